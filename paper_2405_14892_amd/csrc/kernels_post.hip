// Posterior of a Gaussian field observed with noise at m of its n sites
// (arXiv 2405.14892, Section V-B, the equations for Sigma_post and
// mu_post), by one partial Cholesky factorisation of a bordered matrix.
//
// With K = Sigma_oo + sigma_eps^2 I (the observed sites), C = Sigma_o. (m x
// n) and r = y - mu_o, the Woodbury form of the two equations reads
//   Sigma_post = Sigma - C^T K^-1 C,   mu_post = mu + C^T K^-1 r.
// Both are Schur complements of K in
//        [ K    C      0 ]      rows 0 .. m'-1   (observations, padded)
//   B =  [ C^T  Sigma  * ]      rows m' .. m'+n-1 (sites)
//        [ r^T  0      1 ]      row  m'+n         (data)
// (lower triangle stored): factoring only the first m' columns (L_K, then
// W = L_K^-1 C and v = L_K^-1 r below it) leaves in the trailing block
//   Sigma - W^T W = Sigma_post           on the sites,
//   0 - v^T W     = -(mu_post - mu)^T    on the data row.
// So the posterior costs one K factorisation, one panel solve and one
// trailing update of the site block: the library's tiled Cholesky stopped
// after m' columns.  The observations are padded to m' (a multiple of the
// Cholesky tile) with identity rows and columns, which decouple.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch.h"
#include "matern.h"

namespace mvn {

namespace {

__device__ __forceinline__ double& B_at(const PosteriorArgs& p, long i, long j) { return p.B[i * p.ld + j]; }

// Lower triangle of B, 16 x 16 elements per workgroup; clears *info (-1
// and the identity when an observed-site index is out of range).
__global__ __launch_bounds__(256) void posterior_build_kernel(PosteriorArgs p) {
  const bool bad = *p.obs_bad != 0;
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *p.info = bad ? -1 : 0;
  const long i = (long)blockIdx.y * 16 + (threadIdx.x >> 4);
  const long j = (long)blockIdx.x * 16 + (threadIdx.x & 15);
  if (i >= p.ld || j > i) return;
  if (bad) {
    B_at(p, i, j) = (i == j) ? 1.0 : 0.0;
    return;
  }
  const long mp = p.mpad, e = p.mpad + p.n;  // first site row, data row
  auto site = [&](long r) -> long { return r < mp ? p.obs[r] : r - mp; };  // site index of an observation/site row
  auto cov = [&](long a, long b) {  // Sigma between sites a and b (nugget on equal sites)
    const double dx = p.locs[2 * a] - p.locs[2 * b];
    const double dy = p.locs[2 * a + 1] - p.locs[2 * b + 1];
    return matern_cov(p.mk, sqrt(dx * dx + dy * dy)) + (a == b ? p.mk.nugget : 0.0);
  };
  double v;
  const bool obs_i = i < p.m, obs_j = j < p.m;
  const bool pad_i = (i >= p.m && i < mp) || i > e, pad_j = (j >= p.m && j < mp) || j > e;
  if (pad_i || pad_j) {
    v = (i == j) ? 1.0 : 0.0;
  } else if (i == e) {
    v = (j == e) ? 1.0 : (obs_j ? p.y[j] - (p.mu ? p.mu[p.obs[j]] : 0.0) : 0.0);
  } else {
    // both rows are observations or sites (i >= j)
    v = cov(site(i), site(j));
    if (obs_i && i == j) v += p.noise_var;
  }
  B_at(p, i, j) = v;
}

__global__ __launch_bounds__(256) void posterior_moments_kernel(PosteriorArgs p, double* __restrict__ mu_post,
                                                                double* __restrict__ var_post) {
  const long j = (long)blockIdx.x * 256 + threadIdx.x;
  if (j >= p.n) return;
  const long mp = p.mpad, e = p.mpad + p.n;
  const bool ok = *p.info == 0;
  if (mu_post) mu_post[j] = ok ? (p.mu ? p.mu[j] : 0.0) - B_at(p, e, mp + j) : NAN;
  if (var_post) var_post[j] = ok ? B_at(p, mp + j, mp + j) : NAN;
}

}  // namespace

hipError_t launch_posterior(const PosteriorArgs& p, int tile, double* mu_post, double* var_post, hipStream_t st) {
  const dim3 grid((unsigned)(p.ld / 16), (unsigned)(p.ld / 16));
  hipError_t e = launch_index_check(p.obs, p.m, p.n, nullptr, const_cast<int*>(p.obs_bad), st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(posterior_build_kernel, grid, dim3(256), 0, st, p);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the first m' columns only; a non-positive pivot of K lands in *info
  e = launch_cholesky_f64((int)p.ld, tile, p.B, p.info, st, true, (int)p.mpad);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(posterior_moments_kernel, dim3((unsigned)((p.n + 255) / 256)), dim3(256), 0, st, p, mu_post,
                     var_post);
  return hipGetLastError();
}

// ------------------------------------------------------------ exceedance order
// The site order of Algorithm 1 (Section IV-A): decreasing marginal
// exceedance probability p_i = Phi((mu_i - u) / sd_i), ties by increasing
// site index.  Keys are the pairs (-p_i, i) in ascending lexicographic order,
// which makes the order total; they are sorted by a bitonic network over
// npad = the next power of two (padding keys (+inf, i) sort last), one
// launch per compare-exchange stage, each thread owning one pair of
// elements.  A variance <= 0 gives p = 1 if mu_i > u, else 0; a NaN
// variance or a non-finite mean sets *bad.
__global__ __launch_bounds__(256) void exceed_keys_kernel(int n, long npad, const double* __restrict__ mu,
                                                          const double* __restrict__ var, double u,
                                                          double* __restrict__ key, int64_t* __restrict__ idx,
                                                          double* __restrict__ p_out, int* __restrict__ bad) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= npad) return;
  if (i < n) {
    const double v = var[i], m = mu[i];
    const bool ok = !isnan(v) && isfinite(m);
    // a variance at or below zero (a site known exactly, up to rounding) gives p = 1 above u, else 0
    const double p = !ok ? NAN
                         : v > 0.0 ? 0.5 * erfc(-(m - u) / sqrt(v) * 0.70710678118654752440)
                                   : (m > u ? 1.0 : 0.0);
    if (!ok) atomicExch(bad, 1);
    key[i] = ok ? -p : INFINITY;
    if (p_out) p_out[i] = p;
  } else {
    key[i] = INFINITY;
  }
  idx[i] = i;
}

__global__ __launch_bounds__(256) void bitonic_step_kernel(long npad, long j, long k, double* __restrict__ key,
                                                           int64_t* __restrict__ idx) {
  const long t = (long)blockIdx.x * 256 + threadIdx.x;  // one per pair
  if (t >= npad / 2) return;
  const long i = 2 * t - (t & (j - 1));  // the lower element: bit log2(j) clear
  const long l = i + j;
  const bool up = (i & k) == 0;          // ascending block
  const double ki = key[i], kl = key[l];
  const int64_t ii = idx[i], il = idx[l];
  const bool gt = ki > kl || (ki == kl && ii > il);
  if (gt == up) {
    key[i] = kl;
    key[l] = ki;
    idx[i] = il;
    idx[l] = ii;
  }
}

__global__ void exceed_flag_kernel(int* __restrict__ bad) {
  if (threadIdx.x == 0) *bad = 0;
}

__global__ __launch_bounds__(256) void exceed_out_kernel(int n, const int64_t* __restrict__ idx,
                                                         const int* __restrict__ bad, int64_t* __restrict__ perm) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) perm[i] = *bad ? -1 : idx[i];
}

long exceedance_npad(int n) {
  long p = 1;
  while (p < n) p <<= 1;
  return p;
}

hipError_t launch_exceedance_order(int n, const double* mu, const double* var, double u, double* key, int64_t* idx,
                                   int* bad, double* p_out, int64_t* perm, hipStream_t st) {
  const long npad = exceedance_npad(n);
  hipLaunchKernelGGL(exceed_flag_kernel, dim3(1), dim3(64), 0, st, bad);
  hipLaunchKernelGGL(exceed_keys_kernel, dim3((unsigned)((npad + 255) / 256)), dim3(256), 0, st, n, npad, mu, var, u,
                     key, idx, p_out, bad);
  const unsigned g = (unsigned)((npad / 2 + 255) / 256);
  for (long k = 2; k <= npad; k <<= 1)
    for (long j = k >> 1; j > 0; j >>= 1)
      hipLaunchKernelGGL(bitonic_step_kernel, dim3(g > 0 ? g : 1), dim3(256), 0, st, npad, j, k, key, idx);
  hipLaunchKernelGGL(exceed_out_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, (const int64_t*)idx,
                     (const int*)bad, perm);
  return hipGetLastError();
}

}  // namespace mvn
