// Monte Carlo check of detected confidence regions (arXiv 2405.14892,
// Section V-C): fields X = mu + L Z drawn from the fitted distribution, and
// for every sample the first site (in the factor's order) where X leaves
// [a, b].  Because the regions of Algorithm 1 are nested (the first k sites
// in exceedance order), that one index per sample gives the Monte Carlo
// fraction of every nested set: a sample meets the event on the first k
// sites exactly when its first failure comes at or after k.
//
// Normals come from a counter-based generator, so any sample is drawn where
// it is used: Z[i, j] = Phi^-1(U), U = ((SplitMix64 output j n + i) >> 11)
// + 1/2) 2^-53, Phi^-1 by AS 241.
//
// Work: one 64-sample chunk per work item, pulled from a device counter
// (chunk costs differ: see below).  Per block of RB rows the workgroup
//   1. draws Z for the block into its Y scratch,
//   2. forms X - mu = L[block, 0 : i0 + RB] Z[0 : i0 + RB] with the sweep's
//      FP64 MFMA GEMM (the factor's strict upper triangle is zero and its
//      padding the identity, so the diagonal block is just more K),
//   3. finds each sample's first failing row in the block.
// A chunk ends as soon as all its samples have failed: the remaining rows
// cannot change any first failure.  With sites in exceedance order most
// samples fail within the first few hundred sites, so a chunk usually reads
// a small leading part of L.
#include <hip/hip_runtime.h>
#include <limits.h>
#include <stdint.h>

#include "launch.h"
#include "mvn_device.h"
#include "sweep_gemm.h"

namespace mvn {

namespace {

template <int RB>
struct McShape {
  using G = GemmF64T<RB>;
  static constexpr int kT = SweepLdsSize<G>::kT;
  // 70 KB of LDS per workgroup (128 rows) or 36 KB (64 rows)
  static constexpr int kWG = RB == 128 ? 2 : 4;
};

template <int RB>
__global__ __launch_bounds__(256, McShape<RB>::kWG) void mc_kernel(McArgs p) {
  using G = GemmF64T<RB>;
  __shared__ __attribute__((aligned(16))) double T[McShape<RB>::kT];
  __shared__ double s_a[RB], s_b[RB], s_mu[RB];
  __shared__ int s_red[4 * kCols];
  __shared__ long s_item;
  const int t = threadIdx.x, c = t & 63, w = t >> 6;
  const long nchunks = (p.M + kCols - 1) / kCols;
  double* Y = p.yscr + (long)blockIdx.x * p.yslice;
  char* stage0 = (char*)T;
  char* stage1 = (char*)T + G::kStageBytes;
  if (*p.info != 0) {  // no factor: every sample's index is -1
    for (long j = (long)blockIdx.x * 256 + t; j < p.M; j += (long)gridDim.x * 256)
      if (p.first) p.first[j] = -1;
    return;
  }
  for (;;) {
    if (t == 0) s_item = (long)atomicAdd(p.counter, 1ull);
    __syncthreads();
    const long chunk = s_item;
    __syncthreads();
    if (chunk >= nchunks) break;
    const long j = chunk * kCols + c;
    bool alive = w == 0 && j < p.M;
    int my_first = p.n;
    for (int i0 = 0; i0 < p.n; i0 += RB) {
      const int rows = min(RB, p.n - i0);
      // ---- 1: Z of this block (zero in padding rows and past M); limits
      for (int e = t; e < RB * kCols; e += 256) {
        const int r = e >> 6, cc = e & 63;
        const long g = i0 + r, jj = chunk * kCols + cc;
        Y[(long)(i0 + r) * kCols + cc] =
            (g < p.n && jj < p.M) ? normal_from_counter(p.seed, (uint64_t)jj * (uint64_t)p.n + (uint64_t)g) : 0.0;
      }
      if (t < rows) {
        s_a[t] = p.a[i0 + t];
        s_b[t] = p.b[i0 + t];
        s_mu[t] = p.mu ? p.mu[i0 + t] : 0.0;
      }
      __syncthreads();
      // ---- 2: X - mu for the block: K = 0 .. i0 + RB
      typename G::Acc acc;
      G::zero(acc);
      {
        const int nst = (i0 + RB) / G::kK;
        typename G::Regs r;
        G::load(p.L, p.ld, 0, i0, 0, Y, p.ld, r);
        G::store(stage0, r);
        __syncthreads();
        for (int s = 0; s < nst; ++s) {
          const bool odd = s & 1;
          if (s + 1 < nst) G::load(p.L, p.ld, 0, i0, (long)(s + 1) * G::kK, Y, p.ld, r);
          G::mma(odd ? stage1 : stage0, acc);
          if (s + 1 < nst) G::store(odd ? stage0 : stage1, r);
          __syncthreads();
        }
      }
      G::to_block(acc, T);
      __syncthreads();
      // ---- 3: first failing row of the block per sample (wave w scans rows w, w + 4, ...)
      int fr = INT_MAX;
      for (int r = w; r < rows; r += 4) {
        const double x = T[r * kCols + c] + s_mu[r];
        if (!(x >= s_a[r] && x <= s_b[r])) {
          fr = r;
          break;
        }
      }
      s_red[w * kCols + c] = fr;
      __syncthreads();
      if (w == 0) {
        const int m = min(min(s_red[c], s_red[kCols + c]), min(s_red[2 * kCols + c], s_red[3 * kCols + c]));
        if (alive && m != INT_MAX) {
          my_first = i0 + m;
          alive = false;
        }
      }
      if (!__syncthreads_or(alive ? 1 : 0)) break;
    }
    if (w == 0 && j < p.M) {
      if (p.first) p.first[j] = my_first;
      atomicAdd(p.hist + my_first, 1ull);
    }
  }
}

__global__ __launch_bounds__(256) void mc_clear_kernel(unsigned long long* hist, int bins, unsigned long long* counter) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < bins) hist[i] = 0;
  if (i == 0) *counter = 0;
}

// count[k] = M - #{first <= k}: samples inside the limits on sites 0..k.
__global__ __launch_bounds__(1024) void mc_count_kernel(const unsigned long long* __restrict__ hist, int n, long M,
                                                        const int* __restrict__ info, long long* __restrict__ count) {
  __shared__ unsigned long long part[1024];
  const int t = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int lo = min(n, t * per), hi = min(n, lo + per);
  if (*info != 0) {
    for (int k = lo; k < hi; ++k) count[k] = -1;
    return;
  }
  unsigned long long s = 0;
  for (int f = lo; f < hi; ++f) s += hist[f];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {  // inclusive scan of the segment sums
    const unsigned long long v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  unsigned long long below = t ? part[t - 1] : 0;
  for (int k = lo; k < hi; ++k) {
    below += hist[k];
    count[k] = (long long)(M - (long)below);
  }
}

}  // namespace

int mc_wg_per_cu(int rows) { return rows == 128 ? McShape<128>::kWG : McShape<64>::kWG; }

hipError_t launch_mc(const McArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(mc_clear_kernel, dim3((a.n + 1 + 255) / 256), dim3(256), 0, st, a.hist, a.n + 1, a.counter);
  if (a.rows == 128)
    hipLaunchKernelGGL(mc_kernel<128>, dim3(a.grid), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(mc_kernel<64>, dim3(a.grid), dim3(256), 0, st, a);
  hipLaunchKernelGGL(mc_count_kernel, dim3(1), dim3(1024), 0, st, (const unsigned long long*)a.hist, a.n, a.M,
                     a.info, a.count);
  return hipGetLastError();
}

}  // namespace mvn
