// The SOV sweep (arXiv 2405.14892, Algorithms 2-3 with Eq. (sov1)) as one
// persistent kernel, plus the per-call setup and the final mean of
// Algorithm 2 done as a log-sum-exp.
//
// Samples are independent (the recurrence is sequential only along the
// dimension, Section IV-C), so one workgroup owns a block of 64 sample
// columns for the whole sweep and never synchronises with other workgroups;
// only the factor L is shared.  For each block row r of 128 dimensions:
//   1. S = L[r-block, 0:r*128] . Y[0:r*128, cols]   (MFMA, K = r*128, in
//      FP64, or FP32 / BF16 / split BF16 with FP32 accumulation)
//      - the paper's GEMM update of the limit matrices A and B, applied
//        once to a shared shift instead of to two copies of the limits;
//   2. conditioning of the diagonal block, one lane per sample column:
//      s_i = S_i + sum_{k<i in block} L_ik y_k, a' = (a~_i - s_i)/L_ii,
//      b' = (b~_i - s_i)/L_ii, (y_i, d_i) = condition_step(a', b', w),
//      with prod d_i kept as mantissa x 2^exponent and l = log of it at the
//      end of the sweep;
//   3. y of the block goes to the workgroup's Y scratch for later K loops.
// The uniform matrix R of Algorithm 2 is replaced by Richtmyer points
// generated in registers from the lattice table and the SplitMix64 shift.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <limits.h>

#include <type_traits>

#include "gemm_f64.h"
#include "launch.h"
#include "mvn_device.h"
#include "sweep_block.h"
#include "sweep_gemm.h"

namespace mvn {

// ------------------------------------------------------------ setup
__global__ void flag_init_kernel(int* __restrict__ bad) {
  if (threadIdx.x == 0) *bad = INT_MAX;
}

__global__ __launch_bounds__(256) void centre_kernel(int n, int ld, const double* __restrict__ a,
                                                     const double* __restrict__ b,
                                                     const double* __restrict__ mu,
                                                     double* __restrict__ at, double* __restrict__ bt,
                                                     int* __restrict__ bad) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= ld) return;
  if (i >= n) {
    at[i] = -INFINITY;
    bt[i] = INFINITY;
    return;
  }
  const double ai = a[i], bi = b[i], m = mu ? mu[i] : 0.0;
  if (isnan(ai) || isnan(bi) || !isfinite(m) || ai > bi) atomicMin(bad, i + 1);
  at[i] = ai - m;
  bt[i] = bi - m;
}

hipError_t launch_prob_setup(int n, int ld, const double* a, const double* b, const double* mu,
                             double* at, double* bt, int* bad, hipStream_t st) {
  hipLaunchKernelGGL(flag_init_kernel, dim3(1), dim3(64), 0, st, bad);
  hipLaunchKernelGGL(centre_kernel, dim3((ld + 255) / 256), dim3(256), 0, st, n, ld, a, b, mu, at, bt,
                     bad);
  return hipGetLastError();
}

// ------------------------------------------------------------ the sweep
// One workgroup of four wave64s owns 64 sample columns (see sweep_gemm.h for
// the GEMM tiling).  76 KB of LDS and <= 256 registers per lane let two
// workgroups share a CU, so one workgroup's conditioning (VALU) can overlap
// the other's GEMM (MFMA).
int sweep_tile_cols() { return kCols; }

// Shared memory of one sweep workgroup.
struct SweepLds {
  double* T;         // RB x 64 block (also the double-buffered GEMM stages)
  double* slab;
  double* c_at;
  double* c_bt;
  double* c_rl;
  uint64_t* c_lat;
};

// The whole sweep of one 64-column chunk of one problem: for every RB-row
// block, the GEMM (step 1), the conditioning (step 2) and the y write-back
// (step 3).  Writes l of the chunk's valid samples to ell[col].
template <class G, bool PREFIX = false>
__device__ __forceinline__ void sweep_chunk(const SweepLds& sh, const double* __restrict__ L,
                                            const typename G::E* __restrict__ Lg, long lplane, long ld, int n,
                                            const double* __restrict__ at, const double* __restrict__ bt,
                                            const uint64_t* __restrict__ lattice, uint64_t seed, int N, int S,
                                            int periodize, typename G::E* __restrict__ Y,
                                            double* __restrict__ ell, long chunk,
                                            double* __restrict__ prefix = nullptr) {
  constexpr int RB = G::kRows;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const long NS = (long)N * S;
  char* stage0 = (char*)sh.T;
  char* stage1 = (char*)sh.T + G::kStageBytes;
  const long col = chunk * kCols + lane;
  const bool owner = wv == 0;
  const bool valid = owner && col < NS;
  const uint64_t sidx = col < NS ? (uint64_t)(col / N) : 0;  // every lane: its own column
  const uint64_t jpt = col < NS ? (uint64_t)(col % N) + 1 : 1;
  LogProd prod{1.0, 0};
  const PrefixOut pre{prefix, (NS + kCols - 1) / kCols, chunk, (uint64_t)(chunk * kCols / N)};

  for (int i0 = 0; i0 < n; i0 += RB) {
    const int rows = min(RB, n - i0);
    typename G::Acc acc;
    G::zero(acc);
    // ---- step 1: S = L[i0:i0+RB, 0:i0] Y[0:i0, :]
    if (i0 > 0) {
      const int nst = i0 / G::kK;
      typename G::Regs r;
      G::load(Lg, ld, lplane, i0, 0, Y, ld, r);
      G::store(stage0, r);
      __syncthreads();
      for (int s = 0; s < nst; ++s) {
        const bool odd = s & 1;
        if (s + 1 < nst) G::load(Lg, ld, lplane, i0, (long)(s + 1) * G::kK, Y, ld, r);
        G::mma(odd ? stage1 : stage0, acc);
        if (s + 1 < nst) G::store(odd ? stage0 : stage1, r);
        __syncthreads();
      }
    }
    // accumulators -> T[row][col] in FP64; per-row constants -> LDS
    G::to_block(acc, sh.T);
    if (t < rows) {
      const long g = i0 + t;
      sh.c_at[t] = at[g];
      sh.c_bt[t] = bt[g];
      sh.c_rl[t] = 1.0 / L[g * ld + g];
      sh.c_lat[t] = lattice[g];
    }
    // ---- step 2: conditioning of the diagonal block
    prod = condition_block<!std::is_same<typename G::E, double>::value, RB, true, PREFIX>(
        (lds_f64*)sh.T, (lds_f64*)sh.slab, (const lds_f64*)sh.c_at, (const lds_f64*)sh.c_bt,
        (const lds_f64*)sh.c_rl, (const lds_u64*)sh.c_lat, L, ld, i0, rows, n, jpt, sidx, seed, periodize, valid,
        prod, nullptr, 0, pre);
    __syncthreads();
    // ---- step 3: y block -> scratch (in the GEMM's operand type)
    G::put_y(sh.T, Y, ld, i0, rows);
    __syncthreads();
  }
  if (valid) ell[col] = logprod_log(prod);
}

#define MVN_SWEEP_LDS(G)                                                              \
  __shared__ __attribute__((aligned(16))) double lds_T[SweepLdsSize<G>::kT];          \
  __shared__ double lds_slab[kSlab * G::kRows];                                       \
  __shared__ double lds_at[G::kRows], lds_bt[G::kRows], lds_rl[G::kRows];             \
  __shared__ uint64_t lds_lat[G::kRows];                                              \
  const SweepLds sh{lds_T, lds_slab, lds_at, lds_bt, lds_rl, lds_lat}

// Workgroups per CU: two for the 128-row shape; four for the 64-row shape
// (38-41 KB of LDS, <= 128 VGPRs), three for its split-BF16 form (47 KB).
template <class G>
struct SweepOccupancy {
  // LDS of one workgroup (block buffer, slab, per-row constants, work-item
  // slot, AS 241 coefficient table)
  static constexpr int kLds = SweepLdsSize<G>::kT * 8 + kSlab * G::kRows * 8 + 4 * G::kRows * 8 + 16 + 48 * 8;
  static constexpr int kWG = G::kRows == 128 ? 2 : (4 * kLds <= 160 * 1024 ? 4 : 3);
};

template <class G, bool PREFIX = false>
__global__ __launch_bounds__(256, SweepOccupancy<G>::kWG) void sweep_kernel(SweepArgs p) {
  using E = typename G::E;
  MVN_SWEEP_LDS(G);
  const long nchunks = ((long)p.N * p.S + kCols - 1) / kCols;
  E* Y = (E*)p.yscr + (long)blockIdx.x * p.yslice;
  for (long chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x)
    sweep_chunk<G, PREFIX>(sh, p.L, (const E*)p.Llow, (long)p.ld * p.ld, p.ld, p.n, p.at, p.bt, p.lattice,
                           p.seed, p.N, p.S, p.periodize, Y, p.ell, chunk, p.prefix);
}

// Batches: work items (problem rank, chunk) in order of decreasing problem
// size, pulled from a device counter; every workgroup leaves when the
// counter passes the number of items.
template <class G>
__global__ __launch_bounds__(256, SweepOccupancy<G>::kWG) void batch_sweep_kernel(BatchSweepArgs p) {
  using E = typename G::E;
  MVN_SWEEP_LDS(G);
  __shared__ long s_item;
  const long nchunks = ((long)p.N * p.S + kCols - 1) / kCols;
  const long NS = (long)p.N * p.S;
  E* Y = (E*)p.yscr + (long)blockIdx.x * p.yslice;
  for (;;) {
    if (threadIdx.x == 0) s_item = (long)atomicAdd(p.counter, 1ull);
    __syncthreads();
    const long item = s_item;
    __syncthreads();
    if (item >= p.total_items) break;
    const int prob = p.order[item / nchunks];
    const long chunk = item % nchunks;
    const BatchDesc d = p.desc[prob];
    sweep_chunk<G>(sh, p.L + d.factor_off, (const E*)p.Llow + d.factor_off, p.lplane, d.ld, d.n,
                   p.at + d.lim_off, p.bt + d.lim_off, p.lattice, p.seed, p.N, p.S, p.periodize, Y,
                   p.ell + (long)prob * NS, chunk);
  }
}

int sweep_wg_per_cu(int rows, int prec) {
  if (rows != 64) return 2;
  switch (prec) {
    case 0: return SweepOccupancy<GemmF64T<64>>::kWG;
    case 1: return SweepOccupancy<GemmF32T<64>>::kWG;
    case 2: return SweepOccupancy<GemmBF16T<1, 64>>::kWG;
    default: return SweepOccupancy<GemmBF16T<2, 64>>::kWG;
  }
}

long sweep_yslice(int prec, int ld) {
  // elements per workgroup slice of the Y scratch, and bytes per element
  return (long)ld * kCols * (prec == 3 ? 2 : 1);
}

int sweep_elem_bytes(int prec) { return prec == 0 ? 8 : prec == 1 ? 4 : 2; }

template <bool PREFIX>
static hipError_t launch_sweep_t(const SweepArgs& a, hipStream_t st) {
  const dim3 g(a.grid), b(256);
  if (a.rows == 64) {
    switch (a.prec) {
      case 0: hipLaunchKernelGGL((sweep_kernel<GemmF64T<64>, PREFIX>), g, b, 0, st, a); break;
      case 1: hipLaunchKernelGGL((sweep_kernel<GemmF32T<64>, PREFIX>), g, b, 0, st, a); break;
      case 2: hipLaunchKernelGGL((sweep_kernel<GemmBF16T<1, 64>, PREFIX>), g, b, 0, st, a); break;
      case 3: hipLaunchKernelGGL((sweep_kernel<GemmBF16T<2, 64>, PREFIX>), g, b, 0, st, a); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (a.prec) {
      case 0: hipLaunchKernelGGL((sweep_kernel<GemmF64, PREFIX>), g, b, 0, st, a); break;
      case 1: hipLaunchKernelGGL((sweep_kernel<GemmF32, PREFIX>), g, b, 0, st, a); break;
      case 2: hipLaunchKernelGGL((sweep_kernel<GemmBF16, PREFIX>), g, b, 0, st, a); break;
      case 3: hipLaunchKernelGGL((sweep_kernel<GemmBF16x3, PREFIX>), g, b, 0, st, a); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

hipError_t launch_sweep(const SweepArgs& a, hipStream_t st) {
  if (a.narrow) return launch_narrow_sweep(a, st);
  if (a.wide) return launch_wide_sweep(a, st);
  if (a.quad) return launch_quad_sweep(a, st);
  return a.prefix ? launch_sweep_t<true>(a, st) : launch_sweep_t<false>(a, st);
}

// ------------------------------------------------------------ reduction
// Per shift: M_s = max_j l, Z_s = sum_j exp(l - M_s) in a fixed-order tree.
__device__ __forceinline__ void lse_partial_body(const double* __restrict__ ell, int N,
                                                 double* __restrict__ part, int s) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  const double* e = ell + (long)s * N;
  double m = -INFINITY;
  for (int j = t; j < N; j += 256) m = fmax(m, e[j]);
  red[t] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] = fmax(red[t], red[t + w]);
    __syncthreads();
  }
  const double M = red[0];
  __syncthreads();
  double z = 0.0;
  if (M > -INFINITY)
    for (int j = t; j < N; j += 256) z += exp(e[j] - M);
  red[t] = z;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (t == 0) {
    part[2 * s] = M;
    part[2 * s + 1] = red[0];
  }
}

__global__ __launch_bounds__(256) void lse_partial_kernel(const double* __restrict__ ell, int N,
                                                          double* __restrict__ part) {
  lse_partial_body(ell, N, part, blockIdx.x);
}

// log P_s = M_s + log Z_s - log N;  log P = LSE_s log P_s - log S;
// relative standard error = sd_s(P_s) / (sqrt(S) mean_s P_s), in scaled form.
__device__ __forceinline__ void lse_final_body(const double* __restrict__ part, int N, int S,
                                               const int* __restrict__ info_factor,
                                               const int* __restrict__ bad, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  const bool broken = (info_factor && *info_factor != 0) || (bad && *bad != INT_MAX);
  if (broken) {
    for (int k = 0; k < 4 + S; ++k) out[k] = NAN;
    return;
  }
  const double logN = log((double)N);
  double mx = -INFINITY;
  for (int s = 0; s < S; ++s) {
    const double M = part[2 * s], Z = part[2 * s + 1];
    const double lp = (M > -INFINITY && Z > 0.0) ? M + log(Z) - logN : -INFINITY;
    out[4 + s] = lp;
    mx = fmax(mx, lp);
  }
  double sum = 0.0;
  if (mx > -INFINITY)
    for (int s = 0; s < S; ++s) sum += exp(out[4 + s] - mx);
  const double logp = (mx > -INFINITY) ? mx + log(sum) - log((double)S) : -INFINITY;
  out[0] = logp;
  out[1] = exp(logp);
  if (S > 1 && mx > -INFINITY) {
    const double mean = sum / S;
    double var = 0.0;
    for (int s = 0; s < S; ++s) {
      const double d = exp(out[4 + s] - mx) - mean;
      var += d * d;
    }
    var /= (S - 1);
    const double rel = sqrt(var / S) / mean;
    out[3] = rel;
    out[2] = rel * out[1];
  } else {
    out[2] = NAN;
    out[3] = NAN;
  }
}

__global__ void lse_final_kernel(const double* __restrict__ part, int N, int S,
                                 const int* __restrict__ info_factor, const int* __restrict__ bad,
                                 double* __restrict__ out) {
  lse_final_body(part, N, S, info_factor, bad, out);
}

hipError_t launch_reduce(const double* ell, int N, int S, double* part, const int* info_factor,
                         const int* bad_limits, double* out, hipStream_t st) {
  hipLaunchKernelGGL(lse_partial_kernel, dim3(S), dim3(256), 0, st, ell, N, part);
  hipLaunchKernelGGL(lse_final_kernel, dim3(1), dim3(64), 0, st, (const double*)part, N, S,
                     info_factor, bad_limits, out);
  return hipGetLastError();
}

// ------------------------------------------------------------ nested sets
// Per (row, shift): the running products of the shift's N samples after the
// row, summed exactly over the chunk partials of prefix_row in chunk order;
// lps = log(sum 2^E / N), the shift's estimate of P(first row + 1 sites).
__global__ __launch_bounds__(256) void prefix_shift_kernel(const double* __restrict__ part, long nchunks, int cols,
                                                           int n, int N, int S, double* __restrict__ lps) {
  const long id = (long)blockIdx.x * 256 + threadIdx.x;
  if (id >= (long)n * S) return;
  const long row = id / S;
  const int s = (int)(id % S);
  const long c_lo = (long)s * N / cols, c_hi = ((long)(s + 1) * N - 1) / cols;
  int E = kNoExp;
  double sum = 0.0;
  for (long c = c_lo; c <= c_hi; ++c) {
    const int slot = (c * cols / N == s) ? 0 : 1;
    const double* d = part + (row * nchunks + c) * 4 + 2 * slot;
    const double v = d[1];
    if (!(v > 0.0)) continue;
    const int e = (int)d[0];
    if (e > E) {
      sum = ldexp(sum, E - e) + v;
      E = e;
    } else {
      sum += ldexp(v, e - E);
    }
  }
  lps[id] = sum > 0.0 ? log(sum) + (double)E * kLn2 - log((double)N) : -INFINITY;
}

// Per row: the mean over shifts in log space and the relative standard
// error over shifts, as for the full estimate (lse_final_body).
__global__ __launch_bounds__(256) void prefix_final_kernel(const double* __restrict__ lps, int n, int S,
                                                           const int* __restrict__ info_factor,
                                                           const int* __restrict__ bad,
                                                           double* __restrict__ out) {
  const long row = (long)blockIdx.x * 256 + threadIdx.x;
  if (row >= n) return;
  if ((info_factor && *info_factor != 0) || (bad && *bad != INT_MAX)) {
    out[2 * row] = NAN;
    out[2 * row + 1] = NAN;
    return;
  }
  const double* l = lps + row * S;
  double mx = -INFINITY;
  for (int s = 0; s < S; ++s) mx = fmax(mx, l[s]);
  double sum = 0.0;
  if (mx > -INFINITY)
    for (int s = 0; s < S; ++s) sum += exp(l[s] - mx);
  out[2 * row] = (mx > -INFINITY) ? mx + log(sum) - log((double)S) : -INFINITY;
  if (S > 1 && mx > -INFINITY) {
    const double mean = sum / S;
    double var = 0.0;
    for (int s = 0; s < S; ++s) {
      const double d = exp(l[s] - mx) - mean;
      var += d * d;
    }
    var /= (S - 1);
    out[2 * row + 1] = sqrt(var / S) / mean;
  } else {
    out[2 * row + 1] = NAN;
  }
}

hipError_t launch_prefix_reduce(const double* part, long nchunks, int cols, int n, int N, int S, double* lps,
                                const int* info_factor, const int* bad_limits, double* out, hipStream_t st) {
  const long tot = (long)n * S;
  hipLaunchKernelGGL(prefix_shift_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, part, nchunks,
                     cols, n, N, S, lps);
  hipLaunchKernelGGL(prefix_final_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     (const double*)lps, n, S, info_factor, bad_limits, out);
  return hipGetLastError();
}

// ------------------------------------------------------------ batches
__global__ void batch_init_kernel(int* __restrict__ bad, int count, unsigned long long* __restrict__ counter) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < count) bad[i] = INT_MAX;
  if (i == 0) *counter = 0ull;
}

__global__ __launch_bounds__(256) void batch_centre_kernel(const BatchDesc* __restrict__ desc,
                                                           const double* __restrict__ a,
                                                           const double* __restrict__ b,
                                                           const double* __restrict__ mu,
                                                           double* __restrict__ at, double* __restrict__ bt,
                                                           int* __restrict__ bad) {
  const int p = blockIdx.y;
  const BatchDesc d = desc[p];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= d.n) return;
  const long g = d.lim_off + i;
  const double ai = a[g], bi = b[g], m = mu ? mu[g] : 0.0;
  if (isnan(ai) || isnan(bi) || !isfinite(m) || ai > bi) atomicMin(bad + p, i + 1);
  at[g] = ai - m;
  bt[g] = bi - m;
}

hipError_t launch_batch_setup(const BatchDesc* desc, int count, int nmax, const double* a, const double* b,
                              const double* mu, double* at, double* bt, int* bad,
                              unsigned long long* counter, hipStream_t st) {
  hipLaunchKernelGGL(batch_init_kernel, dim3((count + 255) / 256), dim3(256), 0, st, bad, count, counter);
  hipLaunchKernelGGL(batch_centre_kernel, dim3((nmax + 255) / 256, count), dim3(256), 0, st, desc, a, b, mu,
                     at, bt, bad);
  return hipGetLastError();
}

hipError_t launch_batch_sweep(const BatchSweepArgs& a, hipStream_t st) {
  const dim3 g(a.grid), b(256);
  if (a.rows == 64) {
    switch (a.prec) {
      case 0: hipLaunchKernelGGL(batch_sweep_kernel<GemmF64T<64>>, g, b, 0, st, a); break;
      case 1: hipLaunchKernelGGL(batch_sweep_kernel<GemmF32T<64>>, g, b, 0, st, a); break;
      case 2: hipLaunchKernelGGL((batch_sweep_kernel<GemmBF16T<1, 64>>), g, b, 0, st, a); break;
      case 3: hipLaunchKernelGGL((batch_sweep_kernel<GemmBF16T<2, 64>>), g, b, 0, st, a); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (a.prec) {
      case 0: hipLaunchKernelGGL(batch_sweep_kernel<GemmF64>, g, b, 0, st, a); break;
      case 1: hipLaunchKernelGGL(batch_sweep_kernel<GemmF32>, g, b, 0, st, a); break;
      case 2: hipLaunchKernelGGL(batch_sweep_kernel<GemmBF16>, g, b, 0, st, a); break;
      case 3: hipLaunchKernelGGL(batch_sweep_kernel<GemmBF16x3>, g, b, 0, st, a); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void batch_lse_partial_kernel(const double* __restrict__ ell, int N, int S,
                                                                double* __restrict__ part) {
  const int p = blockIdx.y;
  lse_partial_body(ell + (long)p * N * S, N, part + (long)p * 2 * S, blockIdx.x);
}

__global__ void batch_lse_final_kernel(const double* __restrict__ part, int N, int S,
                                       const int* __restrict__ info, const int* __restrict__ bad,
                                       double* __restrict__ out) {
  const int p = blockIdx.x;
  lse_final_body(part + (long)p * 2 * S, N, S, info + p, bad + p, out + (long)p * (4 + S));
}

hipError_t launch_batch_reduce(const double* ell, int count, int N, int S, double* part, const int* info,
                               const int* bad, double* out, hipStream_t st) {
  hipLaunchKernelGGL(batch_lse_partial_kernel, dim3(S, count), dim3(256), 0, st, ell, N, S, part);
  hipLaunchKernelGGL(batch_lse_final_kernel, dim3(count), dim3(64), 0, st, (const double*)part, N, S, info,
                     bad, out);
  return hipGetLastError();
}

}  // namespace mvn
