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

template <class G>
__global__ __launch_bounds__(256, 2) void sweep_kernel(SweepArgs p) {
  using E = typename G::E;
  static_assert(2 * G::kStageBytes <= kTile * kCols * 8, "GEMM stages must fit in the block buffer");
  // 64 KB: double-buffered GEMM stages during step 1, then the 128 x 64
  // FP64 block T (S, overwritten row by row with y) during step 2.
  __shared__ __attribute__((aligned(16))) double lds[kTile * kCols];
  // step 2 operands: a slab of rows of the diagonal block of L, and the
  // block's per-row constants (limits, 1/L_ii, lattice generator)
  __shared__ double slab[kSlab * kTile];
  __shared__ double c_at[kTile], c_bt[kTile], c_rl[kTile];
  __shared__ uint64_t c_lat[kTile];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const long NS = (long)p.N * p.S;
  const long nchunks = (NS + kCols - 1) / kCols;
  const long ld = p.ld;
  const E* Lg = (const E*)p.Llow;
  E* Y = (E*)p.yscr + (long)blockIdx.x * p.yslice;
  char* stage0 = (char*)lds;
  char* stage1 = (char*)lds + G::kStageBytes;

  for (long chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
    const long col = chunk * kCols + lane;
    const bool owner = wv == 0;
    const bool valid = owner && col < NS;
    const uint64_t sidx = valid ? (uint64_t)(col / p.N) : 0;
    const uint64_t jpt = valid ? (uint64_t)(col % p.N) + 1 : 1;
    LogProd prod{1.0, 0};

    for (int i0 = 0; i0 < p.n; i0 += kTile) {
      const int rows = min(kTile, p.n - i0);
      typename G::Acc acc;
      G::zero(acc);
      // ---- step 1: S = L[i0:i0+128, 0:i0] Y[0:i0, :]
      if (i0 > 0) {
        const int nst = i0 / G::kK;
        typename G::Regs r;
        G::load(Lg, ld, i0, 0, Y, ld, r);
        G::store(stage0, r);
        __syncthreads();
        for (int s = 0; s < nst; ++s) {
          const bool odd = s & 1;
          if (s + 1 < nst) G::load(Lg, ld, i0, (long)(s + 1) * G::kK, Y, ld, r);
          G::mma(odd ? stage1 : stage0, acc);
          if (s + 1 < nst) G::store(odd ? stage0 : stage1, r);
          __syncthreads();
        }
      }
      // accumulators -> T[row][col] in FP64; per-row constants -> LDS
      G::to_block(acc, lds);
      if (t < rows) {
        const long g = i0 + t;
        c_at[t] = p.at[g];
        c_bt[t] = p.bt[g];
        c_rl[t] = 1.0 / p.L[g * ld + g];
        c_lat[t] = p.lattice[g];
      }
      // ---- step 2: conditioning of the diagonal block
      prod = condition_block((lds_f64*)lds, (lds_f64*)slab, (const lds_f64*)c_at, (const lds_f64*)c_bt,
                             (const lds_f64*)c_rl, (const lds_u64*)c_lat, p.L, ld, i0, rows, p.n, jpt,
                             sidx, p.seed, p.periodize, valid, prod);
      __syncthreads();
      // ---- step 3: y block -> scratch (in the GEMM's operand type)
      G::put_y(lds, Y, ld, i0, rows);
      __syncthreads();
    }
    if (valid) p.ell[col] = logprod_log(prod);
  }
}

long sweep_yslice(int prec, int ld) {
  // elements per workgroup slice of the Y scratch, and bytes per element
  return (long)ld * kCols * (prec == 3 ? 2 : 1);
}

int sweep_elem_bytes(int prec) { return prec == 0 ? 8 : prec == 1 ? 4 : 2; }

hipError_t launch_sweep(const SweepArgs& a, hipStream_t st) {
  switch (a.prec) {
    case 0: hipLaunchKernelGGL(sweep_kernel<GemmF64>, dim3(a.grid), dim3(256), 0, st, a); break;
    case 1: hipLaunchKernelGGL(sweep_kernel<GemmF32>, dim3(a.grid), dim3(256), 0, st, a); break;
    case 2: hipLaunchKernelGGL(sweep_kernel<GemmBF16>, dim3(a.grid), dim3(256), 0, st, a); break;
    case 3: hipLaunchKernelGGL(sweep_kernel<GemmBF16x3>, dim3(a.grid), dim3(256), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ------------------------------------------------------------ reduction
// Per shift: M_s = max_j l, Z_s = sum_j exp(l - M_s) in a fixed-order tree.
__global__ __launch_bounds__(256) void lse_partial_kernel(const double* __restrict__ ell, int N,
                                                          double* __restrict__ part) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  const double* e = ell + (long)blockIdx.x * N;
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
    part[2 * blockIdx.x] = M;
    part[2 * blockIdx.x + 1] = red[0];
  }
}

// log P_s = M_s + log Z_s - log N;  log P = LSE_s log P_s - log S;
// relative standard error = sd_s(P_s) / (sqrt(S) mean_s P_s), in scaled form.
__global__ void lse_final_kernel(const double* __restrict__ part, int N, int S,
                                 const int* __restrict__ info_factor, const int* __restrict__ bad,
                                 double* __restrict__ out) {
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

hipError_t launch_reduce(const double* ell, int N, int S, double* part, const int* info_factor,
                         const int* bad_limits, double* out, hipStream_t st) {
  hipLaunchKernelGGL(lse_partial_kernel, dim3(S), dim3(256), 0, st, ell, N, part);
  hipLaunchKernelGGL(lse_final_kernel, dim3(1), dim3(64), 0, st, (const double*)part, N, S,
                     info_factor, bad_limits, out);
  return hipGetLastError();
}

}  // namespace mvn
