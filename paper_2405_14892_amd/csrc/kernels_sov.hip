// The SOV sweep (arXiv 2405.14892, Algorithms 2-3 with Eq. (sov1)) as one
// persistent kernel, plus the per-call setup and the final mean of
// Algorithm 2 done as a log-sum-exp.
//
// Samples are independent (the recurrence is sequential only along the
// dimension, Section IV-C), so one workgroup owns a block of 128 sample
// columns for the whole sweep and never synchronises with other workgroups;
// only the factor L is shared.  For each block row r of 128 dimensions:
//   1. S = L[r-block, 0:r*128] . Y[0:r*128, cols]   (FP64 MFMA, K = r*128)
//      - the paper's GEMM update of the limit matrices A and B, applied
//        once to a shared shift instead of to two copies of the limits;
//   2. conditioning of the diagonal block, one lane per sample column:
//      s_i = S_i + sum_{k<i in block} L_ik y_k, a' = (a~_i - s_i)/L_ii,
//      b' = (b~_i - s_i)/L_ii, (y_i, log d_i) = condition(a', b', w),
//      l += log d_i;
//   3. y of the block goes to the workgroup's Y scratch for later K loops.
// The uniform matrix R of Algorithm 2 is replaced by Richtmyer points
// generated in registers from the lattice and shift tables.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <limits.h>

#include "gemm_f64.h"
#include "launch.h"
#include "mvn_device.h"

namespace mvn {

int sweep_tile_cols() { return kTile; }

// ------------------------------------------------------------ setup
__global__ __launch_bounds__(256) void shift_table_kernel(uint64_t seed, int n, int S,
                                                          uint64_t* __restrict__ shift,
                                                          int* __restrict__ bad) {
  const long k = (long)blockIdx.x * 256 + threadIdx.x;
  if (k == 0) *bad = INT_MAX;
  if (k < (long)n * S) shift[k] = splitmix64(seed, (uint64_t)k);
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

hipError_t launch_prob_setup(int n, int ld, int S, uint64_t seed, const double* a, const double* b,
                             const double* mu, double* at, double* bt, uint64_t* shift, int* bad,
                             hipStream_t st) {
  const long tot = (long)n * S;
  hipLaunchKernelGGL(shift_table_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, seed,
                     n, S, shift, bad);
  hipLaunchKernelGGL(centre_kernel, dim3((ld + 255) / 256), dim3(256), 0, st, n, ld, a, b, mu, at, bt,
                     bad);
  return hipGetLastError();
}

// ------------------------------------------------------------ the sweep
__global__ __launch_bounds__(256) void sweep_f64_kernel(SweepArgs p) {
  // 128 KB: two double-buffered GEMM stages during step 1, then the
  // 128 x 128 block T (S, overwritten row by row with y) during step 2.
  __shared__ double lds[kTile * kTile];
  const int t = threadIdx.x;
  const long NS = (long)p.N * p.S;
  const long nchunks = (NS + kTile - 1) / kTile;
  double* Y = p.yscr + (long)blockIdx.x * p.ld * kTile;
  const long ld = p.ld;

  for (long chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
    const long col = chunk * kTile + (t & (kTile - 1));
    const bool owner = t < kTile;
    const bool valid = owner && col < NS;
    const long sidx = valid ? col / p.N : 0;
    const uint64_t jpt = valid ? (uint64_t)(col % p.N) + 1 : 1;
    double ell = 0.0;

    for (int i0 = 0; i0 < p.n; i0 += kTile) {
      const int rows = min(kTile, p.n - i0);
      Acc acc;
      acc_zero(acc);
      // ---- step 1: S = L[i0:i0+128, 0:i0] Y[0:i0, :]
      if (i0 > 0) {
        const int nst = i0 / kStageK;
        double ra[8], rb[8];
        load_rows<false>(p.L, ld, i0, 0, 0, 0, ra);
        load_cols(Y, kTile, 0, rb);
        store_rows(lds, ra);
        store_cols(lds + kStageDoubles, rb);
        __syncthreads();
        for (int s = 0; s < nst; ++s) {
          double* cur = lds + (s & 1) * 2 * kStageDoubles;
          double* nxt = lds + ((s + 1) & 1) * 2 * kStageDoubles;
          if (s + 1 < nst) {
            load_rows<false>(p.L, ld, i0, (long)(s + 1) * kStageK, 0, 0, ra);
            load_cols(Y, kTile, (long)(s + 1) * kStageK, rb);
          }
          mma_stage(cur, cur + kStageDoubles, acc);
          if (s + 1 < nst) {
            store_rows(nxt, ra);
            store_cols(nxt + kStageDoubles, rb);
          }
          __syncthreads();
        }
      }
      // accumulators -> T[row][col]
#pragma unroll
      for (int ib = 0; ib < 4; ++ib)
#pragma unroll
        for (int jb = 0; jb < 4; ++jb)
#pragma unroll
          for (int r = 0; r < 4; ++r) lds[acc_row(ib, r) * kTile + acc_col(jb)] = acc.v[ib][jb][r];
      __syncthreads();
      // ---- step 2: conditioning of the diagonal block, lane = column
      if (owner) {
        const int c = t;
        for (int i = 0; i < rows; ++i) {
          const long g = i0 + i;
          const double* Lg = p.L + g * ld + i0;
          double s = lds[i * kTile + c];
          for (int k = 0; k < i; ++k) s += Lg[k] * lds[k * kTile + c];
          const double lgg = Lg[i];
          const double alpha = (p.at[g] - s) / lgg;
          const double beta = (p.bt[g] - s) / lgg;
          const double w = richtmyer(jpt, p.lattice[g], p.shift[sidx * p.n + g], p.periodize);
          const Step st = condition(alpha, beta, w, 1.0 - w);
          lds[i * kTile + c] = valid ? st.y : 0.0;
          ell += st.logd;
        }
      }
      __syncthreads();
      // ---- step 3: y block -> scratch
      for (int e = t; e < rows * kTile; e += 256) Y[(long)(i0 + e / kTile) * kTile + (e % kTile)] = lds[e];
      __syncthreads();
    }
    if (valid) p.ell[col] = ell;
  }
}

hipError_t launch_sweep_f64(const SweepArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(sweep_f64_kernel, dim3(a.grid), dim3(256), 0, st, a);
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
