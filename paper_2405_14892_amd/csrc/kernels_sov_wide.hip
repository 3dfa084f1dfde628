// The dense FP64 SOV sweep (Algorithms 2-3 with Eq. (sov1)) with 256-row
// blocks and 128 sample columns per workgroup of eight waves, one workgroup
// per CU.
//
// The limit-update GEMM S = L[r-block, 0:i0] Y[0:i0, cols] streams the
// factor once per workgroup pass and the sample block Y once per block row.
// With 128 columns per pass the factor is read half as often as by the
// 64-column sweep, and with 256-row blocks the Y scratch half as often as
// with 128-row ones: 48 KB of operands per K stage of a 256 x 128 x 16
// product instead of 64 KB for two 128 x 128 x 16 ones.  The accumulators of
// the 256 x 128 block (64 doubles per lane, as for two 128 x 128 blocks of
// four waves) stay in the waves' registers through the in-block recurrence:
//   * in a full pass waves 2s and 2s + 1 hold S for the 128-row halves of
//     block x columns [32 s, 32 s + 32);
//   * the block is conditioned in 32-row sub-blocks: the waves write the
//     sub-block's rows of S to LDS, waves 0 and 1 (one lane per sample
//     column, 64 columns each) run the recurrence
//       s_i = S_i + sum_{k in sub-block, k < i} L_ik y_k,
//       (y_i, d_i) = condition_step((a~_i - s_i)/L_ii, (b~_i - s_i)/L_ii, w_i)
//     with the sub-block's triangle of L from LDS, then every wave adds
//     L[later rows, sub-block] y_sub to its later rows' accumulators on MFMA,
//     so a row's dot product runs over its own sub-block only;
//   * y of the sub-block goes to the workgroup's Y scratch ([ld][128]).
// Eight waves give two per SIMD, as two four-wave workgroups would, but they
// share one copy of each L stage.
//
// Columns are dealt to the workgroups in contiguous ranges of whole
// 32-column slices, as evenly as the slice count allows.  A workgroup sweeps
// its range in full passes of four slices, then at most one pass of two and
// one of one slice; in those the waves of a slice split its rows, so all
// four SIMDs still share the MFMA work.
//
// Measured on one box: 7.79 s on the 65536-site field (70% of the FP64 MFMA
// peak) against 8.61 s for 128 x 128 blocks at two four-wave workgroups per
// CU, 1.09 s against 1.10 s on the 16384-site one; 128 x 256 blocks of eight
// waves (the factor read a quarter as often, Y as often as with 128-row
// blocks) took 9.74 s and 1.06 s.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "gemm_f64.h"
#include "launch.h"
#include "mvn_device.h"
#include "sweep_block.h"

namespace mvn {

constexpr int kWT = 512;                // threads per workgroup (8 waves)
constexpr int kWC = 128;                // sample columns of a full pass
constexpr int kWR = 256;                // rows per block
constexpr int kWSub = 32;               // rows per conditioning sub-block
constexpr int kWK = 16;                 // K per LDS stage
constexpr int kWALd = kWR + 1;          // LDS row stride of the L stage (doubles)
constexpr int kWBLd = kWC + 1;          // LDS row stride of the Y stage
constexpr int kWStage = kWK * kWALd + kWK * kWBLd;  // doubles per stage
constexpr int kWLds = 2 * kWStage;
static_assert(kWSub * kWC + kWSub * kWSub + (kWR - kWSub) * kWSub <= kWLds,
              "the sub-block buffers alias the GEMM stages");

int wide_sweep_cols() { return kWC; }
int wide_sweep_wg_per_cu() { return 1; }

// Columns of workgroup g of G: whole 32-column slices, contiguous.
__device__ __forceinline__ long wide_col_start(long g, long G, long NS) {
  const long slices = (NS + 31) / 32;
  const long c = (g * slices / G) * 32;
  return c < NS ? c : NS;
}

struct WideShared {
  double* lds;
  double* c_at;
  double* c_bt;
  double* c_rl;
  uint64_t* c_lat;
  const double* tab;
};

// One pass over `ncols` (<= 32 * NSL) columns starting at global column cb,
// NSL = 4, 2 or 1 slices of 32 columns: the 8 / NSL waves of a slice split
// its kWR block rows, wave w holding rows [RW (w % WPS), + RW) of slice
// w / WPS.
template <int NSL>
__device__ __forceinline__ void wide_pass(const WideShared& sh, const SweepArgs& p, double* __restrict__ Y, long cb,
                                          int ncols) {
  static_assert(NSL == 4 || NSL == 2 || NSL == 1, "slices per pass");
  constexpr int WPS = 8 / NSL;                   // waves per slice
  constexpr int RW = kWR / WPS;                  // rows per wave
  constexpr int NIB = RW / 16;
  constexpr int BC = 32 * NSL;                   // columns staged per K step
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int rw0 = RW * (w % WPS);                // first block row of this wave
  const int cw0 = 32 * (w / WPS);                // first pass column of this wave
  const bool wact = cw0 < ncols;                 // this wave's slice has columns
  const int n = p.n;
  const long ld = p.ld;
  const double* __restrict__ L = p.L;
  double* lds = sh.lds;
  double* T = lds;                               // kWSub x kWC: S, then y, of a sub-block
  double* Ltri = lds + kWSub * kWC;              // kWSub x kWSub: L of the sub-block (k < i), zero elsewhere
  double* Lcol = Ltri + kWSub * kWSub;           // rows below the sub-block x its kWSub columns
  // conditioning lanes: one lane per column, 64 columns per wave
  constexpr int kCondWaves = NSL == 4 ? 2 : 1;
  const int ccol = 64 * w + lane;
  const long gcol = cb + ccol;
  const bool cond = w < kCondWaves;
  const bool valid = cond && ccol < ncols;
  const uint64_t sidx = valid ? (uint64_t)(gcol / p.N) : 0;
  const uint64_t jpt = valid ? (uint64_t)(gcol % p.N) + 1 : 1;
  const auto ninv = [&sh](double x) { return ninv_lower_tab(x, sh.tab); };
  LogProd prod{1.0, 0};
  for (int i0 = 0; i0 < n; i0 += kWR) {
    const int rows = min(kWR, n - i0);
    f64x4 acc[NIB][2];
#pragma unroll
    for (int ib = 0; ib < NIB; ++ib)
#pragma unroll
      for (int jb = 0; jb < 2; ++jb) acc[ib][jb] = f64x4{0.0, 0.0, 0.0, 0.0};
    // ---- S = L[i0:i0+128, 0:i0] Y[0:i0, pass columns]
    if (i0 > 0) {
      const int nst = i0 / kWK;
      // lane t: A row t / 2, k (t % 2) * 8 .. + 8; B: k t / (BC / 8), columns
      // (t % (BC / 8)) * 8 .. + 8
      constexpr int kBLanes = BC / 8 * kWK;  // lanes that load B (256 of the 512 in a full pass)
      // (ld is a multiple of the block rows; the clamp only guards it)
      constexpr int kEA = kWR * kWK / kWT;  // A doubles per lane
      const double* pa = L + (long)min((long)(i0 + t / (kWK / kEA)), ld - 1) * ld + (t % (kWK / kEA)) * kEA;
      const double* pb = Y + (long)(t / (BC / 8)) * kWC + (t % (BC / 8)) * 8;
      double ra[kEA], rb[8];
      auto load = [&](int s) {
        const double2* a2 = reinterpret_cast<const double2*>(pa + (long)s * kWK);
#pragma unroll
        for (int q = 0; q < kEA / 2; ++q) {
          const double2 v = a2[q];
          ra[2 * q] = v.x;
          ra[2 * q + 1] = v.y;
        }
        if (t < kBLanes) {
          const double2* b2 = reinterpret_cast<const double2*>(pb + (long)s * kWK * kWC);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const double2 v = b2[q];
            rb[2 * q] = v.x;
            rb[2 * q + 1] = v.y;
          }
        }
      };
      auto store = [&](int buf) {
        double* As = lds + buf * kWStage;
        double* Bs = As + kWK * kWALd;
#pragma unroll
        for (int q = 0; q < kEA; ++q) As[((t % (kWK / kEA)) * kEA + q) * kWALd + t / (kWK / kEA)] = ra[q];
        if (t < kBLanes) {
          double* d = Bs + (t / (BC / 8)) * kWBLd + (t % (BC / 8)) * 8;
#pragma unroll
          for (int q = 0; q < 8; ++q) d[q] = rb[q];
        }
      };
      load(0);
      store(0);
      __syncthreads();
      for (int s = 0; s < nst; ++s) {
        const int buf = s & 1;
        if (s + 1 < nst) load(s + 1);
        if (wact) {
          const double* As = lds + buf * kWStage;
          const double* Bs = As + kWK * kWALd;
#pragma unroll
          for (int kk = 0; kk < kWK / 4; ++kk) {
            const int k = kk * 4 + (lane >> 4);
            double b[2];
#pragma unroll
            for (int jb = 0; jb < 2; ++jb) b[jb] = Bs[k * kWBLd + cw0 + jb * 16 + (lane & 15)];
#pragma unroll
            for (int ib = 0; ib < NIB; ++ib) {
              const double a = As[k * kWALd + rw0 + ib * 16 + (lane & 15)];
#pragma unroll
              for (int jb = 0; jb < 2; ++jb)
                acc[ib][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[jb], acc[ib][jb], 0, 0, 0);
            }
          }
        }
        if (s + 1 < nst) store(buf ^ 1);
        __syncthreads();
      }
    }
    if (t < rows) {
      const long g = i0 + t;
      sh.c_at[t] = p.at[g];
      sh.c_bt[t] = p.bt[g];
      sh.c_rl[t] = 1.0 / L[g * ld + g];
      sh.c_lat[t] = p.lattice[g];
    }
    // ---- conditioning, 32-row sub-blocks
#pragma unroll 1
    for (int q = 0; q < kWR / kWSub; ++q) {
      const int r0 = q * kWSub;
      if (r0 >= rows) break;  // uniform: rows is the same for every wave
      const int rq = min(kWSub, rows - r0);
      // this sub-block's rows of S -> T (from the waves whose rows hold them)
#pragma unroll
      for (int ib = 0; ib < NIB; ++ib) {
        const int gr = rw0 + 16 * ib;  // block row of local block ib
        if (gr >= r0 && gr < r0 + kWSub) {
#pragma unroll
          for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              T[(gr - r0 + (lane >> 4) + 4 * r) * kWC + cw0 + 16 * jb + (lane & 15)] = acc[ib][jb][r];
        }
      }
      // the sub-block's triangle of L and the rows below it, sub-block columns
      const double* Lq = L + (long)(i0 + r0) * ld + i0 + r0;
      for (int e = t; e < kWSub * kWSub; e += kWT) {
        const int ii = e / kWSub, k = e % kWSub;
        Ltri[e] = k < ii ? Lq[(long)ii * ld + k] : 0.0;
      }
      const int below = kWR - r0 - kWSub;
      for (int e = t; e < below * kWSub; e += kWT) {
        const int ii = e / kWSub, k = e % kWSub;
        Lcol[e] = i0 + r0 + kWSub + ii < ld ? Lq[(long)(kWSub + ii) * ld + k] : 0.0;
      }
      __syncthreads();
      if (cond) {
        for (int i = 0; i < rq; ++i) {
          const double* Li = Ltri + i * kWSub;
          const double* Tc = T + ccol;
          double s0 = Tc[i * kWC], s1 = 0.0, s2 = 0.0, s3 = 0.0;
          const int kend = (i + 3) & ~3;  // Ltri is zero from column i on
          for (int k = 0; k < kend; k += 4) {
            s0 += Li[k] * Tc[k * kWC];
            s1 += Li[k + 1] * Tc[(k + 1) * kWC];
            s2 += Li[k + 2] * Tc[(k + 2) * kWC];
            s3 += Li[k + 3] * Tc[(k + 3) * kWC];
          }
          const double sum = (s0 + s1) + (s2 + s3);
          const int ri = r0 + i;
          const double rl = sh.c_rl[ri];
          const double alpha = (sh.c_at[ri] - sum) * rl;
          const double beta = (sh.c_bt[ri] - sum) * rl;
          const uint64_t gi = (uint64_t)(i0 + ri);
          const double wq = richtmyer(jpt, sh.c_lat[ri], splitmix64(p.seed, sidx * (uint64_t)n + gi), p.periodize);
          const Step st = condition_step_with(alpha, beta, wq, 1.0 - wq, ninv);
          T[i * kWC + ccol] = valid ? st.y : 0.0;
          logprod_mul(prod, st);
        }
      }
      __syncthreads();
      // later rows += L[later rows, sub-block] y_sub (MFMA, K = 32)
      if (wact) {
#pragma unroll
        for (int ib = 0; ib < NIB; ++ib) {
          const int gr = rw0 + 16 * ib;
          if (gr >= r0 + kWSub) {
#pragma unroll
            for (int kk = 0; kk < kWSub / 4; ++kk) {
              const int k = 4 * kk + (lane >> 4);
              const double a = Lcol[(gr - r0 - kWSub + (lane & 15)) * kWSub + k];
#pragma unroll
              for (int jb = 0; jb < 2; ++jb)
                acc[ib][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, T[k * kWC + cw0 + 16 * jb + (lane & 15)],
                                                                  acc[ib][jb], 0, 0, 0);
            }
          }
        }
      }
      // y of the sub-block -> Y scratch rows i0 + r0 .. (the pass's columns)
      for (int e = t; e < kWSub * BC / 2; e += kWT) {
        const int r = e / (BC / 2), c2 = e % (BC / 2);
        reinterpret_cast<double2*>(Y + (long)(i0 + r0 + r) * kWC)[c2] = reinterpret_cast<const double2*>(T + r * kWC)[c2];
      }
      __syncthreads();
    }
  }
  if (valid) p.ell[gcol] = logprod_log(prod);
}

__global__ __launch_bounds__(kWT, 1) void wide_sweep_kernel(SweepArgs p) {
  __shared__ __attribute__((aligned(16))) double lds[kWLds];
  __shared__ double c_at[kWR], c_bt[kWR], c_rl[kWR];
  __shared__ uint64_t c_lat[kWR];
  __shared__ double ninv_tab[48];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  if (w == 1) {
#pragma unroll
    for (int e = 0; e < 48; ++e)
      if (lane == e) ninv_tab[e] = kAs241[e / 16][e % 16];
  }
  const WideShared sh{lds, c_at, c_bt, c_rl, c_lat, ninv_tab};
  const long NS = (long)p.N * p.S;
  double* __restrict__ Y = (double*)p.yscr + (long)blockIdx.x * p.yslice;
  const long cbeg = wide_col_start(blockIdx.x, gridDim.x, NS);
  const long cend = wide_col_start(blockIdx.x + 1, gridDim.x, NS);
  long cb = cbeg;
  for (; cend - cb > 96; cb += kWC) wide_pass<4>(sh, p, Y, cb, (int)min((long)kWC, cend - cb));
  if (cend - cb > 32) {
    wide_pass<2>(sh, p, Y, cb, (int)min(64L, cend - cb));
    cb += 64;
  }
  if (cb < cend) wide_pass<1>(sh, p, Y, cb, (int)(cend - cb));
}

hipError_t launch_wide_sweep(const SweepArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(wide_sweep_kernel, dim3(a.grid), dim3(kWT), 0, st, a);
  return hipGetLastError();
}

}  // namespace mvn
