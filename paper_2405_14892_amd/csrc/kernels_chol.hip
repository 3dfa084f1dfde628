// Covariance generation and dense tiled Cholesky, FP64 (arXiv 2405.14892,
// Algorithm 1: generate Sigma from the Matern kernel, then L <- dpotrf(Sigma)).
//
// The factorisation is right-looking over tiles of width `tile`.  Inside a
// tile column, sub-panels of 32 columns are finished left-looking:
//   chol_diag  - update the 32 x 32 diagonal block by the earlier sub-panels
//                of the same tile column, factor it in LDS (one workgroup);
//   chol_panel - update 128-row blocks below by the same sub-panels on FP64
//                MFMA and solve X L_dd^T = B (one lane per row);
// then chol_syrk subtracts the tile column's outer product from the trailing
// matrix with FP64 MFMA on 128 x 128 lower tiles (the bulk of the flops).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "gemm_f64.h"
#include "launch.h"
#include "sweep_gemm.h"

namespace mvn {

constexpr int kSub = 32;  // sub-panel width

// ------------------------------------------------------------ index arrays
// Device check of a caller's index array (a site permutation or the
// observed sites): every entry in [0, range), and with `seen` (range ints)
// no entry twice.  *flag = 1 on a bad entry; kernels that would index
// through the array read it only when *flag == 0.
__global__ __launch_bounds__(256) void index_clear_kernel(int* __restrict__ seen, long range, int* __restrict__ flag) {
  const long k = (long)blockIdx.x * 256 + threadIdx.x;
  if (k == 0) *flag = 0;
  if (seen && k < range) seen[k] = 0;
}

__global__ __launch_bounds__(256) void index_check_kernel(const int64_t* __restrict__ idx, long count, long range,
                                                          int* __restrict__ seen, int* __restrict__ flag) {
  const long k = (long)blockIdx.x * 256 + threadIdx.x;
  if (k >= count) return;
  const int64_t q = idx[k];
  if (q < 0 || q >= range) {
    atomicExch(flag, 1);
  } else if (seen && atomicExch(seen + q, 1) != 0) {
    atomicExch(flag, 1);
  }
}

hipError_t launch_index_check(const int64_t* idx, long count, long range, int* seen, int* flag, hipStream_t st) {
  const long c = count > range ? count : range;
  hipLaunchKernelGGL(index_clear_kernel, dim3((unsigned)((c + 255) / 256)), dim3(256), 0, st, seen, range, flag);
  if (count > 0)
    hipLaunchKernelGGL(index_check_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, idx, count, range,
                       seen, flag);
  return hipGetLastError();
}

// ------------------------------------------------------------ covariance
// perm_bad (with perm): the permutation check's flag; when set the matrix
// is the identity and *info = -1.
__global__ __launch_bounds__(256) void build_matrix_kernel(int n, int ld, const double* __restrict__ sigma,
                                                           int lds, const int64_t* __restrict__ perm,
                                                           const int* __restrict__ perm_bad,
                                                           const double* __restrict__ locs, Matern mk,
                                                           double* __restrict__ A, int* __restrict__ info) {
  const bool bad = perm && perm_bad && *perm_bad != 0;
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *info = bad ? -1 : 0;
  const long i = (long)blockIdx.y * 16 + (threadIdx.x >> 4);
  const long j = (long)blockIdx.x * 16 + (threadIdx.x & 15);
  if (i >= ld || j > i) return;
  double v;
  if (i >= n || j >= n || bad) {
    v = (i == j) ? 1.0 : 0.0;
  } else if (sigma) {
    const long pi = perm ? perm[i] : i, pj = perm ? perm[j] : j;
    v = pi >= pj ? sigma[pi * lds + pj] : sigma[pj * lds + pi];
  } else {
    const double dx = locs[2 * i] - locs[2 * j];
    const double dy = locs[2 * i + 1] - locs[2 * j + 1];
    v = matern_cov(mk, sqrt(dx * dx + dy * dy));
    if (i == j) v += mk.nugget;
  }
  A[i * ld + j] = v;
}

__global__ __launch_bounds__(256) void clear_u64_kernel(unsigned long long* __restrict__ p, long n) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

hipError_t launch_clear_u64(unsigned long long* p, long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(clear_u64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_build_matrix(int n, int ld, const double* sigma, int lds, const int64_t* perm, const int* perm_bad,
                               const double* locs, const Matern& mk, double* A, int* info, hipStream_t st) {
  dim3 grid(ld / 16, ld / 16);
  hipLaunchKernelGGL(build_matrix_kernel, grid, dim3(256), 0, st, n, ld, sigma, lds, perm, perm_bad, locs, mk, A,
                     info);
  return hipGetLastError();
}

// ------------------------------------------------------------ diagonal block
// Factor the jw x jw diagonal block D = A[j0:j0+jw, j0:j0+jw] in place.  The
// block already holds the updates of every column left of j0: those of
// earlier tile columns from the trailing updates, those of earlier
// sub-panels of its own tile column from their panel solves.  One wave: lane
// r < jw keeps row r of D in registers and column c is finished by the Crout
// step
//   s_r = D[r][c] - sum_{k<c} L[r][k] L[c][k],   L[c][c] = sqrt(s_c),
//   L[r][c] = s_r / L[c][c]  (r > c),
// row c of L being broadcast from lane c with v_readlane.
__device__ __forceinline__ double lane_bcast(double v, int l) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Crout factorisation of the block whose lower rows lane r < jw holds in x
// (rows and columns past jw must be those of the identity, so that all 32
// columns run: no early exit keeps the row in registers).  Returns the
// 1-based index in the block of the first column whose pivot is not
// positive, or 0.
__device__ __forceinline__ int crout32(double (&x)[kSub], int jw) {
  const int r = threadIdx.x & 63;
  int fail = 0;
#pragma unroll
  for (int c = 0; c < kSub; ++c) {
    double s = x[c];
#pragma unroll
    for (int k = 0; k < c; ++k) s -= x[k] * lane_bcast(x[k], c);
    const double piv = lane_bcast(s, c);  // uniform across the wave
    if (fail == 0 && c < jw && !(piv > 0.0)) fail = c + 1;
    const double d = sqrt(piv);
    x[c] = r == c ? d : (r > c ? s / d : 0.0);
  }
  return fail;
}

__device__ __forceinline__ void chol_diag_body(double* __restrict__ A, int ld, int j0, int jw,
                                               int* __restrict__ info) {
  if (*info != 0) return;
  const int r = threadIdx.x & 63;
  const bool live = r < jw;
  double x[kSub];
#pragma unroll
  for (int c = 0; c < kSub; ++c)
    x[c] = (live && c <= r) ? A[(long)(j0 + r) * ld + j0 + c] : (c == r ? 1.0 : 0.0);
  int fail = crout32(x, jw);
  if (fail) fail += j0;
  if (fail) {
    if (r == 0) atomicCAS(info, 0, fail);
    return;
  }
  if (live) {
#pragma unroll
    for (int c = 0; c < kSub; ++c)
      if (c <= r) A[(long)(j0 + r) * ld + j0 + c] = x[c];
  }
}

// One wave.
__global__ __launch_bounds__(64) void chol_diag_kernel(double* __restrict__ A, int ld, int j0, int jw,
                                                       int* __restrict__ info) {
  chol_diag_body(A, ld, j0, jw, info);
}

// ------------------------------------------------------------ panel solve
// Rows i >= j0 + jw, 128 per workgroup: the update
// X = A[i, j0:j0+jw] - A[i, k0:j0] A[j0:j0+jw, k0:j0]^T on FP64 MFMA (four
// waves of 32 rows x 32 columns, K staged 32 deep in LDS, double-buffered),
// then the forward substitution x <- x L_dd^{-T} one lane per row.
// Afterwards the finished columns update the diagonal blocks of the later
// sub-panels of the tile column (rows and columns [q0, q0 + 32), q0 < kend)
// that lie in this workgroup's rows, D_q -= X_q X_q^T, one wave per block on
// FP64 MFMA.  The block right after this sub-panel then holds all its
// updates, and the wave that updated it (wave 0 of row block 0) also factors
// it, so only the first diagonal block of a tile column needs a launch of
// its own.
// FULL: jw == 32 (every sub-panel except the last of a tile whose width is
// not a multiple of 32, which has no later diagonal block); the constant
// bound keeps the substitution in registers.
// PK: k per LDS stage of the panel update.  16 keeps the workgroup at 50 KB of
// LDS (three per CU, and room beside the trailing-update workgroups of the
// lookahead) where 32 took 91 KB; the k order of the products is the same,
// so the factor is too, bit for bit.  Measured: 48.5 -> 47.0 ms at 16 384
// sites (tile 512), 1614 -> 1572 ms at 65 536 (tile 1024), and 35 ms less
// per 2000-problem batch.
constexpr int kPanelK = 16;

template <bool FULL, int PK = kPanelK>
__device__ __forceinline__ void chol_panel_body(double* __restrict__ A, int ld, int k0, int j0, int jw_arg,
                                                int kend, int* __restrict__ info, int rblock) {
  if (*info != 0) return;
  const int jw = FULL ? kSub : jw_arg;
  constexpr int kALd = kTile + 1, kBLd = kSub + 1;
  constexpr int kAS = PK * kALd, kBS = PK * kBLd;
  static_assert(kTile * (kSub + 1) <= 2 * (kAS + kBS), "X must fit in the stage buffers");
  __shared__ double stage[2 * (kAS + kBS)];
  __shared__ double D[kSub][kSub + 1];
  double (*X)[kSub + 1] = reinterpret_cast<double (*)[kSub + 1]>(stage);  // after the K loop
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const long r0 = (long)j0 + jw + (long)rblock * kTile;
  const int K = j0 - k0;  // a multiple of 32
  f64x4 acc[2][2];
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) acc[ib][jb] = f64x4{0.0, 0.0, 0.0, 0.0};
  if (K > 0) {
    // lane t: A row r0 + t/2, PK/2 consecutive k (rows at or past ld read as
    // zero); B row t/8 of the diagonal block, PK/8 consecutive k (masked at jw)
    constexpr int kQA = PK / 2, kQB = PK / 8;
    double ra[kQA], rb[kQB];
    const long arow = r0 + (t >> 1);
    const int brow = t >> 3;
    auto load = [&](int kk) {
      const long kb = (long)k0 + kk + (t & 1) * kQA;
#pragma unroll
      for (int q = 0; q < kQA; ++q) ra[q] = arow < ld ? A[arow * ld + kb + q] : 0.0;
      const long kc = (long)k0 + kk + (t & 7) * kQB;
#pragma unroll
      for (int q = 0; q < kQB; ++q) rb[q] = brow < jw ? A[(long)(j0 + brow) * ld + kc + q] : 0.0;
    };
    auto store = [&](double* s) {
      const int row = t >> 1, kb = (t & 1) * kQA;
#pragma unroll
      for (int q = 0; q < kQA; ++q) s[(kb + q) * kALd + row] = ra[q];
      double* sb = s + kAS;
      const int kc = (t & 7) * kQB;
#pragma unroll
      for (int q = 0; q < kQB; ++q) sb[(kc + q) * kBLd + brow] = rb[q];
    };
    const int nst = K / PK;
    load(0);
    store(stage);
    __syncthreads();
    for (int s = 0; s < nst; ++s) {
      double* cur = stage + (s & 1) * (kAS + kBS);
      double* nxt = stage + ((s + 1) & 1) * (kAS + kBS);
      if (s + 1 < nst) load((s + 1) * PK);
      const double* As = cur;
      const double* Bs = cur + kAS;
#pragma unroll
      for (int kk = 0; kk < PK / 4; ++kk) {
        const int k = kk * 4 + (lane >> 4);
        double a[2], b[2];
#pragma unroll
        for (int ib = 0; ib < 2; ++ib) a[ib] = As[k * kALd + w * 32 + ib * 16 + (lane & 15)];
#pragma unroll
        for (int jb = 0; jb < 2; ++jb) b[jb] = Bs[k * kBLd + jb * 16 + (lane & 15)];
#pragma unroll
        for (int ib = 0; ib < 2; ++ib)
#pragma unroll
          for (int jb = 0; jb < 2; ++jb)
            acc[ib][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ib], b[jb], acc[ib][jb], 0, 0, 0);
      }
      if (s + 1 < nst) store(nxt);
      __syncthreads();
    }
  }
  // X = A[rows, j0:j0+jw] - update (accumulator D[l/16 + 4r][l%16] layout)
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = w * 32 + ib * 16 + (lane >> 4) + 4 * r, c = jb * 16 + (lane & 15);
        const long gi = r0 + row;
        X[row][c] = (gi < ld && c < jw) ? A[gi * ld + j0 + c] - acc[ib][jb][r] : 0.0;
      }
  for (int e = t; e < kSub * kSub; e += 256) {
    const int r = e >> 5, c = e & 31;
    D[r][c] = (r < jw && c <= r) ? A[(long)(j0 + r) * ld + j0 + c] : (r == c ? 1.0 : 0.0);
  }
  __syncthreads();
  // forward substitution over all 32 columns: past jw, X is zero and D the
  // identity, so those columns stay zero and the others are unaffected
  if (t < kTile) {
    double x[kSub];
#pragma unroll
    for (int c = 0; c < kSub; ++c) x[c] = X[t][c];
#pragma unroll
    for (int c = 0; c < kSub; ++c) {
      double v = x[c];
#pragma unroll
      for (int cp = 0; cp < c; ++cp) v -= x[cp] * D[c][cp];
      x[c] = v / D[c][c];
    }
#pragma unroll
    for (int c = 0; c < kSub; ++c) X[t][c] = x[c];
  }
  __syncthreads();
  for (int e = t; e < kTile * kSub; e += 256) {
    const int row = e >> 5, c = e & 31;
    const long gi = r0 + row;
    if (gi < ld && c < jw) A[gi * ld + j0 + c] = X[row][c];
  }
  if (FULL) {
    // the diagonal blocks after j0 + 32 start 32 rows apart, so wave w takes
    // the one at local row 32 w
    const long q0 = r0 + 32 * w;
    if (q0 < kend) {
      const int hq = (int)min((long)kSub, kend - q0);
      const int lr = 32 * w;
      f64x4 dq[3];  // tiles (0, 0), (1, 0), (1, 1)
#pragma unroll
      for (int i = 0; i < 3; ++i) dq[i] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < kSub / 4; ++kk) {
        const int k = kk * 4 + (lane >> 4);
        const double a0 = X[lr + (lane & 15)][k], a1 = X[lr + 16 + (lane & 15)][k];
        dq[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, a0, dq[0], 0, 0, 0);
        dq[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, a0, dq[1], 0, 0, 0);
        dq[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, a1, dq[2], 0, 0, 0);
      }
      if (rblock == 0 && w == 0) {
        // the next diagonal block: updated rows to LDS (D is free after the
        // substitution), one row per lane, factored in registers
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const int ib = i > 0, jb = i > 1;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = ib * 16 + (lane >> 4) + 4 * r, col = jb * 16 + (lane & 15);
            if (row < hq && col <= row) D[row][col] = A[(q0 + row) * ld + q0 + col] - dq[i][r];
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        const int rr = lane;
        double x[kSub];
#pragma unroll
        for (int c = 0; c < kSub; ++c) x[c] = (rr < hq && c <= rr) ? D[rr & 31][c] : (c == rr ? 1.0 : 0.0);
        const int fail = crout32(x, hq);
        if (fail) {
          if (lane == 0) atomicCAS(info, 0, (int)q0 + fail);
        } else if (rr < hq) {
#pragma unroll
          for (int c = 0; c < kSub; ++c)
            if (c <= rr) A[(q0 + rr) * ld + q0 + c] = x[c];
        }
      } else {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const int ib = i > 0, jb = i > 1;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = ib * 16 + (lane >> 4) + 4 * r, col = jb * 16 + (lane & 15);
            if (row < hq && col <= row) A[(q0 + row) * ld + q0 + col] -= dq[i][r];
          }
        }
      }
    }
  }
}

template <bool FULL>
__global__ __launch_bounds__(256) void chol_panel_kernel(double* __restrict__ A, int ld, int k0, int j0, int jw,
                                                         int kend, int* __restrict__ info) {
  chol_panel_body<FULL>(A, ld, k0, j0, jw, kend, info, blockIdx.x);
}

// ------------------------------------------------------------ trailing update
// K stages of 8, double-buffered in LDS (2 x 2 x 8 x 129 doubles = 33 KB, so
// that a panel solve still fits on a CU beside two of these workgroups),
// global loads issued two stages ahead of their use.
constexpr int kSyrkK = 8;
constexpr int kSyrkStage = kSyrkK * kLdsLd;  // doubles, one operand

// Lane t: 4 consecutive k of row t / 2 (zero past ld or klim with MASK).
template <bool MASK>
__device__ __forceinline__ void syrk_load(const double* __restrict__ A, long ld, long row0, long k0, long klim,
                                          double (&r)[4]) {
  const int t = threadIdx.x;
  const long row = row0 + (t >> 1), kb = k0 + (t & 1) * 4;
  const double* p = A + row * ld + kb;
  if (!MASK) {
    const double2 v0 = reinterpret_cast<const double2*>(p)[0], v1 = reinterpret_cast<const double2*>(p)[1];
    r[0] = v0.x;
    r[1] = v0.y;
    r[2] = v1.x;
    r[3] = v1.y;
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) r[q] = (row < ld && kb + q < klim) ? p[q] : 0.0;
  }
}

__device__ __forceinline__ void syrk_store(double* __restrict__ lds, const double (&r)[4]) {
  const int t = threadIdx.x, row = t >> 1, kb = (t & 1) * 4;
#pragma unroll
  for (int q = 0; q < 4; ++q) lds[(kb + q) * kLdsLd + row] = r[q];
}

__device__ __forceinline__ void syrk_mma(const double* __restrict__ As, const double* __restrict__ Bs, Acc& acc) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = w >> 1, wc = w & 1;
#pragma unroll
  for (int kk = 0; kk < kSyrkK / 4; ++kk) {
    const int krow = (kk * 4 + (lane >> 4)) * kLdsLd;
    double a[4], b[4];
#pragma unroll
    for (int ib = 0; ib < 4; ++ib) a[ib] = As[krow + wr * 64 + ib * 16 + (lane & 15)];
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) b[jb] = Bs[krow + wc * 64 + jb * 16 + (lane & 15)];
#pragma unroll
    for (int ib = 0; ib < 4; ++ib)
#pragma unroll
      for (int jb = 0; jb < 4; ++jb)
        acc.v[ib][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ib], b[jb], acc.v[ib][jb], 0, 0, 0);
  }
}

// One 128 x 128 lower tile of C = A[rowA:, rowB:] -= P P^T with
// P = A[:, k0:k0+kw]; only elements with column < clim and column <= row
// are written.
template <bool MASK>
__device__ __forceinline__ void chol_syrk_body(double* __restrict__ A, int ld, int k0, int kw,
                                               const int* __restrict__ info, long rowA, long rowB, long clim) {
  if (*info != 0) return;
  __shared__ double lds[2 * 2 * kSyrkStage];
  Acc acc;
  acc_zero(acc);
  const long klim = (long)k0 + kw;
  const int nst = (kw + kSyrkK - 1) / kSyrkK;
  // stage s lives in register set s & 1 until it is stored to LDS buffer s & 1
  double ra0[4], rb0[4], ra1[4], rb1[4];
  syrk_load<MASK>(A, ld, rowA, k0, klim, ra0);
  syrk_load<MASK>(A, ld, rowB, k0, klim, rb0);
  if (nst > 1) {
    syrk_load<MASK>(A, ld, rowA, (long)k0 + kSyrkK, klim, ra1);
    syrk_load<MASK>(A, ld, rowB, (long)k0 + kSyrkK, klim, rb1);
  }
  syrk_store(lds, ra0);
  syrk_store(lds + kSyrkStage, rb0);
  if (nst > 2) {
    syrk_load<MASK>(A, ld, rowA, (long)k0 + 2 * kSyrkK, klim, ra0);
    syrk_load<MASK>(A, ld, rowB, (long)k0 + 2 * kSyrkK, klim, rb0);
  }
  __syncthreads();
  // step s: MFMAs of stage s, then stage s + 1 (register set (s + 1) & 1) to
  // the other LDS buffer and stage s + 3 loaded into the set just freed
  auto step = [&](int s, double (&ra)[4], double (&rb)[4]) {
    const double* cur = lds + (s & 1) * 2 * kSyrkStage;
    double* nxt = lds + ((s + 1) & 1) * 2 * kSyrkStage;
    syrk_mma(cur, cur + kSyrkStage, acc);
    if (s + 1 < nst) {
      syrk_store(nxt, ra);
      syrk_store(nxt + kSyrkStage, rb);
      if (s + 3 < nst) {
        syrk_load<MASK>(A, ld, rowA, (long)k0 + (long)(s + 3) * kSyrkK, klim, ra);
        syrk_load<MASK>(A, ld, rowB, (long)k0 + (long)(s + 3) * kSyrkK, klim, rb);
      }
    }
    __syncthreads();
  };
  for (int s = 0; s < nst; s += 2) {
    step(s, ra1, rb1);
    if (s + 1 < nst) step(s + 1, ra0, rb0);
  }
#pragma unroll
  for (int ib = 0; ib < 4; ++ib)
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long gi = rowA + acc_row(ib, r), gj = rowB + acc_col(jb);
        if (gi < ld && gj < clim && gj <= gi) A[gi * ld + gj] -= acc.v[ib][jb][r];
      }
}

// (ti, tj), tj <= ti, of lower tile b in row-major order of the triangle.
__device__ __forceinline__ void tri_tile(long b, long& ti, long& tj) {
  ti = (long)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= b) ++ti;
  while (ti * (ti + 1) / 2 > b) --ti;
  tj = b - ti * (ti + 1) / 2;
}

// The lower triangle of tiles of A[r0:, r0:].  MASK = false when every
// 128 x 8 operand tile lies inside the matrix: the tile width is a multiple
// of 128 (so are ld, r0, k0 + kw and kw).
template <bool MASK>
__global__ __launch_bounds__(256, 2) void chol_syrk_kernel(double* __restrict__ A, int ld, int k0, int kw, int r0,
                                                           const int* __restrict__ info) {
  long ti, tj;
  tri_tile(blockIdx.x, ti, tj);
  chol_syrk_body<MASK>(A, ld, k0, kw, info, r0 + ti * kTile, r0 + tj * kTile, ld);
}

// Tile column [c1, c2) of the trailing matrix, c1 = k0 + kw: tile (blockIdx.y,
// blockIdx.x) of A[c1:, c1:c2].
template <bool MASK>
__global__ __launch_bounds__(256, 2) void chol_syrk_col_kernel(double* __restrict__ A, int ld, int k0, int kw,
                                                               int c2, const int* __restrict__ info) {
  if (blockIdx.x > blockIdx.y) return;
  const long c1 = (long)k0 + kw;
  chol_syrk_body<MASK>(A, ld, k0, kw, info, c1 + (long)blockIdx.y * kTile, c1 + (long)blockIdx.x * kTile, c2);
}

__global__ __launch_bounds__(256) void zero_upper_kernel(double* __restrict__ A, int ld) {
  const long i = (long)blockIdx.y * 16 + (threadIdx.x >> 4);
  const long j = (long)blockIdx.x * 16 + (threadIdx.x & 15);
  if (i < ld && j < ld && j > i) A[i * ld + j] = 0.0;
}

SideStream* side_stream(int slot, hipStream_t st) {
  constexpr int kMaxDevices = 64;
  static std::mutex table_mu;
  static SideStream* table[kMaxDevices][kSideSlots] = {};
  static bool failed[kMaxDevices][kSideSlots] = {};
  int dev = 0;
  if (slot < 0 || slot >= kSideSlots || hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return nullptr;
  // a call being captured into a graph runs on the caller's stream alone
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return nullptr;
  std::lock_guard<std::mutex> g(table_mu);
  if (table[dev][slot] || failed[dev][slot]) return table[dev][slot];
  SideStream* sd = new SideStream();
  bool ok = hipStreamCreateWithFlags(&sd->s, hipStreamNonBlocking) == hipSuccess;
  for (int i = 0; ok && i < 3; ++i) ok = hipEventCreateWithFlags(&sd->ev[i], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    failed[dev][slot] = true;
    return nullptr;  // sd and whatever it holds stay allocated: a failure here is not retried
  }
  table[dev][slot] = sd;
  return sd;
}

// The sub-panel chain of tile column [k0, k0 + kw): factor its first 32 x 32
// diagonal block, then per sub-panel solve (and update) the rows below it;
// each panel solve also factors the next diagonal block.
static void chol_column(int ld, int k0, int kw, double* A, int* info, hipStream_t st) {
  const int kend = k0 + kw;
  hipLaunchKernelGGL(chol_diag_kernel, dim3(1), dim3(64), 0, st, A, ld, k0, min(kSub, kw), info);
  for (int j0 = k0; j0 < kend; j0 += kSub) {
    const int jw = min(kSub, kend - j0);
    const int rows = ld - (j0 + jw);  // zero only for the last sub-panel of the matrix
    if (rows > 0) {
      const dim3 pg((rows + kTile - 1) / kTile);
      if (jw == kSub)
        hipLaunchKernelGGL(chol_panel_kernel<true>, pg, dim3(256), 0, st, A, ld, k0, j0, jw, kend, info);
      else
        hipLaunchKernelGGL(chol_panel_kernel<false>, pg, dim3(256), 0, st, A, ld, k0, j0, jw, kend, info);
    }
  }
}

// Right-looking over tile columns.  With a side stream (lookahead), the
// trailing update of tile column k is split: the part that falls on tile
// column k + 1 runs on the caller's stream, which then goes on with that
// column's sub-panel chain, while the rest of the trailing matrix is updated
// on the side stream:
//   st:   chain(k)  [evP]  wait evR(k-1)  next(k)  chain(k+1) ...
//   side:                  wait evP  rest(k)  [evR(k)] ...
// next(k) waits for rest(k-1), which also writes tile column k + 1; the
// regions written concurrently are disjoint column ranges.
struct NoPost {
  void operator()(int, int, hipStream_t) const {}
};

// post(k0, kw, st) runs on the caller's stream after each tile column's
// sub-panel chain, before any of that column's trailing updates.
template <class Next, class Rest, class Post = NoPost>
static hipError_t right_looking(int ld, int tile, double* A, int* info, hipStream_t st, SideStream* sd,
                                Next next, Rest rest, int kstop = 0, Post post = Post()) {
  bool pending = false, used = false;  // a rest() on the side stream not yet waited for; any
  // on an error, let the side stream drain before returning, so that none of
  // its kernels still writes A once the caller sees the failure
  auto fail = [&](hipError_t e) {
    if (used) (void)hipStreamSynchronize(sd->s);
    return e;
  };
  const int kend = kstop > 0 ? kstop : ld;
  for (int k0 = 0; k0 < kend; k0 += tile) {
    const int kw = min(tile, ld - k0);
    chol_column(ld, k0, kw, A, info, st);
    post(k0, kw, st);
    const int c1 = k0 + kw;
    if (c1 < ld) {
      if (!sd) {
        rest(k0, kw, c1, st);
      } else {
        const int c2 = min(c1 + tile, ld);
        hipError_t e = hipEventRecord(sd->ev[0], st);
        if (e == hipSuccess && pending) e = hipStreamWaitEvent(st, sd->ev[1], 0);
        if (e != hipSuccess) return fail(e);
        pending = false;
        next(k0, kw, c2, st);
        if (c2 < ld) {
          used = true;
          e = hipStreamWaitEvent(sd->s, sd->ev[0], 0);
          if (e != hipSuccess) return fail(e);
          rest(k0, kw, c2, sd->s);
          e = hipEventRecord(sd->ev[1], sd->s);
          if (e != hipSuccess) return fail(e);
          pending = true;
        }
      }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(e);
  }
  if (used) {
    hipError_t e = hipEventRecord(sd->ev[2], sd->s);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, sd->ev[2], 0);
    if (e != hipSuccess) return fail(e);
  }
  return hipGetLastError();
}

hipError_t launch_cholesky_f64(int ld, int tile, double* A, int* info, hipStream_t st, bool lookahead, int kstop) {
  SideStream* sd = (lookahead && ld > 2 * tile) ? side_stream(kSideCholesky, st) : nullptr;
  std::unique_lock<std::mutex> lock;
  if (sd) lock = std::unique_lock<std::mutex>(sd->mu);
  const bool mask = tile % kTile != 0;
  auto next = [&](int k0, int kw, int c2, hipStream_t s) {
    const long c1 = (long)k0 + kw;
    const dim3 grid((unsigned)((c2 - c1 + kTile - 1) / kTile), (unsigned)((ld - c1 + kTile - 1) / kTile));
    if (mask) hipLaunchKernelGGL(chol_syrk_col_kernel<true>, grid, dim3(256), 0, s, A, ld, k0, kw, c2, (const int*)info);
    else hipLaunchKernelGGL(chol_syrk_col_kernel<false>, grid, dim3(256), 0, s, A, ld, k0, kw, c2, (const int*)info);
  };
  auto rest = [&](int k0, int kw, int r0, hipStream_t s) {
    const long nt = (ld - r0 + kTile - 1) / kTile;
    const dim3 grid((unsigned)(nt * (nt + 1) / 2));
    if (mask) hipLaunchKernelGGL(chol_syrk_kernel<true>, grid, dim3(256), 0, s, A, ld, k0, kw, r0, (const int*)info);
    else hipLaunchKernelGGL(chol_syrk_kernel<false>, grid, dim3(256), 0, s, A, ld, k0, kw, r0, (const int*)info);
  };
  hipError_t e = right_looking(ld, tile, A, info, st, sd, next, rest, kstop);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(zero_upper_kernel, dim3(ld / 16, ld / 16), dim3(256), 0, st, A, ld);
  return hipGetLastError();
}

// ------------------------------------------------------------ mixed precision
// Trailing update C -= P P^T with the products in FP32 or BF16 on MFMA and
// FP32 accumulation (C stays FP64).  128 x 64 tiles of C on the sweep's GEMM
// policies; P (FP64) is converted while it is staged into LDS.
template <class G>
struct SyrkStage;

template <>
struct SyrkStage<GemmF32> {
  using G = GemmF32;
  struct Regs { double a[16]; double b[8]; };
  static __device__ __forceinline__ void load(const double* A, long ld, long ra0, long rb0, long k0,
                                              long klim, Regs& r) {
    const int t = threadIdx.x;
    const long row = ra0 + (t >> 1), kb = k0 + (t & 1) * 16;
#pragma unroll
    for (int q = 0; q < 16; ++q) r.a[q] = (row < ld && kb + q < klim) ? A[row * ld + kb + q] : 0.0;
    const long cr = rb0 + (t >> 2), kc = k0 + (t & 3) * 8;
#pragma unroll
    for (int q = 0; q < 8; ++q) r.b[q] = (cr < ld && kc + q < klim) ? A[cr * ld + kc + q] : 0.0;
  }
  static __device__ __forceinline__ void store(void* stage, const Regs& r) {
    float* As = (float*)stage;
    float* Bs = As + G::kAStage;
    const int t = threadIdx.x;
    const int row = t >> 1, kb = (t & 1) * 16;
#pragma unroll
    for (int q = 0; q < 16; ++q) As[(kb + q) * G::kALd + row] = (float)r.a[q];
    const int c = t >> 2, kc = (t & 3) * 8;
#pragma unroll
    for (int q = 0; q < 8; ++q) Bs[(kc + q) * G::kBLd + c] = (float)r.b[q];
  }
};

template <int SPLIT>
struct SyrkStage<GemmBF16T<SPLIT, 128>> {
  using G = GemmBF16T<SPLIT, 128>;
  static constexpr int kAH = G::kK / 2, kBQ = G::kK / 4;
  struct Regs { double a[kAH]; double b[kBQ]; };
  static __device__ __forceinline__ void load(const double* A, long ld, long ra0, long rb0, long k0,
                                              long klim, Regs& r) {
    const int t = threadIdx.x;
    const long row = ra0 + (t >> 1), kb = k0 + (t & 1) * kAH;
#pragma unroll
    for (int q = 0; q < kAH; ++q) r.a[q] = (row < ld && kb + q < klim) ? A[row * ld + kb + q] : 0.0;
    const long cr = rb0 + (t >> 2), kc = k0 + (t & 3) * kBQ;
#pragma unroll
    for (int q = 0; q < kBQ; ++q) r.b[q] = (cr < ld && kc + q < klim) ? A[cr * ld + kc + q] : 0.0;
  }
  static __device__ __forceinline__ void store(void* stage, const Regs& r) {
    __bf16* As = (__bf16*)stage;
    __bf16* Bs = As + G::kAStage;
    const int t = threadIdx.x;
    __bf16* da = As + (t >> 1) * G::kALd + (t & 1) * kAH;
#pragma unroll
    for (int q = 0; q < kAH; ++q) {
      const __bf16 hi = to_bf16(r.a[q]);
      da[q] = hi;
      if (SPLIT == 2) da[G::kAPlane + q] = to_bf16(r.a[q] - (double)(float)hi);
    }
    __bf16* db = Bs + (t >> 2) * G::kBLd + (t & 3) * kBQ;
#pragma unroll
    for (int q = 0; q < kBQ; ++q) {
      const __bf16 hi = to_bf16(r.b[q]);
      db[q] = hi;
      if (SPLIT == 2) db[G::kBPlane + q] = to_bf16(r.b[q] - (double)(float)hi);
    }
  }
};

// FP64 operands on the sweep's FP64 policy (the precise path of the
// adaptive map): A rows 8 consecutive k per lane, B rows 4.
template <>
struct SyrkStage<GemmF64T<128>> {
  using G = GemmF64T<128>;
  struct Regs { double a[8]; double b[4]; };
  static __device__ __forceinline__ void load(const double* A, long ld, long ra0, long rb0, long k0,
                                              long klim, Regs& r) {
    const int t = threadIdx.x;
    const long row = ra0 + (t >> 1), kb = k0 + (t & 1) * 8;
#pragma unroll
    for (int q = 0; q < 8; ++q) r.a[q] = (row < ld && kb + q < klim) ? A[row * ld + kb + q] : 0.0;
    const long cr = rb0 + (t >> 2), kc = k0 + (t & 3) * 4;
#pragma unroll
    for (int q = 0; q < 4; ++q) r.b[q] = (cr < ld && kc + q < klim) ? A[cr * ld + kc + q] : 0.0;
  }
  static __device__ __forceinline__ void store(void* stage, const Regs& r) {
    double* As = (double*)stage;
    double* Bs = As + G::kAStage;
    const int t = threadIdx.x;
    const int row = t >> 1, kb = (t & 1) * 8;
#pragma unroll
    for (int q = 0; q < 8; ++q) As[(kb + q) * G::kALd + row] = r.a[q];
    const int c = t >> 2, kc = (t & 3) * 4;
#pragma unroll
    for (int q = 0; q < 4; ++q) Bs[(kc + q) * G::kBLd + c] = r.b[q];
  }
};

// One 128 x 64 tile of C = A[rowA:, colB:] -= P P^T in policy G's
// arithmetic, P = A[:, k0:k0+kw]; only elements with column < clim and
// column <= row are written.  The caller has checked info and that the tile
// reaches the lower triangle.
template <class G>
__device__ __forceinline__ void syrk_lp_tile(double* __restrict__ A, double* lds, int ld, int k0, int kw,
                                             long rowA, long colB, long clim) {
  typename G::Acc acc;
  G::zero(acc);
  const long klim = (long)k0 + kw;
  const int nst = (kw + G::kK - 1) / G::kK;
  char* st0 = (char*)lds;
  char* st1 = (char*)lds + G::kStageBytes;
  typename SyrkStage<G>::Regs r;
  SyrkStage<G>::load(A, ld, rowA, colB, k0, klim, r);
  SyrkStage<G>::store(st0, r);
  __syncthreads();
  for (int s = 0; s < nst; ++s) {
    const bool odd = s & 1;
    if (s + 1 < nst) SyrkStage<G>::load(A, ld, rowA, colB, (long)k0 + (long)(s + 1) * G::kK, klim, r);
    G::mma(odd ? st1 : st0, acc);
    if (s + 1 < nst) SyrkStage<G>::store(odd ? st0 : st1, r);
    __syncthreads();
  }
  G::to_block(acc, lds);
  __syncthreads();
  for (int e = threadIdx.x; e < kTile * kCols; e += 256) {
    const long gi = rowA + e / kCols, gj = colB + e % kCols;
    if (gi < ld && gj < clim && gj <= gi) A[gi * ld + gj] -= lds[e];
  }
}

// Tile-wise precision map of the trailing updates (adaptive mode).  The
// update of tile (i, j) by tile column k subtracts L_ik L_jk^T; rounding its
// operands to a type with unit roundoff u (and accumulating K products in
// FP32) perturbs it by at most about u_K ||L_ik||_F ||L_jk||_F, u_K = u +
// K 2^-24.  A tile runs in the reduced type when that bound is at most
// tol * max_i Sigma_ii, else in FP32 when FP32's bound is, else in FP64;
// near-diagonal tiles, whose panel blocks carry most of the factor's mass,
// therefore stay precise and far tiles with small panel norms do not.
// norms[b] = ||L[r0 + 128 b : r0 + 128 (b + 1), k0 : k0 + kw]||_F for the
// step's rows r0 = k0 + kw (a 64-row B block lies inside one of them).
struct PrecMap {
  const double* norms;        // nullptr: uniform precision (policy G everywhere)
  const double* dmax;         // max diagonal of Sigma (device)
  unsigned long long* counts; // tile updates per path: [0] FP64, [1] FP32, [2] reduced type
  long r0;
  double tol, u_low, u_f32;
};

template <class G>
__device__ __forceinline__ void chol_syrk_lp_body(double* __restrict__ A, int ld, int k0, int kw,
                                                  const int* __restrict__ info, long rowA, long colB, long clim,
                                                  const PrecMap& pm) {
  if (*info != 0) return;
  __shared__ __attribute__((aligned(16))) double lds[kTile * kCols];
  if (colB > rowA + kTile - 1 || rowA >= ld) return;  // tile entirely above the diagonal
  if (!pm.norms) {
    syrk_lp_tile<G>(A, lds, ld, k0, kw, rowA, colB, clim);
    return;
  }
  const double bnd = pm.norms[(rowA - pm.r0) >> 7] * pm.norms[(colB - pm.r0) >> 7];
  const double thr = pm.tol * *pm.dmax;
  const int path = bnd * pm.u_low <= thr ? 2 : (bnd * pm.u_f32 <= thr ? 1 : 0);
  if (threadIdx.x == 0) atomicAdd(pm.counts + path, 1ull);
  if (path == 2) syrk_lp_tile<G>(A, lds, ld, k0, kw, rowA, colB, clim);
  else if (path == 1) syrk_lp_tile<GemmF32>(A, lds, ld, k0, kw, rowA, colB, clim);
  else syrk_lp_tile<GemmF64T<128>>(A, lds, ld, k0, kw, rowA, colB, clim);
}

// Block norms of the finished tile column for the precision map: workgroup b
// covers rows r0 + 128 b .. + 127 of columns [k0, k0 + kw).
__global__ __launch_bounds__(256) void panel_norm_kernel(const double* __restrict__ A, int ld, int k0, int kw,
                                                         int r0, const int* __restrict__ info,
                                                         double* __restrict__ norms) {
  if (*info != 0) return;
  __shared__ double red[256];
  const long rb = (long)r0 + (long)blockIdx.x * 128;
  double s = 0.0;
  for (int e = threadIdx.x; e < 128 * kw; e += 256) {
    const long row = rb + e / kw;
    if (row < ld) {
      const double v = A[row * ld + k0 + e % kw];
      s += v * v;
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) norms[blockIdx.x] = sqrt(red[0]);
}

// max_i A_ii of the matrix about to be factored; clears the path counters.
__global__ __launch_bounds__(1024) void diag_max_kernel(const double* __restrict__ A, int ld,
                                                        double* __restrict__ dmax,
                                                        unsigned long long* __restrict__ counts) {
  __shared__ double red[1024];
  double m = 0.0;
  for (int i = threadIdx.x; i < ld; i += 1024) m = fmax(m, A[(long)i * ld + i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int h = 512; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *dmax = red[0];
  if (threadIdx.x < 3) counts[threadIdx.x] = 0ull;
}

// Tiles (blockIdx.y, blockIdx.x) of A[r0:, r0:].
template <class G>
__global__ __launch_bounds__(256) void chol_syrk_lp_kernel(double* __restrict__ A, int ld, int k0, int kw, int r0,
                                                           const int* __restrict__ info, PrecMap pm) {
  chol_syrk_lp_body<G>(A, ld, k0, kw, info, r0 + (long)blockIdx.y * kTile, r0 + (long)blockIdx.x * kCols, ld, pm);
}

// Tile column [c1, c2) of the trailing matrix, c1 = k0 + kw.
template <class G>
__global__ __launch_bounds__(256) void chol_syrk_lp_col_kernel(double* __restrict__ A, int ld, int k0, int kw, int c2,
                                                               const int* __restrict__ info, PrecMap pm) {
  const long c1 = (long)k0 + kw;
  chol_syrk_lp_body<G>(A, ld, k0, kw, info, c1 + (long)blockIdx.y * kTile, c1 + (long)blockIdx.x * kCols, c2, pm);
}

// Low-precision operand copy of the finished factor for the sweep's GEMM:
// FP32, BF16, or BF16 hi and lo planes (x = hi + lo).
template <class E, int SPLIT>
__global__ __launch_bounds__(256) void convert_factor_flat_kernel(const double* __restrict__ L, long elems,
                                                                  E* __restrict__ out) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= elems) return;
  const double v = L[e];
  const E hi = (E)(float)v;
  out[e] = hi;
  if (SPLIT == 2) out[elems + e] = (E)(float)(v - (double)(float)hi);
}

template <class E, int SPLIT>
__global__ __launch_bounds__(256) void convert_factor_kernel(const double* __restrict__ L, long ld,
                                                             E* __restrict__ out) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= ld * ld) return;
  const double v = L[e];
  const E hi = (E)(float)v;
  out[e] = hi;
  if (SPLIT == 2) out[ld * ld + e] = (E)(float)(v - (double)(float)hi);
}

// Unit roundoff of a tile update's products in policy G's type, with the
// FP32 accumulation of K products (worst case).
template <class G>
static double unit_roundoff(int kw) {
  const double acc = ldexp((double)kw, -24);
  if (std::is_same<G, GemmF32>::value) return ldexp(1.0, -23) + acc;
  if (std::is_same<G, GemmBF16>::value) return ldexp(1.0, -8) + acc;
  return ldexp(1.0, -15) + acc;  // split BF16: hi*hi + hi*lo + lo*hi
}

template <class G>
static hipError_t cholesky_lp(int ld, int tile, double* A, int* info, hipStream_t st, SideStream* sd,
                              const LpMap* map) {
  // panel norms of step k in slot k & 1: the rest of step k (side stream)
  // may still read them while step k + 1 writes the other slot; step k + 2
  // runs after next(k + 1), which waits for rest(k)
  const long nslot = ld / 128 + 1;
  auto pm_of = [&](int k0, int kw) {
    PrecMap pm{};
    if (map) {
      pm.norms = map->norms + (long)(((k0 / tile) & 1)) * nslot;
      pm.dmax = map->dmax;
      pm.counts = map->counts;
      pm.r0 = (long)k0 + kw;
      pm.tol = map->tol;
      pm.u_low = unit_roundoff<G>(kw);
      pm.u_f32 = unit_roundoff<GemmF32>(kw);
    }
    return pm;
  };
  auto post = [&](int k0, int kw, hipStream_t s) {
    if (!map) return;
    const int r0 = k0 + kw;
    if (r0 >= ld) return;
    hipLaunchKernelGGL(panel_norm_kernel, dim3((unsigned)((ld - r0 + 127) / 128)), dim3(256), 0, s, (const double*)A,
                       ld, k0, kw, r0, (const int*)info, map->norms + (long)((k0 / tile) & 1) * nslot);
  };
  auto next = [&](int k0, int kw, int c2, hipStream_t s) {
    const long c1 = (long)k0 + kw;
    const dim3 grid((unsigned)((c2 - c1 + kCols - 1) / kCols), (unsigned)((ld - c1 + kTile - 1) / kTile));
    hipLaunchKernelGGL(chol_syrk_lp_col_kernel<G>, grid, dim3(256), 0, s, A, ld, k0, kw, c2, (const int*)info,
                       pm_of(k0, kw));
  };
  auto rest = [&](int k0, int kw, int r0, hipStream_t s) {
    const dim3 grid((unsigned)((ld - r0 + kCols - 1) / kCols), (unsigned)((ld - r0 + kTile - 1) / kTile));
    hipLaunchKernelGGL(chol_syrk_lp_kernel<G>, grid, dim3(256), 0, s, A, ld, k0, kw, r0, (const int*)info,
                       pm_of(k0, kw));
  };
  if (map)
    hipLaunchKernelGGL(diag_max_kernel, dim3(1), dim3(1024), 0, st, (const double*)A, ld, map->dmax, map->counts);
  return right_looking(ld, tile, A, info, st, sd, next, rest, 0, post);
}

// Low-precision operand copy of the finished factor (prec 1..3).
static hipError_t convert_factor(int prec, int ld, const double* A, void* low, hipStream_t st) {
  const long tot = (long)ld * ld;
  const dim3 cg((unsigned)((tot + 255) / 256));
  switch (prec) {
    case 1: hipLaunchKernelGGL((convert_factor_kernel<float, 1>), cg, dim3(256), 0, st, A, (long)ld, (float*)low); break;
    case 2: hipLaunchKernelGGL((convert_factor_kernel<__bf16, 1>), cg, dim3(256), 0, st, A, (long)ld, (__bf16*)low); break;
    case 3: hipLaunchKernelGGL((convert_factor_kernel<__bf16, 2>), cg, dim3(256), 0, st, A, (long)ld, (__bf16*)low); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_cholesky_lp(int prec, int ld, int tile, double* A, int* info, void* low, hipStream_t st,
                              const LpMap* map, bool fp64_factor) {
  if (prec < 1 || prec > 3) return hipErrorInvalidValue;
  if (fp64_factor) {
    hipError_t e = launch_cholesky_f64(ld, tile, A, info, st);
    if (e != hipSuccess) return e;
    return convert_factor(prec, ld, A, low, st);
  }
  SideStream* sd = ld > 2 * tile ? side_stream(kSideCholesky, st) : nullptr;
  std::unique_lock<std::mutex> lock;
  if (sd) lock = std::unique_lock<std::mutex>(sd->mu);
  hipError_t e;
  switch (prec) {
    case 1: e = cholesky_lp<GemmF32>(ld, tile, A, info, st, sd, map); break;
    case 2: e = cholesky_lp<GemmBF16>(ld, tile, A, info, st, sd, map); break;
    default: e = cholesky_lp<GemmBF16x3>(ld, tile, A, info, st, sd, map); break;
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(zero_upper_kernel, dim3(ld / 16, ld / 16), dim3(256), 0, st, A, ld);
  return convert_factor(prec, ld, A, low, st);
}

// ------------------------------------------------------------ batches
__device__ __forceinline__ int batch_find(const BatchDesc* desc, int count, long b) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (desc[mid].tile_off <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(256) void batch_build_kernel(const BatchDesc* __restrict__ desc, int count,
                                                          const int64_t* __restrict__ idx,
                                                          const double* __restrict__ locs, Matern mk,
                                                          double* __restrict__ factor, int* __restrict__ info) {
  const long b = blockIdx.x;
  const int p = batch_find(desc, count, b);
  const BatchDesc d = desc[p];
  const long lt = b - d.tile_off;
  long ti = (long)((sqrt(8.0 * (double)lt + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= lt) ++ti;
  while (ti * (ti + 1) / 2 > lt) --ti;
  const long tj = lt - ti * (ti + 1) / 2;
  if (lt == 0 && threadIdx.x == 0) info[p] = 0;
  double* A = factor + d.factor_off;
  const int64_t* ix = idx + d.lim_off;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const long i = ti * 64 + (e >> 6), j = tj * 64 + (e & 63);
    if (j > i) continue;
    double v;
    if (i >= d.n || j >= d.n) {
      v = (i == j) ? 1.0 : 0.0;
    } else {
      const long gi = ix[i], gj = ix[j];
      const double dx = locs[2 * gi] - locs[2 * gj];
      const double dy = locs[2 * gi + 1] - locs[2 * gj + 1];
      v = matern_cov(mk, sqrt(dx * dx + dy * dy));
      if (i == j) v += mk.nugget;
    }
    A[i * d.ld + j] = v;
  }
}

hipError_t launch_batch_build(const BatchDesc* desc, int count, long total_tiles, const int64_t* idx,
                              const double* locs, const Matern& mk, double* factor, int* info, hipStream_t st) {
  hipLaunchKernelGGL(batch_build_kernel, dim3((unsigned)total_tiles), dim3(256), 0, st, desc, count, idx,
                     locs, mk, factor, info);
  return hipGetLastError();
}

// Columns per step of the batched factorisation: each step's trailing update
// reads and rewrites the trailing matrix once, so 256-wide steps halve that
// traffic against 128-wide ones (the sub-panels stay 32 wide).
constexpr int kBatchTile = 256;

__global__ __launch_bounds__(64) void batch_diag_kernel(const BatchDesc* __restrict__ desc,
                                                        const int* __restrict__ order, double* factor, int j0,
                                                        int* info) {
  const int p = order[blockIdx.x];
  const BatchDesc d = desc[p];
  chol_diag_body(factor + d.factor_off, d.ld, j0, kSub, info + p);
}

// Compact grids for the batched steps: problems of equal padded size (ranks
// are sorted by size, so they are consecutive) form a group; the host passes
// per group its first rank, problem count, items per problem and the running
// item count, and workgroup b finds its (rank, item) by a binary search.
// Only the items that exist are launched.
constexpr int kMaxGroups = 32;
struct BatchGroups {
  int n;
  int rank0[kMaxGroups];
  int count[kMaxGroups];
  int items[kMaxGroups];
  int cum[kMaxGroups + 1];
};

__device__ __forceinline__ void group_item(const BatchGroups& g, int b, int& rank, int& item) {
  int lo = 0, hi = g.n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (g.cum[mid] <= b) lo = mid;
    else hi = mid;
  }
  const int off = b - g.cum[lo];
  rank = g.rank0[lo] + off / g.items[lo];
  item = off % g.items[lo];
}

__global__ __launch_bounds__(256) void batch_trsm_kernel(const BatchDesc* __restrict__ desc,
                                                         const int* __restrict__ order, double* factor,
                                                         int k0, int j0, int* info, BatchGroups g) {
  int rank, item;
  group_item(g, blockIdx.x, rank, item);
  const int p = order[rank];
  const BatchDesc d = desc[p];
  chol_panel_body<true>(factor + d.factor_off, d.ld, k0, j0, kSub, min(k0 + kBatchTile, d.ld), info + p, item);
}

__global__ __launch_bounds__(256) void batch_syrk_kernel(const BatchDesc* __restrict__ desc,
                                                         const int* __restrict__ order, double* factor,
                                                         int k0, const int* info, BatchGroups g) {
  int rank, item;
  group_item(g, blockIdx.x, rank, item);
  const int p = order[rank];
  const BatchDesc d = desc[p];
  long ti, tj;
  tri_tile(item, ti, tj);
  const long r0 = (long)k0 + kBatchTile;
  chol_syrk_body<false>(factor + d.factor_off, d.ld, k0, kBatchTile, info + p, r0 + ti * kTile, r0 + tj * kTile, d.ld);
}

// Lower 128 x 64 tiles of the trailing matrix: row tile by holds 2 by + 2
// of them, so item t has by = floor((sqrt(4 t + 1) - 1) / 2).
__device__ __forceinline__ void batch_lp_tile(int item, int& by, int& bx) {
  by = (int)((sqrt(4.0 * item + 1.0) - 1.0) * 0.5);
  while ((by + 1) * (by + 2) <= item) ++by;
  while (by * (by + 1) > item) --by;
  bx = item - by * (by + 1);
}

// The BF16 trailing updates of the batch read their operands from a BF16
// copy of the step's panel instead of converting FP64 rows per tile: rows
// [k0 + 256, ld) x columns [k0, k0 + 256) of every problem are rounded once
// per step into the low-precision factor planes (the layout of the FP64
// factor, `plane` elements apart; the final conversion after the last step
// rewrites them with the same rounding), as hi and, for SPLIT 2, lo =
// bf16(x - hi).  Item i of a problem covers its 128-row block i.
template <int SPLIT>
__global__ __launch_bounds__(256) void batch_panel_bf16_kernel(const BatchDesc* __restrict__ desc,
                                                               const int* __restrict__ order,
                                                               const double* __restrict__ factor,
                                                               __bf16* __restrict__ low, long plane, int k0,
                                                               const int* __restrict__ info, BatchGroups g) {
  int rank, item;
  group_item(g, blockIdx.x, rank, item);
  const int p = order[rank];
  if (info[p] != 0) return;
  const BatchDesc d = desc[p];
  const long row0 = (long)k0 + kBatchTile + (long)item * kTile;
  const double* src = factor + d.factor_off + row0 * d.ld + k0;
  __bf16* dst = low + d.factor_off + row0 * d.ld + k0;
  // 128 rows x 256 columns in runs of 8: 16 runs per thread
#pragma unroll 4
  for (int e = threadIdx.x; e < kTile * (kBatchTile / 8); e += 256) {
    const long off = (long)(e / (kBatchTile / 8)) * d.ld + (e % (kBatchTile / 8)) * 8;
    const double2* s = reinterpret_cast<const double2*>(src + off);
    bf16x8 hi, lo;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double2 v = s[q];
      hi[2 * q] = to_bf16(v.x);
      hi[2 * q + 1] = to_bf16(v.y);
      if (SPLIT == 2) {
        lo[2 * q] = to_bf16(v.x - (double)(float)hi[2 * q]);
        lo[2 * q + 1] = to_bf16(v.y - (double)(float)hi[2 * q + 1]);
      }
    }
    *reinterpret_cast<bf16x8*>(dst + off) = hi;
    if (SPLIT == 2) *reinterpret_cast<bf16x8*>(dst + plane + off) = lo;
  }
}

// One lower 128 x 64 tile of a problem's trailing update in BF16 (three
// products of hi and lo planes for SPLIT 2) with FP32 accumulation, the
// operands loaded from the BF16 panel straight into the MFMA registers: no
// LDS and no barrier, so occupancy is set by registers alone.  Wave w owns
// rows 32 w .. 32 w + 31 of the tile; lane (r = lane & 15, q = lane >> 4)
// holds k = 8 q .. 8 q + 7 of each 32-deep block of its A rows and B columns,
// the operand layout of the LDS-staged policy, and the K blocks run in the
// same order, so the tile equals that policy's bit for bit.
template <int SPLIT>
struct BatchBf16Frag {
  bf16x8 a[SPLIT][2];
  bf16x8 b[SPLIT][4];
};

template <int SPLIT>
__device__ __forceinline__ void batch_bf16_load(const __bf16* __restrict__ pa, const __bf16* __restrict__ pb,
                                                long ld, long plane, int k, BatchBf16Frag<SPLIT>& f) {
#pragma unroll
  for (int sp = 0; sp < SPLIT; ++sp) {
#pragma unroll
    for (int ib = 0; ib < 2; ++ib)
      f.a[sp][ib] = *reinterpret_cast<const bf16x8*>(pa + sp * plane + (long)ib * 16 * ld + k);
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
      f.b[sp][jb] = *reinterpret_cast<const bf16x8*>(pb + sp * plane + (long)jb * 16 * ld + k);
  }
}

template <int SPLIT>
__device__ __forceinline__ void batch_bf16_mma(const BatchBf16Frag<SPLIT>& f, f32x4 (&acc)[2][4]) {
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
      acc[ib][jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.a[0][ib], f.b[0][jb], acc[ib][jb], 0, 0, 0);
      if (SPLIT == 2) {
        acc[ib][jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.a[0][ib], f.b[SPLIT - 1][jb], acc[ib][jb], 0, 0, 0);
        acc[ib][jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.a[SPLIT - 1][ib], f.b[0][jb], acc[ib][jb], 0, 0, 0);
      }
    }
}

template <int SPLIT>
__global__ __launch_bounds__(256) void batch_syrk_bf16_kernel(const BatchDesc* __restrict__ desc,
                                                              const int* __restrict__ order, double* factor,
                                                              const __bf16* __restrict__ low, long plane, int k0,
                                                              const int* __restrict__ info, BatchGroups g) {
  int rank, item;
  group_item(g, blockIdx.x, rank, item);
  const int p = order[rank];
  if (info[p] != 0) return;
  const BatchDesc d = desc[p];
  int by, bx;
  batch_lp_tile(item, by, bx);
  const long ld = d.ld;
  const long r0 = (long)k0 + kBatchTile;
  // ld is a multiple of 128 and r0 of 128, so the tile's rows and columns
  // (colB + 63 <= rowA + 127 < ld) and K = [k0, k0 + 256) all exist
  const long rowA = r0 + (long)by * kTile, colB = r0 + (long)bx * kCols;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = lane & 15, q = lane >> 4;
  const __bf16* Lp = low + d.factor_off;
  const __bf16* pa = Lp + (rowA + 32 * w + r) * ld + k0 + 8 * q;
  const __bf16* pb = Lp + (colB + r) * ld + k0 + 8 * q;
  f32x4 acc[2][4];
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) acc[ib][jb] = f32x4{0.f, 0.f, 0.f, 0.f};
  constexpr int kSteps = kBatchTile / 32;
  BatchBf16Frag<SPLIT> f[2];
  batch_bf16_load<SPLIT>(pa, pb, ld, plane, 0, f[0]);
  batch_bf16_load<SPLIT>(pa, pb, ld, plane, 32, f[1]);
#pragma unroll
  for (int s = 0; s < kSteps; ++s) {
    batch_bf16_mma<SPLIT>(f[s & 1], acc);
    if (s + 2 < kSteps) batch_bf16_load<SPLIT>(pa, pb, ld, plane, 32 * (s + 2), f[s & 1]);
  }
  double* A = factor + d.factor_off;
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const long gi = rowA + 32 * w + 16 * ib + 4 * q + v, gj = colB + 16 * jb + r;
        if (gj <= gi) A[gi * ld + gj] -= (double)acc[ib][jb][v];
      }
}

// The FP32 form: the panel rounded to FP32 with each 32-column block stored
// permuted, k = 4 j + q at 8 q + j, so that lane q of a 16 x 16 x 4 MFMA
// finds its eight k of the block (j = 0..7) in 32 contiguous bytes.
__global__ __launch_bounds__(256) void batch_panel_f32_kernel(const BatchDesc* __restrict__ desc,
                                                              const int* __restrict__ order,
                                                              const double* __restrict__ factor,
                                                              float* __restrict__ low, int k0,
                                                              const int* __restrict__ info, BatchGroups g) {
  int rank, item;
  group_item(g, blockIdx.x, rank, item);
  const int p = order[rank];
  if (info[p] != 0) return;
  const BatchDesc d = desc[p];
  const long row0 = (long)k0 + kBatchTile + (long)item * kTile;
  const double* src = factor + d.factor_off + row0 * d.ld + k0;
  float* dst = low + d.factor_off + row0 * d.ld + k0;
  // (row, 32-column block b, q), q fastest: the four lanes of a (row, b)
  // read its 32 contiguous doubles between them
  for (int e = threadIdx.x; e < kTile * (kBatchTile / 32) * 4; e += 256) {
    const int q = e & 3, b = (e >> 2) & (kBatchTile / 32 - 1), row = e / (kBatchTile / 8);
    const double* sp = src + (long)row * d.ld + 32 * b + q;
    const float4 v0{(float)sp[0], (float)sp[4], (float)sp[8], (float)sp[12]};
    const float4 v1{(float)sp[16], (float)sp[20], (float)sp[24], (float)sp[28]};
    float4* o = reinterpret_cast<float4*>(dst + (long)row * d.ld + 32 * b + 8 * q);
    o[0] = v0;
    o[1] = v1;
  }
}

// One lower 128 x 64 tile in FP32 from the permuted FP32 panel, operands
// straight into registers as in the BF16 form; the k order of the products
// is that of the LDS-staged FP32 policy (k = 4 j + q in MFMA j), so the tile
// equals its result bit for bit.
struct BatchF32Frag {
  float4 a[2][2];
  float4 b[4][2];
};

__device__ __forceinline__ void batch_f32_load(const float* __restrict__ pa, const float* __restrict__ pb, long ld,
                                               int k, BatchF32Frag& f) {
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int h = 0; h < 2; ++h) f.a[ib][h] = *reinterpret_cast<const float4*>(pa + (long)ib * 16 * ld + k + 4 * h);
#pragma unroll
  for (int jb = 0; jb < 4; ++jb)
#pragma unroll
    for (int h = 0; h < 2; ++h) f.b[jb][h] = *reinterpret_cast<const float4*>(pb + (long)jb * 16 * ld + k + 4 * h);
}

__device__ __forceinline__ float f4_at(const float4& v, int i) { return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w; }

__device__ __forceinline__ void batch_f32_mma(const BatchF32Frag& f, f32x4 (&acc)[2][4]) {
#pragma unroll
  for (int j = 0; j < 8; ++j)
#pragma unroll
    for (int ib = 0; ib < 2; ++ib)
#pragma unroll
      for (int jb = 0; jb < 4; ++jb)
        acc[ib][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(f4_at(f.a[ib][j >> 2], j & 3), f4_at(f.b[jb][j >> 2], j & 3),
                                                           acc[ib][jb], 0, 0, 0);
}

__global__ __launch_bounds__(256) void batch_syrk_f32_kernel(const BatchDesc* __restrict__ desc,
                                                             const int* __restrict__ order, double* factor,
                                                             const float* __restrict__ low, int k0,
                                                             const int* __restrict__ info, BatchGroups g) {
  int rank, item;
  group_item(g, blockIdx.x, rank, item);
  const int p = order[rank];
  if (info[p] != 0) return;
  const BatchDesc d = desc[p];
  int by, bx;
  batch_lp_tile(item, by, bx);
  const long ld = d.ld;
  const long r0 = (long)k0 + kBatchTile;
  const long rowA = r0 + (long)by * kTile, colB = r0 + (long)bx * kCols;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = lane & 15, q = lane >> 4;
  const float* Lp = low + d.factor_off;
  const float* pa = Lp + (rowA + 32 * w + r) * ld + k0 + 8 * q;
  const float* pb = Lp + (colB + r) * ld + k0 + 8 * q;
  f32x4 acc[2][4];
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) acc[ib][jb] = f32x4{0.f, 0.f, 0.f, 0.f};
  constexpr int kSteps = kBatchTile / 32;
  BatchF32Frag f[2];
  batch_f32_load(pa, pb, ld, 0, f[0]);
  batch_f32_load(pa, pb, ld, 32, f[1]);
#pragma unroll
  for (int s = 0; s < kSteps; ++s) {
    batch_f32_mma(f[s & 1], acc);
    if (s + 2 < kSteps) batch_f32_load(pa, pb, ld, 32 * (s + 2), f[s & 1]);
  }
  double* A = factor + d.factor_off;
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const long gi = rowA + 32 * w + 16 * ib + 4 * q + v, gj = colB + 16 * jb + r;
        if (gj <= gi) A[gi * ld + gj] -= (double)acc[ib][jb][v];
      }
}

// Launches `launch(groups, total)` for the groups of ranks [0, cnt) with
// items(ld) > 0 work items each, at most kMaxGroups groups per launch.
template <class Items, class Launch>
static hipError_t for_groups(const int* ld_rank, int cnt, Items items, Launch launch) {
  BatchGroups g{};
  int r = 0;
  while (r < cnt) {
    int r1 = r;
    while (r1 < cnt && ld_rank[r1] == ld_rank[r]) ++r1;
    const int it = items(ld_rank[r]);
    if (it > 0) {
      g.rank0[g.n] = r;
      g.count[g.n] = r1 - r;
      g.items[g.n] = it;
      g.cum[g.n + 1] = g.cum[g.n] + (r1 - r) * it;
      ++g.n;
    }
    r = r1;
    if (g.n == kMaxGroups || (r >= cnt && g.n > 0)) {
      launch(g, g.cum[g.n]);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      g = BatchGroups{};
    }
  }
  return hipSuccess;
}

hipError_t launch_batch_cholesky(int prec, const BatchDesc* desc, const int* order, const int* ld_rank,
                                 int count, double* factor, int* info, void* low, long factor_elems,
                                 hipStream_t st) {
  const int ldmax = ld_rank[0];
  for (int k0 = 0; k0 < ldmax; k0 += kBatchTile) {
    int cnt = 0;
    while (cnt < count && ld_rank[cnt] > k0) ++cnt;
    for (int j0 = k0; j0 < k0 + kBatchTile; j0 += kSub) {
      if (j0 == k0)
        hipLaunchKernelGGL(batch_diag_kernel, dim3(cnt), dim3(64), 0, st, desc, order, factor, j0, info);
      const hipError_t e = for_groups(
          ld_rank, cnt, [&](int ld) { return (ld - (j0 + kSub) + kTile - 1) / kTile; },
          [&](const BatchGroups& g, int total) {
            hipLaunchKernelGGL(batch_trsm_kernel, dim3(total), dim3(256), 0, st, desc, order, factor, k0, j0, info,
                               g);
          });
      if (e != hipSuccess) return e;
    }
    int cnt2 = 0;
    while (cnt2 < count && ld_rank[cnt2] > k0 + kBatchTile) ++cnt2;
    if (cnt2 > 0) {
      hipError_t e;
      if (prec == 0) {
        e = for_groups(
            ld_rank, cnt2,
            [&](int ld) {
              const int nt = (ld - (k0 + kBatchTile)) / kTile;
              return nt * (nt + 1) / 2;
            },
            [&](const BatchGroups& g, int total) {
              hipLaunchKernelGGL(batch_syrk_kernel, dim3(total), dim3(256), 0, st, desc, order, factor, k0,
                                 (const int*)info, g);
            });
      } else if (prec == 1) {
        // FP32: the step's panel rounded once (permuted), then the tiles
        float* lf = (float*)low;
        e = for_groups(
            ld_rank, cnt2, [&](int ld) { return (ld - (k0 + kBatchTile)) / kTile; },
            [&](const BatchGroups& g, int total) {
              hipLaunchKernelGGL(batch_panel_f32_kernel, dim3(total), dim3(256), 0, st, desc, order,
                                 (const double*)factor, lf, k0, (const int*)info, g);
            });
        if (e == hipSuccess)
          e = for_groups(
              ld_rank, cnt2,
              [&](int ld) {
                const int nt = (ld - (k0 + kBatchTile)) / kTile;
                return nt * (nt + 1);
              },
              [&](const BatchGroups& g, int total) {
                hipLaunchKernelGGL(batch_syrk_f32_kernel, dim3(total), dim3(256), 0, st, desc, order, factor,
                                   (const float*)lf, k0, (const int*)info, g);
              });
      } else {
        // BF16 / split BF16: the step's panel rounded once, then the tiles
        __bf16* lb = (__bf16*)low;
        e = for_groups(
            ld_rank, cnt2, [&](int ld) { return (ld - (k0 + kBatchTile)) / kTile; },
            [&](const BatchGroups& g, int total) {
              if (prec == 2)
                hipLaunchKernelGGL(batch_panel_bf16_kernel<1>, dim3(total), dim3(256), 0, st, desc, order,
                                   (const double*)factor, lb, factor_elems, k0, (const int*)info, g);
              else
                hipLaunchKernelGGL(batch_panel_bf16_kernel<2>, dim3(total), dim3(256), 0, st, desc, order,
                                   (const double*)factor, lb, factor_elems, k0, (const int*)info, g);
            });
        if (e == hipSuccess)
          e = for_groups(
              ld_rank, cnt2,
              [&](int ld) {
                const int nt = (ld - (k0 + kBatchTile)) / kTile;
                return nt * (nt + 1);
              },
              [&](const BatchGroups& g, int total) {
                if (prec == 2)
                  hipLaunchKernelGGL(batch_syrk_bf16_kernel<1>, dim3(total), dim3(256), 0, st, desc, order, factor,
                                     (const __bf16*)lb, factor_elems, k0, (const int*)info, g);
                else
                  hipLaunchKernelGGL(batch_syrk_bf16_kernel<2>, dim3(total), dim3(256), 0, st, desc, order, factor,
                                     (const __bf16*)lb, factor_elems, k0, (const int*)info, g);
              });
      }
      if (e != hipSuccess) return e;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (prec != 0) {
    // one conversion over the whole packed factor; plane stride = factor_elems
    const dim3 cg((unsigned)((factor_elems + 255) / 256));
    switch (prec) {
      case 1: hipLaunchKernelGGL((convert_factor_flat_kernel<float, 1>), cg, dim3(256), 0, st, (const double*)factor, factor_elems, (float*)low); break;
      case 2: hipLaunchKernelGGL((convert_factor_flat_kernel<__bf16, 1>), cg, dim3(256), 0, st, (const double*)factor, factor_elems, (__bf16*)low); break;
      case 3: hipLaunchKernelGGL((convert_factor_flat_kernel<__bf16, 2>), cg, dim3(256), 0, st, (const double*)factor, factor_elems, (__bf16*)low); break;
    }
  }
  return hipGetLastError();
}

}  // namespace mvn
