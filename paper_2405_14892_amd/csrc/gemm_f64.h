// FP64 MFMA macro-tile machinery shared by the Cholesky trailing update and
// the SOV limit-update GEMM.
//
// A workgroup of 256 lanes (4 wave64s in a 2 x 2 arrangement) owns a
// 128 x 128 output tile; each wave owns 64 x 64 = 4 x 4 blocks of the
// 16 x 16 v_mfma_f64_16x16x4_f64 product.  K advances in stages of 16,
// staged through LDS in k-major layout [16][128 + 1] (one double of padding
// to spread the transposing stores over banks), double-buffered so that the
// global loads of stage s+1 overlap the MFMAs of stage s.
//
// MFMA operand layout (16x16x4, f64): lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; the 4 accumulator doubles of lane l are
// D[l/16 + 4 r][l%16], r = 0..3 (rows interleaved across lane groups;
// measured on gfx950).
#pragma once
#include <hip/hip_runtime.h>

namespace mvn {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kTile = 128;            // macro tile edge
constexpr int kStageK = 16;           // k per LDS stage
constexpr int kLdsLd = kTile + 1;     // LDS row stride (doubles)
constexpr int kStageDoubles = kStageK * kLdsLd;  // one operand, one stage

struct Acc {
  f64x4 v[4][4];
};

__device__ __forceinline__ void acc_zero(Acc& a) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) a.v[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
}

// Row / column of accumulator element (ib, jb, r) of this lane in the tile.
__device__ __forceinline__ int acc_row(int ib, int r) {
  const int lane = threadIdx.x & 63, wr = (threadIdx.x >> 6) >> 1;
  return wr * 64 + ib * 16 + (lane >> 4) + 4 * r;
}
__device__ __forceinline__ int acc_col(int jb) {
  const int lane = threadIdx.x & 63, wc = (threadIdx.x >> 6) & 1;
  return wc * 64 + jb * 16 + (lane & 15);
}

// Stage loader for an operand stored row-major as [tile row][k] (L panels,
// P panels): lane t reads 8 consecutive k of row t/2.  With MASK, rows at or
// past row_lim and k at or past k_lim read as zero.
template <bool MASK>
__device__ __forceinline__ void load_rows(const double* __restrict__ src, long ld, long row0,
                                          long k0, long row_lim, long k_lim, double (&r)[8]) {
  const int t = threadIdx.x;
  const long row = row0 + (t >> 1);
  const long kb = k0 + (t & 1) * 8;
  const double* p = src + row * ld + kb;
  if (!MASK) {
    const double2* p2 = reinterpret_cast<const double2*>(p);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double2 v = p2[q];
      r[2 * q] = v.x;
      r[2 * q + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q) r[q] = (row < row_lim && kb + q < k_lim) ? p[q] : 0.0;
  }
}

__device__ __forceinline__ void store_rows(double* __restrict__ lds, const double (&r)[8]) {
  const int t = threadIdx.x;
  const int row = t >> 1, kb = (t & 1) * 8;
#pragma unroll
  for (int q = 0; q < 8; ++q) lds[(kb + q) * kLdsLd + row] = r[q];
}

// Stage loader for an operand stored row-major as [k][tile column] (the Y
// block of the SOV sweep): lane t reads 8 consecutive columns of k row t/16.
__device__ __forceinline__ void load_cols(const double* __restrict__ src, long ld, long k0,
                                          double (&r)[8]) {
  const int t = threadIdx.x;
  const double2* p2 = reinterpret_cast<const double2*>(src + (k0 + (t >> 4)) * ld + (t & 15) * 8);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double2 v = p2[q];
    r[2 * q] = v.x;
    r[2 * q + 1] = v.y;
  }
}

__device__ __forceinline__ void store_cols(double* __restrict__ lds, const double (&r)[8]) {
  const int t = threadIdx.x;
  const int k = t >> 4, cb = (t & 15) * 8;
#pragma unroll
  for (int q = 0; q < 8; ++q) lds[k * kLdsLd + cb + q] = r[q];
}

// One LDS stage of MFMAs: acc += As^T-layout x Bs over 16 k.
__device__ __forceinline__ void mma_stage(const double* __restrict__ As,
                                          const double* __restrict__ Bs, Acc& acc) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = w >> 1, wc = w & 1;
#pragma unroll
  for (int kk = 0; kk < kStageK / 4; ++kk) {
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

// One 128 x 128 tile of C (ldc) = beta C + alpha A B^T with A (M x K, lda)
// and B (N x K, ldb) row-major.  tile_m, tile_n pick the tile.  beta is 0
// (overwrite) or 1 (accumulate).  With MASK the loads are masked at M, N, K;
// without it K must be a multiple of 16 and all 128 rows of both operand
// tiles must be readable (rows past M, N only reach masked-out outputs).
// Stores are always masked at M, N.
template <bool MASK = true>
__device__ __forceinline__ void gemm_nt_tile(double* __restrict__ C, long ldc, const double* __restrict__ A,
                                             long lda, const double* __restrict__ B, long ldb, long M, long N,
                                             long K, double alpha, double beta, long tile_m, long tile_n,
                                             double* lds /* 4 * kStageDoubles */) {
  const long rowA = tile_m * kTile, rowB = tile_n * kTile;
  Acc acc;
  acc_zero(acc);
  const int nst = (int)((K + kStageK - 1) / kStageK);
  if (nst > 0) {
    double ra[8], rb[8];
    load_rows<MASK>(A, lda, rowA, 0, M, K, ra);
    load_rows<MASK>(B, ldb, rowB, 0, N, K, rb);
    store_rows(lds, ra);
    store_rows(lds + kStageDoubles, rb);
    __syncthreads();
    for (int s = 0; s < nst; ++s) {
      double* cur = lds + (s & 1) * 2 * kStageDoubles;
      double* nxt = lds + ((s + 1) & 1) * 2 * kStageDoubles;
      if (s + 1 < nst) {
        load_rows<MASK>(A, lda, rowA, (long)(s + 1) * kStageK, M, K, ra);
        load_rows<MASK>(B, ldb, rowB, (long)(s + 1) * kStageK, N, K, rb);
      }
      mma_stage(cur, cur + kStageDoubles, acc);
      if (s + 1 < nst) {
        store_rows(nxt, ra);
        store_rows(nxt + kStageDoubles, rb);
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int ib = 0; ib < 4; ++ib)
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long gi = rowA + acc_row(ib, r), gj = rowB + acc_col(jb);
        if (gi < M && gj < N) {
          double* c = C + gi * ldc + gj;
          *c = (beta == 0.0 ? 0.0 : *c) + alpha * acc.v[ib][jb][r];
        }
      }
}

}  // namespace mvn
