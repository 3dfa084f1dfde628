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

}  // namespace mvn
