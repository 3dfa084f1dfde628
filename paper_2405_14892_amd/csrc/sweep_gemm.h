// GEMM step of the SOV sweep (S = L_(r,0:r) Y_(0:r), Algorithm 2's limit
// update) in each arithmetic the library offers.  A policy supplies the
// element type of the factor copy and of the Y scratch, the stage loaders,
// the MFMA step, and the mapping of its accumulators onto the 128 x 64 block.
//
// Tile: RB block rows (128 or 64) x 64 sample columns per workgroup of four
// wave64s; wave w owns rows [w RB/4, (w+1) RB/4) x all 64 columns = RB/64 x 4
// MFMA blocks of 16 x 16.  K advances in LDS stages, double-buffered; the
// next stage's global loads are in flight while the current stage's MFMAs
// run.  The 64-row shape needs 38-47 KB of LDS, so four workgroups (three
// for split BF16) share a CU instead of two: more conditioning waves at
// once; the 128-row shape reads the sample block Y half as often.
//
//   GemmF64   v_mfma_f64_16x16x4_f64, FP64 operands; stage 16 deep
//   GemmF32   v_mfma_f32_16x16x4_f32, FP32 operands, FP32 accumulation;
//             stage 32 deep
//   GemmBF16  v_mfma_f32_16x16x32_bf16, BF16 operands, FP32 accumulation;
//             stage 64 deep; the Y scratch is column-major so that each
//             lane's 8 consecutive k are one 16-byte LDS read
//   GemmBF16x3  the same instruction on split operands x = x_hi + x_lo
//             (both BF16): hi*hi + hi*lo + lo*hi, about 16 significant bits
//
// Lane layouts (measured on gfx950): for 16x16x4 f64 and f32 and 16x16x32
// bf16, lane l supplies A[l%16][k-group l/16] and B[k-group l/16][l%16]; the
// f64 accumulator holds D[l/16 + 4r][l%16], the f32 ones D[4(l/16) + r][l%16].
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gemm_f64.h"

namespace mvn {

constexpr int kCols = 64;  // sample columns per workgroup
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ __bf16 to_bf16(double x) { return (__bf16)(float)x; }

// ---------------------------------------------------------------- FP64
template <int RB>
struct GemmF64T {
  using E = double;
  static constexpr int kRows = RB;
  static constexpr int kRW = RB / 4;      // rows per wave
  static constexpr int kIB = kRW / 16;    // 16-row MFMA blocks per wave
  static constexpr int kK = 16;
  static constexpr int kEA = RB * kK / 256;  // A elements per lane per stage
  static constexpr int kALd = RB + 1, kBLd = 64 + 1;
  static constexpr int kAStage = kK * kALd, kBStage = kK * kBLd;  // elements
  static constexpr int kStageBytes = (kAStage + kBStage) * 8;
  struct Acc { f64x4 v[kIB][4]; };
  struct Regs { double a[kEA]; double b[4]; };
  static __device__ __forceinline__ void zero(Acc& acc) {
#pragma unroll
    for (int i = 0; i < kIB; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc.v[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
  }
  // L: row-major [ld][ld]; Y: [ld][64].  Lane t loads kEA consecutive k of
  // row t / (kK / kEA).
  static __device__ __forceinline__ void load(const E* __restrict__ L, long ld, long, long i0, long k0,
                                              const E* __restrict__ Y, long, Regs& r) {
    const int t = threadIdx.x;
    constexpr int tpr = kK / kEA;
    const double2* pa = reinterpret_cast<const double2*>(L + (i0 + t / tpr) * ld + k0 + (t % tpr) * kEA);
#pragma unroll
    for (int q = 0; q < kEA / 2; ++q) {
      const double2 v = pa[q];
      r.a[2 * q] = v.x;
      r.a[2 * q + 1] = v.y;
    }
    const double2* p2 = reinterpret_cast<const double2*>(Y + (k0 + (t >> 4)) * kCols + (t & 15) * 4);
    const double2 v0 = p2[0], v1 = p2[1];
    r.b[0] = v0.x; r.b[1] = v0.y; r.b[2] = v1.x; r.b[3] = v1.y;
  }
  static __device__ __forceinline__ void store(void* stage, const Regs& r) {
    double* As = (double*)stage;
    double* Bs = As + kAStage;
    const int t = threadIdx.x;
    constexpr int tpr = kK / kEA;
    const int row = t / tpr, kb = (t % tpr) * kEA;
#pragma unroll
    for (int q = 0; q < kEA; ++q) As[(kb + q) * kALd + row] = r.a[q];
    double* d = Bs + (t >> 4) * kBLd + (t & 15) * 4;
    d[0] = r.b[0]; d[1] = r.b[1]; d[2] = r.b[2]; d[3] = r.b[3];
  }
  static __device__ __forceinline__ void mma(const void* stage, Acc& acc) {
    const double* As = (const double*)stage;
    const double* Bs = As + kAStage;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int kk = 0; kk < kK / 4; ++kk) {
      const int k = kk * 4 + (lane >> 4);
      double a[kIB], b[4];
#pragma unroll
      for (int ib = 0; ib < kIB; ++ib) a[ib] = As[k * kALd + w * kRW + ib * 16 + (lane & 15)];
#pragma unroll
      for (int jb = 0; jb < 4; ++jb) b[jb] = Bs[k * kBLd + jb * 16 + (lane & 15)];
#pragma unroll
      for (int ib = 0; ib < kIB; ++ib)
#pragma unroll
        for (int jb = 0; jb < 4; ++jb)
          acc.v[ib][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ib], b[jb], acc.v[ib][jb], 0, 0, 0);
    }
  }
  static __device__ __forceinline__ void to_block(const Acc& acc, double* T) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int ib = 0; ib < kIB; ++ib)
#pragma unroll
      for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          T[(w * kRW + ib * 16 + (lane >> 4) + 4 * r) * kCols + jb * 16 + (lane & 15)] = acc.v[ib][jb][r];
  }
  // y block (FP64 in T, rows x 64) -> Y scratch rows i0..i0+rows
  static __device__ __forceinline__ void put_y(const double* T, E* __restrict__ Y, long, int i0, int rows) {
    for (int e = threadIdx.x; e < rows * kCols; e += 256) Y[(long)i0 * kCols + e] = T[e];
  }
};

// ---------------------------------------------------------------- FP32
template <int RB>
struct GemmF32T {
  using E = float;
  static constexpr int kRows = RB;
  static constexpr int kRW = RB / 4;
  static constexpr int kIB = kRW / 16;
  static constexpr int kK = 32;
  static constexpr int kEA = RB * kK / 256;  // 16 or 8
  // (the 64-row shape pads A rows by 2 floats instead of 4 so that four
  // workgroups fit in the CU's LDS)
  static constexpr int kALd = RB + (RB == 64 ? 2 : 4), kBLd = 64 + 4;
  static constexpr int kAStage = kK * kALd, kBStage = kK * kBLd;
  static constexpr int kStageBytes = (kAStage + kBStage) * 4;
  struct Acc { f32x4 v[kIB][4]; };
  struct Regs { float a[kEA]; float b[8]; };
  static __device__ __forceinline__ void zero(Acc& acc) {
#pragma unroll
    for (int i = 0; i < kIB; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc.v[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  static __device__ __forceinline__ void load(const E* __restrict__ L, long ld, long, long i0, long k0,
                                              const E* __restrict__ Y, long, Regs& r) {
    const int t = threadIdx.x;
    constexpr int tpr = kK / kEA;
    const float4* pa = reinterpret_cast<const float4*>(L + (i0 + t / tpr) * ld + k0 + (t % tpr) * kEA);
#pragma unroll
    for (int q = 0; q < kEA / 4; ++q) {
      const float4 v = pa[q];
      r.a[4 * q] = v.x; r.a[4 * q + 1] = v.y; r.a[4 * q + 2] = v.z; r.a[4 * q + 3] = v.w;
    }
    const float4* pb = reinterpret_cast<const float4*>(Y + (k0 + (t >> 3)) * kCols + (t & 7) * 8);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const float4 v = pb[q];
      r.b[4 * q] = v.x; r.b[4 * q + 1] = v.y; r.b[4 * q + 2] = v.z; r.b[4 * q + 3] = v.w;
    }
  }
  static __device__ __forceinline__ void store(void* stage, const Regs& r) {
    float* As = (float*)stage;
    float* Bs = As + kAStage;
    const int t = threadIdx.x;
    constexpr int tpr = kK / kEA;
    const int row = t / tpr, kb = (t % tpr) * kEA;
#pragma unroll
    for (int q = 0; q < kEA; ++q) As[(kb + q) * kALd + row] = r.a[q];
    float* d = Bs + (t >> 3) * kBLd + (t & 7) * 8;
#pragma unroll
    for (int q = 0; q < 8; ++q) d[q] = r.b[q];
  }
  static __device__ __forceinline__ void mma(const void* stage, Acc& acc) {
    const float* As = (const float*)stage;
    const float* Bs = As + kAStage;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int kk = 0; kk < kK / 4; ++kk) {
      const int k = kk * 4 + (lane >> 4);
      float a[kIB], b[4];
#pragma unroll
      for (int ib = 0; ib < kIB; ++ib) a[ib] = As[k * kALd + w * kRW + ib * 16 + (lane & 15)];
#pragma unroll
      for (int jb = 0; jb < 4; ++jb) b[jb] = Bs[k * kBLd + jb * 16 + (lane & 15)];
#pragma unroll
      for (int ib = 0; ib < kIB; ++ib)
#pragma unroll
        for (int jb = 0; jb < 4; ++jb)
          acc.v[ib][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ib], b[jb], acc.v[ib][jb], 0, 0, 0);
    }
  }
  static __device__ __forceinline__ void to_block(const Acc& acc, double* T) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int ib = 0; ib < kIB; ++ib)
#pragma unroll
      for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          T[(w * kRW + ib * 16 + 4 * (lane >> 4) + r) * kCols + jb * 16 + (lane & 15)] =
              (double)acc.v[ib][jb][r];
  }
  static __device__ __forceinline__ void put_y(const double* T, E* __restrict__ Y, long, int i0, int rows) {
    for (int e = threadIdx.x; e < rows * kCols; e += 256) Y[(long)i0 * kCols + e] = (float)T[e];
  }
};

// ---------------------------------------------------------------- BF16
// Split count 1: plain BF16 operands.  Split count 2 (the x3 policy):
// operands are stored as hi and lo planes and three products are accumulated.
template <int SPLIT, int RB>
struct GemmBF16T {
  using E = __bf16;
  static constexpr int kRows = RB;
  static constexpr int kRW = RB / 4;
  static constexpr int kIB = kRW / 16;
  // K per stage: 64 for plain BF16 at 128 rows; 32 otherwise (the 64-row
  // plain shape then fits four workgroups per CU)
  static constexpr int kK = (SPLIT == 1 && RB == 128) ? 64 : 32;
  static constexpr int kALd = kK + 8, kBLd = kK + 8;           // row strides (elements)
  static constexpr int kAPlane = RB * kALd, kBPlane = 64 * kBLd;
  static constexpr int kAStage = SPLIT * kAPlane, kBStage = SPLIT * kBPlane;
  static constexpr int kStageBytes = (kAStage + kBStage) * 2;
  struct Acc { f32x4 v[kIB][4]; };
  // per lane: A row t / (kK / kEA) with kEA consecutive k; B column t/4, k
  // quarter (16-byte chunks)
  static constexpr int kEA = RB * kK / 256;
  static constexpr int kAChunks = kEA / 8;                    // uint4 per lane per plane (A)
  static constexpr int kBChunks = kK / 32;                    // uint4 per lane per plane (B)
  struct Regs { uint4 a[SPLIT][kAChunks]; uint4 b[SPLIT][kBChunks]; };
  static __device__ __forceinline__ void zero(Acc& acc) {
#pragma unroll
    for (int i = 0; i < kIB; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc.v[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  // L planes: row-major [ld][ld] each, `lplane` elements apart; Y planes:
  // column-major [64][ldy] each, plane stride 64*ldy
  static __device__ __forceinline__ void load(const E* __restrict__ L, long ld, long lplane, long i0,
                                              long k0, const E* __restrict__ Y, long ldy, Regs& r) {
    const int t = threadIdx.x;
    constexpr int tpr = kK / kEA;
#pragma unroll
    for (int sp = 0; sp < SPLIT; ++sp) {
      const uint4* pa = reinterpret_cast<const uint4*>(L + sp * lplane + (i0 + t / tpr) * ld + k0 +
                                                       (t % tpr) * kEA);
#pragma unroll
      for (int q = 0; q < kAChunks; ++q) r.a[sp][q] = pa[q];
      const uint4* pb = reinterpret_cast<const uint4*>(Y + sp * (long)kCols * ldy + (long)(t >> 2) * ldy +
                                                       k0 + (t & 3) * (kK / 4));
#pragma unroll
      for (int q = 0; q < kBChunks; ++q) r.b[sp][q] = pb[q];
    }
  }
  static __device__ __forceinline__ void store(void* stage, const Regs& r) {
    E* As = (E*)stage;
    E* Bs = As + kAStage;
    const int t = threadIdx.x;
    constexpr int tpr = kK / kEA;
#pragma unroll
    for (int sp = 0; sp < SPLIT; ++sp) {
      uint4* da = reinterpret_cast<uint4*>(As + sp * kAPlane + (t / tpr) * kALd + (t % tpr) * kEA);
#pragma unroll
      for (int q = 0; q < kAChunks; ++q) da[q] = r.a[sp][q];
      uint4* db = reinterpret_cast<uint4*>(Bs + sp * kBPlane + (t >> 2) * kBLd + (t & 3) * (kK / 4));
#pragma unroll
      for (int q = 0; q < kBChunks; ++q) db[q] = r.b[sp][q];
    }
  }
  static __device__ __forceinline__ void mma(const void* stage, Acc& acc) {
    const E* As = (const E*)stage;
    const E* Bs = As + kAStage;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int kk = 0; kk < kK / 32; ++kk) {
      const int k = kk * 32 + 8 * (lane >> 4);
      bf16x8 a[SPLIT][kIB], b[SPLIT][4];
#pragma unroll
      for (int sp = 0; sp < SPLIT; ++sp) {
#pragma unroll
        for (int ib = 0; ib < kIB; ++ib)
          a[sp][ib] = *reinterpret_cast<const bf16x8*>(As + sp * kAPlane +
                                                      (w * kRW + ib * 16 + (lane & 15)) * kALd + k);
#pragma unroll
        for (int jb = 0; jb < 4; ++jb)
          b[sp][jb] = *reinterpret_cast<const bf16x8*>(Bs + sp * kBPlane + (jb * 16 + (lane & 15)) * kBLd + k);
      }
#pragma unroll
      for (int ib = 0; ib < kIB; ++ib)
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) {
          acc.v[ib][jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][ib], b[0][jb], acc.v[ib][jb], 0, 0, 0);
          if (SPLIT == 2) {
            acc.v[ib][jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][ib], b[SPLIT - 1][jb], acc.v[ib][jb], 0, 0, 0);
            acc.v[ib][jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[SPLIT - 1][ib], b[0][jb], acc.v[ib][jb], 0, 0, 0);
          }
        }
    }
  }
  static __device__ __forceinline__ void to_block(const Acc& acc, double* T) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int ib = 0; ib < kIB; ++ib)
#pragma unroll
      for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          T[(w * kRW + ib * 16 + 4 * (lane >> 4) + r) * kCols + jb * 16 + (lane & 15)] =
              (double)acc.v[ib][jb][r];
  }
  // y block -> column-major Y planes: lane (c = t % 64, quarter t / 64) packs
  // 8 consecutive rows of its column into one 16-byte store.  All RB rows of
  // the block are written (rows past n are never read by later GEMMs).
  static __device__ __forceinline__ void put_y(const double* T, E* __restrict__ Y, long ldy, int i0, int) {
    const int t = threadIdx.x, c = t & 63, rq = t >> 6;
#pragma unroll
    for (int g = 0; g < RB / 32; ++g) {
      const int r0 = rq * (RB / 4) + g * 8;
      bf16x8 hi, lo;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const double v = T[(r0 + e) * kCols + c];
        hi[e] = to_bf16(v);
        if (SPLIT == 2) lo[e] = to_bf16(v - (double)(float)hi[e]);
      }
      *reinterpret_cast<bf16x8*>(Y + (long)c * ldy + i0 + r0) = hi;
      if (SPLIT == 2) *reinterpret_cast<bf16x8*>(Y + (long)kCols * ldy + (long)c * ldy + i0 + r0) = lo;
    }
  }
};

using GemmF64 = GemmF64T<128>;
using GemmF32 = GemmF32T<128>;
using GemmBF16 = GemmBF16T<1, 128>;
using GemmBF16x3 = GemmBF16T<2, 128>;

// LDS block buffer of a sweep workgroup for policy G (doubles): RB x 64 FP64
// or the two GEMM stages, whichever is larger.
template <class G>
struct SweepLdsSize {
  static constexpr int kT = G::kRows * kCols > G::kStageBytes / 4 ? G::kRows * kCols : G::kStageBytes / 4;
};

}  // namespace mvn
