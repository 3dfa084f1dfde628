// The SOV sweep (Algorithms 2-3 with Eq. (sov1)) with 256 sample columns
// per workgroup and every wave conditioning its own 64 of them.
//
// The 64-column sweep conditions a block on one wave while the other three
// wait, so a CU runs at most one conditioning wave per SIMD and a sweep with
// a cheap GEMM (reduced-precision operands, the batches' small problems) is
// bound by that one wave's latency chain.  Here wave w owns columns
// [64 w, 64 w + 64) of the workgroup's chunk for all RB rows of a block
// (RB = 64 or 128):
//   1. S = L[i0:i0+RB, 0:i0] Y[0:i0, chunk]: the L stage is shared through
//      LDS, each wave multiplies it into its own 64 columns (RB/16 x 4 MFMA
//      blocks of 16 x 16), accumulators stay in registers;
//   2. the block is conditioned in 16-row sub-blocks: the wave writes the
//      sub-block's rows of S to its columns of T (LDS, FP64), each lane runs
//      the recurrence over the sub-block for its column,
//        s_i = S_i + sum_{k in sub-block, k < i} L_ik y_k,
//        (y_i, d_i) = condition_step((a~_i - s_i)/L_ii, (b~_i - s_i)/L_ii, w_i),
//      and adds L[later rows, sub-block] y_sub to its later rows'
//      accumulators on MFMA (FP64 for FP64 operands, else FP32, the
//      accumulators' type), so a row's dot product runs over its own
//      sub-block only;
//   3. y of the sub-block goes to the wave's columns of the Y scratch.
// The four waves condition at the same time; the sub-block's triangle and
// fold columns of L are staged in LDS, double-buffered, one workgroup
// barrier per sub-block (the next sub-block's part is fetched into registers
// before the conditioning and written after it).  The factor is read once
// per 256 samples instead of once per 64, and the Y scratch once per RB rows.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "gemm_f64.h"
#include "launch.h"
#include "mvn_device.h"
#include "sweep_block.h"
#include "sweep_gemm.h"

namespace mvn {

constexpr int kQC = 256;  // sample columns per workgroup (64 per wave)
constexpr int kQS = 16;   // rows per conditioning sub-block

// ---------------------------------------------------------------- policies
// A policy gives the GEMM operand type E, the LDS stage layout and loaders
// for an L tile (RB rows x kK) and a Y tile (kK x 256), the MFMA step of wave
// w (RB rows x its 64 columns), the accumulator row of (lane, r) within a
// 16 x 16 block, the fold type F and the y write-back in E.

// FP32 operands, v_mfma_f32_16x16x4_f32; A k-major [kK][RB + 4], B k-major
// [kK][256 + 4]; Y scratch row-major [ld][256].
template <int RB>
struct QuadF32 {
  using E = float;
  using F = float;
  using AccV = f32x4;
  static constexpr int kRows = RB;
  static constexpr bool kMixed = true;
  static constexpr int kK = 16;
  static constexpr int kEA = RB * kK / 256;  // A elements per lane (4 or 8)
  static constexpr int kALd = RB + 4, kBLd = kQC + 4;
  static constexpr int kStageBytes = (kK * kALd + kK * kBLd) * 4;
  static constexpr int kStages = 2;
  struct Regs { float4 a[kEA / 4]; float4 b[4]; };
  static __device__ __forceinline__ void load(const E* __restrict__ L, long ld, long, long i0, long k0,
                                              const E* __restrict__ Y, long, Regs& r) {
    const int t = threadIdx.x;
    constexpr int tpr = kK / kEA;
    const float4* pa = reinterpret_cast<const float4*>(L + (i0 + t / tpr) * ld + k0 + (t % tpr) * kEA);
#pragma unroll
    for (int q = 0; q < kEA / 4; ++q) r.a[q] = pa[q];
    const float4* pb = reinterpret_cast<const float4*>(Y + (k0 + (t >> 4)) * kQC + (t & 15) * 16);
#pragma unroll
    for (int q = 0; q < 4; ++q) r.b[q] = pb[q];
  }
  static __device__ __forceinline__ void store(char* stage, const Regs& r) {
    float* As = (float*)stage;
    float* Bs = As + kK * kALd;
    const int t = threadIdx.x;
    constexpr int tpr = kK / kEA;
    const int row = t / tpr, kb = (t % tpr) * kEA;
#pragma unroll
    for (int q = 0; q < kEA / 4; ++q) {
      As[(kb + 4 * q + 0) * kALd + row] = r.a[q].x;
      As[(kb + 4 * q + 1) * kALd + row] = r.a[q].y;
      As[(kb + 4 * q + 2) * kALd + row] = r.a[q].z;
      As[(kb + 4 * q + 3) * kALd + row] = r.a[q].w;
    }
    float4* d = reinterpret_cast<float4*>(Bs + (t >> 4) * kBLd + (t & 15) * 16);
#pragma unroll
    for (int q = 0; q < 4; ++q) d[q] = r.b[q];
  }
  static __device__ __forceinline__ void mma(const char* stage, AccV (&acc)[RB / 16][4]) {
    const float* As = (const float*)stage;
    const float* Bs = As + kK * kALd;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int kk = 0; kk < kK / 4; ++kk) {
      const int k = kk * 4 + (lane >> 4);
      float a[RB / 16], b[4];
#pragma unroll
      for (int ib = 0; ib < RB / 16; ++ib) a[ib] = As[k * kALd + ib * 16 + (lane & 15)];
#pragma unroll
      for (int jb = 0; jb < 4; ++jb) b[jb] = Bs[k * kBLd + 64 * w + jb * 16 + (lane & 15)];
#pragma unroll
      for (int ib = 0; ib < RB / 16; ++ib)
#pragma unroll
        for (int jb = 0; jb < 4; ++jb)
          acc[ib][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ib], b[jb], acc[ib][jb], 0, 0, 0);
    }
  }
  static __device__ __forceinline__ int row_of(int lane, int r) { return 4 * (lane >> 4) + r; }
  static __device__ __forceinline__ AccV fold(F a, F b, AccV c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // y rows r0 .. r0 + 15 of column c (T column c) -> Y scratch
  static __device__ __forceinline__ void put_y(const double* T, E* __restrict__ Y, long, int r0, int c) {
#pragma unroll
    for (int r = 0; r < kQS; ++r) Y[(long)(r0 + r) * kQC + c] = (float)T[r * kQC + c];
  }
  static long yslice(int ld) { return (long)ld * kQC; }
};

// BF16 operands (SPLIT = 2: hi and lo planes, three products),
// v_mfma_f32_16x16x32_bf16; A row-major [RB][kK + 8], B column-major
// [256][kK + 8] (8 consecutive k of a row / column per lane).  Y scratch
// per plane in groups of 8 rows: element (k, c) at (k / 8) * 2048 + 8 c +
// k % 8, so that a stage's loads (one 16-byte group per lane) and the y
// write-back are contiguous across lanes.
template <int SPLIT, int RB>
struct QuadBF16 {
  using E = __bf16;
  using F = float;
  using AccV = f32x4;
  static constexpr int kRows = RB;
  static constexpr bool kMixed = true;
  static constexpr int kK = 32;
  static constexpr int kEA = RB * kK / 256;  // A elements per lane (8 or 16)
  static constexpr int kALd = kK + 8, kBLd = kK + 8;
  static constexpr int kAPlane = RB * kALd, kBPlane = kQC * kBLd;
  static constexpr int kStageBytes = SPLIT * (kAPlane + kBPlane) * 2;
  // one LDS stage for split operands (two would not leave room for the
  // resident workgroups): the next stage waits in registers
  static constexpr int kStages = SPLIT == 2 ? 1 : 2;
  struct Regs { uint4 a[SPLIT][kEA / 8]; uint4 b[SPLIT][kK / 8]; };
  static __device__ __forceinline__ void load(const E* __restrict__ L, long ld, long lplane, long i0, long k0,
                                              const E* __restrict__ Y, long ldy, Regs& r) {
    const int t = threadIdx.x;
    constexpr int tpr = kK / kEA;
#pragma unroll
    for (int sp = 0; sp < SPLIT; ++sp) {
      const uint4* pa =
          reinterpret_cast<const uint4*>(L + sp * lplane + (i0 + t / tpr) * ld + k0 + (t % tpr) * kEA);
#pragma unroll
      for (int q = 0; q < kEA / 8; ++q) r.a[sp][q] = pa[q];
      const uint4* pb = reinterpret_cast<const uint4*>(Y + (long)sp * kQC * ldy + (k0 / 8) * (kQC * 8) + t * 8);
#pragma unroll
      for (int q = 0; q < kK / 8; ++q) r.b[sp][q] = pb[q * kQC];
    }
  }
  static __device__ __forceinline__ void store(char* stage, const Regs& r) {
    E* As = (E*)stage;
    E* Bs = As + SPLIT * kAPlane;
    const int t = threadIdx.x;
    constexpr int tpr = kK / kEA;
#pragma unroll
    for (int sp = 0; sp < SPLIT; ++sp) {
      uint4* da = reinterpret_cast<uint4*>(As + sp * kAPlane + (t / tpr) * kALd + (t % tpr) * kEA);
#pragma unroll
      for (int q = 0; q < kEA / 8; ++q) da[q] = r.a[sp][q];
      uint4* db = reinterpret_cast<uint4*>(Bs + sp * kBPlane + t * kBLd);
#pragma unroll
      for (int q = 0; q < kK / 8; ++q) db[q] = r.b[sp][q];
    }
  }
  static __device__ __forceinline__ void mma(const char* stage, AccV (&acc)[RB / 16][4]) {
    const E* As = (const E*)stage;
    const E* Bs = As + SPLIT * kAPlane;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int k = 8 * (lane >> 4);
    bf16x8 b[SPLIT][4];
#pragma unroll
    for (int sp = 0; sp < SPLIT; ++sp)
#pragma unroll
      for (int jb = 0; jb < 4; ++jb)
        b[sp][jb] = *reinterpret_cast<const bf16x8*>(Bs + sp * kBPlane + (64 * w + jb * 16 + (lane & 15)) * kBLd + k);
#pragma unroll
    for (int ib = 0; ib < RB / 16; ++ib) {
      bf16x8 a[SPLIT];
#pragma unroll
      for (int sp = 0; sp < SPLIT; ++sp)
        a[sp] = *reinterpret_cast<const bf16x8*>(As + sp * kAPlane + (ib * 16 + (lane & 15)) * kALd + k);
#pragma unroll
      for (int jb = 0; jb < 4; ++jb) {
        acc[ib][jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[0][jb], acc[ib][jb], 0, 0, 0);
        if (SPLIT == 2) {
          acc[ib][jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[SPLIT - 1][jb], acc[ib][jb], 0, 0, 0);
          acc[ib][jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[SPLIT - 1], b[0][jb], acc[ib][jb], 0, 0, 0);
        }
      }
    }
  }
  static __device__ __forceinline__ int row_of(int lane, int r) { return 4 * (lane >> 4) + r; }
  static __device__ __forceinline__ AccV fold(F a, F b, AccV c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ void put_y(const double* T, E* __restrict__ Y, long ldy, int r0, int c) {
#pragma unroll
    for (int h = 0; h < kQS / 8; ++h) {
      bf16x8 hi, lo;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const double v = T[(8 * h + e) * kQC + c];
        hi[e] = to_bf16(v);
        if (SPLIT == 2) lo[e] = to_bf16(v - (double)(float)hi[e]);
      }
      E* d = Y + (long)(r0 / 8 + h) * (kQC * 8) + c * 8;
      *reinterpret_cast<bf16x8*>(d) = hi;
      if (SPLIT == 2) *reinterpret_cast<bf16x8*>(d + (long)kQC * ldy) = lo;
    }
  }
  static long yslice(int ld) { return (long)ld * kQC * SPLIT; }
};

// FP64 operands, v_mfma_f64_16x16x4_f64 (64-row blocks: 128 accumulator
// registers per lane); A k-major [kK][64 + 1], B k-major [kK][256 + 1]; Y
// scratch row-major [ld][256].
struct QuadF64 {
  using E = double;
  using F = double;
  using AccV = f64x4;
  static constexpr int kRows = 64;
  static constexpr bool kMixed = false;
  static constexpr int kK = 8;
  static constexpr int kALd = kRows + 1, kBLd = kQC + 1;
  static constexpr int kStageBytes = (kK * kALd + kK * kBLd) * 8;
  static constexpr int kStages = 2;
  struct Regs { double2 a; double2 b[4]; };
  static __device__ __forceinline__ void load(const E* __restrict__ L, long ld, long, long i0, long k0,
                                              const E* __restrict__ Y, long, Regs& r) {
    const int t = threadIdx.x;
    r.a = *reinterpret_cast<const double2*>(L + (i0 + (t >> 2)) * ld + k0 + (t & 3) * 2);
    const double2* pb = reinterpret_cast<const double2*>(Y + (k0 + (t >> 5)) * kQC + (t & 31) * 8);
#pragma unroll
    for (int q = 0; q < 4; ++q) r.b[q] = pb[q];
  }
  static __device__ __forceinline__ void store(char* stage, const Regs& r) {
    double* As = (double*)stage;
    double* Bs = As + kK * kALd;
    const int t = threadIdx.x;
    const int row = t >> 2, kb = (t & 3) * 2;
    As[kb * kALd + row] = r.a.x;
    As[(kb + 1) * kALd + row] = r.a.y;
    double* d = Bs + (t >> 5) * kBLd + (t & 31) * 8;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      d[2 * q] = r.b[q].x;
      d[2 * q + 1] = r.b[q].y;
    }
  }
  static __device__ __forceinline__ void mma(const char* stage, AccV (&acc)[4][4]) {
    const double* As = (const double*)stage;
    const double* Bs = As + kK * kALd;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int kk = 0; kk < kK / 4; ++kk) {
      const int k = kk * 4 + (lane >> 4);
      double a[4], b[4];
#pragma unroll
      for (int ib = 0; ib < 4; ++ib) a[ib] = As[k * kALd + ib * 16 + (lane & 15)];
#pragma unroll
      for (int jb = 0; jb < 4; ++jb) b[jb] = Bs[k * kBLd + 64 * w + jb * 16 + (lane & 15)];
#pragma unroll
      for (int ib = 0; ib < 4; ++ib)
#pragma unroll
        for (int jb = 0; jb < 4; ++jb)
          acc[ib][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ib], b[jb], acc[ib][jb], 0, 0, 0);
    }
  }
  static __device__ __forceinline__ int row_of(int lane, int r) { return (lane >> 4) + 4 * r; }
  static __device__ __forceinline__ AccV fold(F a, F b, AccV c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ void put_y(const double* T, E* __restrict__ Y, long, int r0, int c) {
#pragma unroll
    for (int r = 0; r < kQS; ++r) Y[(long)(r0 + r) * kQC + c] = T[r * kQC + c];
  }
  static long yslice(int ld) { return (long)ld * kQC; }
};

// LDS of the conditioning phase (aliasing the GEMM stages): T (kQS x kQC
// FP64) and two buffers of a sub-block's strict lower triangle (kQS x kQS
// FP64) and fold columns L[later rows, sub-block] ((RB - kQS) x kQS in the
// accumulators' type).
template <class P>
struct QuadLds {
  using F = typename P::F;
  static constexpr int RB = P::kRows;
  static constexpr int kTri = kQS * kQS;                  // doubles per buffer
  static constexpr int kCol = (RB - kQS) * kQS;           // F per buffer
  static constexpr int kBuf = kTri * 8 + kCol * (int)sizeof(F);
  static constexpr int kCond = kQS * kQC * 8 + 2 * kBuf;
  static constexpr int kRegion = P::kStages * P::kStageBytes > kCond ? P::kStages * P::kStageBytes : kCond;
  // resident workgroups: 128 accumulator registers per lane (FP64, or 128
  // rows) leave room for two, 64 for three
  static constexpr int kWG = (std::is_same<typename P::E, double>::value || RB == 128) ? 2 : 3;
  static_assert(kWG * (kRegion + 4 * RB * 8 + 48 * 8 + 16) <= 160 * 1024, "LDS of the resident workgroups");
};

struct QuadShared {
  char* region;
  double* c_at;
  double* c_bt;
  double* c_rl;
  uint64_t* c_lat;
  const double* tab;
};

// A sub-block's triangle and fold columns of L, fetched into registers by
// all 256 lanes and written to one LDS buffer.
template <class P>
struct QuadStage {
  using F = typename P::F;
  static constexpr int RB = P::kRows;
  static constexpr int kPerC = (QuadLds<P>::kCol + 255) / 256;  // fold entries per lane
  double tri;
  F col[kPerC];
  // rows r0 .. of the block (those < rows are real); the block's L starts at Ld
  __device__ __forceinline__ void fetch(const double* __restrict__ Ld, long ld, int r0, int rows) {
    const int t = threadIdx.x;
    const int i = t / kQS, k = t % kQS;
    tri = (k < i && r0 + i < rows) ? Ld[(long)(r0 + i) * ld + r0 + k] : 0.0;
#pragma unroll
    for (int j = 0; j < kPerC; ++j) {
      const int e = t + 256 * j, ii = r0 + kQS + e / kQS, kk = e % kQS;
      col[j] = (F)((e < (RB - r0 - kQS) * kQS && ii < rows) ? Ld[(long)ii * ld + r0 + kk] : 0.0);
    }
  }
  __device__ __forceinline__ void put(double* tri_l, F* col_l, int r0) const {
    const int t = threadIdx.x;
    tri_l[t] = tri;
#pragma unroll
    for (int j = 0; j < kPerC; ++j) {
      const int e = t + 256 * j;
      if (e < (RB - r0 - kQS) * kQS) col_l[e] = col[j];
    }
  }
};

// This lane's sample column and its QMC indices.
struct QuadLane {
  int c;           // column within the chunk (64 w + lane)
  long col;        // global sample column
  bool valid;
  uint64_t sidx, jpt;
  PrefixOut pre;   // the wave's 64 columns as a chunk of the nested-set partials
  long chunk64;
};

__device__ __forceinline__ QuadLane quad_lane(long chunk, int N, int S, double* prefix) {
  QuadLane q;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const long NS = (long)N * S;
  q.c = 64 * w + lane;
  q.col = chunk * kQC + q.c;
  q.valid = q.col < NS;
  q.sidx = q.valid ? (uint64_t)(q.col / N) : 0;
  q.jpt = q.valid ? (uint64_t)(q.col % N) + 1 : 1;
  q.chunk64 = chunk * 4 + w;
  q.pre = PrefixOut{prefix, (NS + 63) / 64, q.chunk64, (uint64_t)(q.chunk64 * 64 / N)};
  return q;
}

template <class P>
__device__ __forceinline__ void quad_zero(typename P::AccV (&acc)[P::kRows / 16][4]) {
#pragma unroll
  for (int ib = 0; ib < P::kRows / 16; ++ib)
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[ib][jb][r] = 0;
}

// acc += the product of nst LDS stages; load(s, regs) fetches stage s.  Ends
// with a barrier (the stages are free again).
template <class P, class Load>
__device__ __forceinline__ void quad_gemm(const QuadShared& sh, typename P::AccV (&acc)[P::kRows / 16][4], int nst,
                                          Load load) {
  if (nst <= 0) return;
  char* stage0 = sh.region;
  char* stage1 = sh.region + (P::kStages == 2 ? P::kStageBytes : 0);
  typename P::Regs rg;
  load(0, rg);
  P::store(stage0, rg);
  __syncthreads();
  for (int s = 0; s < nst; ++s) {
    const bool odd = s & 1;
    if (s + 1 < nst) load(s + 1, rg);
    P::mma(odd ? stage1 : stage0, acc);
    if (s + 1 < nst) {
      if (P::kStages == 1) __syncthreads();  // every wave is done with the stage
      P::store(odd ? stage0 : stage1, rg);
    }
    __syncthreads();
  }
}

// Steps 2-3 for one block of `rows` rows whose S is in acc: the block's
// diagonal block of L at Ld (leading dimension ld), global first row g0
// (the QMC dimension and the row of the limits, the lattice and Y), y to
// the Y scratch.  Ends with a barrier.
template <class P, bool PREFIX>
__device__ __forceinline__ void quad_condition(const QuadShared& sh, typename P::AccV (&acc)[P::kRows / 16][4],
                                               const double* __restrict__ Ld, long ld, int rows, long g0,
                                               const double* __restrict__ at, const double* __restrict__ bt,
                                               const uint64_t* __restrict__ lattice, uint64_t seed, int n,
                                               int periodize, typename P::E* __restrict__ Y, long ldy,
                                               const QuadLane& ln, LogProd& prod) {
  using F = typename P::F;
  constexpr int NB = P::kRows / 16;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int c = ln.c;
  double* T = (double*)sh.region;                                   // kQS x kQC
  char* bufs = sh.region + kQS * kQC * 8;                           // two triangle + fold buffers
  const auto tri_buf = [bufs](int b) { return (double*)(bufs + b * QuadLds<P>::kBuf); };
  const auto col_buf = [bufs](int b) { return (F*)(bufs + b * QuadLds<P>::kBuf + QuadLds<P>::kTri * 8); };
  const auto ninv = [&sh](double x) { return ninv_lower_tab(x, sh.tab); };
  // the first sub-block's part of L and the per-row constants
  QuadStage<P> stg;
  stg.fetch(Ld, ld, 0, rows);
  stg.put(tri_buf(0), col_buf(0), 0);
  if (t < rows) {
    const long g = g0 + t;
    sh.c_at[t] = at[g];
    sh.c_bt[t] = bt[g];
    sh.c_rl[t] = 1.0 / Ld[(long)t * ld + t];
    sh.c_lat[t] = lattice[g];
  }
#pragma unroll 1
  for (int q = 0; q < NB; ++q) {
    const int r0 = q * kQS;
    if (r0 >= rows) break;  // uniform
    const int rq = min(kQS, rows - r0);
    __syncthreads();  // buffer q % 2 is written; every wave is done with buffer (q + 1) % 2
    const bool more = r0 + kQS < rows;
    if (more) stg.fetch(Ld, ld, r0 + kQS, rows);  // in flight during the conditioning
    const double* Ltri = tri_buf(q & 1);
    const F* Lcol = col_buf(q & 1);
    // S rows of the sub-block -> T (accumulator block ib == q)
#pragma unroll
    for (int ib = 0; ib < NB; ++ib) {
      if (ib == q) {
#pragma unroll
        for (int jb = 0; jb < 4; ++jb)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            T[P::row_of(lane, r) * kQC + 64 * w + 16 * jb + (lane & 15)] = (double)acc[ib][jb][r];
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int i = 0; i < rq; ++i) {
      const double* Li = Ltri + i * kQS;
      const double* Tc = T + c;
      double s0 = Tc[i * kQC], s1 = 0.0, s2 = 0.0, s3 = 0.0;
      const int kend = (i + 3) & ~3;  // the triangle row is zero from column i on
      for (int k = 0; k < kend; k += 4) {
        s0 += Li[k] * Tc[k * kQC];
        s1 += Li[k + 1] * Tc[(k + 1) * kQC];
        s2 += Li[k + 2] * Tc[(k + 2) * kQC];
        s3 += Li[k + 3] * Tc[(k + 3) * kQC];
      }
      const double sum = (s0 + s1) + (s2 + s3);
      const int ri = r0 + i;
      const double rl = sh.c_rl[ri];
      const double alpha = (sh.c_at[ri] - sum) * rl;
      const double beta = (sh.c_bt[ri] - sum) * rl;
      const uint64_t gi = (uint64_t)(g0 + ri);
      const double wq = richtmyer(ln.jpt, sh.c_lat[ri], splitmix64(seed, ln.sidx * (uint64_t)n + gi), periodize);
      const Step st = P::kMixed ? condition_step_mixed_with(alpha, beta, wq, 1.0 - wq, ninv)
                                : condition_step_with(alpha, beta, wq, 1.0 - wq, ninv);
      T[i * kQC + c] = ln.valid ? st.y : 0.0;
      logprod_mul(prod, st);
      if constexpr (PREFIX) {
        if (ln.chunk64 < ln.pre.nchunks) prefix_row(prod, ln.valid, ln.sidx, ln.pre, (long)gi);  // uniform per wave
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // later rows += L[later rows, sub-block] y_sub (K = 16)
#pragma unroll
    for (int ib = 1; ib < NB; ++ib) {
      if (ib > q && 16 * ib < rows) {
#pragma unroll
        for (int kk = 0; kk < kQS / 4; ++kk) {
          const int k = 4 * kk + (lane >> 4);
          const F a = Lcol[(16 * ib - r0 - kQS + (lane & 15)) * kQS + k];
#pragma unroll
          for (int jb = 0; jb < 4; ++jb)
            acc[ib][jb] = P::fold(a, (F)T[k * kQC + 64 * w + 16 * jb + (lane & 15)], acc[ib][jb]);
        }
      }
    }
    // y of the sub-block -> the Y scratch (rows past n are never read)
    P::put_y(T, Y, ldy, (int)(g0 + r0), c);
    if (more) stg.put(tri_buf((q + 1) & 1), col_buf((q + 1) & 1), r0 + kQS);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  __syncthreads();  // the next stages overwrite T and the buffers
}

// The whole sweep of one 256-column chunk of one problem with a dense factor.
template <class P, bool PREFIX>
__device__ __forceinline__ void quad_chunk(const QuadShared& sh, const double* __restrict__ L,
                                           const typename P::E* __restrict__ Lg, long lplane, long ld, int n,
                                           const double* __restrict__ at, const double* __restrict__ bt,
                                           const uint64_t* __restrict__ lattice, uint64_t seed, int N, int S,
                                           int periodize, typename P::E* __restrict__ Y,
                                           double* __restrict__ ell, long chunk, double* __restrict__ prefix) {
  constexpr int RB = P::kRows;
  const QuadLane ln = quad_lane(chunk, N, S, prefix);
  LogProd prod{1.0, 0};
  for (int i0 = 0; i0 < n; i0 += RB) {
    const int rows = min(RB, n - i0);
    typename P::AccV acc[RB / 16][4];
    quad_zero<P>(acc);
    // ---- step 1: S = L[i0:i0+RB, 0:i0] Y[0:i0, chunk]
    quad_gemm<P>(sh, acc, i0 / P::kK, [&](int s, typename P::Regs& rg) {
      P::load(Lg, ld, lplane, i0, (long)s * P::kK, Y, ld, rg);
    });
    quad_condition<P, PREFIX>(sh, acc, L + (long)i0 * ld + i0, ld, rows, i0, at, bt, lattice, seed, n, periodize, Y,
                              ld, ln, prod);
  }
  if (ln.valid) ell[ln.col] = logprod_log(prod);
}

#define MVN_QUAD_LDS(P)                                                               \
  __shared__ __attribute__((aligned(16))) char q_region[QuadLds<P>::kRegion];         \
  __shared__ double q_at[P::kRows], q_bt[P::kRows], q_rl[P::kRows];                   \
  __shared__ uint64_t q_lat[P::kRows];                                                \
  __shared__ double q_tab[48];                                                        \
  if ((threadIdx.x >> 6) == 1) {                                                      \
    _Pragma("unroll") for (int e = 0; e < 48; ++e) if ((threadIdx.x & 63) == e)       \
        q_tab[e] = kAs241[e / 16][e % 16];                                            \
  }                                                                                   \
  const QuadShared sh{q_region, q_at, q_bt, q_rl, q_lat, q_tab}

// Dense factor: chunk c, c + grid, ... of 256 columns per workgroup.  (The
// table written by wave 1 is ordered before its first read by the first
// sub-block's barrier.)
template <class P, bool PREFIX>
__global__ __launch_bounds__(256, QuadLds<P>::kWG) void quad_sweep_kernel(SweepArgs p) {
  using E = typename P::E;
  MVN_QUAD_LDS(P);
  const long nchunks = ((long)p.N * p.S + kQC - 1) / kQC;
  E* Y = (E*)p.yscr + (long)blockIdx.x * p.yslice;
  for (long chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x)
    quad_chunk<P, PREFIX>(sh, p.L, (const E*)p.Llow, (long)p.ld * p.ld, p.ld, p.n, p.at, p.bt, p.lattice, p.seed,
                          p.N, p.S, p.periodize, Y, p.ell, chunk, p.prefix);
}

// Batches: work items (problem rank, chunk) in order of decreasing problem
// size from a device counter, as in the 64-column batch sweep.
template <class P>
__global__ __launch_bounds__(256, QuadLds<P>::kWG) void quad_batch_kernel(BatchSweepArgs p) {
  using E = typename P::E;
  MVN_QUAD_LDS(P);
  __shared__ long s_item;
  const long nchunks = ((long)p.N * p.S + kQC - 1) / kQC;
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
    quad_chunk<P, false>(sh, p.L + d.factor_off, (const E*)p.Llow + d.factor_off, p.lplane, d.ld, d.n,
                         p.at + d.lim_off, p.bt + d.lim_off, p.lattice, p.seed, p.N, p.S, p.periodize, Y,
                         p.ell + (long)prob * NS, chunk, nullptr);
  }
}

// A TLR factor (Section III-E's tiles, the layout of kernels_tlr.hip) with
// 256 columns per workgroup, every wave conditioning its own 64: per
// tile-row i and 64-row block b of it
//   S_b = [U_i0 .. U_i,i-1][b, :] [Z_i0; ..] + L_ii[b, <b] Y_i[<b]
// in one K loop (the packed low-rank columns, then the dense diagonal tile),
// the block conditioned with L_ii as in the dense four-wave sweep, and after
// the tile-row the stacked product of tile column i,
//   [Z_(i+1)i; Z_(i+2)i; ..] = [V'_(i+1)i^T; V'_(i+2)i^T; ..] Y_i,
// in 64-row MFMA tiles whose rows go to their places in the packed Z of the
// tile-rows below.  Against 64 columns per workgroup this reads every U and
// V' column once per 256 samples instead of once per 64, and four waves
// condition at a time instead of one.  Y slice: (nt m) x 256; Z slice:
// Kpad_total x 256, padding rows cleared once.
template <bool PREFIX>
__global__ __launch_bounds__(256, QuadLds<QuadF64>::kWG) void quad_tlr_kernel(TlrSweepArgs p) {
  using P = QuadF64;
  MVN_QUAD_LDS(P);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int m = p.m;
  const TlrSweepHdr h = *p.hdr;
  if ((long)blockIdx.x >= h.grid) return;  // the workspace holds h.grid workgroups
  const double* Vpack = p.vpack_ext ? p.vpack_ext : (const double*)(p.dyn + h.vpack);
  const double* Upack = p.upack_ext ? p.upack_ext : (const double*)(p.dyn + h.upack);
  double* Y = (double*)(p.dyn + h.yscr) + (long)blockIdx.x * p.yslice;
  double* Z = (double*)(p.dyn + h.zscr) + (long)blockIdx.x * h.zslice;
  for (int i = 1; i < p.nt; ++i)
    for (long e = (p.kpad0[i] + p.kval[i]) * kQC + t; e < p.kpad0[i + 1] * kQC; e += 256) Z[e] = 0.0;
  __syncthreads();
  const long nchunks = ((long)p.N * p.S + kQC - 1) / kQC;
  for (long chunk = blockIdx.x; chunk < nchunks; chunk += h.grid) {
    const QuadLane ln = quad_lane(chunk, p.N, p.S, p.prefix);
    LogProd prod{1.0, 0};
    for (int ti = 0; ti < p.nt; ++ti) {
      const long g0 = (long)ti * m;
      const long kp0 = p.kpad0[ti], Kp = p.kpad0[ti + 1] - kp0;
      const int nst_lr = (int)(Kp / P::kK);  // Kp is a multiple of 16
      const double* Ui = Upack + kp0 * m;     // m x Kp
      const double* Zi = Z + kp0 * kQC;       // Kp x 256
      const double* D = p.tiles + (p.diag_compact ? (long)ti : (long)ti * (ti + 1) / 2 + ti) * (long)m * m;
      const double* Yi = Y + g0 * kQC;
      for (int b0 = 0; b0 < m && g0 + b0 < p.n; b0 += P::kRows) {
        const int rows = (int)min((long)P::kRows, p.n - (g0 + b0));
        P::AccV acc[P::kRows / 16][4];
        quad_zero<P>(acc);
        quad_gemm<P>(sh, acc, nst_lr + b0 / P::kK, [&](int s, P::Regs& rg) {
          if (s < nst_lr) P::load(Ui, Kp, 0, b0, (long)s * P::kK, Zi, 0, rg);
          else P::load(D, m, 0, b0, (long)(s - nst_lr) * P::kK, Yi, 0, rg);
        });
        quad_condition<P, PREFIX>(sh, acc, D + (long)b0 * m + b0, m, rows, g0 + b0, p.at, p.bt, p.lattice, p.seed,
                                  p.n, p.periodize, Y, 0, ln, prod);
      }
      // ---- the stacked product of tile column ti (every tile-row but the
      // last is full, so Y_i has all m rows); V' rows past the column's M
      // belong to the next column or to the zero rows after the last, and
      // their products are not stored
      if (ti + 1 < p.nt) {
        const long z0 = p.zcol[ti], M = p.zcol[ti + 1] - z0;
        const double* Vj = Vpack + z0 * m;
        const long* zd = p.zdst + z0;
        for (long r0 = 0; r0 < M; r0 += P::kRows) {
          P::AccV acc[P::kRows / 16][4];
          quad_zero<P>(acc);
          quad_gemm<P>(sh, acc, m / P::kK, [&](int s, P::Regs& rg) {
            P::load(Vj, m, 0, r0, (long)s * P::kK, Yi, 0, rg);
          });
#pragma unroll
          for (int ib = 0; ib < P::kRows / 16; ++ib)
#pragma unroll
            for (int jb = 0; jb < 4; ++jb)
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const long rho = r0 + 16 * ib + P::row_of(lane, r);
                if (rho < M) Z[zd[rho] * kQC + 64 * w + 16 * jb + (lane & 15)] = acc[ib][jb][r];
              }
        }
        __syncthreads();  // Z rows written before the next tile-rows read them
      }
    }
    if (ln.valid) p.ell[ln.col] = logprod_log(prod);
  }
}

hipError_t launch_quad_tlr_sweep(const TlrSweepArgs& a, hipStream_t st) {
  const dim3 g(a.grid), b(256);
  if (a.prefix) hipLaunchKernelGGL(quad_tlr_kernel<true>, g, b, 0, st, a);
  else hipLaunchKernelGGL(quad_tlr_kernel<false>, g, b, 0, st, a);
  return hipGetLastError();
}

int quad_sweep_cols() { return kQC; }

// FP64 always runs 64-row blocks; the reduced precisions take rows = 64 or 128.
int quad_wg_per_cu(int prec, int rows) {
  switch (prec) {
    case 0: return QuadLds<QuadF64>::kWG;
    case 1: return rows == 128 ? QuadLds<QuadF32<128>>::kWG : QuadLds<QuadF32<64>>::kWG;
    case 2: return rows == 128 ? QuadLds<QuadBF16<1, 128>>::kWG : QuadLds<QuadBF16<1, 64>>::kWG;
    default: return rows == 128 ? QuadLds<QuadBF16<2, 128>>::kWG : QuadLds<QuadBF16<2, 64>>::kWG;
  }
}

long quad_yslice(int prec, int ld) {
  switch (prec) {
    case 0: return QuadF64::yslice(ld);
    case 1: return QuadF32<64>::yslice(ld);
    case 2: return QuadBF16<1, 64>::yslice(ld);
    default: return QuadBF16<2, 64>::yslice(ld);
  }
}

template <bool PREFIX>
static hipError_t launch_quad_t(const SweepArgs& a, hipStream_t st) {
  const dim3 g(a.grid), b(256);
  const bool r128 = a.rows == 128;
  switch (a.prec) {
    case 0: hipLaunchKernelGGL((quad_sweep_kernel<QuadF64, PREFIX>), g, b, 0, st, a); break;
    case 1:
      if (r128) hipLaunchKernelGGL((quad_sweep_kernel<QuadF32<128>, PREFIX>), g, b, 0, st, a);
      else hipLaunchKernelGGL((quad_sweep_kernel<QuadF32<64>, PREFIX>), g, b, 0, st, a);
      break;
    case 2:
      if (r128) hipLaunchKernelGGL((quad_sweep_kernel<QuadBF16<1, 128>, PREFIX>), g, b, 0, st, a);
      else hipLaunchKernelGGL((quad_sweep_kernel<QuadBF16<1, 64>, PREFIX>), g, b, 0, st, a);
      break;
    case 3:
      if (r128) hipLaunchKernelGGL((quad_sweep_kernel<QuadBF16<2, 128>, PREFIX>), g, b, 0, st, a);
      else hipLaunchKernelGGL((quad_sweep_kernel<QuadBF16<2, 64>, PREFIX>), g, b, 0, st, a);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_quad_sweep(const SweepArgs& a, hipStream_t st) {
  return a.prefix ? launch_quad_t<true>(a, st) : launch_quad_t<false>(a, st);
}

hipError_t launch_quad_batch_sweep(const BatchSweepArgs& a, hipStream_t st) {
  const dim3 g(a.grid), b(256);
  const bool r128 = a.rows == 128;
  switch (a.prec) {
    case 0: hipLaunchKernelGGL(quad_batch_kernel<QuadF64>, g, b, 0, st, a); break;
    case 1:
      if (r128) hipLaunchKernelGGL(quad_batch_kernel<QuadF32<128>>, g, b, 0, st, a);
      else hipLaunchKernelGGL(quad_batch_kernel<QuadF32<64>>, g, b, 0, st, a);
      break;
    case 2:
      if (r128) hipLaunchKernelGGL((quad_batch_kernel<QuadBF16<1, 128>>), g, b, 0, st, a);
      else hipLaunchKernelGGL((quad_batch_kernel<QuadBF16<1, 64>>), g, b, 0, st, a);
      break;
    case 3:
      if (r128) hipLaunchKernelGGL((quad_batch_kernel<QuadBF16<2, 128>>), g, b, 0, st, a);
      else hipLaunchKernelGGL((quad_batch_kernel<QuadBF16<2, 64>>), g, b, 0, st, a);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace mvn
