// Step 2 of the SOV sweep (conditioning of one 128-row diagonal block),
// shared by the probability sweep and the forward half of the adjoint sweep.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gemm_f64.h"
#include "mvn_device.h"
#include "sweep_gemm.h"

namespace mvn {

constexpr int kSlab = 8;  // rows of the diagonal block of L staged per LDS slab

typedef __attribute__((address_space(3))) double lds_f64;
typedef __attribute__((address_space(3))) uint64_t lds_u64;

// Running products of every row for the nested-set probabilities of
// confidence-region detection (Section III-C with Algorithm 1 of Section IV-A): after row r the
// wave's samples' products m 2^e are summed exactly in base 2, split by
// shift (slot 0: the chunk's first shift, slot 1: the next one; a chunk of
// 64 consecutive samples meets at most two shifts when N >= 64), and stored
// as (E, v) with sum = v 2^E at part[(r * nchunks + chunk) * 4 + 2 slot].
struct PrefixOut {
  double* part;
  long nchunks, chunk;
  uint64_t s_first;
};

constexpr int kNoExp = -(1 << 30);  // exponent of an empty sum

// Wave64 reductions on DPP moves (no LDS crossbar): xor 1 and 2 inside each
// quad, the half-row and row mirrors (8- and 16-lane groups), then the row
// 15 / lane 31 broadcasts that fold rows 0-1 into 1 and 0-1 into 2-3; lane 63
// ends with the whole wave, read back as a uniform value.  Lanes of a row
// that a broadcast does not write take the identity.
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ int dpp_i32(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWS, 0xF, false);
}

template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp_f64(double v) {  // identity 0.0 (all bits zero)
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = dpp_i32<CTRL, ROWS>(0, (int)b), hi = dpp_i32<CTRL, ROWS>(0, (int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ int wave_max_i32(int x) {
  x = max(x, dpp_i32<0xB1>(kNoExp, x));        // quad_perm [1, 0, 3, 2]
  x = max(x, dpp_i32<0x4E>(kNoExp, x));        // quad_perm [2, 3, 0, 1]
  x = max(x, dpp_i32<0x141>(kNoExp, x));       // row_half_mirror
  x = max(x, dpp_i32<0x140>(kNoExp, x));       // row_mirror
  x = max(x, dpp_i32<0x142, 0xA>(kNoExp, x));  // row_bcast15 into rows 1 and 3
  x = max(x, dpp_i32<0x143, 0xC>(kNoExp, x));  // row_bcast31 into rows 2 and 3
  return __builtin_amdgcn_readlane(x, 63);
}

__device__ __forceinline__ double wave_sum_f64(double x) {
  x += dpp_f64<0xB1>(x);
  x += dpp_f64<0x4E>(x);
  x += dpp_f64<0x141>(x);
  x += dpp_f64<0x140>(x);
  x += dpp_f64<0x142, 0xA>(x);
  x += dpp_f64<0x143, 0xC>(x);
  const long long b = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_readlane((int)b, 63), hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ void prefix_row(const LogProd& prod, bool valid, uint64_t sidx, const PrefixOut& pre,
                                           long row) {
  const bool live = valid && prod.m > 0.0;
  const bool first = sidx == pre.s_first;
  const int e0 = wave_max_i32((live && first) ? prod.e : kNoExp);
  const int e1 = wave_max_i32((live && !first) ? prod.e : kNoExp);
  const double v0 = wave_sum_f64((live && first) ? ldexp(prod.m, prod.e - e0) : 0.0);
  const double v1 = wave_sum_f64((live && !first) ? ldexp(prod.m, prod.e - e1) : 0.0);
  if ((threadIdx.x & 63) == 0) {
    double* d = pre.part + (row * pre.nchunks + pre.chunk) * 4;
    d[0] = (double)e0;
    d[1] = v0;
    d[2] = (double)e1;
    d[3] = v1;
  }
}

// The in-block recurrence runs in 32-row sub-blocks: once
// sub-block rows [c0, c0 + 32) hold y, every wave adds L_rr(r, c0:c0+32) y
// to the rows r >= c0 + 32 of T on MFMA (16-row tiles, tile b on wave b mod
// 4), so wave 0's dot product per row only runs over its own sub-block.
constexpr int kCondSub = 32;

__device__ __forceinline__ void subblock_update(lds_f64* T, const double* __restrict__ L, long ld, int i0, int c0,
                                                int rows) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r0 = c0 + kCondSub;
  const int nblk = (rows - r0 + 15) / 16;
  for (int b = w; b < nblk; b += 4) {
    const int rb = r0 + 16 * b;
    f64x4 acc[4];
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[jb][r] = T[(rb + (lane >> 4) + 4 * r) * kCols + jb * 16 + (lane & 15)];
    const double* Lr = L + (long)(i0 + rb + (lane & 15)) * ld + i0 + c0 + (lane >> 4);
#pragma unroll
    for (int kk = 0; kk < kCondSub / 4; ++kk) {
      const double a = Lr[4 * kk];
      const int k = c0 + 4 * kk + (lane >> 4);
#pragma unroll
      for (int jb = 0; jb < 4; ++jb)
        acc[jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, T[k * kCols + jb * 16 + (lane & 15)], acc[jb], 0, 0, 0);
    }
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
      for (int r = 0; r < 4; ++r) T[(rb + (lane >> 4) + 4 * r) * kCols + jb * 16 + (lane & 15)] = acc[jb][r];
  }
}

// Step 2 of the sweep for one 128-row block, called by all 256 lanes once per
// block: rows of the diagonal block of L are staged 8 at a time in LDS (all
// lanes), and wave 0 (lane = sample column) runs the recurrence
//   s_i = S_i + sum_{k<i} L_ik y_k,  a' = (a~_i - s_i)/L_ii,
//   b' = (b~_i - s_i)/L_ii,  (y_i, d_i) = condition_step(a', b', w_i),
// leaving y_i in T and folding d_i into the sample's running product
// (and, for the adjoint, s_i in s_out[(i0 + i) * 64 + lane]).  MIXED selects
// the reduced-precision step (FP32 central Phi / Phi^-1); SL is the slab row
// stride (the block's row count, rows <= SL).  L and the
// row indices are local to a diagonal tile starting at global row goff
// (0 for a dense factor); goff + i0 + i is the QMC dimension of row i.
// This file is compiled without machine loop-invariant code motion: hoisting
// the step's ~60 polynomial constants out of the row loop would pin them in
// registers next to the GEMM's accumulators and force spills (build.py).
// TAB: the AS 241 coefficients from a 384-byte LDS table (else selected
// between constants; for kernels whose LDS is already at its budget).
// PREFIX: the running products of every row go to pre (prefix_row).
template <bool MIXED = false, int SL = kTile, bool TAB = true, bool PREFIX = false>
__device__ __forceinline__ LogProd condition_block(
    lds_f64* T, lds_f64* slab, const lds_f64* c_at, const lds_f64* c_bt, const lds_f64* c_rl,
    const lds_u64* c_lat, const double* __restrict__ L, long ld, int i0, int rows, int n,
    uint64_t jpt, uint64_t sidx, uint64_t seed, int periodize, bool valid, LogProd prod,
    double* __restrict__ s_out = nullptr, int goff = 0, PrefixOut pre = PrefixOut{}) {
  const int t = threadIdx.x, lane = t & 63;
  const bool owner = (t >> 6) == 0;
  // the AS 241 coefficient rows in LDS, written by wave 1 (ordered before
  // wave 0's first read by the slab loop's barrier)
  const lds_f64* tab = nullptr;
  if constexpr (TAB) {
    __shared__ double ninv_tab[48];
    if ((t >> 6) == 1) {
#pragma unroll
      for (int e = 0; e < 48; ++e)
        if (lane == e) ninv_tab[e] = kAs241[e / 16][e % 16];
    }
    tab = (const lds_f64*)ninv_tab;
  }
  const auto ninv = [tab](double x) { return TAB ? ninv_lower_tab(x, tab) : ninv_lower(x); };
  // Slabs of the diagonal block.  128-row blocks: waves 1-3 fetch slab q + 1
  // into registers while wave 0 runs the rows of slab q, so the recurrence
  // does not wait on global memory (the LDS holds one slab; two barriers per
  // slab).  64-row blocks (four workgroups per CU, no register headroom):
  // every lane loads the slab between the two barriers.
  // The slab of a 128-row block holds the 8 rows' entries in the columns of
  // their 32-row sub-block (all that wave 0's dot products read), then the
  // rows' QMC points for the 64 sample columns, which waves 1-3 compute
  // ahead (every lane's jpt and sidx are its own column's).
  constexpr bool kPF = SL >= 128;
  constexpr int kSlabL = kSlab * kCondSub;                   // L part of a slab
  constexpr int kPerL = kPF ? (kSlabL + 191) / 192 : 1;      // L entries per fetching lane
  constexpr int kPerW = (kSlab + 2) / 3;                     // QMC rows per fetching wave
  static_assert(!kPF || kSlabL + kSlab * kCols <= kSlab * SL, "slab too small for the QMC points");
  double pf[kPerL], pw[kPerW];
  const int u = t - 64;         // fetching lane, 0..191 in waves 1-3
  const int wf = (t >> 6) - 1;  // fetching wave, 0..2
  const auto fetch = [&](int q) {
    const int kb = q & ~(kCondSub - 1);
#pragma unroll
    for (int j = 0; j < kPerL; ++j) {
      const int e = u + 192 * j, ii = e / kCondSub, k = kb + e % kCondSub;
      pf[j] = (e < kSlabL && q + ii < rows && k < q + ii) ? L[(long)(i0 + q + ii) * ld + i0 + k] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < kPerW; ++j) {
      const int ii = wf + 3 * j;
      pw[j] = (ii < kSlab && q + ii < rows)
                  ? richtmyer(jpt, c_lat[q + ii], splitmix64(seed, sidx * (uint64_t)n + (uint64_t)(goff + i0 + q + ii)),
                              periodize)
                  : 0.0;
    }
  };
  const auto put = [&]() {
#pragma unroll
    for (int j = 0; j < kPerL; ++j) {
      const int e = u + 192 * j;
      if (e < kSlabL) slab[e] = pf[j];
    }
#pragma unroll
    for (int j = 0; j < kPerW; ++j) {
      const int ii = wf + 3 * j;
      if (ii < kSlab) slab[kSlabL + ii * kCols + lane] = pw[j];
    }
  };
  if constexpr (kPF) {
    __syncthreads();  // T and the per-row constants are complete; slab is free
    if (!owner) {
      fetch(0);
      put();
    }
  }
  for (int q = 0; q < rows; q += kSlab) {
    if constexpr (kPF) {
      __syncthreads();  // slab q in LDS
      if (!owner && q + kSlab < rows) fetch(q + kSlab);
    } else {
      __syncthreads();  // rows < q hold y
      if (q > 0 && q % kCondSub == 0) subblock_update(T, L, ld, i0, q - kCondSub, rows);
      for (int e = t; e < kSlab * SL; e += 256) {
        const int ii = e / SL, k = e % SL;
        slab[e] = (q + ii < rows && k < q + ii) ? L[(long)(i0 + q + ii) * ld + i0 + k] : 0.0;
      }
      __syncthreads();
    }
    if (owner) {
      const int iend = min(q + kSlab, rows);
      for (int i = q; i < iend; ++i) {
        // the slab row is zero from column i on, so the sum runs to a
        // multiple of 8 with four independent partial sums (the LDS reads
        // then pipeline)
        const lds_f64* Tk = T + lane;
        double s0 = T[i * kCols + lane], s1 = 0.0, s2 = 0.0, s3 = 0.0;
        const int kend = (i + 7) & ~7;
        // earlier sub-blocks are already folded into T
        const int kbeg = i & ~(kCondSub - 1);
        // slab row of i, indexed by block column (128-row slabs start at column kbeg)
        const lds_f64* Li = kPF ? slab + (i - q) * kCondSub - kbeg : slab + (i - q) * SL;
        for (int k = kbeg; k < kend; k += 8) {
          s0 += Li[k] * Tk[k * kCols];
          s1 += Li[k + 1] * Tk[(k + 1) * kCols];
          s2 += Li[k + 2] * Tk[(k + 2) * kCols];
          s3 += Li[k + 3] * Tk[(k + 3) * kCols];
          s0 += Li[k + 4] * Tk[(k + 4) * kCols];
          s1 += Li[k + 5] * Tk[(k + 5) * kCols];
          s2 += Li[k + 6] * Tk[(k + 6) * kCols];
          s3 += Li[k + 7] * Tk[(k + 7) * kCols];
        }
        const double sum = (s0 + s1) + (s2 + s3);
        if (s_out) s_out[(long)(i0 + i) * kCols + lane] = sum;
        const double rl = c_rl[i];
        const double alpha = (c_at[i] - sum) * rl;
        const double beta = (c_bt[i] - sum) * rl;
        const uint64_t g = (uint64_t)(goff + i0 + i);
        const double w = kPF ? (double)slab[kSlabL + (i - q) * kCols + lane]
                             : richtmyer(jpt, c_lat[i], splitmix64(seed, sidx * (uint64_t)n + g), periodize);
        const Step st = MIXED ? condition_step_mixed_with(alpha, beta, w, 1.0 - w, ninv)
                              : condition_step_with(alpha, beta, w, 1.0 - w, ninv);
        T[i * kCols + lane] = valid ? st.y : 0.0;
        logprod_mul(prod, st);
        if constexpr (PREFIX) prefix_row(prod, valid, sidx, pre, (long)(goff + i0 + i));
      }
    }
    if constexpr (kPF) {
      if (q + kSlab < rows) {
        __syncthreads();  // wave 0 is done with slab q (and rows <= q + 7 hold y)
        if (!owner) put();
        if ((q + kSlab) % kCondSub == 0) subblock_update(T, L, ld, i0, q + kSlab - kCondSub, rows);
      }
    }
  }
  return prod;
}

}  // namespace mvn
