// The dense FP64 SOV sweep (Algorithms 2-3 with Eq. (sov1)) for few samples:
// 16 or 32 sample columns per workgroup of three waves, with the limit-update
// GEMM of the next block row computed while the current one is conditioned.
//
// With N*S = 10^4 the 64-column sweep has 157 workgroups for 256 CUs, and
// each one's time is its own chain: n conditioning steps (about 1 us each,
// one wave) plus its GEMM on one CU, alone, at half the CU's MFMA rate.  It
// took the same time for 64 samples as for 10^4.  Here:
//   * narrower chunks give 4x / 2x as many workgroups, each with a quarter /
//     half of the GEMM work;
//   * wave 0 only conditions: per 32-row block it runs the recurrence
//       s_i = S_i + sum_{k in block, k < i} L_ik y_k,
//       (y_i, d_i) = condition_step((a~_i - s_i)/L_ii, (b~_i - s_i)/L_ii, w_i)
//     with the block's triangle of L, its limits and QMC points from LDS,
//     P = 64 / C lanes per sample column splitting the dot product (summed
//     by DPP within the quad or pair), and stores y to LDS and to the
//     workgroup's Y scratch;
//   * meanwhile waves 1 and 2 accumulate S_{r+1} = L[block r+1, 0:i0] Y[0:i0]
//     on MFMA, each over all 32 rows and the 16-deep K stages of one parity
//     (so the workgroup reads its Y slice once per block, not once per
//     wave), with operands loaded straight into registers (no LDS stage, so
//     no barrier inside the K loop); they stage the next block's triangle,
//     limits and QMC points into the other half of double-buffered LDS and
//     load L[block r+1, block r];
//   * after the block, each adds its half of L[block r+1, block r] y_r (y_r
//     from LDS) and writes its partial S_{r+1} to LDS (the conditioning
//     wave adds the two): two barriers per 32 rows.
// The recurrence thus never waits on the GEMM except for that last product
// (eight MFMAs per wave), and with several workgroups per CU the MFMA work
// of some overlaps the conditioning of others.
//
// Measured on one box (FP64, 4096 sites): 9.2-10.3 ms for 10^4 samples
// against 11.9 ms for the 64-column sweep, 5.3 against 11.8 ms for 2560.
// The chain alone (the GEMM loop removed in a timing copy) takes 5.9-6.4 ms,
// 1.45 us per row; the rest is the GEMM, whose waves wait on their loads.
// Each workgroup streams the whole factor and re-reads its Y slice once per
// 32 rows; splitting K instead of rows between the two GEMM waves took
// 8192 sites, 10^4 samples from 39 to 31 ms (the 64-column sweep: 32 ms).
//
// The Y scratch is laid out for the B operand: element (k, c) of a
// workgroup's slice at ((k / 4) C + c) 4 + k % 4, so a lane's four k values
// of one MFMA group are 32 contiguous bytes.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "gemm_f64.h"
#include "launch.h"
#include "mvn_device.h"
#include "sweep_block.h"

namespace mvn {

constexpr int kNR = 32;         // rows per block
constexpr int kNThreads = 192;  // wave 0 conditions, waves 1-2 run the GEMM
constexpr int kNFLd = kNR + 1;  // LDS row stride of the closing product's L tile

typedef __attribute__((ext_vector_type(2))) double n_f64x2;

// K columns per register stage: 16 (A 8 doubles for the two 16-row tiles,
// B 4 or 8 per lane).
template <int C>
struct NarrowShape {
  static constexpr int kCT = C / 16;         // 16-column MFMA tiles
  static constexpr int kKS = 16;
  static constexpr int kSub = kKS / 16;      // 16-deep groups per stage
  static constexpr int kP = 64 / C;          // conditioning lanes per sample column
};

// One register stage of the GEMM: a[rt][s][j] = L[16 rt + r, k0 + 16 s + 4 q + j],
// b[t][s][j] = Y(k0 + 16 s + 4 q + j, 16 t + r) for lane (r = lane & 15,
// q = lane >> 4).
template <int C>
struct NarrowRegs {
  double a[2][NarrowShape<C>::kSub][4];
  double b[NarrowShape<C>::kCT][NarrowShape<C>::kSub][4];
};

template <int C>
__device__ __forceinline__ void narrow_load(const double* __restrict__ Arow, long ld, const double* __restrict__ Bq,
                                            int k0, NarrowRegs<C>& g) {
  using Sh = NarrowShape<C>;
#pragma unroll
  for (int s = 0; s < Sh::kSub; ++s) {
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      const n_f64x2* pa = (const n_f64x2*)(Arow + (long)rt * 16 * ld + k0 + 16 * s);
      const n_f64x2 a0 = pa[0], a1 = pa[1];
      g.a[rt][s][0] = a0.x;
      g.a[rt][s][1] = a0.y;
      g.a[rt][s][2] = a1.x;
      g.a[rt][s][3] = a1.y;
    }
#pragma unroll
    for (int t = 0; t < Sh::kCT; ++t) {
      const n_f64x2* pb = (const n_f64x2*)(Bq + (long)(k0 + 16 * s) * C + 64 * t);
      const n_f64x2 b0 = pb[0], b1 = pb[1];
      g.b[t][s][0] = b0.x;
      g.b[t][s][1] = b0.y;
      g.b[t][s][2] = b1.x;
      g.b[t][s][3] = b1.y;
    }
  }
}

// Accumulators: one 16 x 16 tile per row tile and column tile; with one
// column tile, two chains (alternate groups) so that consecutive MFMAs on a
// tile are independent.
template <int C>
struct NarrowAcc {
  static constexpr int kChains = NarrowShape<C>::kCT == 1 ? 2 : 1;
  f64x4 v[kChains][2][NarrowShape<C>::kCT];
};

template <int C>
__device__ __forceinline__ void narrow_mma(const NarrowRegs<C>& g, NarrowAcc<C>& acc) {
  using Sh = NarrowShape<C>;
#pragma unroll
  for (int s = 0; s < Sh::kSub; ++s)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int t = 0; t < Sh::kCT; ++t) {
          f64x4& d = acc.v[(s * 4 + j) % NarrowAcc<C>::kChains][rt][t];
          d = __builtin_amdgcn_mfma_f64_16x16x4f64(g.a[rt][s][j], g.b[t][s][j], d, 0, 0, 0);
        }
}

// LDS of one workgroup: S of the block (written by the GEMM waves), y of the
// block (written by wave 0), the L tile of the closing product, and
// double-buffered per-block inputs of the recurrence.
template <int C>
struct NarrowLds {
  double S[kNR * C];       // S of the block: the even K stages and the closing product's first half
  double S1[kNR * C];      // the odd K stages and its second half (added by the conditioning wave)
  double Yb[kNR * C];
  double F[kNR * kNFLd];  // L[block r+1, block r]
  double W[2][kNR * C];   // QMC points
  double D[2][kNR * kNR]; // the diagonal block of L, strictly lower part (row-major)
  double at[2][kNR], bt[2][kNR], rl[2][kNR];
  double tab[48];         // AS 241 coefficients
};

// Stage the inputs of block i0 (rows < n) into buffer `buf` (GEMM waves,
// u = thread - 64 in 0..127).  Rows and columns up to the padded leading
// dimension exist, so the tile copies need no guard.
// The lane index is passed through an empty asm statement so that the
// per-lane offsets are recomputed per block instead of being hoisted out of
// the sweep and held in registers for its whole length.
__device__ __forceinline__ int narrow_opaque(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

template <int C>
__device__ __forceinline__ void narrow_stage(NarrowLds<C>& sh, int buf, int u0, const double* __restrict__ L, long ld,
                                             int n, int i0, const double* __restrict__ at,
                                             const double* __restrict__ bt, const uint64_t* __restrict__ lattice,
                                             uint64_t seed, uint64_t sidx, uint64_t jpt, int periodize) {
  const int u = narrow_opaque(u0);
  const int rows = min(kNR, n - i0);
  // the strictly lower part, zeros from the diagonal on (the recurrence's dot
  // products then run over every k without a branch)
  const double* src = L + (long)(i0 + u / kNR) * ld + i0 + u % kNR;
#pragma unroll
  for (int j = 0; j < kNR * kNR / 128; ++j) {
    const int i = u / kNR + (128 / kNR) * j, k = u % kNR;
    const double v = src[(long)(128 / kNR) * j * ld];
    sh.D[buf][i * kNR + k] = k < i ? v : 0.0;
  }
  if (u < kNR) {
    sh.at[buf][u] = u < rows ? at[i0 + u] : 0.0;
  } else if (u < 2 * kNR) {
    const int i = u - kNR;
    sh.bt[buf][i] = i < rows ? bt[i0 + i] : 0.0;
  } else if (u < 3 * kNR) {
    const int i = u - 2 * kNR;
    sh.rl[buf][i] = i < rows ? 1.0 / L[(long)(i0 + i) * (ld + 1)] : 1.0;
  }
  // QMC points: lane u serves column u % C, rows u / C + (128 / C) j
#pragma unroll
  for (int j = 0; j < kNR * C / 128; ++j) {
    const int i = u / C + (128 / C) * j;
    const uint64_t g = (uint64_t)(i0 + i);
    sh.W[buf][i * C + u % C] =
        i < rows ? richtmyer(jpt, lattice[g], splitmix64(seed, sidx * (uint64_t)n + g), periodize) : 0.5;
  }
}

// Workgroups per CU: three with 16 columns (42 KB of LDS), two with 32
// (58 KB).
constexpr int narrow_wg(int C) { return C == 16 ? 3 : 2; }

template <int C, bool PREFIX>
__global__ __launch_bounds__(kNThreads, narrow_wg(C)) void narrow_sweep_kernel(SweepArgs p) {
  using Sh = NarrowShape<C>;
  __shared__ __attribute__((aligned(16))) NarrowLds<C> sh;
  const int t = threadIdx.x, lane = t & 63;
  // the wave index as a uniform value, so the role branches are scalar
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
  const long NS = (long)p.N * p.S;
  const long nchunks = (NS + C - 1) / C;
  const int n = p.n;
  const long ld = p.ld;
  const int nb = (n + kNR - 1) / kNR;
  double* Y = (double*)p.yscr + (long)blockIdx.x * p.yslice;
  if (t < 48) sh.tab[t] = kAs241[t / 16][t % 16];
  for (int e = t; e < kNR * C; e += kNThreads) sh.Yb[e] = 0.0;
  const lds_f64* tab = (const lds_f64*)sh.tab;
  const auto ninv = [tab](double x) { return ninv_lower_tab(x, tab); };
  // wave 0: sample column lane / P, part lane % P of its dot products
  const int ccol = lane / Sh::kP, part = lane % Sh::kP;
  // GEMM waves: u in 0..127 for staging; wave 1 + kp takes every row of the
  // next block and the K stages of parity kp, so each wave reads its half of
  // the Y slice once per block
  const int u = t - 64, kp = wv - 1;
  for (long chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
    const long col = chunk * C + ccol;
    const bool valid = wv == 0 && col < NS;
    const uint64_t sidx = col < NS ? (uint64_t)(col / p.N) : 0;
    const uint64_t jpt = col < NS ? (uint64_t)(col % p.N) + 1 : 1;
    LogProd prod{1.0, 0};
    const PrefixOut pre{p.prefix, nchunks, chunk, (uint64_t)(chunk * C / p.N)};
    // the staging lane's column (fixed across its rows)
    const long scol = chunk * C + (u & (C - 1));
    const uint64_t ssidx = (wv > 0 && scol < NS) ? (uint64_t)(scol / p.N) : 0;
    const uint64_t sjpt = (wv > 0 && scol < NS) ? (uint64_t)(scol % p.N) + 1 : 1;
    NarrowAcc<C> acc;
#pragma unroll
    for (int c = 0; c < NarrowAcc<C>::kChains; ++c)
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < Sh::kCT; ++ct) acc.v[c][rt][ct] = f64x4{0.0, 0.0, 0.0, 0.0};
      if (wv > 0) narrow_stage<C>(sh, 0, u, p.L, ld, n, 0, p.at, p.bt, p.lattice, p.seed, ssidx, sjpt, p.periodize);
    for (int r = 0; r < nb; ++r) {
      const int i0 = r * kNR, buf = r & 1;
      // ---- phase A: S_r = (L[block r, 0:i0 - 32] Y) + L[block r, block r-1] y_{r-1},
      // as two partial sums: each K parity adds its 16 of the closing
      // product's 32 columns and writes its own array
      if (wv > 0) {
        if (r > 0) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int k = 16 * kp + 4 * (lane >> 4) + j;
#pragma unroll
            for (int rt = 0; rt < 2; ++rt) {
              const double a = sh.F[(16 * rt + (lane & 15)) * kNFLd + k];
#pragma unroll
              for (int ct = 0; ct < Sh::kCT; ++ct) {
                f64x4& d = acc.v[j % NarrowAcc<C>::kChains][rt][ct];
                d = __builtin_amdgcn_mfma_f64_16x16x4f64(a, sh.Yb[k * C + 16 * ct + (lane & 15)], d, 0, 0, 0);
              }
            }
          }
        }
        double* Sd = kp ? sh.S1 : sh.S;
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
          for (int ct = 0; ct < Sh::kCT; ++ct)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              double x = acc.v[0][rt][ct][v];
              if constexpr (NarrowAcc<C>::kChains == 2) x += acc.v[1][rt][ct][v];
              Sd[(16 * rt + (lane >> 4) + 4 * v) * C + 16 * ct + (lane & 15)] = x;
            }
      }
      __syncthreads();  // S_r and the block's inputs are in LDS; Yb is free
      // ---- phase B
      if (wv == 0) {
        const int rows = min(kNR, n - i0);
        const lds_f64* D = (const lds_f64*)sh.D[buf];
        const lds_f64* Wb = (const lds_f64*)sh.W[buf];
        lds_f64* Yb = (lds_f64*)sh.Yb;
        double* Yg = Y + (long)i0 * C + ((long)ccol) * 4;
        for (int i = 0; i < rows; ++i) {
          const int pt = narrow_opaque(part);
          // D is zero from column i on and Yb holds finite values (or the
          // zeros it starts with), so every term of the part can be summed;
          // the part-0 lane starts from the two halves of S (read off the
          // recurrence's dependency chain, summed once by the DPP reduction)
          double s0 = part == 0 ? sh.S[i * C + ccol] : 0.0;
          double s1 = part == 0 ? sh.S1[i * C + ccol] : 0.0;
          const lds_f64* Di = D + i * kNR;
#pragma unroll
          for (int kk = 0; kk < kNR / Sh::kP; kk += 2) {
            const int k = pt + Sh::kP * kk;
            s0 += Di[k] * Yb[k * C + ccol];
            s1 += Di[k + Sh::kP] * Yb[(k + Sh::kP) * C + ccol];
          }
          double s = s0 + s1;
          s += dpp_f64<0xB1>(s);                 // partner lane xor 1
          if constexpr (Sh::kP == 4) s += dpp_f64<0x4E>(s);  // xor 2
          const double rl = sh.rl[buf][i];
          const double alpha = (sh.at[buf][i] - s) * rl;
          const double beta = (sh.bt[buf][i] - s) * rl;
          const double w = Wb[i * C + ccol];
          const Step st = condition_step_with(alpha, beta, w, 1.0 - w, ninv);
          const double y = valid ? st.y : 0.0;
          Yb[i * C + ccol] = y;
          if (part == 0) Yg[(long)(i / 4) * C * 4 + (i & 3)] = y;
          logprod_mul(prod, st);
          if constexpr (PREFIX) prefix_row(prod, valid && part == 0, sidx, pre, (long)(i0 + i));
        }
      } else if (r + 1 < nb) {
        const int i1 = i0 + kNR;
        narrow_stage<C>(sh, buf ^ 1, u, p.L, ld, n, i1, p.at, p.bt, p.lattice, p.seed, ssidx, sjpt, p.periodize);
        const double* Arow = p.L + (long)(i1 + (lane & 15)) * ld + 4 * (lane >> 4);
        const double* Bq = Y + ((long)(lane >> 4) * C + (lane & 15)) * 4;
#pragma unroll
        for (int c = 0; c < NarrowAcc<C>::kChains; ++c)
#pragma unroll
          for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int ct = 0; ct < Sh::kCT; ++ct) acc.v[c][rt][ct] = f64x4{0.0, 0.0, 0.0, 0.0};
        // S_{r+1} over the finished blocks 0..r-1 (K = i0, a multiple of
        // 2 kKS): this wave's stages k0 = kp kKS + 2 kKS m < i0, two register
        // sets in flight
        int k0 = kp * Sh::kKS;
        if (k0 < i0) {
          NarrowRegs<C> g0, g1;
          narrow_load<C>(Arow, ld, Bq, k0, g0);
          for (;;) {
            const int k1 = k0 + 2 * Sh::kKS;
            if (k1 < i0) narrow_load<C>(Arow, ld, Bq, k1, g1);
            narrow_mma<C>(g0, acc);
            if (k1 >= i0) break;
            const int k2 = k1 + 2 * Sh::kKS;
            if (k2 < i0) narrow_load<C>(Arow, ld, Bq, k2, g0);
            narrow_mma<C>(g1, acc);
            if (k2 >= i0) break;
            k0 = k2;
          }
        }
        // the L tile of the closing product with y_r
        const int uf = narrow_opaque(u);
        const double* fsrc = p.L + (long)(i1 + uf / kNR) * ld + i0 + uf % kNR;
#pragma unroll
        for (int j = 0; j < kNR * kNR / 128; ++j)
          sh.F[(uf / kNR + (128 / kNR) * j) * kNFLd + uf % kNR] = fsrc[(long)(128 / kNR) * j * ld];
      }
      __syncthreads();  // y_r in Yb and the Y scratch; the next block's inputs staged
    }
    if (valid && part == 0) p.ell[col] = logprod_log(prod);
  }
}

int narrow_sweep_wg_per_cu(int cols) { return narrow_wg(cols); }

hipError_t launch_narrow_sweep(const SweepArgs& a, hipStream_t st) {
  const dim3 g(a.grid), b(kNThreads);
  if (a.narrow == 16) {
    if (a.prefix)
      hipLaunchKernelGGL((narrow_sweep_kernel<16, true>), g, b, 0, st, a);
    else
      hipLaunchKernelGGL((narrow_sweep_kernel<16, false>), g, b, 0, st, a);
  } else if (a.narrow == 32) {
    if (a.prefix)
      hipLaunchKernelGGL((narrow_sweep_kernel<32, true>), g, b, 0, st, a);
    else
      hipLaunchKernelGGL((narrow_sweep_kernel<32, false>), g, b, 0, st, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace mvn
