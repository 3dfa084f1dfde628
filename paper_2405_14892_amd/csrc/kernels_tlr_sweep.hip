// SOV sweep through a tile low-rank factor (arXiv 2405.14892, Algorithm 2's
// limit update applied through the low-rank tiles of Section III-E; the
// factor layout is described in kernels_tlr.hip).
//
// This file is compiled without machine loop-invariant code motion, like the
// dense sweep: the conditioning step is inlined into the row loop.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "gemm_f64.h"
#include "launch.h"
#include "mvn_device.h"
#include "sweep_block.h"
#include "sweep_gemm.h"

namespace mvn {

// ------------------------------------------------------------ index tables
// The tables of tlr_tables.h (stacked V' rows by tile column, packed K of
// every tile-row, the Z row of every stacked row), built from the ranks on
// the device so that a call never reads them back; then the layout of the
// rank-dependent region (packed operands, then per workgroup a Y and a Z
// slice) and how many workgroups it holds.  One workgroup; pair p = (i, j),
// i > j, has index i (i - 1) / 2 + j.
__device__ __forceinline__ long align256(long x) { return (x + 255) / 256 * 256; }

__global__ __launch_bounds__(1024) void tlr_tables_kernel(TlrTableArgs a) {
  const int t = threadIdx.x, nt = a.nt;
  const long np = (long)nt * (nt - 1) / 2;
  for (long p = t; p < np; p += 1024) {
    const long r = a.ranks[p] < 0 ? -(long)a.ranks[p] : (long)a.ranks[p];
    a.kk[p] = (int)(r > a.rs ? a.rs : r);
  }
  __syncthreads();
  // per tile column j: the sum of its ranks (zcol[j + 1] holds it for now);
  // per tile-row i: the sum of its ranks, and each pair's column within it
  for (int j = t; j < nt; j += 1024) {
    long c = 0;
    for (int i = j + 1; i < nt; ++i) c += a.kk[(long)i * (i - 1) / 2 + j];
    a.zcol[j + 1] = c;
  }
  for (int i = t; i < nt; i += 1024) {
    long c = 0;
    for (int j = 0; j < i; ++j) {
      const long p = (long)i * (i - 1) / 2 + j;
      a.ucol0[p] = c;
      c += a.kk[p];
    }
    a.kval[i] = (int)c;
  }
  __syncthreads();
  if (t == 0) {
    a.zcol[0] = 0;
    a.kpad0[0] = 0;
    for (int j = 0; j < nt; ++j) {
      a.zcol[j + 1] += a.zcol[j];
      a.kpad0[j + 1] = a.kpad0[j] + ((long)a.kval[j] + 15) / 16 * 16;
    }
    TlrSweepHdr h{};
    h.ksum = a.zcol[nt];
    h.kpad = a.kpad0[nt];
    const long m = a.m;
    h.vpack = 0;
    h.upack = a.ext_pack ? 0 : align256(8 * (h.ksum + 128) * m);
    h.yscr = a.ext_pack ? 0 : align256(h.upack + 8 * m * (h.kpad > 0 ? h.kpad : 1));
    h.zslice = (h.kpad > 0 ? h.kpad : 1) * (a.cols > 0 ? a.cols : kCols);
    const long per = align256(8 * a.yslice) + align256(8 * h.zslice);
    const long room = (long)a.dyn_bytes - h.yscr;
    long g = room > 0 ? room / per : 0;
    if (g > a.grid_max) g = a.grid_max;
    h.grid = g;
    h.zscr = align256(h.yscr + 8 * g * a.yslice);
    *a.hdr = h;
    if (g < 1) *a.bad = 0;  // no sweep workgroup fits: the reduction reports NaN
  }
  __syncthreads();
  // first stacked row of each pair, then every stacked row's Z row
  for (int j = t; j < nt; j += 1024) {
    long row = a.zcol[j];
    for (int i = j + 1; i < nt; ++i) {
      const long p = (long)i * (i - 1) / 2 + j;
      a.vrow0[p] = row;
      row += a.kk[p];
    }
  }
  __syncthreads();
  for (long p = t; p < np; p += 1024) {
    int i = (int)((1.0 + sqrt(1.0 + 8.0 * (double)p)) * 0.5);
    while ((long)i * (i - 1) / 2 > p) --i;
    while ((long)(i + 1) * i / 2 <= p) ++i;
    const long base = a.kpad0[i] + a.ucol0[p], r0 = a.vrow0[p];
    for (int q = 0; q < a.kk[p]; ++q) a.zdst[r0 + q] = base + q;
  }
}

hipError_t launch_tlr_tables(const TlrTableArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(tlr_tables_kernel, dim3(1), dim3(1024), 0, st, a);
  return hipGetLastError();
}

// ------------------------------------------------------------ operand packing
// Once per probability call the low-rank factors are copied into the order
// the sweep reads them (tlr_tables.h): the V' rows of every tile (i, j),
// i > j, stacked by tile column j in order of i (Vpack, then 128 zero rows so
// that a 128-row MFMA tile may run past the last column), and per tile-row i
// the U columns of its tiles side by side (Upack_i, m x Kpad_i, zero columns
// up to the multiple of 16).

// Block (p, c): pair p's rows of V' (k_p rows of m doubles), a slice of
// them; block p == np clears the zero tail.
__global__ __launch_bounds__(256) void tlr_pack_v_kernel(const double* __restrict__ Vt, int m, int rs, int np,
                                                         const int* __restrict__ kk,
                                                         const long* __restrict__ vrow0,
                                                         const TlrSweepHdr* __restrict__ hdr, char* dyn) {
  const int p = blockIdx.x;
  const long ksum = hdr->ksum;
  if (hdr->grid < 1) return;
  double* Vpack = (double*)(dyn + hdr->vpack);
  if (p == np) {
    for (long e = (long)blockIdx.y * 256 + threadIdx.x; e < 128L * m; e += 256L * gridDim.y)
      Vpack[ksum * m + e] = 0.0;
    return;
  }
  const long cnt = (long)kk[p] * m;
  const double* src = Vt + (long)p * rs * m;
  double* dst = Vpack + vrow0[p] * m;
  for (long e = (long)blockIdx.y * 256 + threadIdx.x; e < cnt; e += 256L * gridDim.y) dst[e] = src[e];
}

// Block (p, rb): rows rb*64 .. rb*64+63 of pair p = (i, j): U_ij[:, 0:k_p]
// into Upack_i at column ucol0[p]; the block of the pair (i, i - 1) also
// clears the padding columns [K_i, Kpad_i).
__global__ __launch_bounds__(256) void tlr_pack_u_kernel(const double* __restrict__ U, int m, int rs,
                                                         const int* __restrict__ kk,
                                                         const long* __restrict__ ucol0,
                                                         const long* __restrict__ kpad0,
                                                         const int* __restrict__ kval,
                                                         const TlrSweepHdr* __restrict__ hdr, char* dyn) {
  if (hdr->grid < 1) return;
  double* Upack = (double*)(dyn + hdr->upack);
  const int p = blockIdx.x;
  int i = (int)((1.0 + sqrt(1.0 + 8.0 * (double)p)) * 0.5);
  while (i * (i - 1) / 2 > p) --i;
  while ((i + 1) * i / 2 <= p) ++i;
  const int j = p - i * (i - 1) / 2;
  const long Kp = kpad0[i + 1] - kpad0[i];
  double* dst = Upack + kpad0[i] * m;
  const double* src = U + (long)p * m * rs;
  const int r0 = blockIdx.y * 64, kp = kk[p];
  const long c0 = ucol0[p];
  for (int e = threadIdx.x; e < 64 * kp; e += 256) {
    const int row = r0 + e / kp, q = e % kp;
    dst[(long)row * Kp + c0 + q] = src[(long)row * rs + q];
  }
  if (j == i - 1) {
    const int kv = kval[i], pw = (int)(Kp - kv);
    for (int e = threadIdx.x; e < 64 * pw; e += 256) {
      const int row = r0 + e / pw, q = e % pw;
      dst[(long)row * Kp + kv + q] = 0.0;
    }
  }
}

hipError_t launch_tlr_pack(const TlrPackArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(tlr_pack_v_kernel, dim3(a.np + 1, 16), dim3(256), 0, st, a.Vt, a.m, a.rs, a.np, a.kk, a.vrow0,
                     a.hdr, a.dyn);
  if (a.np > 0)
    hipLaunchKernelGGL(tlr_pack_u_kernel, dim3(a.np, a.m / 64), dim3(256), 0, st, a.U, a.m, a.rs, a.kk, a.ucol0,
                       a.kpad0, a.kval, a.hdr, a.dyn);
  return hipGetLastError();
}

// ------------------------------------------------------------ TLR sweep
// Rows [r0, r0 + 32) of the stacked product V_j^T Y_j (rows at or past M
// are dropped; row rho goes to Z row zdst[rho]): a 32 x 64 product with
// K = m split over the four waves, wave w taking k = 64 s + 16 w ..
// 64 s + 16 w + 15 of every 64-deep stage; the four partial products are
// summed through LDS.  Used for the last <= 64 rows of a tile column, where
// a 128-row MFMA tile would be mostly padding.  lds: 8192 doubles.
__device__ __forceinline__ void z_rows32(const double* __restrict__ Vj, int m, long r0, const double* __restrict__ Yj,
                                         double* __restrict__ Z, const long* __restrict__ zdst, long M,
                                         double* lds) {
  constexpr int kALd = 32 + 1, kBLd = 64 + 1;
  constexpr int kAW = 16 * kALd, kBW = 16 * kBLd;  // one wave's A / B slice
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  double* As = lds;
  double* Bs = lds + 4 * kAW;
  f64x4 acc[2][4];
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) acc[ib][jb] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int nst = m / 64;
  double ra[8], rb[16];
  // lane t loads 8 k of A row t / 8 and 16 columns of B row t / 4
  auto load = [&](int s) {
    const double2* pa = reinterpret_cast<const double2*>(Vj + (r0 + (t >> 3)) * m + s * 64 + (t & 7) * 8);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double2 v = pa[q];
      ra[2 * q] = v.x;
      ra[2 * q + 1] = v.y;
    }
    const double2* pb = reinterpret_cast<const double2*>(Yj + (long)(s * 64 + (t >> 2)) * kCols + (t & 3) * 16);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double2 v = pb[q];
      rb[2 * q] = v.x;
      rb[2 * q + 1] = v.y;
    }
  };
  load(0);
  for (int s = 0; s < nst; ++s) {
    {
      const int wa = (t & 7) >> 1, k0 = (t & 1) * 8, row = t >> 3;
#pragma unroll
      for (int q = 0; q < 8; ++q) As[wa * kAW + (k0 + q) * kALd + row] = ra[q];
      const int kb = t >> 2, c0 = (t & 3) * 16;
#pragma unroll
      for (int q = 0; q < 16; ++q) Bs[(kb >> 4) * kBW + (kb & 15) * kBLd + c0 + q] = rb[q];
    }
    __syncthreads();
    if (s + 1 < nst) load(s + 1);
    const double* Aw = As + w * kAW;
    const double* Bw = Bs + w * kBW;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int k = kk * 4 + (lane >> 4);
      double a[2], b[4];
#pragma unroll
      for (int ib = 0; ib < 2; ++ib) a[ib] = Aw[k * kALd + ib * 16 + (lane & 15)];
#pragma unroll
      for (int jb = 0; jb < 4; ++jb) b[jb] = Bw[k * kBLd + jb * 16 + (lane & 15)];
#pragma unroll
      for (int ib = 0; ib < 2; ++ib)
#pragma unroll
        for (int jb = 0; jb < 4; ++jb)
          acc[ib][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ib], b[jb], acc[ib][jb], 0, 0, 0);
    }
    __syncthreads();
  }
  double* part = lds;  // 4 x 32 x 64
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        part[w * 2048 + (ib * 16 + (lane >> 4) + 4 * q) * kCols + jb * 16 + (lane & 15)] = acc[ib][jb][q];
  __syncthreads();
  for (int e = t; e < 32 * kCols; e += 256) {
    const long rho = r0 + e / kCols;
    if (rho < M)
      Z[zdst[rho] * kCols + (e & (kCols - 1))] = (part[e] + part[2048 + e]) + (part[4096 + e] + part[6144 + e]);
  }
  __syncthreads();
}

// The sweep of one 64-column chunk through a TLR factor.  For tile-row i:
//   for each RB-row block b of the tile:
//     S_b = [U_i0 .. U_i,i-1][b, :] [Z_i0; ..] + L_ii[b, <b] Y_i[<b]
//         (one K loop: the packed low-rank products, then the dense part)
//     conditioning of the block with the dense L_ii, as in the dense sweep;
//   then, Y_i being known, the stacked product of tile column i:
//     [Z_(i+1)i; Z_(i+2)i; ..] = [V'_(i+1)i^T; V'_(i+2)i^T; ..] Y_i
//         (M = sum of the column's ranks, K = m; FP64 MFMA in RB-row tiles,
//         with 32-row split-K products for the last <= 64 rows when RB is
//         128), whose rows are stored at their places in the packed Z of the
//         tile-rows below.
// Z lives in the workgroup's slice of the Z scratch (Kpad_total x 64), whose
// padding rows are cleared once and never written.  RB = 128: two
// workgroups per CU; RB = 64: four (more sample chunks conditioned at once).
template <int RB, bool PREFIX = false>
__global__ __launch_bounds__(256, RB == 128 ? 2 : 4) void tlr_sweep_kernel(TlrSweepArgs p) {
  using G = GemmF64T<RB>;
  constexpr int kT = SweepLdsSize<G>::kT;
  static_assert(RB == 64 || kT >= 8192, "the 32-row split-K product needs 8192 doubles");
  __shared__ __attribute__((aligned(16))) double lds_T[kT];
  __shared__ double lds_slab[kSlab * RB];
  __shared__ double c_at[RB], c_bt[RB], c_rl[RB];
  __shared__ uint64_t c_lat[RB];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int m = p.m;
  const long NS = (long)p.N * p.S;
  const long nchunks = (NS + kCols - 1) / kCols;
  const TlrSweepHdr h = *p.hdr;
  if ((long)blockIdx.x >= h.grid) return;  // the workspace holds h.grid workgroups
  const double* Vpack = p.vpack_ext ? p.vpack_ext : (const double*)(p.dyn + h.vpack);
  const double* Upack = p.upack_ext ? p.upack_ext : (const double*)(p.dyn + h.upack);
  double* Y = (double*)(p.dyn + h.yscr) + (long)blockIdx.x * p.yslice;
  double* Z = (double*)(p.dyn + h.zscr) + (long)blockIdx.x * h.zslice;
  char* stage0 = (char*)lds_T;
  char* stage1 = (char*)lds_T + G::kStageBytes;

  for (int i = 1; i < p.nt; ++i)
    for (long e = (p.kpad0[i] + p.kval[i]) * kCols + t; e < p.kpad0[i + 1] * kCols; e += 256) Z[e] = 0.0;

  for (long chunk = blockIdx.x; chunk < nchunks; chunk += h.grid) {
    const long col = chunk * kCols + lane;
    const bool owner = wv == 0;
    const bool valid = owner && col < NS;
    const uint64_t sidx = col < NS ? (uint64_t)(col / p.N) : 0;  // every lane: its own column
    const uint64_t jpt = col < NS ? (uint64_t)(col % p.N) + 1 : 1;
    LogProd prod{1.0, 0};
    const PrefixOut pre{p.prefix, nchunks, chunk, (uint64_t)(chunk * kCols / p.N)};
    for (int ti = 0; ti < p.nt; ++ti) {
      const long g0 = (long)ti * m;
      const long kp0 = p.kpad0[ti], Kp = p.kpad0[ti + 1] - kp0;
      const int nst_lr = (int)(Kp / G::kK);
      const double* Ui = Upack + kp0 * m;  // m x Kp
      const double* Zi = Z + kp0 * kCols;
      const double* D = p.tiles + (p.diag_compact ? (long)ti : (long)ti * (ti + 1) / 2 + ti) * (long)m * m;
      for (int b0 = 0; b0 < m && g0 + b0 < p.n; b0 += RB) {
        const int rows = (int)min((long)RB, p.n - (g0 + b0));
        typename G::Acc acc;
        G::zero(acc);
        const int nst = nst_lr + b0 / G::kK;
        if (nst > 0) {
          auto load_stage = [&](int s, typename G::Regs& rg) {
            if (s < nst_lr) G::load(Ui, Kp, 0, b0, (long)s * G::kK, Zi, Kp, rg);
            else G::load(D, m, 0, b0, (long)(s - nst_lr) * G::kK, Y + g0 * kCols, m, rg);
          };
          typename G::Regs rg;
          load_stage(0, rg);
          G::store(stage0, rg);
          __syncthreads();
          for (int s = 0; s < nst; ++s) {
            const bool odd = s & 1;
            if (s + 1 < nst) load_stage(s + 1, rg);
            G::mma(odd ? stage1 : stage0, acc);
            if (s + 1 < nst) G::store(odd ? stage0 : stage1, rg);
            __syncthreads();
          }
        }
        G::to_block(acc, lds_T);
        if (t < rows) {
          const long g = g0 + b0 + t;
          c_at[t] = p.at[g];
          c_bt[t] = p.bt[g];
          c_rl[t] = 1.0 / D[(long)(b0 + t) * m + b0 + t];
          c_lat[t] = p.lattice[g];
        }
        prod = condition_block<false, RB, true, PREFIX>((lds_f64*)lds_T, (lds_f64*)lds_slab, (const lds_f64*)c_at,
                                                        (const lds_f64*)c_bt, (const lds_f64*)c_rl,
                                                        (const lds_u64*)c_lat, D, m, b0, rows, p.n, jpt, sidx, p.seed,
                                                        p.periodize, valid, prod, nullptr, (int)g0, pre);
        __syncthreads();
        for (int e = t; e < rows * kCols; e += 256) Y[(g0 + b0) * kCols + e] = lds_T[e];
        __syncthreads();
      }
      // ---- stacked product of tile column ti
      if (ti + 1 < p.nt) {
        const long z0 = p.zcol[ti], M = p.zcol[ti + 1] - z0;
        const double* Vj = Vpack + z0 * m;
        const double* Yj = Y + g0 * kCols;
        const long* zd = p.zdst + z0;
        long r0 = 0;
        for (; M - r0 > (RB == 128 ? 64 : 0); r0 += RB) {
          typename G::Acc acc;
          G::zero(acc);
          const int nst = m / G::kK;
          typename G::Regs rg;
          G::load(Vj, m, 0, r0, 0, Yj, m, rg);
          G::store(stage0, rg);
          __syncthreads();
          for (int s = 0; s < nst; ++s) {
            const bool odd = s & 1;
            if (s + 1 < nst) G::load(Vj, m, 0, r0, (long)(s + 1) * G::kK, Yj, m, rg);
            G::mma(odd ? stage1 : stage0, acc);
            if (s + 1 < nst) G::store(odd ? stage0 : stage1, rg);
            __syncthreads();
          }
          G::to_block(acc, lds_T);
          __syncthreads();
          for (int e = t; e < RB * kCols; e += 256) {
            const long rho = r0 + e / kCols;
            if (rho < M) Z[zd[rho] * kCols + (e & (kCols - 1))] = lds_T[e];
          }
          __syncthreads();
        }
        if constexpr (RB == 128)
          for (; r0 < M; r0 += 32) z_rows32(Vj, m, r0, Yj, Z, zd, M, lds_T);
      }
    }
    if (valid) p.ell[col] = logprod_log(prod);
  }
}

hipError_t launch_tlr_sweep(const TlrSweepArgs& a, hipStream_t st) {
  if (a.rows == 256) return launch_quad_tlr_sweep(a, st);
  const dim3 g(a.grid), b(256);
  if (a.prefix) {
    if (a.rows == 64) hipLaunchKernelGGL((tlr_sweep_kernel<64, true>), g, b, 0, st, a);
    else hipLaunchKernelGGL((tlr_sweep_kernel<128, true>), g, b, 0, st, a);
  } else {
    if (a.rows == 64) hipLaunchKernelGGL((tlr_sweep_kernel<64, false>), g, b, 0, st, a);
    else hipLaunchKernelGGL((tlr_sweep_kernel<128, false>), g, b, 0, st, a);
  }
  return hipGetLastError();
}

}  // namespace mvn
