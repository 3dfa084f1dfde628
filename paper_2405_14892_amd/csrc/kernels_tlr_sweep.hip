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

// ------------------------------------------------------------ TLR sweep
// Rows [r0, r0 + 32) of Z = V'^T Y_j (rows at or past rs are dropped): a
// 32 x 64 product with K = m split over the four waves, wave w taking
// k = 64 s + 16 w .. 64 s + 16 w + 15 of every 64-deep stage; the four
// partial products are summed through LDS.  Used for ranks <= 64, where a
// 128-row MFMA tile would be mostly zero rows.  lds: 8192 doubles.
__device__ __forceinline__ void z_rows32(const double* __restrict__ Vp, int m, int r0, const double* __restrict__ Yj,
                         double* __restrict__ Zj, int rs, double* lds) {
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
    const double2* pa = reinterpret_cast<const double2*>(Vp + (long)(r0 + (t >> 3)) * m + s * 64 + (t & 7) * 8);
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
  for (int e = t; e < 32 * kCols; e += 256)
    if (r0 + e / kCols < rs) Zj[(long)r0 * kCols + e] = (part[e] + part[2048 + e]) + (part[4096 + e] + part[6144 + e]);
  __syncthreads();
}


// The sweep of one 64-column chunk through a TLR factor.  For tile-row i:
//   Z_ij = V'^T_ij Y_j for j < i                       (r_ij x 64, FP64 MFMA,
//                                                      K = m)
//   for each 128-row block b of the tile:
//     S_b = sum_{j<i} U_ij[b, :] Z_ij + L_ii[b, <b] Y_i[<b]   (one K loop
//                                                      over all terms)
//     conditioning of the block with the dense L_ii, as in the dense sweep.
// Z lives in the workgroup's slice of the Z scratch ((nt - 1) x rs x 64).
__global__ __launch_bounds__(256, 2) void tlr_sweep_kernel(TlrSweepArgs p) {
  using G = GemmF64;
  static_assert(2 * G::kStageBytes <= kTile * kCols * 8, "GEMM stages must fit in the block buffer");
  __shared__ __attribute__((aligned(16))) double lds_T[kTile * kCols];
  __shared__ double lds_slab[kSlab * kTile];
  __shared__ double c_at[kTile], c_bt[kTile], c_rl[kTile];
  __shared__ uint64_t c_lat[kTile];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int m = p.m, rs = p.rs;
  const long NS = (long)p.N * p.S;
  const long nchunks = (NS + kCols - 1) / kCols;
  double* Y = p.yscr + (long)blockIdx.x * p.yslice;
  double* Z = p.zscr + (long)blockIdx.x * p.zslice;
  char* stage0 = (char*)lds_T;
  char* stage1 = (char*)lds_T + G::kStageBytes;

  for (long chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
    const long col = chunk * kCols + lane;
    const bool owner = wv == 0;
    const bool valid = owner && col < NS;
    const uint64_t sidx = valid ? (uint64_t)(col / p.N) : 0;
    const uint64_t jpt = valid ? (uint64_t)(col % p.N) + 1 : 1;
    LogProd prod{1.0, 0};
    for (int ti = 0; ti < p.nt; ++ti) {
      const long g0 = (long)ti * m;
      const long prow = (long)ti * (ti - 1) / 2;  // panel index of (ti, 0)
      // ---- Z_ij = V'^T_ij Y_j, j < ti
      for (int tj = 0; tj < ti; ++tj) {
        const int rk = abs(p.ranks[prow + tj]);
        const double* Vp = p.Vt + (prow + tj) * (long)rs * m;
        const double* Yj = Y + (long)tj * m * kCols;
        double* Zj = Z + (long)tj * rs * kCols;
        if (rk <= 64) {
          for (int r0 = 0; r0 < rk; r0 += 32) z_rows32(Vp, m, r0, Yj, Zj, rs, lds_T);
          continue;
        }
        for (int r0 = 0; r0 < rk; r0 += kTile) {
          G::Acc acc;
          G::zero(acc);
          const int nst = m / G::kK;
          G::Regs rg;
          G::load(Vp, m, 0, r0, 0, Yj, m, rg);
          G::store(stage0, rg);
          __syncthreads();
          for (int s = 0; s < nst; ++s) {
            const bool odd = s & 1;
            if (s + 1 < nst) G::load(Vp, m, 0, r0, (long)(s + 1) * G::kK, Yj, m, rg);
            G::mma(odd ? stage1 : stage0, acc);
            if (s + 1 < nst) G::store(odd ? stage0 : stage1, rg);
            __syncthreads();
          }
          G::to_block(acc, lds_T);
          __syncthreads();
          for (int e = t; e < kTile * kCols; e += 256)
            if (r0 + e / kCols < rs) Zj[(long)r0 * kCols + e] = lds_T[e];
          __syncthreads();
        }
      }
      // K stages of the low-rank terms of this tile-row
      int nst_lr = 0;
      for (int tj = 0; tj < ti; ++tj) nst_lr += (abs(p.ranks[prow + tj]) + G::kK - 1) / G::kK;
      const double* D = p.tiles + ((long)ti * (ti + 1) / 2 + ti) * (long)m * m;
      for (int b0 = 0; b0 < m && g0 + b0 < p.n; b0 += kTile) {
        const int rows = (int)min((long)kTile, p.n - (g0 + b0));
        G::Acc acc;
        G::zero(acc);
        const int nst = nst_lr + b0 / G::kK;
        if (nst > 0) {
          int cj = 0, ck = 0;  // cursor over the low-rank stages: panel (ti, cj), stage ck
          auto load_stage = [&](int s, G::Regs& rg) {
            if (s < nst_lr) {
              while (ck * G::kK >= abs(p.ranks[prow + cj])) {
                ++cj;
                ck = 0;
              }
              G::load(p.U + (prow + cj) * (long)m * rs, rs, 0, b0, (long)ck * G::kK,
                      Z + (long)cj * rs * kCols, rs, rg);
              ++ck;
            } else {
              G::load(D, m, 0, b0, (long)(s - nst_lr) * G::kK, Y + g0 * kCols, m, rg);
            }
          };
          G::Regs rg;
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
        prod = condition_block((lds_f64*)lds_T, (lds_f64*)lds_slab, (const lds_f64*)c_at, (const lds_f64*)c_bt,
                               (const lds_f64*)c_rl, (const lds_u64*)c_lat, D, m, b0, rows, p.n, jpt, sidx,
                               p.seed, p.periodize, valid, prod, nullptr, (int)g0);
        __syncthreads();
        for (int e = t; e < rows * kCols; e += 256) Y[(g0 + b0) * kCols + e] = lds_T[e];
        __syncthreads();
      }
    }
    if (valid) p.ell[col] = logprod_log(prod);
  }
}

hipError_t launch_tlr_sweep(const TlrSweepArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(tlr_sweep_kernel, dim3(a.grid), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace mvn
