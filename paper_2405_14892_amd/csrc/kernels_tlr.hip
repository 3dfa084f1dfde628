// Tile low-rank (TLR) factorisation (arXiv 2405.14892, Section III-E for the
// tile compression; Algorithm 1's factorisation in its TLR form).  The sweep
// through a TLR factor is in kernels_tlr_sweep.hip.
//
// Storage (device, inside the caller's factor buffer):
//   tiles  lower m x m tiles, tile-major: tile (i, j), j <= i, at
//          (i(i+1)/2 + j) m^2 doubles, row-major with leading dimension m;
//          rows / columns past n hold the identity.  After the
//          factorisation the diagonal tiles hold L_ii (upper part zero) and
//          the off-diagonal tiles the updated A_ij they were compressed from.
//   U      panel (i, k), i > k, at (i(i-1)/2 + k) m rs doubles: m x rs
//          row-major (rs = rank stride, a multiple of 16)
//   Vt     panel (i, k) at (i(i-1)/2 + k) rs m doubles: rs x m row-major,
//          holding V'^T = (L_kk^{-1} V)^T, so that L_ik = U_ik V'^T_ik;
//          followed by 128 rows of slack so that 128-row GEMM loads of the
//          last panel stay inside the buffer
//   ranks  int per panel; negative if the rank cap stopped the compression
//          before the residual reached eps (|rank| is used)
// Columns of U and rows of Vt past the rank are zero, so GEMMs whose K is
// the rank rounded up to 16 are exact.
//
// Factorisation over tile columns; the tiles not yet factored are kept
// dense and every update uses the low-rank factors:
//   1. L_kk = chol(A_kk)                        (the dense tiled Cholesky)
//   2. A_ik ~ U_ik V_ik^T, i > k                (adaptive cross
//      approximation, stopped only when the exact residual Frobenius norm is
//      <= eps, so ||A_ik - U V^T||_2 <= eps as for the truncated SVD)
//   3. V'^T_ik = V^T_ik L_kk^{-T}               (row solves)
//   4. A_ij -= U_ik (V'^T_ik V'_jk) U_jk^T       (FP64 MFMA GEMMs whose
//      dimensions come from the device rank table)
// The updates are applied left-looking: all of a tile's updates are summed
// in one segmented-K GEMM just before its column is factored.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "gemm_f64.h"
#include "launch.h"
#include "mvn_device.h"

namespace mvn {

__device__ __forceinline__ long tri_lo(long i, long j) { return i * (i + 1) / 2 + j; }   // j <= i
__device__ __forceinline__ long tri_st(long i, long k) { return i * (i - 1) / 2 + k; }   // k < i

// b = i(i+1)/2 + j with 0 <= j <= i
__device__ __forceinline__ void tri_inverse(long b, long& i, long& j) {
  long t = (long)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
  while ((t + 1) * (t + 2) / 2 <= b) ++t;
  while (t * (t + 1) / 2 > b) --t;
  i = t;
  j = b - t * (t + 1) / 2;
}

// ------------------------------------------------------------ build
// One 64 x 64 sub-block of one lower tile per workgroup; clears *info.
__global__ __launch_bounds__(256) void tlr_build_kernel(int n, int m, const double* __restrict__ sigma, int lds,
                                                        const int64_t* __restrict__ perm,
                                                        const int* __restrict__ perm_bad,
                                                        const double* __restrict__ locs, Matern mk,
                                                        double* __restrict__ tiles, int* __restrict__ info) {
  const long per = (long)(m / 64) * (m / 64);
  const long t = blockIdx.x / per, sb = blockIdx.x % per;
  const bool bad = perm && perm_bad && *perm_bad != 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) *info = bad ? -1 : 0;
  long ti, tj;
  tri_inverse(t, ti, tj);
  const long r0 = (sb / (m / 64)) * 64, c0 = (sb % (m / 64)) * 64;
  double* A = tiles + t * (long)m * m;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const long lr = r0 + (e >> 6), lc = c0 + (e & 63);
    const long i = ti * m + lr, j = tj * m + lc;
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
    A[lr * m + lc] = v;
  }
}

// ------------------------------------------------------------ compression
// Block-wide reductions over the 256 lanes: a shuffle tree inside each
// wave64, then the four wave results through LDS (ties to the lower index).
__device__ __forceinline__ void block_argmax(double v, int idx, double* sv, int* si, double& best, int& bidx) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(v, off);
    const int oi = __shfl_xor(idx, off);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
  if (lane == 0) {
    sv[w] = v;
    si[w] = idx;
  }
  __syncthreads();
  best = sv[0];
  bidx = si[0];
#pragma unroll
  for (int q = 1; q < 4; ++q)
    if (sv[q] > best || (sv[q] == best && si[q] < bidx)) {
      best = sv[q];
      bidx = si[q];
    }
  __syncthreads();
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ __forceinline__ double block_sum(double v, double* sv) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  v = wave_sum(v);
  if (lane == 0) sv[w] = v;
  __syncthreads();
  const double r = (sv[0] + sv[1]) + (sv[2] + sv[3]);
  __syncthreads();
  return r;
}

// Two sums in one exchange.
__device__ __forceinline__ void block_sum2(double& a, double& b, double* sv) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  a = wave_sum(a);
  b = wave_sum(b);
  if (lane == 0) {
    sv[w] = a;
    sv[4 + w] = b;
  }
  __syncthreads();
  a = (sv[0] + sv[1]) + (sv[2] + sv[3]);
  b = (sv[4] + sv[5]) + (sv[6] + sv[7]);
  __syncthreads();
}

// ||A - U V^T||_F^2 for one m x m tile: U (m x rs, row-major) and V^T
// (rs x m, row-major), both zero past column / row kr (a multiple of 16).
// The product runs on FP64 MFMA in 128 x 128 blocks (the kernel's LDS stage
// buffers); every lane then folds its accumulator entries against A.
__device__ __forceinline__ double residual_norm2(const double* __restrict__ A, int m, const double* __restrict__ Up, int rs,
                                 const double* __restrict__ Vp, int kr, double* lds, double* sv) {
  double res2 = 0.0;
  const int nb = m / kTile, nst = kr / kStageK;
  for (int bb = 0; bb < nb * nb; ++bb) {
    const int bi = bb / nb, bj = bb % nb;
    Acc acc;
    acc_zero(acc);
    if (nst > 0) {
      double ra[8], rb[8];
      load_rows<false>(Up, rs, (long)bi * kTile, 0, 0, 0, ra);
      load_cols(Vp + (long)bj * kTile, m, 0, rb);
      store_rows(lds, ra);
      store_cols(lds + kStageDoubles, rb);
      __syncthreads();
      for (int s = 0; s < nst; ++s) {
        double* cur = lds + (s & 1) * 2 * kStageDoubles;
        double* nxt = lds + ((s + 1) & 1) * 2 * kStageDoubles;
        if (s + 1 < nst) {
          load_rows<false>(Up, rs, (long)bi * kTile, (long)(s + 1) * kStageK, 0, 0, ra);
          load_cols(Vp + (long)bj * kTile, m, (long)(s + 1) * kStageK, rb);
        }
        mma_stage(cur, cur + kStageDoubles, acc);
        if (s + 1 < nst) {
          store_rows(nxt, ra);
          store_cols(nxt + kStageDoubles, rb);
        }
        __syncthreads();
      }
    }
#pragma unroll
    for (int ib = 0; ib < 4; ++ib)
#pragma unroll
      for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const long gi = (long)bi * kTile + acc_row(ib, q), gj = (long)bj * kTile + acc_col(jb);
          const double d = A[gi * m + gj] - acc.v[ib][jb][q];
          res2 += d * d;
        }
  }
  return block_sum(res2, sv);
}

// Partially pivoted cross approximation of panel tile (k + 1 + i0 + blockIdx.x,
// k), one workgroup per tile.  Each step takes the residual row at the pivot row,
// the pivot column at its largest entry among unused columns, the residual
// column there, and the next pivot row at that column's largest entry among
// unused rows.  When ||u|| ||v|| <= eps / 4 (or the rank reaches the cap) the
// exact residual ||A - U V^T||_F is formed, and the approximation is accepted
// only if it is <= eps; otherwise the crosses continue and the next check
// waits max(2, r / 8) crosses.  (A first check at eps / 2 usually fails on
// the adjacent tiles and its retry lands past the needed rank.)  A row whose residual
// vanishes is skipped; if every row has been used the approximation is exact.
// Lane t owns columns (row residual) and rows (column residual) 4t .. 4t + 3,
// read as 16-byte pairs; the columns of U are also kept transposed in the
// workgroup's slot of Ut (rs x m) for that.  The residuals are summed in the
// same order as with any other lane mapping, and ties in the pivot search go
// to the lowest index, so the crosses do not depend on the mapping.
__global__ __launch_bounds__(256) void tlr_aca_kernel(const double* __restrict__ tiles, int k, int i0, int m,
                                                      int rs, int rcap, double eps, double* __restrict__ U,
                                                      double* __restrict__ Vt, int* __restrict__ ranks,
                                                      double* __restrict__ Ut, const int* __restrict__ info) {
  if (*info != 0) return;
  __shared__ double row[kTlrMaxTile];
  __shared__ unsigned char urow[kTlrMaxTile], ucol[kTlrMaxTile];
  __shared__ double sv[256];
  __shared__ int si[256];
  __shared__ int s_next;
  __shared__ double lds[4 * kStageDoubles];
  __shared__ double uq[kTlrMaxRank];  // U row irow, then V^T column jp
  const int t = threadIdx.x;
  const long i = k + 1 + i0 + blockIdx.x;
  const double* A = tiles + tri_lo(i, k) * (long)m * m;
  double* Utp = Ut + (long)blockIdx.x * rs * m;
  const long pid = tri_st(i, k);
  double* Up = U + pid * (long)m * rs;
  double* Vp = Vt + pid * (long)rs * m;
  for (long e = t; e < (long)m * rs; e += 256) {
    Up[e] = 0.0;
    Vp[e] = 0.0;
  }
  for (int e = t; e < m; e += 256) urow[e] = ucol[e] = 0;
  __syncthreads();
  int r = 0, irow = 0, flag = 0, next_check = 0;
  for (int guard = 0; guard < 2 * m; ++guard) {
    bool check = false;
    // residual row irow: lane t holds columns 4t .. 4t + 3 (lanes past m / 4
    // idle), read as 16-byte pairs so that each load instruction moves 1 KB
    const bool act = 4 * t < m;
    double best = -1.0;
    int bj = 0;
    {
      double v[4] = {0.0, 0.0, 0.0, 0.0};
      if (act) {
        const double2* pa = reinterpret_cast<const double2*>(A + (long)irow * m + 4 * t);
        const double2 a0 = pa[0], a1 = pa[1];
        v[0] = a0.x; v[1] = a0.y; v[2] = a1.x; v[3] = a1.y;
      }
      if (t < r) uq[t] = Up[(long)irow * rs + t];
      __syncthreads();
      if (act) {
#pragma unroll 8
        for (int q = 0; q < r; ++q) {
          const double u = uq[q];
          const double2* pv = reinterpret_cast<const double2*>(Vp + (long)q * m + 4 * t);
          const double2 b0 = pv[0], b1 = pv[1];
          v[0] -= u * b0.x;
          v[1] -= u * b0.y;
          v[2] -= u * b1.x;
          v[3] -= u * b1.y;
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int j = 4 * t + c;
          row[j] = v[c];
          if (!ucol[j] && fabs(v[c]) > best) {
            best = fabs(v[c]);
            bj = j;
          }
        }
      }
    }
    double piv;
    int jp;
    block_argmax(best, bj, sv, si, piv, jp);
    if (t == 0) urow[irow] = 1;
    __syncthreads();
    if (!(piv > 0.0)) {
      // this row's residual is zero: take the first unused row, or stop
      if (t == 0) {
        int nx = -1;
        for (int e = 0; e < m; ++e)
          if (!urow[e]) {
            nx = e;
            break;
          }
        s_next = nx;
      }
      __syncthreads();
      const int nx = s_next;
      __syncthreads();
      if (nx < 0) break;  // every row used: the approximation is exact
      irow = nx;
      continue;
    }
    if (r == rcap) {
      flag = 1;  // a further cross is needed but the cap is reached
      break;
    }
    double nu2 = 0.0, nv2 = 0.0;
    const double p = row[jp];
    if (act) {
      double2 w0, w1;
      w0.x = row[4 * t] / p;
      w0.y = row[4 * t + 1] / p;
      w1.x = row[4 * t + 2] / p;
      w1.y = row[4 * t + 3] / p;
      double2* pv = reinterpret_cast<double2*>(Vp + (long)r * m + 4 * t);
      pv[0] = w0;
      pv[1] = w1;
      nv2 = (w0.x * w0.x + w0.y * w0.y) + (w1.x * w1.x + w1.y * w1.y);
    }
    // residual column jp (U_(:, r)), lane t holding rows 4t .. 4t + 3 and
    // reading the earlier columns of U from their transposed copy; next
    // pivot row
    double cb = -1.0;
    int bi = 0;
    {
      double v[4] = {0.0, 0.0, 0.0, 0.0};
      if (act) {
#pragma unroll
        for (int c = 0; c < 4; ++c) v[c] = A[(long)(4 * t + c) * m + jp];
      }
      __syncthreads();  // every lane is done with uq (row residual)
      if (t < r) uq[t] = Vp[(long)t * m + jp];
      __syncthreads();
      if (act) {
#pragma unroll 8
        for (int q = 0; q < r; ++q) {
          const double vq = uq[q];
          const double2* pu = reinterpret_cast<const double2*>(Utp + (long)q * m + 4 * t);
          const double2 u0 = pu[0], u1 = pu[1];
          v[0] -= u0.x * vq;
          v[1] -= u0.y * vq;
          v[2] -= u1.x * vq;
          v[3] -= u1.y * vq;
        }
        double2* pw = reinterpret_cast<double2*>(Utp + (long)r * m + 4 * t);
        pw[0] = double2{v[0], v[1]};
        pw[1] = double2{v[2], v[3]};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int ii = 4 * t + c;
          Up[(long)ii * rs + r] = v[c];
          nu2 += v[c] * v[c];
          if (!urow[ii] && fabs(v[c]) > cb) {
            cb = fabs(v[c]);
            bi = ii;
          }
        }
      }
    }
    if (t == 0) ucol[jp] = 1;
    block_sum2(nu2, nv2, sv);
    double cbest;
    int ip;
    block_argmax(cb, bi, sv, si, cbest, ip);
    ++r;
    if (cbest >= 0.0) {
      irow = ip;
    } else {
      check = true;  // every row used
    }
    if ((sqrt(nu2 * nv2) <= 0.25 * eps && r >= next_check) || r == rcap) check = true;
    if (!check) continue;
    // exact residual; after a failed check the next one waits a few crosses
    const double res2 = residual_norm2(A, m, Up, rs, Vp, (r + 15) & ~15, lds, sv);
    next_check = r + max(2, r / 8);
    if (res2 <= eps * eps) break;
    if (cbest < 0.0) break;  // rows exhausted; what is left is rounding
    if (r == rcap) {
      flag = 1;
      break;
    }
  }
  if (t == 0) ranks[pid] = flag ? -r : r;
}

// ------------------------------------------------------------ row solves
// x L_kk^T = b for every rank row of every panel of step k (the rows of Vt),
// one wave per row and four rows per workgroup (grid: panels x rs / 4).
// Lane c owns column c0 + c of the current 64-column block: the part of its
// sum over earlier blocks is a dot product against rows of L_kk staged in
// LDS; inside the block a 64-step forward substitution broadcasts each
// solved value from its lane.
__global__ __launch_bounds__(256) void tlr_trsm_rows_kernel(const double* __restrict__ tiles, int k, int m,
                                                            int rs, double* __restrict__ Vt,
                                                            const int* __restrict__ ranks,
                                                            const int* __restrict__ info) {
  if (*info != 0) return;
  __shared__ double Ls[64][64 + 1];
  __shared__ double rd[64];
  __shared__ double xs[4][kTlrMaxTile];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const long i = k + 1 + blockIdx.x;
  const long pid = tri_st(i, k);
  const int rk = abs(ranks[pid]);
  if ((int)blockIdx.y * 4 >= rk) return;  // uniform over the workgroup
  const int row = blockIdx.y * 4 + w;
  const bool live = row < rk;
  const double* L = tiles + tri_lo(k, k) * (long)m * m;
  double* x = Vt + pid * (long)rs * m + (long)(live ? row : 0) * m;
  for (int c0 = 0; c0 < m; c0 += 64) {
    double acc = live ? x[c0 + lane] : 0.0;
    for (int l0 = 0; l0 < c0; l0 += 64) {
      __syncthreads();
      for (int e = t; e < 64 * 64; e += 256) Ls[e >> 6][e & 63] = L[(long)(c0 + (e >> 6)) * m + l0 + (e & 63)];
      __syncthreads();
      double a0 = 0.0, a1 = 0.0;
#pragma unroll 8
      for (int ll = 0; ll < 64; ll += 2) {
        a0 += xs[w][l0 + ll] * Ls[lane][ll];
        a1 += xs[w][l0 + ll + 1] * Ls[lane][ll + 1];
      }
      acc -= a0 + a1;
    }
    __syncthreads();
    for (int e = t; e < 64 * 64; e += 256) {
      const int rr = e >> 6, ll = e & 63;
      Ls[rr][ll] = ll <= rr ? L[(long)(c0 + rr) * m + c0 + ll] : 0.0;
    }
    if (t < 64) rd[t] = 1.0 / L[(long)(c0 + t) * m + c0 + t];
    __syncthreads();
    double xv = 0.0;
    for (int c = 0; c < 64; ++c) {
      const double xc = __shfl(acc, c) * rd[c];
      if (lane == c) xv = xc;
      if (lane > c) acc -= xc * Ls[lane][c];
    }
    xs[w][c0 + lane] = xv;
    if (live) x[c0 + lane] = xv;
  }
}

// ------------------------------------------------------------ recompression
// After the factorisation every panel L_ik = U V'^T (rank 2 <= r <= 192,
// not capped) is recompressed to the smallest rank whose error in the tile
// it approximates stays within eps (Section III-E: the truncated SVD of the
// tile, here taken within the column and row spaces the cross approximation
// found).  With V = L_kk V' (A_ik ~ U V^T):
//   1. G_u = U^T U = D_u Lu Lu^T D_u and G_v = V^T V = D_v Lv Lv^T D_v
//      (D: square roots of the diagonals, Lu, Lv: Cholesky factors of the
//      equilibrated Grams), so Q_u = U D_u^-1 Lu^-T and
//      Q_v = V D_v^-1 Lv^-T are orthonormal bases of those spaces;
//   2. B = Q_u^T A Q_v = Lu^-1 (D_u^-1 U^T A V D_v^-1) Lv^-T: the tile's
//      projection onto them, whose residual ||A - Q_u B Q_v^T|| is orthogonal
//      to any change inside them;
//   3. B B^T = W diag(sigma^2) W^T by cyclic Jacobi (the disjoint rotations of
//      a round-robin schedule applied together; the matrix packed in LDS, so
//      ranks up to 192; W in the scratch);
//   4. k = the smallest rank whose discarded sum of sigma^2 is <= f eps^2
//      (f = 0.95, then 0.7, 0.4), and with W_k the top k vectors
//        U2 = U X_u, X_u = D_u^-1 Lu^-T W_k;  V2'^T = X_v^T V'^T,
//        X_v = D_v^-1 Lv^-T B^T W_k
//      (U2 V2^T = Q_u W_k W_k^T B Q_v^T, the best rank-k approximation of
//      the tile within those spaces);
//   5. the new factors replace the old ones only if the exact residual
//      ||A - U2 V2^T||_F (V2^T = X_v^T V^T) is <= eps.
// Small products on MFMA in 128 x 128 blocks with masked, double-buffered
// LDS stages; triangular solves one vector per lane against the factor
// packed in LDS.  One workgroup per CU takes the panels in order of
// distance from the diagonal, each with its own scratch.
// Stage loads of the small products, masked at the operand edges: lane t
// holds 8 values of one stage (k row t / 16, columns 8 (t % 16) .. + 7 for a
// k-major operand; row t / 2, k 8 (t % 2) .. + 7 for a row-major one).
__device__ __forceinline__ void rc_load8(const double* __restrict__ p, bool full, int nv, double (&r)[8]) {
  if (full && (((uintptr_t)p & 15) == 0)) {
    const double2* p2 = reinterpret_cast<const double2*>(p);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double2 v = p2[q];
      r[2 * q] = v.x;
      r[2 * q + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q) r[q] = q < nv ? p[q] : 0.0;
  }
}
__device__ __forceinline__ void rc_load_kmaj(const double* __restrict__ A, long lda, int na, int K, int k0,
                                             double (&r)[8]) {
  const int t = threadIdx.x, k = k0 + (t >> 4), cb = (t & 15) * 8;
  const int nv = k < K ? min(8, na - cb) : 0;
  rc_load8(A + (long)k * lda + cb, nv >= 8, nv, r);
}
__device__ __forceinline__ void rc_load_rmaj(const double* __restrict__ A, long lda, int na, int K, int k0,
                                             double (&r)[8]) {
  const int t = threadIdx.x, row = t >> 1, kb = k0 + (t & 1) * 8;
  const int nv = row < na ? min(8, K - kb) : 0;
  rc_load8(A + (long)row * lda + kb, nv >= 8, nv, r);
}

// One 128 x 128 block: acc = A^T B (TN: both operands k-major) or A B^T
// (both row-major), K in stages of 16 through double-buffered LDS.
template <bool TN>
__device__ __forceinline__ void rc_block(const double* __restrict__ A, long lda, int na, const double* __restrict__ B,
                                         long ldb, int nb, int K, Acc& acc, double* lds) {
  const int nst = (K + kStageK - 1) / kStageK;
  if (nst == 0) return;
  double ra[8], rb[8];
  const auto load = [&](int k0) {
    if (TN) {
      rc_load_kmaj(A, lda, na, K, k0, ra);
      rc_load_kmaj(B, ldb, nb, K, k0, rb);
    } else {
      rc_load_rmaj(A, lda, na, K, k0, ra);
      rc_load_rmaj(B, ldb, nb, K, k0, rb);
    }
  };
  const auto store = [&](double* st) {
    if (TN) {
      store_cols(st, ra);
      store_cols(st + kStageDoubles, rb);
    } else {
      store_rows(st, ra);
      store_rows(st + kStageDoubles, rb);
    }
  };
  load(0);
  __syncthreads();  // the LDS's previous use is over
  store(lds);
  __syncthreads();
  for (int s = 0; s < nst; ++s) {
    double* cur = lds + (s & 1) * 2 * kStageDoubles;
    double* nxt = lds + ((s + 1) & 1) * 2 * kStageDoubles;
    if (s + 1 < nst) load((s + 1) * kStageK);
    mma_stage(cur, cur + kStageDoubles, acc);
    if (s + 1 < nst) store(nxt);
    __syncthreads();
  }
}

// C = A^T B (TN; A[k lda + i], B[k ldb + j]) or A B^T (NT; A[i lda + k],
// B[j ldb + k]) for i < M, j < N (operands zero past na / nb, k past K), in
// 128 x 128 blocks; out of line so that the recompression's many products
// share one body and its registers.
template <bool TN>
__device__ __noinline__ void rc_gemm(const double* __restrict__ A, long lda, int na, const double* __restrict__ B,
                                     long ldb, int nb, int K, double* __restrict__ C, long ldc, int M, int N,
                                     double* lds) {
  for (int tm = 0; tm * kTile < M; ++tm)
    for (int tn = 0; tn * kTile < N; ++tn) {
      const double* Ab = TN ? A + tm * kTile : A + (long)tm * kTile * lda;
      const double* Bb = TN ? B + tn * kTile : B + (long)tn * kTile * ldb;
      Acc acc;
      acc_zero(acc);
      rc_block<TN>(Ab, lda, na - tm * kTile, Bb, ldb, nb - tn * kTile, K, acc, lds);
      const int mm = min(kTile, M - tm * kTile), nn = min(kTile, N - tn * kTile);
      double* Cb = C + (long)tm * kTile * ldc + tn * kTile;
#pragma unroll
      for (int ib = 0; ib < 4; ++ib)
#pragma unroll
        for (int jb = 0; jb < 4; ++jb)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int i = acc_row(ib, q), j = acc_col(jb);
            if (i < mm && j < nn) Cb[(long)i * ldc + j] = acc.v[ib][jb][q];
          }
    }
}

// Thin products for ranks up to 32, operands loaded straight into registers
// (each entry of the m x m tile is used once: no LDS stage, no barrier).
// Wave w takes the 16-row tiles w, w + 4, ...; for MFMA j of a 16-deep step
// k0, lane (r = lane & 15, q = lane >> 4) supplies its A row's and its B row's
// values at k = k0 + 4q + j (the same bijection of k for both operands).
struct RcThin {
  double a[4];
  double b[2][4];
};

__device__ __forceinline__ void rc_thin_load(const double* __restrict__ pa, const double* __restrict__ pb0,
                                             const double* __restrict__ pb1, bool v0, bool v1, int k0, RcThin& g) {
  const double2* a2 = reinterpret_cast<const double2*>(pa + k0);
  const double2 a0 = a2[0], a1 = a2[1];
  g.a[0] = a0.x; g.a[1] = a0.y; g.a[2] = a1.x; g.a[3] = a1.y;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    g.b[0][j] = v0 ? pb0[k0 + j] : 0.0;
    g.b[1][j] = v1 ? pb1[k0 + j] : 0.0;
  }
}

__device__ __forceinline__ void rc_thin_mma(const RcThin& g, f64x4& c0, f64x4& c1) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(g.a[j], g.b[0][j], c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(g.a[j], g.b[1][j], c1, 0, 0, 0);
  }
}

// C = A B^T: rows i < M (a multiple of 16) of A (lda), rows j < N <= 32 of
// B (ldb), k < K (a multiple of 16), or k < 16 (tile + 1) with LOWER (A lower
// triangular).  TRANSC stores C^T (C[j ldc + i]).
template <bool LOWER, bool TRANSC>
__device__ __noinline__ void rc_thin_nt(const double* __restrict__ A, long lda, int M, const double* __restrict__ B,
                                        long ldb, int N, int K, double* __restrict__ C, long ldc) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, r = lane & 15, q = lane >> 4;
  const bool v0 = r < N, v1 = 16 + r < N;
  const double* pb0 = B + (long)(v0 ? r : 0) * ldb + 4 * q;
  const double* pb1 = B + (long)(v1 ? 16 + r : 0) * ldb + 4 * q;
  for (int rt = w; rt * 16 < M; rt += 4) {
    const int kmax = LOWER ? min(K, 16 * (rt + 1)) : K;
    const double* pa = A + (long)(16 * rt + r) * lda + 4 * q;
    f64x4 c0 = {0.0, 0.0, 0.0, 0.0}, c1 = {0.0, 0.0, 0.0, 0.0};
    RcThin g0, g1, g2;
    rc_thin_load(pa, pb0, pb1, v0, v1, 0, g0);
    if (16 < kmax) rc_thin_load(pa, pb0, pb1, v0, v1, 16, g1);
    for (int k0 = 0; k0 < kmax; k0 += 48) {
      if (k0 + 32 < kmax) rc_thin_load(pa, pb0, pb1, v0, v1, k0 + 32, g2);
      rc_thin_mma(g0, c0, c1);
      if (k0 + 16 >= kmax) break;
      if (k0 + 48 < kmax) rc_thin_load(pa, pb0, pb1, v0, v1, k0 + 48, g0);
      rc_thin_mma(g1, c0, c1);
      if (k0 + 32 >= kmax) break;
      if (k0 + 64 < kmax) rc_thin_load(pa, pb0, pb1, v0, v1, k0 + 64, g1);
      rc_thin_mma(g2, c0, c1);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const long i = 16 * rt + q + 4 * v;
      if (v0) {
        if (TRANSC) C[(long)r * ldc + i] = c0[v]; else C[i * ldc + r] = c0[v];
      }
      if (v1) {
        if (TRANSC) C[(long)(16 + r) * ldc + i] = c1[v]; else C[i * ldc + 16 + r] = c1[v];
      }
    }
  }
}

// ||A - U2 V2^T||_F^2 for the m x m tile A, U2 and V2 (m x K row-major, ld,
// K <= 32 and a multiple of 16, columns past the rank zero): per 16-row tile
// and pair of 16-column tiles, the product on MFMA folded against A, with the
// next pair's operands loaded ahead.
__device__ __noinline__ double rc_thin_residual(const double* __restrict__ A, int m, const double* __restrict__ U2,
                                                const double* __restrict__ V2, int ld, int K, double* sv) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, r = lane & 15, q = lane >> 4;
  double res2 = 0.0;
  for (int rt = w; rt * 16 < m; rt += 4) {
    const double* pa = U2 + (long)(16 * rt + r) * ld + 4 * q;
    double ua[2][4];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int j = 0; j < 4; ++j) ua[s][j] = 16 * s < K ? pa[16 * s + j] : 0.0;
    const double* arow = A + (long)(16 * rt + q) * m + r;
    // stage: B operands of two column tiles and the A entries they meet
    double vb[2][2][4], av[2][4];
    const auto load = [&](int ct) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const double* pv = V2 + (long)(16 * (ct + h) + r) * ld + 4 * q;
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int j = 0; j < 4; ++j) vb[h][s][j] = 16 * s < K ? pv[16 * s + j] : 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) av[h][v] = arow[(long)4 * v * m + 16 * (ct + h)];
      }
    };
    load(0);
    for (int ct = 0; ct < m / 16; ct += 2) {
      f64x4 c0 = {0.0, 0.0, 0.0, 0.0}, c1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ua[s][j], vb[0][s][j], c0, 0, 0, 0);
          c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ua[s][j], vb[1][s][j], c1, 0, 0, 0);
        }
      double a0[4], a1[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        a0[v] = av[0][v];
        a1[v] = av[1][v];
      }
      if (ct + 2 < m / 16) load(ct + 2);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double d0 = a0[v] - c0[v], d1 = a1[v] - c1[v];
        res2 += d0 * d0 + d1 * d1;
      }
    }
  }
  return block_sum(res2, sv);
}

__device__ __noinline__ double rc_residual(const double* __restrict__ A, int m, const double* __restrict__ Up, int ld,
                                           const double* __restrict__ Vp, int kr, double* lds, double* sv) {
  return residual_norm2(A, m, Up, ld, Vp, kr, lds, sv);
}

// Pair p of round rho of the round-robin schedule on n (even) indices.
__device__ __forceinline__ void rc_pair(int n, int rho, int p, int& a, int& b) {
  if (p == 0) {
    a = n - 1;
    b = rho;
  } else {
    a = (rho + p) % (n - 1);
    b = (rho - p + n - 1) % (n - 1);
  }
}

constexpr int kRcMaxRank = 192;  // largest rank recompressed: its packed working matrix fills the LDS
constexpr int kRcPacked = kRcMaxRank * (kRcMaxRank + 1) / 2;
constexpr int kRcSweeps = 15;

// Packed symmetric / lower-triangular storage: (i, j), j <= i, at i(i+1)/2 + j.
__device__ __forceinline__ int rc_pk(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

typedef __attribute__((address_space(3))) double rc_lds;

// Shared state of one workgroup's recompression.
struct RcShared {
  double* S;         // packed kr x kr working matrix (LDS), also the GEMM stages
  double *cs, *sn, *lam, *du, *dv, *tail, *sv;
  int *pa, *pb, *ord, *flag;
};

// Lower Cholesky factor of the Gram matrix G (kr x kr, row stride R,
// indices >= r the identity) after equilibration by d = sqrt of its
// diagonal, written back to G (upper part zero); false if not positive
// definite.
__device__ __forceinline__ bool rc_gram_chol(const RcShared& sh, double* __restrict__ G, int R, int kr, int r,
                                             double* d) {
  const int t = threadIdx.x;
  rc_lds* S = (rc_lds*)sh.S;
  for (int e = t; e < kr; e += 256) d[e] = e < r ? sqrt(G[(long)e * R + e]) : 1.0;
  if (t == 0) *sh.flag = 0;
  __syncthreads();
  for (int e = t; e < kr * kr; e += 256) {
    const int p = e / kr, q = e % kr;
    if (q <= p) S[rc_pk(p, q)] = (p < r && q < r) ? G[(long)p * R + q] / (d[p] * d[q]) : (p == q ? 1.0 : 0.0);
  }
  __syncthreads();
  for (int j = 0; j < kr; ++j) {
    if (t == 0) {
      const double piv = S[rc_pk(j, j)];
      if (!(piv > 0.0) || !isfinite(piv)) *sh.flag = 1;
      S[rc_pk(j, j)] = piv > 0.0 ? sqrt(piv) : 1.0;
    }
    __syncthreads();
    const double dj = S[rc_pk(j, j)];
    for (int e = j + 1 + t; e < kr; e += 256) S[rc_pk(e, j)] /= dj;
    __syncthreads();
    const int nr = kr - j - 1;
    for (int e = t; e < nr * nr; e += 256) {
      const int ii = j + 1 + e / nr, ll = j + 1 + e % nr;
      if (ll <= ii) S[rc_pk(ii, ll)] -= S[rc_pk(ii, j)] * S[rc_pk(ll, j)];
    }
    __syncthreads();
  }
  const bool ok = *sh.flag == 0;
  for (int e = t; e < kr * kr; e += 256) {
    const int p = e / kr, q = e % kr;
    G[(long)p * R + q] = q <= p ? S[rc_pk(p, q)] : 0.0;
  }
  __syncthreads();
  return ok;
}

// Lower factor (kr x kr, row stride R) into the packed working matrix.
__device__ __forceinline__ void rc_load_factor(const RcShared& sh, const double* __restrict__ Lg, int R, int kr) {
  for (int e = threadIdx.x; e < kr * kr; e += 256) {
    const int p = e / kr, q = e % kr;
    if (q <= p) ((rc_lds*)sh.S)[rc_pk(p, q)] = Lg[(long)p * R + q];
  }
  __syncthreads();
}

// With the lower factor F packed in the working matrix, vector x (stride sx)
// in place: forward F x = b, or (TRANS) backward F^T x = b.
template <bool TRANS>
__device__ __forceinline__ void rc_solve(const RcShared& sh, int kr, double* __restrict__ x, long sx) {
  const rc_lds* S = (const rc_lds*)sh.S;
  if (!TRANS) {
    for (int p = 0; p < kr; ++p) {
      const rc_lds* Sp = S + p * (p + 1) / 2;
      double v0 = x[p * sx], v1 = 0.0;
      int l = 0;
      for (; l + 1 < p; l += 2) {
        v0 -= Sp[l] * x[l * sx];
        v1 -= Sp[l + 1] * x[(l + 1) * sx];
      }
      if (l < p) v0 -= Sp[l] * x[l * sx];
      x[p * sx] = (v0 + v1) / Sp[p];
    }
  } else {
    for (int p = kr - 1; p >= 0; --p) {
      double v0 = x[p * sx], v1 = 0.0;
      int l = p + 1;
      for (; l + 1 < kr; l += 2) {
        v0 -= S[l * (l + 1) / 2 + p] * x[l * sx];
        v1 -= S[(l + 1) * (l + 2) / 2 + p] * x[(l + 1) * sx];
      }
      if (l < kr) v0 -= S[l * (l + 1) / 2 + p] * x[l * sx];
      x[p * sx] = (v0 + v1) / S[p * (p + 1) / 2 + p];
    }
  }
}

// Eigen-decomposition of the symmetric kr x kr matrix packed in the working
// matrix by cyclic Jacobi: the disjoint rotations of a round of a round-robin
// schedule are applied together, as 2 x 2 block transforms between pairs
// (J_P^T [S_PQ] J_Q, each block read and written once) in one phase; the
// accumulated rotations are kept transposed (Wt = W^T, kr x kr, row stride
// R, scratch), so that a rotation of columns a, b of W updates rows a, b of
// Wt with consecutive lanes on consecutive entries.  A rotation is skipped
// when |S_ab| <= 1e-14 sqrt(S_aa S_bb); a sweep without rotations ends.  On
// return the diagonal holds the eigenvalues and Wt the eigenvectors as rows.
__device__ __forceinline__ void rc_jacobi(const RcShared& sh, int kr, double* __restrict__ Wt, int R) {
  const int t = threadIdx.x, np = kr / 2;
  rc_lds* S = (rc_lds*)sh.S;
  const int nh = kr <= 128 ? 256 / kr : 1;  // lanes per column of Wt (kr >= 16)
  const int jc = t % kr, hh = t / kr;
  for (int e = t; e < kr * kr; e += 256) {
    const int p = e / kr, q = e - (e / kr) * kr;
    Wt[(long)p * R + q] = p == q ? 1.0 : 0.0;
  }
  // the block items (P, Q), P <= Q, of this lane: P rows of the triangle in
  // order, precomputed once (np (np + 1) / 2 <= 4656 items, <= 19 per lane)
  constexpr int kMaxItems = (kRcMaxRank / 2) * (kRcMaxRank / 2 + 1) / 2 / 256 + 1;
  short iP[kMaxItems], iQ[kMaxItems];
  int nitems = 0;
  {
    int P = 0, Q = 0, e = 0;
    for (int it = 0; it < kMaxItems; ++it) {
      const int target = t + 256 * it;
      // advance (P, Q) to the target-th pair of the triangle (row P, Q >= P)
      while (e < target && P < np) {
        ++e;
        if (++Q == np) {
          ++P;
          Q = P;
        }
      }
      if (P < np && e == target) {
        iP[it] = (short)P;
        iQ[it] = (short)Q;
        nitems = it + 1;
      } else {
        iP[it] = iQ[it] = -1;
      }
    }
  }
  for (int sw = 0; sw < kRcSweeps; ++sw) {
    if (t == 0) *sh.flag = 0;
    __syncthreads();
    for (int rho = 0; rho < kr - 1; ++rho) {
      if (t < np) {
        int a, b;
        rc_pair(kr, rho, t, a, b);
        const double app = S[rc_pk(a, a)], aqq = S[rc_pk(b, b)], apq = S[rc_pk(a, b)];
        double c = 1.0, s = 0.0;
        if (apq != 0.0 && fabs(apq) > 1e-14 * sqrt(fabs(app * aqq))) {
          const double th = (aqq - app) / (2.0 * apq);
          const double tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
          c = 1.0 / sqrt(1.0 + tt * tt);
          s = tt * c;
          *sh.flag = 1;
        }
        sh.cs[t] = c;
        sh.sn[t] = s;
        sh.pa[t] = a;
        sh.pb[t] = b;
      }
      __syncthreads();
      // blocks (P, Q), P <= Q: rows by P's rotation, columns by Q's
      for (int it = 0; it < nitems; ++it) {
        const int P = iP[it], Q = iQ[it];
        if (P < 0) continue;
        const double sP = sh.sn[P], sQ = sh.sn[Q];
        if (sP == 0.0 && sQ == 0.0) continue;
        const double cP = sh.cs[P], cQ = sh.cs[Q];
        const int a = sh.pa[P], b = sh.pb[P], c = sh.pa[Q], d = sh.pb[Q];
        const int iac = rc_pk(a, c), iad = rc_pk(a, d), ibc = rc_pk(b, c), ibd = rc_pk(b, d);
        const double xac = S[iac], xad = S[iad], xbc = S[ibc], xbd = S[ibd];
        const double rac = cP * xac - sP * xbc, rad = cP * xad - sP * xbd;
        const double rbc = sP * xac + cP * xbc, rbd = sP * xad + cP * xbd;
        S[iac] = cQ * rac - sQ * rad;
        S[ibd] = sQ * rbc + cQ * rbd;
        S[iad] = sQ * rac + cQ * rad;                 // for P == Q the pair's own (a, b) entry
        if (P != Q) S[ibc] = cQ * rbc - sQ * rbd;
      }
      // rows a, b of Wt: lane t takes column jc of every nh-th pair from hh,
      // the loads of 16 pairs issued before their stores
      if (hh < nh) {
        for (int P0 = hh; P0 < np; P0 += 16 * nh) {
          double xa[16], xb[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            const int P = P0 + u * nh;
            if (P < np && sh.sn[P] != 0.0) {
              xa[u] = Wt[(long)sh.pa[P] * R + jc];
              xb[u] = Wt[(long)sh.pb[P] * R + jc];
            }
          }
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            const int P = P0 + u * nh;
            if (P < np && sh.sn[P] != 0.0) {
              const double cP = sh.cs[P], sP = sh.sn[P];
              Wt[(long)sh.pa[P] * R + jc] = cP * xa[u] - sP * xb[u];
              Wt[(long)sh.pb[P] * R + jc] = sP * xa[u] + cP * xb[u];
            }
          }
        }
      }
      __syncthreads();
    }
    const bool more = *sh.flag != 0;
    __syncthreads();
    if (!more) break;
  }
}

// The recompression of one panel (see above).  Scratch slots: Yt, V2t, V2p
// R x m, U2 m x R, the R x R slots Lu, Lv, W, Bm, Tm, Xu, Xv.
__device__ __forceinline__ void rc_panel(const RcShared& sh, const double* __restrict__ A,
                                         const double* __restrict__ Lkk, double* __restrict__ Up,
                                         double* __restrict__ Vp, int* __restrict__ rank_out, int m, int rs, int r,
                                         double eps, double* ws) {
  const int t = threadIdx.x, R = rs, kr = (r + 15) & ~15;
  double* Yt = ws;
  double* U2 = Yt + (long)R * m;
  double* V2t = U2 + (long)R * m;
  double* V2p = V2t + (long)R * m;
  double* Lu = V2p + (long)R * m;
  double* Lv = Lu + (long)R * R;
  double* W = Lv + (long)R * R;          // B B^T, then the eigenvectors as rows
  double* Bm = W + (long)R * R;
  double* Tm = Bm + (long)R * R;
  double* Xu = Tm + (long)R * R;
  double* Xv = Xu + (long)R * R;
  double* S = sh.S;
  const bool thin = kr <= 32;
  // V^T = V'^T L_kk^T (column block tn of L_kk^T needs L_kk's first 128 (tn + 1) columns)
  if (thin) {
    rc_thin_nt<true, true>(Lkk, m, m, Vp, m, kr, m, Yt, m);
  } else {
    for (int tn = 0; tn < m / kTile; ++tn)
      rc_gemm<false>(Vp, m, kr, Lkk + (long)tn * kTile * m, m, kTile, (tn + 1) * kTile, Yt + tn * kTile, m, kr,
                     kTile, S);
  }
  __syncthreads();
  rc_gemm<true>(Up, rs, kr, Up, rs, kr, m, Lu, R, kr, kr, S);
  rc_gemm<false>(Yt, m, kr, Yt, m, kr, m, Lv, R, kr, kr, S);
  __syncthreads();
  if (!rc_gram_chol(sh, Lu, R, kr, r, sh.du)) return;
  if (!rc_gram_chol(sh, Lv, R, kr, r, sh.dv)) return;
  // U^T A V (A V staged in U2's buffer), scaled by D_u^-1 . D_v^-1
  if (thin)
    rc_thin_nt<false, false>(A, m, m, Yt, m, kr, m, U2, R);
  else
    rc_gemm<false>(A, m, m, Yt, m, kr, m, U2, R, m, kr, S);
  __syncthreads();
  rc_gemm<true>(Up, rs, kr, U2, R, kr, m, Tm, R, kr, kr, S);
  __syncthreads();
  for (int e = t; e < kr * kr; e += 256) {
    const int p = e / kr, q = e % kr;
    Tm[(long)p * R + q] /= sh.du[p] * sh.dv[q];
  }
  __syncthreads();
  // B = Lu^-1 T Lv^-T: columns by forward solves with Lu, then rows with Lv
  rc_load_factor(sh, Lu, R, kr);
  for (int c = t; c < kr; c += 256) rc_solve<false>(sh, kr, Tm + c, R);
  __syncthreads();
  rc_load_factor(sh, Lv, R, kr);
  for (int c = t; c < kr; c += 256) rc_solve<false>(sh, kr, Tm + (long)c * R, 1);
  __syncthreads();
  for (int e = t; e < kr * kr; e += 256) Bm[(long)(e / kr) * R + e % kr] = Tm[(long)(e / kr) * R + e % kr];
  __syncthreads();
  // B B^T (via W's slot) packed into the working matrix, then its eigenvectors
  rc_gemm<false>(Bm, R, kr, Bm, R, kr, kr, W, R, kr, kr, S);
  __syncthreads();
  for (int e = t; e < kr * kr; e += 256) {
    const int p = e / kr, q = e % kr;
    if (q <= p) S[rc_pk(p, q)] = 0.5 * (W[(long)p * R + q] + W[(long)q * R + p]);  // symmetric against rounding
  }
  __syncthreads();
  rc_jacobi(sh, kr, W, R);
  // sigma^2 in decreasing order and the discarded sums
  for (int e = t; e < kr; e += 256) sh.lam[e] = fmax(S[rc_pk(e, e)], 0.0);
  __syncthreads();
  for (int e = t; e < kr; e += 256) {
    int rk = 0;
    const double v = sh.lam[e];
    for (int q = 0; q < kr; ++q) rk += (sh.lam[q] > v || (sh.lam[q] == v && q < e)) ? 1 : 0;
    sh.ord[rk] = e;
  }
  __syncthreads();
  if (t == 0) {
    double acc = 0.0;
    sh.tail[kr] = 0.0;
    for (int q = kr - 1; q >= 0; --q) {
      acc += sh.lam[sh.ord[q]];
      sh.tail[q] = acc;
    }
  }
  __syncthreads();
  for (int at = 0; at < 3; ++at) {
    const double f = at == 0 ? 0.95 : (at == 1 ? 0.7 : 0.4);
    int kk = 0;
    while (kk < r && sh.tail[kk] > f * eps * eps) ++kk;
    if (kk >= r) return;  // uniform: no smaller rank
    const int kr2 = (kk + 15) & ~15;
    // W_k ([l][j], columns past kk zero); X_v = D_v^-1 Lv^-T B^T W_k
    for (int e = t; e < kr * kr; e += 256) {
      const int l = e / kr, j = e % kr;
      Tm[(long)l * R + j] = j < kk ? W[(long)sh.ord[j] * R + l] : 0.0;
    }
    __syncthreads();
    rc_gemm<true>(Bm, R, kr, Tm, R, kr, kr, Xv, R, kr, kr, S);
    __syncthreads();
    rc_load_factor(sh, Lv, R, kr);
    for (int c = t; c < kk; c += 256) {
      rc_solve<true>(sh, kr, Xv + c, R);
      for (int p = 0; p < kr; ++p) Xv[(long)p * R + c] /= sh.dv[p];
    }
    __syncthreads();
    // X_u^T row j = (D_u^-1 Lu^-T W_k(:, j))^T
    rc_load_factor(sh, Lu, R, kr);
    for (int c = t; c < kr; c += 256) {
      double* z = Xu + (long)c * R;
      for (int p = 0; p < kr; ++p) z[p] = c < kk ? Tm[(long)p * R + c] : 0.0;
      if (c < kk) {
        rc_solve<true>(sh, kr, z, 1);
        for (int p = 0; p < kr; ++p) z[p] /= sh.du[p];
      }
    }
    __syncthreads();
    // U2 = U X_u (m x kr2); V2 = V X_v (m x kr2, thin) or V2^T (kr2 x m) for
    // the check; V2'^T = X_v^T V'^T (kr2 x m)
    if (kr2 > 0) {
      rc_gemm<false>(Up, rs, m, Xu, R, kr2, kr, U2, R, m, kr2, S);
      if (thin)
        rc_gemm<true>(Yt, m, m, Xv, R, kr2, kr, V2t, R, m, kr2, S);
      else
        rc_gemm<true>(Xv, R, kr2, Yt, m, m, kr, V2t, m, kr2, m, S);
      rc_gemm<true>(Xv, R, kr2, Vp, m, m, kr, V2p, m, kr2, m, S);
    }
    __syncthreads();
    const double res = kr2 == 0 ? rc_thin_residual(A, m, U2, V2t, R, 0, sh.sv)
                       : thin   ? rc_thin_residual(A, m, U2, V2t, R, kr2, sh.sv)
                                : rc_residual(A, m, U2, R, V2t, kr2, S, sh.sv);
    if (!(res <= eps * eps)) continue;  // uniform: try a larger rank
    for (long e = t; e < (long)m * r; e += 256) {
      const long row = e / r;
      const int c = (int)(e % r);
      Up[row * rs + c] = c < kk ? U2[row * R + c] : 0.0;
    }
    for (long e = t; e < (long)r * m; e += 256) {
      const int q = (int)(e / m);
      Vp[e] = q < kk ? V2p[e] : 0.0;
    }
    if (t == 0) *rank_out = kk;
    return;
  }
}

__global__ void tlr_rc_queue_init_kernel(unsigned long long* __restrict__ q) {
  if (threadIdx.x == 0) *q = 0ull;
}

__global__ __launch_bounds__(256, 1) void tlr_recompress_kernel(double* __restrict__ tiles, int m, int nt, int rs,
                                                                double eps, double* __restrict__ U,
                                                                double* __restrict__ Vt, int* __restrict__ ranks,
                                                                double* __restrict__ scratch,
                                                                unsigned long long* __restrict__ queue,
                                                                const int* __restrict__ info) {
  if (*info != 0) return;
  __shared__ double S[kRcPacked];  // packed working matrix, and the GEMM stages
  __shared__ double cs[kRcMaxRank / 2], sn[kRcMaxRank / 2], lam[kRcMaxRank], du[kRcMaxRank], dv[kRcMaxRank],
      tail[kRcMaxRank + 1], sv[8];
  __shared__ int pa[kRcMaxRank / 2], pb[kRcMaxRank / 2], ord[kRcMaxRank];
  __shared__ int s_flag;
  __shared__ long s_w;
  static_assert(4 * kStageDoubles <= kRcPacked, "the GEMM stages alias S");
  const long npan = (long)nt * (nt - 1) / 2;
  double* ws = scratch + (long)blockIdx.x * tlr_rc_scratch_doubles(m, rs);
  const RcShared sh{S, cs, sn, lam, du, dv, tail, sv, pa, pb, ord, &s_flag};
  // panels in order of distance from the diagonal (the largest ranks first),
  // taken from a device counter, so that workgroups with cheap panels take
  // more; every workgroup leaves once the counter passes the panel count
  for (;;) {
    __syncthreads();  // the previous panel is done with the LDS and s_w
    if (threadIdx.x == 0) s_w = (long)atomicAdd(queue, 1ull);
    __syncthreads();
    const long w = s_w;
    if (w >= npan) break;
    long d = 1, rem = w;
    while (rem >= nt - d) {
      rem -= nt - d;
      ++d;
    }
    const long k = rem, i = k + d;
    const long pid = tri_st(i, k);
    const int r = ranks[pid];
    if (r < 2 || r > kRcMaxRank || r > rs) continue;  // uniform
    rc_panel(sh, tiles + tri_lo(i, k) * (long)m * m, tiles + tri_lo(k, k) * (long)m * m, U + pid * (long)m * rs,
             Vt + pid * (long)rs * m, ranks + pid, m, rs, r, eps, ws);
  }
}

hipError_t launch_tlr_recompress(double* tiles, int m, int nt, int rs, double eps, double* U, double* Vt, int* ranks,
                                 double* scratch, int grid, const int* info, hipStream_t st) {
  if (nt < 2 || grid < 1) return hipSuccess;
  unsigned long long* queue = (unsigned long long*)(scratch + (long)grid * tlr_rc_scratch_doubles(m, rs));
  hipLaunchKernelGGL(tlr_rc_queue_init_kernel, dim3(1), dim3(64), 0, st, queue);
  hipLaunchKernelGGL(tlr_recompress_kernel, dim3(grid), dim3(256), 0, st, tiles, m, nt, rs, eps, U, Vt, ranks, scratch,
                     queue, info);
  return hipGetLastError();
}

// ------------------------------------------------------------ updates
// Left-looking: before column j is factored, every tile (i, j), i >= j,
// takes all of its updates at once,
//   A_ij -= sum_{k<j} U_ik W_ijk U_jk^T,   W_ijk = V'^T_ik V'_jk,
// so each tile is read and written once.  The (i, k) pairs of one launch
// are z = (i - i0) nk + (k - k0) for i in [i0, i0 + ni), k in [k0, k0 + nk).

// WT_z = V'^T_jk (V'^T_ik)^T: r_jk x r_ik.  Grid (pairs, rs/128, rs/128):
// the pair is the fastest grid index, so that the workgroups that have work
// (mostly tile (0, 0)) are consecutive and spread over all XCDs.
__global__ __launch_bounds__(256, 2) void tlr_w_kernel(int j, int i0, int k0, int nk, int m, int rs,
                                                    const double* __restrict__ Vt, const int* __restrict__ ranks,
                                                    double* __restrict__ WT, const int* __restrict__ info) {
  if (*info != 0) return;
  __shared__ double lds[4 * kStageDoubles];
  const long z = blockIdx.x;
  const long i = i0 + z / nk, k = k0 + z % nk;
  const int ri = abs(ranks[tri_st(i, k)]), rj = abs(ranks[tri_st(j, k)]);
  if ((long)blockIdx.y * kTile >= rj || (long)blockIdx.z * kTile >= ri) return;
  // unmasked loads: K = m, and the 128-row operand tiles stay inside the Vt
  // arena (its 128 rows of slack cover the last panel)
  gemm_nt_tile<false>(WT + z * rs * rs, rs, Vt + tri_st(j, k) * (long)rs * m, m, Vt + tri_st(i, k) * (long)rs * m,
                      m, rj, ri, m, 1.0, 0.0, blockIdx.y, blockIdx.z, lds);
}

// T_z = U_ik W_ijk: m x r_jk (B operand WT_z, K = r_ik); columns r_jk up to
// the next multiple of 16 are set to zero for the segmented K loop below.
__global__ __launch_bounds__(256, 2) void tlr_t_kernel(int j, int i0, int k0, int nk, int m, int rs,
                                                    const double* __restrict__ U, const int* __restrict__ ranks,
                                                    const double* __restrict__ WT, double* __restrict__ T,
                                                    const int* __restrict__ info) {
  if (*info != 0) return;
  __shared__ double lds[4 * kStageDoubles];
  const long i = i0 + blockIdx.z / nk, k = k0 + blockIdx.z % nk;
  const int ri = abs(ranks[tri_st(i, k)]), rj = abs(ranks[tri_st(j, k)]);
  if ((long)blockIdx.y * kTile >= rj) return;
  double* Tz = T + (long)blockIdx.z * m * rs;
  gemm_nt_tile(Tz, rs, U + tri_st(i, k) * (long)m * rs, rs, WT + (long)blockIdx.z * rs * rs, rs, m, rj, ri, 1.0,
               0.0, blockIdx.x, blockIdx.y, lds);
  const int r16 = (rj + 15) & ~15;
  if ((int)blockIdx.y == rj / kTile && r16 > rj) {
    const int w = r16 - rj;
    for (int e = threadIdx.x; e < kTile * w; e += 256)
      Tz[((long)blockIdx.x * kTile + e / w) * rs + rj + e % w] = 0.0;
  }
}

// A_ij -= sum_k T_z U_jk^T for k in [k0, k0 + nk): one 128 x 128 block of
// tile (i0 + blockIdx.z, j) per workgroup, K running over the k segments
// (each rounded up to 16; T_z and U_jk are zero past r_jk).  Of a diagonal
// tile only the lower blocks are updated.
__global__ __launch_bounds__(256, 2) void tlr_u_kernel(int j, int i0, int k0, int nk, int m, int rs,
                                                    double* __restrict__ tiles, const double* __restrict__ U,
                                                    const int* __restrict__ ranks, const double* __restrict__ T,
                                                    const int* __restrict__ info) {
  if (*info != 0) return;
  __shared__ double lds[4 * kStageDoubles];
  const long i = i0 + blockIdx.z;
  const long tr = blockIdx.y, tc = blockIdx.x;
  if (i == j && tc > tr) return;
  int nst = 0;
  for (int kk = 0; kk < nk; ++kk) nst += (abs(ranks[tri_st(j, k0 + kk)]) + kStageK - 1) / kStageK;
  if (nst == 0) return;
  Acc acc;
  acc_zero(acc);
  int ck = 0, cs = 0;  // cursor: segment k0 + ck, stage cs inside it
  auto load = [&](double (&ra)[8], double (&rb)[8]) {
    while (cs * kStageK >= abs(ranks[tri_st(j, k0 + ck)])) {
      ++ck;
      cs = 0;
    }
    const long z = (long)blockIdx.z * nk + ck;
    load_rows<false>(T + z * m * rs, rs, tr * kTile, (long)cs * kStageK, 0, 0, ra);
    load_rows<false>(U + tri_st(j, k0 + ck) * (long)m * rs, rs, tc * kTile, (long)cs * kStageK, 0, 0, rb);
    ++cs;
  };
  double ra[8], rb[8];
  load(ra, rb);
  store_rows(lds, ra);
  store_rows(lds + kStageDoubles, rb);
  __syncthreads();
  for (int s = 0; s < nst; ++s) {
    double* cur = lds + (s & 1) * 2 * kStageDoubles;
    double* nxt = lds + ((s + 1) & 1) * 2 * kStageDoubles;
    if (s + 1 < nst) load(ra, rb);
    mma_stage(cur, cur + kStageDoubles, acc);
    if (s + 1 < nst) {
      store_rows(nxt, ra);
      store_rows(nxt + kStageDoubles, rb);
    }
    __syncthreads();
  }
  double* C = tiles + tri_lo(i, j) * (long)m * m;
#pragma unroll
  for (int ib = 0; ib < 4; ++ib)
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double* c = C + (tr * kTile + acc_row(ib, q)) * (long)m + tc * kTile + acc_col(jb);
        *c -= acc.v[ib][jb][q];
      }
}

// local = info (so that a failed earlier step skips the tile's kernels)
__global__ void tlr_info_copy_kernel(const int* __restrict__ info, int* __restrict__ local) {
  if (threadIdx.x == 0) *local = *info;
}

// info = first failing global pivot (1-based) from the tile's local info
__global__ void tlr_info_kernel(int* __restrict__ info, const int* __restrict__ local, int offset) {
  if (threadIdx.x == 0 && *local != 0 && *info == 0) *info = *local + offset;
}

// ------------------------------------------------------------ dense form
// The TLR factor written out as a dense row-major factor (leading dimension
// ldd <= nt m): one 128 x 128 block per workgroup.  A diagonal tile's block
// is copied (identity past n, as the tiles hold it); an off-diagonal tile's
// block is U_ij V'^T_ij on FP64 MFMA with K the rank rounded up to 16 (U's
// columns past the rank are zero), zero past n.  Blocks above the diagonal
// are not written (the sweep reads only the lower triangle).
__global__ __launch_bounds__(256) void tlr_expand_kernel(int n, int m, int rs, const double* __restrict__ tiles,
                                                         const double* __restrict__ U, const double* __restrict__ Vt,
                                                         const int* __restrict__ ranks, double* __restrict__ D,
                                                         long ldd) {
  __shared__ __attribute__((aligned(16))) double lds[4 * kStageDoubles];
  const int sb = m / kTile;
  long ti, tj;
  tri_inverse(blockIdx.x, ti, tj);
  const int br = blockIdx.y / sb, bc = blockIdx.y % sb;
  const long R0 = ti * m + (long)br * kTile, C0 = tj * m + (long)bc * kTile;
  if (R0 >= ldd || C0 >= ldd || (ti == tj && bc > br)) return;  // uniform per workgroup
  const int t = threadIdx.x;
  if (ti == tj) {
    const double* src = tiles + tri_lo(ti, ti) * (long)m * m + (long)br * kTile * m + (long)bc * kTile;
    for (int e = t; e < kTile * kTile; e += 256) {
      const int r = e / kTile, c = e % kTile;
      if (R0 + r < ldd && C0 + c < ldd) D[(R0 + r) * ldd + C0 + c] = src[(long)r * m + c];
    }
    return;
  }
  const long pid = tri_st(ti, tj);
  const int r = abs(ranks[pid]);
  const int K = min(rs, (r + 15) & ~15);
  const double* Up = U + pid * (long)m * rs;
  const double* Vp = Vt + pid * (long)rs * m + (long)bc * kTile;
  Acc acc;
  acc_zero(acc);
  const int nst = K / kStageK;
  if (nst > 0) {
    double ra[8], rb[8];
    load_rows<false>(Up, rs, (long)br * kTile, 0, 0, 0, ra);
    load_cols(Vp, m, 0, rb);
    store_rows(lds, ra);
    store_cols(lds + kStageDoubles, rb);
    __syncthreads();
    for (int s = 0; s < nst; ++s) {
      double* cur = lds + (s & 1) * 2 * kStageDoubles;
      double* nxt = lds + ((s + 1) & 1) * 2 * kStageDoubles;
      if (s + 1 < nst) {
        load_rows<false>(Up, rs, (long)br * kTile, (long)(s + 1) * kStageK, 0, 0, ra);
        load_cols(Vp, m, (long)(s + 1) * kStageK, rb);
      }
      mma_stage(cur, cur + kStageDoubles, acc);
      if (s + 1 < nst) {
        store_rows(nxt, ra);
        store_cols(nxt + kStageDoubles, rb);
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int ib = 0; ib < 4; ++ib)
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const long gi = R0 + acc_row(ib, q), gj = C0 + acc_col(jb);
        if (gi < ldd && gj < ldd) D[gi * ldd + gj] = (gi < n && gj < n) ? acc.v[ib][jb][q] : 0.0;
      }
}

hipError_t launch_tlr_expand(int n, int m, int nt, int rs, const double* tiles, const double* U, const double* Vt,
                             const int* ranks, double* D, long ldd, hipStream_t st) {
  const long ntiles = (long)nt * (nt + 1) / 2;
  const unsigned sb = (unsigned)(m / kTile);
  hipLaunchKernelGGL(tlr_expand_kernel, dim3((unsigned)ntiles, sb * sb), dim3(256), 0, st, n, m, rs, tiles, U, Vt,
                     ranks, D, ldd);
  return hipGetLastError();
}

hipError_t launch_tlr_build(int n, int m, int nt, const double* sigma, int lds, const int64_t* perm,
                            const int* perm_bad, const double* locs, const Matern& mk, double* tiles, int* info,
                            hipStream_t st) {
  const long sub = (long)(m / 64) * (m / 64) * ((long)nt * (nt + 1) / 2);
  hipLaunchKernelGGL(tlr_build_kernel, dim3((unsigned)sub), dim3(256), 0, st, n, m, sigma, lds, perm, perm_bad,
                     locs, mk, tiles, info);
  return hipGetLastError();
}

hipError_t launch_tlr_cholesky(const TlrCholArgs& a, hipStream_t st) {
  const int m = a.m, nt = a.nt, rs = a.rs;
  const unsigned rt = (unsigned)((rs + kTile - 1) / kTile), mt = (unsigned)(m / kTile);
  SideStream* sd = side_stream(kSideTlr, st);
  std::unique_lock<std::mutex> lock;
  if (sd) lock = std::unique_lock<std::mutex>(sd->mu);
  for (int j = 0; j < nt; ++j) {
    // updates of column j from the panels k < j, in launches of at most
    // kTlrPairBatch (i, k) pairs
    if (j > 0) {
      const int nk = (int)std::min<long>(j, kTlrPairBatch);
      const int ni_max = (int)std::max<long>(1, kTlrPairBatch / nk);
      for (int i0 = j; i0 < nt; i0 += ni_max) {
        const int ni = std::min(ni_max, nt - i0);
        for (int k0 = 0; k0 < j; k0 += nk) {
          const int nkc = std::min(nk, j - k0);
          const unsigned np = (unsigned)(ni * nkc);
          hipLaunchKernelGGL(tlr_w_kernel, dim3(np, rt, rt), dim3(256), 0, st, j, i0, k0, nkc, m, rs,
                             (const double*)a.Vt, (const int*)a.ranks, a.WT, (const int*)a.info);
          hipLaunchKernelGGL(tlr_t_kernel, dim3(mt, rt, np), dim3(256), 0, st, j, i0, k0, nkc, m, rs,
                             (const double*)a.U, (const int*)a.ranks, (const double*)a.WT, a.T,
                             (const int*)a.info);
          hipLaunchKernelGGL(tlr_u_kernel, dim3(mt, mt, (unsigned)ni), dim3(256), 0, st, j, i0, k0, nkc, m, rs,
                             a.tiles, (const double*)a.U, (const int*)a.ranks, (const double*)a.T,
                             (const int*)a.info);
        }
      }
    }
    // the dense factor of the diagonal tile; the cross approximation of the
    // tiles below does not read it, so with a side stream the two overlap and
    // join before the row solves
    double* Djj = a.tiles + (long)(j * (j + 1) / 2 + j) * m * m;
    const int P = nt - j - 1;
    const bool overlap = sd && P > 0;
    hipStream_t ps = overlap ? sd->s : st;
    // on an error, let the side stream drain before returning, so that none
    // of its kernels still writes the tiles once the caller sees the failure
    auto fail = [&](hipError_t e) {
      if (overlap) (void)hipStreamSynchronize(ps);
      return e;
    };
    if (overlap) {
      hipError_t e = hipEventRecord(sd->ev[0], st);
      if (e == hipSuccess) e = hipStreamWaitEvent(ps, sd->ev[0], 0);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(tlr_info_copy_kernel, dim3(1), dim3(64), 0, ps, (const int*)a.info, a.local_info);
    hipError_t e = launch_cholesky_f64(m, 128, Djj, a.local_info, ps, false);
    if (e != hipSuccess) return fail(e);
    hipLaunchKernelGGL(tlr_info_kernel, dim3(1), dim3(64), 0, ps, a.info, (const int*)a.local_info, j * m);
    if (overlap) {
      e = hipEventRecord(sd->ev[1], ps);
      if (e != hipSuccess) return fail(e);
    }
    if (P > 0) {
      // the T workspace (idle between the updates of two tile columns) holds
      // the transposed U columns, kTlrPairBatch tiles per launch
      const int pb = (int)std::min<long>(P, kTlrPairBatch);
      for (int i0 = 0; i0 < P; i0 += pb)
        hipLaunchKernelGGL(tlr_aca_kernel, dim3(std::min(pb, P - i0)), dim3(256), 0, st, (const double*)a.tiles, j,
                           i0, m, rs, a.rcap, a.eps, a.U, a.Vt, a.ranks, a.T, (const int*)a.info);
      if (overlap) {
        e = hipStreamWaitEvent(st, sd->ev[1], 0);
        if (e != hipSuccess) return fail(e);
      }
      hipLaunchKernelGGL(tlr_trsm_rows_kernel, dim3(P, rs / 4), dim3(256), 0, st, (const double*)a.tiles, j, m, rs,
                         a.Vt, (const int*)a.ranks, (const int*)a.info);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return fail(e);
  }
  if (a.rc_scratch) return launch_tlr_recompress(a.tiles, m, nt, rs, a.eps, a.U, a.Vt, a.ranks, a.rc_scratch,
                                                 a.rc_grid, a.info, st);
  return hipGetLastError();
}

}  // namespace mvn
