// Adjoint of the SOV estimator at fixed QMC points: d log P-hat / d a~, d b~
// (and d/d mu = -(d/da~ + d/db~)).  The paper does not differentiate the
// estimator; this is the reverse-mode chain rule of the recurrence of
// Eq. (sov1) as swept by Algorithms 2-3:
//
//   forward   s_i = sum_{k<i} L_ik y_k, a'_i = (a~_i - s_i)/L_ii,
//             b'_i = (b~_i - s_i)/L_ii, d_i = Phi(b') - Phi(a'),
//             y_i = Phi^-1(Phi(a') + w_i d_i), l = sum_i log d_i
//   reverse   with l-bar = omega (the sample's weight in the log-sum-exp)
//             and y-bar_i = sum_{k>i} L_ki s-bar_k:
//             a'-bar = -omega phi(a')/d + y-bar (1-w) phi(a')/phi(y)
//             b'-bar =  omega phi(b')/d + y-bar  w    phi(b')/phi(y)
//             a~-bar_i += a'-bar / L_ii,  b~-bar_i += b'-bar / L_ii,
//             s-bar_i = -(a'-bar + b'-bar) / L_ii
//
// One persistent workgroup owns a 64-column chunk for both passes: the
// forward pass keeps the shifts s_i in the workgroup's scratch (instead of y),
// the reverse pass recomputes (a', b', y, d) from them with the same code and
// forms y-bar block by block: a transposed GEMM Y-bar_r = L_(>r, r)^T S-bar_(>r)
// on FP64 MFMA (rows of L are contiguous in the block's columns, so the
// operand needs no transpose), then the in-block part as a dot product over
// the later rows of the block.  Chunks weight their samples by
// exp(l - max_chunk l); a final fixed-order reduction rescales them.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "gemm_f64.h"
#include "launch.h"
#include "mvn_device.h"
#include "sweep_block.h"
#include "sweep_gemm.h"

namespace mvn {

constexpr double kInvSqrt2Pi = 0.39894228040143267794;

// A operand of the reverse GEMM: As[k][row] = L[j0 + k][i0 + row].
struct RevOperand {
  static __device__ __forceinline__ void load(const double* __restrict__ L, long ld, long j0, long i0,
                                              double (&r)[8]) {
    const int t = threadIdx.x;
    const double2* p2 = reinterpret_cast<const double2*>(L + (j0 + (t >> 4)) * ld + i0 + (t & 15) * 8);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double2 v = p2[q];
      r[2 * q] = v.x;
      r[2 * q + 1] = v.y;
    }
  }
  static __device__ __forceinline__ void store(double* As, const double (&r)[8]) {
    const int t = threadIdx.x;
    double* d = As + (t >> 4) * GemmF64::kALd + (t & 15) * 8;
#pragma unroll
    for (int q = 0; q < 8; ++q) d[q] = r[q];
  }
};

// B operand of the reverse GEMM: S-bar rows j0..j0+15 of the chunk, [j][64].
__device__ __forceinline__ void load_sbar(const double* __restrict__ Sb, long j0, double (&r)[4]) {
  const int t = threadIdx.x;
  const double2* p2 = reinterpret_cast<const double2*>(Sb + (j0 + (t >> 4)) * kCols + (t & 15) * 4);
  const double2 v0 = p2[0], v1 = p2[1];
  r[0] = v0.x; r[1] = v0.y; r[2] = v1.x; r[3] = v1.y;
}
__device__ __forceinline__ void store_sbar(double* stage, const double (&r)[4]) {
  const int t = threadIdx.x;
  double* d = stage + GemmF64::kAStage + (t >> 4) * GemmF64::kBLd + (t & 15) * 4;
  d[0] = r[0]; d[1] = r[1]; d[2] = r[2]; d[3] = r[3];
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// G: the forward pass's limit-update GEMM (FP64, or FP32 / BF16 / split BF16
// on the factor's operand copy with FP32 accumulation; Y in G's operand
// type).  The reverse GEMM is FP64 on the FP64 factor in every mode, and
// the conditioning step is the FP64 one, so the reverse pass differentiates
// exactly the forward recurrence it recomputes from the stored shifts.
template <class G>
__global__ __launch_bounds__(256, 2) void grad_kernel(GradArgs p) {
  using E = typename G::E;
  using R = GemmF64;  // reverse GEMM
  static_assert(2 * G::kStageBytes <= kTile * kCols * 8 && 2 * R::kStageBytes <= kTile * kCols * 8,
                "GEMM stages fit the block buffer");
  __shared__ __attribute__((aligned(16))) double lds[kTile * kCols];
  __shared__ double slab[kSlab * kTile];
  __shared__ double c_at[kTile], c_bt[kTile], c_rl[kTile];
  __shared__ uint64_t c_lat[kTile];
  __shared__ double sslab[kSlab * kCols];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const long NS = (long)p.N * p.S;
  const long nchunks = (NS + kCols - 1) / kCols;
  const long ld = p.ld;
  const long slice = ld * kCols;
  E* Y = (E*)(p.yscr + (long)blockIdx.x * slice);
  const E* Lg = (const E*)p.Llow;
  const long lplane = ld * ld;
  double* Sf = p.sfw + (long)blockIdx.x * slice;
  double* Sb = p.sbar + (long)blockIdx.x * slice;
  char* stage0 = (char*)lds;
  char* stage1 = (char*)lds + G::kStageBytes;
  char* rstage0 = (char*)lds;
  char* rstage1 = (char*)lds + R::kStageBytes;
  const int nblk = (p.n + kTile - 1) / kTile;

  // rows n..ld-1 of the s-bar scratch are read by the reverse GEMMs (as
  // zeros: the matching rows of L are zero there) and never written
  for (long e = (long)p.n * kCols + t; e < slice; e += 256) Sb[e] = 0.0;

  for (long chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
    const long col = chunk * kCols + lane;
    const bool owner = wv == 0;
    const bool valid = owner && col < NS;
    const uint64_t sidx = col < NS ? (uint64_t)(col / p.N) : 0;  // every lane: its own column
    const uint64_t jpt = col < NS ? (uint64_t)(col % p.N) + 1 : 1;
    LogProd prod{1.0, 0};

    // ================= forward pass (the probability sweep, keeping s_i)
    for (int i0 = 0; i0 < p.n; i0 += kTile) {
      const int rows = min(kTile, p.n - i0);
      typename G::Acc acc;
      G::zero(acc);
      if (i0 > 0) {
        const int nst = i0 / G::kK;
        typename G::Regs r;
        G::load(Lg, ld, lplane, i0, 0, Y, ld, r);
        G::store(stage0, r);
        __syncthreads();
        for (int s = 0; s < nst; ++s) {
          const bool odd = s & 1;
          if (s + 1 < nst) G::load(Lg, ld, lplane, i0, (long)(s + 1) * G::kK, Y, ld, r);
          G::mma(odd ? stage1 : stage0, acc);
          if (s + 1 < nst) G::store(odd ? stage0 : stage1, r);
          __syncthreads();
        }
      }
      G::to_block(acc, lds);
      if (t < rows) {
        const long g = i0 + t;
        c_at[t] = p.at[g];
        c_bt[t] = p.bt[g];
        c_rl[t] = 1.0 / p.L[g * ld + g];
        c_lat[t] = p.lattice[g];
      }
      prod = condition_block<false, kTile, false>((lds_f64*)lds, (lds_f64*)slab, (const lds_f64*)c_at, (const lds_f64*)c_bt,
                             (const lds_f64*)c_rl, (const lds_u64*)c_lat, p.L, ld, i0, rows, p.n, jpt,
                             sidx, p.seed, p.periodize, valid, prod, owner ? Sf : nullptr);
      __syncthreads();
      G::put_y(lds, Y, ld, i0, rows);
      __syncthreads();
    }
    // chunk weights omega_c = exp(l_c - max_chunk l)
    double omega = 0.0;
    if (owner) {
      const double l = valid ? logprod_log(prod) : -INFINITY;
      if (valid) p.ell[col] = l;
      const double M = wave_max(l);
      omega = (M > -INFINITY && l > -INFINITY) ? exp(l - M) : 0.0;
      const double Z = wave_sum(omega);
      if (lane == 0) {
        p.mz[2 * chunk] = M;
        p.mz[2 * chunk + 1] = Z;
      }
    }
    double* ga = p.gpart + chunk * 2 * ld;
    double* gb = ga + ld;

    // ================= reverse pass
    for (int r = nblk - 1; r >= 0; --r) {
      const int i0 = r * kTile;
      const int rows = min(kTile, p.n - i0);
      R::Acc acc;
      R::zero(acc);
      // ---- Y-bar of the block from the later blocks: K over rows j >= i0 + 128
      const long j0 = (long)i0 + kTile;
      const int nst = (int)((ld - j0) / R::kK);
      if (nst > 0) {
        double ra[8], rb[4];
        RevOperand::load(p.L, ld, j0, i0, ra);
        load_sbar(Sb, j0, rb);
        RevOperand::store((double*)rstage0, ra);
        store_sbar((double*)rstage0, rb);
        __syncthreads();
        for (int s = 0; s < nst; ++s) {
          const bool odd = s & 1;
          if (s + 1 < nst) {
            RevOperand::load(p.L, ld, j0 + (long)(s + 1) * R::kK, i0, ra);
            load_sbar(Sb, j0 + (long)(s + 1) * R::kK, rb);
          }
          R::mma(odd ? rstage1 : rstage0, acc);
          if (s + 1 < nst) {
            RevOperand::store((double*)(odd ? rstage0 : rstage1), ra);
            store_sbar((double*)(odd ? rstage0 : rstage1), rb);
          }
          __syncthreads();
        }
      }
      R::to_block(acc, lds);
      if (t < rows) {
        const long g = i0 + t;
        c_at[t] = p.at[g];
        c_bt[t] = p.bt[g];
        c_rl[t] = 1.0 / p.L[g * ld + g];
        c_lat[t] = p.lattice[g];
      }
      // ---- reverse recurrence over the block, slabs of 8 rows from the end
      for (int q = ((rows - 1) / kSlab) * kSlab; q >= 0; q -= kSlab) {
        __syncthreads();
        // columns q..q+7 of the block's L (rows below them) and the slab's s
        for (int e = t; e < kTile * kSlab; e += 256) {
          const int i = e / kSlab, kk = e % kSlab;
          slab[e] = (i < rows && i > q + kk) ? p.L[(long)(i0 + i) * ld + i0 + q + kk] : 0.0;
        }
        for (int e = t; e < kSlab * kCols; e += 256) {
          const int kk = e / kCols;
          sslab[e] = (q + kk < rows) ? Sf[(long)(i0 + q + kk) * kCols + (e % kCols)] : 0.0;
        }
        __syncthreads();
        if (owner) {
          for (int k = min(q + kSlab, rows) - 1; k >= q; --k) {
            // y-bar_k = GEMM part + sum over the block's rows i > k (T[i] = s-bar_i)
            double s0 = lds[k * kCols + lane], s1 = 0.0, s2 = 0.0, s3 = 0.0;
            const int kk = k - q;
            const int ib = (k + 1) & ~7, ie = (rows + 7) & ~7;
            for (int i = ib; i < ie; i += 8) {
              s0 += slab[i * kSlab + kk] * lds[i * kCols + lane];
              s1 += slab[(i + 1) * kSlab + kk] * lds[(i + 1) * kCols + lane];
              s2 += slab[(i + 2) * kSlab + kk] * lds[(i + 2) * kCols + lane];
              s3 += slab[(i + 3) * kSlab + kk] * lds[(i + 3) * kCols + lane];
              s0 += slab[(i + 4) * kSlab + kk] * lds[(i + 4) * kCols + lane];
              s1 += slab[(i + 5) * kSlab + kk] * lds[(i + 5) * kCols + lane];
              s2 += slab[(i + 6) * kSlab + kk] * lds[(i + 6) * kCols + lane];
              s3 += slab[(i + 7) * kSlab + kk] * lds[(i + 7) * kCols + lane];
            }
            const double ybar = (s0 + s1) + (s2 + s3);
            // recompute the forward step from the stored shift
            const double s = sslab[kk * kCols + lane];
            const double rl = c_rl[k];
            const double alpha = (c_at[k] - s) * rl;
            const double beta = (c_bt[k] - s) * rl;
            const uint64_t g = (uint64_t)(i0 + k);
            const double w = richtmyer(jpt, c_lat[k], splitmix64(p.seed, sidx * (uint64_t)p.n + g),
                                       p.periodize);
            const Step st = condition_step(alpha, beta, w, 1.0 - w);
            double abar = 0.0, bbar = 0.0;
            if (omega > 0.0 && st.m > 0.0) {
              // phi(x)/d, in log scale when d is kept as m 2^e
              const double logd = st.e == 0 ? 0.0 : log(st.m) + (double)st.e * kLn2;
              double ra_d = 0.0, rb_d = 0.0;
              if (isfinite(alpha))
                ra_d = st.e == 0 ? kInvSqrt2Pi * exp(-0.5 * alpha * alpha) / st.m
                                 : exp(-0.5 * alpha * alpha - 0.5 * kLog2Pi - logd);
              if (isfinite(beta))
                rb_d = st.e == 0 ? kInvSqrt2Pi * exp(-0.5 * beta * beta) / st.m
                                 : exp(-0.5 * beta * beta - 0.5 * kLog2Pi - logd);
              const double y = st.y;
              // phi(x)/phi(y) = exp((y - x)(y + x)/2)
              const double ra_y = isfinite(alpha) ? (1.0 - w) * exp(0.5 * (y - alpha) * (y + alpha)) : 0.0;
              const double rb_y = isfinite(beta) ? w * exp(0.5 * (y - beta) * (y + beta)) : 0.0;
              abar = -omega * ra_d + ybar * ra_y;
              bbar = omega * rb_d + ybar * rb_y;
            }
            lds[k * kCols + lane] = -(abar + bbar) * rl;
            const double sa = wave_sum(abar * rl);
            const double sb = wave_sum(bbar * rl);
            if (lane == 0) {
              ga[i0 + k] = sa;
              gb[i0 + k] = sb;
            }
          }
        }
      }
      __syncthreads();
      // s-bar of the block -> scratch for the GEMMs of earlier blocks
      for (int e = t; e < rows * kCols; e += 256) Sb[(long)i0 * kCols + e] = lds[e];
      __syncthreads();
    }
  }
}

// scale_c = exp(M_c - M) / Z with M = max_c M_c, Z = sum_c Z_c exp(M_c - M).
__global__ __launch_bounds__(256) void grad_scale_kernel(const double* __restrict__ mz, long nchunks,
                                                         double* __restrict__ scale) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  double m = -INFINITY;
  for (long c = t; c < nchunks; c += 256) m = fmax(m, mz[2 * c]);
  red[t] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] = fmax(red[t], red[t + w]);
    __syncthreads();
  }
  const double M = red[0];
  __syncthreads();
  double z = 0.0;
  if (M > -INFINITY)
    for (long c = t; c < nchunks; c += 256)
      if (mz[2 * c] > -INFINITY) z += mz[2 * c + 1] * exp(mz[2 * c] - M);
  red[t] = z;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  const double Z = red[0];
  for (long c = t; c < nchunks; c += 256)
    scale[c] = (M > -INFINITY && mz[2 * c] > -INFINITY && Z > 0.0) ? exp(mz[2 * c] - M) / Z : 0.0;
  if (t == 0) scale[nchunks] = (M > -INFINITY && Z > 0.0) ? 1.0 : NAN;
}

// d/da_i = sum_c scale_c ga_c[i], same for b; d/dmu = -(d/da + d/db).
__global__ __launch_bounds__(256) void grad_sum_kernel(const double* __restrict__ gpart,
                                                       const double* __restrict__ scale, long nchunks, int n,
                                                       long ld, const int* __restrict__ info_factor,
                                                       const int* __restrict__ bad, double* __restrict__ da,
                                                       double* __restrict__ db, double* __restrict__ dmu) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const bool broken = (info_factor && *info_factor != 0) || (bad && *bad != INT_MAX) || isnan(scale[nchunks]);
  double sa = 0.0, sb = 0.0;
  for (long c = 0; c < nchunks; ++c) {
    const double f = scale[c];
    if (f != 0.0) {
      sa += f * gpart[c * 2 * ld + i];
      sb += f * gpart[c * 2 * ld + ld + i];
    }
  }
  if (broken) sa = sb = NAN;
  if (da) da[i] = sa;
  if (db) db[i] = sb;
  if (dmu) dmu[i] = -(sa + sb);
}

hipError_t launch_grad(const GradArgs& a, const int* info_factor, const int* bad, double* scale,
                       double* da, double* db, double* dmu, hipStream_t st) {
  switch (a.prec) {
    case 0: hipLaunchKernelGGL(grad_kernel<GemmF64>, dim3(a.grid), dim3(256), 0, st, a); break;
    case 1: hipLaunchKernelGGL(grad_kernel<GemmF32>, dim3(a.grid), dim3(256), 0, st, a); break;
    case 2: hipLaunchKernelGGL(grad_kernel<GemmBF16>, dim3(a.grid), dim3(256), 0, st, a); break;
    case 3: hipLaunchKernelGGL(grad_kernel<GemmBF16x3>, dim3(a.grid), dim3(256), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  const long nchunks = ((long)a.N * a.S + kCols - 1) / kCols;
  hipLaunchKernelGGL(grad_scale_kernel, dim3(1), dim3(256), 0, st, (const double*)a.mz, nchunks, scale);
  hipLaunchKernelGGL(grad_sum_kernel, dim3((a.n + 255) / 256), dim3(256), 0, st, (const double*)a.gpart,
                     (const double*)scale, nchunks, a.n, (long)a.ld, info_factor, bad, da, db, dmu);
  return hipGetLastError();
}

}  // namespace mvn
