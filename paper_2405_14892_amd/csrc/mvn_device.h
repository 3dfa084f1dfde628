// Device (and host-testable) arithmetic of the SOV conditioning step.
//
// The step is Eq. (sov1) of arXiv 2405.14892, Section III-B: for a sample with
// conditional limits a', b' and uniform w,
//     d = Phi(b') - Phi(a'),   y = Phi^-1( Phi(a') + w d ),   l += log d.
// It is evaluated with exact identities that avoid cancellation:
//   * reflection (a', b', w) -> (-b', -a', 1-w), y -> -y when a' > 0, so the
//     lower end never sits in the upper tail;
//   * y from Phi^-1(p) when p = Phi(a') + u d <= 1/2, else from -Phi^-1(q)
//     with q = Phi(-b') + (1-u) d = 1 - p;
//   * log-scale d and p when b' < -35 (both ends deep in the lower tail).
// Phi uses erfc/erfcx; Phi^-1 is Wichura's algorithm AS 241 (PPND16, Applied
// Statistics 37, 1988), and the log-scale inverse is Newton's method on
// log Phi(y) = lp from the asymptotic expansion of the normal tail.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

#define MVN_HD __host__ __device__ __forceinline__
// Rare paths and check wrappers are kept out of line on the device so they
// add no register pressure where the common path is inlined.  (Host builds
// of this header, used to check the arithmetic on the CPU, inline them.)
#if defined(__HIP_DEVICE_COMPILE__)
#define MVN_HD_COLD __host__ __device__ __attribute__((noinline))
#else
#define MVN_HD_COLD __host__ __device__ inline
#endif

namespace mvn {

constexpr double kSqrt1_2 = 0.70710678118654752440;       // 1/sqrt(2)
constexpr double kSqrt2OverPi = 0.79788456080286535588;   // sqrt(2/pi)
constexpr double kLog2Pi = 1.83787706640934548356;        // log(2 pi)
constexpr double kDeepTail = -35.0;

// ---------------------------------------------------------------- Phi
// Phi(x) = erfc(-x/sqrt 2)/2; relative accuracy in the lower tail.
MVN_HD double ncdf(double x) { return 0.5 * erfc(-x * kSqrt1_2); }

// log Phi(x) for x <= 0 (any depth): log(erfcx(-x/sqrt2)/2) - x^2/2.
MVN_HD double log_ncdf_lower(double x) {
  if (x == -INFINITY) return -INFINITY;
  if (x > -5.0) return log(ncdf(x));
  return log(0.5 * erfcx(-x * kSqrt1_2)) - 0.5 * x * x;
}

// ---------------------------------------------------------------- Phi^-1
// AS 241 PPND16 for 0 < p <= 1/2 (returns a value <= 0).  Its three ranges
// (|p - 1/2| <= 0.425; sqrt(-log p) <= 5; beyond) are degree-7/7 rationals
// in a transformed variable.  Here each lane selects its variable and
// coefficients and evaluates one rational with one division, so a wave whose
// lanes fall in different ranges does not run every branch (the result is
// the same, operation for operation, as evaluating the lane's own branch).
//
// kAs241[g] = coefficients of range g (0 central, 1 near tail, 2 far tail):
// numerator n0 .. n7, denominator d1 .. d7 (d0 = 1), one zero of padding.
constexpr double kAs241[3][16] = {
    {3.3871328727963666080e+0, 1.3314166789178437745e+2, 1.9715909503065514427e+3, 1.3731693765509461125e+4,
     4.5921953931549871457e+4, 6.7265770927008700853e+4, 3.3430575583588128105e+4, 2.5090809287301226727e+3,
     4.2313330701600911252e+1, 6.8718700749205790830e+2, 5.3941960214247511077e+3, 2.1213794301586595867e+4,
     3.9307895800092710610e+4, 2.8729085735721942674e+4, 5.2264952788528545610e+3, 0.0},
    {1.42343711074968357734e+0, 4.63033784615654529590e+0, 5.76949722146069140550e+0, 3.64784832476320460504e+0,
     1.27045825245236838258e+0, 2.41780725177450611770e-1, 2.27238449892691845833e-2, 7.74545014278341407640e-4,
     2.05319162663775882187e+0, 1.67638483018380384940e+0, 6.89767334985100004550e-1, 1.48103976427480074590e-1,
     1.51986665636164571966e-2, 5.47593808499534494600e-4, 1.05075007164441684324e-9, 0.0},
    {6.65790464350110377720e+0, 5.46378491116411436990e+0, 1.78482653991729133580e+0, 2.96560571828504891230e-1,
     2.65321895265761230930e-2, 1.24266094738807843860e-3, 2.71155556874348757815e-5, 2.01033439929228813265e-7,
     5.99832206555887937690e-1, 1.36929880922735805310e-1, 1.48753612908506148525e-2, 7.86869131145613259100e-4,
     1.84631831751005468180e-5, 1.42151175831644588870e-7, 2.04426310338993978564e-15, 0.0}};

// The rational of range g in x from coefficient row c (16 entries as above).
template <class C>
MVN_HD void as241_rational(C c, double x, double& num, double& den) {
  num = (((((((c[7] * x + c[6]) * x + c[5]) * x + c[4]) * x + c[3]) * x + c[2]) * x + c[1]) * x + c[0]);
  den = (((((((c[14] * x + c[13]) * x + c[12]) * x + c[11]) * x + c[10]) * x + c[9]) * x + c[8]) * x + 1.0);
}

// Coefficients chosen per lane with selects between literal constants.
MVN_HD double ninv_lower(double p) {
  const double q = p - 0.5;
  const bool central = fabs(q) <= 0.425;
  const double rt = central ? 1.0 : sqrt(-log(p));
  const bool near = rt <= 5.0;
  const double x = central ? 0.180625 - q * q : (near ? rt - 1.6 : rt - 5.0);
  double c[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) c[k] = central ? kAs241[0][k] : (near ? kAs241[1][k] : kAs241[2][k]);
  double num, den;
  as241_rational(c, x, num, den);
  const double r = (central ? q * num : num) / den;
  return central ? r : -r;
}

// The same with the coefficients read from a copy of kAs241 (48 doubles,
// e.g. in LDS): one row address per lane instead of 31 two-way selects of
// 64-bit constants.  Same operations, same result.
template <class T>
MVN_HD double ninv_lower_tab(double p, T tab) {
  const double q = p - 0.5;
  const bool central = fabs(q) <= 0.425;
  const double rt = central ? 1.0 : sqrt(-log(p));
  const bool near = rt <= 5.0;
  const double x = central ? 0.180625 - q * q : (near ? rt - 1.6 : rt - 5.0);
  double num, den;
  as241_rational(tab + (central ? 0 : (near ? 16 : 32)), x, num, den);
  const double r = (central ? q * num : num) / den;
  return central ? r : -r;
}

// Phi^-1 from lp = log p, p tiny (lp < log 1e-300 allowed).  Start from the
// tail expansion log Phi(y) ~ -y^2/2 - log|y| - log(2 pi)/2, then Newton
// steps y <- y - (log Phi(y) - lp) / (phi(y)/Phi(y)).
MVN_HD double ninv_log(double lp) {
  if (lp > -680.0) return ninv_lower(exp(lp));
  if (lp == -INFINITY) return -INFINITY;
  const double t = -2.0 * lp - kLog2Pi;
  double y = -sqrt(t - log(t));
  for (int it = 0; it < 4; ++it) {
    const double z = -y * kSqrt1_2;
    const double ex = erfcx(z);
    const double f = log(0.5 * ex) - 0.5 * y * y - lp;
    const double mills = kSqrt2OverPi / ex;  // phi(y)/Phi(y)
    y -= f / mills;
  }
  return y;
}

// ---------------------------------------------------------------- the step
// Result of one step: y, and the factor d = m * 2^e (e = 0 except in the
// log-scale branch, where d itself would underflow; m = 0 marks a sample
// whose interval has zero mass).
struct Step {
  double y;
  double m;
  int e;
};

constexpr double kLn2 = 0.69314718055994530942;

// Both ends below -35: d and p from log Phi (y and d in the unreflected
// frame of (lo, hi)).  Rare, so out of line.
MVN_HD_COLD Step deep_tail(double lo, double hi, double u) {
  const double la = log_ncdf_lower(lo);
  const double lb = log_ncdf_lower(hi);
  const double logd = lb + log1p(-exp(la - lb));
  const double t = log(u) + logd;
  // logaddexp(la, t)
  const double mx = la > t ? la : t;
  const double lp = (mx == -INFINITY) ? -INFINITY : mx + log1p(exp(-fabs(la - t)));
  if (!(logd > -INFINITY)) return Step{0.0, 0.0, 0};
  const double ef = floor(logd / kLn2);
  return Step{ninv_log(lp), exp(logd - ef * kLn2), (int)ef};
}

// One conditioning step (see header comment).  w in (0,1); cw = 1 - w.
// ninv(p) is Phi^-1 on (0, 1/2] (ninv_lower or ninv_lower_tab).
template <class NInv>
MVN_HD Step condition_step_with(double alpha, double beta, double w, double cw, NInv ninv) {
  const bool refl = alpha > 0.0;
  const double lo = refl ? -beta : alpha;
  const double hi = refl ? -alpha : beta;
  const double u = refl ? cw : w;
  const double v = refl ? w : cw;
  Step st;
  if (!(hi < kDeepTail)) {
    // Phi(-inf) = 0 needs no erfc (every row with an infinite lower limit)
    const double pa = (lo == -INFINITY) ? 0.0 : ncdf(lo);
    // one erfc serves both Phi(hi) and Phi(-hi)
    const double e = 0.5 * erfc(fabs(hi) * kSqrt1_2);
    const double pb = hi > 0.0 ? 1.0 - e : e;
    const double qb = hi > 0.0 ? e : 1.0 - e;
    const double d = pb - pa;
    const double p = pa + u * d;
    // one Phi^-1 evaluation: the argument is chosen first, so lanes of a
    // wave that take different sides do not run the function twice
    const bool low = p <= 0.5;
    const double t = ninv(low ? p : qb + v * d);
    st.y = low ? t : -t;
    st.m = d;
    st.e = 0;
  } else {
    st = deep_tail(lo, hi, u);
  }
  if (!(st.m > 0.0)) {  // zero mass (or NaN): dead sample
    st.y = 0.0;
    st.m = 0.0;
    st.e = 0;
  }
  if (refl) st.y = -st.y;
  return st;
}

MVN_HD Step condition_step(double alpha, double beta, double w, double cw) {
  return condition_step_with(alpha, beta, w, cw, [](double x) { return ninv_lower(x); });
}

// ---------------------------------------------------------------- the step, reduced precision
// Single-precision AS 241 (PPND7, about 7 significant digits) for
// 0 < p <= 1/2, with the same range selection as ninv_lower.
MVN_HD float ninv_lower_f32(float p) {
  const float q = p - 0.5f;
  const bool central = fabsf(q) <= 0.425f;
  const float rt = central ? 1.0f : sqrtf(-logf(p));
  const bool near = rt <= 5.0f;
  const float x = central ? 0.180625f - q * q : (near ? rt - 1.6f : rt - 5.0f);
#define MVN_SEL(c, n, f) (central ? (c) : (near ? (n) : (f)))
  const float n3 = MVN_SEL(5.9109374720e+1f, 1.7023821103e-1f, 1.7337203997e-2f);
  const float n2 = MVN_SEL(1.5929113202e+2f, 1.3067284816e+0f, 4.2868294337e-1f);
  const float n1 = MVN_SEL(5.0434271938e+1f, 2.7568153900e+0f, 3.0812263860e+0f);
  const float n0 = MVN_SEL(3.3871327179e+0f, 1.4234372777e+0f, 6.6579051150e+0f);
  const float d3 = MVN_SEL(6.7187563600e+1f, 0.0f, 0.0f);
  const float d2 = MVN_SEL(7.8757757664e+1f, 1.2021132975e-1f, 1.2258202635e-2f);
  const float d1 = MVN_SEL(1.7895169469e+1f, 7.3700164250e-1f, 2.4197894225e-1f);
#undef MVN_SEL
  const float num = ((n3 * x + n2) * x + n1) * x + n0;
  const float den = ((d3 * x + d2) * x + d1) * x + 1.0f;
  const float r = (central ? q * num : num) / den;
  return central ? r : -r;
}

// The conditioning step of the reduced-precision modes: Phi and Phi^-1 in
// FP32 where that keeps log d and y within a few 1e-6: both limits at or
// above -5 (rounding a limit x to FP32 moves log Phi(x) by about
// x^2 * 6e-8) and d = Phi(b') - Phi(a') at least half of Phi(b') (at most one
// bit cancels).  Every other lane (lower tails, narrow intervals) takes the
// FP64 step.  The factor d is returned in
// FP64 and accumulated in log space as in the FP64 step.
template <class NInv>
MVN_HD Step condition_step_mixed_with(double alpha, double beta, double w, double cw, NInv ninv) {
  const bool refl = alpha > 0.0;
  const double lo = refl ? -beta : alpha;
  const double hi = refl ? -alpha : beta;
  bool ok = hi >= -5.0 && (lo == -INFINITY || lo >= -5.0);
  Step st{0.0, 0.0, 0};
  if (ok) {
    const float his = (float)hi;
    const float e = 0.5f * erfcf(fabsf(his) * 0.70710678f);
    const float pb = his > 0.0f ? 1.0f - e : e;
    const float qb = his > 0.0f ? e : 1.0f - e;
    const float pa = (lo == -INFINITY) ? 0.0f : 0.5f * erfcf(-(float)lo * 0.70710678f);
    const float d = pb - pa;
    ok = d >= 0.5f * pb && d > 0.0f;
    const float u = (float)(refl ? cw : w), v = (float)(refl ? w : cw);
    const float p = pa + u * d;
    const bool low = p <= 0.5f;
    const float t = ninv_lower_f32(low ? p : qb + v * d);
    st.y = (double)(low ? t : -t);
    st.m = (double)d;
    if (refl) st.y = -st.y;
  }
  if (!ok) st = condition_step_with(alpha, beta, w, cw, ninv);
  return st;
}

MVN_HD Step condition_step_mixed(double alpha, double beta, double w, double cw) {
  return condition_step_mixed_with(alpha, beta, w, cw, [](double x) { return ninv_lower(x); });
}

// Running product of the d_i as m * 2^e with m renormalised into [1/2, 1)
// after every factor: exact exponent bookkeeping, one log per sample at
// the end instead of one per step.
struct LogProd {
  double m;
  int e;
};

MVN_HD void logprod_mul(LogProd& a, const Step& s) {
  int k;
  a.m = frexp(a.m * s.m, &k);
  a.e += k + s.e;
}

MVN_HD double logprod_log(const LogProd& a) {
  return a.m > 0.0 ? log(a.m) + (double)a.e * kLn2 : -INFINITY;
}

// (y, log d) of one step, for checks of the arithmetic.
struct StepLog {
  double y;
  double logd;
};

MVN_HD_COLD StepLog condition(double alpha, double beta, double w, double cw) {
  const Step s = condition_step(alpha, beta, w, cw);
  return StepLog{s.y, s.m > 0.0 ? log(s.m) + (double)s.e * kLn2 : -INFINITY};
}

// ---------------------------------------------------------------- QMC points
// SplitMix64 output k (0-based) from state `seed` (Steele, Lea & Flood 2014).
MVN_HD uint64_t splitmix64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Standard normal number k from the counter-based stream of `seed`:
// Phi^-1(U), U = ((SplitMix64 output k) >> 11) + 1/2) 2^-53, Phi^-1 by AS 241
// (the upper half by symmetry; 1 - U is exact there).
MVN_HD double normal_from_counter(uint64_t seed, uint64_t k) {
  const double u = ((double)(splitmix64(seed, k) >> 11) + 0.5) * 0x1.0p-53;
  return u <= 0.5 ? ninv_lower(u) : -ninv_lower(1.0 - u);
}

// Richtmyer point j (1-based) of dimension with generator A and shift D.
MVN_HD double richtmyer(uint64_t j, uint64_t A, uint64_t D, int periodize) {
  const uint64_t x = j * A + D;
  double w = ((double)(x >> 11) + 0.5) * 0x1.0p-53;
  if (periodize) w = 1.0 - fabs(2.0 * w - 1.0);
  return w;
}

}  // namespace mvn
