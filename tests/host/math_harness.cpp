// Host build of the device conditioning arithmetic, for CPU checks of the
// AS 241 coefficients and the branch structure against SciPy.
// Reads lines "op x [y w]" from stdin and prints results with %.17g.
#include <cmath>
#include <cstdio>
#include <cstring>

// erfcx for the host build only: exp(x^2) erfc(x) in long double, with the
// continued-fraction tail for large x.
static double host_erfcx(double x) {
  if (x < 25.0) return (double)(expl((long double)x * x) * erfcl((long double)x));
  long double t = x, s = 1.0L / (t * sqrtl(3.14159265358979323846264338327950288L));
  long double x2 = 2.0L * t * t;
  return (double)(s * (1.0L - 1.0L / x2 + 3.0L / (x2 * x2) - 15.0L / (x2 * x2 * x2)));
}
__host__ double erfcx(double x) { return host_erfcx(x); }

#include "../../paper_2405_14892_amd/csrc/matern.h"
#include "../../paper_2405_14892_amd/csrc/mvn_device.h"

int main() {
  char op[32];
  double x, y, w;
  while (scanf("%31s", op) == 1) {
    if (!strcmp(op, "ninv")) {
      scanf("%lf", &x);
      printf("%.17g\n", mvn::ninv_lower(x));
    } else if (!strcmp(op, "ninvtab")) {  // table form == select form, bit for bit
      scanf("%lf", &x);
      const double a = mvn::ninv_lower(x), b = mvn::ninv_lower_tab(x, &mvn::kAs241[0][0]);
      printf("%d\n", memcmp(&a, &b, sizeof a) == 0 ? 1 : 0);
    } else if (!strcmp(op, "ninvlog")) {
      scanf("%lf", &x);
      printf("%.17g\n", mvn::ninv_log(x));
    } else if (!strcmp(op, "lncdf")) {
      scanf("%lf", &x);
      printf("%.17g\n", mvn::log_ncdf_lower(x));
    } else if (!strcmp(op, "cond")) {
      scanf("%lf %lf %lf", &x, &y, &w);
      mvn::StepLog s = mvn::condition(x, y, w, 1.0 - w);
      printf("%.17g %.17g\n", s.y, s.logd);
    } else if (!strcmp(op, "condmix")) {
      scanf("%lf %lf %lf", &x, &y, &w);
      mvn::Step s = mvn::condition_step_mixed(x, y, w, 1.0 - w);
      const double ld = s.m > 0.0 ? std::log(s.m) + (double)s.e * mvn::kLn2 : -INFINITY;
      printf("%.17g %.17g\n", s.y, ld);
    } else if (!strcmp(op, "ninv32")) {
      scanf("%lf", &x);
      printf("%.17g\n", (double)mvn::ninv_lower_f32((float)x));
    } else if (!strcmp(op, "sm")) {
      unsigned long long seed, k;
      scanf("%llu %llu", &seed, &k);
      printf("%llu\n", (unsigned long long)mvn::splitmix64(seed, k));
    } else if (!strcmp(op, "lkv")) {  // log(e^x K_nu(x))
      scanf("%lf %lf", &x, &y);
      printf("%.17g\n", mvn::log_bessel_k_scaled(x, y));
    } else if (!strcmp(op, "matern")) {  // sigma2 beta nu h
      double s2, be, nu, hh;
      scanf("%lf %lf %lf %lf", &s2, &be, &nu, &hh);
      printf("%.17g\n", mvn::matern_cov(mvn::make_matern(s2, be, nu, 0.0), hh));
    } else if (!strcmp(op, "mcn")) {  // normal number k of the counter-based stream
      unsigned long long seed, k;
      scanf("%llu %llu", &seed, &k);
      printf("%.17g\n", mvn::normal_from_counter(seed, k));
    }
  }
  return 0;
}
