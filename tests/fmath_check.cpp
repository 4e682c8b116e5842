// Host check of the library's double exp, log and reciprocal-based division against long double
// (x86 80-bit) references: prints the largest error in ulp of the double result over argument
// sweeps, then the special cases.  Built and run by test_fmath.py.
#include <stdio.h>
#include <math.h>
#include <stdint.h>
#include "fmath.h"

static double ulp_err(double got, long double ref) {
  const double r = (double)ref;
  const double u = nextafter(fabs(r), INFINITY) - fabs(r);
  return (double)(fabsl((long double)got - ref) / (long double)u);
}

int main() {
  uint64_t s = 0x9e3779b97f4a7c15ull;
  auto uni = [&]() {  // splitmix64 -> [0, 1)
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return (double)((z ^ (z >> 31)) >> 11) * 0x1p-53;
  };
  double emax = 0.0, lmax = 0.0, exw = 0.0, lxw = 0.0;
  for (int i = 0; i < 4000000; ++i) {
    // exp: arguments across the normal range, denser near 0
    const double x = i % 2 ? -708.0 + 1417.0 * uni() : (uni() - 0.5) * 40.0 * uni();
    const double e = ulp_err(ism::fexp(x), expl((long double)x));
    if (e > emax) { emax = e; exw = x; }
    // log: log-uniform over the normal range, and near 1
    const double y = i % 2 ? exp2(-1020.0 + 2040.0 * uni()) : 1.0 + (uni() - 0.5) * 1e-3 * uni();
    const double l = ulp_err(ism::flog(y), logl((long double)y));
    if (l > lmax) { lmax = l; lxw = y; }
  }
  // division: quotients of log-uniform operands over the range the callers allow
  double dmax = 0.0, dxw = 0.0;
  for (int i = 0; i < 2000000; ++i) {
    const double a = exp2(-300.0 + 600.0 * uni()) * (uni() < 0.5 ? -1.0 : 1.0);
    const double b = exp2(-990.0 + 1980.0 * uni());
    const double d = ulp_err(ism::fdivp(a, b), (long double)a / (long double)b);
    if (d > dmax) { dmax = d; dxw = b; }
  }
  printf("div_max_ulp %.4f at %.17g\n", dmax, dxw);
  printf("exp_max_ulp %.4f at %.17g\n", emax, exw);
  printf("log_max_ulp %.4f at %.17g\n", lmax, lxw);
  // special cases: saturation, exact values, non-finite arguments
  printf("exp_special %d\n", ism::fexp(-800.0) == 0.0 && isinf(ism::fexp(800.0)) && ism::fexp(0.0) == 1.0 &&
                                 ism::fexp(NAN) == 0.0 && ism::fexp(-INFINITY) == 0.0);
  printf("log_special %d\n", ism::flog(1.0) == 0.0 && isinf(ism::flog(0.0)) && ism::flog(0.0) < 0 &&
                                 isinf(ism::flog(INFINITY)) && isnan(ism::flog(-1.0)) && isnan(ism::flog(NAN)));
  return 0;
}
