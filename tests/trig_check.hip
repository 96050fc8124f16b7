// Host-side accuracy check of dst::fast_sincos against long-double libm.
#include <cmath>
#include <cstdio>
#include <random>

#include "dst_trig.h"

int main() {
  std::mt19937_64 rng(1309);
  std::uniform_real_distribution<double> wide(-7.0, 7.0), huge(-2.0e5, 2.0e5);
  long double worst_s = 0, worst_c = 0;
  long n = 0;
  auto check = [&](double x) {
    double s, c;
    dst::fast_sincos(x, &s, &c);
    const long double rs = sinl((long double)x), rc = cosl((long double)x);
    const long double es = fabsl((long double)s - rs), ec = fabsl((long double)c - rc);
    if (es > worst_s) worst_s = es;
    if (ec > worst_c) worst_c = ec;
    ++n;
  };
  for (int i = 0; i < 2000000; ++i) check(wide(rng));
  for (int i = 0; i < 200000; ++i) check(huge(rng));
  // quadrant edges and multiples of pi/4
  for (int k = -64; k <= 64; ++k) {
    const double b = k * 0.7853981633974483;
    for (double d : {0.0, 1e-12, -1e-12, 1e-6, -1e-6}) check(b + d);
  }
  check(0.0);
  check(-0.0);
  std::printf("%ld %.3Le %.3Le\n", n, worst_s, worst_c);
  return 0;
}
