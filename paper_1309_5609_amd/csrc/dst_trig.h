// cos(x) and sin(x) in FP64 for the polarisation rows cos 2psi, sin 2psi
// (Eqs. 3-6 of arXiv:1309.5609), cheaper than a general-purpose sincos.
//
// Method (Cody-Waite reduction plus Taylor series):
//   k = nearest integer to x * 2/pi,  r = x - k pi/2  with pi/2 split in three
//   parts C1 + C2 + C3 (C1, C2 carry 33 significant bits, so k*C1 and k*C2 are
//   exact for |k| < 2^16); then |r| <= pi/4 and
//     sin r = r - r^3/3! + ... + r^17/17!   (next term < 1e-19)
//     cos r = 1 - r^2/2! + ... + r^18/18!   (next term < 4e-21)
//   evaluated by Horner's rule in r^2; the quadrant k mod 4 selects signs and
//   swaps.  Error: a few units in the last place.  Arguments with |x| > 1e5
//   fall back to the standard library.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace dst {

__host__ __device__ __forceinline__ void fast_sincos(double x, double* s_out, double* c_out) {
  if (!(fabs(x) <= 1.0e5)) {
    *s_out = sin(x);
    *c_out = cos(x);
    return;
  }
  constexpr double kTwoOverPi = 0.6366197723675814;
  constexpr double C1 = 1.5707963267341256;
  constexpr double C2 = 6.077100506303966e-11;
  constexpr double C3 = 2.0222662487959506e-21;
  const double k = rint(x * kTwoOverPi);
  double r = fma(-k, C1, x);
  r = fma(-k, C2, r);
  r = fma(-k, C3, r);
  const double z = r * r;
  // inverse factorials
  constexpr double f2 = 1.0 / 2.0, f3 = 1.0 / 6.0, f4 = 1.0 / 24.0, f5 = 1.0 / 120.0, f6 = 1.0 / 720.0,
                   f7 = 1.0 / 5040.0, f8 = 1.0 / 40320.0, f9 = 1.0 / 362880.0, f10 = 1.0 / 3628800.0,
                   f11 = 1.0 / 39916800.0, f12 = 1.0 / 479001600.0, f13 = 1.0 / 6227020800.0,
                   f14 = 1.0 / 87178291200.0, f15 = 1.0 / 1307674368000.0, f16 = 1.0 / 20922789888000.0,
                   f17 = 1.0 / 355687428096000.0, f18 = 1.0 / 6402373705728000.0;
  double ps = fma(z, f17, -f15);
  ps = fma(z, ps, f13);
  ps = fma(z, ps, -f11);
  ps = fma(z, ps, f9);
  ps = fma(z, ps, -f7);
  ps = fma(z, ps, f5);
  ps = fma(z, ps, -f3);
  const double sr = fma(r * z, ps, r);
  double pc = fma(z, -f18, f16);
  pc = fma(z, pc, -f14);
  pc = fma(z, pc, f12);
  pc = fma(z, pc, -f10);
  pc = fma(z, pc, f8);
  pc = fma(z, pc, -f6);
  pc = fma(z, pc, f4);
  pc = fma(z, pc, -f2);
  const double cr = fma(z, pc, 1.0);
  const int q = (int)k & 3;
  const double s = (q & 1) ? cr : sr;
  const double c = (q & 1) ? sr : cr;
  *s_out = (q & 2) ? -s : s;
  *c_out = ((q + 1) & 2) ? -c : c;
}

}  // namespace dst
