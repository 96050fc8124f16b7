// Pointing expansion on the GPU: pixel index (HEALPix RING) and polarisation
// angle per sample of a spinning ground scan at fixed elevation, the input the
// destriper takes (the pointing of the Polarimeters data section and the
// parallactic-angle footnote of the Algorithm section), computed where it is
// used instead of streamed from the host.
//
// Geometry: the telescope spins about the vertical at constant elevation; the
// textbook alt-az -> equatorial transform gives declination, hour angle and
// parallactic angle, which repeat every spin period, so they are tabulated
// once per period on the host (n_period entries, C library functions).  Per
// sample only the local sidereal time advances: RA = LST - H.  The RING index
// follows the HEALPix geometry (Gorski et al. 2005): equal-area rings, belt
// pixels bounded by the lines tt -+ 3z/4 = const in the (tt = 2 phi / pi, z)
// plane, cap pixels by tp N sqrt(3 (1 - |z|)) = const and
// (1 - tp) N sqrt(3 (1 - |z|)) = const.
//
// Every step is a correctly rounded IEEE operation (add, multiply, divide,
// sqrt, floor, fmod) evaluated in a fixed order with contraction off, so the
// result is reproducible bit for bit by any implementation that evaluates the
// same expressions in the same order on the same table.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <vector>

#include "dst_internal.h"

#pragma clang fp contract(off)

namespace dst {
namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ int64_t ring_pixel(int64_t n, double z, double phi) {
  const double twopi = 2.0 * M_PI;
  const double za = fabs(z);
  // floor modulo (result in [0, 2 pi)), then the wrap of a result equal to 2 pi
  double ph = fmod(phi, twopi);
  if (ph != 0.0 && ((ph < 0.0) != (twopi < 0.0))) ph += twopi;
  if (ph >= twopi) ph = 0.0;
  const double tt = ph / (0.5 * M_PI);
  const double nd = (double)n;
  if (za <= 2.0 / 3.0) {
    const double a = nd * (0.5 + tt);
    const double b = (0.75 * nd) * z;
    const int64_t jp = (int64_t)floor(a - b);
    const int64_t jm = (int64_t)floor(a + b);
    const int64_t ir = n + 1 + jp - jm;
    const int64_t kshift = 1 - (ir & 1);
    int64_t ip = (jp + jm - n + kshift + 1) / 2;
    ip %= 4 * n;
    if (ip < 0) ip += 4 * n;
    return 2 * n * (n - 1) + (ir - 1) * 4 * n + ip;
  }
  const double tp = tt - floor(tt);
  const double tmp = nd * sqrt(3.0 * (1.0 - za));
  const int64_t jp = (int64_t)floor(tp * tmp);
  const int64_t jm = (int64_t)floor((1.0 - tp) * tmp);
  const int64_t ir = jp + jm + 1;
  int64_t ip = (int64_t)floor(tt * (double)ir);
  ip %= 4 * ir;
  if (ip < 0) ip += 4 * ir;
  return z > 0.0 ? 2 * ir * (ir - 1) + ip : 12 * n * n - 2 * ir * (ir + 1) + ip;
}

// tab: [3][n_per] = hour angle, cos(colatitude), polarisation angle.
template <typename PT>
__global__ void __launch_bounds__(kBlock) k_expand(int64_t nside, int64_t start, int64_t n, int64_t n_per,
                                                   double rate, double lst0, double sidereal,
                                                   const double* __restrict__ tab, int32_t* __restrict__ pix,
                                                   PT* __restrict__ psi) {
  const double* ha = tab;
  const double* zt = tab + n_per;
  const double* pt = tab + 2 * n_per;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t idx = start + k;
    const int64_t ph = idx % n_per;
    const double t = (double)idx / rate;
    const double lst = lst0 + ((2.0 * M_PI) * t) / sidereal;
    const double ra = lst - ha[ph];
    pix[k] = (int32_t)ring_pixel(nside, zt[ph], ra);
    if (psi) psi[k] = (PT)pt[ph];
  }
}

}  // namespace

// Host table of one spin period, evaluated in the order the expressions are
// written (C library sin, cos, tan, asin, atan2).
void scan_period_table(const dst_scan& s, int64_t n_per, std::vector<double>& tab) {
  tab.assign(3 * (size_t)n_per, 0.0);
  const double d2r = M_PI / 180.0;
  const double el = s.elevation_deg * d2r;
  const double lat = s.latitude_deg * d2r;
  const double az0 = s.az0_deg * d2r;
  const double psi0 = s.psi0_deg * d2r;
  for (int64_t i = 0; i < n_per; ++i) {
    const double t = (double)i / s.sample_rate_hz;
    const double az = az0 + ((2.0 * M_PI) * t) / s.spin_period_s;
    const double sin_dec = std::sin(el) * std::sin(lat) + (std::cos(el) * std::cos(lat)) * std::cos(az);
    const double dec = std::asin(std::fmin(1.0, std::fmax(-1.0, sin_dec)));
    const double h = std::atan2((-std::sin(az)) * std::cos(el),
                                std::cos(lat) * std::sin(el) - (std::sin(lat) * std::cos(el)) * std::cos(az));
    const double q = std::atan2(std::sin(h), std::tan(lat) * std::cos(dec) - std::sin(dec) * std::cos(h));
    tab[i] = h;
    tab[n_per + i] = std::cos(0.5 * M_PI - dec);
    tab[2 * n_per + i] = q + psi0;
  }
}

hipError_t launch_expand(int64_t nside, int64_t start, int64_t n, int64_t n_per, const dst_scan& s, const double* tab,
                         int32_t* pix, void* psi, int psi_f32, hipStream_t st) {
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  if (psi_f32)
    hipLaunchKernelGGL(k_expand<float>, dim3((unsigned)g), dim3(kBlock), 0, st, nside, start, n, n_per,
                       s.sample_rate_hz, s.lst0_rad, s.sidereal_day_s, tab, pix, static_cast<float*>(psi));
  else
    hipLaunchKernelGGL(k_expand<double>, dim3((unsigned)g), dim3(kBlock), 0, st, nside, start, n, n_per,
                       s.sample_rate_hz, s.lst0_rad, s.sidereal_day_s, tab, pix, static_cast<double*>(psi));
  return hipGetLastError();
}

}  // namespace dst
