// Monte Carlo noise on the GPU: white + 1/f timelines with the spectrum of
// Eq. 1 of arXiv:1309.5609, made by filtering white noise in the Fourier
// domain, segment by segment.
//
// * Random bits: Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC 2011), a
//   counter-based generator: block b of segment j of a stream is the
//   function of counter (b, j, 0, 0) and key (seed, stream), so any sample
//   can be drawn by any thread with no state.
// * Normals: Box-Muller on the top 53 bits of two words,
//   u1 in (0, 1], u2 in [0, 1): sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2).
// * Filter: segments of S = 2^m samples; two real segments travel as the real
//   and imaginary parts of one complex transform (the gain is real and even
//   in frequency, so it acts on each part separately); radix-4 / radix-2
//   Stockham passes (self-sorting, ping-pong buffers), gain
//   sqrt(1 + (f_k / |f|)^alpha) with the zero-frequency bin kept, inverse
//   transform, 1/S.  The last segment is drawn at full length and cut.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "dst_internal.h"

namespace dst {
namespace {

constexpr int kBlock = 256;
constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull, kM1 = 0xCA5A826395121157ull;
constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull, kW1 = 0xBB67AE8584CAA73Bull;

__device__ __forceinline__ void philox4x64_10(uint64_t (&x)[4], uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += kW0;
      k1 += kW1;
    }
    const uint64_t hi0 = __umul64hi(kM0, x[0]), lo0 = kM0 * x[0];
    const uint64_t hi1 = __umul64hi(kM1, x[2]), lo1 = kM1 * x[2];
    const uint64_t y0 = hi1 ^ x[1] ^ k0, y2 = hi0 ^ x[3] ^ k1;
    x[0] = y0;
    x[1] = lo1;
    x[2] = y2;
    x[3] = lo0;
  }
}

// Four unit normals of block b of segment seg.
__device__ __forceinline__ void normals4(uint64_t seed, uint64_t stream, uint64_t seg, uint64_t b, double (&z)[4]) {
  uint64_t x[4] = {b, seg, 0ull, 0ull};
  philox4x64_10(x, seed, stream);
  const double scale = 1.1102230246251565e-16;  // 2^-53
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const double u1 = ((double)(x[2 * p] >> 11) + 1.0) * scale;
    const double u2 = (double)(x[2 * p + 1] >> 11) * scale;
    const double r = sqrt(-2.0 * log(u1));
    double s, c;
    sincos((2.0 * M_PI) * u2, &s, &c);
    z[2 * p] = r * c;
    z[2 * p + 1] = r * s;
  }
}

// buf[p][k] = sigma (white(seg 2 (p0 + p), k), white(seg 2 (p0 + p) + 1, k)); imaginary part 0 past n_seg.
__global__ void __launch_bounds__(kBlock) k_white_pairs(uint64_t seed, uint64_t stream, int64_t p0, int64_t n_pairs,
                                                        int64_t n_seg, int64_t S, double sigma,
                                                        double2* __restrict__ buf) {
  const int64_t nb = S / 4;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_pairs * nb;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = g / nb, b = g - p * nb;
    const int64_t sa = 2 * (p0 + p), sb = sa + 1;
    double za[4], zb[4] = {0.0, 0.0, 0.0, 0.0};
    normals4(seed, stream, (uint64_t)sa, (uint64_t)b, za);
    if (sb < n_seg) normals4(seed, stream, (uint64_t)sb, (uint64_t)b, zb);
    double2* o = buf + p * S + 4 * b;
#pragma unroll
    for (int i = 0; i < 4; ++i) o[i] = make_double2(sigma * za[i], sigma * zb[i]);
  }
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// One self-sorting (Stockham) radix-R pass over `batch` transforms of N
// points at span Ns (the product of the radices of the earlier passes).
template <int R>
__global__ void __launch_bounds__(kBlock) k_fft_pass(const double2* __restrict__ in, double2* __restrict__ out,
                                                     int64_t N, int64_t Ns, int64_t batch, double sign) {
  const int64_t T = N / R;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < T * batch;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t bt = g / T, j = g - bt * T;
    const double2* x = in + bt * N;
    double2* y = out + bt * N;
    double2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = x[j + r * T];
    const int64_t k = j & (Ns - 1);
    if (Ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        double s, c;
        sincos(sign * (2.0 * M_PI) * (double)(r * k) / (double)(Ns * R), &s, &c);
        v[r] = cmul(v[r], make_double2(c, s));
      }
    }
    double2 X[R];
    if (R == 2) {
      X[0] = make_double2(v[0].x + v[1].x, v[0].y + v[1].y);
      X[1] = make_double2(v[0].x - v[1].x, v[0].y - v[1].y);
    } else {
      const double2 t0 = make_double2(v[0].x + v[2].x, v[0].y + v[2].y);
      const double2 t1 = make_double2(v[0].x - v[2].x, v[0].y - v[2].y);
      const double2 t2 = make_double2(v[1].x + v[3].x, v[1].y + v[3].y);
      const double2 d = make_double2(v[1].x - v[3].x, v[1].y - v[3].y);
      const double2 t3 = make_double2(-sign * d.y, sign * d.x);  // (sign i) d
      X[0] = make_double2(t0.x + t2.x, t0.y + t2.y);
      X[2] = make_double2(t0.x - t2.x, t0.y - t2.y);
      X[1] = make_double2(t1.x + t3.x, t1.y + t3.y);
      X[3] = make_double2(t1.x - t3.x, t1.y - t3.y);
    }
    const int64_t idx = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) y[idx + r * Ns] = X[r];
  }
}

// X[k] *= sqrt(1 + (f_k / |f|)^alpha) with |f| of bin k, bin 0 unchanged.
__global__ void __launch_bounds__(kBlock) k_filter(double2* __restrict__ buf, int64_t S, int64_t batch, double rate,
                                                   double fknee, double alpha) {
  const double d = 1.0 / rate;
  const double val = 1.0 / ((double)S * d);
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < S * batch;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = g & (S - 1);
    const int64_t kk = k <= S / 2 ? k : S - k;
    if (kk == 0) continue;
    const double f = (double)kk * val;
    const double h = sqrt(1.0 + pow(fknee / f, alpha));
    buf[g] = make_double2(buf[g].x * h, buf[g].y * h);
  }
}

template <typename OT>
__global__ void __launch_bounds__(kBlock) k_unpack(const double2* __restrict__ buf, int64_t p0, int64_t n_pairs,
                                                   int64_t S, int64_t n, double inv_s, int accumulate,
                                                   OT* __restrict__ out) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_pairs * S;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = g / S, k = g - p * S;
    const int64_t ta = 2 * (p0 + p) * S + k, tb = ta + S;
    const double2 v = buf[g];
    if (ta < n) out[ta] = accumulate ? (OT)((double)out[ta] + v.x * inv_s) : (OT)(v.x * inv_s);
    if (tb < n) out[tb] = accumulate ? (OT)((double)out[tb] + v.y * inv_s) : (OT)(v.y * inv_s);
  }
}

unsigned grid_for(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (unsigned)g;
}

// In-place (via the second buffer) transform of `batch` segments; returns the
// buffer holding the result.
double2* fft(double2* a, double2* b, int64_t S, int64_t batch, double sign, hipStream_t st) {
  int m = 0;
  while (((int64_t)1 << m) < S) ++m;
  int64_t Ns = 1;
  const unsigned g2 = grid_for(S / 2 * batch), g4 = grid_for(S / 4 * batch);
  if (m & 1) {
    hipLaunchKernelGGL(k_fft_pass<2>, dim3(g2), dim3(kBlock), 0, st, a, b, S, Ns, batch, sign);
    double2* t = a;
    a = b;
    b = t;
    Ns *= 2;
  }
  while (Ns < S) {
    hipLaunchKernelGGL(k_fft_pass<4>, dim3(g4), dim3(kBlock), 0, st, a, b, S, Ns, batch, sign);
    double2* t = a;
    a = b;
    b = t;
    Ns *= 4;
  }
  return a;
}

}  // namespace

int64_t noise_pairs_per_chunk(int64_t S) {
  const int64_t cap = (int64_t)1 << 24;  // complex values per buffer (256 MiB)
  return S >= cap ? 1 : cap / S;
}

hipError_t launch_noise(uint64_t seed, uint64_t stream, int64_t n, int64_t S, double rate, double sigma, double fknee,
                        double alpha, void* out, int out_f32, int accumulate, double2* buf0, double2* buf1,
                        hipStream_t st) {
  const int64_t n_seg = (n + S - 1) / S;
  const int64_t n_pairs = (n_seg + 1) / 2;
  const int64_t chunk = noise_pairs_per_chunk(S);
  for (int64_t p0 = 0; p0 < n_pairs; p0 += chunk) {
    const int64_t np = n_pairs - p0 < chunk ? n_pairs - p0 : chunk;
    hipLaunchKernelGGL(k_white_pairs, dim3(grid_for(np * (S / 4))), dim3(kBlock), 0, st, seed, stream, p0, np, n_seg,
                       S, sigma, buf0);
    double2* x = fft(buf0, buf1, S, np, -1.0, st);
    if (fknee > 0.0) {
      hipLaunchKernelGGL(k_filter, dim3(grid_for(S * np)), dim3(kBlock), 0, st, x, S, np, rate, fknee, alpha);
    }
    double2* other = x == buf0 ? buf1 : buf0;
    x = fft(x, other, S, np, 1.0, st);
    if (out_f32)
      hipLaunchKernelGGL(k_unpack<float>, dim3(grid_for(S * np)), dim3(kBlock), 0, st, x, p0, np, S, n,
                         1.0 / (double)S, accumulate, static_cast<float*>(out));
    else
      hipLaunchKernelGGL(k_unpack<double>, dim3(grid_for(S * np)), dim3(kBlock), 0, st, x, p0, np, S, n,
                         1.0 / (double)S, accumulate, static_cast<double*>(out));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace dst
