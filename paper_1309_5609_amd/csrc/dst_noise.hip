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
//   in frequency, so it acts on each part separately); self-sorting
//   Stockham passes of radix up to 256, each computed in LDS (see fft), gain
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

// ---------------------------------------------------------------- FFT
// Self-sorting (Stockham) transform of length S = 2^m in passes of radix
// R = 2^r (r <= kFftMaxLog, the bits of m spread evenly over the passes).
// Pass with span Ns (the product of the earlier radices), for column j of
// each transform (0 <= j < T = S / R, k = j mod Ns):
//   v_r = x[j + r T] w^{r k},  w = exp(sign 2 pi i / (Ns R)),
//   X_q = sum_r v_r exp(sign 2 pi i r q / R),
//   y[(j / Ns) Ns R + k + q Ns] = X_q.
// A workgroup holds TC = kFftElems / R columns in LDS (loaded so that
// neighbouring lanes touch neighbouring addresses) and computes their
// length-R transforms there by the same recursion with radices 2 and 4, so a
// pass reads and writes each value once.  Twiddles: w^E for E in units of
// 1 / S of a turn, from two tables, hi[E >> h] lo[E mod 2^h], made once per
// length with sincospi.
constexpr int kFftElems = 2048;  // complex values per workgroup
constexpr int kFftMaxLog = 8;

struct Twiddles {
  const double2* hi;  // exp(-2 pi i a 2^h / S), a < S / 2^h
  const double2* lo;  // exp(-2 pi i b / S), b < 2^h
  int h;
  int64_t S;
};

// exp(sign 2 pi i E / S)
__device__ __forceinline__ double2 twiddle(const Twiddles& t, int64_t E, double sign) {
  E &= t.S - 1;
  double2 w = cmul(t.hi[E >> t.h], t.lo[E & (((int64_t)1 << t.h) - 1)]);
  if (sign > 0.0) w.y = -w.y;
  return w;
}

__global__ void __launch_bounds__(kBlock) k_twiddles(double2* __restrict__ hi, double2* __restrict__ lo, int h,
                                                     int m) {
  const int64_t nh = (int64_t)1 << (m - h), nl = (int64_t)1 << h;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nh + nl; i += (int64_t)gridDim.x * blockDim.x) {
    // angle -2 pi x, x = a / nh or b / S, as sincospi of -2x (exact arguments)
    double s, c;
    if (i < nh) {
      sincospi(-2.0 * (double)i / (double)nh, &s, &c);
      hi[i] = make_double2(c, s);
    } else {
      sincospi(-2.0 * (double)(i - nh) / (double)(nh * nl), &s, &c);
      lo[i - nh] = make_double2(c, s);
    }
  }
}

// One radix-RAD stage of the in-LDS transforms of length R (columns of
// stride LS), span ns; WR[i] = exp(sign 2 pi i i / R).
template <int RAD>
__device__ __forceinline__ void lds_stage(double2* L, int R, int LS, int ns, const double2* WR, double sign) {
  constexpr int PER = kFftElems / RAD / kBlock;  // butterflies per thread
  const int nbf = R / RAD;
  double2 v[PER][RAD];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int idx = threadIdx.x + kBlock * i;
    const int c = idx / nbf, j = idx - c * nbf;
#pragma unroll
    for (int q = 0; q < RAD; ++q) v[i][q] = L[c * LS + j + q * nbf];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int idx = threadIdx.x + kBlock * i;
    const int c = idx / nbf, j = idx - c * nbf;
    const int k = j & (ns - 1);
    if (ns > 1) {
      const int unit = R / (ns * RAD);
#pragma unroll
      for (int q = 1; q < RAD; ++q) v[i][q] = cmul(v[i][q], WR[q * k * unit]);
    }
    double2 X[RAD];
    if (RAD == 2) {
      X[0] = make_double2(v[i][0].x + v[i][1].x, v[i][0].y + v[i][1].y);
      X[1] = make_double2(v[i][0].x - v[i][1].x, v[i][0].y - v[i][1].y);
    } else {
      const double2 t0 = make_double2(v[i][0].x + v[i][2].x, v[i][0].y + v[i][2].y);
      const double2 t1 = make_double2(v[i][0].x - v[i][2].x, v[i][0].y - v[i][2].y);
      const double2 t2 = make_double2(v[i][1].x + v[i][3].x, v[i][1].y + v[i][3].y);
      const double2 d = make_double2(v[i][1].x - v[i][3].x, v[i][1].y - v[i][3].y);
      const double2 t3 = make_double2(-sign * d.y, sign * d.x);  // (sign i) d
      X[0] = make_double2(t0.x + t2.x, t0.y + t2.y);
      X[2] = make_double2(t0.x - t2.x, t0.y - t2.y);
      X[1] = make_double2(t1.x + t3.x, t1.y + t3.y);
      X[3] = make_double2(t1.x - t3.x, t1.y - t3.y);
    }
    const int o = (j / ns) * ns * RAD + k;
#pragma unroll
    for (int q = 0; q < RAD; ++q) L[c * LS + o + q * ns] = X[q];
  }
  __syncthreads();
}

// The gain of Eq. 1's filter at bin k of a length-S transform:
// sqrt(1 + (f_k / |f|)^alpha), 1 at zero frequency.
struct Gain {
  double fknee = 0.0, alpha = 0.0, df = 0.0;  // df: bin spacing (rate / S); fknee = 0: no filter
};
__device__ __forceinline__ double gain_at(const Gain& G, int64_t k, int64_t S) {
  const int64_t kk = k <= S / 2 ? k : S - k;
  if (kk == 0) return 1.0;
  return sqrt(1.0 + pow(G.fknee / ((double)kk * G.df), G.alpha));
}

// One pass of radix R = 2^LOGR over `batch` transforms of length S, span Ns;
// with G.fknee > 0 (first pass only) the inputs are first scaled by the gain
// of their bin.
template <int LOGR>
__global__ void __launch_bounds__(kBlock) k_fft_lds(const double2* __restrict__ in, double2* __restrict__ out,
                                                    int64_t S, int64_t Ns, int64_t batch, double sign, Twiddles tw,
                                                    Gain G) {
  constexpr int R = 1 << LOGR, TC = kFftElems / R, LS = R + 1;  // LS: padded column stride
  __shared__ double2 L[TC * LS];
  __shared__ double2 WR[R];
  for (int i = threadIdx.x; i < R; i += kBlock) WR[i] = twiddle(tw, (int64_t)i * (S / R), sign);
  const int64_t T = S / R, ncol = batch * T;
  const bool in_cfast = T >= TC, out_cfast = Ns >= TC;  // lane order that keeps accesses contiguous
  for (int64_t g0 = (int64_t)blockIdx.x * TC; g0 < ncol; g0 += (int64_t)gridDim.x * TC) {
#pragma unroll 4
    for (int i = 0; i < kFftElems / kBlock; ++i) {
      const int idx = threadIdx.x + kBlock * i;
      const int c = in_cfast ? idx % TC : idx / R, r = in_cfast ? idx / TC : idx % R;
      const int64_t g = g0 + c;
      double2 x = make_double2(0.0, 0.0);
      if (g < ncol) {
        const int64_t bt = g / T, j = g - bt * T;
        x = in[bt * S + j + r * T];
        const int64_t k = j & (Ns - 1);
        if (Ns > 1 && r > 0) x = cmul(x, twiddle(tw, (int64_t)r * k * (S / (Ns * R)), sign));
      }
      L[c * LS + r] = x;
    }
    __syncthreads();
    if (G.fknee > 0.0) {  // first pass (Ns = 1): element (c, r) is bin j + r T
      for (int idx = threadIdx.x; idx < kFftElems; idx += kBlock) {
        const int c = idx / R, r = idx % R;
        const int64_t g = g0 + c;
        if (g >= ncol) continue;
        const int64_t j = g % T;
        const double h = gain_at(G, j + r * T, S);
        L[c * LS + r] = make_double2(L[c * LS + r].x * h, L[c * LS + r].y * h);
      }
      __syncthreads();
    }
    int ns = 1;
    if (LOGR & 1) {
      lds_stage<2>(L, R, LS, ns, WR, sign);
      ns = 2;
    }
#pragma unroll 1
    for (; ns < R; ns *= 4) lds_stage<4>(L, R, LS, ns, WR, sign);
#pragma unroll 4
    for (int i = 0; i < kFftElems / kBlock; ++i) {
      const int idx = threadIdx.x + kBlock * i;
      const int c = out_cfast ? idx % TC : idx / R, q = out_cfast ? idx / TC : idx % R;
      const int64_t g = g0 + c;
      if (g < ncol) {
        const int64_t bt = g / T, j = g - bt * T;
        out[bt * S + (j / Ns) * Ns * R + (j & (Ns - 1)) + q * Ns] = L[c * LS + q];
      }
    }
    __syncthreads();  // the next column group reuses L
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

int log2_of(int64_t S) {
  int m = 0;
  while (((int64_t)1 << m) < S) ++m;
  return m;
}

// Transform of `batch` segments through the two buffers (a holds the input);
// returns the buffer holding the result.
double2* fft(double2* a, double2* b, int64_t S, int64_t batch, double sign, const Twiddles& tw, const Gain& gain,
             hipStream_t st) {
  const int m = log2_of(S);
  const int P = (m + kFftMaxLog - 1) / kFftMaxLog;  // passes
  int64_t Ns = 1;
  for (int p = 0; p < P; ++p) {
    const int r = m / P + (p < m % P ? 1 : 0);
    const int64_t groups = (batch * (S >> r) + (kFftElems >> r) - 1) / (kFftElems >> r);
    const unsigned g = (unsigned)(groups < 65536 ? groups : 65536);
    const Gain G = p == 0 ? gain : Gain{};
    switch (r) {
      case 1: hipLaunchKernelGGL(k_fft_lds<1>, dim3(g), dim3(kBlock), 0, st, a, b, S, Ns, batch, sign, tw, G); break;
      case 2: hipLaunchKernelGGL(k_fft_lds<2>, dim3(g), dim3(kBlock), 0, st, a, b, S, Ns, batch, sign, tw, G); break;
      case 3: hipLaunchKernelGGL(k_fft_lds<3>, dim3(g), dim3(kBlock), 0, st, a, b, S, Ns, batch, sign, tw, G); break;
      case 4: hipLaunchKernelGGL(k_fft_lds<4>, dim3(g), dim3(kBlock), 0, st, a, b, S, Ns, batch, sign, tw, G); break;
      case 5: hipLaunchKernelGGL(k_fft_lds<5>, dim3(g), dim3(kBlock), 0, st, a, b, S, Ns, batch, sign, tw, G); break;
      case 6: hipLaunchKernelGGL(k_fft_lds<6>, dim3(g), dim3(kBlock), 0, st, a, b, S, Ns, batch, sign, tw, G); break;
      case 7: hipLaunchKernelGGL(k_fft_lds<7>, dim3(g), dim3(kBlock), 0, st, a, b, S, Ns, batch, sign, tw, G); break;
      default: hipLaunchKernelGGL(k_fft_lds<8>, dim3(g), dim3(kBlock), 0, st, a, b, S, Ns, batch, sign, tw, G); break;
    }
    double2* t = a;
    a = b;
    b = t;
    Ns <<= r;
  }
  return a;
}

}  // namespace

int64_t noise_twiddle_count(int64_t S) {
  const int m = log2_of(S), h = (m + 1) / 2;
  return ((int64_t)1 << (m - h)) + ((int64_t)1 << h);
}

int64_t noise_pairs_per_chunk(int64_t S) {
  const int64_t cap = (int64_t)1 << 24;  // complex values per buffer (256 MiB)
  return S >= cap ? 1 : cap / S;
}

hipError_t launch_noise(uint64_t seed, uint64_t stream, int64_t n, int64_t S, double rate, double sigma, double fknee,
                        double alpha, void* out, int out_f32, int accumulate, double2* buf0, double2* buf1,
                        double2* twbuf, hipStream_t st) {
  if (S < 4 || (S & (S - 1))) return hipErrorInvalidValue;
  const int m = log2_of(S), h = (m + 1) / 2;
  Twiddles tw;
  tw.hi = twbuf;
  tw.lo = twbuf + ((int64_t)1 << (m - h));
  tw.h = h;
  tw.S = S;
  hipLaunchKernelGGL(k_twiddles, dim3(grid_for(noise_twiddle_count(S))), dim3(kBlock), 0, st, twbuf,
                     twbuf + ((int64_t)1 << (m - h)), h, m);
  const int64_t n_seg = (n + S - 1) / S;
  const int64_t n_pairs = (n_seg + 1) / 2;
  const int64_t chunk = noise_pairs_per_chunk(S);
  for (int64_t p0 = 0; p0 < n_pairs; p0 += chunk) {
    const int64_t np = n_pairs - p0 < chunk ? n_pairs - p0 : chunk;
    hipLaunchKernelGGL(k_white_pairs, dim3(grid_for(np * (S / 4))), dim3(kBlock), 0, st, seed, stream, p0, np, n_seg,
                       S, sigma, buf0);
    double2* x = fft(buf0, buf1, S, np, -1.0, tw, Gain{}, st);
    // the filter is applied as the inverse transform reads the spectrum
    Gain gain;
    if (fknee > 0.0) {
      gain.fknee = fknee;
      gain.alpha = alpha;
      gain.df = rate / (double)S;
    }
    double2* other = x == buf0 ? buf1 : buf0;
    x = fft(x, other, S, np, 1.0, tw, gain, st);
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
