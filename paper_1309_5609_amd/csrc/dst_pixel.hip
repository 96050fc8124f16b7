// Pixel-major form of the destriping operator for the iterative solve.
//
// The pointing of a problem is fixed for every CG iteration, so the solver
// builds once a transpose of it: samples sorted by pixel (stable, so in time
// order inside a pixel), with each sample's baseline index and angle.  The
// binning A^T W F p of every iteration then becomes a per-pixel gather of the
// (small, cache-resident) baseline vector followed by the per-pixel inverse,
// with no atomics and a fixed summation order.  The rescan and baseline sum
// F^T W A m stays in time order (one workgroup per baseline).
//
// Paper: arXiv:1309.5609, Algorithm section (Eqs. 9-13).
#include <hip/hip_runtime.h>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "dst_internal.h"
#include "dst_trig.h"
#include "dst_pixel.h"
#include "dst_cg.h"
#include "dst_comp.h"

namespace dst {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// cos(2 psi), sin(2 psi) in FP64 (pointing rows of Eqs. 3-6).
__device__ __forceinline__ void rot2(double psi, double& c, double& s) { fast_sincos(2.0 * psi, &s, &c); }

template <int N>
__device__ __forceinline__ void wave_sum(double (&v)[N]) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += __shfl_xor(v[i], off, 64);
  }
}

template <int N, typename T>
__device__ __forceinline__ void block_sum(T (&v)[N], T* lds) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += __shfl_xor(v[i], off, 64);
  }
  const int wid = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  if (lane_id() == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) lds[i * 16 + wid] = v[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      T acc = lds[i * 16];
      for (int w = 1; w < nw; ++w) acc += lds[i * 16 + w];
      v[i] = acc;
    }
  }
  __syncthreads();
}

// Workgroup i runs on XCD i mod 8 (round-robin dispatch); give each XCD a
// contiguous range of baselines so the map entries a range touches stay in
// that XCD's L2.  Returns -1 for the padding groups past n_b.
__device__ __forceinline__ int64_t xcd_baseline(int64_t n_b) {
  const int64_t per = (n_b + 7) / 8;
  const int64_t i = blockIdx.x;
  const int64_t b = (i & 7) * per + (i >> 3);
  return b < n_b ? b : -1;
}

// ---------------------------------------------------------------- transpose build

// Sort keys: pixel, or n_pix for masked samples; flags out-of-range pixels.
__global__ void __launch_bounds__(kBlock) k_sort_keys(const int32_t* __restrict__ pix, int64_t n_t, int64_t n_pix,
                                                      uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                      int* __restrict__ err) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_t; t += (int64_t)gridDim.x * blockDim.x) {
    const int p = pix[t];
    uint32_t k = (uint32_t)n_pix;
    if (p >= 0) {
      if (p < n_pix)
        k = (uint32_t)p;
      else
        atomicOr(err, 1);
    }
    keys[t] = k;
    vals[t] = (uint32_t)t;
  }
}

// seg[2k] = first sorted position of key k, seg[2k+1] = one past its last.
__global__ void __launch_bounds__(kBlock) k_segments(const uint32_t* __restrict__ keys, int64_t n_t,
                                                     int64_t* __restrict__ seg) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n_t; j += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t k = keys[j];
    if (j == 0 || keys[j - 1] != k) seg[2 * (int64_t)k] = j;
    if (j == n_t - 1 || keys[j + 1] != k) seg[2 * (int64_t)k + 1] = j + 1;
  }
}

// First sample of each pixel (the sort is stable, so it heads the segment);
// unobserved pixels get UINT32_MAX.  Counts observed pixels.
__global__ void __launch_bounds__(kBlock) k_first_visit(const int64_t* __restrict__ seg,
                                                        const uint32_t* __restrict__ perm, int64_t n_pix,
                                                        uint32_t* __restrict__ first, uint32_t* __restrict__ pidx,
                                                        unsigned long long* __restrict__ n_obs) {
  __shared__ unsigned long long lds[16];
  unsigned long long cnt[1] = {0};
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n_pix; p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j0 = seg[2 * p], j1 = seg[2 * p + 1];
    const bool hit = j1 > j0;
    first[p] = hit ? perm[j0] : 0xffffffffu;
    pidx[p] = (uint32_t)p;
    cnt[0] += hit;
  }
  block_sum<1>(cnt, lds);
  if (threadIdx.x == 0) atomicAdd(n_obs, cnt[0]);
}

// Compact ids: observed pixels numbered in order of first visit.
__global__ void __launch_bounds__(kBlock) k_compact_ids(const uint32_t* __restrict__ order, int64_t n_obs,
                                                        const int64_t* __restrict__ seg, int32_t* __restrict__ cid,
                                                        int64_t* __restrict__ chits) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c <= n_obs; c += (int64_t)gridDim.x * blockDim.x) {
    if (c == n_obs) {
      chits[c] = 0;
      continue;
    }
    const uint32_t p = order[c];
    cid[p] = (int32_t)c;
    chits[c] = seg[2 * (int64_t)p + 1] - seg[2 * (int64_t)p];
  }
}

// Compact pixel id of every sample (-1 for masked samples).
__global__ void __launch_bounds__(kBlock) k_cpix(const int32_t* __restrict__ pix, int64_t n_t, int64_t n_pix,
                                                 const int32_t* __restrict__ cid, int32_t* __restrict__ cpix) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_t; t += (int64_t)gridDim.x * blockDim.x) {
    const int p = pix[t];
    cpix[t] = (p >= 0 && p < n_pix) ? cid[p] : -1;
  }
}

// Full-sky outputs from compact arrays: hits, and a map m = a (- b).
__global__ void __launch_bounds__(kBlock) k_scatter(int64_t n_pix, const int32_t* __restrict__ cid,
                                                    const int32_t* __restrict__ chits32, int32_t* __restrict__ hits,
                                                    const double* __restrict__ a4, const double* __restrict__ b4,
                                                    double* __restrict__ out3, int b_dense) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n_pix; p += (int64_t)gridDim.x * blockDim.x) {
    const int c = cid[p];
    if (hits) hits[p] = c >= 0 ? chits32[c] : 0;
    if (out3) {
      double m0 = 0.0, m1 = 0.0, m2 = 0.0;
      if (c >= 0) {
        m0 = a4[4 * (int64_t)c + 0];
        m1 = a4[4 * (int64_t)c + 1];
        m2 = a4[4 * (int64_t)c + 2];
        if (b4 && b_dense) {
          m0 -= b4[c];
        } else if (b4) {
          m0 -= b4[4 * (int64_t)c + 0];
          m1 -= b4[4 * (int64_t)c + 1];
          m2 -= b4[4 * (int64_t)c + 2];
        }
      }
      out3[3 * p + 0] = m0;
      out3[3 * p + 1] = m1;
      out3[3 * p + 2] = m2;
    }
  }
}

// One wavefront per compact pixel c (first-visit order): lay out the pixel's
// samples -- sample index, baseline index, angle -- at [cstart[c], cstart[c+1])
// in time order; sum its weight block (hits, M_QQ, M_QU, M_UU; the T block is
// w_T h) and, with TOD, its sum map A^T W d; then invert the block with the
// validity cut (Eqs. 9-11 and the remark after them) and form the binned map.
// Fixed summation order per pixel; no atomics on pixel data.
template <typename PT, typename TT, bool HAS_T, bool HAS_QU, bool TOD>
__global__ void __launch_bounds__(kBlock) k_setup_pixels(View v, const uint32_t* __restrict__ order, int64_t n_obs,
                                                         const int64_t* __restrict__ seg,
                                                         const int64_t* __restrict__ cstart,
                                                         const uint32_t* __restrict__ perm,
                                                         const TT* __restrict__ tod, double rcond_cut,
                                                         uint32_t* __restrict__ cperm, int32_t* __restrict__ sb,
                                                         PT* __restrict__ spsi, int32_t* __restrict__ hits,
                                                         double* __restrict__ Minv4, uint8_t* __restrict__ valid,
                                                         double* __restrict__ m4_zero, double* __restrict__ sd4,
                                                         double* __restrict__ md4,
                                                         unsigned long long* __restrict__ counts) {
  __shared__ unsigned long long lds[4 * 16];
  unsigned long long cnt[4] = {0, 0, 0, 0};
  const int lane = lane_id();
  const int64_t nw = (int64_t)gridDim.x * kWaves;
  const PT* psi = static_cast<const PT*>(v.psi);
  const int64_t n_t = v.n_t;
  const uint32_t L = (uint32_t)v.L;
  for (int64_t c = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); c < n_obs; c += nw) {
    const int64_t src = seg[2 * (int64_t)order[c]];
    const int64_t dst = cstart[c];
    const int64_t h = cstart[c + 1] - dst;
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // cc, cs, ss, d_I, d_Q, d_U
    for (int64_t k = lane; k < h; k += 64) {
      const uint32_t t = perm[src + k];
      cperm[dst + k] = t;
      sb[dst + k] = (int32_t)(t / L);
      double cs = 1.0, sn = 0.0;
      if (HAS_QU) {
        const PT a = psi[t];
        spsi[dst + k] = a;
        rot2((double)a, cs, sn);
        acc[0] += cs * cs;
        acc[1] += cs * sn;
        acc[2] += sn * sn;
      }
      if (TOD) {
        if (HAS_T) acc[3] += (double)tod[v.rowT * n_t + t];
        if (HAS_QU) {
          const double xq = v.w[1] * (double)tod[v.rowQ * n_t + t];
          const double xu = v.w[2] * (double)tod[v.rowU * n_t + t];
          acc[4] += cs * xq - sn * xu;
          acc[5] += sn * xq + cs * xu;
        }
      }
    }
    wave_sum<6>(acc);
    if (lane == 0) {
      double inv[4] = {0.0, 0.0, 0.0, 0.0};
      uint8_t f = 0;
      const double mII = HAS_T ? v.w[0] * (double)h : 0.0;
      if (HAS_T && h > 0) {
        f |= 1;
        inv[0] = 1.0 / mII;
      }
      if (HAS_QU && h > 0) {
        const double wq = v.w[1], wu = v.w[2];
        const double a = wq * acc[0] + wu * acc[2];
        const double b = (wq - wu) * acc[1];
        const double d = wq * acc[2] + wu * acc[0];
        // eigenvalues of the symmetric 2x2 block [[a, b], [b, d]]
        const double half = 0.5 * (a - d);
        const double rad = sqrt(half * half + b * b);
        const double lmax = 0.5 * (a + d) + rad;
        const double det = a * d - b * b;
        const double lmin = lmax > 0.0 ? det / lmax : 0.0;
        if (lmax > 0.0 && lmin > 0.0 && lmin >= rcond_cut * lmax) {
          f |= 2;
          inv[1] = d / det;
          inv[2] = -b / det;
          inv[3] = a / det;
        }
      }
      hits[c] = (int32_t)h;
      double2* mi = reinterpret_cast<double2*>(Minv4 + 4 * c);
      mi[0] = make_double2(inv[0], inv[1]);
      mi[1] = make_double2(inv[2], inv[3]);
      valid[c] = f;
      double2* mz = reinterpret_cast<double2*>(m4_zero + 4 * c);
      mz[0] = make_double2(0.0, 0.0);
      mz[1] = make_double2(0.0, 0.0);
      if (TOD) {
        const double sI = (f & 1) ? v.w[0] * acc[3] : 0.0;
        const double sQ = (f & 2) ? acc[4] : 0.0;
        const double sU = (f & 2) ? acc[5] : 0.0;
        double2* sp = reinterpret_cast<double2*>(sd4 + 4 * c);
        sp[0] = make_double2(sI, sQ);
        sp[1] = make_double2(sU, 0.0);
        double2* mp = reinterpret_cast<double2*>(md4 + 4 * c);
        mp[0] = make_double2(inv[0] * sI, inv[1] * sQ + inv[2] * sU);
        mp[1] = make_double2(inv[2] * sQ + inv[3] * sU, 0.0);
      }
      cnt[0] += f & 1;
      cnt[1] += (f >> 1) & 1;
      cnt[2] += (f & 1) ? (unsigned long long)h : 0ull;
      cnt[3] += (f & 2) ? (unsigned long long)h : 0ull;
    }
  }
  block_sum<4>(cnt, lds);
  if (threadIdx.x == 0 && counts) {
#pragma unroll
    for (int i = 0; i < 4; ++i) atomicAdd(&counts[i], cnt[i]);
  }
}

// Time-major pass over each baseline (one workgroup, XCD-local order):
// valid-sample counts n_valid and the Jacobi diagonal 1/(w_k n_valid), and
// with TOD the right-hand side of Eq. 13,
//   b_k[beta] = w_k sum_{t in beta, valid_k} (d_k(t) - A_k(t) . m_d[p(t)]).
template <typename PT, typename TT, bool HAS_T, bool HAS_QU, bool TOD>
__global__ void __launch_bounds__(kBlock) k_rhs_unbin(View v, const TT* __restrict__ tod,
                                                      const double* __restrict__ md4,
                                                      const uint8_t* __restrict__ valid, int32_t* __restrict__ nvalid,
                                                      double* __restrict__ J, double* __restrict__ b_out) {
  __shared__ double lds[5 * 16];
  const PT* psi = static_cast<const PT*>(v.psi);
  const int64_t n_b = v.n_b, n_t = v.n_t;
  const int64_t b = xcd_baseline(n_b);
  if (b < 0) return;
  const int64_t t0 = b * v.L;
  const int64_t t1 = min(t0 + v.L, n_t);
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // d_T - m, d_q - A m, d_u - A m, n_T, n_QU
  constexpr int U = 8;
  for (int64_t tb = t0 + threadIdx.x; tb < t1; tb += U * kBlock) {
    int pp[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t t = tb + u * kBlock;
      pp[u] = t < t1 ? v.pix[t] : -1;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int pu = pp[u];
      if (pu < 0 || pu >= v.n_pix) continue;
      const int64_t t = tb + u * kBlock;
      const uint8_t f = valid[pu];
      const double2* mp = reinterpret_cast<const double2*>(md4 + 4 * (int64_t)pu);
      if (HAS_T && (f & 1)) {
        acc[3] += 1.0;
        if (TOD) acc[0] += (double)tod[v.rowT * n_t + t] - mp[0].x;
      }
      if (HAS_QU && (f & 2)) {
        acc[4] += 1.0;
        if (TOD) {
          const double mQ = mp[0].y, mU = mp[1].x;
          double c, s;
          rot2((double)psi[t], c, s);
          acc[1] += (double)tod[v.rowQ * n_t + t] - (c * mQ + s * mU);
          acc[2] += (double)tod[v.rowU * n_t + t] - (c * mU - s * mQ);
        }
      }
    }
  }
  block_sum<5>(acc, lds);
  if (threadIdx.x == 0) {
    const int nT = (int)acc[3], nQ = (int)acc[4];
    nvalid[b] = nT;
    nvalid[n_b + b] = nQ;
    if (HAS_T) {
      J[v.rowT * n_b + b] = nT ? 1.0 / (v.w[0] * nT) : 0.0;
      if (TOD) b_out[v.rowT * n_b + b] = v.w[0] * acc[0];
    }
    if (HAS_QU) {
      J[v.rowQ * n_b + b] = nQ ? 1.0 / (v.w[1] * nQ) : 0.0;
      J[v.rowU * n_b + b] = nQ ? 1.0 / (v.w[2] * nQ) : 0.0;
      if (TOD) {
        b_out[v.rowQ * n_b + b] = v.w[1] * acc[1];
        b_out[v.rowU * n_b + b] = v.w[2] * acc[2];
      }
    }
  }
}

// ---------------------------------------------------------------- iteration kernels

// m_p = M_p^-1 sum_{t in p} A(t)^T (w .* p)[beta(t)]  (the binning of F p and the
// per-pixel inverse, Eqs. 10-12), pixel-major.  pw4 = [n_b][4] (w_T p_T, w_q p_q, w_u p_u, 0).
template <typename PT, bool HAS_T, bool HAS_QU>
__global__ void __launch_bounds__(kBlock) k_bin_pixel(int64_t n_pix, const int64_t* __restrict__ cstart,
                                                      const int32_t* __restrict__ sb, const PT* __restrict__ spsi,
                                                      const double* __restrict__ pw4,
                                                      const double* __restrict__ Minv4,
                                                      const uint8_t* __restrict__ valid, double* __restrict__ m4,
                                                      const CgCtl* __restrict__ gate) {
  if (gate && gate->done) return;
  const int lane = lane_id();
  const int64_t nw = (int64_t)gridDim.x * kWaves;
  for (int64_t p = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); p < n_pix; p += nw) {
    if (valid[p] == 0) continue;  // m stays 0 on invalid pixels
    const int64_t j0 = cstart[p], j1 = cstart[p + 1];
    double acc[3] = {0.0, 0.0, 0.0};
    // U samples per lane per step: all streaming loads first, then the gathers
    constexpr int U = 4;
    for (int64_t jb = j0 + lane; jb < j1; jb += 64 * U) {
      int32_t bb[U];
      double aa[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t j = jb + 64 * u;
        const bool in = j < j1;
        bb[u] = in ? sb[j] : -1;
        aa[u] = (HAS_QU && in) ? (double)spsi[j] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (bb[u] < 0) continue;
        const double2* q0 = reinterpret_cast<const double2*>(pw4 + 4 * (int64_t)bb[u]);
        const double2 x0 = q0[0];
        if (HAS_T) acc[0] += x0.x;
        if (HAS_QU) {
          const double u0 = q0[1].x;
          double c0, s0;
          rot2(aa[u], c0, s0);
          acc[1] += c0 * x0.y - s0 * u0;
          acc[2] += s0 * x0.y + c0 * u0;
        }
      }
    }
    wave_sum<3>(acc);
    if (lane == 0) {
      const double2* ip = reinterpret_cast<const double2*>(Minv4 + 4 * p);
      const double2 i01 = ip[0], i23 = ip[1];
      double2* mp = reinterpret_cast<double2*>(m4 + 4 * p);
      mp[0] = make_double2(i01.x * acc[0], i01.y * acc[1] + i23.x * acc[2]);
      mp[1] = make_double2(i23.x * acc[1] + i23.y * acc[2], 0.0);
    }
  }
}

// q_k[b] = w_k (n_valid_k(b) p_k[b] - sum_{t in b} A_k(t) . m[p(t)])  (F^T Z F p,
// the baseline sums of Eq. 13), one workgroup per baseline in XCD-local order.
// m is zero on invalid blocks, so invalid samples add nothing to the sum.
// With ctl: per-baseline partials of p.q and of the T-projection sums
// (finished by k_cg_alpha).
template <typename PT, bool HAS_T, bool HAS_QU, bool CG>
__global__ void __launch_bounds__(kBlock) k_unbin_cg(View v, const double* __restrict__ m4,
                                                     const int32_t* __restrict__ nvalid,
                                                     const double* __restrict__ p, double* __restrict__ q,
                                                     CgCtl* __restrict__ ctl, double* __restrict__ partials) {
  if (CG && ctl->done) return;
  __shared__ double lds[4 * 16];
  const PT* psi = static_cast<const PT*>(v.psi);
  const int64_t n_b = v.n_b;
  const int64_t b = xcd_baseline(n_b);
  if (b >= 0) {
    const int64_t t0 = b * v.L;
    const int64_t t1 = min(t0 + v.L, v.n_t);
    double acc[3] = {0.0, 0.0, 0.0};
    constexpr int U = 8;
    for (int64_t tb = t0 + threadIdx.x; tb < t1; tb += U * kBlock) {
      int pp[U];
      double ang[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t t = tb + u * kBlock;
        pp[u] = t < t1 ? v.pix[t] : -1;
        if (HAS_QU) ang[u] = t < t1 ? (double)psi[t] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int pu = pp[u];
        if (pu < 0 || pu >= v.n_pix) continue;
        const double2* mp = reinterpret_cast<const double2*>(m4 + 4 * (int64_t)pu);
        const double2 m01 = mp[0];
        if (HAS_T) acc[0] += m01.x;
        if (HAS_QU) {
          const double mU = mp[1].x;
          double c, s;
          rot2(ang[u], c, s);
          acc[1] += c * m01.y + s * mU;
          acc[2] += c * mU - s * m01.y;
        }
      }
    }
    block_sum<3>(acc, lds);
    if (threadIdx.x == 0) {
      const int nT = nvalid[b], nQ = nvalid[n_b + b];
      double pq = 0.0, eq = 0.0, ep = 0.0;
      if (HAS_T) {
        const double pb = p[v.rowT * n_b + b];
        const double o = v.w[0] * (pb * (double)nT - acc[0]);
        q[v.rowT * n_b + b] = o;
        pq += pb * o;
        if (nT > 0) {
          eq = o;
          ep = pb;
        }
      }
      if (HAS_QU) {
        const double pbq = p[v.rowQ * n_b + b], pbu = p[v.rowU * n_b + b];
        const double oq = v.w[1] * (pbq * (double)nQ - acc[1]);
        const double ou = v.w[2] * (pbu * (double)nQ - acc[2]);
        q[v.rowQ * n_b + b] = oq;
        q[v.rowU * n_b + b] = ou;
        pq += pbq * oq + pbu * ou;
      }
      if (CG) {
        partials[b] = pq;
        partials[n_b + b] = eq;
        partials[2 * n_b + b] = ep;
      }
    }
  }
}

__global__ void __launch_bounds__(1024) k_cg_alpha(int64_t n_part, CgCtl* __restrict__ ctl,
                                                   const double* __restrict__ partials, CompView cv,
                                                   double* __restrict__ q, const double* __restrict__ p) {
  __shared__ double lds[3 * 16];
  __shared__ double clds[16 * 64];
  cg_alpha_body(n_part, ctl, partials, cv, q, p, lds, clds);
}

__global__ void __launch_bounds__(1024) k_cg_beta(int n_part, CgCtl* __restrict__ ctl,
                                                  const double* __restrict__ partials) {
  __shared__ double lds[2 * 16];
  cg_beta_body(n_part, ctl, partials, lds);
}

__global__ void __launch_bounds__(kBlock) k_p_update4(View v, double* __restrict__ p, const double* __restrict__ z,
                                                      double* __restrict__ pw4, const CgCtl* __restrict__ ctl,
                                                      int use_beta, int dense_t) {
  p_update4_body(v, p, z, pw4, ctl, use_beta, dense_t, blockIdx.x, gridDim.x);
}

unsigned grid_for(int64_t n, int64_t per_block, unsigned cap) {
  int64_t g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

}  // namespace

// ---------------------------------------------------------------- host side

// Key bits to sort: keys run over 0..n_pix (n_pix marks masked samples).
static unsigned sort_end_bit(int64_t n_pix) {
  unsigned end_bit = 1;
  while (end_bit < 32 && ((uint64_t)1 << end_bit) <= (uint64_t)n_pix) ++end_bit;
  return end_bit;
}

#define DST_CHECK(x)                  \
  do {                                \
    hipError_t e_ = (x);              \
    if (e_ != hipSuccess) return e_;  \
  } while (0)

hipError_t transpose_tmp_bytes(int64_t n_t, int64_t n_pix, size_t* bytes) {
  size_t a = 0, b = 0, c = 0;
  {
    rocprim::double_buffer<uint32_t> keys(nullptr, nullptr);
    rocprim::double_buffer<uint32_t> vals(nullptr, nullptr);
    DST_CHECK(rocprim::radix_sort_pairs(nullptr, a, keys, vals, (size_t)n_t, 0u, sort_end_bit(n_pix)));
    DST_CHECK(rocprim::radix_sort_pairs(nullptr, b, keys, vals, (size_t)n_pix, 0u, 32u));
  }
  DST_CHECK(rocprim::exclusive_scan(nullptr, c, static_cast<const int64_t*>(nullptr), static_cast<int64_t*>(nullptr),
                                    (int64_t)0, (size_t)n_pix + 1, rocprim::plus<int64_t>()));
  *bytes = std::max(a, std::max(b, c));
  return hipSuccess;
}

hipError_t transpose_build(const View& v, Transpose& T, int* err, hipStream_t st) {
  const int64_t n_t = v.n_t, n_pix = v.n_pix;
  const unsigned g = grid_for(n_t, kBlock, 8192);
  const unsigned gp = grid_for(n_pix, kBlock, 4096);
  // 1. stable sort of sample indices by pixel
  hipLaunchKernelGGL(k_sort_keys, dim3(g), dim3(kBlock), 0, st, v.pix, n_t, n_pix, T.keys[0], T.vals[0], err);
  DST_CHECK(hipGetLastError());
  {
    rocprim::double_buffer<uint32_t> keys(T.keys[0], T.keys[1]);
    rocprim::double_buffer<uint32_t> vals(T.vals[0], T.vals[1]);
    size_t tmp = T.tmp_bytes;
    DST_CHECK(rocprim::radix_sort_pairs(T.tmp, tmp, keys, vals, (size_t)n_t, 0u, sort_end_bit(n_pix), st));
    T.perm = vals.current();
    // 2. segment of every pixel in the sorted order
    hipLaunchKernelGGL(k_segments, dim3(g), dim3(kBlock), 0, st, keys.current(), n_t, T.seg);
    DST_CHECK(hipGetLastError());
  }
  // 3. order observed pixels by first visit
  hipLaunchKernelGGL(k_first_visit, dim3(gp), dim3(kBlock), 0, st, T.seg, T.perm, n_pix, T.pk[0], T.pv[0],
                     T.n_obs_dev);
  DST_CHECK(hipGetLastError());
  {
    rocprim::double_buffer<uint32_t> keys(T.pk[0], T.pk[1]);
    rocprim::double_buffer<uint32_t> vals(T.pv[0], T.pv[1]);
    size_t tmp = T.tmp_bytes;
    DST_CHECK(rocprim::radix_sort_pairs(T.tmp, tmp, keys, vals, (size_t)n_pix, 0u, 32u, st));
    T.order = vals.current();
  }
  unsigned long long nobs = 0;
  DST_CHECK(hipMemcpyAsync(&nobs, T.n_obs_dev, sizeof nobs, hipMemcpyDeviceToHost, st));
  DST_CHECK(hipStreamSynchronize(st));
  T.n_obs = (int64_t)nobs;
  // 4. compact ids and per-pixel offsets of the transposed arrays
  hipLaunchKernelGGL(k_compact_ids, dim3(grid_for(T.n_obs + 1, kBlock, 4096)), dim3(kBlock), 0, st, T.order,
                     T.n_obs, T.seg, T.cid, T.chits);
  DST_CHECK(hipGetLastError());
  {
    size_t tmp = T.tmp_bytes;
    DST_CHECK(rocprim::exclusive_scan(T.tmp, tmp, T.chits, T.cstart, (int64_t)0, (size_t)T.n_obs + 1,
                                      rocprim::plus<int64_t>(), st));
  }
  hipLaunchKernelGGL(k_cpix, dim3(g), dim3(kBlock), 0, st, v.pix, n_t, n_pix, T.cid, T.cpix);
  return hipGetLastError();
}

template <typename PT, typename TT, bool HAS_T, bool HAS_QU>
static void setup_pixels_dispatch(const View& v, const Transpose& T, const void* tod, double rcond_cut,
                                  int32_t* hits, double* Minv4, uint8_t* valid, double* m4_zero, double* sd4,
                                  double* md4, unsigned long long* counts, hipStream_t st) {
  const unsigned g = grid_for(T.n_obs, kWaves, 4096);
  const TT* x = static_cast<const TT*>(tod);
  PT* sp = static_cast<PT*>(T.spsi);
  if (tod)
    hipLaunchKernelGGL((k_setup_pixels<PT, TT, HAS_T, HAS_QU, true>), dim3(g), dim3(kBlock), 0, st, v, T.order,
                       T.n_obs, T.seg, T.cstart, T.perm, x, rcond_cut, T.cperm, T.sb, sp, hits, Minv4, valid, m4_zero,
                       sd4, md4, counts);
  else
    hipLaunchKernelGGL((k_setup_pixels<PT, TT, HAS_T, HAS_QU, false>), dim3(g), dim3(kBlock), 0, st, v, T.order,
                       T.n_obs, T.seg, T.cstart, T.perm, x, rcond_cut, T.cperm, T.sb, sp, hits, Minv4, valid, m4_zero,
                       sd4, md4, counts);
}

template <typename PT, typename TT>
static void setup_pixels_streams(const View& v, const Transpose& T, const void* tod, double rcond_cut, int32_t* hits,
                                 double* Minv4, uint8_t* valid, double* m4_zero, double* sd4, double* md4,
                                 unsigned long long* counts, hipStream_t st) {
  if (v.rowT >= 0 && v.rowQ >= 0)
    setup_pixels_dispatch<PT, TT, true, true>(v, T, tod, rcond_cut, hits, Minv4, valid, m4_zero, sd4, md4, counts, st);
  else if (v.rowQ >= 0)
    setup_pixels_dispatch<PT, TT, false, true>(v, T, tod, rcond_cut, hits, Minv4, valid, m4_zero, sd4, md4, counts,
                                               st);
  else
    setup_pixels_dispatch<PT, TT, true, false>(v, T, tod, rcond_cut, hits, Minv4, valid, m4_zero, sd4, md4, counts,
                                               st);
}

hipError_t launch_setup_pixels(const View& v, int psi_f32, const Transpose& T, const void* tod, int tod_f32,
                               double rcond_cut, int32_t* hits, double* Minv4, uint8_t* valid, double* m4_zero,
                               double* sd4, double* md4, unsigned long long* counts, hipStream_t st) {
  if (T.n_obs == 0) return hipSuccess;
  const bool pf = psi_f32 && v.rowQ >= 0;
  if (pf && tod_f32)
    setup_pixels_streams<float, float>(v, T, tod, rcond_cut, hits, Minv4, valid, m4_zero, sd4, md4, counts, st);
  else if (pf)
    setup_pixels_streams<float, double>(v, T, tod, rcond_cut, hits, Minv4, valid, m4_zero, sd4, md4, counts, st);
  else if (tod_f32)
    setup_pixels_streams<double, float>(v, T, tod, rcond_cut, hits, Minv4, valid, m4_zero, sd4, md4, counts, st);
  else
    setup_pixels_streams<double, double>(v, T, tod, rcond_cut, hits, Minv4, valid, m4_zero, sd4, md4, counts, st);
  return hipGetLastError();
}

template <typename PT, typename TT, bool HAS_T, bool HAS_QU>
static void rhs_dispatch(const View& vc, const void* tod, const double* md4, const uint8_t* valid, int32_t* nvalid,
                         double* J, double* b, hipStream_t st) {
  const unsigned g = (unsigned)(8 * ((vc.n_b + 7) / 8));
  const TT* x = static_cast<const TT*>(tod);
  if (tod)
    hipLaunchKernelGGL((k_rhs_unbin<PT, TT, HAS_T, HAS_QU, true>), dim3(g), dim3(kBlock), 0, st, vc, x, md4, valid,
                       nvalid, J, b);
  else
    hipLaunchKernelGGL((k_rhs_unbin<PT, TT, HAS_T, HAS_QU, false>), dim3(g), dim3(kBlock), 0, st, vc, x, md4, valid,
                       nvalid, J, b);
}

template <typename PT, typename TT>
static void rhs_streams(const View& vc, const void* tod, const double* md4, const uint8_t* valid, int32_t* nvalid,
                        double* J, double* b, hipStream_t st) {
  if (vc.rowT >= 0 && vc.rowQ >= 0)
    rhs_dispatch<PT, TT, true, true>(vc, tod, md4, valid, nvalid, J, b, st);
  else if (vc.rowQ >= 0)
    rhs_dispatch<PT, TT, false, true>(vc, tod, md4, valid, nvalid, J, b, st);
  else
    rhs_dispatch<PT, TT, true, false>(vc, tod, md4, valid, nvalid, J, b, st);
}

hipError_t launch_rhs_unbin(const View& vc, int psi_f32, const void* tod, int tod_f32, const double* md4,
                            const uint8_t* valid, int32_t* nvalid, double* J, double* b, hipStream_t st) {
  const bool pf = psi_f32 && vc.rowQ >= 0;
  if (pf && tod_f32)
    rhs_streams<float, float>(vc, tod, md4, valid, nvalid, J, b, st);
  else if (pf)
    rhs_streams<float, double>(vc, tod, md4, valid, nvalid, J, b, st);
  else if (tod_f32)
    rhs_streams<double, float>(vc, tod, md4, valid, nvalid, J, b, st);
  else
    rhs_streams<double, double>(vc, tod, md4, valid, nvalid, J, b, st);
  return hipGetLastError();
}

hipError_t launch_scatter(int64_t n_pix, const int32_t* cid, const int32_t* chits, int32_t* hits, const double* a4,
                          const double* b4, double* out3, hipStream_t st, int b_dense) {
  hipLaunchKernelGGL(k_scatter, dim3(grid_for(n_pix, kBlock, 4096)), dim3(kBlock), 0, st, n_pix, cid, chits, hits,
                     a4, b4, out3, b_dense);
  return hipGetLastError();
}

template <typename PT>
static void bin_pixel_dispatch(const View& v, const Transpose& T, const double* pw4, const double* Minv4,
                               const uint8_t* valid, double* m4, const CgCtl* gate, hipStream_t st) {
  const unsigned g = grid_for(v.n_pix, kWaves, 65536);
  const PT* sp = static_cast<const PT*>(T.spsi);
  if (v.rowT >= 0 && v.rowQ >= 0)
    hipLaunchKernelGGL((k_bin_pixel<PT, true, true>), dim3(g), dim3(kBlock), 0, st, v.n_pix, T.cstart, T.sb, sp, pw4,
                       Minv4, valid, m4, gate);
  else if (v.rowQ >= 0)
    hipLaunchKernelGGL((k_bin_pixel<PT, false, true>), dim3(g), dim3(kBlock), 0, st, v.n_pix, T.cstart, T.sb, sp, pw4,
                       Minv4, valid, m4, gate);
  else
    hipLaunchKernelGGL((k_bin_pixel<PT, true, false>), dim3(g), dim3(kBlock), 0, st, v.n_pix, T.cstart, T.sb, sp, pw4,
                       Minv4, valid, m4, gate);
}

hipError_t launch_bin_pixel(const View& v, int psi_f32, const Transpose& T, const double* pw4, const double* Minv4,
                            const uint8_t* valid, double* m4, const CgCtl* gate, hipStream_t st) {
  if (psi_f32 && v.rowQ >= 0)
    bin_pixel_dispatch<float>(v, T, pw4, Minv4, valid, m4, gate, st);
  else
    bin_pixel_dispatch<double>(v, T, pw4, Minv4, valid, m4, gate, st);
  return hipGetLastError();
}

template <typename PT, bool CG>
static void unbin_cg_dispatch(const View& v, const double* m4, const int32_t* nvalid, const double* p, double* q,
                              CgCtl* ctl, double* partials, hipStream_t st) {
  const unsigned g = (unsigned)(8 * ((v.n_b + 7) / 8));
  if (v.rowT >= 0 && v.rowQ >= 0)
    hipLaunchKernelGGL((k_unbin_cg<PT, true, true, CG>), dim3(g), dim3(kBlock), 0, st, v, m4, nvalid, p, q, ctl,
                       partials);
  else if (v.rowQ >= 0)
    hipLaunchKernelGGL((k_unbin_cg<PT, false, true, CG>), dim3(g), dim3(kBlock), 0, st, v, m4, nvalid, p, q, ctl,
                       partials);
  else
    hipLaunchKernelGGL((k_unbin_cg<PT, true, false, CG>), dim3(g), dim3(kBlock), 0, st, v, m4, nvalid, p, q, ctl,
                       partials);
}

hipError_t launch_unbin_cg(const View& v, int psi_f32, const double* m4, const int32_t* nvalid, const double* p,
                           double* q, CgCtl* ctl, double* partials, hipStream_t st) {
  const bool pf = psi_f32 && v.rowQ >= 0;
  if (ctl) {
    if (pf)
      unbin_cg_dispatch<float, true>(v, m4, nvalid, p, q, ctl, partials, st);
    else
      unbin_cg_dispatch<double, true>(v, m4, nvalid, p, q, ctl, partials, st);
  } else {
    if (pf)
      unbin_cg_dispatch<float, false>(v, m4, nvalid, p, q, ctl, partials, st);
    else
      unbin_cg_dispatch<double, false>(v, m4, nvalid, p, q, ctl, partials, st);
  }
  return hipGetLastError();
}

hipError_t launch_cg_alpha(int64_t n_part, CgCtl* ctl, const double* partials, const CompView& cv, double* q,
                           const double* p, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(1024), 0, st, n_part, ctl, partials, cv, q, p);
  return hipGetLastError();
}

hipError_t launch_cg_beta(int n_part, CgCtl* ctl, const double* partials, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(1024), 0, st, n_part, ctl, partials);
  return hipGetLastError();
}

hipError_t launch_p_update4(const View& v, double* p, const double* z, double* pw4, const CgCtl* ctl, int use_beta,
                            int dense_t, hipStream_t st) {
  const unsigned g = grid_for(v.n_b, kBlock, 1024);
  hipLaunchKernelGGL(k_p_update4, dim3(g), dim3(kBlock), 0, st, v, p, z, pw4, ctl, use_beta, dense_t);
  return hipGetLastError();
}


}  // namespace dst
