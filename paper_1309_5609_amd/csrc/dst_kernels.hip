// HIP kernels of the destriping hot path for gfx950 (CDNA4, wave64).
//
// Paper: Zonca et al., "Destriping Cosmic Microwave Background Polarimeter
// data" (arXiv:1309.5609), Algorithm section.  Operators:
//   bin    s = A^T W x        (sum maps of Eqs. 10-11, weighted reading of Eq. 12)
//   apply  m = M^-1 s         (per-pixel weight-matrix inverse, remark after Eqs. 10-11)
//   unbin  y = A m            (rescan, the R P~ of Eq. 13)
//   reduce F^T W (x - A m)    (baseline sums of Eq. 13)
// plus the preconditioned-CG recurrences of the destriping equation.
//
// Layout: timelines [n_streams][n_t]; per-pixel arrays [n_pix][4] doubles;
// baseline vectors [n_streams][n_b].  Samples are streamed in time order with
// each wavefront owning 64 consecutive samples, so pixel indices along the
// scan arrive in runs; bin() sums each run across the wavefront before one
// atomic per run.  Baseline reductions give one workgroup per baseline, so the
// per-baseline sums need no atomics.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "dst_cg.h"
#include "dst_internal.h"
#include "dst_trig.h"

namespace dst {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// cos(2 psi), sin(2 psi) in FP64 (pointing rows of Eqs. 3-6).
__device__ __forceinline__ void rot2(double psi, double& c, double& s) { fast_sincos(2.0 * psi, &s, &c); }

// Sum of N doubles over each run of equal consecutive keys of the wavefront.
// The first lane of a run gets the run total and its length; returns whether
// the calling lane heads a run.  All 64 lanes must call it together.
template <int N>
__device__ __forceinline__ bool wave_run_sum(int key, double (&v)[N], int& run_len) {
  const int lane = lane_id();
  const int prev = __shfl_up(key, 1, 64);
  const bool head = (lane == 0) || (prev != key);
  const unsigned long long heads = __ballot(head);
  const unsigned long long upto = (lane == 63) ? ~0ull : ((1ull << (lane + 1)) - 1ull);
  const int rid = __popcll(heads & upto);
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int orid = __shfl_down(rid, off, 64);
    const bool take = (lane + off < 64) && (orid == rid);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const double o = __shfl_down(v[i], off, 64);
      if (take) v[i] += o;
    }
  }
  const unsigned long long above = heads & ~upto;
  const int next = above ? (__ffsll((unsigned long long)above) - 1) : 64;
  run_len = next - lane;
  return head;
}

// Block-wide sum of N values (fixed order).  Result valid in thread 0.
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

// Arrival counter for "last block finishes the reduction".  Every thread of
// the last block returns true after an acquire fence.
__device__ __forceinline__ bool arrive_last(uint32_t* counter, bool* flag) {
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t prev = atomicAdd(counter, 1u);
    *flag = (prev == gridDim.x - 1);
  }
  __syncthreads();
  const bool last = *flag;
  if (last) __threadfence();
  return last;
}

// Fixed-order sum of `n` partials per column for the last block.
template <int N>
__device__ __forceinline__ void sum_partials(const double* part, int64_t n, double (&out)[N], double* lds) {
#pragma unroll
  for (int i = 0; i < N; ++i) out[i] = 0.0;
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
#pragma unroll
    for (int i = 0; i < N; ++i) out[i] += part[i * n + j];
  }
  block_sum<N>(out, lds);
}

__device__ __forceinline__ int64_t baseline_of(int64_t t0, int64_t b0, int64_t L, int lane) {
  // t0 = first sample of the chunk (multiple of 64), b0 = t0 / L
  const int64_t rem = t0 - b0 * L + lane;  // < L + 64
  if (L >= 64) return b0 + (rem >= L ? 1 : 0);
  return b0 + (int64_t)((uint32_t)rem / (uint32_t)L);
}

// ---------------------------------------------------------------- setup

template <typename PT>
__global__ void __launch_bounds__(kBlock) k_pointing(View v, int32_t* __restrict__ hits, double* __restrict__ M4,
                                                     int* __restrict__ err) {
  const int lane = lane_id();
  const int64_t wave = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
  const int64_t nw = (int64_t)gridDim.x * kWaves;
  const PT* psi = static_cast<const PT*>(v.psi);
  const bool qu = v.rowQ >= 0;
  const double wq = v.w[1], wu = v.w[2];
  for (int64_t t0 = wave * 64; t0 < v.n_t; t0 += nw * 64) {
    const int64_t t = t0 + lane;
    int key = -1;
    double m[3] = {0.0, 0.0, 0.0};
    if (t < v.n_t) {
      int p = v.pix[t];
      if (p >= v.n_pix) {
        atomicOr(err, 1);
        p = -1;
      }
      if (p >= 0) {
        key = p;
        if (qu) {
          double c, s;
          rot2((double)psi[t], c, s);
          m[0] = wq * c * c + wu * s * s;
          m[1] = (wq - wu) * c * s;
          m[2] = wq * s * s + wu * c * c;
        }
      }
    }
    int len;
    const bool head = wave_run_sum<3>(key, m, len);
    if (head && key >= 0) {
      atomicAdd(&hits[key], len);
      if (qu) {
        unsafeAtomicAdd(&M4[4 * (int64_t)key + 1], m[0]);
        unsafeAtomicAdd(&M4[4 * (int64_t)key + 2], m[1]);
        unsafeAtomicAdd(&M4[4 * (int64_t)key + 3], m[2]);
      }
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_invert(View v, const int32_t* __restrict__ hits,
                                                   const double* __restrict__ M4, double rcond_cut,
                                                   double* __restrict__ Minv4, uint8_t* __restrict__ valid,
                                                   double* __restrict__ blocks_out,
                                                   unsigned long long* __restrict__ counts) {
  __shared__ unsigned long long lds[2 * 16];
  unsigned long long cnt[2] = {0, 0};
  const bool has_t = v.rowT >= 0, has_qu = v.rowQ >= 0;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < v.n_pix;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int h = hits[p];
    double inv[4] = {0.0, 0.0, 0.0, 0.0};
    uint8_t f = 0;
    const double mII = has_t ? v.w[0] * (double)h : 0.0;
    double a = 0.0, b = 0.0, d = 0.0;
    if (has_t && h > 0) {
      f |= 1;
      inv[0] = 1.0 / mII;
    }
    if (has_qu) {
      a = M4[4 * p + 1];
      b = M4[4 * p + 2];
      d = M4[4 * p + 3];
      if (h > 0) {
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
    }
    double2* mi = reinterpret_cast<double2*>(Minv4 + 4 * p);
    mi[0] = make_double2(inv[0], inv[1]);
    mi[1] = make_double2(inv[2], inv[3]);
    valid[p] = f;
    if (blocks_out) {
      blocks_out[4 * p + 0] = mII;
      blocks_out[4 * p + 1] = a;
      blocks_out[4 * p + 2] = b;
      blocks_out[4 * p + 3] = d;
    }
    cnt[0] += f & 1;
    cnt[1] += (f >> 1) & 1;
  }
  block_sum<2>(cnt, lds);
  if (threadIdx.x == 0 && counts) {
    atomicAdd(&counts[0], cnt[0]);
    atomicAdd(&counts[1], cnt[1]);
  }
}

// Valid samples per baseline and stream class, and the Jacobi diagonal
// 1/(w_k n_valid) of F^T W F (0 for baselines without valid samples).
__global__ void __launch_bounds__(kBlock) k_baseline_counts(View v, const uint8_t* __restrict__ valid,
                                                            int32_t* __restrict__ nvalid, double* __restrict__ J,
                                                            unsigned long long* __restrict__ counts) {
  __shared__ int lds[2 * 16];
  const int64_t b = blockIdx.x;
  const int64_t t0 = b * v.L;
  const int64_t t1 = min(t0 + v.L, v.n_t);
  int c[2] = {0, 0};
  for (int64_t t = t0 + threadIdx.x; t < t1; t += blockDim.x) {
    const int p = v.pix[t];
    if (p >= 0 && p < v.n_pix) {
      const uint8_t f = valid[p];
      c[0] += f & 1;
      c[1] += (f >> 1) & 1;
    }
  }
  block_sum<2>(c, lds);
  if (threadIdx.x == 0) {
    nvalid[b] = c[0];
    nvalid[v.n_b + b] = c[1];
    if (v.rowT >= 0) J[v.rowT * v.n_b + b] = c[0] ? 1.0 / (v.w[0] * c[0]) : 0.0;
    if (v.rowQ >= 0) {
      J[v.rowQ * v.n_b + b] = c[1] ? 1.0 / (v.w[1] * c[1]) : 0.0;
      J[v.rowU * v.n_b + b] = c[1] ? 1.0 / (v.w[2] * c[1]) : 0.0;
    }
    if (counts) {
      atomicAdd(&counts[0], (unsigned long long)c[0]);
      atomicAdd(&counts[1], (unsigned long long)c[1]);
    }
  }
}

// ---------------------------------------------------------------- operators

// s[p] += sum over valid samples of sum_k w_k A_k(t)^T x_k(t),
// x = tod (USE_TOD) + bsign * F base (USE_BASE).
template <typename PT, typename TT, bool USE_TOD, bool USE_BASE>
__global__ void __launch_bounds__(kBlock) k_bin(View v, const TT* __restrict__ tod, const double* __restrict__ base,
                                                double bsign, const uint8_t* __restrict__ valid,
                                                double* __restrict__ s4, int* __restrict__ err,
                                                const CgCtl* __restrict__ gate) {
  if (gate && gate->done) return;
  const int lane = lane_id();
  const int64_t wave = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
  const int64_t nw = (int64_t)gridDim.x * kWaves;
  const PT* psi = static_cast<const PT*>(v.psi);
  const int64_t n_t = v.n_t, n_b = v.n_b;
  for (int64_t t0 = wave * 64; t0 < n_t; t0 += nw * 64) {
    const int64_t t = t0 + lane;
    int key = -1;
    double c3[3] = {0.0, 0.0, 0.0};
    if (t < n_t) {
      int p = v.pix[t];
      if (p >= v.n_pix) {
        if (err) atomicOr(err, 1);
        p = -1;
      }
      if (p >= 0) {
        key = p;
        const uint8_t f = valid[p];
        const int64_t b = USE_BASE ? baseline_of(t0, t0 / v.L, v.L, lane) : 0;
        if (f & 1) {
          double x = 0.0;
          if (USE_TOD) x = (double)tod[v.rowT * n_t + t];
          if (USE_BASE) x += bsign * base[v.rowT * n_b + b];
          c3[0] = v.w[0] * x;
        }
        if (f & 2) {
          double xq = 0.0, xu = 0.0;
          if (USE_TOD) {
            xq = (double)tod[v.rowQ * n_t + t];
            xu = (double)tod[v.rowU * n_t + t];
          }
          if (USE_BASE) {
            xq += bsign * base[v.rowQ * n_b + b];
            xu += bsign * base[v.rowU * n_b + b];
          }
          double c, s;
          rot2((double)psi[t], c, s);
          const double wq = v.w[1] * xq, wu = v.w[2] * xu;
          c3[1] = c * wq - s * wu;
          c3[2] = s * wq + c * wu;
        }
      }
    }
    int len;
    const bool head = wave_run_sum<3>(key, c3, len);
    if (head && key >= 0) {
      double* sp = s4 + 4 * (int64_t)key;
      if (c3[0] != 0.0) unsafeAtomicAdd(sp + 0, c3[0]);
      if (c3[1] != 0.0) unsafeAtomicAdd(sp + 1, c3[1]);
      if (c3[2] != 0.0) unsafeAtomicAdd(sp + 2, c3[2]);
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_apply(int64_t n_pix, const double* __restrict__ s4,
                                                  const double* __restrict__ Minv4, double* __restrict__ m,
                                                  int m_stride, double* __restrict__ s_clear,
                                                  const CgCtl* __restrict__ gate) {
  if (gate && gate->done) return;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n_pix;
       p += (int64_t)gridDim.x * blockDim.x) {
    const double2* sp = reinterpret_cast<const double2*>(s4 + 4 * p);
    const double2* ip = reinterpret_cast<const double2*>(Minv4 + 4 * p);
    const double2 s01 = sp[0], s23 = sp[1];
    const double2 i01 = ip[0], i23 = ip[1];
    const double mI = i01.x * s01.x;
    const double mQ = i01.y * s01.y + i23.x * s23.x;
    const double mU = i23.x * s01.y + i23.y * s23.x;
    if (m_stride == 4) {
      double2* mp = reinterpret_cast<double2*>(m + 4 * p);
      mp[0] = make_double2(mI, mQ);
      mp[1] = make_double2(mU, 0.0);
    } else {
      m[3 * p + 0] = mI;
      m[3 * p + 1] = mQ;
      m[3 * p + 2] = mU;
    }
    if (s_clear) {
      double2* sc = reinterpret_cast<double2*>(s_clear + 4 * p);
      sc[0] = make_double2(0.0, 0.0);
      sc[1] = make_double2(0.0, 0.0);
    }
  }
}

// One workgroup per baseline:
//   out_k[b] = w_k * sum_{t in b, valid_k} (x_k(t) - A_k(t) . m[p(t)])
// With CG, base is the search direction p (bsign = +1) and the last block
// computes mu (projection of the T part) and alpha = r.z / p.(P K p).
template <typename PT, typename TT, bool USE_TOD, bool USE_BASE, bool CG>
__global__ void __launch_bounds__(kBlock) k_unbin_reduce(View v, const TT* __restrict__ tod,
                                                         const double* __restrict__ base, double bsign,
                                                         const double* __restrict__ m4,
                                                         const uint8_t* __restrict__ valid,
                                                         const int32_t* __restrict__ nvalid,
                                                         double* __restrict__ out, CgCtl* __restrict__ ctl,
                                                         double* __restrict__ partials) {
  if (CG && ctl->done) return;
  __shared__ double lds[4 * 16];
  __shared__ bool last;
  const PT* psi = static_cast<const PT*>(v.psi);
  const int64_t b = blockIdx.x;
  const int64_t t0 = b * v.L;
  const int64_t t1 = min(t0 + v.L, v.n_t);
  const int64_t n_t = v.n_t, n_b = v.n_b;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t t = t0 + threadIdx.x; t < t1; t += blockDim.x) {
    const int p = v.pix[t];
    if (p < 0 || p >= v.n_pix) continue;
    const uint8_t f = valid[p];
    if (f == 0) continue;
    const double2* mp = reinterpret_cast<const double2*>(m4 + 4 * (int64_t)p);
    const double2 m01 = mp[0];
    if (f & 1) {
      double x = 0.0;
      if (USE_TOD) x = (double)tod[v.rowT * n_t + t];
      acc[0] += x - m01.x;
    }
    if (f & 2) {
      const double mU = mp[1].x;
      double c, s;
      rot2((double)psi[t], c, s);
      double xq = 0.0, xu = 0.0;
      if (USE_TOD) {
        xq = (double)tod[v.rowQ * n_t + t];
        xu = (double)tod[v.rowU * n_t + t];
      }
      acc[1] += xq - (c * m01.y + s * mU);
      acc[2] += xu - (c * mU - s * m01.y);
    }
  }
  block_sum<3>(acc, lds);
  if (threadIdx.x == 0) {
    const int nT = nvalid[b], nQ = nvalid[n_b + b];
    double pq = 0.0, eq = 0.0, ep = 0.0;
    if (v.rowT >= 0) {
      double a = acc[0];
      double pb = 0.0;
      if (USE_BASE) {
        pb = base[v.rowT * n_b + b];
        a += bsign * pb * (double)nT;
      }
      const double o = v.w[0] * a;
      out[v.rowT * n_b + b] = o;
      pq += pb * o;
      if (nT > 0) {
        eq = o;
        ep = pb;
      }
    }
    if (v.rowQ >= 0) {
      double aq = acc[1], au = acc[2];
      double pbq = 0.0, pbu = 0.0;
      if (USE_BASE) {
        pbq = base[v.rowQ * n_b + b];
        pbu = base[v.rowU * n_b + b];
        aq += bsign * pbq * (double)nQ;
        au += bsign * pbu * (double)nQ;
      }
      const double oq = v.w[1] * aq, ou = v.w[2] * au;
      out[v.rowQ * n_b + b] = oq;
      out[v.rowU * n_b + b] = ou;
      pq += pbq * oq + pbu * ou;
    }
    if (CG) {
      partials[b] = pq;
      partials[n_b + b] = eq;
      partials[2 * n_b + b] = ep;
    }
  }
  if (!CG) return;
  if (!arrive_last(&ctl->counter[0], &last)) return;
  double tot[3];
  sum_partials<3>(partials, n_b, tot, lds);
  if (threadIdx.x == 0) {
    const double mu = ctl->n_e > 0.0 ? tot[1] / ctl->n_e : 0.0;
    const double pkp = tot[0] - mu * tot[2];
    ctl->mu = mu;
    if (!isfinite(pkp)) {
      ctl->done = DONE_NAN;
    } else if (pkp <= 0.0) {
      ctl->done = DONE_BREAKDOWN;
    } else {
      ctl->alpha = ctl->rz / pkp;
    }
    ctl->counter[0] = 0;
  }
}

template <typename PT>
__global__ void __launch_bounds__(kBlock) k_scan(View v, const double* __restrict__ map3, double* __restrict__ out,
                                                 int* __restrict__ err) {
  const PT* psi = static_cast<const PT*>(v.psi);
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < v.n_t;
       t += (int64_t)gridDim.x * blockDim.x) {
    int p = v.pix[t];
    if (p >= v.n_pix) {
      atomicOr(err, 1);
      p = -1;
    }
    double yT = 0.0, yq = 0.0, yu = 0.0;
    if (p >= 0) {
      const double* mp = map3 + 3 * (int64_t)p;
      yT = mp[0];
      if (v.rowQ >= 0) {
        double c, s;
        rot2((double)psi[t], c, s);
        yq = c * mp[1] + s * mp[2];
        yu = -s * mp[1] + c * mp[2];
      }
    }
    if (v.rowT >= 0) out[v.rowT * v.n_t + t] = yT;
    if (v.rowQ >= 0) {
      out[v.rowQ * v.n_t + t] = yq;
      out[v.rowU * v.n_t + t] = yu;
    }
  }
}

template <typename TT>
__global__ void __launch_bounds__(kBlock) k_reduce(View v, const TT* __restrict__ x, const uint8_t* __restrict__ valid,
                                                   double* __restrict__ out) {
  __shared__ double lds[3 * 16];
  const int64_t b = blockIdx.x;
  const int64_t t0 = b * v.L;
  const int64_t t1 = min(t0 + v.L, v.n_t);
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t t = t0 + threadIdx.x; t < t1; t += blockDim.x) {
    const int p = v.pix[t];
    if (p < 0 || p >= v.n_pix) continue;
    const uint8_t f = valid[p];
    if (f & 1) acc[0] += (double)x[v.rowT * v.n_t + t];
    if (f & 2) {
      acc[1] += (double)x[v.rowQ * v.n_t + t];
      acc[2] += (double)x[v.rowU * v.n_t + t];
    }
  }
  block_sum<3>(acc, lds);
  if (threadIdx.x == 0) {
    if (v.rowT >= 0) out[v.rowT * v.n_b + b] = v.w[0] * acc[0];
    if (v.rowQ >= 0) {
      out[v.rowQ * v.n_b + b] = v.w[1] * acc[1];
      out[v.rowU * v.n_b + b] = v.w[2] * acc[2];
    }
  }
}

// ---------------------------------------------------------------- CG vectors

__device__ __forceinline__ bool t_valid_row(const View& v, int64_t i, const double* J) {
  return v.rowT >= 0 && i < v.n_b && J[i] > 0.0;  // the T row is row 0 when present
}

// Means over T-valid baselines of b_T and (K a0)_T, and their count.
__global__ void __launch_bounds__(kBlock) k_cg_means(View v, const double* __restrict__ b,
                                                     const double* __restrict__ ka, const double* __restrict__ J,
                                                     CgCtl* __restrict__ ctl, double* __restrict__ partials) {
  __shared__ double lds[3 * 16];
  __shared__ bool last;
  double acc[3] = {0.0, 0.0, 0.0};
  if (v.rowT >= 0) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < v.n_b;
         i += (int64_t)gridDim.x * blockDim.x) {
      if (J[i] > 0.0) {
        acc[0] += b[i];
        acc[1] += ka ? ka[i] : 0.0;
        acc[2] += 1.0;
      }
    }
  }
  block_sum<3>(acc, lds);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = acc[0];
    partials[gridDim.x + blockIdx.x] = acc[1];
    partials[2 * gridDim.x + blockIdx.x] = acc[2];
  }
  if (!arrive_last(&ctl->counter[1], &last)) return;
  double tot[3];
  sum_partials<3>(partials, gridDim.x, tot, lds);
  if (threadIdx.x == 0) {
    ctl->n_e = tot[2];
    ctl->mu_b = tot[2] > 0.0 ? tot[0] / tot[2] : 0.0;
    ctl->mu_ka = tot[2] > 0.0 ? tot[1] / tot[2] : 0.0;
    ctl->counter[1] = 0;
  }
}

// b <- P b;  a = a0 (or 0);  r = P b - P K a0;  z = J r;  p = z.
__global__ void __launch_bounds__(kBlock) k_cg_init(View v, double* __restrict__ b, const double* __restrict__ ka,
                                                    const double* __restrict__ a0, double* __restrict__ a,
                                                    double* __restrict__ r, double* __restrict__ z,
                                                    double* __restrict__ p, const double* __restrict__ J,
                                                    CgCtl* __restrict__ ctl, double* __restrict__ partials,
                                                    double tol, int max_iter) {
  __shared__ double lds[3 * 16];
  __shared__ bool last;
  const int64_t N = (int64_t)v.n_streams * v.n_b;
  const double mu_b = ctl->mu_b, mu_ka = ctl->mu_ka;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    const bool e = t_valid_row(v, i, J);
    const double bi = b[i] - (e ? mu_b : 0.0);
    b[i] = bi;
    double ri = bi;
    if (ka) ri -= ka[i] - (e ? mu_ka : 0.0);
    a[i] = a0 ? a0[i] : 0.0;
    r[i] = ri;
    const double zi = J[i] * ri;
    z[i] = zi;
    p[i] = zi;
    acc[0] += ri * zi;
    acc[1] += bi * bi;
    acc[2] += ri * ri;
  }
  block_sum<3>(acc, lds);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = acc[0];
    partials[gridDim.x + blockIdx.x] = acc[1];
    partials[2 * gridDim.x + blockIdx.x] = acc[2];
  }
  if (!arrive_last(&ctl->counter[2], &last)) return;
  double tot[3];
  sum_partials<3>(partials, gridDim.x, tot, lds);
  if (threadIdx.x == 0) {
    ctl->rz = tot[0];
    ctl->b_norm = sqrt(tot[1]);
    ctl->r_norm = sqrt(tot[2]);
    ctl->tol = tol;
    ctl->max_iter = max_iter;
    ctl->iter = 0;
    ctl->alpha = 0.0;
    ctl->beta = 0.0;
    ctl->mu = 0.0;
    if (!isfinite(tot[0]) || !isfinite(tot[1]) || !isfinite(tot[2])) {
      ctl->done = DONE_NAN;
    } else if (ctl->b_norm == 0.0 || ctl->r_norm <= tol * ctl->b_norm) {
      ctl->done = DONE_CONVERGED;
    } else if (max_iter <= 0) {
      ctl->done = DONE_MAXITER;
    } else {
      ctl->done = DONE_RUNNING;
    }
    ctl->counter[2] = 0;
  }
}

// a += alpha p;  r -= alpha P q;  z = J r;  per-block partials of r.z and r.r
// (finished by a single-workgroup kernel).
__global__ void __launch_bounds__(kBlock) k_cg_update(View v, double* __restrict__ a, double* __restrict__ r,
                                                      double* __restrict__ z, const double* __restrict__ p,
                                                      const double* __restrict__ q, const double* __restrict__ J,
                                                      CgCtl* __restrict__ ctl, double* __restrict__ partials) {
  __shared__ double lds[2 * 16];
  cg_update_body(v, a, r, z, p, q, J, ctl, partials, blockIdx.x, gridDim.x, lds);
}

__global__ void __launch_bounds__(kBlock) k_p_update(int64_t N, double* __restrict__ p, const double* __restrict__ z,
                                                     const CgCtl* __restrict__ ctl) {
  if (ctl->done) return;
  const double beta = ctl->beta;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = z[i] + beta * p[i];
}

// Canonical T baselines: zero mean over baselines with valid T samples; the
// others are set to 0.
__global__ void __launch_bounds__(kBlock) k_canon_mean(View v, const double* __restrict__ a,
                                                       const double* __restrict__ J, CgCtl* __restrict__ ctl,
                                                       double* __restrict__ partials) {
  __shared__ double lds[2 * 16];
  __shared__ bool last;
  double acc[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < v.n_b; i += (int64_t)gridDim.x * blockDim.x) {
    if (J[i] > 0.0) {
      acc[0] += a[i];
      acc[1] += 1.0;
    }
  }
  block_sum<2>(acc, lds);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = acc[0];
    partials[gridDim.x + blockIdx.x] = acc[1];
  }
  if (!arrive_last(&ctl->counter[3], &last)) return;
  double tot[2];
  sum_partials<2>(partials, gridDim.x, tot, lds);
  if (threadIdx.x == 0) {
    ctl->mu = tot[1] > 0.0 ? tot[0] / tot[1] : 0.0;
    ctl->counter[3] = 0;
  }
}

__global__ void __launch_bounds__(kBlock) k_canon_apply(View v, double* __restrict__ a, const double* __restrict__ J,
                                                        const CgCtl* __restrict__ ctl) {
  const double mu = ctl->mu;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < v.n_b; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = J[i] > 0.0 ? a[i] - mu : 0.0;
}

// || P b - P K a ||_2 with the T projection of K a recomputed here.
__global__ void __launch_bounds__(kBlock) k_resid_norm(View v, const double* __restrict__ b,
                                                       const double* __restrict__ ka, const double* __restrict__ J,
                                                       CgCtl* __restrict__ ctl, double* __restrict__ partials,
                                                       double* __restrict__ out_norm) {
  // one pass over x = b - K a: sum of x^2, sum of x and count over T-valid
  // rows; then ||x - mean_T(x) e||^2 = sum x^2 - (sum_T x)^2 / n_e by the last block
  __shared__ double lds[3 * 16];
  __shared__ bool last;
  double acc[3] = {0.0, 0.0, 0.0};
  const int64_t N = (int64_t)v.n_streams * v.n_b;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    const double x = b[i] - ka[i];
    acc[0] += x * x;
    if (t_valid_row(v, i, J)) {
      acc[1] += x;
      acc[2] += 1.0;
    }
  }
  block_sum<3>(acc, lds);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = acc[0];
    partials[gridDim.x + blockIdx.x] = acc[1];
    partials[2 * gridDim.x + blockIdx.x] = acc[2];
  }
  if (!arrive_last(&ctl->counter[3], &last)) return;
  double tot[3];
  sum_partials<3>(partials, gridDim.x, tot, lds);
  if (threadIdx.x == 0) {
    const double s2 = tot[0] - (tot[2] > 0.0 ? tot[1] * tot[1] / tot[2] : 0.0);
    *out_norm = sqrt(s2 > 0.0 ? s2 : 0.0);
    ctl->counter[3] = 0;
  }
}

__global__ void k_fill(double* x, int64_t n, double value) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = value;
}

__global__ void k_fill_u32(uint32_t* x, int64_t n, uint32_t value) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = value;
}

unsigned grid_for(int64_t n, int64_t per_block, unsigned cap) {
  int64_t g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

constexpr unsigned kStreamGrid = 8192;   // grid-stride kernels over samples
constexpr unsigned kVectorGrid = 1024;   // grid-stride kernels over baseline vectors / pixels

}  // namespace

// ---------------------------------------------------------------- launchers

hipError_t launch_pointing(const View& v, int psi_f32, int32_t* hits, double* M4, int* err, hipStream_t st) {
  const unsigned g = grid_for(v.n_t, kBlock, kStreamGrid);
  if (psi_f32)
    hipLaunchKernelGGL(k_pointing<float>, dim3(g), dim3(kBlock), 0, st, v, hits, M4, err);
  else
    hipLaunchKernelGGL(k_pointing<double>, dim3(g), dim3(kBlock), 0, st, v, hits, M4, err);
  return hipGetLastError();
}

hipError_t launch_invert(const View& v, const int32_t* hits, const double* M4, double rcond_cut, double* Minv4,
                         uint8_t* valid, double* blocks_out, unsigned long long* counts, hipStream_t st) {
  const unsigned g = grid_for(v.n_pix, kBlock, kVectorGrid);
  hipLaunchKernelGGL(k_invert, dim3(g), dim3(kBlock), 0, st, v, hits, M4, rcond_cut, Minv4, valid, blocks_out,
                     counts);
  return hipGetLastError();
}

hipError_t launch_baseline_counts(const View& v, const uint8_t* valid, int32_t* nvalid, double* J,
                                  unsigned long long* counts, hipStream_t st) {
  hipLaunchKernelGGL(k_baseline_counts, dim3((unsigned)v.n_b), dim3(kBlock), 0, st, v, valid, nvalid, J, counts);
  return hipGetLastError();
}

template <typename PT, typename TT>
static void bin_dispatch(const View& v, const void* tod, const double* base, double bsign, const uint8_t* valid,
                         double* s4, int* err, const CgCtl* gate, hipStream_t st) {
  const unsigned g = grid_for(v.n_t, kBlock, kStreamGrid);
  const TT* x = static_cast<const TT*>(tod);
  if (tod && base)
    hipLaunchKernelGGL((k_bin<PT, TT, true, true>), dim3(g), dim3(kBlock), 0, st, v, x, base, bsign, valid, s4, err,
                       gate);
  else if (tod)
    hipLaunchKernelGGL((k_bin<PT, TT, true, false>), dim3(g), dim3(kBlock), 0, st, v, x, base, bsign, valid, s4,
                       err, gate);
  else if (base)
    hipLaunchKernelGGL((k_bin<PT, TT, false, true>), dim3(g), dim3(kBlock), 0, st, v, x, base, bsign, valid, s4,
                       err, gate);
}

hipError_t launch_bin(const View& v, int psi_f32, const void* tod, int tod_f32, const double* base, double bsign,
                      const uint8_t* valid, double* s4, int* err, const CgCtl* gate, hipStream_t st) {
  if (psi_f32) {
    if (tod_f32)
      bin_dispatch<float, float>(v, tod, base, bsign, valid, s4, err, gate, st);
    else
      bin_dispatch<float, double>(v, tod, base, bsign, valid, s4, err, gate, st);
  } else {
    if (tod_f32)
      bin_dispatch<double, float>(v, tod, base, bsign, valid, s4, err, gate, st);
    else
      bin_dispatch<double, double>(v, tod, base, bsign, valid, s4, err, gate, st);
  }
  return hipGetLastError();
}

hipError_t launch_apply(int64_t n_pix, const double* s4, const double* Minv4, double* m, int m_stride, double* s_clear,
                        const CgCtl* gate, hipStream_t st) {
  const unsigned g = grid_for(n_pix, kBlock, 4096);
  hipLaunchKernelGGL(k_apply, dim3(g), dim3(kBlock), 0, st, n_pix, s4, Minv4, m, m_stride, s_clear, gate);
  return hipGetLastError();
}

template <typename PT, typename TT>
static void unbin_dispatch(const View& v, const void* tod, const double* base, double bsign, const double* m4,
                           const uint8_t* valid, const int32_t* nvalid, double* out, CgCtl* ctl, double* partials,
                           hipStream_t st) {
  const dim3 g((unsigned)v.n_b), blk(kBlock);
  const TT* x = static_cast<const TT*>(tod);
  if (ctl)
    hipLaunchKernelGGL((k_unbin_reduce<PT, TT, false, true, true>), g, blk, 0, st, v, x, base, bsign, m4, valid,
                       nvalid, out, ctl, partials);
  else if (tod && base)
    hipLaunchKernelGGL((k_unbin_reduce<PT, TT, true, true, false>), g, blk, 0, st, v, x, base, bsign, m4, valid,
                       nvalid, out, ctl, partials);
  else if (tod)
    hipLaunchKernelGGL((k_unbin_reduce<PT, TT, true, false, false>), g, blk, 0, st, v, x, base, bsign, m4, valid,
                       nvalid, out, ctl, partials);
  else if (base)
    hipLaunchKernelGGL((k_unbin_reduce<PT, TT, false, true, false>), g, blk, 0, st, v, x, base, bsign, m4, valid,
                       nvalid, out, ctl, partials);
  else
    hipLaunchKernelGGL((k_unbin_reduce<PT, TT, false, false, false>), g, blk, 0, st, v, x, base, bsign, m4, valid,
                       nvalid, out, ctl, partials);
}

hipError_t launch_unbin_reduce(const View& v, int psi_f32, const void* tod, int tod_f32, const double* base,
                               double bsign, const double* m4, const uint8_t* valid, const int32_t* nvalid,
                               double* out, CgCtl* ctl, double* partials, hipStream_t st) {
  if (psi_f32) {
    if (tod_f32)
      unbin_dispatch<float, float>(v, tod, base, bsign, m4, valid, nvalid, out, ctl, partials, st);
    else
      unbin_dispatch<float, double>(v, tod, base, bsign, m4, valid, nvalid, out, ctl, partials, st);
  } else {
    if (tod_f32)
      unbin_dispatch<double, float>(v, tod, base, bsign, m4, valid, nvalid, out, ctl, partials, st);
    else
      unbin_dispatch<double, double>(v, tod, base, bsign, m4, valid, nvalid, out, ctl, partials, st);
  }
  return hipGetLastError();
}

hipError_t launch_scan(const View& v, int psi_f32, const double* map3, double* out, int* err, hipStream_t st) {
  const unsigned g = grid_for(v.n_t, kBlock, kStreamGrid);
  if (psi_f32)
    hipLaunchKernelGGL(k_scan<float>, dim3(g), dim3(kBlock), 0, st, v, map3, out, err);
  else
    hipLaunchKernelGGL(k_scan<double>, dim3(g), dim3(kBlock), 0, st, v, map3, out, err);
  return hipGetLastError();
}

hipError_t launch_reduce(const View& v, const void* x, int x_f32, const uint8_t* valid, double* out, hipStream_t st) {
  if (x_f32)
    hipLaunchKernelGGL(k_reduce<float>, dim3((unsigned)v.n_b), dim3(kBlock), 0, st, v,
                       static_cast<const float*>(x), valid, out);
  else
    hipLaunchKernelGGL(k_reduce<double>, dim3((unsigned)v.n_b), dim3(kBlock), 0, st, v,
                       static_cast<const double*>(x), valid, out);
  return hipGetLastError();
}

static unsigned vec_grid(const View& v) { return grid_for((int64_t)v.n_streams * v.n_b, kBlock, kVectorGrid); }

hipError_t launch_cg_start(const View& v, double* b, const double* ka, const double* a0, double* a, double* r,
                           double* z, double* p, const double* J, CgCtl* ctl, double* partials, double tol,
                           int max_iter, hipStream_t st) {
  const unsigned g1 = grid_for(v.n_b, kBlock, kVectorGrid);
  hipLaunchKernelGGL(k_cg_means, dim3(g1), dim3(kBlock), 0, st, v, b, ka, J, ctl, partials);
  hipLaunchKernelGGL(k_cg_init, dim3(vec_grid(v)), dim3(kBlock), 0, st, v, b, ka, a0, a, r, z, p, J, ctl, partials,
                     tol, max_iter);
  return hipGetLastError();
}

int cg_update_blocks(const View& v) { return (int)vec_grid(v); }

hipError_t launch_cg_update(const View& v, double* a, double* r, double* z, const double* p, const double* q,
                            const double* J, CgCtl* ctl, double* partials, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_update, dim3(vec_grid(v)), dim3(kBlock), 0, st, v, a, r, z, p, q, J, ctl, partials);
  return hipGetLastError();
}

hipError_t launch_p_update(const View& v, double* p, const double* z, const CgCtl* ctl, hipStream_t st) {
  const int64_t N = (int64_t)v.n_streams * v.n_b;
  hipLaunchKernelGGL(k_p_update, dim3(vec_grid(v)), dim3(kBlock), 0, st, N, p, z, ctl);
  return hipGetLastError();
}

hipError_t launch_canonicalise(const View& v, double* a, const double* J, double* partials, CgCtl* ctl,
                               hipStream_t st) {
  if (v.rowT < 0) return hipSuccess;
  const unsigned g = grid_for(v.n_b, kBlock, kVectorGrid);
  hipLaunchKernelGGL(k_canon_mean, dim3(g), dim3(kBlock), 0, st, v, a, J, ctl, partials);
  hipLaunchKernelGGL(k_canon_apply, dim3(g), dim3(kBlock), 0, st, v, a, J, ctl);
  return hipGetLastError();
}

hipError_t launch_residual_norm(const View& v, const double* b, const double* ka, const double* J, CgCtl* ctl,
                                double* partials, double* out_norm, hipStream_t st) {
  hipLaunchKernelGGL(k_resid_norm, dim3(vec_grid(v)), dim3(kBlock), 0, st, v, b, ka, J, ctl, partials, out_norm);
  return hipGetLastError();
}

hipError_t launch_fill(double* x, int64_t n, double value, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, st, x, n, value);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* x, int64_t n, uint32_t value, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, st, x, n, value);
  return hipGetLastError();
}

}  // namespace dst
