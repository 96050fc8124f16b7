// Multi-right-hand-side kernels: one pass over the run records applies the
// destriping operator (Eq. 13 of arXiv:1309.5609) to every realization of a
// batch that shares the pointing.  Lanes of a wavefront are split into
// 64 / Rp slots of Rp realization lanes: the lanes of one slot read the same
// run record (one broadcast access) and gather the Rp values of their
// realizations from one contiguous stretch, so the run stream is read once
// per iteration for the whole batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <type_traits>

#include "dst_device.h"
#include "dst_multi.h"

namespace dst {
namespace {

using dev::kBlock;
using dev::kWaves;
using dev::lane_id;
using dev::rot2;

// ---------------------------------------------------------------- setup

// Pixel-order position of every time-order run: runs of compact pixel c sit
// at pstart[c] .. pstart[c + 1] in the order of the sorted run keys of its
// original pixel (seg gives that pixel's range of sorted keys).
__global__ void __launch_bounds__(kBlock) k_run_positions(int64_t n_obs, const uint32_t* __restrict__ order,
                                                          const int64_t* __restrict__ seg,
                                                          const uint32_t* __restrict__ rperm,
                                                          const int64_t* __restrict__ pstart,
                                                          uint32_t* __restrict__ ipos) {
  const int lane = lane_id();
  const int64_t nw = (int64_t)gridDim.x * kWaves;
  for (int64_t c = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); c < n_obs; c += nw) {
    const uint32_t p = order[c];
    const int64_t j0 = seg[2 * (int64_t)p], j1 = seg[2 * (int64_t)p + 1];
    const int64_t d0 = pstart[c];
    for (int64_t j = j0 + lane; j < j1; j += 64) ipos[rperm[j]] = (uint32_t)(d0 + (j - j0));
  }
}

// One wavefront per baseline; one lane per run; NR realizations per pass
// (their timelines share the angle loads and the trigonometry).  Per run and
// realization: w_T sum d_T and the rotated, weighted q/u sums, stored in the
// run's record (one 128-byte line holding every realization of the pass) at
// its pixel-order position, so each scattered store writes a whole line; per
// baseline: w_k sum d_k over valid samples (the data part of b = F^T Z d).
// When the samples of 64 consecutive runs fit kStageM (half that with FP64
// timelines), the wavefront first
// copies them (angles and timelines) into LDS with coalesced loads and the
// lanes read their runs from there.
constexpr int kStageM = 256;

template <typename PT, typename TT, bool HAS_T, bool HAS_QU, int NR>
__global__ void __launch_bounds__(kBlock) k_multi_tod(View v, TodSet tods, const uint32_t* __restrict__ bstart,
                                                      const uint32_t* __restrict__ t0,
                                                      const int32_t* __restrict__ tpix, const int32_t* __restrict__ tn,
                                                      const uint32_t* __restrict__ ipos,
                                                      const uint8_t* __restrict__ valid, int Rp, int ri0,
                                                      double* __restrict__ prs, double* __restrict__ braw) {
  constexpr int NROW = (HAS_T ? 1 : 0) + (HAS_QU ? 2 : 0);  // timeline rows per realization
  constexpr int iT = 0, iQ = HAS_T ? 1 : 0, iU = iQ + 1;
  constexpr int SM = sizeof(TT) == 4 ? kStageM : kStageM / 2;  // staged samples (LDS per workgroup ~64 KB)
  __shared__ PT s_psi[HAS_QU ? kWaves : 1][HAS_QU ? SM : 1];
  __shared__ TT s_tod[kWaves][NR * NROW][SM];
  const PT* psi = static_cast<const PT*>(v.psi);
  const int lane = lane_id();
  const int wave = threadIdx.x >> 6;
  const int64_t b = (int64_t)blockIdx.x * kWaves + wave;
  if (b >= v.n_b) return;  // the block's waves never synchronise with each other
  const int64_t n_t = v.n_t;
  const int64_t r0 = bstart[b], r1 = bstart[b + 1];
  double acc[3 * NR];
#pragma unroll
  for (int i = 0; i < 3 * NR; ++i) acc[i] = 0.0;
  constexpr int U = NR >= 3 ? 1 : (NR == 2 ? 2 : 4);  // samples whose loads are issued together
  for (int64_t jb = r0; jb < r1; jb += 64) {
    const int64_t j = jb + lane;
    const bool has = j < r1;
    const int64_t ts = has ? (int64_t)t0[j] : 0;
    const int n = has ? tn[j] : 0;
    const uint8_t f = has ? valid[tpix[j]] : 0;
    // samples spanned by these runs (lane 0 always holds one)
    const int last = r1 - 1 - jb < 63 ? (int)(r1 - 1 - jb) : 63;
    const int64_t lo = __shfl(ts, 0, 64), hi = __shfl(ts + n, last, 64);
    const bool staged = hi - lo <= SM;
    if (staged) {
      for (int e = lane; e < hi - lo; e += 64) {
        const int64_t t = lo + e;
        if (HAS_QU) s_psi[HAS_QU ? wave : 0][e] = psi[t];
#pragma unroll
        for (int i = 0; i < NR; ++i) {
          const TT* tod = static_cast<const TT*>(tods.p[i]);
          if (HAS_T) s_tod[wave][NROW * i + iT][e] = tod[v.rowT * n_t + t];
          if (HAS_QU) {
            s_tod[wave][NROW * i + iQ][e] = tod[v.rowQ * n_t + t];
            s_tod[wave][NROW * i + iU][e] = tod[v.rowU * n_t + t];
          }
        }
      }
      // LDS operations of one wavefront execute in issue order; the barrier
      // keeps the compiler from moving the reads above the writes.
      __builtin_amdgcn_wave_barrier();
    }
    double dT[NR], dq[NR], du[NR], dQ[NR], dU[NR];
#pragma unroll
    for (int i = 0; i < NR; ++i) dT[i] = dq[i] = du[i] = dQ[i] = dU[i] = 0.0;
    for (int k0 = 0; k0 < n; k0 += U) {
      double ang[U], xT[U][NR], xq[U][NR], xu[U][NR];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t t = ts + k0 + u;
        const bool in = k0 + u < n;
        const int64_t e = t - lo;
        if (staged) {
          ang[u] = (HAS_QU && in) ? (double)s_psi[HAS_QU ? wave : 0][HAS_QU ? e : 0] : 0.0;
#pragma unroll
          for (int i = 0; i < NR; ++i) {
            xT[u][i] = (HAS_T && in) ? (double)s_tod[wave][NROW * i + iT][e] : 0.0;
            xq[u][i] = (HAS_QU && in) ? (double)s_tod[wave][NROW * i + iQ][e] : 0.0;
            xu[u][i] = (HAS_QU && in) ? (double)s_tod[wave][NROW * i + iU][e] : 0.0;
          }
        } else {
          ang[u] = (HAS_QU && in) ? (double)psi[t] : 0.0;
#pragma unroll
          for (int i = 0; i < NR; ++i) {
            const TT* tod = static_cast<const TT*>(tods.p[i]);
            xT[u][i] = (HAS_T && in) ? (double)tod[v.rowT * n_t + t] : 0.0;
            xq[u][i] = (HAS_QU && in) ? (double)tod[v.rowQ * n_t + t] : 0.0;
            xu[u][i] = (HAS_QU && in) ? (double)tod[v.rowU * n_t + t] : 0.0;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (k0 + u >= n) break;
        double c = 1.0, s = 0.0;
        if (HAS_QU) rot2(ang[u], c, s);
#pragma unroll
        for (int i = 0; i < NR; ++i) {
          if (HAS_T) dT[i] += xT[u][i];
          if (HAS_QU) {
            dq[i] += xq[u][i];
            du[i] += xu[u][i];
            const double wq = v.w[1] * xq[u][i], wu = v.w[2] * xu[u][i];
            dQ[i] += c * wq - s * wu;
            dU[i] += s * wq + c * wu;
          }
        }
      }
    }
    if (staged) __builtin_amdgcn_wave_barrier();  // reads done before the next stage overwrites
    if (!has) continue;
    const bool vT = HAS_T && (f & 1), vQ = HAS_QU && (f & 2);
    const int64_t pos = ipos[j];
    double rec[kRunRec];
#pragma unroll
    for (int e = 0; e < kRunRec; ++e) rec[e] = 0.0;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      rec[3 * i] = vT ? v.w[0] * dT[i] : 0.0;
      rec[3 * i + 1] = vQ ? dQ[i] : 0.0;
      rec[3 * i + 2] = vQ ? dU[i] : 0.0;
    }
    double2* o = reinterpret_cast<double2*>(prs + (int64_t)kRunRec * pos);
#pragma unroll
    for (int e = 0; e < kRunRec / 2; ++e) o[e] = make_double2(rec[2 * e], rec[2 * e + 1]);
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      if (vT) acc[3 * i] += dT[i];
      if (vQ) {
        acc[3 * i + 1] += dq[i];
        acc[3 * i + 2] += du[i];
      }
    }
  }
  dev::wave_sum<3 * NR>(acc);
  if (lane == 0) {
    const int64_t o = b * v.n_streams * Rp + ri0;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      if (HAS_T) braw[o + v.rowT * Rp + i] = v.w[0] * acc[3 * i];
      if (HAS_QU) {
        braw[o + v.rowQ * Rp + i] = v.w[1] * acc[3 * i + 1];
        braw[o + v.rowU * Rp + i] = v.w[2] * acc[3 * i + 2];
      }
    }
  }
}

// One wavefront per compact pixel: md = M^-1 (sum of its run sums), columns
// ri0 .. ri0 + nr - 1 (the pixel's run records are contiguous).
template <int NR>
__global__ void __launch_bounds__(kBlock) k_multi_pixsum(int64_t n_obs, View vc, const int64_t* __restrict__ pstart,
                                                         const double* __restrict__ prs,
                                                         const double* __restrict__ Minv4, int Rp, int ri0,
                                                         double* __restrict__ md) {
  const int lane = lane_id();
  const int64_t nw = (int64_t)gridDim.x * kWaves;
  for (int64_t c = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); c < n_obs; c += nw) {
    const int64_t j0 = pstart[c], j1 = pstart[c + 1];
    const double2* ip = reinterpret_cast<const double2*>(Minv4 + 4 * c);
    const double2 i01 = ip[0], i23 = ip[1];
    double acc[3 * NR];
#pragma unroll
    for (int i = 0; i < 3 * NR; ++i) acc[i] = 0.0;
    // two records per lane in flight; the first 3 NR doubles of each
    constexpr int ND = (3 * NR + 1) / 2;
    for (int64_t jb = j0 + lane; jb < j1; jb += 128) {
      double2 x[2][ND];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int64_t j = jb + 64 * u;
        const double2* xr = reinterpret_cast<const double2*>(prs + (int64_t)kRunRec * j);
#pragma unroll
        for (int e = 0; e < ND; ++e) x[u][e] = j < j1 ? xr[e] : make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
#pragma unroll
        for (int e = 0; e < 3 * NR; ++e) acc[e] += (e & 1) ? x[u][e >> 1].y : x[u][e >> 1].x;
      }
    }
    dev::wave_sum<3 * NR>(acc);
    if (lane == 0) {
#pragma unroll
      for (int i = 0; i < NR; ++i) {
        const int64_t o = c * vc.n_streams * Rp + ri0 + i;
        if (vc.rowT >= 0) md[o + vc.rowT * Rp] = i01.x * acc[3 * i];
        if (vc.rowQ >= 0) {
          md[o + vc.rowQ * Rp] = i01.y * acc[3 * i + 1] + i23.x * acc[3 * i + 2];
          md[o + vc.rowU * Rp] = i23.x * acc[3 * i + 1] + i23.y * acc[3 * i + 2];
        }
      }
    }
  }
}


// ---------------------------------------------------------------- operator

// Steps of the run loops whose gathers are issued together (each step takes
// one run per slot of lanes): two in the binning, four in the rescan (four in
// both, or two in both, measured slower).
constexpr int kStepsBin = 2, kStepsUnbin = 4;

// Value of v in the lane whose byte address (4 x lane) is a4.
template <typename T>
__device__ __forceinline__ T from_lane(int a4, T v) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_ds_bpermute(a4, __builtin_bit_cast(int, v)));
  } else {
    static_assert(sizeof(T) == 8, "32- or 64-bit values");
    const int2 w = __builtin_bit_cast(int2, v);
    return __builtin_bit_cast(
        T, make_int2(__builtin_amdgcn_ds_bpermute(a4, w.x), __builtin_amdgcn_ds_bpermute(a4, w.y)));
  }
}

__device__ __forceinline__ bool lane_active(int r, int R, const MultiCtl* ctl) {
  return r < R && (ctl == nullptr || ctl->done[r] == DONE_RUNNING);
}

// V consecutive realizations' values of one row (V = 1 or 2; 16-byte aligned
// when V = 2 because Rp is even then).
template <int V, typename GT>
__device__ __forceinline__ void load_v(const GT* q, double (&x)[V]) {
  if constexpr (V == 2 && sizeof(GT) == 8) {
    const double2 t = *reinterpret_cast<const double2*>(q);
    x[0] = t.x;
    x[1] = t.y;
  } else if constexpr (V == 2) {
    const float2 t = *reinterpret_cast<const float2*>(q);
    x[0] = (double)t.x;
    x[1] = (double)t.y;
  } else {
    x[0] = (double)q[0];
  }
}

// m = M^-1 A^T W F p per compact pixel (one wavefront per pixel), for every
// active realization.  p is unweighted; the weights are applied here.  Each
// lane carries V consecutive realizations, so one gather instruction serves
// 64 V / Rp runs.  GT: the storage type of p and m (double, or float in the
// mixed-precision iterations; sums in FP64 either way).
template <typename RT, bool HAS_T, bool HAS_QU, int V, typename GT>
__global__ void __launch_bounds__(kBlock) k_multi_bin(View vc, int R, int Rp, const int64_t* __restrict__ pstart,
                                                      const int32_t* __restrict__ pb, const int32_t* __restrict__ pn,
                                                      const RT* __restrict__ pcs, const GT* __restrict__ p,
                                                      const double* __restrict__ Minv4,
                                                      GT* __restrict__ m, const MultiCtl* __restrict__ ctl) {
  if (ctl && ctl->running == 0) return;
  const int lane = lane_id();
  const int Rl = Rp / V;  // lanes per slot
  const int r0 = (lane & (Rl - 1)) * V;
  const int slot = lane / Rl;
  const int slots = 64 / Rl;
  const int slot4 = 4 * slot;
  bool actv[V];
  bool any = false;
#pragma unroll
  for (int v = 0; v < V; ++v) {
    actv[v] = lane_active(r0 + v, R, ctl);
    any = any || actv[v];
  }
  const int nS = vc.n_streams;
  const int oT = vc.rowT * Rp, oQ = vc.rowQ * Rp, oU = vc.rowU * Rp;
  const double w0 = vc.w[0], w1 = vc.w[1], w2 = vc.w[2];
  // each XCD (workgroup i runs on XCD i mod 8) sweeps a contiguous eighth of
  // the compact pixels, so the pixels it works on at a time are neighbours,
  // visited by the same baselines, whose p rows stay in its L2
  const int64_t n_obs = vc.n_pix;
  const int64_t per = (n_obs + 7) / 8;
  const int64_t xcd = blockIdx.x & 7, kb = blockIdx.x >> 3, nk = gridDim.x >> 3;
  const int64_t lo = xcd * per, hi = std::min(n_obs, lo + per);
  for (int64_t c = lo + kb * kWaves + (threadIdx.x >> 6); c < hi; c += nk * kWaves) {
    const int64_t j0 = pstart[c], j1 = pstart[c + 1];
    // per realization: sum n p_T, and the four products of the angle sums
    // with p_Q, p_U (the weights of the rows are applied once per pixel)
    double aT[V], aCQ[V], aSU[V], aSQ[V], aCU[V];
#pragma unroll
    for (int v = 0; v < V; ++v) aT[v] = aCQ[v] = aSU[v] = aSQ[v] = aCU[v] = 0.0;
    // The run data of 63 runs at a time are loaded once, one run per lane
    // (coalesced), and handed to the slots by shuffles, so the only loads
    // left in the run loop are the gathers of p: those of kStepsBin steps are
    // issued together, with no branch between them.  Lane 63 never holds a
    // run (zero length and angle sums, baseline -1), so a step past the
    // window reads it and gathers row 0 with zero weight.
    const int o0 = HAS_T ? oT : oQ;  // the first row gathered
    const GT* pT = p + r0 + o0;
    const int64_t dQ = oQ - o0, dU = oU - o0;
    const uint32_t rowB = (uint32_t)(nS * Rp * sizeof(GT));  // bytes per baseline's block of rows
    for (int64_t wb = j0; wb < j1; wb += 63) {
      const int64_t jl = wb + lane;
      const bool inw = lane < 63 && jl < j1;
      const int w_b = inw ? pb[jl] : -1;
      const int w_n = (HAS_T && inw) ? pn[jl] : 0;
      const CS2<RT> w_cs = (HAS_QU && inw) ? reinterpret_cast<const CS2<RT>*>(pcs)[jl] : make_cs<RT>(0.0, 0.0);
      const RT w_c = w_cs.x, w_s = w_cs.y;
      const int nwin = j1 - wb < 63 ? (int)(j1 - wb) : 63;
      for (int k0 = 0; k0 < nwin; k0 += kStepsBin * slots) {  // uniform: every lane takes part in the shuffles
        int nn[kStepsBin];
        RT cu[kStepsBin], su[kStepsBin];
        const GT* pr[kStepsBin];
#pragma unroll
        for (int u = 0; u < kStepsBin; ++u) {
          const int a4 = min(4 * (k0 + u * slots) + slot4, 4 * 63);
          const int bb = from_lane(a4, w_b);
          nn[u] = from_lane(a4, w_n);
          cu[u] = from_lane(a4, w_c);
          su[u] = from_lane(a4, w_s);
          pr[u] = reinterpret_cast<const GT*>(reinterpret_cast<const char*>(pT) +
                                              (uint64_t)(uint32_t)max(bb, 0) * rowB);
        }
        if (!any) continue;
        double t[kStepsBin][V], tq[kStepsBin][V], tu[kStepsBin][V];
#pragma unroll
        for (int u = 0; u < kStepsBin; ++u) {
          if (HAS_T) load_v<V>(pr[u], t[u]);
          if (HAS_QU) {
            load_v<V>(pr[u] + dQ, tq[u]);
            load_v<V>(pr[u] + dU, tu[u]);
          }
        }
#pragma unroll
        for (int u = 0; u < kStepsBin; ++u) {
          const double N = (double)nn[u], C = (double)cu[u], S = (double)su[u];
#pragma unroll
          for (int v = 0; v < V; ++v) {
            if (HAS_T) aT[v] = fma(N, t[u][v], aT[v]);
            if (HAS_QU) {
              aCQ[v] = fma(C, tq[u][v], aCQ[v]);
              aSU[v] = fma(S, tu[u][v], aSU[v]);
              aSQ[v] = fma(S, tq[u][v], aSQ[v]);
              aCU[v] = fma(C, tu[u][v], aCU[v]);
            }
          }
        }
      }
    }
    double acc[3 * V];  // [row][v]: the weighted sums A^T W F p
#pragma unroll
    for (int v = 0; v < V; ++v) {
      acc[v] = w0 * aT[v];
      acc[V + v] = w1 * aCQ[v] - w2 * aSU[v];
      acc[2 * V + v] = w1 * aSQ[v] + w2 * aCU[v];
    }
    dev::lane_group_sum<3 * V>(acc, Rl);
    if (slot == 0 && any) {
      const double2* ip = reinterpret_cast<const double2*>(Minv4 + 4 * c);
      const double2 i01 = ip[0], i23 = ip[1];
      GT* mo = m + c * nS * Rp + r0;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        if (!actv[v]) continue;
        if (HAS_T) mo[oT + v] = (GT)(i01.x * acc[v]);
        if (HAS_QU) {
          mo[oQ + v] = (GT)(i01.y * acc[V + v] + i23.x * acc[2 * V + v]);
          mo[oU + v] = (GT)(i23.x * acc[V + v] + i23.y * acc[2 * V + v]);
        }
      }
    }
  }
}

// Rescan and baseline sums, one wavefront per baseline, each XCD (workgroup
// i runs on XCD i mod 8) sweeping a contiguous eighth of the baselines in the
// rescan order (baselines sorted by the smallest compact id they visit, so
// those over the same sky are processed together and share map lines in L2).
//   OPERATOR / CG:  q = w (n_valid p - sum_runs A . m)  (= K p)
//   RHS:            q = braw - w sum_runs A . m         (= F^T Z d with m = m_d)
// CG also writes per-workgroup partials [block][3][Rp] of p.q and of the
// T-projection sums (q_T and p_T over T-valid baselines).
template <typename RT, bool HAS_T, bool HAS_QU, int MODE, int V, typename GT>
__global__ void __launch_bounds__(kBlock) k_multi_unbin(View vc, int R, int Rp, const uint32_t* __restrict__ bstart,
                                                        const uint32_t* __restrict__ border,
                                                        const int32_t* __restrict__ tpix,
                                                        const int32_t* __restrict__ tn, const RT* __restrict__ tcs,
                                                        const GT* __restrict__ m,
                                                        const int32_t* __restrict__ nvalid,
                                                        const double* __restrict__ p, const double* __restrict__ braw,
                                                        double* __restrict__ q, MultiCtl* __restrict__ ctl,
                                                        double* __restrict__ partials) {
  __shared__ double lds[kWaves][3][64];
  if (MODE == UNBIN_CG && ctl->running == 0) return;
  const int lane = lane_id();
  const int wave = threadIdx.x >> 6;
  const int Rl = Rp / V;  // lanes per slot; each lane carries V consecutive realizations
  const int r0 = (lane & (Rl - 1)) * V;
  const int slot = lane / Rl;
  const int slots = 64 / Rl;
  const int slot4 = 4 * slot;
  bool actv[V];
  bool any = false;
#pragma unroll
  for (int v = 0; v < V; ++v) {
    actv[v] = lane_active(r0 + v, R, MODE == UNBIN_CG ? ctl : nullptr);
    any = any || actv[v];
  }
  const int nS = vc.n_streams;
  const int oT = vc.rowT * Rp, oQ = vc.rowQ * Rp, oU = vc.rowU * Rp;
  const double w0 = vc.w[0], w1 = vc.w[1], w2 = vc.w[2];
  const int64_t n_b = vc.n_b;
  const int64_t per = (n_b + 7) / 8;
  const int64_t x = blockIdx.x & 7, k = blockIdx.x >> 3, nk = gridDim.x >> 3;
  const int64_t lo = x * per, hi = std::min(n_b, lo + per);
  const int o0 = HAS_T ? oT : oQ;  // the first row gathered
  const GT* mT = m + r0 + o0;
  const int64_t dQ = oQ - o0, dU = oU - o0;
  const uint32_t rowB = (uint32_t)(nS * Rp * sizeof(GT));  // bytes per pixel row block
  double dots[3 * V];  // [kind][v]
#pragma unroll
  for (int i = 0; i < 3 * V; ++i) dots[i] = 0.0;
  for (int64_t bk = lo + k * kWaves + wave; bk < hi; bk += nk * kWaves) {
    const int64_t b = border[bk];
    const int64_t rs0 = bstart[b], rs1 = bstart[b + 1];
    double acc[3 * V];  // [row][v]
#pragma unroll
    for (int i = 0; i < 3 * V; ++i) acc[i] = 0.0;
    // run data of 63 runs at a time: one coalesced load per lane, handed to
    // the slots by shuffles; the run loop only gathers m, kStepsUnbin steps at
    // a time with no branch between the gathers (lane 63 holds no run, so a
    // step past the window reads it and gathers row 0 with zero weight)
    for (int64_t wb = rs0; wb < rs1; wb += 63) {
      const int64_t jl = wb + lane;
      const bool inw = lane < 63 && jl < rs1;
      const int w_c = inw ? tpix[jl] : -1;
      const int w_n = (HAS_T && inw) ? tn[jl] : 0;
      const CS2<RT> w_cs = (HAS_QU && inw) ? reinterpret_cast<const CS2<RT>*>(tcs)[jl] : make_cs<RT>(0.0, 0.0);
      const RT w_C = w_cs.x, w_S = w_cs.y;
      const int nwin = rs1 - wb < 63 ? (int)(rs1 - wb) : 63;
      for (int k0 = 0; k0 < nwin; k0 += kStepsUnbin * slots) {  // uniform: every lane takes part in the shuffles
        int nn[kStepsUnbin];
        RT cu[kStepsUnbin], su[kStepsUnbin];
        const GT* mr[kStepsUnbin];
#pragma unroll
        for (int u = 0; u < kStepsUnbin; ++u) {
          const int a4 = min(4 * (k0 + u * slots) + slot4, 4 * 63);
          const int cc = from_lane(a4, w_c);
          nn[u] = from_lane(a4, w_n);
          cu[u] = from_lane(a4, w_C);
          su[u] = from_lane(a4, w_S);
          mr[u] = reinterpret_cast<const GT*>(reinterpret_cast<const char*>(mT) +
                                              (uint64_t)(uint32_t)max(cc, 0) * rowB);
        }
        if (!any) continue;
        double t[kStepsUnbin][V], mQ[kStepsUnbin][V], mU[kStepsUnbin][V];
#pragma unroll
        for (int u = 0; u < kStepsUnbin; ++u) {
          if (HAS_T) load_v<V>(mr[u], t[u]);
          if (HAS_QU) {
            load_v<V>(mr[u] + dQ, mQ[u]);
            load_v<V>(mr[u] + dU, mU[u]);
          }
        }
#pragma unroll
        for (int u = 0; u < kStepsUnbin; ++u) {
          const double N = (double)nn[u], C = (double)cu[u], S = (double)su[u];
#pragma unroll
          for (int v = 0; v < V; ++v) {
            if (HAS_T) acc[v] = fma(N, t[u][v], acc[v]);
            if (HAS_QU) {
              acc[V + v] = fma(C, mQ[u][v], acc[V + v]);
              acc[V + v] = fma(S, mU[u][v], acc[V + v]);
              acc[2 * V + v] = fma(C, mU[u][v], acc[2 * V + v]);
              acc[2 * V + v] = fma(-S, mQ[u][v], acc[2 * V + v]);
            }
          }
        }
      }
    }
    dev::lane_group_sum<3 * V>(acc, Rl);
    if (slot == 0 && any) {
#pragma unroll
      for (int v = 0; v < V; ++v) {
        if (!actv[v]) continue;
        const int64_t o = b * nS * Rp + r0 + v;
        if (MODE == UNBIN_RHS) {
          if (HAS_T) q[o + oT] = braw[o + oT] - w0 * acc[v];
          if (HAS_QU) {
            q[o + oQ] = braw[o + oQ] - w1 * acc[V + v];
            q[o + oU] = braw[o + oU] - w2 * acc[2 * V + v];
          }
        } else {
          const double nT = (double)nvalid[b], nQ = (double)nvalid[n_b + b];
          if (HAS_T) {
            const double pv = p[o + oT];
            const double out = w0 * (pv * nT - acc[v]);
            q[o + oT] = out;
            dots[v] += pv * out;
            if (nT > 0.0) {
              dots[V + v] += out;
              dots[2 * V + v] += pv;
            }
          }
          if (HAS_QU) {
            const double pq = p[o + oQ], pu = p[o + oU];
            const double oq = w1 * (pq * nQ - acc[V + v]);
            const double ou = w2 * (pu * nQ - acc[2 * V + v]);
            q[o + oQ] = oq;
            q[o + oU] = ou;
            dots[v] += pq * oq + pu * ou;
          }
        }
      }
    }
  }
  if (MODE == UNBIN_CG) {
    if (slot == 0) {
#pragma unroll
      for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int v = 0; v < V; ++v) lds[wave][i][r0 + v] = dots[i * V + v];
      }
    }
    __syncthreads();
    if ((int)threadIdx.x < Rp) {
      const int t = threadIdx.x;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        double s = lds[0][i][t];
        for (int w = 1; w < kWaves; ++w) s += lds[w][i][t];
        partials[((int64_t)blockIdx.x * 3 + i) * Rp + t] = s;
      }
    }
  }
}

// ---------------------------------------------------------------- CG pieces

// Sum over threads with equal (thread mod Rp) in fixed order; the result for
// realization t sits in lds[i][t], t < Rp.
template <int N>
__device__ __forceinline__ void block_sum_by_rhs(double (&v)[N], double (*lds)[kBlock], int Rp) {
  const int t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < N; ++i) lds[i][t] = v[i];
  __syncthreads();
  for (int h = kBlock / 2; h >= Rp; h >>= 1) {
    if (t < h) {
#pragma unroll
      for (int i = 0; i < N; ++i) lds[i][t] += lds[i][t + h];
    }
    __syncthreads();
  }
}

// Sum of per-block partials [n_part][N][Rp] per realization, by one
// workgroup, in fixed order; the result for realization t sits in lds[i][t].
template <int N>
__device__ __forceinline__ void sum_partials_by_rhs(const double* __restrict__ part, int n_part, int Rp,
                                                    double (*lds)[kBlock]) {
  const int t = threadIdx.x;
  const int r = t & (Rp - 1), ch = t / Rp, nch = kBlock / Rp;
  double s[N];
#pragma unroll
  for (int i = 0; i < N; ++i) s[i] = 0.0;
  // the loads of eight blocks are issued together; the sums keep their order
#pragma unroll 8
  for (int blk = ch; blk < n_part; blk += nch) {
#pragma unroll
    for (int i = 0; i < N; ++i) s[i] += part[((int64_t)blk * N + i) * Rp + r];
  }
  block_sum_by_rhs<N>(s, lds, Rp);
}

__device__ __forceinline__ bool t_valid(const View& v, int row, int64_t b, const double* J) {
  return row == v.rowT && J[(int64_t)row * v.n_b + b] > 0.0;
}

// Per block and realization: sum of x over T-valid baselines and their count.
__global__ void __launch_bounds__(kBlock) k_multi_tsum(View v, int Rp, const double* __restrict__ x,
                                                       const double* __restrict__ J, double* __restrict__ partials) {
  __shared__ double lds[2][kBlock];
  double acc[2] = {0.0, 0.0};
  if (v.rowT >= 0) {
    const int nS = v.n_streams;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < v.n_b * Rp;
         i += (int64_t)gridDim.x * blockDim.x) {
      const int64_t b = i / Rp;
      const int r = (int)(i & (Rp - 1));
      if (J[v.rowT * v.n_b + b] > 0.0) {
        acc[0] += x[(b * nS + v.rowT) * Rp + r];
        acc[1] += 1.0;
      }
    }
  }
  block_sum_by_rhs<2>(acc, lds, Rp);
  if ((int)threadIdx.x < Rp) {
    partials[((int64_t)blockIdx.x * 2 + 0) * Rp + threadIdx.x] = lds[0][threadIdx.x];
    partials[((int64_t)blockIdx.x * 2 + 1) * Rp + threadIdx.x] = lds[1][threadIdx.x];
  }
}

// which = 0: mu_b and n_e (start-up); which = 1: mu (canonicalisation).
__global__ void __launch_bounds__(kBlock) k_multi_tsum_fin(int n_part, int Rp, MultiCtl* __restrict__ ctl,
                                                           const double* __restrict__ partials, int which) {
  __shared__ double lds[2][kBlock];
  sum_partials_by_rhs<2>(partials, n_part, Rp, lds);
  const int t = threadIdx.x;
  if (t < Rp) {
    const double mean = lds[1][t] > 0.0 ? lds[0][t] / lds[1][t] : 0.0;
    if (which == 0) {
      ctl->mu_b[t] = mean;
      if (t == 0) ctl->n_e = lds[1][0];
    } else {
      ctl->mu[t] = mean;
    }
  }
}

// b <- P b;  a = 0;  r = b;  z = J r;  p = z;  per-block partials of r.z, b.b.
__global__ void __launch_bounds__(kBlock) k_multi_init(View v, int R, int Rp, double* __restrict__ b,
                                                       double* __restrict__ a, double* __restrict__ r,
                                                       double* __restrict__ z, double* __restrict__ p,
                                                       const double* __restrict__ J,
                                                       const MultiCtl* __restrict__ ctl,
                                                       double* __restrict__ partials) {
  __shared__ double lds[2][kBlock];
  const int nS = v.n_streams;
  const int64_t N = v.n_b * nS * Rp;
  const int ri = threadIdx.x & (Rp - 1);
  const bool real = ri < R;
  const double mu_b = ctl->mu_b[ri];
  double acc[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t rowb = i / Rp;
    const int row = (int)(rowb % nS);
    const int64_t bb = rowb / nS;
    const double Ji = J[(int64_t)row * v.n_b + bb];
    double bi = real ? b[i] - (t_valid(v, row, bb, J) ? mu_b : 0.0) : 0.0;
    b[i] = bi;
    a[i] = 0.0;
    r[i] = bi;
    const double zi = Ji * bi;
    z[i] = zi;
    p[i] = zi;
    acc[0] += bi * zi;
    acc[1] += bi * bi;
  }
  block_sum_by_rhs<2>(acc, lds, Rp);
  if ((int)threadIdx.x < Rp) {
    partials[((int64_t)blockIdx.x * 2 + 0) * Rp + threadIdx.x] = lds[0][threadIdx.x];
    partials[((int64_t)blockIdx.x * 2 + 1) * Rp + threadIdx.x] = lds[1][threadIdx.x];
  }
}

__global__ void __launch_bounds__(kBlock) k_multi_init_fin(int n_part, int R, int Rp, MultiCtl* __restrict__ ctl,
                                                           const double* __restrict__ partials, double tol,
                                                           int max_iter) {
  __shared__ double lds[2][kBlock];
  sum_partials_by_rhs<2>(partials, n_part, Rp, lds);
  const int t = threadIdx.x;
  if (t < kMaxRhs) {
    ctl->iter[t] = 0;
    ctl->alpha[t] = 0.0;
    ctl->beta[t] = 0.0;
    ctl->mu[t] = 0.0;
    ctl->true_norm[t] = 0.0;
    if (t >= R) {
      ctl->rz[t] = ctl->b_norm[t] = ctl->r_norm[t] = 0.0;
      ctl->done[t] = DONE_PAD;
    } else {
      const double rz = lds[0][t], bb = lds[1][t];
      ctl->rz[t] = rz;
      ctl->b_norm[t] = sqrt(bb);
      ctl->r_norm[t] = sqrt(bb);
      if (!isfinite(rz) || !isfinite(bb))
        ctl->done[t] = DONE_NAN;
      else if (bb == 0.0)
        ctl->done[t] = DONE_CONVERGED;
      else if (max_iter <= 0)
        ctl->done[t] = DONE_MAXITER;
      else
        ctl->done[t] = DONE_RUNNING;
    }
  }
  __syncthreads();
  if (t == 0) {
    int run = 0;
    for (int i = 0; i < R; ++i) run += ctl->done[i] == DONE_RUNNING;
    ctl->running = run;
    ctl->tol = tol;
    ctl->max_iter = max_iter;
    ctl->n_rhs = R;
  }
}

// Several components: q loses each component's mean (per right-hand side)
// and ctl->corr[r] = sum over components of mean * (sum of p over the component).
__global__ void __launch_bounds__(1024) k_multi_comp(CompView cv, double* __restrict__ q,
                                                     const double* __restrict__ p, int64_t sb, int Rp,
                                                     MultiCtl* __restrict__ ctl) {
  if (ctl->running == 0) return;
  const int ncomp = *cv.ncomp;
  if (ncomp <= 1) return;
  __shared__ double lds[16 * 64];
  const double corr = comp_project_block(cv, ncomp, q, p, sb, Rp, lds);
  if ((int)threadIdx.x < Rp) ctl->corr[threadIdx.x] = corr;
}

// alpha_r = r.z / (p.K p) with K p projected on the T null space (one
// component: the mean mu of its T part, applied by the update; several: q
// was projected in place by k_multi_comp).
__global__ void __launch_bounds__(kBlock) k_multi_alpha(int n_part, int Rp, MultiCtl* __restrict__ ctl,
                                                        const double* __restrict__ partials,
                                                        const int32_t* __restrict__ ncomp_dev) {
  if (ctl->running == 0) return;
  __shared__ double lds[3][kBlock];
  sum_partials_by_rhs<3>(partials, n_part, Rp, lds);
  const int t = threadIdx.x;
  const bool split = ncomp_dev && *ncomp_dev > 1;
  if (t < Rp && ctl->done[t] == DONE_RUNNING) {
    const double mu = split ? 0.0 : (ctl->n_e > 0.0 ? lds[1][t] / ctl->n_e : 0.0);
    const double pkp = split ? lds[0][t] - ctl->corr[t] : lds[0][t] - mu * lds[2][t];
    ctl->mu[t] = mu;
    if (!isfinite(pkp))
      ctl->done[t] = DONE_NAN;
    else if (pkp <= 0.0)
      ctl->done[t] = DONE_BREAKDOWN;
    else
      ctl->alpha[t] = ctl->rz[t] / pkp;
  }
}

// a += alpha p;  r -= alpha P q;  z = J r;  per-block partials of r.z and r.r.
__global__ void __launch_bounds__(kBlock) k_multi_update(View v, int Rp, double* __restrict__ a,
                                                         double* __restrict__ r, double* __restrict__ z,
                                                         const double* __restrict__ q, const double* __restrict__ p,
                                                         const double* __restrict__ J, MultiCtl* __restrict__ ctl,
                                                         double* __restrict__ partials) {
  if (ctl->running == 0) return;
  __shared__ double lds[2][kBlock];
  const int nS = v.n_streams;
  const int64_t N = v.n_b * nS * Rp;
  const int ri = threadIdx.x & (Rp - 1);
  const bool run = ctl->done[ri] == DONE_RUNNING;
  const double alpha = ctl->alpha[ri], mu = ctl->mu[ri];
  double acc[2] = {0.0, 0.0};
  if (run) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
      const int64_t rowb = i / Rp;
      const int row = (int)(rowb % nS);
      const int64_t bb = rowb / nS;
      const double Ji = J[(int64_t)row * v.n_b + bb];
      const double qi = q[i] - ((row == v.rowT && Ji > 0.0) ? mu : 0.0);
      a[i] += alpha * p[i];
      const double rr = r[i] - alpha * qi;
      r[i] = rr;
      const double zz = Ji * rr;
      z[i] = zz;
      acc[0] += rr * zz;
      acc[1] += rr * rr;
    }
  }
  block_sum_by_rhs<2>(acc, lds, Rp);
  if ((int)threadIdx.x < Rp) {
    partials[((int64_t)blockIdx.x * 2 + 0) * Rp + threadIdx.x] = lds[0][threadIdx.x];
    partials[((int64_t)blockIdx.x * 2 + 1) * Rp + threadIdx.x] = lds[1][threadIdx.x];
  }
}

// Stopping test per realization and beta = r'.z' / r.z.
__global__ void __launch_bounds__(kBlock) k_multi_beta(int n_part, int Rp, MultiCtl* __restrict__ ctl,
                                                       const double* __restrict__ partials) {
  if (ctl->running == 0) return;
  __shared__ double lds[2][kBlock];
  sum_partials_by_rhs<2>(partials, n_part, Rp, lds);
  const int t = threadIdx.x;
  if (t < Rp && ctl->done[t] == DONE_RUNNING) {
    const double rz_new = lds[0][t];
    const double rn = sqrt(lds[1][t]);
    const int it = ctl->iter[t] + 1;
    ctl->iter[t] = it;
    ctl->r_norm[t] = rn;
    if (!isfinite(rz_new) || !isfinite(rn))
      ctl->done[t] = DONE_NAN;
    else if (rn <= ctl->tol * ctl->b_norm[t])
      ctl->done[t] = DONE_CONVERGED;
    else if (it >= ctl->max_iter)
      ctl->done[t] = DONE_MAXITER;
    else {
      ctl->beta[t] = rz_new / ctl->rz[t];
      ctl->rz[t] = rz_new;
    }
  }
  __syncthreads();
  if (t == 0) {
    int run = 0;
    for (int i = 0; i < ctl->n_rhs; ++i) run += ctl->done[i] == DONE_RUNNING;
    ctl->running = run;
  }
}

// p = z + beta p; with p32, its FP32 copy too (the mixed-precision gathers).
__global__ void __launch_bounds__(kBlock) k_multi_p(int64_t N, int Rp, double* __restrict__ p,
                                                    const double* __restrict__ z, const MultiCtl* __restrict__ ctl,
                                                    float* __restrict__ p32) {
  if (ctl->running == 0) return;
  const int ri = threadIdx.x & (Rp - 1);
  if (ctl->done[ri] != DONE_RUNNING) return;
  const double beta = ctl->beta[ri];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    const double x = z[i] + beta * p[i];
    p[i] = x;
    if (p32) p32[i] = (float)x;
  }
}

__global__ void __launch_bounds__(kBlock) k_to_f32(int64_t N, const double* __restrict__ x, float* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}

__global__ void __launch_bounds__(kBlock) k_multi_canon_apply(View v, int Rp, double* __restrict__ a,
                                                              const double* __restrict__ J,
                                                              const MultiCtl* __restrict__ ctl) {
  if (v.rowT < 0) return;
  const int nS = v.n_streams;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < v.n_b * Rp;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = i / Rp;
    const int r = (int)(i & (Rp - 1));
    const int64_t o = (b * nS + v.rowT) * Rp + r;
    a[o] = J[v.rowT * v.n_b + b] > 0.0 ? a[o] - ctl->mu[r] : 0.0;
  }
}

// Per block and realization, x = b - K a: sum of x^2 and sum of x over T-valid rows.
__global__ void __launch_bounds__(kBlock) k_multi_resid(View v, int Rp, const double* __restrict__ b,
                                                        const double* __restrict__ ka, const double* __restrict__ J,
                                                        double* __restrict__ partials) {
  __shared__ double lds[2][kBlock];
  const int nS = v.n_streams;
  const int64_t N = v.n_b * nS * Rp;
  double acc[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t rowb = i / Rp;
    const int row = (int)(rowb % nS);
    const int64_t bb = rowb / nS;
    const double x = b[i] - ka[i];
    acc[0] += x * x;
    if (t_valid(v, row, bb, J)) acc[1] += x;
  }
  block_sum_by_rhs<2>(acc, lds, Rp);
  if ((int)threadIdx.x < Rp) {
    partials[((int64_t)blockIdx.x * 2 + 0) * Rp + threadIdx.x] = lds[0][threadIdx.x];
    partials[((int64_t)blockIdx.x * 2 + 1) * Rp + threadIdx.x] = lds[1][threadIdx.x];
  }
}

// ||P x||^2 = sum x^2 - n_e mean_T(x)^2.
__global__ void __launch_bounds__(kBlock) k_multi_resid_fin(int n_part, int Rp, MultiCtl* __restrict__ ctl,
                                                            const double* __restrict__ partials) {
  __shared__ double lds[2][kBlock];
  sum_partials_by_rhs<2>(partials, n_part, Rp, lds);
  const int t = threadIdx.x;
  if (t < Rp) {
    const double n_e = ctl->n_e;
    const double s2 = lds[0][t] - (n_e > 0.0 ? lds[1][t] * lds[1][t] / n_e : 0.0);
    ctl->true_norm[t] = sqrt(s2 > 0.0 ? s2 : 0.0);
  }
}

__global__ void __launch_bounds__(kBlock) k_multi_extract(View v, int Rp, int ri, const double* __restrict__ x,
                                                          double* __restrict__ out) {
  const int nS = v.n_streams;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nS * v.n_b;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = i / v.n_b, b = i - row * v.n_b;
    out[i] = x[(b * nS + row) * Rp + ri];
  }
}

__global__ void __launch_bounds__(kBlock) k_multi_scatter(int64_t n_pix, View vc, const int32_t* __restrict__ cid,
                                                          int Rp, int ri, const double* __restrict__ md,
                                                          const double* __restrict__ m, double* __restrict__ out3) {
  const int nS = vc.n_streams;
  const int rows[3] = {vc.rowT, vc.rowQ, vc.rowU};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_pix; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = cid[i];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double val = 0.0;
      if (c >= 0 && rows[k] >= 0) {
        const int64_t o = (c * nS + rows[k]) * Rp + ri;
        val = md[o] - (m ? m[o] : 0.0);
      }
      out3[3 * i + k] = val;
    }
  }
}

// ---------------------------------------------------------------- dispatch

template <typename T>
struct type_tag {
  using type = T;
};
template <typename F>
void by_float(bool f32, F&& f) {
  if (f32)
    f(type_tag<float>{});
  else
    f(type_tag<double>{});
}
template <typename F>
void by_streams(const View& v, F&& f) {
  if (v.rowT >= 0 && v.rowQ >= 0)
    f(std::true_type{}, std::true_type{});
  else if (v.rowQ >= 0)
    f(std::false_type{}, std::true_type{});
  else
    f(std::true_type{}, std::false_type{});
}

unsigned grid_for(int64_t n, int64_t per_block, int64_t cap) {
  int64_t g = (n + per_block - 1) / per_block;
  return (unsigned)std::max<int64_t>(1, std::min(g, cap));
}

constexpr int kTsumBlocks = 256;

}  // namespace

int multi_padded(int R) {
  int Rp = 1;
  while (Rp < R) Rp <<= 1;
  return Rp;
}

hipError_t launch_run_positions(const Runs& W, uint32_t* ipos, hipStream_t st) {
  hipLaunchKernelGGL(k_run_positions, dim3(grid_for(W.n_obs, kWaves, 16384)), dim3(kBlock), 0, st, W.n_obs, W.order,
                     W.seg, W.rperm, W.pstart, ipos);
  return hipGetLastError();
}

hipError_t launch_multi_tod(const View& vc, int psi_f32, const TodSet& tods, int nr, int tod_f32, const Runs& W,
                            const uint32_t* ipos, const uint8_t* valid, int Rp, int ri0, double* prs, double* braw,
                            hipStream_t st) {
  const unsigned g = grid_for(vc.n_b, kWaves, INT32_MAX);
  by_float(psi_f32, [&](auto pt) {
    using PT = typename decltype(pt)::type;
    by_float(tod_f32, [&](auto tt) {
      using TT = typename decltype(tt)::type;
      by_streams(vc, [&](auto T, auto Q) {
        constexpr bool HT = decltype(T)::value, HQ = decltype(Q)::value;
        auto launch = [&](auto kern) {
          hipLaunchKernelGGL(kern, dim3(g), dim3(kBlock), 0, st, vc, tods, W.bstart, W.t0, W.tpix, W.tn, ipos, valid,
                             Rp, ri0, prs, braw);
        };
        if (nr >= 5)
          launch(k_multi_tod<PT, TT, HT, HQ, 5>);
        else if (nr == 4)
          launch(k_multi_tod<PT, TT, HT, HQ, 4>);
        else if (nr == 3)
          launch(k_multi_tod<PT, TT, HT, HQ, 3>);
        else if (nr == 2)
          launch(k_multi_tod<PT, TT, HT, HQ, 2>);
        else
          launch(k_multi_tod<PT, TT, HT, HQ, 1>);
      });
    });
  });
  return hipGetLastError();
}

hipError_t launch_multi_pixsum(int64_t n_obs, const View& vc, const Runs& W, const double* prs, int nr,
                               const double* Minv4, int Rp, int ri0, double* md, hipStream_t st) {
  const dim3 g(grid_for(n_obs, kWaves, 16384));
  if (nr >= 5)
    hipLaunchKernelGGL(k_multi_pixsum<5>, g, dim3(kBlock), 0, st, n_obs, vc, W.pstart, prs, Minv4, Rp, ri0, md);
  else if (nr == 4)
    hipLaunchKernelGGL(k_multi_pixsum<4>, g, dim3(kBlock), 0, st, n_obs, vc, W.pstart, prs, Minv4, Rp, ri0, md);
  else if (nr == 3)
    hipLaunchKernelGGL(k_multi_pixsum<3>, g, dim3(kBlock), 0, st, n_obs, vc, W.pstart, prs, Minv4, Rp, ri0, md);
  else if (nr == 2)
    hipLaunchKernelGGL(k_multi_pixsum<2>, g, dim3(kBlock), 0, st, n_obs, vc, W.pstart, prs, Minv4, Rp, ri0, md);
  else
    hipLaunchKernelGGL(k_multi_pixsum<1>, g, dim3(kBlock), 0, st, n_obs, vc, W.pstart, prs, Minv4, Rp, ri0, md);
  return hipGetLastError();
}

template <typename GT>
hipError_t multi_bin_impl(const View& vc, const Runs& W, const Multi& mu, const GT* p, const double* Minv4, GT* m,
                          const MultiCtl* ctl, hipStream_t st) {
  const int64_t per = (vc.n_pix + 7) / 8;
  const unsigned g = (unsigned)(8 * std::max<int64_t>(1, std::min<int64_t>((per + kWaves - 1) / kWaves, 2048)));
  by_float(W.f32, [&](auto rt) {
    using RT = typename decltype(rt)::type;
    by_streams(vc, [&](auto T, auto Q) {
      auto launch = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(g), dim3(kBlock), 0, st, vc, mu.R, mu.Rp, W.pstart, W.pb, W.pn,
                           static_cast<const RT*>(W.pcs), p, Minv4, m, ctl);
      };
      if (mu.Rp >= 2)
        launch(k_multi_bin<RT, decltype(T)::value, decltype(Q)::value, 2, GT>);
      else
        launch(k_multi_bin<RT, decltype(T)::value, decltype(Q)::value, 1, GT>);
    });
  });
  return hipGetLastError();
}

hipError_t launch_multi_bin(const View& vc, const Runs& W, const Multi& mu, const double* p, const double* Minv4,
                            double* m, const MultiCtl* ctl, hipStream_t st) {
  return multi_bin_impl<double>(vc, W, mu, p, Minv4, m, ctl, st);
}

hipError_t launch_multi_bin(const View& vc, const Runs& W, const Multi& mu, const float* p, const double* Minv4,
                            float* m, const MultiCtl* ctl, hipStream_t st) {
  return multi_bin_impl<float>(vc, W, mu, p, Minv4, m, ctl, st);
}

int multi_unbin_blocks(const View& vc) {
  const int64_t per = (vc.n_b + 7) / 8;
  const int64_t g = std::max<int64_t>(1, std::min<int64_t>((per + kWaves - 1) / kWaves, 256));
  return (int)(8 * g);
}

template <typename GT>
hipError_t multi_unbin_impl(const View& vc, const Runs& W, const Multi& mu, int mode, const GT* m,
                            const int32_t* nvalid, const double* p, const double* braw, double* q, MultiCtl* ctl,
                            double* partials, hipStream_t st) {
  const unsigned g = (unsigned)multi_unbin_blocks(vc);
  by_float(W.f32, [&](auto rt) {
    using RT = typename decltype(rt)::type;
    by_streams(vc, [&](auto T, auto Q) {
      constexpr bool HT = decltype(T)::value, HQ = decltype(Q)::value;
      auto launch = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(g), dim3(kBlock), 0, st, vc, mu.R, mu.Rp, W.bstart, W.border, W.tpix, W.tn,
                           static_cast<const RT*>(W.tcs), m, nvalid, p, braw, q, ctl, partials);
      };
      auto by_mode = [&](auto VV) {
        constexpr int V = decltype(VV)::value;
        if (mode == UNBIN_CG)
          launch(k_multi_unbin<RT, HT, HQ, UNBIN_CG, V, GT>);
        else if (mode == UNBIN_RHS)
          launch(k_multi_unbin<RT, HT, HQ, UNBIN_RHS, V, GT>);
        else
          launch(k_multi_unbin<RT, HT, HQ, UNBIN_OPERATOR, V, GT>);
      };
      if (mu.Rp >= 2)
        by_mode(std::integral_constant<int, 2>{});
      else
        by_mode(std::integral_constant<int, 1>{});
    });
  });
  return hipGetLastError();
}

hipError_t launch_multi_unbin(const View& vc, const Runs& W, const Multi& mu, int mode, const double* m,
                              const int32_t* nvalid, const double* p, const double* braw, double* q, MultiCtl* ctl,
                              double* partials, hipStream_t st) {
  return multi_unbin_impl<double>(vc, W, mu, mode, m, nvalid, p, braw, q, ctl, partials, st);
}

hipError_t launch_multi_unbin(const View& vc, const Runs& W, const Multi& mu, int mode, const float* m,
                              const int32_t* nvalid, const double* p, const double* braw, double* q, MultiCtl* ctl,
                              double* partials, hipStream_t st) {
  return multi_unbin_impl<float>(vc, W, mu, mode, m, nvalid, p, braw, q, ctl, partials, st);
}

int multi_update_blocks(const View& v, const Multi& mu) {
  return (int)grid_for((int64_t)v.n_b * v.n_streams * mu.Rp, kBlock, 1024);
}

hipError_t launch_multi_start(const View& v, const Multi& mu, double* b, double* a, double* r, double* z, double* p,
                              const double* J, MultiCtl* ctl, double* partials, double tol, int max_iter,
                              hipStream_t st) {
  const unsigned gt = grid_for((int64_t)v.n_b * mu.Rp, kBlock, kTsumBlocks);
  hipLaunchKernelGGL(k_multi_tsum, dim3(gt), dim3(kBlock), 0, st, v, mu.Rp, b, J, partials);
  hipLaunchKernelGGL(k_multi_tsum_fin, dim3(1), dim3(kBlock), 0, st, (int)gt, mu.Rp, ctl, partials, 0);
  const unsigned gu = (unsigned)multi_update_blocks(v, mu);
  hipLaunchKernelGGL(k_multi_init, dim3(gu), dim3(kBlock), 0, st, v, mu.R, mu.Rp, b, a, r, z, p, J, ctl, partials);
  hipLaunchKernelGGL(k_multi_init_fin, dim3(1), dim3(kBlock), 0, st, (int)gu, mu.R, mu.Rp, ctl, partials, tol,
                     max_iter);
  return hipGetLastError();
}

hipError_t launch_multi_comp(const View& v, const Multi& mu, const CompView& cv, double* q, const double* p,
                             MultiCtl* ctl, hipStream_t st) {
  if (!cv.ncomp) return hipSuccess;
  hipLaunchKernelGGL(k_multi_comp, dim3(1), dim3(1024), 0, st, cv, q, p, (int64_t)v.n_streams * mu.Rp, mu.Rp, ctl);
  return hipGetLastError();
}

hipError_t launch_multi_alpha(const View& vc, const Multi& mu, MultiCtl* ctl, const double* partials,
                              const CompView& cv, hipStream_t st) {
  hipLaunchKernelGGL(k_multi_alpha, dim3(1), dim3(kBlock), 0, st, multi_unbin_blocks(vc), mu.Rp, ctl, partials,
                     cv.ncomp);
  return hipGetLastError();
}

hipError_t launch_multi_update(const View& v, const Multi& mu, double* a, double* r, double* z, const double* q,
                               const double* p, const double* J, MultiCtl* ctl, double* partials, hipStream_t st) {
  hipLaunchKernelGGL(k_multi_update, dim3(multi_update_blocks(v, mu)), dim3(kBlock), 0, st, v, mu.Rp, a, r, z, q, p,
                     J, ctl, partials);
  return hipGetLastError();
}

hipError_t launch_multi_beta(const View& v, const Multi& mu, MultiCtl* ctl, const double* partials, hipStream_t st) {
  hipLaunchKernelGGL(k_multi_beta, dim3(1), dim3(kBlock), 0, st, multi_update_blocks(v, mu), mu.Rp, ctl, partials);
  return hipGetLastError();
}

hipError_t launch_multi_p(const View& v, const Multi& mu, double* p, const double* z, const MultiCtl* ctl,
                          hipStream_t st, float* p32) {
  const int64_t N = (int64_t)v.n_b * v.n_streams * mu.Rp;
  hipLaunchKernelGGL(k_multi_p, dim3(grid_for(N, kBlock, 2048)), dim3(kBlock), 0, st, N, mu.Rp, p, z, ctl, p32);
  return hipGetLastError();
}

hipError_t launch_to_f32(const double* x, float* y, int64_t N, hipStream_t st) {
  hipLaunchKernelGGL(k_to_f32, dim3(grid_for(N, kBlock, 2048)), dim3(kBlock), 0, st, N, x, y);
  return hipGetLastError();
}

hipError_t launch_multi_canonicalise(const View& v, const Multi& mu, double* a, const double* J, MultiCtl* ctl,
                                     double* partials, hipStream_t st) {
  const unsigned gt = grid_for((int64_t)v.n_b * mu.Rp, kBlock, kTsumBlocks);
  hipLaunchKernelGGL(k_multi_tsum, dim3(gt), dim3(kBlock), 0, st, v, mu.Rp, a, J, partials);
  hipLaunchKernelGGL(k_multi_tsum_fin, dim3(1), dim3(kBlock), 0, st, (int)gt, mu.Rp, ctl, partials, 1);
  hipLaunchKernelGGL(k_multi_canon_apply, dim3(gt), dim3(kBlock), 0, st, v, mu.Rp, a, J, ctl);
  return hipGetLastError();
}

hipError_t launch_multi_resid(const View& v, const Multi& mu, const double* b, const double* ka, const double* J,
                              MultiCtl* ctl, double* partials, hipStream_t st) {
  const unsigned g = (unsigned)multi_update_blocks(v, mu);
  hipLaunchKernelGGL(k_multi_resid, dim3(g), dim3(kBlock), 0, st, v, mu.Rp, b, ka, J, partials);
  hipLaunchKernelGGL(k_multi_resid_fin, dim3(1), dim3(kBlock), 0, st, (int)g, mu.Rp, ctl, partials);
  return hipGetLastError();
}

hipError_t launch_multi_extract(const View& v, const Multi& mu, int ri, const double* x, double* out,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_multi_extract, dim3(grid_for((int64_t)v.n_b * v.n_streams, kBlock, 4096)), dim3(kBlock), 0,
                     st, v, mu.Rp, ri, x, out);
  return hipGetLastError();
}

hipError_t launch_multi_scatter(const View& full, const View& vc, const int32_t* cid, const Multi& mu, int ri,
                                const double* md, const double* m, double* out3, hipStream_t st) {
  hipLaunchKernelGGL(k_multi_scatter, dim3(grid_for(full.n_pix, kBlock, 8192)), dim3(kBlock), 0, st, full.n_pix, vc,
                     cid, mu.Rp, ri, md, m, out3);
  return hipGetLastError();
}

}  // namespace dst
