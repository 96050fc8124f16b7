// Run-compressed pointing for the iterative solve.
//
// Inside one baseline the baseline offset is a constant, so every sample of a
// run -- a maximal stretch of consecutive samples on the same pixel within one
// baseline -- meets the same p[beta] in the binning of F p, and the same map
// values in the rescan.  Grouping the terms of A^T W F p and F^T W A m
// (Eqs. 10-13 of arXiv:1309.5609) by run gives, exactly up to rounding order,
//   T:  n_r p_T[beta]            and  n_r m_I
//   Q:  C_r w_q p_q - S_r w_u p_u    U: S_r w_q p_q + C_r w_u p_u
//   q:  C_r m_Q + S_r m_U            u: C_r m_U - S_r m_Q
// with n_r the run length and C_r, S_r the sums of cos 2psi, sin 2psi over the
// run.  The runs are built once per solve; each CG iteration then reads one
// small record per run (no trigonometry), in pixel order for the binning and
// in time order for the rescan.
#include <hip/hip_runtime.h>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <type_traits>

#include "dst_internal.h"
#include "dst_runs.h"
#include "dst_cg.h"
#include "dst_group.h"
#include "dst_trig.h"

namespace dst {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

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

// Smallest and largest eigenvalue of the symmetric 3x3 matrix
// [[a00, a01, a02], [a01, a11, a12], [a02, a12, a22]] by the trigonometric
// form of the roots of its characteristic cubic (Smith 1961).
__device__ __forceinline__ void sym3_eig_range(double a00, double a01, double a02, double a11, double a12,
                                               double a22, double& lmin, double& lmax) {
  const double p1 = a01 * a01 + a02 * a02 + a12 * a12;
  const double q = (a00 + a11 + a22) / 3.0;
  const double b00 = a00 - q, b11 = a11 - q, b22 = a22 - q;
  const double p2 = b00 * b00 + b11 * b11 + b22 * b22 + 2.0 * p1;
  if (!(p2 > 0.0)) {  // a multiple of the identity
    lmin = lmax = q;
    return;
  }
  const double pp = sqrt(p2 / 6.0);
  const double detb = b00 * (b11 * b22 - a12 * a12) - a01 * (a01 * b22 - a12 * a02) + a02 * (a01 * a12 - b11 * a02);
  double r = detb / (2.0 * pp * pp * pp);
  r = r < -1.0 ? -1.0 : (r > 1.0 ? 1.0 : r);
  const double phi = acos(r) / 3.0;
  lmax = q + 2.0 * pp * cos(phi);
  lmin = q + 2.0 * pp * cos(phi + 2.0943951023931957);  // + 2 pi / 3
}

unsigned grid_for(int64_t n, int64_t per_block, unsigned cap) {
  int64_t g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

// ---------------------------------------------------------------- run building

// Run detection in tiles of kTile samples, one wavefront per tile, 64
// samples at a time.  Sample t starts a run when its pixel is valid and it is
// the first sample of its baseline or follows a sample on another pixel (or
// a masked one), or when t is a multiple of the split length (a power of two
// chosen so that a compact pixel id or a baseline index and the run length
// fit one 32-bit key; no split when whole baselines fit).  A run ends before
// the next start, at the end of its baseline or at the first sample off its
// pixel.  Splitting a run changes no sum, only how it is grouped.
constexpr int64_t kTile = 4096;
constexpr int kChunks = 4;  // 64-sample chunks whose loads are issued together

// Pixels of kChunks consecutive 64-sample chunks from c0 (lane = sample),
// each sample's predecessor, and the run-start flags; samples at or past z
// read as masked.  Sample indices are below 2^32.
struct ChunkHeads {
  int p[kChunks];
  uint64_t head[kChunks];
};
__device__ __forceinline__ void chunk_heads(const int32_t* __restrict__ pix, int64_t c0, int64_t z, int64_t n_pix,
                                            uint32_t L, uint32_t smask, ChunkHeads& o) {
  const int lane = lane_id();
#pragma unroll
  for (int k = 0; k < kChunks; ++k) {
    const int64_t t = c0 + 64 * k + lane;
    o.p[k] = t < z ? pix[t] : -1;
  }
  const int before = (lane == 0 && c0 > 0) ? pix[c0 - 1] : -1;  // the sample before the first chunk
#pragma unroll
  for (int k = 0; k < kChunks; ++k) {
    const int64_t t = c0 + 64 * k + lane;
    // both shuffles run on every lane (a lane reading an inactive lane gets no data)
    const int up = __shfl_up(o.p[k], 1, 64);
    const int last = k == 0 ? before : __shfl(o.p[k > 0 ? k - 1 : 0], 63, 64);
    const int prev = lane == 0 ? last : up;
    const int p = o.p[k];
    const bool on = t < z && p >= 0 && p < n_pix;
    o.head[k] = __ballot(on && (((uint32_t)t % L) == 0u || ((uint32_t)t & smask) == 0u || prev != p));
  }
}

// Per tile: number of run starts; samples off the map (masked or out of
// range) are counted into n_out, indices >= n_pix raise err.
__global__ void __launch_bounds__(kBlock) k_tile_heads(const int32_t* __restrict__ pix, int64_t n_t, int64_t n_pix,
                                                       int64_t L, uint32_t smask, int64_t n_tiles,
                                                       uint32_t* __restrict__ tcount,
                                                       int* __restrict__ err, unsigned long long* __restrict__ n_out) {
  const int lane = lane_id();
  const int64_t nw = (int64_t)gridDim.x * kWaves;
  for (int64_t tile = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); tile < n_tiles; tile += nw) {
    const int64_t a = tile * kTile, z = min(n_t, a + kTile);
    uint32_t cnt = 0, out = 0;
    bool bad = false;
    for (int64_t c0 = a; c0 < z; c0 += 64 * kChunks) {
      ChunkHeads h;
      chunk_heads(pix, c0, z, n_pix, (uint32_t)L, smask, h);
#pragma unroll
      for (int k = 0; k < kChunks; ++k) {
        const bool in = c0 + 64 * k + lane < z;
        bad |= in && h.p[k] >= n_pix;
        cnt += (uint32_t)__popcll(h.head[k]);
        out += (uint32_t)__popcll(__ballot(in && (h.p[k] < 0 || h.p[k] >= n_pix)));
      }
    }
    if (__ballot(bad) != 0ull && lane == 0) atomicOr(err, 1);
    if (lane == 0) {
      tcount[tile] = cnt;
      if (out) atomicAdd(n_out, (unsigned long long)out);
    }
  }
}

// First sample of each run (t0, time order) and the first run of each
// baseline (bstart); toff = exclusive scan of the tile counts, R runs in all.
// skey / sval: each run's pixel and index, the input of the sort by pixel.
__global__ void __launch_bounds__(kBlock) k_tile_starts(const int32_t* __restrict__ pix, int64_t n_t, int64_t n_pix,
                                                        int64_t L, uint32_t smask, int64_t n_b, int64_t n_tiles,
                                                        const uint32_t* __restrict__ toff, uint32_t R,
                                                        uint32_t* __restrict__ t0, uint32_t* __restrict__ bstart,
                                                        uint32_t* __restrict__ skey, uint32_t* __restrict__ sval) {
  const int lane = lane_id();
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));  // lanes below this one
  const int64_t nw = (int64_t)gridDim.x * kWaves;
  for (int64_t tile = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); tile < n_tiles; tile += nw) {
    const int64_t a = tile * kTile, z = min(n_t, a + kTile);
    uint32_t run = toff[tile];
    for (int64_t c0 = a; c0 < z; c0 += 64 * kChunks) {
      ChunkHeads h;
      chunk_heads(pix, c0, z, n_pix, (uint32_t)L, smask, h);
#pragma unroll
      for (int k = 0; k < kChunks; ++k) {
        const int64_t t = c0 + 64 * k + lane;
        const uint32_t idx = run + (uint32_t)__popcll(h.head[k] & lt);
        if ((h.head[k] >> lane) & 1ull) {
          t0[idx] = (uint32_t)t;
          skey[idx] = (uint32_t)h.p[k];  // the run's pixel and index: the sort's input
          sval[idx] = idx;
        }
        if (t < z && ((uint32_t)t % (uint32_t)L) == 0u) bstart[(uint32_t)t / (uint32_t)L] = idx;
        run += (uint32_t)__popcll(h.head[k]);
      }
    }
    if (tile == n_tiles - 1 && lane == 0) bstart[n_b] = R;
  }
}

// One thread per run: length, sums of cos 2psi and sin 2psi, and the setup
// sums.  Time-order outputs feed the rescan and the right-hand side (pixel,
// length, C, S, and per baseline and 64-run window the sums of d_T, d_q,
// d_u); a 64-byte record per run
// feeds the per-pixel setup, which reads it in pixel order with one aligned
// access.  Samples are summed in time order.  A wavefront takes 64
// consecutive runs; when the samples they span fit kStage, the wavefront
// first copies them (angles and timelines) into LDS with coalesced loads and
// each lane then reads its run from there.
constexpr int kStage = 256;
// Runs per wavefront of the run build: windows [k kRunWindow, (k + 1) kRunWindow)
// of the time-order runs, whose per-baseline sums of d the right-hand side reads.
constexpr int kRunWindow = 64;

template <typename PT, typename TT, typename RT, bool HAS_T, bool HAS_QU, bool IQU, bool TOD>
__global__ void __launch_bounds__(kBlock) k_run_build(View v, const TT* __restrict__ tod,
                                                      const uint32_t* __restrict__ t0,
                                                      const unsigned long long* __restrict__ n_out, int64_t R,
                                                      int32_t* __restrict__ rpix, int32_t* __restrict__ rn,
                                                      RT* __restrict__ rcs, double* __restrict__ raw,
                                                      RunRecord* __restrict__ rec) {
  constexpr bool SA = HAS_QU || IQU;                 // angles used
  constexpr bool TONLY = HAS_T && !HAS_QU && !IQU;   // intensity only: 16-byte records
  constexpr bool ST = TOD && (HAS_T || IQU);         // T (or radiometer) timeline used
  constexpr bool SQ = TOD && HAS_QU && !IQU;         // q/u timelines used
  constexpr int NROW = (ST ? 1 : 0) + (SQ ? 2 : 0);
  __shared__ PT s_psi[SA ? kWaves : 1][SA ? kStage : 1];
  __shared__ TT s_tod[NROW > 0 ? kWaves : 1][NROW > 0 ? NROW : 1][NROW > 0 ? kStage : 1];
  const PT* psi = static_cast<const PT*>(v.psi);
  const int64_t n_t = v.n_t;
  const int lane = lane_id();
  const int wave = threadIdx.x >> 6;
  constexpr int iT = 0, iQ = ST ? 1 : 0, iU = iQ + 1;
  constexpr int U = 2;  // samples whose loads are issued together (direct path)
  const bool gaps = *n_out != 0;
  static_assert(kRunWindow == 64, "one run per lane");
  for (int64_t rb = ((int64_t)blockIdx.x * kWaves + wave) * kRunWindow; rb < R;
       rb += (int64_t)gridDim.x * kWaves * kRunWindow) {
    const int64_t r = rb + lane;
    const bool has = r < R;
    int64_t ts = 0, te = 0;
    if (has) {
      ts = t0[r];
      // a run ends at the next run's start, the end of its baseline, or (with
      // masked samples in the timeline) the first sample off its pixel
      te = r + 1 < R ? (int64_t)t0[r + 1] : n_t;
      te = min(te, (ts / v.L + 1) * v.L);
      if (gaps) {
        const int p = v.pix[ts];
        int64_t t = ts + 1;
        while (t < te && v.pix[t] == p) ++t;
        te = t;
      }
    }
    const int32_t n = (int32_t)(te - ts);
    // samples spanned by the wavefront's runs (lane 0 always holds one)
    const int last = R - 1 - rb < 63 ? (int)(R - 1 - rb) : 63;
    const int64_t lo = __shfl(ts, 0, 64), hi = __shfl(te, last, 64);
    const bool staged = hi - lo <= kStage;
    if (staged) {
      // the span's angles and timelines go straight into LDS, every row in
      // flight at once (LDS-direct loads: no registers)
      const int span = (int)(hi - lo);
      if (SA) dev::lds_copy_words(psi + lo, &s_psi[SA ? wave : 0][0], span * (int)sizeof(PT) / 4);
      const int nw = span * (int)sizeof(TT) / 4;
      if (ST) dev::lds_copy_words(tod + v.rowT * n_t + lo, &s_tod[wave][iT][0], nw);
      if (SQ) {
        dev::lds_copy_words(tod + v.rowQ * n_t + lo, &s_tod[wave][iQ][0], nw);
        dev::lds_copy_words(tod + v.rowU * n_t + lo, &s_tod[wave][SQ ? iU : 0][0], nw);
      }
      dev::lds_copy_wait();
    }
    double C = 0.0, S = 0.0, cc = 0.0, cs = 0.0;
    double dT = 0.0, dq = 0.0, du = 0.0, dQ = 0.0, dU = 0.0;
    // one sample: angle and timeline values in, the run's sums updated
    auto take = [&](double ps, double xT, double xq, double xu) {
      double c = 1.0, s = 0.0;
      if (SA) {
        rot2(ps, c, s);
        C += c;
        S += s;
        cc += c * c;
        cs += c * s;
      }
      if (TOD && IQU) {
        // radiometer row (1, c, s): sums of d and of the weighted c d, s d
        const double wx = v.w[0] * xT;
        dT += xT;
        dQ += c * wx;
        dU += s * wx;
      } else if (TOD) {
        if (HAS_T) dT += xT;
        if (HAS_QU) {
          dq += xq;
          du += xu;
          const double wq = v.w[1] * xq, wu = v.w[2] * xu;
          dQ += c * wq - s * wu;
          dU += s * wq + c * wu;
        }
      }
    };
    if (staged) {
      const int i0 = (int)(ts - lo);
#pragma unroll 1
      for (int k = 0; k < n; ++k) {
        const int i = i0 + k;
        take(SA ? (double)s_psi[SA ? wave : 0][SA ? i : 0] : 0.0,
             ST ? (double)s_tod[NROW > 0 ? wave : 0][0][NROW > 0 ? i : 0] : 0.0,
             SQ ? (double)s_tod[wave][iQ][i] : 0.0, SQ ? (double)s_tod[wave][SQ ? iU : 0][i] : 0.0);
      }
    } else {
      for (int k0 = 0; k0 < n; k0 += U) {
        double ps_[U], xT[U], xq[U], xu[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t t = ts + k0 + u;
          const bool in = k0 + u < n;
          ps_[u] = (SA && in) ? (double)psi[t] : 0.0;
          xT[u] = (ST && in) ? (double)tod[v.rowT * n_t + t] : 0.0;
          xq[u] = (SQ && in) ? (double)tod[v.rowQ * n_t + t] : 0.0;
          xu[u] = (SQ && in) ? (double)tod[v.rowU * n_t + t] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (k0 + u >= n) break;
          take(ps_[u], xT[u], xq[u], xu[u]);
        }
      }
    }
    if (staged) __builtin_amdgcn_wave_barrier();  // reads done before the next stage overwrites
    if (TOD) {
      // sums of d over the wavefront's runs of each baseline (the data part
      // of b = F^T Z d before the invalid pixels' runs are taken out): a scan
      // inside each stretch of lanes with the same baseline; the stretch's
      // last lane stores it at its run, so that raw holds, at every run that
      // ends a baseline or a 64-run window, the sum over that baseline's runs
      // in the window (the other entries are never read)
      const int bl = has ? (int)(ts / v.L) : -1 - lane;
      double s0 = dT, s1 = dq, s2 = du;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int bo = __shfl_up(bl, off, 64);
        const double a0 = __shfl_up(s0, off, 64);
        const double a1 = TONLY ? 0.0 : __shfl_up(s1, off, 64);
        const double a2 = TONLY ? 0.0 : __shfl_up(s2, off, 64);
        if (lane >= off && bo == bl) {
          s0 += a0;
          s1 += a1;
          s2 += a2;
        }
      }
      const int bn = __shfl_down(bl, 1, 64);
      if (has && (lane == kRunWindow - 1 || bn != bl)) {
        if (TONLY) {
          raw[r] = s0;
        } else {
          raw[3 * r + 0] = s0;
          raw[3 * r + 1] = s1;
          raw[3 * r + 2] = s2;
        }
      }
    }
    if (!has) continue;
    rpix[r] = v.pix[ts];
    rn[r] = n;
    if (SA) reinterpret_cast<CS2<RT>*>(rcs)[r] = make_cs<RT>(C, S);
    if (TONLY) {
      RunRecordT x;
      x.n = n;
      x.b = (int32_t)(ts / v.L);
      x.dT = dT;
      reinterpret_cast<RunRecordT*>(rec)[r] = x;
      continue;
    }
    RunRecord x;
    x.n = n;
    x.b = (int32_t)(ts / v.L);
    x.C = C;
    x.S = S;
    x.cc = cc;
    x.cs = cs;
    x.dT = dT;
    x.dQ = dQ;
    x.dU = dU;
    rec[r] = x;
  }
}

// seg[2k], seg[2k+1]: range of key k in the sorted key array.  Four keys
// per thread, loaded together.
__global__ void __launch_bounds__(kBlock) k_key_segments(const uint32_t* __restrict__ keys, int64_t n,
                                                         int64_t* __restrict__ seg) {
  const int64_t nq = (n + 3) / 4;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j0 = 4 * q;
    uint32_t k[6];  // keys j0 - 1 .. j0 + 4; absent neighbours differ from every key
    if (j0 + 4 <= n) {
      const uint4 x = reinterpret_cast<const uint4*>(keys)[q];
      k[1] = x.x;
      k[2] = x.y;
      k[3] = x.z;
      k[4] = x.w;
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) k[1 + i] = j0 + i < n ? keys[j0 + i] : 0u;
    }
    k[0] = j0 > 0 ? keys[j0 - 1] : ~k[1];
    k[5] = j0 + 4 < n ? keys[j0 + 4] : ~k[4];
#pragma unroll
    for (int i = 1; i <= 4; ++i) {
      const int64_t j = j0 + i - 1;
      if (j >= n) break;
      const uint32_t nx = j == n - 1 ? ~k[i] : k[i + 1];
      if (k[i - 1] != k[i]) seg[2 * (int64_t)k[i]] = j;
      if (nx != k[i]) seg[2 * (int64_t)k[i] + 1] = j + 1;
    }
  }
}

// First visit of each pixel (start of its earliest run; the run sort is
// stable, so that run heads the pixel's segment); `none` (n_t, after every
// sample) if unobserved.
__global__ void __launch_bounds__(kBlock) k_first_visit(const int64_t* __restrict__ seg,
                                                        const uint32_t* __restrict__ rperm,
                                                        const uint32_t* __restrict__ t0, int64_t n_pix,
                                                        uint32_t none, uint32_t* __restrict__ first,
                                                        uint32_t* __restrict__ pidx,
                                                        unsigned long long* __restrict__ n_obs) {
  __shared__ unsigned long long lds[16];
  unsigned long long cnt[1] = {0};
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n_pix; p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j0 = seg[2 * p], j1 = seg[2 * p + 1];
    const bool hit = j1 > j0;
    first[p] = hit ? t0[rperm[j0]] : none;
    pidx[p] = (uint32_t)p;
    cnt[0] += hit;
  }
  block_sum<1>(cnt, lds);
  if (threadIdx.x == 0) atomicAdd(n_obs, cnt[0]);
}

// Compact ids in order of first visit (pixels a stretch of the scan touches
// get neighbouring ids), and run counts per compact pixel.
__global__ void __launch_bounds__(kBlock) k_compact(const uint32_t* __restrict__ order, int64_t n_obs,
                                                    const int64_t* __restrict__ seg, int32_t* __restrict__ cid,
                                                    int64_t* __restrict__ ccount) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c <= n_obs; c += (int64_t)gridDim.x * blockDim.x) {
    if (c == n_obs) {
      ccount[c] = 0;
      continue;
    }
    const uint32_t p = order[c];
    cid[p] = (int32_t)c;
    ccount[c] = seg[2 * (int64_t)p + 1] - seg[2 * (int64_t)p];
  }
}

// 32 lanes per compact pixel: its runs (pixel order, time order within
// the pixel) -> the pixel-order run arrays; hits, weight blocks, inverse,
// validity; with TOD the sum map and binned map.  The sum of sin^2 2psi over
// a run is its length minus the sum of cos^2 2psi.
template <typename RT, bool HAS_T, bool HAS_QU, bool IQU, bool TOD>
__global__ void __launch_bounds__(kBlock) k_pixels_from_runs(
    View v, int64_t n_obs, const uint32_t* __restrict__ order, const int64_t* __restrict__ seg,
    const uint32_t* __restrict__ rperm, const RunRecord* __restrict__ rec, double rcond_cut,
    int32_t* __restrict__ pb, int32_t* __restrict__ pn, int nb, uint32_t* __restrict__ pkey, RT* __restrict__ pcs,
    const int64_t* __restrict__ pstart, int32_t* __restrict__ hits, double* __restrict__ Minv4,
    uint8_t* __restrict__ valid, double* __restrict__ m4_zero, double* __restrict__ sd4, double* __restrict__ md4,
    unsigned long long* __restrict__ counts) {
  constexpr bool TONLY = HAS_T && !HAS_QU && !IQU;  // 16-byte records
  __shared__ unsigned long long lds[4 * 16];
  unsigned long long cnt[4] = {0, 0, 0, 0};
  // LPP lanes per pixel (two pixels per wavefront), U runs per lane and step
  constexpr int LPP = 32, PPW = 64 / LPP, U = 4;
  const int lane = lane_id();
  const int grp = lane / LPP, sub = lane % LPP;
  const int64_t nw = (int64_t)gridDim.x * kWaves * PPW;
  for (int64_t cb = ((int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6)) * PPW; cb < n_obs; cb += nw) {
    const int64_t c = cb + grp;
    const bool have = c < n_obs;
    int64_t j0 = 0, j1 = 0, d0 = 0;
    if (have) {
      const uint32_t p = order[c];
      j0 = seg[2 * (int64_t)p];
      j1 = seg[2 * (int64_t)p + 1];
      d0 = pstart[c];
    }
    constexpr int NA = IQU ? 8 : 6;
    double acc[NA];  // h, cc, cs, dT, dQ, dU (and C, S for the radiometer block)
#pragma unroll
    for (int i = 0; i < NA; ++i) acc[i] = 0.0;
    for (int64_t jb = j0 + sub; jb < j1; jb += LPP * U) {
      uint32_t q[U];
#pragma unroll
      for (int u = 0; u < U; ++u) q[u] = jb + LPP * u < j1 ? rperm[jb + LPP * u] : 0u;
      RunRecord xs[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (jb + LPP * u >= j1) continue;
        if (TONLY) {
          const RunRecordT y = reinterpret_cast<const RunRecordT*>(rec)[q[u]];
          xs[u].n = y.n;
          xs[u].b = y.b;
          xs[u].dT = y.dT;
        } else {
          xs[u] = rec[q[u]];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t j = jb + LPP * u;
        if (j >= j1) break;
        const RunRecord& x = xs[u];
        const int64_t d = d0 + (j - j0);
        pb[d] = x.b;
        pn[d] = x.n;
        if (nb > 0) pkey[d] = ((uint32_t)x.b << nb) | (uint32_t)(x.n - 1);
        acc[0] += (double)x.n;
        if (HAS_QU || IQU) {
          reinterpret_cast<CS2<RT>*>(pcs)[d] = make_cs<RT>(x.C, x.S);
          acc[1] += x.cc;
          acc[2] += x.cs;
        }
        if (IQU) {
          acc[NA - 2] += x.C;
          acc[NA - 1] += x.S;
        }
        if (TOD) {
          acc[3] += x.dT;
          acc[4] += x.dQ;
          acc[5] += x.dU;
        }
      }
    }
#pragma unroll
    for (int off = LPP / 2; off > 0; off >>= 1) {
#pragma unroll
      for (int i = 0; i < NA; ++i) acc[i] += __shfl_xor(acc[i], off, 64);
    }
    if (IQU && have && sub == 0) {
      // full 3x3 block w [[h, C, S], [C, cc, cs], [S, cs, ss]] of the radiometer row
      const int64_t h = (int64_t)acc[0];
      const double w = v.w[0];
      const double a00 = w * acc[0], a01 = w * acc[NA - 2], a02 = w * acc[NA - 1];
      const double a11 = w * acc[1], a12 = w * acc[2], a22 = w * (acc[0] - acc[1]);
      double inv[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      uint8_t f = 0;
      if (h > 0) {
        double lmin, lmax;
        sym3_eig_range(a00, a01, a02, a11, a12, a22, lmin, lmax);
        if (lmax > 0.0 && lmin > 0.0 && lmin >= rcond_cut * lmax) {
          const double c00 = a11 * a22 - a12 * a12, c01 = a02 * a12 - a01 * a22, c02 = a01 * a12 - a02 * a11;
          const double c11 = a00 * a22 - a02 * a02, c12 = a01 * a02 - a00 * a12, c22 = a00 * a11 - a01 * a01;
          const double det = a00 * c00 + a01 * c01 + a02 * c02;
          if (det > 0.0) {
            f = 3;
            inv[0] = c00 / det;
            inv[1] = c01 / det;
            inv[2] = c02 / det;
            inv[3] = c11 / det;
            inv[4] = c12 / det;
            inv[5] = c22 / det;
          }
        }
      }
      hits[c] = (int32_t)h;
      double2* mi = reinterpret_cast<double2*>(Minv4 + 8 * c);
      mi[0] = make_double2(inv[0], inv[1]);
      mi[1] = make_double2(inv[2], inv[3]);
      mi[2] = make_double2(inv[4], inv[5]);
      mi[3] = make_double2(0.0, 0.0);
      valid[c] = f;
      double2* mz = reinterpret_cast<double2*>(m4_zero + 4 * c);
      mz[0] = make_double2(0.0, 0.0);
      mz[1] = make_double2(0.0, 0.0);
      if (TOD) {
        const double sI = f ? w * acc[3] : 0.0, sQ = f ? acc[4] : 0.0, sU = f ? acc[5] : 0.0;
        double2* sp = reinterpret_cast<double2*>(sd4 + 4 * c);
        sp[0] = make_double2(sI, sQ);
        sp[1] = make_double2(sU, 0.0);
        double2* mp = reinterpret_cast<double2*>(md4 + 4 * c);
        mp[0] = make_double2(inv[0] * sI + inv[1] * sQ + inv[2] * sU, inv[1] * sI + inv[3] * sQ + inv[4] * sU);
        mp[1] = make_double2(inv[2] * sI + inv[4] * sQ + inv[5] * sU, 0.0);
      }
      cnt[0] += f ? 1 : 0;
      cnt[2] += f ? (unsigned long long)h : 0ull;
    }
    if (!IQU && have && sub == 0) {
      const int64_t h = (int64_t)acc[0];
      double inv[4] = {0.0, 0.0, 0.0, 0.0};
      uint8_t f = 0;
      if (HAS_T && h > 0) {
        f |= 1;
        inv[0] = 1.0 / (v.w[0] * (double)h);
      }
      if (HAS_QU && h > 0) {
        const double wq = v.w[1], wu = v.w[2];
        const double scc = acc[1], sss = acc[0] - acc[1];
        const double a = wq * scc + wu * sss;
        const double b = (wq - wu) * acc[2];
        const double d = wq * sss + wu * scc;
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

// One wavefront per baseline: its time-order runs take compact pixel ids
// (pixel -> cid) and, with nb > 0, the packed iteration keys
// c << nb | (length - 1); key[b] = the smallest compact id the baseline
// visits (n_obs when none), which orders baselines for the rescan;
// val[b] = b.
__global__ void __launch_bounds__(kBlock) k_compact_baselines(int64_t n_b, int64_t n_obs, int nb,
                                                              const uint32_t* __restrict__ bstart,
                                                              const int32_t* __restrict__ cid,
                                                              int32_t* __restrict__ tpix,
                                                              const int32_t* __restrict__ tn,
                                                              uint32_t* __restrict__ tkey, uint32_t* __restrict__ key,
                                                              uint32_t* __restrict__ val) {
  constexpr int U = 4;  // runs per lane whose loads are issued together
  const int lane = lane_id();
  const int64_t nw = (int64_t)gridDim.x * kWaves;
  for (int64_t b = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); b < n_b; b += nw) {
    uint32_t m = (uint32_t)n_obs;
    const int64_t r0 = bstart[b], r1 = bstart[b + 1];
    for (int64_t rb = r0 + lane; rb < r1; rb += 64 * U) {
      int32_t p[U], len[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t r = rb + 64 * u;
        p[u] = r < r1 ? tpix[r] : 0;
        len[u] = (nb > 0 && r < r1) ? tn[r] : 1;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t r = rb + 64 * u;
        if (r >= r1) break;
        const int32_t c = cid[p[u]];
        tpix[r] = c;
        if (nb > 0) tkey[r] = ((uint32_t)c << nb) | (uint32_t)(len[u] - 1);
        m = min(m, (uint32_t)c);
      }
    }
    for (int off = 32; off > 0; off >>= 1) m = min(m, (uint32_t)__shfl_xor((int)m, off, 64));
    if (lane == 0) {
      key[b] = m;
      val[b] = (uint32_t)b;
    }
  }
}

// Per baseline (time-order runs): n_valid, the Jacobi diagonal and with TOD
//   b_k = w_k sum_{runs, valid_k} (sum of d_k over the run - A-weighted m_d).
// The sums of d come from the run build's per-window sums (all runs of the
// baseline) less the runs on pixels not valid for stream k, whose samples are
// read again here.  The rescan's layout: 16 lanes per baseline, four
// baselines per wavefront in the rescan order, the loads of four runs per
// lane issued together.
template <typename RT, typename TT, bool HAS_T, bool HAS_QU, bool IQU, bool TOD, bool PK>
__global__ void __launch_bounds__(kBlock) k_rhs_runs(View v, const uint32_t* __restrict__ bstart,
                                                     const uint32_t* __restrict__ border,
                                                     const uint32_t* __restrict__ rkey,
                                                     const int32_t* __restrict__ rn, int nb,
                                                     const RT* __restrict__ rcs,
                                                     const double* __restrict__ raw, const double* __restrict__ md4,
                                                     const TT* __restrict__ tod, const uint32_t* __restrict__ t0,
                                                     const uint8_t* __restrict__ valid, int32_t* __restrict__ nvalid,
                                                     double* __restrict__ J, double* __restrict__ b_out) {
  constexpr int BPW = 4, SEG = 64 / BPW;
  const int lane = lane_id();
  const int64_t n_b = v.n_b;
  const int64_t n_g = ((n_b + BPW - 1) / BPW + kWaves - 1) / kWaves;
  const int64_t per = (n_g + 7) / 8;
  const int64_t gi = blockIdx.x;
  const int64_t g = (gi & 7) * per + (gi >> 3);
  if (g >= n_g) return;  // whole workgroup
  const int sl = lane % SEG;
  const int64_t k = (g * kWaves + (threadIdx.x >> 6)) * BPW + lane / SEG;
  const int64_t b = k < n_b ? (int64_t)border[k] : n_b;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // T, q, u residual sums; n_T, n_QU
  if (b < n_b) {
    const int64_t r0 = bstart[b], r1 = bstart[b + 1];
    constexpr int U = 4;
    for (int64_t rb = r0 + sl; rb < r1; rb += SEG * U) {
      int c[U], nn[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t r = rb + SEG * u;
        const bool in = r < r1;
        const uint32_t key = in ? rkey[r] : 0u;
        // packed keys (PK): compact pixel << nb | (length - 1); else pixel, lengths in rn
        c[u] = in ? (int)(PK ? key >> nb : key) : -1;
        nn[u] = in ? (PK ? (int)(key & ((1u << nb) - 1u)) + 1 : rn[r]) : 0;
      }
      uint8_t f[U];
      double2 m01[U];
      double m2x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        f[u] = 0;
        m01[u] = make_double2(0.0, 0.0);
        m2x[u] = 0.0;
        if (c[u] < 0) continue;
        f[u] = valid[c[u]];
        if (TOD) {
          const double2* mp = reinterpret_cast<const double2*>(md4 + 4 * (int64_t)c[u]);
          m01[u] = mp[0];
          m2x[u] = mp[1].x;
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (c[u] < 0) continue;
        const int64_t r = rb + SEG * u;
        const double n = (double)nn[u];
        constexpr int RW = HAS_T && !HAS_QU && !IQU ? 1 : 3;  // raw sums per run
        if (TOD && (r % kRunWindow == kRunWindow - 1 || r == r1 - 1)) {
          // the run ends the baseline or a 64-run window: raw holds the sums
          // of d over the baseline's runs in that window
          if (HAS_T || IQU) acc[0] += raw[RW * r];
          if (HAS_QU && !IQU) {
            acc[1] += raw[RW * r + 1];
            acc[2] += raw[RW * r + 2];
          }
        }
        const bool tin = (HAS_T || IQU) && !(f[u] & 1), qin = HAS_QU && !IQU && !(f[u] & 2);
        if (TOD && (tin || qin)) {
          // a run on a pixel left out of the map (for T or for q/u): its own
          // sums of d come out of the baseline's data part again
          const int64_t ts = t0[r];
          double sT = 0.0, sq = 0.0, su = 0.0;
          for (int k = 0; k < nn[u]; ++k) {
            if (tin) sT += (double)tod[v.rowT * v.n_t + ts + k];
            if (qin) {
              sq += (double)tod[v.rowQ * v.n_t + ts + k];
              su += (double)tod[v.rowU * v.n_t + ts + k];
            }
          }
          acc[0] -= sT;
          acc[1] -= sq;
          acc[2] -= su;
        }
        if (IQU && (f[u] & 1)) {
          acc[3] += n;
          if (TOD) {
            const CS2<RT> cs = reinterpret_cast<const CS2<RT>*>(rcs)[r];
            const double C = (double)cs.x, S = (double)cs.y;
            acc[0] -= n * m01[u].x + C * m01[u].y + S * m2x[u];
          }
        } else if (HAS_T && (f[u] & 1)) {
          acc[3] += n;
          if (TOD) acc[0] -= n * m01[u].x;
        }
        if (HAS_QU && (f[u] & 2)) {
          acc[4] += n;
          if (TOD) {
            const CS2<RT> cs = reinterpret_cast<const CS2<RT>*>(rcs)[r];
            const double C = (double)cs.x, S = (double)cs.y;
            const double mQ = m01[u].y, mU = m2x[u];
            acc[1] -= C * mQ + S * mU;
            acc[2] -= C * mU - S * mQ;
          }
        }
      }
    }
  }
#pragma unroll
  for (int off = SEG / 2; off > 0; off >>= 1) {
#pragma unroll
    for (int i = 0; i < 5; ++i) acc[i] += __shfl_xor(acc[i], off, 64);
  }
  if (sl == 0 && b < n_b) {
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

// Run stream of U runs j, j + stride, ... (key, length, and the interleaved
// pair of sums of cos 2psi and sin 2psi, one load).  Every load is issued, with index 0 for runs at or past j1, so
// the loads of all U runs are in flight together with no branches between
// them; the caller zeroes those runs' terms.  PK: packed keys (index << nb |
// length - 1), else index keys with the lengths in len_arr.
template <typename RT, bool LEN, bool ANG, bool PK, int U>
__device__ __forceinline__ void load_runs(const uint32_t* __restrict__ key_arr, const int32_t* __restrict__ len_arr,
                                          const RT* __restrict__ cs_arr, int64_t j,
                                          int64_t stride, int64_t j1, uint32_t (&key)[U], int32_t (&len)[U],
                                          RT (&C)[U], RT (&S)[U]) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t jj = j + stride * u < j1 ? j + stride * u : 0;
    key[u] = key_arr[jj];
    len[u] = (LEN && !PK) ? len_arr[jj] : 0;
    const CS2<RT> cs = ANG ? reinterpret_cast<const CS2<RT>*>(cs_arr)[jj] : make_cs<RT>(0.0, 0.0);
    C[u] = cs.x;
    S[u] = cs.y;
  }
}

// Index, length and angle sums of a loaded run; zero terms past j1.
template <typename RT, bool PK>
__device__ __forceinline__ void decode_run(uint32_t key, int32_t len, RT c, RT s, bool in, int nb, int32_t& idx,
                                           double& n, double& C, double& S) {
  idx = (int32_t)(PK ? key >> nb : key);
  n = in ? (double)(PK ? (int32_t)(key & ((1u << nb) - 1u)) + 1 : len) : 0.0;
  C = in ? (double)c : 0.0;
  S = in ? (double)s : 0.0;
}

// m = M^-1 A^T W F p per compact pixel from its pixel-order runs.  LPP lanes
// work on one pixel (64 / LPP pixels per wavefront, each with its own chain of
// dependent loads in flight); pw4[b] = (w_T p_T, w_q p_q, w_u p_u, 0).
// The body takes the workgroup's place (vblock of vgrid) in its problem's grid.
template <typename RT, bool HAS_T, bool HAS_QU, bool IQU, int LPP, bool PK>
__device__ __forceinline__ void bin_runs_body(int64_t n_obs, const int64_t* __restrict__ pstart,
                                              const uint32_t* __restrict__ pb, const int32_t* __restrict__ pn,
                                              int nb, const RT* __restrict__ pcs, const double* __restrict__ pw4,
                                              const double* __restrict__ Minv4, const uint8_t* __restrict__ valid,
                                              double* __restrict__ m4, int64_t vblock, int64_t vgrid) {
  constexpr int PPW = 64 / LPP;
  constexpr int U = LPP >= 64 ? 2 : (LPP == 32 ? 4 : 8);
  // intensity-only problems keep p and m as one double per baseline / pixel
  constexpr bool TONLY = HAS_T && !HAS_QU && !IQU;
  const int lane = lane_id();
  const int grp = lane / LPP, sub = lane % LPP;
  const int64_t step = vgrid * kWaves * PPW;
  for (int64_t cb = (vblock * kWaves + (threadIdx.x >> 6)) * PPW; cb < n_obs; cb += step) {
    const int64_t c = cb + grp;
    const bool have = c < n_obs && valid[c] != 0;  // m stays 0 on invalid pixels
    int64_t j0 = 0, j1 = 0;
    if (have) {
      j0 = pstart[c];
      j1 = pstart[c + 1];
    }
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t jb = j0 + sub; jb < j1; jb += LPP * U) {
      uint32_t key[U];
      int32_t len[U];
      RT cr[U], sr[U];
      // packed keys (PK): baseline << nb | (length - 1); else baseline, lengths in pn
      load_runs<RT, HAS_T, HAS_QU || IQU, PK, U>(pb, pn, pcs, jb, LPP, j1, key, len, cr, sr);
      double2 x0[U];
      double u0[U], nn[U], cc[U], ss[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        int32_t bb;
        decode_run<RT, PK>(key[u], len[u], cr[u], sr[u], jb + LPP * u < j1, nb, bb, nn[u], cc[u], ss[u]);
        // runs past j1 read baseline pw4 of run 0 (a valid index) and add nothing
        if (TONLY) {
          x0[u] = make_double2(pw4[bb], 0.0);
          u0[u] = 0.0;
        } else {
          const double2* q0 = reinterpret_cast<const double2*>(pw4 + 4 * (int64_t)bb);
          x0[u] = q0[0];
          u0[u] = HAS_QU ? q0[1].x : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (IQU) {
          acc[0] += nn[u] * x0[u].x;
          acc[1] += cc[u] * x0[u].x;
          acc[2] += ss[u] * x0[u].x;
          continue;
        }
        if (HAS_T) acc[0] += nn[u] * x0[u].x;
        if (HAS_QU) {
          acc[1] += cc[u] * x0[u].y - ss[u] * u0[u];
          acc[2] += ss[u] * x0[u].y + cc[u] * u0[u];
        }
      }
    }
#pragma unroll
    for (int off = LPP / 2; off > 0; off >>= 1) {
#pragma unroll
      for (int i = 0; i < 3; ++i) acc[i] += __shfl_xor(acc[i], off, 64);
    }
    if (IQU && have && sub == 0) {
      const double2* ip = reinterpret_cast<const double2*>(Minv4 + 8 * c);
      const double2 i01 = ip[0], i23 = ip[1], i45 = ip[2];  // (00, 01), (02, 11), (12, 22)
      double2* mp = reinterpret_cast<double2*>(m4 + 4 * c);
      mp[0] = make_double2(i01.x * acc[0] + i01.y * acc[1] + i23.x * acc[2],
                           i01.y * acc[0] + i23.y * acc[1] + i45.x * acc[2]);
      mp[1] = make_double2(i23.x * acc[0] + i45.x * acc[1] + i45.y * acc[2], 0.0);
    }
    if (TONLY && have && sub == 0) m4[c] = Minv4[4 * c] * acc[0];
    if (!IQU && !TONLY && have && sub == 0) {
      const double2* ip = reinterpret_cast<const double2*>(Minv4 + 4 * c);
      const double2 i01 = ip[0], i23 = ip[1];
      double2* mp = reinterpret_cast<double2*>(m4 + 4 * c);
      mp[0] = make_double2(i01.x * acc[0], i01.y * acc[1] + i23.x * acc[2]);
      mp[1] = make_double2(i23.x * acc[1] + i23.y * acc[2], 0.0);
    }
  }
}

template <typename RT, bool HAS_T, bool HAS_QU, bool IQU, int LPP, bool PK>
__global__ void __launch_bounds__(kBlock) k_bin_runs(int64_t n_obs, const int64_t* __restrict__ pstart,
                                                     const uint32_t* __restrict__ pb, const int32_t* __restrict__ pn,
                                                     int nb,
                                                     const RT* __restrict__ pcs,
                                                     const double* __restrict__ pw4,
                                                     const double* __restrict__ Minv4,
                                                     const uint8_t* __restrict__ valid, double* __restrict__ m4,
                                                     const CgCtl* __restrict__ gate) {
  if (gate && gate->done) return;
  bin_runs_body<RT, HAS_T, HAS_QU, IQU, LPP, PK>(n_obs, pstart, pb, pn, nb, pcs, pw4, Minv4, valid, m4, blockIdx.x,
                                                  gridDim.x);
}

// The same binning with a three-stage software pipeline over the
// wavefront's pixels (launch shape -LPP): while the baseline values of one
// pixel's first LPP * U runs are gathered, the run stream of its next pixel
// and the run range of the one after are loaded.  More registers, so fewer
// wavefronts: measured slower than the plain kernel at 32 lanes per pixel in
// both precisions, kept as a launch shape for the autotuner.
template <typename RT, bool HAS_T, bool HAS_QU, bool IQU, int LPP>
__global__ void __launch_bounds__(kBlock) k_bin_runs_pipe(int64_t n_obs, const int64_t* __restrict__ pstart,
                                                          const uint32_t* __restrict__ pb,
                                                          const int32_t* __restrict__ pn, int nb,
                                                          const RT* __restrict__ pcs,
                                                          const double* __restrict__ pw4,
                                                          const double* __restrict__ Minv4,
                                                          const uint8_t* __restrict__ valid, double* __restrict__ m4,
                                                          const CgCtl* __restrict__ gate) {
  if (gate && gate->done) return;
  constexpr int PPW = 64 / LPP;
  constexpr int U = LPP >= 64 ? 2 : (LPP == 32 ? 4 : 8);
  const int lane = lane_id();
  const int grp = lane / LPP, sub = lane % LPP;
  const int64_t step = (int64_t)gridDim.x * kWaves * PPW;
  // run range of compact pixel cx; empty when invalid or past the end
  auto head = [&](int64_t cx, int64_t& j0x, int64_t& j1x) {
    const bool inr = cx < n_obs;
    const bool h = inr && valid[cx] != 0;  // m stays 0 on invalid pixels
    j0x = inr ? pstart[cx] : 0;
    const int64_t e = inr ? pstart[cx + 1] : 0;
    j1x = h ? e : j0x;
  };
  uint32_t nkey[U];
  int32_t nlen[U];
  RT nC[U], nS[U];
  auto fetch = [&](int64_t j0x, int64_t j1x) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t j = j0x + sub + LPP * u;
      const bool in = j < j1x;
      nkey[u] = in ? pb[j] : 0u;
      nlen[u] = (HAS_T && !nb && in) ? pn[j] : 0;
      const CS2<RT> cs = ((HAS_QU || IQU) && in) ? reinterpret_cast<const CS2<RT>*>(pcs)[j] : make_cs<RT>(0.0, 0.0);
      nC[u] = cs.x;
      nS[u] = cs.y;
    }
  };
  int64_t cb = ((int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6)) * PPW;
  int64_t a0, a1, b0, b1;
  head(cb + grp, a0, a1);
  fetch(a0, a1);
  head(cb + step + grp, b0, b1);
  for (; cb < n_obs; cb += step) {
    const int64_t c = cb + grp;
    const int64_t j0 = a0, j1 = a1;
    const bool have = j1 > j0;  // valid observed pixels have runs; the range is empty otherwise
    int32_t bb[U], nn[U];
    double cc[U], ss[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool in = j0 + sub + LPP * u < j1;
      // packed keys (nb > 0): baseline << nb | (length - 1); else baseline, lengths in pn
      bb[u] = in ? (int32_t)(nb ? nkey[u] >> nb : nkey[u]) : -1;
      nn[u] = (HAS_T && in) ? (nb ? (int32_t)(nkey[u] & ((1u << nb) - 1u)) + 1 : nlen[u]) : 0;
      cc[u] = (double)nC[u];
      ss[u] = (double)nS[u];
    }
    double2 x0[U];
    double u0[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      x0[u] = make_double2(0.0, 0.0);
      u0[u] = 0.0;
      if (bb[u] < 0) continue;
      const double2* q0 = reinterpret_cast<const double2*>(pw4 + 4 * (int64_t)bb[u]);
      x0[u] = q0[0];
      if (HAS_QU) u0[u] = q0[1].x;
    }
    fetch(b0, b1);
    a0 = b0;
    a1 = b1;
    head(cb + 2 * step + grp, b0, b1);
    double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (IQU) {
        acc[0] += (double)nn[u] * x0[u].x;
        acc[1] += cc[u] * x0[u].x;
        acc[2] += ss[u] * x0[u].x;
        continue;
      }
      if (HAS_T) acc[0] += (double)nn[u] * x0[u].x;
      if (HAS_QU) {
        acc[1] += cc[u] * x0[u].y - ss[u] * u0[u];
        acc[2] += ss[u] * x0[u].y + cc[u] * u0[u];
      }
    }
    // runs past the first LPP * U of a long pixel, with the next step's run
    // stream loaded while this step's baseline values are gathered
    int64_t jb = j0 + sub + LPP * U;
    if (jb < j1) {
      uint32_t rkey[U];
      int32_t rlen[U];
      RT rC[U], rS[U];
      auto rfetch = [&](int64_t jx) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t j = jx + LPP * u;
          const bool in = j < j1;
          rkey[u] = in ? pb[j] : 0u;
          rlen[u] = (HAS_T && !nb && in) ? pn[j] : 0;
          const CS2<RT> cs =
              ((HAS_QU || IQU) && in) ? reinterpret_cast<const CS2<RT>*>(pcs)[j] : make_cs<RT>(0.0, 0.0);
          rC[u] = cs.x;
          rS[u] = cs.y;
        }
      };
      rfetch(jb);
      for (; jb < j1; jb += LPP * U) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const bool in = jb + LPP * u < j1;
          bb[u] = in ? (int32_t)(nb ? rkey[u] >> nb : rkey[u]) : -1;
          nn[u] = (HAS_T && in) ? (nb ? (int32_t)(rkey[u] & ((1u << nb) - 1u)) + 1 : rlen[u]) : 0;
          cc[u] = (double)rC[u];
          ss[u] = (double)rS[u];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          x0[u] = make_double2(0.0, 0.0);
          u0[u] = 0.0;
          if (bb[u] < 0) continue;
          const double2* q0 = reinterpret_cast<const double2*>(pw4 + 4 * (int64_t)bb[u]);
          x0[u] = q0[0];
          if (HAS_QU) u0[u] = q0[1].x;
        }
        rfetch(jb + LPP * U);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (IQU) {
            acc[0] += (double)nn[u] * x0[u].x;
            acc[1] += cc[u] * x0[u].x;
            acc[2] += ss[u] * x0[u].x;
            continue;
          }
          if (HAS_T) acc[0] += (double)nn[u] * x0[u].x;
          if (HAS_QU) {
            acc[1] += cc[u] * x0[u].y - ss[u] * u0[u];
            acc[2] += ss[u] * x0[u].y + cc[u] * u0[u];
          }
        }
      }
    }
#pragma unroll
    for (int off = LPP / 2; off > 0; off >>= 1) {
#pragma unroll
      for (int i = 0; i < 3; ++i) acc[i] += __shfl_xor(acc[i], off, 64);
    }
    if (IQU && have && sub == 0) {
      const double2* ip = reinterpret_cast<const double2*>(Minv4 + 8 * c);
      const double2 i01 = ip[0], i23 = ip[1], i45 = ip[2];  // (00, 01), (02, 11), (12, 22)
      double2* mp = reinterpret_cast<double2*>(m4 + 4 * c);
      mp[0] = make_double2(i01.x * acc[0] + i01.y * acc[1] + i23.x * acc[2],
                           i01.y * acc[0] + i23.y * acc[1] + i45.x * acc[2]);
      mp[1] = make_double2(i23.x * acc[0] + i45.x * acc[1] + i45.y * acc[2], 0.0);
    }
    if (!IQU && have && sub == 0) {
      const double2* ip = reinterpret_cast<const double2*>(Minv4 + 4 * c);
      const double2 i01 = ip[0], i23 = ip[1];
      double2* mp = reinterpret_cast<double2*>(m4 + 4 * c);
      mp[0] = make_double2(i01.x * acc[0], i01.y * acc[1] + i23.x * acc[2]);
      mp[1] = make_double2(i23.x * acc[1] + i23.y * acc[2], 0.0);
    }
  }
}

// q = K p = F^T W (F p - A m) per baseline from its time-order runs.  BPW
// baselines share a wavefront (64 / BPW lanes each), taken in the order
// `border` (baselines sorted by the smallest compact pixel they visit), so
// the baselines of one wavefront cross nearly the same pixels — for a scan
// that repeats every sidereal day, the same stretch of sky on different
// days — and one gather instruction touches fewer distinct map lines.
// Consecutive workgroups run on one XCD and take consecutive wavefront tasks.
// m is zero on invalid blocks.  With CG: per-workgroup partials of p.q and of
// the T-projection sums, partials[j * gridDim.x + blockIdx.x] for j = 0, 1, 2
// (summed in a fixed order: a wavefront butterfly, then the wavefronts in
// turn), so the step length is finished from a few thousand numbers.
// The body takes the workgroup's place (vblock of vgrid, vgrid a multiple of
// 8 and the problem's first workgroup on a multiple of 8, so vblock % 8 is
// the hardware's XCD of the workgroup) in its problem's grid.
template <typename RT, bool HAS_T, bool HAS_QU, bool IQU, bool CG, int BPW, bool PK>
__device__ __forceinline__ void unbin_runs_body(const View& v, const uint32_t* __restrict__ bstart,
                                                const uint32_t* __restrict__ border,
                                                const uint32_t* __restrict__ rpix, const int32_t* __restrict__ rn,
                                                int nb, const RT* __restrict__ rcs, const double* __restrict__ m4,
                                                const int32_t* __restrict__ nvalid, const double* __restrict__ p,
                                                double* __restrict__ q, double* __restrict__ partials, int64_t vblock,
                                                int64_t vgrid) {
  constexpr int SEG = 64 / BPW;  // lanes per baseline
  constexpr bool TONLY = HAS_T && !HAS_QU && !IQU;  // m: one double per pixel
  const int lane = lane_id();
  const int64_t n_b = v.n_b;
  const int64_t n_g = ((n_b + BPW - 1) / BPW + kWaves - 1) / kWaves;
  const int64_t per = (n_g + 7) / 8;
  const int64_t i = vblock;
  const int64_t g = (i & 7) * per + (i >> 3);
  if (g >= n_g) {  // whole workgroup
    if (CG && threadIdx.x == 0) {
#pragma unroll
      for (int j = 0; j < 3; ++j) partials[j * vgrid + i] = 0.0;
    }
    return;
  }
  const int sl = lane % SEG;
  const int64_t k = (g * kWaves + (threadIdx.x >> 6)) * BPW + lane / SEG;
  const int64_t b = k < n_b ? (int64_t)border[k] : n_b;
  double acc[3] = {0.0, 0.0, 0.0};
  if (b < n_b) {
    const int64_t r0 = bstart[b], r1 = bstart[b + 1];
    constexpr int U = 4;
    // Software pipeline: the run stream of the next step is loaded while the
    // map values of this step are gathered.
    uint32_t key[U];
    int32_t len[U];
    RT C[U], S[U];
    auto fetch = [&](int64_t rb) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t r = rb + SEG * u;
        const bool in = r < r1;
        key[u] = in ? rpix[r] : 0u;
        len[u] = (HAS_T && !PK && in) ? rn[r] : 0;
        const CS2<RT> cs =
            ((HAS_QU || IQU) && in) ? reinterpret_cast<const CS2<RT>*>(rcs)[r] : make_cs<RT>(0.0, 0.0);
        C[u] = cs.x;
        S[u] = cs.y;
      }
    };
    fetch(r0 + sl);
    for (int64_t rb = r0 + sl; rb < r1; rb += SEG * U) {
      int32_t cc_[U], nn[U];
      double Cd[U], Sd[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        // packed keys (PK): compact pixel << nb | (length - 1); else pixel, lengths in rn
        const bool in = rb + SEG * u < r1;
        cc_[u] = in ? (int32_t)(PK ? key[u] >> nb : key[u]) : -1;
        nn[u] = (HAS_T && in) ? (PK ? (int32_t)(key[u] & ((1u << nb) - 1u)) + 1 : len[u]) : 0;
        Cd[u] = (double)C[u];
        Sd[u] = (double)S[u];
      }
      double2 m01[U];
      double mU[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        m01[u] = make_double2(0.0, 0.0);
        mU[u] = 0.0;
        if (cc_[u] < 0) continue;
        if (TONLY) {
          m01[u].x = m4[cc_[u]];
          continue;
        }
        const double2* mp = reinterpret_cast<const double2*>(m4 + 4 * (int64_t)cc_[u]);
        m01[u] = mp[0];
        if (HAS_QU || IQU) mU[u] = mp[1].x;
      }
      fetch(rb + SEG * U);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (IQU) {
          acc[0] += (double)nn[u] * m01[u].x + Cd[u] * m01[u].y + Sd[u] * mU[u];
          continue;
        }
        if (HAS_T) acc[0] += (double)nn[u] * m01[u].x;
        if (HAS_QU) {
          acc[1] += Cd[u] * m01[u].y + Sd[u] * mU[u];
          acc[2] += Cd[u] * mU[u] - Sd[u] * m01[u].y;
        }
      }
    }
  }
#pragma unroll
  for (int off = SEG / 2; off > 0; off >>= 1) {
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] += __shfl_xor(acc[c], off, 64);
  }
  double pq = 0.0, eq = 0.0, ep = 0.0;
  if (sl == 0 && b < n_b) {
    const int nT = nvalid[b], nQ = nvalid[n_b + b];
    if (HAS_T) {
      const double pbv = p[v.rowT * n_b + b];
      const double o = v.w[0] * (pbv * (double)nT - acc[0]);
      q[v.rowT * n_b + b] = o;
      pq += pbv * o;
      if (nT > 0) {
        eq = o;
        ep = pbv;
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
  }
  if (CG) {
    __shared__ double red[kWaves][3];
    double t[3] = {pq, eq, ep};
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
      for (int j = 0; j < 3; ++j) t[j] += __shfl_xor(t[j], off, 64);
    }
    if (lane == 0) {
#pragma unroll
      for (int j = 0; j < 3; ++j) red[threadIdx.x >> 6][j] = t[j];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        double x = 0.0;
        for (int w = 0; w < kWaves; ++w) x += red[w][j];
        partials[j * vgrid + i] = x;
      }
    }
  }
}

template <typename RT, bool HAS_T, bool HAS_QU, bool IQU, bool CG, int BPW, bool PK>
__global__ void __launch_bounds__(kBlock) k_unbin_runs(View v, const uint32_t* __restrict__ bstart,
                                                       const uint32_t* __restrict__ border,
                                                       const uint32_t* __restrict__ rpix,
                                                       const int32_t* __restrict__ rn, int nb, const RT* __restrict__ rcs,
                                                       const double* __restrict__ m4,
                                                       const int32_t* __restrict__ nvalid,
                                                       const double* __restrict__ p, double* __restrict__ q,
                                                       CgCtl* __restrict__ ctl, double* __restrict__ partials) {
  if (CG && ctl->done) return;
  unbin_runs_body<RT, HAS_T, HAS_QU, IQU, CG, BPW, PK>(v, bstart, border, rpix, rn, nb, rcs, m4, nvalid, p, q,
                                                       partials, blockIdx.x, gridDim.x);
}

// Stable sort of the runs by pixel: onesweep passes of ten bits, so the
// 20-bit pixel indices of N_side 256 take two passes where the library's
// eight-bit passes take three (setup 6.29 -> 6.09 ms on the 30-day workload;
// eleven bits: 6.12 ms).
constexpr unsigned kRunSortBits = 10;
using RunSortConfig = rocprim::radix_sort_config<
    rocprim::default_config, rocprim::default_config,
    rocprim::radix_sort_onesweep_config<rocprim::kernel_config<1024, 16>, rocprim::kernel_config<1024, 16>,
                                        kRunSortBits, rocprim::block_radix_rank_algorithm::match>>;
// Pixels by first visit (keys 0..n_t): the same passes, also below the
// library's merge-sort limit (its merge sort took about 130 us for the
// 786,432 pixels of N_side 256).
using PixSortConfig = rocprim::radix_sort_config<
    rocprim::default_config, rocprim::default_config,
    rocprim::radix_sort_onesweep_config<rocprim::kernel_config<1024, 16>, rocprim::kernel_config<1024, 16>,
                                        kRunSortBits, rocprim::block_radix_rank_algorithm::match>,
    0>;

// Key bits to sort: keys run over 0..n_pix - 1.
unsigned key_bits(int64_t n) {
  unsigned bits = 1;
  while (bits < 32 && ((uint64_t)1 << bits) < (uint64_t)n) ++bits;
  return bits;
}

#define DST_CHECK(x)                 \
  do {                               \
    hipError_t e_ = (x);             \
    if (e_ != hipSuccess) return e_; \
  } while (0)

}  // namespace

// ---------------------------------------------------------------- host side

hipError_t runs_tmp_bytes(int64_t n_t, int64_t n_pix, int64_t n_b, size_t* bytes) {
  size_t a = 0, b = 0, c = 0;
  DST_CHECK(rocprim::exclusive_scan(nullptr, a, static_cast<const uint32_t*>(nullptr),
                                    static_cast<uint32_t*>(nullptr), 0u, (size_t)run_tiles(n_t),
                                    rocprim::plus<uint32_t>()));
  {
    rocprim::double_buffer<uint32_t> keys(nullptr, nullptr);
    rocprim::double_buffer<uint32_t> vals(nullptr, nullptr);
    DST_CHECK(rocprim::radix_sort_pairs<RunSortConfig>(nullptr, b, keys, vals, (size_t)n_t, 0u, key_bits(n_pix)));
  }
  size_t d = 0;
  {
    rocprim::double_buffer<uint32_t> keys(nullptr, nullptr);
    rocprim::double_buffer<uint32_t> vals(nullptr, nullptr);
    DST_CHECK(rocprim::radix_sort_pairs<PixSortConfig>(nullptr, d, keys, vals, (size_t)n_pix, 0u, 32u));
  }
  DST_CHECK(rocprim::exclusive_scan(nullptr, c, static_cast<const int64_t*>(nullptr), static_cast<int64_t*>(nullptr),
                                    (int64_t)0, (size_t)n_pix + 1, rocprim::plus<int64_t>()));
  size_t e = 0;
  {
    rocprim::double_buffer<uint32_t> keys(nullptr, nullptr);
    rocprim::double_buffer<uint32_t> vals(nullptr, nullptr);
    DST_CHECK(rocprim::radix_sort_pairs(nullptr, e, keys, vals, (size_t)n_b, 0u, 32u));
  }
  *bytes = std::max(std::max(std::max(a, b), std::max(c, d)), e);
  return hipSuccess;
}

int64_t run_tiles(int64_t n_t) { return (n_t + kTile - 1) / kTile; }

hipError_t runs_count(const View& v, Runs& W, int* err, hipStream_t st) {
  const int64_t n_t = v.n_t, n_tiles = run_tiles(n_t);
  // run-length bits of the packed keys: all of L when it fits beside the
  // pixel (bounded by n_pix) and baseline indices, else runs are split
  int room = 32 - (int)std::max(key_bits(std::max<int64_t>(v.n_pix, 1)), key_bits(std::max<int64_t>(v.n_b, 1)));
  if (W.split_bits > 0) room = std::min(room, W.split_bits);
  if ((int)key_bits(v.L) <= room || room < 1) {
    W.len_bits = (int)key_bits(v.L);
    W.smask = 0xffffffffu;
  } else {
    W.len_bits = room;
    W.smask = (1u << room) - 1u;
  }
  const unsigned g = grid_for(n_tiles, kWaves, 8192);
  hipLaunchKernelGGL(k_tile_heads, dim3(g), dim3(kBlock), 0, st, v.pix, n_t, v.n_pix, v.L, W.smask, n_tiles, W.tcount, err,
                     W.n_out);
  DST_CHECK(hipGetLastError());
  size_t tmp = W.tmp_bytes;
  DST_CHECK(rocprim::exclusive_scan(W.tmp, tmp, W.tcount, W.toff, 0u, (size_t)n_tiles, rocprim::plus<uint32_t>(),
                                    st));
  uint32_t last[2] = {0, 0};
  DST_CHECK(hipMemcpyAsync(&last[0], W.toff + n_tiles - 1, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  DST_CHECK(hipMemcpyAsync(&last[1], W.tcount + n_tiles - 1, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  DST_CHECK(hipStreamSynchronize(st));
  W.R = (int64_t)last[0] + last[1];
  return hipSuccess;
}

// Compile-time dispatch helpers: f(tag) for a float type chosen at run time,
// and f(T, Q) for the problem's stream set (T and/or the q/u pair).
template <typename T>
struct type_tag {
  using type = T;
};
template <typename F>
static void by_float(bool f32, F&& f) {
  if (f32)
    f(type_tag<float>{});
  else
    f(type_tag<double>{});
}
template <typename F>
static void by_streams(const View& v, F&& f) {
  if (v.iqu)
    f(std::true_type{}, std::false_type{}, std::true_type{});
  else if (v.rowT >= 0 && v.rowQ >= 0)
    f(std::true_type{}, std::true_type{}, std::false_type{});
  else if (v.rowQ >= 0)
    f(std::false_type{}, std::true_type{}, std::false_type{});
  else
    f(std::true_type{}, std::false_type{}, std::false_type{});
}
template <typename F>
static void by_bool(bool b, F&& f) {
  if (b)
    f(std::true_type{});
  else
    f(std::false_type{});
}

hipError_t runs_build(const View& v, int psi_f32, const void* tod, int tod_f32, double rcond_cut, Runs& W,
                      int32_t* hits, double* Minv4, uint8_t* valid, double* m4_zero, double* sd4, double* md4,
                      unsigned long long* counts, hipStream_t st) {
  const int64_t n_t = v.n_t, n_pix = v.n_pix, R = W.R;
  const unsigned g = grid_for(n_t, kBlock, 8192);
  // 1. run starts and per-baseline run ranges
  hipLaunchKernelGGL(k_tile_starts, dim3(grid_for(run_tiles(n_t), kWaves, 8192)), dim3(kBlock), 0, st, v.pix, n_t,
                     v.n_pix, v.L, W.smask, v.n_b, run_tiles(n_t), W.toff, (uint32_t)R, W.t0, W.bstart, W.keys[0],
                     W.vals[0]);
  DST_CHECK(hipGetLastError());
  // 2. run records and setup moments (time order)
  const bool pf = psi_f32 && (v.rowQ >= 0 || v.iqu);
  const unsigned grb = grid_for(R, kBlock, 16384);  // 64 runs per wavefront, 256 per workgroup
  by_float(pf, [&](auto pt) {
    using PT = typename decltype(pt)::type;
    by_float(tod_f32, [&](auto tt) {
      using TT = typename decltype(tt)::type;
      by_float(W.f32, [&](auto rt) {
        using RT = typename decltype(rt)::type;
        by_streams(v, [&](auto T, auto Q, auto I) {
          by_bool(tod != nullptr, [&](auto D) {
            hipLaunchKernelGGL((k_run_build<PT, TT, RT, decltype(T)::value, decltype(Q)::value, decltype(I)::value,
                                            decltype(D)::value>),
                               dim3(grb), dim3(kBlock), 0, st, v, static_cast<const TT*>(tod), W.t0, W.n_out, W.R,
                               W.tpix, W.tn,
                               static_cast<RT*>(W.tcs), W.raw, W.rec);
          });
        });
      });
    });
  });
  DST_CHECK(hipGetLastError());
  // 3. runs sorted by pixel (stable: time order inside a pixel)
  const unsigned gr = grid_for(R, kBlock, 8192);
  {
    rocprim::double_buffer<uint32_t> keys(W.keys[0], W.keys[1]);
    rocprim::double_buffer<uint32_t> vals(W.vals[0], W.vals[1]);
    size_t tmp = W.tmp_bytes;
    DST_CHECK(rocprim::radix_sort_pairs<RunSortConfig>(W.tmp, tmp, keys, vals, (size_t)R, 0u, key_bits(n_pix), st));
    W.rperm = vals.current();
    hipLaunchKernelGGL(k_key_segments, dim3(gr), dim3(kBlock), 0, st, keys.current(), R, W.seg);
    DST_CHECK(hipGetLastError());
  }
  // 4. observed pixels -> compact ids in order of first visit; run offsets
  const unsigned gp = grid_for(n_pix, kBlock, 4096);
  hipLaunchKernelGGL(k_first_visit, dim3(gp), dim3(kBlock), 0, st, W.seg, W.rperm, W.t0, n_pix, (uint32_t)n_t,
                     W.pk[0], W.pv[0],
                     W.n_obs_dev);
  DST_CHECK(hipGetLastError());
  {
    rocprim::double_buffer<uint32_t> keys(W.pk[0], W.pk[1]);
    rocprim::double_buffer<uint32_t> vals(W.pv[0], W.pv[1]);
    size_t tmp = W.tmp_bytes;
    DST_CHECK(rocprim::radix_sort_pairs<PixSortConfig>(W.tmp, tmp, keys, vals, (size_t)n_pix, 0u,
                                                       key_bits(n_t + 1), st));
    W.order = vals.current();
  }
  unsigned long long nobs = 0;
  DST_CHECK(hipMemcpyAsync(&nobs, W.n_obs_dev, sizeof nobs, hipMemcpyDeviceToHost, st));
  DST_CHECK(hipStreamSynchronize(st));
  W.n_obs = (int64_t)nobs;
  hipLaunchKernelGGL(k_compact, dim3(grid_for(W.n_obs + 1, kBlock, 4096)), dim3(kBlock), 0, st, W.order, W.n_obs,
                     W.seg, W.cid, W.ccount);
  DST_CHECK(hipGetLastError());
  {
    size_t tmp = W.tmp_bytes;
    DST_CHECK(rocprim::exclusive_scan(W.tmp, tmp, W.ccount, W.pstart, (int64_t)0, (size_t)W.n_obs + 1,
                                      rocprim::plus<int64_t>(), st));
  }
  // one 32-bit key per run for the iterations (index and length) when both fit
  const unsigned nb = (unsigned)W.len_bits;
  W.nb = 0;
  if (W.tkey && W.pkey && key_bits(std::max<int64_t>(W.n_obs, 1)) + nb <= 32 && key_bits(v.n_b) + nb <= 32)
    W.nb = (int)nb;
  // 5. per-pixel setup from the runs; pixel-order run arrays and keys
  if (W.n_obs > 0) {
    // two pixels per wavefront; at most 16384 workgroups, each taking pixels
    // 131072 apart (4096: setup +0.04 ms, 1024: +0.24 ms; one step per
    // workgroup, about 39000 of them: +1.0 ms)
    const unsigned gw = grid_for(W.n_obs, 2 * kWaves, 16384);
    by_float(W.f32, [&](auto rt) {
      using RT = typename decltype(rt)::type;
      by_streams(v, [&](auto T, auto Q, auto I) {
        by_bool(tod != nullptr, [&](auto D) {
          hipLaunchKernelGGL((k_pixels_from_runs<RT, decltype(T)::value, decltype(Q)::value, decltype(I)::value,
                                                 decltype(D)::value>),
                             dim3(gw), dim3(kBlock), 0, st, v, W.n_obs, W.order, W.seg, W.rperm, W.rec, rcond_cut,
                             W.pb, W.pn, W.nb, W.pkey, static_cast<RT*>(W.pcs), W.pstart, hits, Minv4,
                             valid, m4_zero, sd4, md4, counts);
        });
      });
    });
    DST_CHECK(hipGetLastError());
  }
  // 6. time-order runs carry compact ids from here on, and their keys; the
  // rescan order of the baselines: by the smallest compact id each visits (stable)
  if (v.n_b > 0) {
    hipLaunchKernelGGL(k_compact_baselines, dim3(grid_for(v.n_b, kWaves, 16384)), dim3(kBlock), 0, st, v.n_b,
                       W.n_obs, W.nb, W.bstart, W.cid, W.tpix, W.tn, W.tkey, W.bkey[0], W.bord[0]);
    DST_CHECK(hipGetLastError());
    rocprim::double_buffer<uint32_t> keys(W.bkey[0], W.bkey[1]);
    rocprim::double_buffer<uint32_t> vals(W.bord[0], W.bord[1]);
    size_t tmp = W.tmp_bytes;
    DST_CHECK(rocprim::radix_sort_pairs(W.tmp, tmp, keys, vals, (size_t)v.n_b, 0u, key_bits(W.n_obs + 1), st));
    W.border = vals.current();
  }
  return hipGetLastError();
}

hipError_t launch_rhs_runs(const View& vc, const Runs& W, const void* tod, int tod_f32, const double* md4,
                           const uint8_t* valid, int32_t* nvalid, double* J, double* b, hipStream_t st) {
  const int64_t n_g = ((vc.n_b + 3) / 4 + kWaves - 1) / kWaves;  // four baselines per wavefront
  const unsigned g = (unsigned)(8 * ((n_g + 7) / 8));
  by_float(W.f32, [&](auto rt) {
    using RT = typename decltype(rt)::type;
    by_float(tod_f32 != 0, [&](auto tt) {
      using TT = typename decltype(tt)::type;
      by_streams(vc, [&](auto T, auto Q, auto I) {
        by_bool(tod != nullptr, [&](auto D) {
          by_bool(W.nb != 0, [&](auto K) {
            hipLaunchKernelGGL((k_rhs_runs<RT, TT, decltype(T)::value, decltype(Q)::value, decltype(I)::value,
                                            decltype(D)::value, decltype(K)::value>),
                               dim3(g), dim3(kBlock), 0, st, vc, W.bstart, W.border,
                               W.nb ? W.tkey : reinterpret_cast<const uint32_t*>(W.tpix), W.tn, W.nb,
                               static_cast<const RT*>(W.tcs), W.raw, md4, static_cast<const TT*>(tod), W.t0,
                               valid, nvalid, J, b);
          });
        });
      });
    });
  });
  return hipGetLastError();
}

int bin_lanes_for(int64_t runs, int64_t n_obs, bool t_only) {
  // sparse pixels (few runs each) take fewer lanes, so that most lanes are
  // not idle: lanes per pixel times runs per lane and step (8 for LPP <= 16)
  // near the mean runs per pixel; dense ones 32 lanes.  Intensity-only runs
  // (one 4-byte key each) do best with 8 pixels per wavefront even when
  // dense (measured: 365 days at N_side 512, 285 runs per pixel).
  const double mean = n_obs > 0 ? (double)runs / (double)n_obs : 0.0;
  if (mean <= 32.0) return 4;
  if (mean <= 64.0 || t_only) return 8;
  return 32;
}

hipError_t launch_bin_runs(const View& vc, const Runs& W, const double* pw4, const double* Minv4,
                           const uint8_t* valid, double* m4, const CgCtl* gate, int lpp, hipStream_t st) {
  if (lpp == 0) lpp = 32;  // the default
  if (lpp != 64 && lpp != 32 && lpp != 16 && lpp != 8 && lpp != 4 && lpp != -64) lpp = 32;
  const bool pipe = lpp < 0;
  if (pipe) lpp = -lpp;
  const int64_t ppb = kWaves * (64 / lpp);
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((W.n_obs + ppb - 1) / ppb, 16384));
  by_float(W.f32, [&](auto rt) {
    using RT = typename decltype(rt)::type;
    by_streams(vc, [&](auto T, auto Q, auto I) {
      constexpr bool HT = decltype(T)::value, HQ = decltype(Q)::value, HI = decltype(I)::value;
      auto launch = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(g), dim3(kBlock), 0, st, W.n_obs, W.pstart,
                           W.nb ? W.pkey : reinterpret_cast<const uint32_t*>(W.pb), W.pn, W.nb,
                           static_cast<const RT*>(W.pcs), pw4, Minv4, valid, m4, gate);
      };
      // the pipelined variant keeps the four-double layout: not for intensity-only problems
      if (pipe && !(HT && !HQ && !HI)) {
        launch(k_bin_runs_pipe<RT, HT, HQ, HI, 64>);
        return;
      }
      if (pipe) lpp = 64;
      by_bool(W.nb != 0, [&](auto K) {
        constexpr bool PK = decltype(K)::value;
        if (lpp == 4)
          launch(k_bin_runs<RT, HT, HQ, HI, 4, PK>);
        else if (lpp == 8)
          launch(k_bin_runs<RT, HT, HQ, HI, 8, PK>);
        else if (lpp == 16)
          launch(k_bin_runs<RT, HT, HQ, HI, 16, PK>);
        else if (lpp == 32)
          launch(k_bin_runs<RT, HT, HQ, HI, 32, PK>);
        else
          launch(k_bin_runs<RT, HT, HQ, HI, 64, PK>);
      });
    });
  });
  return hipGetLastError();
}

int64_t unbin_runs_parts(const View& vc, int bpw) {
  if (bpw != 1 && bpw != 2 && bpw != 4 && bpw != 8) bpw = 4;
  const int64_t n_g = ((vc.n_b + bpw - 1) / bpw + kWaves - 1) / kWaves;
  return 8 * ((n_g + 7) / 8);
}

hipError_t launch_unbin_runs(const View& vc, const Runs& W, const double* m4, const int32_t* nvalid, const double* p,
                             double* q, CgCtl* ctl, double* partials, int bpw, hipStream_t st) {
  if (bpw != 1 && bpw != 2 && bpw != 4 && bpw != 8) bpw = 4;
  const unsigned g = (unsigned)unbin_runs_parts(vc, bpw);
  by_float(W.f32, [&](auto rt) {
    using RT = typename decltype(rt)::type;
    by_streams(vc, [&](auto T, auto Q, auto I) {
      by_bool(ctl != nullptr, [&](auto CG) {
        constexpr bool HT = decltype(T)::value, HQ = decltype(Q)::value, HI = decltype(I)::value;
        constexpr bool C = decltype(CG)::value;
        auto launch = [&](auto kern) {
          hipLaunchKernelGGL(kern, dim3(g), dim3(kBlock), 0, st, vc, W.bstart, W.border,
                             W.nb ? W.tkey : reinterpret_cast<const uint32_t*>(W.tpix), W.tn, W.nb,
                             static_cast<const RT*>(W.tcs), m4, nvalid, p, q, ctl,
                             partials);
        };
        by_bool(W.nb != 0, [&](auto K) {
          constexpr bool PK = decltype(K)::value;
          if (bpw == 8)
            launch(k_unbin_runs<RT, HT, HQ, HI, C, 8, PK>);
          else if (bpw == 4)
            launch(k_unbin_runs<RT, HT, HQ, HI, C, 4, PK>);
          else if (bpw == 2)
            launch(k_unbin_runs<RT, HT, HQ, HI, C, 2, PK>);
          else
            launch(k_unbin_runs<RT, HT, HQ, HI, C, 1, PK>);
        });
      });
    });
  });
  return hipGetLastError();
}

// ---------------------------------------------------------------- problem groups

namespace {

// Problem of workgroup b: the i with start[i] <= b < start[i + 1].
__device__ __forceinline__ int group_of(const uint32_t* start, int n, uint32_t b) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (start[mid] <= b)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

template <typename RT, int KIND, int LPP>
__global__ void __launch_bounds__(kBlock) k_group_bin(GroupLaunch G) {
  constexpr bool HT = KIND != GK_QU, HQ = KIND == GK_QU || KIND == GK_TQU, HI = KIND == GK_IQU;
  const GroupSlice& S = G.kind[KIND];
  const uint32_t b = blockIdx.x;
  const int j = group_of(S.bin_start, S.count, b);
  const GroupProblem& P = G.prob[S.first + j];
  if (P.ctl->done) return;
  const int64_t vb = b - S.bin_start[j], vg = S.bin_start[j + 1] - S.bin_start[j];
  bin_runs_body<RT, HT, HQ, HI, LPP, true>(P.v.n_pix, P.pstart, P.pkey, nullptr, P.nb, static_cast<const RT*>(P.pcs),
                                           P.pw4, P.Minv4, P.valid, P.m4, vb, vg);
}

template <typename RT, int KIND, int BPW>
__global__ void __launch_bounds__(kBlock) k_group_unbin(GroupLaunch G) {
  constexpr bool HT = KIND != GK_QU, HQ = KIND == GK_QU || KIND == GK_TQU, HI = KIND == GK_IQU;
  const GroupSlice& S = G.kind[KIND];
  const uint32_t b = blockIdx.x;
  const int j = group_of(S.unbin_start, S.count, b);
  const GroupProblem& P = G.prob[S.first + j];
  if (P.ctl->done) return;
  const int64_t vb = b - S.unbin_start[j], vg = S.unbin_start[j + 1] - S.unbin_start[j];
  unbin_runs_body<RT, HT, HQ, HI, true, BPW, true>(P.v, P.bstart, P.border, P.tkey, nullptr, P.nb,
                                                   static_cast<const RT*>(P.tcs), P.m4, P.nvalid, P.p, P.q,
                                                   P.part_unbin, vb, vg);
}

// One workgroup per problem.
__global__ void __launch_bounds__(1024) k_group_alpha(GroupLaunch G) {
  __shared__ double lds[3 * 16];
  __shared__ double clds[16 * 64];
  const int i = blockIdx.x;
  const GroupProblem& P = G.prob[i];
  cg_alpha_body(P.unbin_n, P.ctl, P.part_unbin, P.cv, P.q, P.p, lds, clds);
}

__global__ void __launch_bounds__(kBlock) k_group_update(GroupLaunch G) {
  __shared__ double lds[2 * 16];
  const uint32_t b = blockIdx.x;
  const int i = group_of(G.vec_start, G.n, b);
  const GroupProblem& P = G.prob[i];
  const int64_t vb = b - G.vec_start[i], vg = G.vec_start[i + 1] - G.vec_start[i];
  cg_update_body(P.v, P.a, P.r, P.z, P.p, P.q, P.J, P.ctl, P.part_update, vb, vg, lds);
}

__global__ void __launch_bounds__(1024) k_group_beta(GroupLaunch G) {
  __shared__ double lds[2 * 16];
  const int i = blockIdx.x;
  const GroupProblem& P = G.prob[i];
  cg_beta_body((int)P.vec_n, P.ctl, P.part_update, lds);
}

__global__ void __launch_bounds__(kBlock) k_group_p(GroupLaunch G) {
  const uint32_t b = blockIdx.x;
  const int i = group_of(G.vec_start, G.n, b);
  const GroupProblem& P = G.prob[i];
  const int64_t vb = b - G.vec_start[i], vg = G.vec_start[i + 1] - G.vec_start[i];
  p_update4_body(P.v, P.p, P.z, P.pw4, P.ctl, 1, P.dense_t, vb, vg);
}

}  // namespace

uint32_t group_bin_blocks(int64_t n_obs, int lpp) {
  const int64_t ppb = kWaves * (64 / lpp);
  return (uint32_t)std::max<int64_t>(1, std::min<int64_t>((n_obs + ppb - 1) / ppb, 16384));
}

uint32_t group_unbin_blocks(const View& vc, int bpw) { return (uint32_t)unbin_runs_parts(vc, bpw); }

uint32_t group_vec_blocks(const View& v) {
  const int64_t n = (int64_t)v.n_streams * v.n_b;
  return (uint32_t)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, 1024));
}

hipError_t launch_group_phase(const GroupLaunch& G, int phase, hipStream_t st) {
  if (G.n <= 0) return hipSuccess;
  by_float(G.f32 != 0, [&](auto rt) {
    using RT = typename decltype(rt)::type;
    auto per_kind = [&](auto kind) {
      constexpr int K = decltype(kind)::value;
      const GroupSlice& S = G.kind[K];
      if (S.count == 0) return;
      if (phase == 1) {
        switch (S.bpw) {
          case 1: hipLaunchKernelGGL((k_group_unbin<RT, K, 1>), dim3(S.unbin_total), dim3(kBlock), 0, st, G); break;
          case 2: hipLaunchKernelGGL((k_group_unbin<RT, K, 2>), dim3(S.unbin_total), dim3(kBlock), 0, st, G); break;
          case 8: hipLaunchKernelGGL((k_group_unbin<RT, K, 8>), dim3(S.unbin_total), dim3(kBlock), 0, st, G); break;
          default: hipLaunchKernelGGL((k_group_unbin<RT, K, 4>), dim3(S.unbin_total), dim3(kBlock), 0, st, G); break;
        }
        return;
      }
      switch (S.lpp) {
        case 4: hipLaunchKernelGGL((k_group_bin<RT, K, 4>), dim3(S.bin_total), dim3(kBlock), 0, st, G); break;
        case 8: hipLaunchKernelGGL((k_group_bin<RT, K, 8>), dim3(S.bin_total), dim3(kBlock), 0, st, G); break;
        case 16: hipLaunchKernelGGL((k_group_bin<RT, K, 16>), dim3(S.bin_total), dim3(kBlock), 0, st, G); break;
        default: hipLaunchKernelGGL((k_group_bin<RT, K, 32>), dim3(S.bin_total), dim3(kBlock), 0, st, G); break;
      }
    };
    if (phase <= 1) {
      per_kind(std::integral_constant<int, GK_T>{});
      per_kind(std::integral_constant<int, GK_QU>{});
      per_kind(std::integral_constant<int, GK_TQU>{});
      per_kind(std::integral_constant<int, GK_IQU>{});
      if (phase == 1) hipLaunchKernelGGL(k_group_alpha, dim3(G.n), dim3(1024), 0, st, G);
    } else {
      hipLaunchKernelGGL(k_group_update, dim3(G.vec_total), dim3(kBlock), 0, st, G);
      hipLaunchKernelGGL(k_group_beta, dim3(G.n), dim3(1024), 0, st, G);
      hipLaunchKernelGGL(k_group_p, dim3(G.vec_total), dim3(kBlock), 0, st, G);
    }
  });
  return hipGetLastError();
}

hipError_t launch_group_iteration(const GroupLaunch& G, hipStream_t st) {
  for (int phase = 0; phase < 3; ++phase) {
    const hipError_t e = launch_group_phase(G, phase, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace dst
