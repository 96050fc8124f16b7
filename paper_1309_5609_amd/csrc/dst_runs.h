// Run-compressed pointing used by the iterative solve (default form).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "dst_internal.h"

namespace dst {

// Per-run pair (sum of cos 2psi, sum of sin 2psi) in the run sums' precision:
// one 16-byte (FP64) or 8-byte (FP32) load per run in the iterations.
template <typename RT>
using CS2 = typename std::conditional<std::is_same<RT, double>::value, double2, float2>::type;

template <typename RT>
__host__ __device__ inline CS2<RT> make_cs(double c, double s) {
  CS2<RT> v;
  v.x = (RT)c;
  v.y = (RT)s;
  return v;
}

// Per-run record read by the per-pixel setup (one aligned 64-byte access):
// length, baseline, sums over the run of cos 2psi, sin 2psi, cos^2 2psi,
// cos 2psi sin 2psi, d_T and of the rotated, weighted q/u pair
// (w_q d_q c - w_u d_u s, w_q d_q s + w_u d_u c).
struct alignas(64) RunRecord {
  int32_t n;
  int32_t b;
  double C, S, cc, cs, dT, dQ, dU;
};
static_assert(sizeof(RunRecord) == 64, "run record must be one 64-byte line");

// Intensity-only problems keep a 16-byte record per run (length, baseline,
// sum of d_T) and one raw sum per run: the angle moments are not needed.
struct alignas(16) RunRecordT {
  int32_t n;
  int32_t b;
  double dT;
};
static_assert(sizeof(RunRecordT) == 16, "intensity run record must be 16 bytes");

// A run is a maximal stretch of consecutive unmasked samples on one pixel
// inside one baseline.  Runs are kept twice: in time order (t*: rescan and
// baseline sums; bstart[b] .. bstart[b+1] are the runs of baseline b) and in
// pixel order (p*: binning; pstart[c] .. pstart[c+1] are the runs of compact
// pixel c, in time order).  Compact ids number observed pixels in order of
// first visit, so pixels that a stretch of the scan crosses sit close
// together in per-pixel arrays.
//
// Buffers belong to the caller's workspace.  Sizes: tcount, toff
// [run_tiles(n_t)];
// bstart [n_b + 1]; t0, tpix, tn, pb, pn [R] and the pairs tcs, pcs [2 R] (FP32
// when f32, else FP64);
// raw [3 R]; rec [R]; keys, vals 2 x [R]; seg [2 n_pix] (zero-filled before
// runs_build); pk, pv 2 x [n_pix]; cid [n_pix] (filled with -1 before
// runs_build); ccount, pstart [n_pix + 1]; bkey, bord 2 x [n_b].
struct Runs {
  uint32_t* tcount = nullptr;  // run starts per tile of the run detection
  uint32_t* toff = nullptr;    // their exclusive scan
  void* tmp = nullptr;
  size_t tmp_bytes = 0;
  int64_t R = 0;
  uint32_t* t0 = nullptr;
  unsigned long long* n_out = nullptr;  // samples in no run (masked or out of range); zero-filled before runs_count
  uint32_t* bstart = nullptr;
  bool f32 = false;  // run sums of cos 2psi, sin 2psi (tcs, pcs) stored in FP32 (else FP64)
  int32_t* tpix = nullptr;
  int32_t* tn = nullptr;
  void* tcs = nullptr;  // [2 R] CS2 pairs per run, time order
  double* raw = nullptr;       // [3 R] ([R] for T only), time order: at each run that ends its baseline or a
                               // 64-run window, the sums of d_T, d_q, d_u over the baseline's runs in the window
  RunRecord* rec = nullptr;    // [R] per-run records (time order); RunRecordT for T only
  uint32_t* keys[2] = {nullptr, nullptr};
  uint32_t* vals[2] = {nullptr, nullptr};
  const uint32_t* rperm = nullptr;
  int64_t* seg = nullptr;
  uint32_t* pk[2] = {nullptr, nullptr};
  uint32_t* pv[2] = {nullptr, nullptr};
  unsigned long long* n_obs_dev = nullptr;  // zero-filled before runs_build
  int32_t* cid = nullptr;
  int64_t* ccount = nullptr;
  const uint32_t* order = nullptr;  // compact id -> pixel (set by runs_build)
  int64_t n_obs = 0;
  int32_t* pb = nullptr;
  int32_t* pn = nullptr;
  void* pcs = nullptr;  // [2 R] CS2 pairs per run, pixel order
  int64_t* pstart = nullptr;
  // Iteration keys [R] (time and pixel order): index << nb | (length - 1),
  // used when nb > 0 (index and length fit 32 bits together).
  uint32_t* tkey = nullptr;
  uint32_t* pkey = nullptr;
  int nb = 0;
  // Set by runs_count: bits of the run length in a packed key, and the mask
  // of the forced run splits (t & smask == 0 starts a run; all ones: none).
  int len_bits = 0;
  uint32_t smask = 0xffffffffu;
  int split_bits = 0;  // > 0: split runs at 2^split_bits samples at most (set by the caller)
  // Rescan order of the baselines (set by runs_build): sorted by the smallest
  // compact id each visits, so baselines over the same sky sit together.
  uint32_t* bkey[2] = {nullptr, nullptr};
  uint32_t* bord[2] = {nullptr, nullptr};
  const uint32_t* border = nullptr;
};

// Number of tiles the run detection splits n_t samples into.
int64_t run_tiles(int64_t n_t);
hipError_t runs_tmp_bytes(int64_t n_t, int64_t n_pix, int64_t n_b, size_t* bytes);
// Marks run heads and counts the runs (W.R); synchronises `st`.
hipError_t runs_count(const View& v, Runs& W, int* err, hipStream_t st);
// Builds the time- and pixel-order runs, compact ids (synchronises `st` once
// for n_obs), and per compact pixel: hits, block inverse, validity, zeroed
// m4 and, with tod, the sum map sd4 and binned map md4.
// counts: [valid T pixels, valid QU pixels, valid T samples, valid QU samples].
hipError_t runs_build(const View& v, int psi_f32, const void* tod, int tod_f32, double rcond_cut, Runs& W,
                      int32_t* hits, double* Minv4, uint8_t* valid, double* m4_zero, double* sd4, double* md4,
                      unsigned long long* counts, hipStream_t st);
// Per baseline: n_valid, Jacobi diagonal, and with tod b = F^T W (d - A m_d)
// (tod as given to runs_build; the data part comes from the run build's
// per-baseline window sums, less the runs on pixels left out of the map).
hipError_t launch_rhs_runs(const View& vc, const Runs& W, const void* tod, int tod_f32, const double* md4,
                           const uint8_t* valid, int32_t* nvalid, double* J, double* b, hipStream_t st);
// Lanes per pixel of the binning for `runs` runs over n_obs pixels
// (t_only: an intensity-only problem).
int bin_lanes_for(int64_t runs, int64_t n_obs, bool t_only);
// m = M^-1 A^T W F p (pw4 = interleaved w .* p).
// lpp: lanes per pixel (64, 32, 16, 8 or 4; -64: 64 with the pixel pipeline; 0: 32).
hipError_t launch_bin_runs(const View& vc, const Runs& W, const double* pw4, const double* Minv4,
                           const uint8_t* valid, double* m4, const CgCtl* gate, int lpp, hipStream_t st);
// q = K p; with ctl the per-workgroup CG partials, unbin_runs_parts(vc, bpw)
// of each kind (finished by launch_cg_alpha).
// bpw: baselines per wavefront (1, 2, 4 or 8; else 4), taken in the order
// W.border.
int64_t unbin_runs_parts(const View& vc, int bpw);
hipError_t launch_unbin_runs(const View& vc, const Runs& W, const double* m4, const int32_t* nvalid, const double* p,
                             double* q, CgCtl* ctl, double* partials, int bpw, hipStream_t st);

}  // namespace dst
