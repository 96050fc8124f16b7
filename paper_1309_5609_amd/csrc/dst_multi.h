// Multi-right-hand-side form of the solve: up to kMaxRhs problems that share
// pointing, weights and the rcond cut (Monte Carlo realizations of one
// channel) are solved together.  The operator K = F^T Z F depends only on the
// pointing and the weights (Eq. 13 of arXiv:1309.5609), so one pass over the
// run records applies it to every right-hand side at once; each realization
// keeps its own CG scalars and stops on its own.
//
// Layouts (Rp = number of right-hand sides rounded up to a power of two; the
// padding slots are inert):
//   per-baseline vectors  [n_b][n_streams][Rp]
//   per-pixel maps        [n_obs][n_streams][Rp]   (component row = stream row:
//                                                    I with T, Q with q, U with u)
// so that the Rp values one run needs are contiguous.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "dst_comp.h"
#include "dst_internal.h"
#include "dst_runs.h"

namespace dst {

constexpr int kMaxRhs = 64;

// CG state of every right-hand side, in device memory.
struct MultiCtl {
  double rz[kMaxRhs];
  double alpha[kMaxRhs];
  double beta[kMaxRhs];
  double mu[kMaxRhs];       // T mean of K p over T-valid baselines (null-space projection)
  double b_norm[kMaxRhs];
  double r_norm[kMaxRhs];
  double mu_b[kMaxRhs];     // T mean of b removed at start-up
  double true_norm[kMaxRhs];
  double corr[kMaxRhs];     // p.(K p - P K p) when the graph has several components
  int32_t iter[kMaxRhs];
  int32_t done[kMaxRhs];    // DONE_* codes; DONE_PAD marks padding slots
  double n_e;               // number of T-valid baselines
  double tol;
  int32_t max_iter;
  int32_t n_rhs;
  int32_t running;          // right-hand sides still iterating; 0 stops every kernel
  int32_t pad;
};

enum { DONE_PAD = 5 };

struct Multi {
  int R = 0;   // right-hand sides
  int Rp = 0;  // padded count (power of two, <= kMaxRhs)
};

int multi_padded(int R);

// ipos[run] = position of time-order run `run` in the pixel-order arrays.
hipError_t launch_run_positions(const Runs& W, uint32_t* ipos, hipStream_t st);

// Timelines of up to kTodBatch realizations handled by one setup pass; their
// per-run data sums share one record of kRunRec doubles (one 128-byte line).
constexpr int kTodBatch = 5;
constexpr int kRunRec = 16;
static_assert(3 * kTodBatch <= kRunRec, "a pass's run sums must fit one record");
struct TodSet {
  const void* p[kTodBatch];
};

// Realizations ri0 .. ri0 + nr - 1 (nr <= kTodBatch, same tod dtype): per-run
// sums of the weighted data at each run's pixel-order position, one record of
// kRunRec doubles per run (one 128-byte line: realization i at [3 i .. 3 i + 2]
// = w_T d_T, rotated Q, rotated U), and per-baseline sums w_k d_k over valid
// samples into braw ([n_b][n_streams][Rp]).  prs holds kRunRec R doubles.
hipError_t launch_multi_tod(const View& vc, int psi_f32, const TodSet& tods, int nr, int tod_f32, const Runs& W,
                            const uint32_t* ipos, const uint8_t* valid, int Rp, int ri0, double* prs, double* braw,
                            hipStream_t st);
// Realizations ri0 .. ri0 + nr - 1: binned maps md = M^-1 (sum of the pixel's run sums).
hipError_t launch_multi_pixsum(int64_t n_obs, const View& vc, const Runs& W, const double* prs, int nr,
                               const double* Minv4, int Rp, int ri0, double* md, hipStream_t st);

// m = M^-1 A^T W F p for every active right-hand side (ctl NULL: all R).
// The float form reads p and writes m in FP32 (sums in FP64): the
// mixed-precision iterations of a batch with FP32 angles and timelines.
hipError_t launch_multi_bin(const View& vc, const Runs& W, const Multi& mu, const double* p, const double* Minv4,
                            double* m, const MultiCtl* ctl, hipStream_t st);
hipError_t launch_multi_bin(const View& vc, const Runs& W, const Multi& mu, const float* p, const double* Minv4,
                            float* m, const MultiCtl* ctl, hipStream_t st);
// Modes of the rescan + baseline sum.
enum MultiUnbinMode { UNBIN_OPERATOR = 0, UNBIN_CG = 1, UNBIN_RHS = 2 };
// OPERATOR: q = K p.  CG: q = K p for running right-hand sides plus per-block
// partials of p.q and of the T-projection sums.  RHS: q = braw - F^T W A m.
int multi_unbin_blocks(const View& vc);
hipError_t launch_multi_unbin(const View& vc, const Runs& W, const Multi& mu, int mode, const double* m,
                              const int32_t* nvalid, const double* p, const double* braw, double* q, MultiCtl* ctl,
                              double* partials, hipStream_t st);
hipError_t launch_multi_unbin(const View& vc, const Runs& W, const Multi& mu, int mode, const float* m,
                              const int32_t* nvalid, const double* p, const double* braw, double* q, MultiCtl* ctl,
                              double* partials, hipStream_t st);

// CG pieces (N = n_b * n_streams * Rp).
hipError_t launch_multi_start(const View& v, const Multi& mu, double* b, double* a, double* r, double* z, double* p,
                              const double* J, MultiCtl* ctl, double* partials, double tol, int max_iter,
                              hipStream_t st);
// With several components of the baseline-pixel graph, q = K p loses each
// component's mean in place (per right-hand side) and ctl->corr the matching
// p.q correction; nothing happens with one component.
hipError_t launch_multi_comp(const View& v, const Multi& mu, const CompView& cv, double* q, const double* p,
                             MultiCtl* ctl, hipStream_t st);
hipError_t launch_multi_alpha(const View& vc, const Multi& mu, MultiCtl* ctl, const double* partials,
                              const CompView& cv, hipStream_t st);
int multi_update_blocks(const View& v, const Multi& mu);
hipError_t launch_multi_update(const View& v, const Multi& mu, double* a, double* r, double* z, const double* q,
                               const double* p, const double* J, MultiCtl* ctl, double* partials, hipStream_t st);
hipError_t launch_multi_beta(const View& v, const Multi& mu, MultiCtl* ctl, const double* partials, hipStream_t st);
// p = z + beta p; with p32, its FP32 copy too.
hipError_t launch_multi_p(const View& v, const Multi& mu, double* p, const double* z, const MultiCtl* ctl,
                          hipStream_t st, float* p32 = nullptr);
// y = (float) x, N values.
hipError_t launch_to_f32(const double* x, float* y, int64_t N, hipStream_t st);
// a_T -= its mean over T-valid baselines (0 elsewhere), per right-hand side.
hipError_t launch_multi_canonicalise(const View& v, const Multi& mu, double* a, const double* J, MultiCtl* ctl,
                                     double* partials, hipStream_t st);
// ctl->true_norm[r] = || P (b - K a) || per right-hand side.
hipError_t launch_multi_resid(const View& v, const Multi& mu, const double* b, const double* ka, const double* J,
                              MultiCtl* ctl, double* partials, hipStream_t st);

// Column ri of a multi vector -> [n_streams][n_b].
hipError_t launch_multi_extract(const View& v, const Multi& mu, int ri, const double* x, double* out,
                                hipStream_t st);
// Column ri of the maps -> full-sky user map [n_pix][3]: md - m (m may be NULL), zero where unobserved.
hipError_t launch_multi_scatter(const View& full, const View& vc, const int32_t* cid, const Multi& mu, int ri,
                                const double* md, const double* m, double* out3, hipStream_t st);

}  // namespace dst
