// Internal declarations shared by the kernels and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "dst.h"

namespace dst {

// Problem as the kernels see it.  Rows give the position of each stream in
// [n_streams][...] arrays (-1 when the stream is absent).
struct View {
  const int32_t* pix;
  const void* psi;
  int64_t n_t;
  int64_t n_pix;
  int64_t L;
  int64_t n_b;
  double w[3];  // T, q, u
  int rowT, rowQ, rowU, n_streams;
  int iqu;      // 1: one radiometer stream (row 0) with pointing row (1, cos 2psi, sin 2psi)
};

// CG scalars and reduction scratch, resident in device memory.
struct CgCtl {
  double rz;       // r.z of the current residual
  double alpha;    // step of the current iteration
  double beta;     // p update coefficient
  double mu;       // mean of the T part of K p over T-valid baselines (null-space projection)
  double b_norm;   // ||P b||
  double r_norm;   // ||r|| of the recurrence
  double tol;
  double n_e;      // number of baselines with valid T samples
  double mu_b;     // projection means of b and of K a0 at start-up
  double mu_ka;
  int32_t iter;
  int32_t done;    // 0 running, 1 converged, 2 breakdown, 3 non-finite, 4 max_iter
  int32_t max_iter;
  int32_t pad;
  uint32_t counter[4];  // arrival counters of the last-block reductions
};

enum { DONE_RUNNING = 0, DONE_CONVERGED = 1, DONE_BREAKDOWN = 2, DONE_NAN = 3, DONE_MAXITER = 4 };

// Kernel-side layout of per-pixel data: [n_pix][4] doubles.
//   sums / map:  (I, Q, U, unused)
//   inverse:     (1/M_II, (M_QU^-1)_QQ, (M_QU^-1)_QU, (M_QU^-1)_UU)
// valid: bit 0 = T block valid, bit 1 = QU block valid.

// ---- launchers (all asynchronous on `st`) --------------------------------
hipError_t launch_pointing(const View& v, int psi_f32, int32_t* hits, double* M4, int* err, hipStream_t st);
hipError_t launch_invert(const View& v, const int32_t* hits, const double* M4, double rcond_cut, double* Minv4,
                         uint8_t* valid, double* blocks_out, unsigned long long* counts, hipStream_t st);
hipError_t launch_baseline_counts(const View& v, const uint8_t* valid, int32_t* nvalid, double* jacobi,
                                  unsigned long long* counts, hipStream_t st);
// s[p] += sum_k w_k A_k^T x_k over valid samples, x = tod (if tod) + base_sign * F base (if base)
hipError_t launch_bin(const View& v, int psi_f32, const void* tod, int tod_f32, const double* base, double base_sign,
                      const uint8_t* valid, double* s4, int* err, const CgCtl* gate, hipStream_t st);
// m[p] = Minv[p] s[p]; optional clearing of s; m_stride 3 (user layout) or 4
hipError_t launch_apply(int64_t n_pix, const double* s4, const double* Minv4, double* m, int m_stride, double* s_clear,
                        const CgCtl* gate, hipStream_t st);
// out_k[b] = sum_{t in b} v_k(t) w_k (x_k(t) - A_k(t) . m[p(t)]), x as in launch_bin.
// With ctl: also the CG step (alpha, mu) from p.q with base = p.
hipError_t launch_unbin_reduce(const View& v, int psi_f32, const void* tod, int tod_f32, const double* base,
                               double base_sign, const double* m4, const uint8_t* valid, const int32_t* nvalid,
                               double* out, CgCtl* ctl, double* partials, hipStream_t st);
hipError_t launch_scan(const View& v, int psi_f32, const double* map3, double* out, int* err, hipStream_t st);
hipError_t launch_reduce(const View& v, const void* x, int x_f32, const uint8_t* valid, double* out, hipStream_t st);

// CG vector kernels; N = n_streams * n_b, J = Jacobi diagonal [n_streams][n_b].
hipError_t launch_cg_start(const View& v, double* b, const double* ka, const double* a0, double* a, double* r,
                           double* z, double* p, const double* J, CgCtl* ctl, double* partials, double tol,
                           int max_iter, hipStream_t st);
// per-block partials of r.z and r.r at partials[0 .. 2 * cg_update_blocks(v))
hipError_t launch_cg_update(const View& v, double* a, double* r, double* z, const double* p, const double* q,
                            const double* J, CgCtl* ctl, double* partials, hipStream_t st);
int cg_update_blocks(const View& v);
hipError_t launch_p_update(const View& v, double* p, const double* z, const CgCtl* ctl, hipStream_t st);
// a_T -= mean of a_T over baselines with valid T samples (J_T > 0).
hipError_t launch_canonicalise(const View& v, double* a, const double* J, double* partials, CgCtl* ctl,
                               hipStream_t st);
// ||x - P y||_2 into ctl->r_norm slot given (used for the true residual)
hipError_t launch_residual_norm(const View& v, const double* b, const double* ka, const double* J, CgCtl* ctl,
                                double* partials, double* out_norm, hipStream_t st);
// Copy kernel layout [n_pix][4] -> user [n_pix][3]
hipError_t launch_fill(double* x, int64_t n, double value, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* x, int64_t n, uint32_t value, hipStream_t st);

// ---- pointing expansion (dst_pointing.hip) ---------------------------------
// [3][n_per] table of one spin period: hour angle, cos(colatitude), psi.
void scan_period_table(const dst_scan& s, int64_t n_per, std::vector<double>& tab);
hipError_t launch_expand(int64_t nside, int64_t start, int64_t n, int64_t n_per, const dst_scan& s, const double* tab,
                         int32_t* pix, void* psi, int psi_f32, hipStream_t st);

// ---- Monte Carlo noise (dst_noise.hip) -------------------------------------
int64_t noise_pairs_per_chunk(int64_t S);
int64_t noise_twiddle_count(int64_t S);
// buf0, buf1: noise_pairs_per_chunk(S) * S complex values each; tw:
// noise_twiddle_count(S) complex values.
hipError_t launch_noise(uint64_t seed, uint64_t stream, int64_t n, int64_t S, double rate, double sigma, double fknee,
                        double alpha, void* out, int out_f32, int accumulate, double2* buf0, double2* buf1,
                        double2* tw, hipStream_t st);

// ---- restarted GMRES on the device (dst_gmres.hip) ------------------------
constexpr int kMaxKrylov = 128;  // basis vectors + the T mask in one dot launch; restart <= kMaxKrylov - 2
constexpr int kMaxRestart = kMaxKrylov - 2;
// ctl.done of a cycle that stopped early on an invariant Krylov space (new
// basis vector of norm zero): the steps left in the cycle do nothing and the
// restart resumes.
constexpr int DONE_PAUSE = 5;

// Device state of one GMRES solve.  ctl.done gates every kernel of the
// iteration (the operator's included); ctl.iter counts Arnoldi steps.
struct GmState {
  CgCtl ctl;
  double bnorm, n_e, tol, rel, inv_h;
  int32_t m, k, pad0, pad1;  // restart length; columns of the current cycle
  double h1[kMaxKrylov];     // e.w, v_0.w .. v_j.w of the step
  double h2[kMaxKrylov];     // the reorthogonalisation's v_i.w
  double cs[kMaxRestart], sn[kMaxRestart], g[kMaxRestart + 1], y[kMaxRestart];
  double H[(kMaxRestart + 1) * kMaxRestart];  // Hessenberg (i, j) at i * kMaxRestart + j
};
// What the host reads back (pinned memory written by the kernels).
struct GmStatus {
  int32_t iter, done, k, pad;
  double rel;
};

int gmres_dot_blocks(int64_t N);
hipError_t launch_tmask(const View& v, const double* J, double* e, hipStream_t st);
hipError_t launch_gm_init(GmState* s, double bnorm, double n_e, double tol, int max_iter, int m, double beta,
                          double rel, int done, GmStatus* status, hipStream_t st);
// v_j = inv_h src; z = J v_j; pw4 = the per-baseline weighted z (binning layout).
hipError_t launch_gm_next(const View& v, GmState* s, const double* src, double* vj, const double* J, double* z,
                          double* pw4, int dense_t, hipStream_t st);
// out[i] = V_i . w for i < k (V_i = V + i N); partial: k * gmres_dot_blocks(N) doubles.
hipError_t launch_gm_dots(GmState* s, const double* V, int k, const double* w, int64_t N, double* partial,
                          double* out, hipStream_t st);
// mode 1: w -= (h1_0 / n_e) e + sum_{i <= j} h1_{i+1} v_i, then partial dots v_i . w (i <= j) into h2;
// mode 2: w -= sum_{i <= j} h2_i v_i, then ||w||^2, the Givens step j and the status.
hipError_t launch_gm_orth(GmState* s, int mode, const double* V, int j, double* w, int64_t N, double* partial,
                          GmStatus* status, hipStream_t st);
// y = R^-1 g over the cycle's k columns, then a += J sum_i y_i v_i; resumes a paused solve.
hipError_t launch_gm_update(GmState* s, const double* J, const double* V, double* a, int64_t N, hipStream_t st);
// r = b - (q - (e.q / n_e) e) with e.q in h1_0, beta = ||r||, the next cycle's start, the status.
hipError_t launch_gm_restart(GmState* s, const double* b, const double* q, const double* e, double* r, int64_t N,
                             double* partial, GmStatus* status, hipStream_t st);

}  // namespace dst
