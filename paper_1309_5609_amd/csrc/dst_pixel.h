// Pixel-major (transposed) pointing used by the iterative solve.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "dst_internal.h"
#include "dst_comp.h"

namespace dst {

// The pointing of one problem, reorganised once for the iterations.
//
// Observed pixels get compact ids in order of first visit, so the pixels a
// stretch of the scan touches sit close together in memory.  The samples of
// compact pixel c, in time order, occupy [cstart[c], cstart[c+1]) of cperm
// (sample index), sb (baseline index) and spsi (angle).  cpix[t] is the
// compact id of sample t (-1 if masked).
//
// Buffers belong to the caller's workspace.  Sizes: keys, vals 2 x [n_t];
// pk, pv 2 x [n_pix]; seg [2 (n_pix + 1)] (zero-filled before the build);
// cid [n_pix] (filled with -1 before the build); chits, cstart [n_pix + 1];
// cperm, sb, cpix [n_t]; spsi [n_t] of the angle's type; tmp tmp_bytes.
struct Transpose {
  uint32_t* keys[2] = {nullptr, nullptr};
  uint32_t* vals[2] = {nullptr, nullptr};
  uint32_t* pk[2] = {nullptr, nullptr};
  uint32_t* pv[2] = {nullptr, nullptr};
  void* tmp = nullptr;
  size_t tmp_bytes = 0;
  unsigned long long* n_obs_dev = nullptr;  // zero-filled before the build
  int64_t* seg = nullptr;
  int32_t* cid = nullptr;
  int64_t* chits = nullptr;
  int64_t* cstart = nullptr;
  uint32_t* cperm = nullptr;
  int32_t* sb = nullptr;
  void* spsi = nullptr;
  int32_t* cpix = nullptr;
  // set by transpose_build
  const uint32_t* perm = nullptr;
  const uint32_t* order = nullptr;  // compact id -> pixel
  int64_t n_obs = 0;
};

hipError_t transpose_tmp_bytes(int64_t n_t, int64_t n_pix, size_t* bytes);
// Sort, segments, first-visit compact ids, offsets and cpix; synchronises `st`
// once to learn n_obs.  The per-sample arrays (cperm, sb, spsi) are filled by
// launch_setup_pixels.
hipError_t transpose_build(const View& v, Transpose& T, int* err, hipStream_t st);
// Per compact pixel: the transposed sample arrays, hits, block inverse and
// validity, zeroed m4, and (tod != NULL) the sum map sd4 and binned map md4.
// counts: [valid T pixels, valid QU pixels, valid T samples, valid QU samples].
hipError_t launch_setup_pixels(const View& v, int psi_f32, const Transpose& T, const void* tod, int tod_f32,
                               double rcond_cut, int32_t* hits, double* Minv4, uint8_t* valid, double* m4_zero,
                               double* sd4, double* md4, unsigned long long* counts, hipStream_t st);
// Per baseline: n_valid, Jacobi diagonal and (tod != NULL) b = F^T W (d - A m_d).
hipError_t launch_rhs_unbin(const View& vc, int psi_f32, const void* tod, int tod_f32, const double* md4,
                            const uint8_t* valid, int32_t* nvalid, double* J, double* b, hipStream_t st);
hipError_t launch_bin_pixel(const View& vc, int psi_f32, const Transpose& T, const double* pw4, const double* Minv4,
                            const uint8_t* valid, double* m4, const CgCtl* gate, hipStream_t st);
hipError_t launch_unbin_cg(const View& vc, int psi_f32, const double* m4, const int32_t* nvalid, const double* p,
                           double* q, CgCtl* ctl, double* partials, hipStream_t st);
// Single-workgroup finishes of the CG step (alpha) and of the residual update (beta).
// alpha reads n_part partials of each kind (n_b from k_unbin_cg); when the
// baseline-pixel graph has several components it projects q = K p in place
// (p: the search direction).
hipError_t launch_cg_alpha(int64_t n_part, CgCtl* ctl, const double* partials, const CompView& cv, double* q,
                           const double* p, hipStream_t st);
hipError_t launch_cg_beta(int n_part, CgCtl* ctl, const double* partials, hipStream_t st);
// p = z + beta p (z == NULL: p unchanged) and pw4 = interleaved w .* p
// (dense_t: intensity-only run form, pw4[b] = w_T p_T)
hipError_t launch_p_update4(const View& v, double* p, const double* z, double* pw4, const CgCtl* ctl, int use_beta,
                            int dense_t, hipStream_t st);
// Full-sky outputs: hits[p] and out3[p] = a4[cid[p]] - b4[cid[p]] (0 where unobserved;
// any of hits / b4 / out3 may be NULL; b_dense: b4 holds one double per pixel, the I value).
hipError_t launch_scatter(int64_t n_pix, const int32_t* cid, const int32_t* chits, int32_t* hits, const double* a4,
                          const double* b4, double* out3, hipStream_t st, int b_dense = 0);

}  // namespace dst
