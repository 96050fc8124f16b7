// Bodies of the PCG vector steps (the solver paragraph closing the Algorithm
// section of arXiv:1309.5609, applied to Eq. 13), shared by the single
// solve's kernels and by the kernels that advance several independent
// problems in one launch.  A body takes the workgroup's position in its own
// problem's grid (vblock of vgrid) instead of blockIdx / gridDim.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "dst_comp.h"
#include "dst_device.h"
#include "dst_internal.h"

namespace dst {

// Step length from the rescan's partials (n_part of each kind: p.q, T sum of
// q, T sum of p): the null-space projection of q = K p (one component: the
// mean mu over T-valid baselines, applied by the residual update; several:
// each component's mean removed from q in place) and alpha = r.z / p.(P K p).
// One workgroup; fixed summation order.  lds: 48 doubles; clds: 16 * 64.
__device__ inline void cg_alpha_body(int64_t n_part, CgCtl* ctl, const double* partials, const CompView& cv,
                                     double* q, const double* p, double* lds, double* clds) {
  if (ctl->done) return;
  double tot[3] = {0.0, 0.0, 0.0};
  for (int64_t j = threadIdx.x; j < n_part; j += blockDim.x) {
    tot[0] += partials[j];
    tot[1] += partials[n_part + j];
    tot[2] += partials[2 * n_part + j];
  }
  dev::block_sum<3>(tot, lds);
  const int ncomp = cv.ncomp ? *cv.ncomp : 0;
  double corr = 0.0;
  if (ncomp > 1) corr = comp_project_block(cv, ncomp, q, p, 1, 1, clds);
  if (threadIdx.x == 0) {
    const double mu = ncomp > 1 ? 0.0 : (ctl->n_e > 0.0 ? tot[1] / ctl->n_e : 0.0);
    const double pkp = ncomp > 1 ? tot[0] - corr : tot[0] - mu * tot[2];
    ctl->mu = mu;
    if (!isfinite(pkp)) {
      ctl->done = DONE_NAN;
    } else if (pkp <= 0.0) {
      ctl->done = DONE_BREAKDOWN;
    } else {
      ctl->alpha = ctl->rz / pkp;
    }
  }
}

// Stopping test on ||r|| and beta = r'.z' / r.z from the update's n_part
// partials of each kind.  One workgroup.  lds: 32 doubles.
__device__ inline void cg_beta_body(int n_part, CgCtl* ctl, const double* partials, double* lds) {
  if (ctl->done) return;
  double tot[2] = {0.0, 0.0};
  for (int j = threadIdx.x; j < n_part; j += blockDim.x) {
    tot[0] += partials[j];
    tot[1] += partials[n_part + j];
  }
  dev::block_sum<2>(tot, lds);
  if (threadIdx.x == 0) {
    const double rz_new = tot[0];
    const double rn = sqrt(tot[1]);
    ctl->iter += 1;
    ctl->r_norm = rn;
    if (!isfinite(rz_new) || !isfinite(rn)) {
      ctl->done = DONE_NAN;
    } else if (rn <= ctl->tol * ctl->b_norm) {
      ctl->done = DONE_CONVERGED;
    } else if (ctl->iter >= ctl->max_iter) {
      ctl->done = DONE_MAXITER;
    } else {
      ctl->beta = rz_new / ctl->rz;
      ctl->rz = rz_new;
    }
  }
}

// a += alpha p;  r -= alpha P q;  z = J r;  the workgroup's partials of r.z
// and r.r at partials[vblock] and partials[vgrid + vblock].  lds: 32 doubles.
__device__ inline void cg_update_body(const View& v, double* a, double* r, double* z, const double* p,
                                      const double* q, const double* J, const CgCtl* ctl, double* partials,
                                      int64_t vblock, int64_t vgrid, double* lds) {
  if (ctl->done) return;
  const int64_t N = (int64_t)v.n_streams * v.n_b;
  const double alpha = ctl->alpha, mu = ctl->mu;
  double acc[2] = {0.0, 0.0};
  for (int64_t i = vblock * blockDim.x + threadIdx.x; i < N; i += vgrid * blockDim.x) {
    const double ji = J[i];
    const double qi = q[i] - ((v.rowT >= 0 && i < v.n_b && ji > 0.0) ? mu : 0.0);
    a[i] += alpha * p[i];
    const double ri = r[i] - alpha * qi;
    r[i] = ri;
    const double zi = ji * ri;
    z[i] = zi;
    acc[0] += ri * zi;
    acc[1] += ri * ri;
  }
  dev::block_sum<2>(acc, lds);
  if (threadIdx.x == 0) {
    partials[vblock] = acc[0];
    partials[vgrid + vblock] = acc[1];
  }
}

// p = z + beta p (z == NULL: p unchanged) and its weighted interleaved copy
// pw4[b] = (w_T p_T, w_q p_q, w_u p_u, 0) read by the pixel-order binning
// (dense_t: intensity-only, pw4[b] = w_T p_T, one double per baseline).
__device__ inline void p_update4_body(const View& v, double* p, const double* z, double* pw4, const CgCtl* ctl,
                                      int use_beta, int dense_t, int64_t vblock, int64_t vgrid) {
  if (ctl && ctl->done) return;
  const double beta = use_beta ? ctl->beta : 0.0;
  const int64_t n_b = v.n_b;
  if (dense_t) {
    for (int64_t b = vblock * blockDim.x + threadIdx.x; b < n_b; b += vgrid * blockDim.x) {
      double pi = z ? z[b] + beta * p[b] : p[b];
      if (z) p[b] = pi;
      pw4[b] = v.w[0] * pi;
    }
    return;
  }
  for (int64_t b = vblock * blockDim.x + threadIdx.x; b < n_b; b += vgrid * blockDim.x) {
    double w4[4] = {0.0, 0.0, 0.0, 0.0};
    const int rows[3] = {v.rowT, v.rowQ, v.rowU};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (rows[k] < 0) continue;
      const int64_t i = rows[k] * n_b + b;
      double pi = z ? z[i] + beta * p[i] : p[i];
      if (z) p[i] = pi;
      w4[k] = v.w[k] * pi;
    }
    double2* o = reinterpret_cast<double2*>(pw4 + 4 * b);
    o[0] = make_double2(w4[0], w4[1]);
    o[1] = make_double2(w4[2], 0.0);
  }
}

}  // namespace dst
