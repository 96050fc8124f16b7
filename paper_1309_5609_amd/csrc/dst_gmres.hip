// Restarted GMRES on Eq. 13 (Saad & Schultz 1986; the solver the paper's
// implementation uses), with its whole state on the device: the Arnoldi
// coefficients, the Hessenberg matrix, the Givens rotations, the residual
// estimate and the small triangular solve live in a GmState that the kernels
// read and write, so the host only enqueues launches and reads a status
// written into pinned memory, one step behind the GPU.
//
// One Arnoldi step j (classical Gram-Schmidt with one reorthogonalisation,
// w = P K J v_j, P the projection off the T null vector e / per component):
//   next   v_j = src / h_{j-1}, z = J v_j and the binning's weighted z
//   (the operator: binning and rescan, then the component projection)
//   dots   h1 = (e.w, v_0.w .. v_j.w)
//   orth 1 w -= (h1_0 / n_e) e + sum_i h1_{i+1} v_i, then h2 = (v_i.w)
//   orth 2 w -= sum_i h2_i v_i, then ||w||, the new column of H, the
//          rotations and the residual estimate |g_{j+1}| / ||b||
// Every kernel of a step returns at once when ctl.done is set, so steps
// enqueued past the stop cost a launch each.  Vectors are [n_streams][n_b];
// the basis V holds e at slot 0 and v_i at slot i + 1.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "dst_internal.h"

namespace dst {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

__device__ __forceinline__ double wave_sum(double x) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Sum of x over the workgroup, in a fixed order; valid in thread 0.
__device__ __forceinline__ double block_sum(double x, double* lds) {
  x = wave_sum(x);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = x;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += lds[w];
  __syncthreads();
  return s;
}

__device__ __forceinline__ double& Hat(GmState* s, int i, int j) { return s->H[i * kMaxRestart + j]; }

__device__ __forceinline__ void write_status(const GmState* s, GmStatus* out) {
  if (!out) return;
  out->iter = s->ctl.iter;
  out->done = s->ctl.done;
  out->k = s->k;
  out->rel = s->rel;
  __threadfence_system();
}

// e = 1 on the T rows of baselines with valid T samples (J_T > 0), else 0.
__global__ void __launch_bounds__(kBlock) k_tmask(View v, const double* __restrict__ J, double* __restrict__ e) {
  const int64_t N = (int64_t)v.n_streams * v.n_b;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
    e[i] = (v.rowT >= 0 && i < v.n_b && J[i] > 0.0) ? 1.0 : 0.0;
}

__global__ void k_gm_init(GmState* s, double bnorm, double n_e, double tol, int max_iter, int m, double beta,
                          double rel, int done, GmStatus* status) {
  if (threadIdx.x != 0) return;
  s->ctl.done = done;
  s->ctl.iter = 0;
  s->ctl.max_iter = max_iter;
  s->ctl.b_norm = bnorm;
  s->bnorm = bnorm;
  s->n_e = n_e;
  s->tol = tol;
  s->rel = rel;
  s->m = m;
  s->k = 0;
  s->g[0] = beta;
  s->inv_h = beta > 0.0 ? 1.0 / beta : 0.0;
  write_status(s, status);
}

// v_j = inv_h src, z = J v_j and pw4 (per baseline: w_T z_T, w_q z_q, w_u z_u, 0;
// with dense_t, one w_T z_T per baseline), one thread per baseline.
__global__ void __launch_bounds__(kBlock) k_gm_next(View v, const GmState* __restrict__ s,
                                                    const double* __restrict__ src, double* __restrict__ vj,
                                                    const double* __restrict__ J, double* __restrict__ z,
                                                    double* __restrict__ pw4, int dense_t) {
  if (s->ctl.done) return;
  const double h = s->inv_h;
  const int64_t n_b = v.n_b;
  const int rows[3] = {v.rowT, v.rowQ, v.rowU};
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < n_b; b += (int64_t)gridDim.x * blockDim.x) {
    double w4[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (rows[k] < 0) continue;
      const int64_t i = rows[k] * n_b + b;
      const double x = h * src[i];
      const double zi = J[i] * x;
      vj[i] = x;
      z[i] = zi;
      w4[k] = v.w[k] * zi;
    }
    if (dense_t) {
      pw4[b] = w4[0];
    } else {
      double2* o = reinterpret_cast<double2*>(pw4 + 4 * b);
      o[0] = make_double2(w4[0], w4[1]);
      o[1] = make_double2(w4[2], 0.0);
    }
  }
}

// partial[i][bx] = block bx's slice of V_i . w  (V_i = V + i N), i = blockIdx.y.
__global__ void __launch_bounds__(kBlock) k_gm_dots(const GmState* __restrict__ s, const double* __restrict__ V,
                                                    const double* __restrict__ w, int64_t N,
                                                    double* __restrict__ partial) {
  if (s->ctl.done) return;
  __shared__ double lds[kWaves];
  const double* x = V + (int64_t)blockIdx.y * N;
  double acc = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < N; t += (int64_t)gridDim.x * blockDim.x)
    acc += x[t] * w[t];
  acc = block_sum(acc, lds);
  if (threadIdx.x == 0) partial[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = acc;
}

// out[i] = sum_bx partial[i][bx], one workgroup per vector i = blockIdx.x.
__global__ void __launch_bounds__(kBlock) k_gm_dots_fin(const GmState* __restrict__ s,
                                                        const double* __restrict__ partial, int nbx,
                                                        double* __restrict__ out) {
  if (s->ctl.done) return;
  __shared__ double lds[kWaves];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nbx; b += blockDim.x) acc += partial[(int64_t)blockIdx.x * nbx + b];
  acc = block_sum(acc, lds);
  if (threadIdx.x == 0) out[blockIdx.x] = acc;
}

// Orthogonalisation pass (mode 1 or 2, see launch_gm_orth), the slices of
// k_gm_dots: each wavefront takes 64 consecutive elements at a time, updates
// w there and adds the wave's sums of the products into its LDS row.
__global__ void __launch_bounds__(kBlock) k_gm_orth(GmState* __restrict__ s, int mode, const double* __restrict__ V,
                                                    int j, double* __restrict__ w, int64_t N,
                                                    double* __restrict__ partial) {
  if (s->ctl.done) return;
  __shared__ double coef[kMaxKrylov];
  __shared__ double acc[kWaves][kMaxKrylov];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // combined vectors: mode 1 e, v_0 .. v_j (from V); mode 2 v_0 .. v_j (from V + N)
  const int ncomb = mode == 1 ? j + 2 : j + 1;
  const double* C = mode == 1 ? V : V + N;
  const int nd = mode == 1 ? j + 1 : 1;  // dot products per slice
  for (int i = threadIdx.x; i < ncomb; i += blockDim.x) {
    double c;
    if (mode == 1)
      c = i == 0 ? (s->n_e > 0.0 ? s->h1[0] / s->n_e : 0.0) : s->h1[i];
    else
      c = s->h2[i];
    coef[i] = c;
  }
  for (int i = threadIdx.x; i < kWaves * kMaxKrylov; i += blockDim.x) (&acc[0][0])[i] = 0.0;
  __syncthreads();
  for (int64_t base = ((int64_t)blockIdx.x * kWaves + wave) * 64; base < N; base += (int64_t)gridDim.x * kBlock) {
    const int64_t t = base + lane;
    const bool in = t < N;
    double x = in ? w[t] : 0.0;
    double sum = 0.0;
    for (int i = 0; i < ncomb; ++i) sum += coef[i] * (in ? C[(int64_t)i * N + t] : 0.0);
    x -= sum;
    if (in) w[t] = x;
    if (mode == 1) {
      for (int i = 0; i < nd; ++i) {
        const double pr = wave_sum(x * (in ? V[(int64_t)(i + 1) * N + t] : 0.0));
        if (lane == 0) acc[wave][i] += pr;
      }
    } else {
      const double pr = wave_sum(x * x);
      if (lane == 0) acc[wave][0] += pr;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nd; i += blockDim.x) {
    double t = 0.0;
    for (int wv = 0; wv < kWaves; ++wv) t += acc[wv][i];
    partial[(int64_t)i * gridDim.x + blockIdx.x] = t;
  }
}

// Step j's end: h = ||w|| from the partial sums; column j of H = h1 + h2 with
// h below the diagonal; the earlier rotations, a new one zeroing h; g and the
// residual estimate; the stop (converged, iteration limit, breakdown, or a
// pause on h = 0); 1 / h for the next basis vector.  One workgroup.
__global__ void __launch_bounds__(kBlock) k_gm_givens(GmState* __restrict__ s, int j,
                                                      const double* __restrict__ partial, int nbx,
                                                      GmStatus* status) {
  __shared__ double lds[kWaves];
  const bool run = s->ctl.done == DONE_RUNNING;
  double acc = 0.0;
  if (run)
    for (int b = threadIdx.x; b < nbx; b += blockDim.x) acc += partial[b];
  acc = block_sum(acc, lds);
  if (threadIdx.x != 0) return;
  if (run) {
    const double hn = sqrt(fmax(acc, 0.0));
    for (int i = 0; i <= j; ++i) Hat(s, i, j) = s->h1[i + 1] + s->h2[i];
    Hat(s, j + 1, j) = hn;
    for (int i = 0; i < j; ++i) {
      const double a = Hat(s, i, j), b = Hat(s, i + 1, j);
      Hat(s, i, j) = s->cs[i] * a + s->sn[i] * b;
      Hat(s, i + 1, j) = -s->sn[i] * a + s->cs[i] * b;
    }
    const double den = hypot(Hat(s, j, j), Hat(s, j + 1, j));
    if (!(den > 0.0) || !isfinite(den)) {
      s->ctl.done = isfinite(den) ? DONE_BREAKDOWN : DONE_NAN;
    } else {
      const double c = Hat(s, j, j) / den, sn = Hat(s, j + 1, j) / den;
      s->cs[j] = c;
      s->sn[j] = sn;
      Hat(s, j, j) = den;
      Hat(s, j + 1, j) = 0.0;
      const double gj = s->g[j];
      s->g[j + 1] = -sn * gj;
      s->g[j] = c * gj;
      s->ctl.iter += 1;
      s->k = j + 1;
      const double rel = fabs(s->g[j + 1]) / s->bnorm;
      s->rel = rel;
      s->inv_h = hn > 0.0 ? 1.0 / hn : 0.0;
      if (!isfinite(rel))
        s->ctl.done = DONE_NAN;
      else if (rel <= s->tol)
        s->ctl.done = DONE_CONVERGED;
      else if (s->ctl.iter >= s->ctl.max_iter)
        s->ctl.done = DONE_MAXITER;
      else if (hn == 0.0)
        s->ctl.done = DONE_PAUSE;
    }
  }
  write_status(s, status);
}

// y = R^-1 g over the cycle's k columns (one wavefront: each row's sum split
// over the lanes); a paused solve resumes.
__global__ void __launch_bounds__(64) k_gm_solve(GmState* __restrict__ s) {
  __shared__ double y[kMaxRestart];
  const int k = s->k;
  for (int i = k - 1; i >= 0; --i) {
    double part = 0.0;
    for (int l = i + 1 + (int)threadIdx.x; l < k; l += 64) part += Hat(s, i, l) * y[l];
    part = wave_sum(part);
    if (threadIdx.x == 0) y[i] = (s->g[i] - part) / Hat(s, i, i);
    __syncthreads();
  }
  for (int i = threadIdx.x; i < k; i += 64) s->y[i] = y[i];
  if (threadIdx.x == 0 && s->ctl.done == DONE_PAUSE) s->ctl.done = DONE_RUNNING;
}

// a += J sum_{i < k} y_i v_i.
__global__ void __launch_bounds__(kBlock) k_gm_xupdate(const GmState* __restrict__ s, const double* __restrict__ J,
                                                       const double* __restrict__ V, double* __restrict__ a,
                                                       int64_t N) {
  const int k = s->k;
  if (k == 0) return;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < N; t += (int64_t)gridDim.x * blockDim.x) {
    double sum = 0.0;
    for (int i = 0; i < k; ++i) sum += s->y[i] * V[(int64_t)(i + 1) * N + t];
    a[t] += J[t] * sum;
  }
}

// r = b - (q - mu e), mu = e.q / n_e (in h1_0), and block partials of r.r.
__global__ void __launch_bounds__(kBlock) k_gm_rresid(const GmState* __restrict__ s, const double* __restrict__ b,
                                                      const double* __restrict__ q, const double* __restrict__ e,
                                                      double* __restrict__ r, int64_t N,
                                                      double* __restrict__ partial) {
  if (s->ctl.done) return;
  __shared__ double lds[kWaves];
  const double mu = s->n_e > 0.0 ? s->h1[0] / s->n_e : 0.0;
  double acc = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < N; t += (int64_t)gridDim.x * blockDim.x) {
    const double x = b[t] - (q[t] - mu * e[t]);
    r[t] = x;
    acc += x * x;
  }
  acc = block_sum(acc, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// The next cycle's start: beta = ||r||, g = beta e_1, no columns, 1 / beta for
// v_0; a zero residual ends the solve.  One workgroup.
__global__ void __launch_bounds__(kBlock) k_gm_begin(GmState* __restrict__ s, const double* __restrict__ partial,
                                                     int nbx, GmStatus* status) {
  __shared__ double lds[kWaves];
  const bool run = s->ctl.done == DONE_RUNNING;
  double acc = 0.0;
  if (run)
    for (int b = threadIdx.x; b < nbx; b += blockDim.x) acc += partial[b];
  acc = block_sum(acc, lds);
  if (threadIdx.x != 0) return;
  if (run) {
    const double beta = sqrt(fmax(acc, 0.0));
    s->g[0] = beta;
    s->k = 0;
    s->inv_h = beta > 0.0 ? 1.0 / beta : 0.0;
    if (!isfinite(beta)) {
      s->ctl.done = DONE_NAN;
    } else if (beta == 0.0) {
      s->rel = 0.0;
      s->ctl.done = DONE_CONVERGED;
    }
  }
  write_status(s, status);
}

unsigned vec_grid(int64_t N) {
  int64_t g = (N + kBlock - 1) / kBlock;
  if (g > 2048) g = 2048;
  if (g < 1) g = 1;
  return (unsigned)g;
}

}  // namespace

int gmres_dot_blocks(int64_t N) {
  int64_t g = (N + 4 * kBlock - 1) / (4 * kBlock);
  if (g > 256) g = 256;
  if (g < 1) g = 1;
  return (int)g;
}

hipError_t launch_tmask(const View& v, const double* J, double* e, hipStream_t st) {
  hipLaunchKernelGGL(k_tmask, dim3(vec_grid((int64_t)v.n_streams * v.n_b)), dim3(kBlock), 0, st, v, J, e);
  return hipGetLastError();
}

hipError_t launch_gm_init(GmState* s, double bnorm, double n_e, double tol, int max_iter, int m, double beta,
                          double rel, int done, GmStatus* status, hipStream_t st) {
  hipLaunchKernelGGL(k_gm_init, dim3(1), dim3(64), 0, st, s, bnorm, n_e, tol, max_iter, m, beta, rel, done, status);
  return hipGetLastError();
}

hipError_t launch_gm_next(const View& v, GmState* s, const double* src, double* vj, const double* J, double* z,
                          double* pw4, int dense_t, hipStream_t st) {
  hipLaunchKernelGGL(k_gm_next, dim3(vec_grid(v.n_b)), dim3(kBlock), 0, st, v, s, src, vj, J, z, pw4, dense_t);
  return hipGetLastError();
}

hipError_t launch_gm_dots(GmState* s, const double* V, int k, const double* w, int64_t N, double* partial,
                          double* out, hipStream_t st) {
  const int nbx = gmres_dot_blocks(N);
  hipLaunchKernelGGL(k_gm_dots, dim3(nbx, k), dim3(kBlock), 0, st, s, V, w, N, partial);
  hipLaunchKernelGGL(k_gm_dots_fin, dim3(k), dim3(kBlock), 0, st, s, partial, nbx, out);
  return hipGetLastError();
}

hipError_t launch_gm_orth(GmState* s, int mode, const double* V, int j, double* w, int64_t N, double* partial,
                          GmStatus* status, hipStream_t st) {
  if (mode != 1 && mode != 2) return hipErrorInvalidValue;
  if (j < 0 || j + 2 > kMaxKrylov) return hipErrorInvalidValue;
  const int nbx = gmres_dot_blocks(N);
  hipLaunchKernelGGL(k_gm_orth, dim3(nbx), dim3(kBlock), 0, st, s, mode, V, j, w, N, partial);
  if (mode == 1)
    hipLaunchKernelGGL(k_gm_dots_fin, dim3(j + 1), dim3(kBlock), 0, st, s, partial, nbx, s->h2);
  else
    hipLaunchKernelGGL(k_gm_givens, dim3(1), dim3(kBlock), 0, st, s, j, partial, nbx, status);
  return hipGetLastError();
}

hipError_t launch_gm_update(GmState* s, const double* J, const double* V, double* a, int64_t N, hipStream_t st) {
  hipLaunchKernelGGL(k_gm_solve, dim3(1), dim3(64), 0, st, s);
  hipLaunchKernelGGL(k_gm_xupdate, dim3(vec_grid(N)), dim3(kBlock), 0, st, s, J, V, a, N);
  return hipGetLastError();
}

hipError_t launch_gm_restart(GmState* s, const double* b, const double* q, const double* e, double* r, int64_t N,
                             double* partial, GmStatus* status, hipStream_t st) {
  const int nbx = gmres_dot_blocks(N);
  hipError_t err = launch_gm_dots(s, e, 1, q, N, partial, s->h1, st);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_gm_rresid, dim3(nbx), dim3(kBlock), 0, st, s, b, q, e, r, N, partial);
  hipLaunchKernelGGL(k_gm_begin, dim3(1), dim3(kBlock), 0, st, s, partial, nbx, status);
  return hipGetLastError();
}

}  // namespace dst
