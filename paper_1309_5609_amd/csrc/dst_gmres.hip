// Vector kernels of the restarted GMRES solve of Eq. 13 (Saad & Schultz
// 1986; the solver the paper's implementation uses): batched dot products
// against the Krylov basis, basis combinations, the right-preconditioned
// solution update and the restart residual.  The Arnoldi coefficients, the
// Givens rotations and the small triangular solve run on the host between
// launches; every vector operation runs here.  Vectors are [n_streams][n_b].
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dst_internal.h"

namespace dst {
namespace {

constexpr int kBlock = 256;

// e = 1 on the T rows of baselines with valid T samples (J_T > 0), else 0.
__global__ void __launch_bounds__(kBlock) k_tmask(View v, const double* __restrict__ J, double* __restrict__ e) {
  const int64_t N = (int64_t)v.n_streams * v.n_b;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
    e[i] = (v.rowT >= 0 && i < v.n_b && J[i] > 0.0) ? 1.0 : 0.0;
}

// partial[i][bx] = sum over block bx's slice of V_i . w  (V_i = V + i * ldv).
__global__ void __launch_bounds__(kBlock) k_dots(const double* __restrict__ V, int64_t ldv,
                                                 const double* __restrict__ w, int64_t N,
                                                 double* __restrict__ partial) {
  __shared__ double lds[kBlock / 64];
  const double* x = V + (int64_t)blockIdx.y * ldv;
  double acc = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < N; t += (int64_t)gridDim.x * blockDim.x)
    acc += x[t] * w[t];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = lds[0];
    for (int i = 1; i < kBlock / 64; ++i) s += lds[i];
    partial[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
  }
}

// out[i] = sum_bx partial[i][bx], one workgroup per vector.
__global__ void __launch_bounds__(kBlock) k_dots_fin(const double* __restrict__ partial, int nbx,
                                                     double* __restrict__ out) {
  __shared__ double lds[kBlock / 64];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nbx; b += blockDim.x) acc += partial[(int64_t)blockIdx.x * nbx + b];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = lds[0];
    for (int i = 1; i < kBlock / 64; ++i) s += lds[i];
    out[blockIdx.x] = s;
  }
}

// w -= sum_i c_i V_i.
__global__ void __launch_bounds__(kBlock) k_combine(double* __restrict__ w, const double* __restrict__ V, int64_t ldv,
                                                    int k, GmresCoef c, int64_t N) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < N; t += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < k; ++i) s += c.c[i] * V[(int64_t)i * ldv + t];
    w[t] -= s;
  }
}

// out = s w, or out = J w (the right preconditioner) with J non-null.
__global__ void __launch_bounds__(kBlock) k_scale(const double* __restrict__ w, double s,
                                                  const double* __restrict__ J, double* __restrict__ out,
                                                  int64_t N) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < N; t += (int64_t)gridDim.x * blockDim.x)
    out[t] = J ? J[t] * w[t] : s * w[t];
}

// x += J (sum_i y_i V_i).
__global__ void __launch_bounds__(kBlock) k_xupdate(double* __restrict__ x, const double* __restrict__ J,
                                                    const double* __restrict__ V, int64_t ldv, int k, GmresCoef y,
                                                    int64_t N) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < N; t += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < k; ++i) s += y.c[i] * V[(int64_t)i * ldv + t];
    x[t] += J[t] * s;
  }
}

// r = b - (q - mu e): the residual with K x projected off the T null vector.
__global__ void __launch_bounds__(kBlock) k_restart_resid(const double* __restrict__ b, const double* __restrict__ q,
                                                          double mu, const double* __restrict__ e,
                                                          double* __restrict__ r, int64_t N) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < N; t += (int64_t)gridDim.x * blockDim.x)
    r[t] = b[t] - (q[t] - mu * e[t]);
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

hipError_t launch_dots(const double* V, int64_t ldv, int k, const double* w, int64_t N, double* partial, double* out,
                       hipStream_t st) {
  const int nbx = gmres_dot_blocks(N);
  hipLaunchKernelGGL(k_dots, dim3(nbx, k), dim3(kBlock), 0, st, V, ldv, w, N, partial);
  hipLaunchKernelGGL(k_dots_fin, dim3(k), dim3(kBlock), 0, st, partial, nbx, out);
  return hipGetLastError();
}

hipError_t launch_combine(double* w, const double* V, int64_t ldv, int k, const GmresCoef& c, int64_t N,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_combine, dim3(vec_grid(N)), dim3(kBlock), 0, st, w, V, ldv, k, c, N);
  return hipGetLastError();
}

hipError_t launch_scale(const double* w, double s, const double* J, double* out, int64_t N, hipStream_t st) {
  hipLaunchKernelGGL(k_scale, dim3(vec_grid(N)), dim3(kBlock), 0, st, w, s, J, out, N);
  return hipGetLastError();
}

hipError_t launch_xupdate(double* x, const double* J, const double* V, int64_t ldv, int k, const GmresCoef& y,
                          int64_t N, hipStream_t st) {
  hipLaunchKernelGGL(k_xupdate, dim3(vec_grid(N)), dim3(kBlock), 0, st, x, J, V, ldv, k, y, N);
  return hipGetLastError();
}

hipError_t launch_restart_resid(const double* b, const double* q, double mu, const double* e, double* r, int64_t N,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_restart_resid, dim3(vec_grid(N)), dim3(kBlock), 0, st, b, q, mu, e, r, N);
  return hipGetLastError();
}

}  // namespace dst
