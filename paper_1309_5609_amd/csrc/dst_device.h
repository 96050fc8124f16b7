// Device helpers shared by the multi-right-hand-side kernels: wavefront and
// workgroup sums (fixed order, so results do not depend on scheduling) and the
// 2psi rotation.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "dst_trig.h"

namespace dst {
namespace dev {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ void rot2(double psi, double& c, double& s) { fast_sincos(2.0 * psi, &s, &c); }

// Butterfly sum over lanes that differ in bits [log2(from), 6): after the
// call every lane holds the sum over its group of 64 / from lanes with equal
// (lane mod from).
template <int N>
__device__ __forceinline__ void lane_group_sum(double (&v)[N], int from) {
  for (int off = 32; off >= from; off >>= 1) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += __shfl_xor(v[i], off, 64);
  }
}

template <int N>
__device__ __forceinline__ void wave_sum(double (&v)[N]) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += __shfl_xor(v[i], off, 64);
  }
}

// Sum over the whole workgroup; the result is valid in thread 0.
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

// Copies n 4-byte words from global memory to a wavefront's own LDS range
// through the LDS-direct load path (one word per lane and instruction; lane l
// writes dst + 4 (i + l)), so a whole stage is in flight at once with no
// registers.  The source needs 4-byte alignment only.  Call from the whole
// wavefront with dst uniform; the data are in LDS after lds_copy_wait().
__device__ __forceinline__ void lds_copy_words(const void* src, void* dst, int n) {
  const uint32_t* s = static_cast<const uint32_t*>(src);
  uint32_t* d = static_cast<uint32_t*>(dst);
  const int lane = lane_id();
  for (int i = 0; i < n; i += 64) {
    if (i + lane < n) __builtin_amdgcn_global_load_lds(s + i + lane, d + i, 4, 0, 0);
  }
}

// Waits for every outstanding load of the wavefront (the LDS-direct ones
// included); the wave barrier keeps the compiler from moving LDS reads above.
__device__ __forceinline__ void lds_copy_wait() {
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
}

}  // namespace dev
}  // namespace dst
