// Connected components of the baseline-pixel graph and the null-space
// projection they define.
//
// A constant added to the T baselines (or to the baselines of a radiometer
// stream) of one connected component of the bipartite graph
// baseline <-> pixel, linked by the samples valid for that stream, is
// indistinguishable from the same constant added to the I map of the
// component's pixels (the full data model, Eq. 8).  So K = F^T Z F (Eq. 13)
// has one null vector per component: the indicator e_c of the component's
// baselines.  The solvers remove the component means from b and from every
// K p, and the solution is reported with zero mean per component.
//
// Layout of a baseline-indexed quantity x for Rp right-hand sides: element
// (baseline b, right-hand side r) at x[b * sb + r] (single solve: sb = 1,
// Rp = 1; batched solve: [n_b][n_streams][Rp] with the T row first, so
// sb = n_streams * Rp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dst {

// Device-side description of the components, built once per pointing.
//   ncomp   number of components (0 when no baseline holds a valid sample)
//   start   [ncomp + 1] offsets into member (written only when ncomp > 1)
//   member  baselines of each component in increasing order (ncomp > 1)
struct CompView {
  const int32_t* ncomp = nullptr;  // NULL: no T-like stream, no projection
  const uint32_t* start = nullptr;
  const uint32_t* member = nullptr;
};

// Buffers of the component build (caller's workspace), sizes in elements:
// parent, label [n_b]; start [n_b + 1]; member, cursor [n_b]; ncomp [4];
// pmin [n_obs]; flags [kCompFlags].
constexpr int kCompFlags = 32;
struct Comp {
  int32_t* parent = nullptr;
  int32_t* label = nullptr;
  uint32_t* start = nullptr;
  uint32_t* member = nullptr;
  uint32_t* cursor = nullptr;
  int32_t* ncomp = nullptr;
  int32_t* pmin = nullptr;
  int32_t* flags = nullptr;
  CompView view() const {
    CompView c;
    c.ncomp = ncomp;
    c.start = start;
    c.member = member;
    return c;
  }
};

// The time-order elements of each baseline: the runs (bstart [n_b + 1], keys
// c << nb | length - 1, or c when nb = 0) or, without runs, the samples with
// their compact pixels cpix [n_t] (-1 masked).
struct ChainSource {
  const uint32_t* bstart = nullptr;
  const uint32_t* tkey = nullptr;
  int nb = 0;
  const int32_t* cpix = nullptr;
  int64_t L = 1, n_t = 0;
};

// Components over the pixels whose T block is valid (bit 0 of valid).
// Elements elem_start[c] .. elem_start[c + 1] - 1 belong to compact pixel c
// (runs or samples in pixel order); eb[e] is the baseline of element e;
// nvalid_T[b] the number of valid samples of baseline b.  Asynchronous.
hipError_t launch_components(int64_t n_b, int64_t n_obs, const int64_t* elem_start, const int32_t* eb,
                             const uint8_t* valid, const int32_t* nvalid_T, const ChainSource& cs, Comp& C,
                             hipStream_t st);

// x <- x - (component mean of x) on every baseline of a component, for each of
// R right-hand sides, when there is more than one component (one component
// is left to the solvers' own global projection).  Asynchronous.
hipError_t launch_comp_project(const CompView& cv, double* x, int64_t sb, int Rp, hipStream_t st);

// One workgroup: for every component c and right-hand side r,
//   mean = sum_{b in c} x[b][r] / |c|,   x[b][r] -= mean  (b in c),
//   corr[r] += mean * sum_{b in c} y[b][r]        (y may be NULL),
// with corr[r] (r < Rp) valid in threads 0 .. Rp - 1 on return (0 without y).
// Waves take components round robin and every sum runs in a fixed order, so
// the result does not depend on scheduling.  lds: at least 16 * 64 doubles.
__device__ inline double comp_project_block(const CompView& cv, int ncomp, double* x, const double* y, int64_t sb,
                                            int Rp, double* lds) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const int G = 64 / Rp;  // member groups per wave
  const int r = lane & (Rp - 1);
  const int g = lane / Rp;
  double corr = 0.0;
  for (int c = wave; c < ncomp; c += nw) {
    const uint32_t m0 = cv.start[c], m1 = cv.start[c + 1];
    double sx = 0.0, sy = 0.0;
    for (uint32_t m = m0 + g; m < m1; m += G) {
      const int64_t i = (int64_t)cv.member[m] * sb + r;
      sx += x[i];
      if (y) sy += y[i];
    }
    for (int off = 32; off >= Rp; off >>= 1) {
      sx += __shfl_xor(sx, off, 64);
      sy += __shfl_xor(sy, off, 64);
    }
    const double mean = sx / (double)(m1 - m0);
    for (uint32_t m = m0 + g; m < m1; m += G) x[(int64_t)cv.member[m] * sb + r] -= mean;
    corr += mean * sy;
  }
  if (lane < Rp) lds[wave * 64 + lane] = corr;
  __syncthreads();
  double tot = 0.0;
  if ((int)threadIdx.x < Rp)
    for (int w = 0; w < nw; ++w) tot += lds[w * 64 + threadIdx.x];
  __syncthreads();
  return tot;
}

}  // namespace dst
