// Several independent destriping problems advanced together: one launch per
// PCG phase serves every problem of the group (the channels of a survey,
// each with its own pointing, map and baselines; per-horn independence,
// Introduction of arXiv:1309.5609).  A launch's workgroups are split into
// consecutive ranges, one per problem; a workgroup finds its problem by
// binary search over the range starts and runs the same body the
// single-problem kernels run, with its place in that problem's range.  A
// problem whose solve has stopped leaves its workgroups idle.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "dst_comp.h"
#include "dst_internal.h"

namespace dst {

enum GroupKind { GK_T = 0, GK_QU = 1, GK_TQU = 2, GK_IQU = 3 };

// One problem of a group, in device memory.  All arrays are the problem's
// own (compact pixel space, packed run keys).
struct GroupProblem {
  View v;  // compact view: n_pix = observed pixels
  int kind;
  int nb;       // length bits of the packed run keys (> 0)
  int dense_t;  // intensity only: pw4 and m4 hold one double per baseline / pixel
  uint32_t unbin_n, vec_n;  // workgroups of the problem in the rescan and vector launches
  const int64_t* pstart;
  const uint32_t* pkey;
  const void* pcs;
  const uint32_t* bstart;
  const uint32_t* border;
  const uint32_t* tkey;
  const void* tcs;
  const double* Minv4;
  const uint8_t* valid;
  double* m4;
  double* pw4;
  const int32_t* nvalid;
  const double* J;
  double *a, *r, *z, *p, *q;
  CgCtl* ctl;
  double* part_unbin;   // [3][unbin_n]
  double* part_update;  // [2][vec_n]
  CompView cv;
};

// The group's launches.  Problems are ordered by kind; the binning and the
// rescan take one launch per kind present (the slice of problems of that
// kind, each owning workgroups start[i] .. start[i + 1] - 1, every rescan
// range a multiple of 8), since the kinds' kernels differ twofold in
// registers per lane; the vector phases take one launch for all problems.
struct GroupSlice {
  int first = 0, count = 0;
  const uint32_t* bin_start = nullptr;    // device [count + 1]
  const uint32_t* unbin_start = nullptr;  // device [count + 1]
  uint32_t bin_total = 0, unbin_total = 0;
  int lpp = 32;  // lanes per pixel of the binning (4, 8, 16 or 32)
  int bpw = 4;   // baselines per wavefront of the rescan (1, 2, 4 or 8)
};
struct GroupLaunch {
  const GroupProblem* prob = nullptr;  // device [n]
  int n = 0;
  const uint32_t* vec_start = nullptr;  // device [n + 1]
  uint32_t vec_total = 0;
  int f32 = 0;  // run sums of cos 2psi, sin 2psi in FP32 (every problem with angles agrees)
  GroupSlice kind[4];
};

// Workgroups each phase gives one problem.
uint32_t group_bin_blocks(int64_t n_obs, int lpp);
uint32_t group_unbin_blocks(const View& vc, int bpw);  // a multiple of 8
uint32_t group_vec_blocks(const View& v);

// One PCG iteration of every running problem: binning (m = M^-1 A^T W F p),
// rescan (q = K p and the step-length partials), step length (with the
// component projection), residual update, stopping test and beta, new p.
hipError_t launch_group_iteration(const GroupLaunch& G, hipStream_t st);
// The phases one by one, for timing (phase 0: bin; 1: rescan and step
// length; 2: update, beta and p).
hipError_t launch_group_phase(const GroupLaunch& G, int phase, hipStream_t st);

}  // namespace dst
