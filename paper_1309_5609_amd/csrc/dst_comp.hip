// Connected components of the baseline-pixel graph (the null vectors of the
// destriping operator, Eq. 13 with the full model of Eq. 8) and the
// per-component projection.
//
// Build: a lock-free union-find over the baselines (hooks by compare-and-swap,
// always the larger root under the smaller, so every parent is smaller than
// its child, no cycle can form and a set's root is its smallest member;
// finds halve their path).  Loads may return an earlier parent, which is
// still an ancestor: a find then ends at a node that was a root, and a hook
// on a node that is no longer a root fails its compare-and-swap and retries
// from the new parent, so stale reads cost retries, never correctness.
// Minimum-label rounds over sampled edges settle a scan's graph first
// (below); the union-find pass over all elements runs only when they leave
// more than one self-labelled baseline.  Then
// each baseline takes its root, roots are numbered in increasing order and,
// when there is more than one component, the members of each are listed in
// increasing baseline order (a deterministic order, so sums over a component
// do not depend on scheduling).
#include <hip/hip_runtime.h>

#include "dst_comp.h"

namespace dst {
namespace {

constexpr int kBlk = 256;

// Parent reads and path-halving writes of the union-find: relaxed and
// cacheable (an earlier value is an ancestor, see above).
__device__ __forceinline__ int32_t uf_load(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void uf_store(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Values of the component lists that other wavefronts wrote: read at device
// scope.
__device__ __forceinline__ int32_t dev_load(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void dev_store(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Loads and stores of values other threads wrote through atomics or in
// other wavefronts, at device scope (not served from a stale L1 line).
__device__ __forceinline__ uint32_t ld_u32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_u32(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x with path halving.  Parents only ever point to smaller indices,
// so the walk ends.
__device__ int32_t uf_find(int32_t* parent, int32_t x) {
  int32_t p = uf_load(parent + x);
  while (p != x) {
    const int32_t gp = uf_load(parent + p);
    if (gp != p) uf_store(parent + x, gp);  // gp is an ancestor of x: the invariant holds
    x = p;
    p = gp;
  }
  return x;
}

__device__ void uf_union(int32_t* parent, int32_t a, int32_t b) {
  a = uf_find(parent, a);
  b = uf_find(parent, b);
  while (a != b) {
    if (a < b) {
      const int32_t t = a;
      a = b;
      b = t;
    }
    // hook root a (the larger) under b; on failure a was hooked meanwhile
    const int32_t old = atomicCAS(parent + a, a, b);
    if (old == a) return;
    a = uf_find(parent, old);
    b = uf_find(parent, b);
  }
}

// Labels by minimum propagation over a subset of the graph's edges (every
// kStride-th element of each pixel, the pixel's last, and every kStride-th
// element of each baseline): a round takes, per valid pixel, the smallest
// label of its sampled baselines (pixel order), then lowers each baseline's
// label to the smallest of its sampled pixels' and jumps once to that label's
// own label (time order).  Labels only decrease and always name a smaller
// baseline of the same component (every edge used is one of the graph's).
// The rounds end when one changes nothing or when a single baseline with
// valid samples is still its own label (the graph is then connected);
// otherwise the labels seed the union-find (each label a valid parent) and
// the pass over all elements settles the components exactly.
constexpr int kRounds = 12;
constexpr int kStride = 8;
static_assert(2 * kRounds + 1 <= kCompFlags, "the round flags live in the flags buffer");

// flags: [0, kRounds) round r changed a label; [kRounds, 2 kRounds) after
// round r, the baselines with valid samples still labelled by themselves (0
// when the round did not run); 2 kRounds: the union-find pass is needed.
// Every label names a smaller baseline of the same component, so following
// labels from any baseline ends at a self-labelled one: when one is left the
// graph is connected, which ends the rounds and skips the union-find pass.
constexpr int kSelf = kRounds, kGate = 2 * kRounds;

__global__ void __launch_bounds__(kBlk) k_lp_zero(int32_t* __restrict__ flags, int32_t* __restrict__ ncomp) {
  if (threadIdx.x < kCompFlags) flags[threadIdx.x] = 0;
  if (threadIdx.x < 4) ncomp[threadIdx.x] = 0;
}

__global__ void __launch_bounds__(kBlk) k_lp_init(int64_t n_b, const int32_t* __restrict__ nvalid_T,
                                                  int32_t* __restrict__ label) {
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < n_b; b += (int64_t)gridDim.x * blockDim.x)
    label[b] = nvalid_T[b] > 0 ? (int32_t)b : INT32_MAX;
}

// Rounds go on while the previous round changed a label and left more than
// one self-labelled baseline.
__device__ __forceinline__ bool lp_done(int r, const int32_t* flags) {
  return r > 0 && (flags[r - 1] == 0 || flags[kSelf + r - 1] <= 1);
}

// Minimum over the `width` lanes (a power of two) of each lane group.
__device__ __forceinline__ int32_t group_min(int32_t x, int width) {
  for (int off = width / 2; off > 0; off >>= 1) x = min(x, __shfl_xor(x, off, 64));
  return x;
}

constexpr int kPixLanes = 8;    // lanes per pixel in the pixel sweep (8 pixels per wavefront)
constexpr int kBaseLanes = 16;  // lanes per baseline in the baseline sweep (4 baselines per wavefront)

// Round r, pixel side: pmin[c] = smallest label of the baselines of valid pixel c.
__global__ void __launch_bounds__(kBlk) k_lp_pix(int r, int64_t n_obs, const int64_t* __restrict__ elem_start,
                                                 const int32_t* __restrict__ eb, const uint8_t* __restrict__ valid,
                                                 const int32_t* __restrict__ label, int32_t* __restrict__ pmin,
                                                 const int32_t* __restrict__ flags) {
  if (lp_done(r, flags)) return;
  const int sub = threadIdx.x % kPixLanes;
  const int64_t ngroup = (int64_t)gridDim.x * (kBlk / kPixLanes);
  for (int64_t cb = ((int64_t)blockIdx.x * (kBlk / kPixLanes) + threadIdx.x / kPixLanes); cb - (cb % (64 / kPixLanes)) < n_obs;
       cb += ngroup) {
    const int64_t c = cb;
    const bool on = c < n_obs && (valid[c] & 1);
    int32_t mn = INT32_MAX;
    if (on) {
      const int64_t e0 = elem_start[c], e1 = elem_start[c + 1];
      if (sub == 0) mn = label[eb[e1 - 1]];
      for (int64_t e = e0 + (int64_t)sub * kStride; e < e1; e += kPixLanes * kStride) mn = min(mn, label[eb[e]]);
    }
    mn = group_min(mn, kPixLanes);
    if (on && sub == 0) pmin[c] = mn;
  }
}

// Round r, baseline side: label[b] = min(label[b], pmin of b's valid pixels);
// flags[r] marks a change.  Time-order elements of baseline b: runs
// bstart[b] .. bstart[b + 1] - 1 with keys c << nb | length - 1 (c when
// nb = 0), or, without runs, samples b L .. (b + 1) L - 1 with compact pixels
// cpix (-1 masked).
__global__ void __launch_bounds__(kBlk) k_lp_base(int r, int64_t n_b, const uint32_t* __restrict__ bstart,
                                                  const uint32_t* __restrict__ tkey, int nb,
                                                  const int32_t* __restrict__ cpix, int64_t L, int64_t n_t,
                                                  const uint8_t* __restrict__ valid, const int32_t* __restrict__ pmin,
                                                  int32_t* __restrict__ label, int32_t* __restrict__ flags) {
  if (lp_done(r, flags)) return;
  __shared__ int32_t s_self;
  if (threadIdx.x == 0) s_self = 0;
  __syncthreads();
  int32_t self = 0;
  const int sub = threadIdx.x % kBaseLanes;
  const int64_t ngroup = (int64_t)gridDim.x * (kBlk / kBaseLanes);
  for (int64_t bb = ((int64_t)blockIdx.x * (kBlk / kBaseLanes) + threadIdx.x / kBaseLanes);
       bb - (bb % (64 / kBaseLanes)) < n_b; bb += ngroup) {
    const int64_t b = bb;
    const bool on = b < n_b;
    int32_t mn = INT32_MAX;
    if (on) {
      int64_t e0, e1;
      if (bstart) {
        e0 = bstart[b];
        e1 = bstart[b + 1];
      } else {
        e0 = b * L;
        e1 = min(n_t, (b + 1) * L);
      }
      for (int64_t e = e0 + (int64_t)sub * kStride; e < e1; e += kBaseLanes * kStride) {
        const int64_t c = bstart ? (int64_t)(nb > 0 ? tkey[e] >> nb : tkey[e]) : (int64_t)cpix[e];
        if (c >= 0 && (valid[c] & 1)) mn = min(mn, pmin[c]);
      }
    }
    mn = group_min(mn, kBaseLanes);
    if (on && sub == 0) {
      const int32_t old = label[b];
      int32_t nw = min(old, mn);
      if (nw < old) nw = min(nw, label[nw]);  // one jump: the new label's own label
      if (nw < old) {
        label[b] = nw;
        flags[r] = 1;
      }
      self += nw == (int32_t)b ? 1 : 0;
    }
  }
  // one atomic per workgroup that still holds a self-labelled baseline
  if (self) atomicAdd(&s_self, self);
  __syncthreads();
  if (threadIdx.x == 0 && s_self) atomicAdd(flags + kSelf + r, s_self);
}

// The union-find forest seeded from the labels; flags[kGate] = 1 when the
// pass over all elements is needed (the last round that ran left more than
// one self-labelled baseline; every round that runs leaves at least one when
// any baseline holds a valid sample).
__global__ void __launch_bounds__(kBlk) k_lp_seed(int64_t n_b, const int32_t* __restrict__ label,
                                                  int32_t* __restrict__ parent, int32_t* __restrict__ flags) {
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < n_b; b += (int64_t)gridDim.x * blockDim.x)
    parent[b] = label[b] < (int32_t)b ? label[b] : (int32_t)b;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    int32_t left = 0;
    for (int r = 0; r < kRounds; ++r)
      if (flags[kSelf + r] > 0) left = flags[kSelf + r];
    flags[kGate] = left > 1 ? 1 : 0;
  }
}


// One wavefront per compact pixel with a valid T block: every element whose
// baseline differs from its predecessor's is linked to the pixel's first
// (nothing to do when the label rounds showed one component: *gate == 0).
// Fast path: a baseline whose parent is already the root of the pixel's
// first baseline is joined (parents only move to ancestors, so any value
// read, even a stale one, that equals that root proves the link).
__global__ void __launch_bounds__(kBlk) k_uf_link(int64_t n_obs, const int64_t* __restrict__ elem_start,
                                                  const int32_t* __restrict__ eb, const uint8_t* __restrict__ valid,
                                                  int32_t* __restrict__ parent, const int32_t* __restrict__ gate) {
  if (*gate == 0) return;
  const int lane = threadIdx.x & 63;
  const int64_t nwave = (int64_t)gridDim.x * (kBlk / 64);
  for (int64_t c = (int64_t)blockIdx.x * (kBlk / 64) + (threadIdx.x >> 6); c < n_obs; c += nwave) {
    if (!(valid[c] & 1)) continue;
    const int64_t e0 = elem_start[c], e1 = elem_start[c + 1];
    if (e1 - e0 < 2) continue;
    const int32_t first = eb[e0];
    const int32_t rf = uf_find(parent, first);
    for (int64_t e = e0 + 1 + lane; e < e1; e += 64) {
      const int32_t b = eb[e];
      if (b != eb[e - 1] && b != rf && uf_load(parent + b) != rf) uf_union(parent, rf, b);
    }
  }
}

// label[b] = root of b for baselines with valid samples (-1 otherwise); roots
// are counted.
__global__ void __launch_bounds__(kBlk) k_uf_label(int64_t n_b, const int32_t* __restrict__ nvalid_T,
                                                   int32_t* __restrict__ parent, int32_t* __restrict__ label,
                                                   int32_t* __restrict__ ncomp) {
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < n_b; b += (int64_t)gridDim.x * blockDim.x) {
    if (nvalid_T[b] > 0) {
      const int32_t r = uf_find(parent, (int32_t)b);
      label[b] = r;
      if (r == (int32_t)b) atomicAdd(ncomp, 1);
    } else {
      label[b] = -1;
    }
  }
}

// Exclusive scan over one workgroup of 1024 threads; returns the exclusive
// prefix of v and writes the total to *total (all threads).
__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* lds, uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  uint32_t inc = v;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(inc, off, 64);
    if (lane >= off) inc += t;
  }
  if (lane == 63) lds[wave] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int w = 0; w < nw; ++w) {
      const uint32_t t = lds[w];
      lds[w] = run;
      run += t;
    }
    lds[32] = run;
  }
  __syncthreads();
  const uint32_t out = lds[wave] + inc - v;
  *total = lds[32];
  __syncthreads();
  return out;
}

// Component lists when there is more than one component (one workgroup of
// 1024 threads; returns at once otherwise).  label[b] becomes the compact
// component id; cursor holds the id of each root, then the fill cursors.
__global__ void __launch_bounds__(1024) k_comp_lists(int64_t n_b, int32_t* __restrict__ label,
                                                     uint32_t* __restrict__ start, uint32_t* __restrict__ member,
                                                     uint32_t* __restrict__ cursor,
                                                     const int32_t* __restrict__ ncomp_dev) {
  const int ncomp = *ncomp_dev;
  if (ncomp <= 1) return;
  __shared__ uint32_t lds[64];
  // compact ids of the roots, in increasing order
  uint32_t run = 0;
  for (int64_t b0 = 0; b0 < n_b; b0 += blockDim.x) {
    const int64_t b = b0 + threadIdx.x;
    const uint32_t f = (b < n_b && dev_load(label + b) == (int32_t)b) ? 1u : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(f, lds, &tot);
    if (f) st_u32(cursor + b, run + ex);
    run += tot;
  }
  for (int64_t c = threadIdx.x; c <= ncomp; c += blockDim.x) st_u32(start + c, 0u);
  __syncthreads();
  // relabel with the compact id (each thread reads and writes only its own
  // label; the roots' ids stay in cursor) and count the members
  for (int64_t b = threadIdx.x; b < n_b; b += blockDim.x) {
    const int32_t r = dev_load(label + b);
    if (r >= 0) {
      const uint32_t c = ld_u32(cursor + r);
      dev_store(label + b, (int32_t)c);
      atomicAdd(start + c, 1u);
    }
  }
  __syncthreads();
  // counts -> offsets
  run = 0;
  for (int64_t c0 = 0; c0 <= ncomp; c0 += blockDim.x) {
    const int64_t c = c0 + threadIdx.x;
    const uint32_t v = c < ncomp ? ld_u32(start + c) : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(v, lds, &tot);
    if (c <= ncomp) st_u32(start + c, run + ex);
    run += tot;
  }
  __syncthreads();
  for (int64_t c = threadIdx.x; c < ncomp; c += blockDim.x) st_u32(cursor + c, ld_u32(start + c));
  __syncthreads();
  // members in increasing baseline order: wavefront 0 takes 64 baselines at a
  // time; lanes of one component get consecutive slots in lane order
  if (threadIdx.x >= 64) return;
  const int lane = threadIdx.x;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  for (int64_t b0 = 0; b0 < n_b; b0 += 64) {
    const int64_t b = b0 + lane;
    const int32_t c = b < n_b ? dev_load(label + b) : -1;
    bool pending = c >= 0;
    while (__ballot(pending)) {
      const uint64_t pm = __ballot(pending);
      const int leader = __ffsll((unsigned long long)pm) - 1;
      const int32_t lc = __shfl(c, leader, 64);
      const bool mine = pending && c == lc;
      const uint64_t mm = __ballot(mine);
      // the leader takes the component's next slots (read-modify-write, so
      // later chunks see every earlier update)
      uint32_t base = lane == leader ? atomicAdd(cursor + lc, (uint32_t)__popcll(mm)) : 0u;
      base = __shfl(base, leader, 64);
      if (mine) {
        st_u32(member + base + __popcll(mm & below), (uint32_t)b);
        pending = false;
      }
    }
  }
}

__global__ void __launch_bounds__(1024) k_comp_project(CompView cv, double* __restrict__ x, int64_t sb, int Rp) {
  __shared__ double lds[16 * 64];
  const int ncomp = *cv.ncomp;
  if (ncomp <= 1) return;
  (void)comp_project_block(cv, ncomp, x, nullptr, sb, Rp, lds);
}

unsigned grid_of(int64_t n, int64_t per, unsigned cap) {
  int64_t g = (n + per - 1) / per;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

}  // namespace

hipError_t launch_components(int64_t n_b, int64_t n_obs, const int64_t* elem_start, const int32_t* eb,
                             const uint8_t* valid, const int32_t* nvalid_T, const ChainSource& cs, Comp& C,
                             hipStream_t st) {
  const unsigned gb = grid_of(n_b, kBlk, 4096);
  hipLaunchKernelGGL(k_lp_zero, dim3(1), dim3(kBlk), 0, st, C.flags, C.ncomp);
  hipLaunchKernelGGL(k_lp_init, dim3(gb), dim3(kBlk), 0, st, n_b, nvalid_T, C.label);
  for (int r = 0; r < kRounds; ++r) {
    if (n_obs > 0)
      hipLaunchKernelGGL(k_lp_pix, dim3(grid_of(n_obs, kBlk / kPixLanes, 65536)), dim3(kBlk), 0, st, r, n_obs,
                         elem_start, eb, valid, C.label, C.pmin, C.flags);
    hipLaunchKernelGGL(k_lp_base, dim3(grid_of(n_b, kBlk / kBaseLanes, 65536)), dim3(kBlk), 0, st, r, n_b, cs.bstart,
                       cs.tkey, cs.nb, cs.cpix, cs.L, cs.n_t, valid, C.pmin, C.label, C.flags);
  }
  hipLaunchKernelGGL(k_lp_seed, dim3(gb), dim3(kBlk), 0, st, n_b, C.label, C.parent, C.flags);
  if (n_obs > 0)
    hipLaunchKernelGGL(k_uf_link, dim3(grid_of(n_obs, kBlk / 64, 65536)), dim3(kBlk), 0, st, n_obs, elem_start, eb,
                       valid, C.parent, C.flags + kGate);
  hipLaunchKernelGGL(k_uf_label, dim3(gb), dim3(kBlk), 0, st, n_b, nvalid_T, C.parent, C.label, C.ncomp);
  hipLaunchKernelGGL(k_comp_lists, dim3(1), dim3(1024), 0, st, n_b, C.label, C.start, C.member, C.cursor, C.ncomp);
  return hipGetLastError();
}

hipError_t launch_comp_project(const CompView& cv, double* x, int64_t sb, int Rp, hipStream_t st) {
  if (!cv.ncomp) return hipSuccess;
  hipLaunchKernelGGL(k_comp_project, dim3(1), dim3(1024), 0, st, cv, x, sb, Rp);
  return hipGetLastError();
}

}  // namespace dst
