// C-ABI layer of the destriping library: argument checks, workspace, the
// pointing setup shared by every entry point, and the PCG driver of the
// destriping equation (Eq. 13 of arXiv:1309.5609, solved as the closing
// paragraph of its Algorithm section describes: by an iterative solver that
// only applies the operator).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <string>
#include <map>
#include <tuple>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "dst.h"
#include "dst_comp.h"
#include "dst_group.h"
#include "dst_internal.h"
#include "dst_multi.h"
#include "dst_pixel.h"
#include "dst_runs.h"

using dst::CgCtl;
using dst::View;

constexpr int kMaxGroup = 64;  // problems advanced together by one group of launches

struct dst_ctx {
  int device = 0;
  std::string err;
  struct Buf {
    void* ptr = nullptr;
    size_t bytes = 0;
  };
  std::unordered_map<std::string, Buf> ws;
  std::string ws_prefix;      // prepended to slot names (one namespace per problem of a group)
  std::unordered_set<std::string> ws_shared;  // slots that stay unprefixed (setup-only arrays)
  CgCtl* ctl_host = nullptr;  // pinned mirror of the device CG scalars
  int* err_host = nullptr;    // pinned mirror of the device error flag
  int* err_dev = nullptr;     // device error flag (sticky: set by kernels, cleared when reported)
  unsigned char* scratch = nullptr;  // device address of this device's fixed scratch (dst_bin_noalloc)
  // pinned mirrors of the setup's four counts and of the true residual norm
  struct Readback {
    unsigned long long counts[4];
    int32_t ncomp[4];
    double rnorm;
  };
  Readback* rb_host = nullptr;
  dst::MultiCtl* mctl_host = nullptr;  // pinned mirror of the batched CG state
  CgCtl* gctl_host = nullptr;          // pinned mirrors of the CG scalars of a problem group [kMaxGroup]
  // GMRES status written by the kernels into pinned memory: slots 0, 1 for
  // alternate Arnoldi steps, slot 2 for the end of a cycle; gm_dev is the
  // device's address of the same memory; gm_ev marks the steps.
  dst::GmStatus* gm_host = nullptr;
  dst::GmStatus* gm_dev = nullptr;
  hipEvent_t gm_ev[2] = {nullptr, nullptr};
  // instantiated iteration graphs kept between solves (single solve,
  // shared-pointing batch, problem group), updated in place by each capture
  hipGraphExec_t graphs[3] = {nullptr, nullptr, nullptr};
  hipStream_t cap = nullptr;  // private stream on which iteration graphs are captured
  int unbin_bpw = 4;          // launch shape of the run rescan (baselines per wavefront)
  int bin_lpp = 0;            // launch shape of the run binning (lanes per pixel; 0: default 32)
  int run_split_bits = 0;     // > 0: longest run 2^bits samples (runs split beyond; results unchanged)
  // launch shapes chosen by the autotuner, per problem shape
  std::map<std::tuple<int64_t, int64_t, int, int>, std::pair<int, int>> tuned;
};

namespace {

constexpr int64_t kMaxBaselines = (int64_t)1 << 31;

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

int fail(dst_ctx* ctx, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (ctx) ctx->err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                             \
  do {                                                                                            \
    hipError_t e_ = (expr);                                                                       \
    if (e_ != hipSuccess) return fail(ctx, DST_EHIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                                      __FILE__, __LINE__);                                        \
  } while (0)

#define DST_TRY(expr)         \
  do {                        \
    int rc_ = (expr);         \
    if (rc_ != DST_OK) return rc_; \
  } while (0)

// Device workspace slot `name` (inside the context's current slot prefix),
// grown to at least `bytes`.
int ws_get(dst_ctx* ctx, const char* name, size_t bytes, void** out) {
  if (bytes == 0) bytes = 256;
  auto& b = ctx->ws[(ctx->ws_prefix.empty() || ctx->ws_shared.count(name)) ? std::string(name)
                                                                           : ctx->ws_prefix + name];
  if (b.bytes < bytes) {
    if (b.ptr) (void)hipFree(b.ptr);
    b.ptr = nullptr;
    b.bytes = 0;
    size_t want = (bytes + 255) & ~(size_t)255;
    if (hipMalloc(&b.ptr, want) != hipSuccess) {
      (void)hipGetLastError();
      b.ptr = nullptr;
      return fail(ctx, DST_ENOMEM, "cannot allocate %zu bytes of workspace '%s'", want, name);
    }
    b.bytes = want;
  }
  *out = b.ptr;
  return DST_OK;
}

// Frees slot `name` of the current prefix (no-op when absent).
void ws_release(dst_ctx* ctx, const char* name) {
  auto it = ctx->ws.find(ctx->ws_prefix + name);
  if (it == ctx->ws.end()) return;
  if (it->second.ptr) (void)hipFree(it->second.ptr);
  ctx->ws.erase(it);
}

template <typename T>
int ws(dst_ctx* ctx, const char* name, size_t count, T** out) {
  void* p = nullptr;
  int rc = ws_get(ctx, name, count * sizeof(T), &p);
  *out = static_cast<T*>(p);
  return rc;
}

int stream_rows(uint32_t streams, View& v) {
  v.rowT = v.rowQ = v.rowU = -1;
  v.iqu = 0;
  switch (streams) {
    case DST_T:
      v.rowT = 0;
      v.n_streams = 1;
      return 0;
    case DST_QU:
      v.rowQ = 0;
      v.rowU = 1;
      v.n_streams = 2;
      return 0;
    case DST_TQU:
      v.rowT = 0;
      v.rowQ = 1;
      v.rowU = 2;
      v.n_streams = 3;
      return 0;
    case DST_IQU:
      v.rowT = 0;
      v.n_streams = 1;
      v.iqu = 1;
      return 0;
    default:
      return -1;
  }
}

bool is_dtype(int32_t d) { return d == DST_F32 || d == DST_F64; }

// Checks common to every entry point; fills the kernel view.
int check_problem(dst_ctx* ctx, const dst_problem* prob, bool need_tod, View& v) {
  if (!ctx) return DST_EINVAL;
  if (!prob) return fail(ctx, DST_EINVAL, "problem is NULL");
  if (prob->reserved != 0) return fail(ctx, DST_EINVAL, "problem.reserved must be 0");
  if (prob->n_samples < 1) return fail(ctx, DST_EINVAL, "n_samples must be >= 1 (got %lld)", (long long)prob->n_samples);
  if (prob->n_pix < 1 || prob->n_pix > INT32_MAX)
    return fail(ctx, DST_EINVAL, "n_pix must be in [1, 2^31) (got %lld)", (long long)prob->n_pix);
  if (prob->baseline_length < 1 || prob->baseline_length > INT32_MAX)
    return fail(ctx, DST_EINVAL, "baseline_length must be in [1, 2^31) (got %lld)",
                (long long)prob->baseline_length);
  if (stream_rows(prob->streams, v) != 0)
    return fail(ctx, DST_EINVAL, "streams must be DST_T, DST_QU, DST_TQU or DST_IQU (got %u)", prob->streams);
  if (!prob->pix) return fail(ctx, DST_EINVAL, "pix is NULL");
  if (v.rowQ >= 0 || v.iqu) {
    if (!prob->psi) return fail(ctx, DST_EINVAL, "psi is NULL but the streams need the angle");
    if (!is_dtype(prob->psi_dtype)) return fail(ctx, DST_EINVAL, "psi_dtype must be DST_F32 or DST_F64");
  }
  if (need_tod) {
    if (!prob->tod) return fail(ctx, DST_EINVAL, "tod is NULL");
    if (!is_dtype(prob->tod_dtype)) return fail(ctx, DST_EINVAL, "tod_dtype must be DST_F32 or DST_F64");
  }
  static const char* names[3] = {"w_T", "w_q", "w_u"};
  const int rows[3] = {v.rowT, v.rowQ, v.rowU};
  for (int k = 0; k < 3; ++k) {
    if (rows[k] < 0) continue;
    const double w = prob->weight[k];
    if (!(w > 0.0) || !std::isfinite(w)) return fail(ctx, DST_EINVAL, "%s must be > 0 and finite", names[k]);
  }
  if (!(prob->rcond_cut >= 0.0 && prob->rcond_cut < 1.0))
    return fail(ctx, DST_EINVAL, "rcond_cut must be in [0, 1)");
  const int64_t n_b = (prob->n_samples + prob->baseline_length - 1) / prob->baseline_length;
  if (n_b >= kMaxBaselines) return fail(ctx, DST_EINVAL, "too many baselines (%lld)", (long long)n_b);
  v.pix = prob->pix;
  v.psi = prob->psi;
  v.n_t = prob->n_samples;
  v.n_pix = prob->n_pix;
  v.L = prob->baseline_length;
  v.n_b = n_b;
  for (int k = 0; k < 3; ++k) v.w[k] = rows[k] >= 0 ? prob->weight[k] : 0.0;
  return DST_OK;
}

// Per-pixel and per-baseline data every operator needs.
struct Setup {
  View v;
  int psi_f32 = 0;
  int tod_f32 = 0;
  int32_t* hits = nullptr;
  double* M4 = nullptr;
  double* Minv4 = nullptr;
  uint8_t* valid = nullptr;
  int32_t* nvalid = nullptr;
  double* J = nullptr;
  unsigned long long* counts = nullptr;  // [0..1] valid pixels T/QU, [2..3] valid samples T/QU
  int* err = nullptr;
};

// Hits, blocks, inverse and validity into the buffers S already names
// (hits, M4, Minv4, valid, counts); allocates nothing.
int setup_pixels(dst_ctx* ctx, const dst_problem* prob, Setup& S, double* blocks_out, hipStream_t st) {
  const View& v = S.v;
  S.psi_f32 = prob->psi_dtype == DST_F32;
  S.tod_f32 = prob->tod_dtype == DST_F32;
  S.err = ctx->err_dev;
  HIP_TRY(dst::launch_fill_u32(reinterpret_cast<uint32_t*>(S.hits), v.n_pix, 0u, st));
  HIP_TRY(dst::launch_fill(S.M4, 4 * v.n_pix, 0.0, st));
  HIP_TRY(dst::launch_fill_u32(reinterpret_cast<uint32_t*>(S.counts), 8, 0u, st));
  HIP_TRY(dst::launch_pointing(v, S.psi_f32, S.hits, S.M4, S.err, st));
  HIP_TRY(dst::launch_invert(v, S.hits, S.M4, prob->rcond_cut, S.Minv4, S.valid, blocks_out, S.counts, st));
  return DST_OK;
}

int run_setup(dst_ctx* ctx, const dst_problem* prob, Setup& S, bool baselines, double* blocks_out, hipStream_t st) {
  const View& v = S.v;
  DST_TRY(ws(ctx, "hits", v.n_pix, &S.hits));
  DST_TRY(ws(ctx, "M4", 4 * v.n_pix, &S.M4));
  DST_TRY(ws(ctx, "Minv4", 4 * v.n_pix, &S.Minv4));
  DST_TRY(ws(ctx, "valid", v.n_pix, &S.valid));
  DST_TRY(ws(ctx, "counts", 4, &S.counts));
  DST_TRY(setup_pixels(ctx, prob, S, blocks_out, st));
  if (baselines) {
    DST_TRY(ws(ctx, "nvalid", 2 * v.n_b, &S.nvalid));
    DST_TRY(ws(ctx, "J", (size_t)v.n_streams * v.n_b, &S.J));
    HIP_TRY(dst::launch_baseline_counts(v, S.valid, S.nvalid, S.J, S.counts + 2, st));
  }
  return DST_OK;
}

// Wait for the stream and report a pixel index out of range found by any
// kernel of this context since the last report (the flag is sticky until
// reported, so asynchronous calls report at the next synchronisation).
int finish(dst_ctx* ctx, const Setup* S, hipStream_t st) {
  (void)S;
  // the error flag rides on the same synchronisation (pinned mirror)
  HIP_TRY(hipMemcpyAsync(ctx->err_host, ctx->err_dev, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (*ctx->err_host) {
    HIP_TRY(dst::launch_fill_u32(reinterpret_cast<uint32_t*>(ctx->err_dev), 4, 0u, st));
    HIP_TRY(hipStreamSynchronize(st));
    *ctx->err_host = 0;
    return fail(ctx, DST_EBOUNDS, "a pixel index >= n_pix was found in the pointing");
  }
  return DST_OK;
}

// End of an asynchronous entry point: launch errors only.
int issued(dst_ctx* ctx) {
  HIP_TRY(hipGetLastError());
  return DST_OK;
}

// [n_pix][4] kernel layout -> [n_pix][3] user layout.
hipError_t copy4to3(double* dst3, const double* src4, int64_t n_pix, hipStream_t st) {
  return hipMemcpy2DAsync(dst3, 3 * sizeof(double), src4, 4 * sizeof(double), 3 * sizeof(double), (size_t)n_pix,
                          hipMemcpyDeviceToDevice, st);
}

int check_bin_args(dst_ctx* ctx, const dst_problem* prob, uint32_t flags, const double* map_out, View& v) {
  DST_TRY(check_problem(ctx, prob, (flags & DST_BIN_USE_TOD) != 0, v));
  if (v.iqu) return fail(ctx, DST_EINVAL, "DST_IQU streams are not supported by this entry point");
  if (!map_out) return fail(ctx, DST_EINVAL, "map_out is NULL");
  if (flags & ~(uint32_t)(DST_BIN_USE_TOD | DST_BIN_MAP)) return fail(ctx, DST_EINVAL, "unknown flags %u", flags);
  return DST_OK;
}

// Binning after the pixel setup: s = A^T W (d - F a) into s4, then the sum
// map or M^-1 s into map_out, and the hits.  Allocates nothing.
int bin_pass(dst_ctx* ctx, const dst_problem* prob, const Setup& S, const double* baselines, uint32_t flags,
             double* s4, double* map_out, int32_t* hits_out, hipStream_t st) {
  const View& v = S.v;
  const bool use_tod = flags & DST_BIN_USE_TOD;
  HIP_TRY(dst::launch_fill(s4, 4 * v.n_pix, 0.0, st));
  if (use_tod || baselines)
    HIP_TRY(dst::launch_bin(v, S.psi_f32, use_tod ? prob->tod : nullptr, S.tod_f32, baselines, -1.0, S.valid, s4,
                            S.err, nullptr, st));
  if (flags & DST_BIN_MAP) {
    HIP_TRY(dst::launch_apply(v.n_pix, s4, S.Minv4, map_out, 3, nullptr, nullptr, st));
  } else {
    HIP_TRY(copy4to3(map_out, s4, v.n_pix, st));
  }
  if (hits_out) HIP_TRY(hipMemcpyAsync(hits_out, S.hits, v.n_pix * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
  return issued(ctx);
}

// Fixed scratch of dst_bin_noalloc: per pixel the hits (4 B), blocks (32 B),
// block inverse (32 B), validity (1 B) and sums (32 B), plus four counters,
// each array on a 256-byte boundary, for up to kNoAllocMaxPix pixels (a full
// N_side 256 sky).  Host code reaches it only through the device address
// hipGetSymbolAddress gives at context creation (dst_ctx::scratch).
constexpr int64_t kNoAllocMaxPix = 12 * 256 * 256;
constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t kScratchBytes = align256(4 * kNoAllocMaxPix) + 2 * align256(32 * kNoAllocMaxPix) +
                                 align256(kNoAllocMaxPix) + align256(32 * kNoAllocMaxPix) + 256;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

void carve_scratch(unsigned char* base, int64_t n_pix, Setup& S, double** s4) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    unsigned char* p = base + off;
    off += align256(bytes);
    return p;
  };
  S.hits = reinterpret_cast<int32_t*>(take(4 * (size_t)n_pix));
  S.M4 = reinterpret_cast<double*>(take(32 * (size_t)n_pix));
  S.Minv4 = reinterpret_cast<double*>(take(32 * (size_t)n_pix));
  S.valid = take((size_t)n_pix);
  *s4 = reinterpret_cast<double*>(take(32 * (size_t)n_pix));
  S.counts = reinterpret_cast<unsigned long long*>(take(4 * sizeof(unsigned long long)));
}


// out = F^T Z x with x = tod + bsign * F base (either may be NULL).
int operator_pass(dst_ctx* ctx, Setup& S, const void* tod, const double* base, double bsign, double* out,
                  hipStream_t st) {
  const View& v = S.v;
  double *s4 = nullptr, *m4 = nullptr;
  DST_TRY(ws(ctx, "s4", 4 * v.n_pix, &s4));
  DST_TRY(ws(ctx, "m4", 4 * v.n_pix, &m4));
  HIP_TRY(dst::launch_fill(s4, 4 * v.n_pix, 0.0, st));
  if (tod || base) HIP_TRY(dst::launch_bin(v, S.psi_f32, tod, S.tod_f32, base, bsign, S.valid, s4, S.err, nullptr, st));
  HIP_TRY(dst::launch_apply(v.n_pix, s4, S.Minv4, m4, 4, nullptr, nullptr, st));
  HIP_TRY(dst::launch_unbin_reduce(v, S.psi_f32, tod, S.tod_f32, base, bsign, m4, S.valid, S.nvalid, out, nullptr,
                                   nullptr, st));
  return DST_OK;
}


// Solver setup: the pixel-major transpose of the pointing with compact pixel
// ids, per-pixel blocks from it (no atomics), and the per-baseline counts and
// Jacobi diagonal.  Every solver kernel works in compact pixel space (S.v has
// pix = the compact ids, n_pix = observed pixels); outputs are scattered back.
struct Plan {
  Setup S;
  View full;
  bool runs = true;       // run-compressed form (default) or per-sample form
  dst::Transpose T;       // per-sample form
  dst::Runs W;            // run form
  double* m4 = nullptr;   // per-iteration map (zero on invalid pixels)
  double* pw4 = nullptr;  // weighted interleaved baseline vector
  int lpp = 0;            // launch shapes of the run binning (0: default) and rescan
  int bpw = 4;
  dst::Comp C;            // components of the baseline-pixel graph (streams with a T-like row)
  int dense_t = 0;        // run form, intensity only: p and m kept as one double per baseline / pixel
  const int32_t* cid() const { return runs ? W.cid : T.cid; }
  dst::CompView cv() const { return C.ncomp ? C.view() : dst::CompView{}; }
};

// Components of the baseline-pixel graph over T-valid samples (after the
// per-baseline counts); elements elem_start / eb in pixel order.
int build_components(dst_ctx* ctx, Plan& P, int64_t n_obs, const int64_t* elem_start, const int32_t* eb,
                     const dst::ChainSource& cs, hipStream_t st) {
  const View& v = P.full;
  if (v.rowT < 0) return DST_OK;
  dst::Comp& C = P.C;
  DST_TRY(ws(ctx, "comp_parent", v.n_b, &C.parent));
  DST_TRY(ws(ctx, "comp_label", v.n_b, &C.label));
  DST_TRY(ws(ctx, "comp_start", v.n_b + 1, &C.start));
  DST_TRY(ws(ctx, "comp_member", v.n_b, &C.member));
  DST_TRY(ws(ctx, "comp_cursor", v.n_b, &C.cursor));
  DST_TRY(ws(ctx, "comp_n", 4, &C.ncomp));
  DST_TRY(ws(ctx, "comp_pmin", std::max<int64_t>(n_obs, 1), &C.pmin));
  DST_TRY(ws(ctx, "comp_flags", dst::kCompFlags, &C.flags));
  HIP_TRY(dst::launch_components(v.n_b, n_obs, elem_start, eb, P.S.valid, P.S.nvalid, cs, C, st));
  return DST_OK;
}

// Run form of the setup: runs in time and pixel order, compact ids in pixel
// order, per-pixel blocks and (with tod) binned map, per-baseline counts and b.
int build_runs_plan(dst_ctx* ctx, const dst_problem* prob, Plan& P, const void* tod, double** sd4, double** md4,
                    double* b, hipStream_t st) {
  Setup& S = P.S;
  const View& v = P.full;
  if ((uint64_t)v.n_t >= ((uint64_t)1 << 32))
    return fail(ctx, DST_EINVAL, "the solver needs n_samples < 2^32 (got %lld)", (long long)v.n_t);
  S.psi_f32 = prob->psi_dtype == DST_F32;
  S.tod_f32 = prob->tod_dtype == DST_F32;
  dst::Runs& W = P.W;
  P.dense_t = (v.rowT >= 0 && v.rowQ < 0 && !v.iqu) ? 1 : 0;
  DST_TRY(ws(ctx, "r_tcount", dst::run_tiles(v.n_t), &W.tcount));
  DST_TRY(ws(ctx, "r_toff", dst::run_tiles(v.n_t), &W.toff));
  size_t tmp_bytes = 0;
  HIP_TRY(dst::runs_tmp_bytes(v.n_t, v.n_pix, v.n_b, &tmp_bytes));
  DST_TRY(ws_get(ctx, "r_tmp", tmp_bytes, &W.tmp));
  W.tmp_bytes = tmp_bytes;
  DST_TRY(ws(ctx, "r_bstart", v.n_b + 1, &W.bstart));
  DST_TRY(ws(ctx, "r_bkey0", v.n_b, &W.bkey[0]));
  DST_TRY(ws(ctx, "r_bkey1", v.n_b, &W.bkey[1]));
  DST_TRY(ws(ctx, "r_bord0", v.n_b, &W.bord[0]));
  DST_TRY(ws(ctx, "r_bord1", v.n_b, &W.bord[1]));
  DST_TRY(ws(ctx, "r_seg", 2 * (size_t)v.n_pix, &W.seg));
  DST_TRY(ws(ctx, "r_pk0", v.n_pix, &W.pk[0]));
  DST_TRY(ws(ctx, "r_pk1", v.n_pix, &W.pk[1]));
  DST_TRY(ws(ctx, "r_pv0", v.n_pix, &W.pv[0]));
  DST_TRY(ws(ctx, "r_pv1", v.n_pix, &W.pv[1]));
  DST_TRY(ws(ctx, "r_nobs", 1, &W.n_obs_dev));
  DST_TRY(ws(ctx, "r_nout", 1, &W.n_out));
  DST_TRY(ws(ctx, "r_cid", v.n_pix, &W.cid));
  DST_TRY(ws(ctx, "r_ccount", v.n_pix + 1, &W.ccount));
  DST_TRY(ws(ctx, "r_pstart", v.n_pix + 1, &W.pstart));
  DST_TRY(ws(ctx, "counts", 4, &S.counts));
  S.err = ctx->err_dev;
  HIP_TRY(dst::launch_fill_u32(reinterpret_cast<uint32_t*>(W.seg), 4 * v.n_pix, 0u, st));
  HIP_TRY(dst::launch_fill_u32(reinterpret_cast<uint32_t*>(W.cid), v.n_pix, 0xffffffffu, st));
  HIP_TRY(dst::launch_fill_u32(reinterpret_cast<uint32_t*>(W.n_obs_dev), 2, 0u, st));
  HIP_TRY(dst::launch_fill_u32(reinterpret_cast<uint32_t*>(W.n_out), 2, 0u, st));
  HIP_TRY(dst::launch_fill_u32(reinterpret_cast<uint32_t*>(S.counts), 8, 0u, st));
  W.split_bits = ctx->run_split_bits;
  HIP_TRY(dst::runs_count(v, W, S.err, st));
  const int64_t R = W.R;
  DST_TRY(ws(ctx, "r_t0", R, &W.t0));
  DST_TRY(ws(ctx, "r_tpix", R, &W.tpix));
  DST_TRY(ws(ctx, "r_tn", R, &W.tn));
  // FP32 angles (mixed precision): run sums of cos 2psi, sin 2psi kept in FP32
  W.f32 = S.psi_f32 && (v.rowQ >= 0 || v.iqu);
  const size_t rsz = W.f32 ? sizeof(float) : sizeof(double);
  DST_TRY(ws_get(ctx, "r_tcs", 2 * R * rsz, &W.tcs));
  // intensity-only problems: one raw sum and a 16-byte record per run
  const bool t_only = v.rowT >= 0 && v.rowQ < 0 && !v.iqu;
  DST_TRY(ws(ctx, "r_raw", (t_only ? 1 : 3) * (size_t)R, &W.raw));
  DST_TRY(ws_get(ctx, "r_rec", (size_t)R * (t_only ? sizeof(dst::RunRecordT) : sizeof(dst::RunRecord)),
                 reinterpret_cast<void**>(&W.rec)));
  DST_TRY(ws(ctx, "r_keys0", R, &W.keys[0]));
  DST_TRY(ws(ctx, "r_keys1", R, &W.keys[1]));
  DST_TRY(ws(ctx, "r_vals0", R, &W.vals[0]));
  DST_TRY(ws(ctx, "r_vals1", R, &W.vals[1]));
  DST_TRY(ws(ctx, "r_pb", R, &W.pb));
  DST_TRY(ws(ctx, "r_tkey", R, &W.tkey));
  DST_TRY(ws(ctx, "r_pkey", R, &W.pkey));
  DST_TRY(ws(ctx, "r_pn", R, &W.pn));
  DST_TRY(ws_get(ctx, "r_pcs", 2 * R * rsz, &W.pcs));
  // per-pixel arrays sized for every pixel (the observed count is known later)
  DST_TRY(ws(ctx, "hits", v.n_pix, &S.hits));
  DST_TRY(ws(ctx, "Minv4", (v.iqu ? 8 : 4) * (size_t)v.n_pix, &S.Minv4));  // IQU: 6 entries of a 3x3 inverse
  DST_TRY(ws(ctx, "valid", v.n_pix, &S.valid));
  DST_TRY(ws(ctx, "m4", 4 * v.n_pix, &P.m4));
  DST_TRY(ws(ctx, "pw4", 4 * v.n_b, &P.pw4));
  DST_TRY(ws(ctx, "nvalid", 2 * v.n_b, &S.nvalid));
  DST_TRY(ws(ctx, "J", (size_t)v.n_streams * v.n_b, &S.J));
  double *s4 = nullptr, *m4d = nullptr;
  if (tod) {
    DST_TRY(ws(ctx, "sd4", 4 * v.n_pix, &s4));
    DST_TRY(ws(ctx, "md4", 4 * v.n_pix, &m4d));
  }
  if (sd4) *sd4 = s4;
  if (md4) *md4 = m4d;
  HIP_TRY(dst::runs_build(v, S.psi_f32, tod, S.tod_f32, prob->rcond_cut, W, S.hits, S.Minv4, S.valid, P.m4, s4, m4d,
                          S.counts, st));
  S.v = v;
  S.v.n_pix = W.n_obs;
  HIP_TRY(dst::launch_rhs_runs(S.v, W, tod, S.tod_f32, m4d, S.valid, S.nvalid, S.J, b, st));
  dst::ChainSource cs;
  cs.bstart = W.bstart;
  cs.tkey = W.nb ? W.tkey : reinterpret_cast<const uint32_t*>(W.tpix);
  cs.nb = W.nb;
  return build_components(ctx, P, W.n_obs, W.pstart, W.pb, cs, st);
}

// With tod: also the sum map sd4, binned map md4 (compact [n_obs][4]) and the
// right-hand side b = F^T W (d - A m_d) ([n_streams][n_b]).
int build_sample_plan(dst_ctx* ctx, const dst_problem* prob, Plan& P, const void* tod, double** sd4,
                      double** md4, double* b, hipStream_t st) {
  Setup& S = P.S;
  const View& v = P.full;
  if ((uint64_t)v.n_t >= ((uint64_t)1 << 32))
    return fail(ctx, DST_EINVAL, "the solver needs n_samples < 2^32 (got %lld)", (long long)v.n_t);
  S.psi_f32 = prob->psi_dtype == DST_F32;
  S.tod_f32 = prob->tod_dtype == DST_F32;
  dst::Transpose& T = P.T;
  DST_TRY(ws(ctx, "keys0", v.n_t, &T.keys[0]));
  DST_TRY(ws(ctx, "keys1", v.n_t, &T.keys[1]));
  DST_TRY(ws(ctx, "vals0", v.n_t, &T.vals[0]));
  DST_TRY(ws(ctx, "vals1", v.n_t, &T.vals[1]));
  DST_TRY(ws(ctx, "pk0", v.n_pix, &T.pk[0]));
  DST_TRY(ws(ctx, "pk1", v.n_pix, &T.pk[1]));
  DST_TRY(ws(ctx, "pv0", v.n_pix, &T.pv[0]));
  DST_TRY(ws(ctx, "pv1", v.n_pix, &T.pv[1]));
  size_t tmp_bytes = 0;
  HIP_TRY(dst::transpose_tmp_bytes(v.n_t, v.n_pix, &tmp_bytes));
  DST_TRY(ws_get(ctx, "sort_tmp", tmp_bytes, &T.tmp));
  T.tmp_bytes = tmp_bytes;
  DST_TRY(ws(ctx, "n_obs", 1, &T.n_obs_dev));
  DST_TRY(ws(ctx, "seg", 2 * (size_t)(v.n_pix + 1), &T.seg));
  DST_TRY(ws(ctx, "cid", v.n_pix, &T.cid));
  DST_TRY(ws(ctx, "chits", v.n_pix + 1, &T.chits));
  DST_TRY(ws(ctx, "cstart", v.n_pix + 1, &T.cstart));
  DST_TRY(ws(ctx, "cperm", v.n_t, &T.cperm));
  DST_TRY(ws(ctx, "sb", v.n_t, &T.sb));
  DST_TRY(ws(ctx, "cpix", v.n_t, &T.cpix));
  const size_t psz = S.psi_f32 ? sizeof(float) : sizeof(double);
  DST_TRY(ws_get(ctx, "spsi", (v.rowQ >= 0 ? (size_t)v.n_t : 1) * psz, &T.spsi));
  DST_TRY(ws(ctx, "counts", 4, &S.counts));
  S.err = ctx->err_dev;
  HIP_TRY(dst::launch_fill_u32(reinterpret_cast<uint32_t*>(T.seg), 4 * (v.n_pix + 1), 0u, st));
  HIP_TRY(dst::launch_fill_u32(reinterpret_cast<uint32_t*>(T.cid), v.n_pix, 0xffffffffu, st));
  HIP_TRY(dst::launch_fill_u32(reinterpret_cast<uint32_t*>(T.n_obs_dev), 2, 0u, st));
  HIP_TRY(dst::launch_fill_u32(reinterpret_cast<uint32_t*>(S.counts), 8, 0u, st));
  HIP_TRY(dst::transpose_build(v, T, S.err, st));
  // compact view: pixel ids are the compact ids, n_pix the observed pixels
  S.v = v;
  S.v.pix = T.cpix;
  S.v.n_pix = T.n_obs;
  const int64_t n_obs = T.n_obs;
  DST_TRY(ws(ctx, "hits", n_obs, &S.hits));
  DST_TRY(ws(ctx, "Minv4", 4 * n_obs, &S.Minv4));
  DST_TRY(ws(ctx, "valid", n_obs, &S.valid));
  DST_TRY(ws(ctx, "m4", 4 * n_obs, &P.m4));
  DST_TRY(ws(ctx, "pw4", 4 * v.n_b, &P.pw4));
  DST_TRY(ws(ctx, "nvalid", 2 * v.n_b, &S.nvalid));
  DST_TRY(ws(ctx, "J", (size_t)v.n_streams * v.n_b, &S.J));
  double *s4 = nullptr, *m4d = nullptr;
  if (tod) {
    DST_TRY(ws(ctx, "sd4", 4 * n_obs, &s4));
    DST_TRY(ws(ctx, "md4", 4 * n_obs, &m4d));
  }
  if (sd4) *sd4 = s4;
  if (md4) *md4 = m4d;
  HIP_TRY(dst::launch_setup_pixels(v, S.psi_f32, T, tod, S.tod_f32, prob->rcond_cut, S.hits, S.Minv4, S.valid, P.m4,
                                   s4, m4d, S.counts, st));
  HIP_TRY(dst::launch_rhs_unbin(S.v, S.psi_f32, tod, S.tod_f32, m4d, S.valid, S.nvalid, S.J, b, st));
  dst::ChainSource cs;
  cs.cpix = T.cpix;
  cs.L = v.L;
  cs.n_t = v.n_t;
  return build_components(ctx, P, T.n_obs, T.cstart, T.sb, cs, st);
}

int build_plan(dst_ctx* ctx, const dst_problem* prob, Plan& P, const void* tod, double** sd4, double** md4,
               double* b, hipStream_t st) {
  P.lpp = ctx->bin_lpp;
  P.bpw = ctx->unbin_bpw;
  if (!P.runs) return build_sample_plan(ctx, prob, P, tod, sd4, md4, b, st);
  DST_TRY(build_runs_plan(ctx, prob, P, tod, sd4, md4, b, st));
  if (P.lpp == 0) {
    const View& v = P.S.v;
    P.lpp = dst::bin_lanes_for(P.W.R, P.W.n_obs, v.rowT >= 0 && v.rowQ < 0 && !v.iqu);
  }
  return DST_OK;
}

// The two halves of K p: m = M^-1 A^T W F p (pixel order), then
// q = F^T W (F p - A m) (time order).  With ctl, the CG partials.
int plan_bin(dst_ctx* ctx, Plan& P, const CgCtl* gate, hipStream_t st) {
  Setup& S = P.S;
  if (P.runs)
    HIP_TRY(dst::launch_bin_runs(S.v, P.W, P.pw4, S.Minv4, S.valid, P.m4, gate, P.lpp, st));
  else
    HIP_TRY(dst::launch_bin_pixel(S.v, S.psi_f32, P.T, P.pw4, S.Minv4, S.valid, P.m4, gate, st));
  return DST_OK;
}

int plan_unbin(dst_ctx* ctx, Plan& P, const double* p, double* q, CgCtl* ctl, double* partials, hipStream_t st) {
  Setup& S = P.S;
  if (P.runs)
    HIP_TRY(dst::launch_unbin_runs(S.v, P.W, P.m4, S.nvalid, p, q, ctl, partials, P.bpw, st));
  else
    HIP_TRY(dst::launch_unbin_cg(S.v, S.psi_f32, P.m4, S.nvalid, p, q, ctl, partials, st));
  return DST_OK;
}

// out = K v = F^T Z F v through the solver's kernels.
int plan_operator(dst_ctx* ctx, Plan& P, const double* vin, double* out, hipStream_t st) {
  Setup& S = P.S;
  HIP_TRY(dst::launch_p_update4(S.v, const_cast<double*>(vin), nullptr, P.pw4, nullptr, 0, P.dense_t, st));
  DST_TRY(plan_bin(ctx, P, nullptr, st));
  DST_TRY(plan_unbin(ctx, P, vin, out, nullptr, nullptr, st));
  return DST_OK;
}

// The iteration kernels read their scalars from device memory and return at
// once after the stop (convergence or the iteration limit, both decided on
// the device), so one graph of check_every iterations, replayed between the
// host's checks, serves the whole solve.
// Captures `reps` calls of body(stream) on the context's private stream into
// the graph kept in ctx->graphs[slot]: the new capture
// updates the kept executable graph in place when its topology is unchanged
// (same kernels in the same order: only arguments and grids differ), which
// costs far less than instantiating it again; otherwise the new graph is
// instantiated and kept.  *exec stays owned by the context.
template <typename F>
int capture_graph_kept(dst_ctx* ctx, int slot, int reps, F&& body, hipGraphExec_t* exec) {
  *exec = nullptr;
  if (!ctx->cap) HIP_TRY(hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal));
  int rc = DST_OK;
  for (int i = 0; i < reps && rc == DST_OK; ++i) rc = body(ctx->cap);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(ctx->cap, &g);
  if (rc != DST_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(ctx, DST_EHIP, "graph capture: %s", hipGetErrorString(e));
  hipGraphExec_t& kept = ctx->graphs[slot];
  if (kept) {
    hipGraphNode_t err_node = nullptr;
    hipGraphExecUpdateResult res = hipGraphExecUpdateError;
    if (hipGraphExecUpdate(kept, g, &err_node, &res) == hipSuccess && res == hipGraphExecUpdateSuccess) {
      (void)hipGraphDestroy(g);
      *exec = kept;
      return DST_OK;
    }
    (void)hipGetLastError();
    (void)hipGraphExecDestroy(kept);
    kept = nullptr;
  }
  const hipError_t e2 = hipGraphInstantiate(&kept, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e2 != hipSuccess) {
    kept = nullptr;
    return fail(ctx, DST_EHIP, "graph instantiation: %s", hipGetErrorString(e2));
  }
  *exec = kept;
  return DST_OK;
}

struct EventSet {
  std::vector<hipEvent_t> ev;
  ~EventSet() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
  hipError_t add(hipEvent_t* out) {
    hipError_t e = hipEventCreate(out);
    if (e == hipSuccess) ev.push_back(*out);
    return e;
  }
};

// Status of one finished right-hand side.
int done_status(int done) {
  switch (done) {
    case dst::DONE_CONVERGED:
      return DST_OK;
    case dst::DONE_BREAKDOWN:
      return DST_EBREAKDOWN;
    case dst::DONE_NAN:
      return DST_ENAN;
    default:
      return DST_ENOCONV;
  }
}

// Worse of two statuses: errors (negative) over the ENOCONV warning over OK.
int worse(int a, int b) {
  if (a < 0) return a;
  if (b < 0) return b;
  return std::max(a, b);
}

bool same_operator(const dst_problem& a, const dst_problem& b) {
  if (a.streams == DST_IQU || b.streams == DST_IQU) return false;  // the batched kernels have no IQU rows
  return a.pix == b.pix && a.psi == b.psi && a.n_samples == b.n_samples && a.n_pix == b.n_pix &&
         a.baseline_length == b.baseline_length && a.streams == b.streams && a.psi_dtype == b.psi_dtype &&
         a.weight[0] == b.weight[0] && a.weight[1] == b.weight[1] && a.weight[2] == b.weight[2] &&
         a.rcond_cut == b.rcond_cut;
}

struct BatchOut {
  double* const* baselines;
  double* const* maps;
  double* const* binned;
  int32_t* const* hits;
  dst_solve_info* infos;
};

// Multi-right-hand-side solve of the problems idx (same pointing, weights and
// cut): shared run setup, one binned map and right-hand side per problem, then
// PCG on every right-hand side at once with per-problem stopping.
int solve_group(dst_ctx* ctx, const dst_problem* problems, const std::vector<int>& idx, const dst_solve_opts& opts,
                int check_every, const BatchOut& out, hipStream_t st, int* status) {
  const dst_problem& p0 = problems[idx[0]];
  const bool profile = opts.flags & DST_SOLVE_PROFILE;
  const bool use_graph = !(opts.flags & (DST_SOLVE_NO_GRAPH | DST_SOLVE_PROFILE));
  View v{};
  DST_TRY(check_problem(ctx, &p0, true, v));
  EventSet evs;
  hipEvent_t ev[4];
  for (auto& e : ev) HIP_TRY(evs.add(&e));
  HIP_TRY(hipEventRecord(ev[0], st));

  // shared pointing setup (runs, compact pixels, blocks, counts, Jacobi)
  Plan P;
  P.full = v;
  P.runs = true;
  DST_TRY(build_runs_plan(ctx, &p0, P, nullptr, nullptr, nullptr, nullptr, st));
  Setup& S = P.S;
  const View& vc = S.v;
  dst::Runs& W = P.W;
  dst::Multi mu;
  mu.R = (int)idx.size();
  mu.Rp = dst::multi_padded(mu.R);
  const int64_t n_obs = W.n_obs;
  const size_t NV = (size_t)v.n_b * v.n_streams * mu.Rp;
  const size_t NM = (size_t)std::max<int64_t>(n_obs, 1) * v.n_streams * mu.Rp;
  uint32_t* ipos;
  double *prs, *braw, *b, *a, *r, *z, *p, *q, *ka, *md, *m, *part, *part2;
  dst::MultiCtl* ctl;
  DST_TRY(ws(ctx, "mb_ipos", (size_t)std::max<int64_t>(W.R, 1), &ipos));
  DST_TRY(ws(ctx, "mb_prs", (size_t)dst::kRunRec * std::max<int64_t>(W.R, 1), &prs));
  DST_TRY(ws(ctx, "mb_braw", NV, &braw));
  DST_TRY(ws(ctx, "mb_b", NV, &b));
  DST_TRY(ws(ctx, "mb_a", NV, &a));
  DST_TRY(ws(ctx, "mb_r", NV, &r));
  DST_TRY(ws(ctx, "mb_z", NV, &z));
  DST_TRY(ws(ctx, "mb_p", NV, &p));
  DST_TRY(ws(ctx, "mb_q", NV, &q));
  DST_TRY(ws(ctx, "mb_ka", NV, &ka));
  DST_TRY(ws(ctx, "mb_md", NM, &md));
  DST_TRY(ws(ctx, "mb_m", NM, &m));
  DST_TRY(ws(ctx, "mb_part", (size_t)dst::multi_unbin_blocks(vc) * 3 * mu.Rp, &part));
  DST_TRY(ws(ctx, "mb_part2", (size_t)std::max(dst::multi_update_blocks(v, mu), 256) * 2 * mu.Rp, &part2));
  DST_TRY(ws(ctx, "mb_ctl", 1, &ctl));
  // With FP32 angles and timelines the iterations keep FP32 copies of p and m
  // for the gathers of the binning and the rescan (sums, the CG and the
  // final outputs stay FP64).
  bool g32 = W.f32 != 0;
  for (int k = 0; k < mu.R; ++k) g32 = g32 && problems[idx[k]].tod_dtype == DST_F32;
  float *p32 = nullptr, *m32 = nullptr;
  if (g32) {
    DST_TRY(ws(ctx, "mb_p32", NV, &p32));
    DST_TRY(ws(ctx, "mb_m32", NM, &m32));
  }
  HIP_TRY(dst::launch_fill(m, NM, 0.0, st));
  HIP_TRY(dst::launch_fill(md, NM, 0.0, st));
  HIP_TRY(dst::launch_fill(braw, NV, 0.0, st));
  HIP_TRY(dst::launch_fill_u32(reinterpret_cast<uint32_t*>(ctl), sizeof(dst::MultiCtl) / 4, 0u, st));

  // per problem: run sums of the data, binned map; then every b at once
  HIP_TRY(dst::launch_run_positions(W, ipos, st));
  // realizations in passes of up to kTodBatch with one timeline dtype
  for (int k = 0; k < mu.R;) {
    const int32_t dt = problems[idx[k]].tod_dtype;
    dst::TodSet tods{};
    int nr = 0;
    while (k + nr < mu.R && nr < dst::kTodBatch && problems[idx[k + nr]].tod_dtype == dt) {
      tods.p[nr] = problems[idx[k + nr]].tod;
      ++nr;
    }
    HIP_TRY(dst::launch_multi_tod(vc, S.psi_f32, tods, nr, dt == DST_F32, W, ipos, S.valid, mu.Rp, k, prs, braw, st));
    HIP_TRY(dst::launch_multi_pixsum(n_obs, vc, W, prs, nr, S.Minv4, mu.Rp, k, md, st));
    k += nr;
  }
  HIP_TRY(dst::launch_multi_unbin(vc, W, mu, dst::UNBIN_RHS, md, S.nvalid, nullptr, braw, b, nullptr, nullptr, st));
  const dst::CompView cv = P.cv();
  const int64_t sbm = (int64_t)v.n_streams * mu.Rp;  // stride of one baseline in the multi layout
  HIP_TRY(dst::launch_comp_project(cv, b, sbm, mu.Rp, st));
  HIP_TRY(dst::launch_multi_start(v, mu, b, a, r, z, p, S.J, ctl, part2, opts.tol, opts.max_iter, st));
  if (g32) HIP_TRY(dst::launch_to_f32(p, p32, (int64_t)NV, st));
  HIP_TRY(hipEventRecord(ev[1], st));
  dst::MultiCtl& h = *ctx->mctl_host;
  HIP_TRY(hipMemcpyAsync(&h, ctl, sizeof(dst::MultiCtl), hipMemcpyDeviceToHost, st));
  DST_TRY(finish(ctx, &S, st));
  unsigned long long counts[4];
  HIP_TRY(hipMemcpy(counts, S.counts, sizeof counts, hipMemcpyDeviceToHost));
  int32_t ncomp = 0;
  if (P.C.ncomp) HIP_TRY(hipMemcpy(&ncomp, P.C.ncomp, sizeof ncomp, hipMemcpyDeviceToHost));
  if (counts[2] + counts[3] == 0) return fail(ctx, DST_EDEGENERATE, "no valid sample in the problem");

  // PCG: bin (m = M^-1 A^T W F p) -> rescan + sums (q = K p, alpha) ->
  // a, r, z (beta) -> p, for every running right-hand side
  EventSet pev;
  auto iteration = [&](hipStream_t s, bool timed) -> int {
    hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
    if (timed) {
      for (auto& x : e) HIP_TRY(pev.add(&x));
      HIP_TRY(hipEventRecord(e[0], s));
    }
    if (g32)
      HIP_TRY(dst::launch_multi_bin(vc, W, mu, p32, S.Minv4, m32, ctl, s));
    else
      HIP_TRY(dst::launch_multi_bin(vc, W, mu, p, S.Minv4, m, ctl, s));
    if (timed) HIP_TRY(hipEventRecord(e[1], s));
    if (g32)
      HIP_TRY(dst::launch_multi_unbin(vc, W, mu, dst::UNBIN_CG, m32, S.nvalid, p, nullptr, q, ctl, part, s));
    else
      HIP_TRY(dst::launch_multi_unbin(vc, W, mu, dst::UNBIN_CG, m, S.nvalid, p, nullptr, q, ctl, part, s));
    if (ncomp > 1) HIP_TRY(dst::launch_multi_comp(v, mu, cv, q, p, ctl, s));
    HIP_TRY(dst::launch_multi_alpha(vc, mu, ctl, part, cv, s));
    if (timed) HIP_TRY(hipEventRecord(e[2], s));
    HIP_TRY(dst::launch_multi_update(v, mu, a, r, z, q, p, S.J, ctl, part2, s));
    HIP_TRY(dst::launch_multi_beta(v, mu, ctl, part2, s));
    HIP_TRY(dst::launch_multi_p(v, mu, p, z, ctl, s, p32));
    if (timed) HIP_TRY(hipEventRecord(e[3], s));
    return DST_OK;
  };
  // check_every iterations captured once, replayed once per check
  struct {
    hipGraphExec_t exec = nullptr;  // kept by the context
  } gg;
  if (use_graph && h.running > 0)
    DST_TRY(capture_graph_kept(ctx, 1, check_every, [&](hipStream_t s) { return iteration(s, false); }, &gg.exec));
  HIP_TRY(hipEventRecord(ev[2], st));
  int launched = 0;
  while (h.running > 0 && launched < opts.max_iter) {
    const int k = std::min(check_every, opts.max_iter - launched);
    if (gg.exec) {
      HIP_TRY(hipGraphLaunch(gg.exec, st));  // check_every iterations (those past the stop return at once)
    } else {
      for (int i = 0; i < k; ++i) DST_TRY(iteration(st, profile));
    }
    launched += k;
    HIP_TRY(hipMemcpyAsync(&h, ctl, sizeof(dst::MultiCtl), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  HIP_TRY(hipEventRecord(ev[3], st));

  // canonical baselines, true residuals, outputs
  if (!(opts.flags & DST_SOLVE_NO_CANON)) {
    HIP_TRY(dst::launch_comp_project(cv, a, sbm, mu.Rp, st));
    HIP_TRY(dst::launch_multi_canonicalise(v, mu, a, S.J, ctl, part2, st));
  }
  HIP_TRY(dst::launch_multi_bin(vc, W, mu, a, S.Minv4, m, nullptr, st));
  HIP_TRY(dst::launch_multi_unbin(vc, W, mu, dst::UNBIN_OPERATOR, m, S.nvalid, a, nullptr, ka, nullptr, nullptr, st));
  HIP_TRY(dst::launch_comp_project(cv, ka, sbm, mu.Rp, st));
  HIP_TRY(dst::launch_multi_resid(v, mu, b, ka, S.J, ctl, part2, st));
  for (int k = 0; k < mu.R; ++k) {
    const int i = idx[k];
    HIP_TRY(dst::launch_multi_extract(v, mu, k, a, out.baselines[i], st));
    if (out.maps && out.maps[i]) HIP_TRY(dst::launch_multi_scatter(v, vc, W.cid, mu, k, md, m, out.maps[i], st));
    if (out.binned && out.binned[i])
      HIP_TRY(dst::launch_multi_scatter(v, vc, W.cid, mu, k, md, nullptr, out.binned[i], st));
    if (out.hits && out.hits[i])
      HIP_TRY(dst::launch_scatter(v.n_pix, W.cid, S.hits, out.hits[i], md, nullptr, nullptr, st));
  }
  HIP_TRY(hipMemcpyAsync(&h, ctl, sizeof(dst::MultiCtl), hipMemcpyDeviceToHost, st));
  DST_TRY(finish(ctx, &S, st));

  int max_it = 0;
  for (int k = 0; k < mu.R; ++k) max_it = std::max(max_it, h.iter[k]);
  float t_setup = 0.f, t_iter = 0.f, t_total = 0.f;
  HIP_TRY(hipEventElapsedTime(&t_setup, ev[0], ev[1]));
  HIP_TRY(hipEventElapsedTime(&t_iter, ev[2], ev[3]));
  HIP_TRY(hipEventElapsedTime(&t_total, ev[0], ev[3]));
  double tk[3] = {0.0, 0.0, 0.0};
  if (profile && !pev.ev.empty()) {
    const size_t n_it = pev.ev.size() / 4;
    const size_t used = std::min<size_t>(n_it, (size_t)max_it);
    for (size_t i = 0; i < used; ++i)
      for (int j = 0; j < 3; ++j) {
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, pev.ev[4 * i + j], pev.ev[4 * i + j + 1]));
        tk[j] += t;
      }
    for (auto& x : tk) x = used ? x / used : 0.0;
  }
  for (int k = 0; k < mu.R; ++k) {
    *status = worse(*status, done_status(h.done[k]));
    if (!out.infos) continue;
    dst_solve_info& in = out.infos[idx[k]];
    in = dst_solve_info{};
    in.iterations = h.iter[k];
    in.converged = h.done[k] == dst::DONE_CONVERGED;
    in.b_norm = h.b_norm[k];
    in.rel_residual = h.b_norm[k] > 0.0 ? h.r_norm[k] / h.b_norm[k] : 0.0;
    in.true_rel_residual = h.b_norm[k] > 0.0 ? h.true_norm[k] / h.b_norm[k] : 0.0;
    in.n_valid_pix[0] = (int64_t)counts[0];
    in.n_valid_pix[1] = (int64_t)counts[1];
    in.n_valid_samples[0] = (int64_t)counts[2];
    in.n_valid_samples[1] = (int64_t)counts[3];
    in.n_components = ncomp;
    in.t_setup_ms = t_setup;
    in.t_iter_ms = max_it > 0 ? t_iter / max_it : 0.0;
    in.t_total_ms = t_total;
    in.t_bin_ms = tk[0];
    in.t_unbin_ms = tk[1];
    in.t_update_ms = tk[2];
    in.n_runs = W.R;
  }
  return DST_OK;
}

// Baselines per wavefront of a group's rescan for problems of one kind.
int group_bpw(const dst_ctx* ctx, int kind) {
  (void)kind;
  const int b = ctx->unbin_bpw;
  return (b == 1 || b == 2 || b == 8) ? b : 4;
}

// Independent problems with different pointing (the channels of a survey)
// solved together: each problem gets its own run setup, right-hand side and
// PCG state (workspace slots under its own prefix; the setup-only arrays are
// freed once built), then every iteration advances all of them with one
// launch per phase (bin, rescan, step length, update, beta, p) over one
// list of workgroups, replayed from one captured graph; a problem that has
// stopped leaves its workgroups idle.  Outputs as dst_solve per problem.
int solve_uneven(dst_ctx* ctx, const dst_problem* problems, const std::vector<int>& idx, const dst_solve_opts& opts,
                 int check_every, const BatchOut& out, hipStream_t st, int* status) {
  const int n = (int)idx.size();
  const bool profile = opts.flags & DST_SOLVE_PROFILE;
  const bool use_graph = !(opts.flags & (DST_SOLVE_NO_GRAPH | DST_SOLVE_PROFILE));
  struct Member {
    Plan P;
    View v;
    double *b = nullptr, *a = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *ka = nullptr;
    double *part = nullptr, *part2 = nullptr, *rnorm = nullptr, *sd4 = nullptr, *md4 = nullptr;
    CgCtl* ctl = nullptr;
    std::string prefix;
    unsigned long long counts[4] = {0, 0, 0, 0};
    int32_t ncomp = 0;
  };
  std::vector<Member> M(n);
  EventSet evs;
  hipEvent_t ev[4];
  for (auto& e : ev) HIP_TRY(evs.add(&e));
  HIP_TRY(hipEventRecord(ev[0], st));
  struct PrefixGuard {
    dst_ctx* c;
    ~PrefixGuard() {
      c->ws_prefix.clear();
      c->ws_shared.clear();
    }
  } pg{ctx};
  CgCtl* ctls = nullptr;
  {
    ctx->ws_prefix.clear();
    DST_TRY(ws(ctx, "grp_ctl", kMaxGroup, &ctls));
  }
  // arrays only the setup reads: one set serves every problem's setup in turn
  for (const char* name : {"r_tcount", "r_toff", "r_rec", "r_raw", "r_keys0", "r_keys1", "r_vals0", "r_vals1",
                           "r_t0", "r_tmp", "r_pb", "r_pn", "r_tpix", "r_tn", "r_seg", "r_pk0", "r_pk1", "r_bkey0",
                           "r_bkey1", "r_nobs", "r_nout", "r_ccount", "sd4", "comp_parent", "comp_cursor", "comp_pmin", "comp_flags", "counts"})
    ctx->ws_shared.insert(name);
  for (int k = 0; k < n; ++k) {
    Member& m = M[k];
    const dst_problem& pr = problems[idx[k]];
    DST_TRY(check_problem(ctx, &pr, true, m.v));
    m.prefix = "grp" + std::to_string(k) + "/";
    ctx->ws_prefix = m.prefix;
    const View& v = m.v;
    const int64_t N = (int64_t)v.n_streams * v.n_b;
    m.P.full = v;
    m.P.runs = true;
    m.P.lpp = 32;
    m.P.bpw = 4;
    DST_TRY(ws(ctx, "cg_b", N, &m.b));
    DST_TRY(build_runs_plan(ctx, &pr, m.P, pr.tod, &m.sd4, &m.md4, m.b, st));
    if (m.P.W.nb <= 0) return fail(ctx, DST_EHIP, "problem %d: run keys do not pack (internal)", idx[k]);
    DST_TRY(ws(ctx, "cg_a", N, &m.a));
    DST_TRY(ws(ctx, "cg_r", N, &m.r));
    DST_TRY(ws(ctx, "cg_z", N, &m.z));
    DST_TRY(ws(ctx, "cg_p", N, &m.p));
    DST_TRY(ws(ctx, "cg_q", N, &m.q));
    DST_TRY(ws(ctx, "cg_ka", N, &m.ka));
    const View& vc = m.P.S.v;
    DST_TRY(ws(ctx, "cg_part", 3 * (size_t)std::max<int64_t>({(int64_t)dst::group_unbin_blocks(vc, 1), v.n_b, 4096}),
               &m.part));
    DST_TRY(ws(ctx, "cg_part2", 2 * (size_t)dst::group_vec_blocks(v), &m.part2));
    DST_TRY(ws(ctx, "cg_rnorm", 1, &m.rnorm));
    m.ctl = ctls + k;
    HIP_TRY(dst::launch_fill_u32(reinterpret_cast<uint32_t*>(m.ctl), sizeof(CgCtl) / 4, 0u, st));
    const dst::CompView cv = m.P.cv();
    HIP_TRY(dst::launch_comp_project(cv, m.b, 1, 1, st));
    HIP_TRY(dst::launch_cg_start(v, m.b, nullptr, nullptr, m.a, m.r, m.z, m.p, m.P.S.J, m.ctl, m.part, opts.tol,
                                 opts.max_iter, st));
    HIP_TRY(dst::launch_p_update4(v, m.p, nullptr, m.P.pw4, nullptr, 0, m.P.dense_t, st));
    HIP_TRY(hipMemcpyAsync(m.counts, m.P.S.counts, sizeof m.counts, hipMemcpyDeviceToHost, st));
    if (m.P.C.ncomp) HIP_TRY(hipMemcpyAsync(&m.ncomp, m.P.C.ncomp, sizeof m.ncomp, hipMemcpyDeviceToHost, st));
    DST_TRY(finish(ctx, &m.P.S, st));
  }
  ctx->ws_prefix.clear();
  ctx->ws_shared.clear();
  for (int k = 0; k < n; ++k)
    if (M[k].counts[2] + M[k].counts[3] == 0)
      return fail(ctx, DST_EDEGENERATE, "problem %d: no valid sample in the problem", idx[k]);

  // the group's work list, problems ordered by kind: per problem its arrays
  // and its workgroup ranges
  auto kind_of = [](const View& v) {
    return v.iqu ? dst::GK_IQU : (v.rowT >= 0 && v.rowQ >= 0 ? dst::GK_TQU : (v.rowQ >= 0 ? dst::GK_QU : dst::GK_T));
  };
  std::vector<int> order(n);
  for (int k = 0; k < n; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return kind_of(M[x].P.S.v) < kind_of(M[y].P.S.v); });
  std::vector<dst::GroupProblem> gp(n);
  std::vector<int64_t> n_runs(n);
  std::vector<uint32_t> vec_start(n + 1, 0u);
  std::vector<uint32_t> ranges;  // per kind: bin starts [count + 1], then rescan starts [count + 1]
  dst::GroupLaunch G;
  int f32 = -1;
  for (int o = 0; o < n; ++o) {
    Member& m = M[order[o]];
    const Setup& S = m.P.S;
    const dst::Runs& W = m.P.W;
    dst::GroupProblem& g = gp[o];
    n_runs[o] = W.R;
    g.v = S.v;
    g.kind = kind_of(S.v);
    g.nb = W.nb;
    g.dense_t = m.P.dense_t;
    g.unbin_n = dst::group_unbin_blocks(S.v, group_bpw(ctx, g.kind));
    g.vec_n = dst::group_vec_blocks(S.v);
    g.pstart = W.pstart;
    g.pkey = W.pkey;
    g.pcs = W.pcs;
    g.bstart = W.bstart;
    g.border = W.border;
    g.tkey = W.tkey;
    g.tcs = W.tcs;
    g.Minv4 = S.Minv4;
    g.valid = S.valid;
    g.m4 = m.P.m4;
    g.pw4 = m.P.pw4;
    g.nvalid = S.nvalid;
    g.J = S.J;
    g.a = m.a;
    g.r = m.r;
    g.z = m.z;
    g.p = m.p;
    g.q = m.q;
    g.ctl = m.ctl;
    g.part_unbin = m.part;
    g.part_update = m.part2;
    g.cv = m.P.cv();
    if (g.kind != dst::GK_T) {
      if (f32 >= 0 && f32 != (int)W.f32) return fail(ctx, DST_EINVAL, "internal: mixed angle precision in a group");
      f32 = (int)W.f32;
    }
    vec_start[o + 1] = vec_start[o] + g.vec_n;
    dst::GroupSlice& sl = G.kind[g.kind];
    if (sl.count++ == 0) sl.first = o;
  }
  std::vector<size_t> roff(4, 0);
  for (int K = 0; K < 4; ++K) {
    dst::GroupSlice& sl = G.kind[K];
    if (sl.count == 0) continue;
    // lanes per pixel of the kind's binning from its runs per observed pixel
    int64_t runs = 0, obs = 0;
    for (int j = 0; j < sl.count; ++j) {
      runs += n_runs[sl.first + j];
      obs += gp[sl.first + j].v.n_pix;
    }
    sl.lpp = dst::bin_lanes_for(runs, obs, K == dst::GK_T);
    sl.bpw = group_bpw(ctx, K);
    if (ctx->bin_lpp == 4 || ctx->bin_lpp == 8 || ctx->bin_lpp == 16 || ctx->bin_lpp == 32) sl.lpp = ctx->bin_lpp;
    roff[K] = ranges.size();
    ranges.resize(ranges.size() + 2 * (sl.count + 1), 0u);
    uint32_t* bs = ranges.data() + roff[K];
    uint32_t* us = bs + sl.count + 1;
    for (int j = 0; j < sl.count; ++j) {
      const dst::GroupProblem& g = gp[sl.first + j];
      bs[j + 1] = bs[j] + dst::group_bin_blocks(g.v.n_pix, sl.lpp);
      us[j + 1] = us[j] + g.unbin_n;
    }
    sl.bin_total = bs[sl.count];
    sl.unbin_total = us[sl.count];
  }
  dst::GroupProblem* gp_dev = nullptr;
  uint32_t *vec_dev = nullptr, *ranges_dev = nullptr;
  DST_TRY(ws(ctx, "grp_desc", n, &gp_dev));
  DST_TRY(ws(ctx, "grp_vec", n + 1, &vec_dev));
  DST_TRY(ws(ctx, "grp_ranges", std::max<size_t>(ranges.size(), 1), &ranges_dev));
  HIP_TRY(hipMemcpyAsync(gp_dev, gp.data(), n * sizeof(dst::GroupProblem), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(vec_dev, vec_start.data(), (n + 1) * sizeof(uint32_t), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(ranges_dev, ranges.data(), ranges.size() * sizeof(uint32_t), hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  G.prob = gp_dev;
  G.n = n;
  G.vec_start = vec_dev;
  G.vec_total = vec_start[n];
  G.f32 = f32 > 0 ? 1 : 0;
  for (int K = 0; K < 4; ++K) {
    dst::GroupSlice& sl = G.kind[K];
    if (sl.count == 0) continue;
    sl.bin_start = ranges_dev + roff[K];
    sl.unbin_start = sl.bin_start + sl.count + 1;
  }
  HIP_TRY(hipEventRecord(ev[1], st));

  CgCtl* h = ctx->gctl_host;
  HIP_TRY(hipMemcpyAsync(h, ctls, n * sizeof(CgCtl), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  auto running = [&]() {
    for (int k = 0; k < n; ++k)
      if (h[k].done == dst::DONE_RUNNING) return true;
    return false;
  };
  EventSet pev;
  auto iteration = [&](hipStream_t s, bool timed) -> int {
    if (!timed) {
      HIP_TRY(dst::launch_group_iteration(G, s));
      return DST_OK;
    }
    hipEvent_t e[4];
    for (auto& x : e) HIP_TRY(pev.add(&x));
    HIP_TRY(hipEventRecord(e[0], s));
    for (int phase = 0; phase < 3; ++phase) {
      HIP_TRY(dst::launch_group_phase(G, phase, s));
      HIP_TRY(hipEventRecord(e[phase + 1], s));
    }
    return DST_OK;
  };
  struct {
    hipGraphExec_t exec = nullptr;  // kept by the context
  } gg;
  if (use_graph && running())
    DST_TRY(capture_graph_kept(ctx, 2, check_every, [&](hipStream_t s) { return iteration(s, false); }, &gg.exec));
  HIP_TRY(hipEventRecord(ev[2], st));
  int launched = 0;
  while (running() && launched < opts.max_iter) {
    const int k = std::min(check_every, opts.max_iter - launched);
    if (gg.exec) {
      HIP_TRY(hipGraphLaunch(gg.exec, st));  // check_every iterations (those past the stop return at once)
    } else {
      for (int i = 0; i < k; ++i) DST_TRY(iteration(st, profile));
    }
    launched += k;
    HIP_TRY(hipMemcpyAsync(h, ctls, n * sizeof(CgCtl), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  HIP_TRY(hipEventRecord(ev[3], st));
  std::vector<CgCtl> fin(h, h + n);

  // per problem: canonical baselines, true residual, outputs
  for (int k = 0; k < n; ++k) {
    Member& m = M[k];
    const int i = idx[k];
    ctx->ws_prefix = m.prefix;
    const View& v = m.v;
    const int64_t N = (int64_t)v.n_streams * v.n_b;
    const dst::CompView cv = m.P.cv();
    if (!(opts.flags & DST_SOLVE_NO_CANON)) {
      HIP_TRY(dst::launch_comp_project(cv, m.a, 1, 1, st));
      HIP_TRY(dst::launch_canonicalise(v, m.a, m.P.S.J, m.part, m.ctl, st));
    }
    DST_TRY(plan_operator(ctx, m.P, m.a, m.ka, st));
    HIP_TRY(dst::launch_comp_project(cv, m.ka, 1, 1, st));
    HIP_TRY(dst::launch_residual_norm(v, m.b, m.ka, m.P.S.J, m.ctl, m.part, m.rnorm, st));
    HIP_TRY(hipMemcpyAsync(out.baselines[i], m.a, N * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (out.maps && out.maps[i])
      HIP_TRY(dst::launch_scatter(v.n_pix, m.P.cid(), nullptr, nullptr, m.md4, m.P.m4, out.maps[i], st, m.P.dense_t));
    if (out.binned && out.binned[i])
      HIP_TRY(dst::launch_scatter(v.n_pix, m.P.cid(), nullptr, nullptr, m.md4, nullptr, out.binned[i], st));
    if (out.hits && out.hits[i])
      HIP_TRY(dst::launch_scatter(v.n_pix, m.P.cid(), m.P.S.hits, out.hits[i], m.md4, nullptr, nullptr, st));
  }
  ctx->ws_prefix.clear();
  std::vector<double> rn(n, 0.0);
  for (int k = 0; k < n; ++k) HIP_TRY(hipMemcpyAsync(&rn[k], M[k].rnorm, sizeof(double), hipMemcpyDeviceToHost, st));
  DST_TRY(finish(ctx, nullptr, st));

  int max_it = 0;
  for (int k = 0; k < n; ++k) max_it = std::max(max_it, fin[k].iter);
  float t_setup = 0.f, t_iter = 0.f, t_total = 0.f;
  HIP_TRY(hipEventElapsedTime(&t_setup, ev[0], ev[1]));
  HIP_TRY(hipEventElapsedTime(&t_iter, ev[2], ev[3]));
  HIP_TRY(hipEventElapsedTime(&t_total, ev[0], ev[3]));
  double tk[3] = {0.0, 0.0, 0.0};
  if (profile && !pev.ev.empty()) {
    const size_t used = std::min<size_t>(pev.ev.size() / 4, (size_t)max_it);
    for (size_t it = 0; it < used; ++it)
      for (int j = 0; j < 3; ++j) {
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, pev.ev[4 * it + j], pev.ev[4 * it + j + 1]));
        tk[j] += t;
      }
    for (auto& x : tk) x = used ? x / used : 0.0;
  }
  for (int k = 0; k < n; ++k) {
    const CgCtl& f = fin[k];
    *status = worse(*status, done_status(f.done));
    if (!out.infos) continue;
    dst_solve_info& in = out.infos[idx[k]];
    in = dst_solve_info{};
    in.iterations = f.iter;
    in.converged = f.done == dst::DONE_CONVERGED;
    in.b_norm = f.b_norm;
    in.rel_residual = f.b_norm > 0.0 ? f.r_norm / f.b_norm : 0.0;
    in.true_rel_residual = f.b_norm > 0.0 ? rn[k] / f.b_norm : 0.0;
    in.n_valid_pix[0] = (int64_t)M[k].counts[0];
    in.n_valid_pix[1] = (int64_t)M[k].counts[1];
    in.n_valid_samples[0] = (int64_t)M[k].counts[2];
    in.n_valid_samples[1] = (int64_t)M[k].counts[3];
    in.n_components = M[k].ncomp;
    in.t_setup_ms = t_setup;
    in.t_iter_ms = max_it > 0 ? t_iter / max_it : 0.0;
    in.t_total_ms = t_total;
    in.t_bin_ms = tk[0];
    in.t_unbin_ms = tk[1];
    in.t_update_ms = tk[2];
    in.n_runs = M[k].P.W.R;
  }
  return DST_OK;
}

// Restarted GMRES on K a = b (Eq. 13), right-preconditioned by the Jacobi
// diagonal J, with the same T null-space projection as the PCG (b and every
// K v lose their mean over T-valid baselines, and their component means
// first when the baseline-pixel graph has several components: cv set).
// Arnoldi by classical Gram-Schmidt with one reorthogonalisation; the
// coefficients, rotations and triangular solve stay on the device (GmState).
// The host enqueues the steps of a cycle and, while the GPU runs step j,
// reads the status that step j - 1 wrote into pinned memory, so it stops
// enqueueing one step after the stop with no idle GPU in between; the cycle's
// end (solution update, restart residual) is followed by one wait.  On entry
// b is projected, a holds a0 (or 0), r = b - P K a0 and ctl_host the start-up
// scalars (b_norm, r_norm, n_e).  q is scratch; partials is the scratch of
// the rescan's gated form.  *fin receives iterations, stop code and the
// residual estimate for the common exit path.
int gmres_loop(dst_ctx* ctx, Plan& P, const View& v, const double* b, double* a, double* r, double* q,
               double* partials, const dst_solve_opts& opts, const dst::CompView& cv, CgCtl* fin, hipStream_t st) {
  Setup& S = P.S;
  const int64_t N = (int64_t)v.n_streams * v.n_b;
  const int m = opts.restart > 0 ? opts.restart : 50;
  const CgCtl h0 = *ctx->ctl_host;
  const double bnorm = h0.b_norm, n_e = h0.n_e;
  double *V, *z, *part, *gsw;
  DST_TRY(ws(ctx, "gm_V", (size_t)(m + 2) * N, &V));  // slot 0: T mask e; slots 1..m+1: basis
  DST_TRY(ws(ctx, "gm_z", N, &z));
  DST_TRY(ws(ctx, "gm_part", (size_t)(m + 2) * dst::gmres_dot_blocks(N), &part));
  DST_TRY(ws(ctx, "gm_state", (sizeof(dst::GmState) + sizeof(double) - 1) / sizeof(double), &gsw));
  dst::GmState* gs = reinterpret_cast<dst::GmState*>(gsw);
  dst::GmStatus* hs = ctx->gm_host;
  dst::GmStatus* ds = ctx->gm_dev;
  double* e = V;
  auto slot = [&](int i) { return V + (int64_t)(i + 1) * N; };  // basis vector i
  HIP_TRY(dst::launch_tmask(v, S.J, e, st));
  const double beta = h0.r_norm;
  if (h0.done == dst::DONE_NAN || !std::isfinite(bnorm) || !std::isfinite(beta)) {
    // a non-finite right-hand side or start-up residual: nothing to iterate on
    *fin = h0;
    fin->iter = 0;
    fin->done = dst::DONE_NAN;
    return DST_OK;
  }
  const double rel0 = bnorm > 0.0 ? beta / bnorm : 0.0;
  const bool run = bnorm > 0.0 && beta > 0.0 && rel0 > opts.tol && opts.max_iter > 0;
  HIP_TRY(dst::launch_gm_init(gs, bnorm, n_e, opts.tol, opts.max_iter, m, beta, rel0,
                              run ? dst::DONE_RUNNING : dst::DONE_CONVERGED, ds + 2, st));
  CgCtl* gate = &gs->ctl;
  int iters = 0;
  double rel = rel0;
  if (run) {
    for (int s = 0; s < 3; ++s) hs[s].done = dst::DONE_RUNNING;
    for (;;) {
      for (int j = 0; j < m; ++j) {
        // w = P K J v_j, then the two orthogonalisation passes and the Givens step
        HIP_TRY(dst::launch_gm_next(v, gs, j == 0 ? r : q, slot(j), S.J, z, P.pw4, P.dense_t, st));
        DST_TRY(plan_bin(ctx, P, gate, st));
        DST_TRY(plan_unbin(ctx, P, z, q, gate, partials, st));
        HIP_TRY(dst::launch_comp_project(cv, q, 1, 1, st));
        HIP_TRY(dst::launch_gm_dots(gs, V, j + 2, q, N, part, gs->h1, st));  // e.w, v_0.w .. v_j.w
        HIP_TRY(dst::launch_gm_orth(gs, 1, V, j, q, N, part, nullptr, st));
        HIP_TRY(dst::launch_gm_orth(gs, 2, V, j, q, N, part, ds + (j & 1), st));
        HIP_TRY(hipEventRecord(ctx->gm_ev[j & 1], st));
        if (j > 0) {
          HIP_TRY(hipEventSynchronize(ctx->gm_ev[(j - 1) & 1]));
          if (hs[(j - 1) & 1].done != dst::DONE_RUNNING) break;
        }
      }
      // a += J V y, then the restart residual r = b - P K a and v_0 = r / ||r||
      HIP_TRY(dst::launch_gm_update(gs, S.J, V, a, N, st));
      HIP_TRY(dst::launch_p_update4(S.v, a, nullptr, P.pw4, gate, 0, P.dense_t, st));
      DST_TRY(plan_bin(ctx, P, gate, st));
      DST_TRY(plan_unbin(ctx, P, a, q, gate, partials, st));
      HIP_TRY(dst::launch_comp_project(cv, q, 1, 1, st));
      HIP_TRY(dst::launch_gm_restart(gs, b, q, e, r, N, part, ds + 2, st));
      HIP_TRY(hipStreamSynchronize(st));
      if (hs[2].done != dst::DONE_RUNNING) break;
    }
    iters = hs[2].iter;
    rel = hs[2].rel;
  }
  *fin = h0;
  fin->iter = iters;
  fin->r_norm = rel * bnorm;
  fin->done = !std::isfinite(rel) ? dst::DONE_NAN : (rel <= opts.tol ? dst::DONE_CONVERGED : dst::DONE_MAXITER);
  return DST_OK;
}

// Autotuner: times every launch shape of the run binning and rescan on the
// problem itself (operator mode, best of two launches each) and keeps the
// fastest for this problem shape in the context.  p: any baseline vector;
// scratch: [n_streams][n_b] written by the rescan.
int autotune(dst_ctx* ctx, Plan& P, const double* p, double* scratch, hipStream_t st) {
  if (!P.runs) return DST_OK;
  Setup& S = P.S;
  const auto key = std::make_tuple(P.W.n_obs, S.v.n_b, S.v.n_streams, (int)P.W.f32);
  auto it = ctx->tuned.find(key);
  if (it == ctx->tuned.end()) {
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    struct Ev {
      hipEvent_t a, b;
      ~Ev() {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
      }
    } ev{e0, e1};
    auto time_of = [&](auto launch) -> float {
      float best = 1e30f;
      for (int rep = 0; rep < 2; ++rep) {
        if (hipEventRecord(e0, st) != hipSuccess || launch() != hipSuccess || hipEventRecord(e1, st) != hipSuccess ||
            hipEventSynchronize(e1) != hipSuccess)
          return -1.0f;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.0f;
        best = std::min(best, ms);
      }
      return best;
    };
    int best_lpp = P.lpp, best_bpw = P.bpw;
    float tb = 1e30f, tu = 1e30f;
    for (int lpp : {64, 32, 16, 8, 4, -64}) {
      const float t = time_of([&] {
        return dst::launch_bin_runs(S.v, P.W, P.pw4, S.Minv4, S.valid, P.m4, nullptr, lpp, st);
      });
      if (t < 0.f) return fail(ctx, DST_EHIP, "autotuner: a bin launch failed");
      if (t < tb) {
        tb = t;
        best_lpp = lpp;
      }
    }
    for (int bpw : {1, 2, 4, 8}) {
      const float t = time_of([&] {
        return dst::launch_unbin_runs(S.v, P.W, P.m4, S.nvalid, p, scratch, nullptr, nullptr, bpw, st);
      });
      if (t < 0.f) return fail(ctx, DST_EHIP, "autotuner: a rescan launch failed");
      if (t < tu) {
        tu = t;
        best_bpw = bpw;
      }
    }
    it = ctx->tuned.emplace(key, std::make_pair(best_lpp, best_bpw)).first;
  }
  P.lpp = it->second.first;
  P.bpw = it->second.second;
  return DST_OK;
}

}  // namespace

extern "C" {

int dst_version(void) { return DST_ABI_VERSION; }

int dst_create(dst_ctx** out, int device) {
  if (!out) return DST_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return DST_EINVAL;
  dst_ctx* ctx = new (std::nothrow) dst_ctx();
  if (!ctx) return DST_ENOMEM;
  ctx->device = device;
  if (const char* e = std::getenv("DST_UNBIN_BPW")) ctx->unbin_bpw = std::atoi(e);
  if (const char* e = std::getenv("DST_BIN_LPP")) ctx->bin_lpp = std::atoi(e);
  if (const char* e = std::getenv("DST_RUN_SPLIT_BITS")) ctx->run_split_bits = std::atoi(e);
  DeviceGuard g(device);
  if (hipHostMalloc(reinterpret_cast<void**>(&ctx->ctl_host), sizeof(CgCtl), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&ctx->err_host), sizeof(int), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&ctx->rb_host), sizeof(dst_ctx::Readback), hipHostMallocDefault) !=
          hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&ctx->mctl_host), sizeof(dst::MultiCtl), hipHostMallocDefault) !=
          hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&ctx->gctl_host), kMaxGroup * sizeof(CgCtl), hipHostMallocDefault) !=
          hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&ctx->gm_host), 3 * sizeof(dst::GmStatus), hipHostMallocCoherent) !=
          hipSuccess ||
      hipHostGetDevicePointer(reinterpret_cast<void**>(&ctx->gm_dev), ctx->gm_host, 0) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->gm_ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->gm_ev[1], hipEventDisableTiming) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&ctx->err_dev), 4 * sizeof(int)) != hipSuccess ||
      hipMemset(ctx->err_dev, 0, 4 * sizeof(int)) != hipSuccess) {
    (void)hipGetLastError();
    dst_destroy(ctx);
    return DST_ENOMEM;
  }
  // the fixed scratch of dst_bin_noalloc: its address on this device (each
  // device holds its own copy of the array)
  if (hipGetSymbolAddress(reinterpret_cast<void**>(&ctx->scratch), HIP_SYMBOL(scratch)) != hipSuccess) {
    (void)hipGetLastError();
    ctx->scratch = nullptr;
  }
  *out = ctx;
  return DST_OK;
}

int dst_destroy(dst_ctx* ctx) {
  if (!ctx) return DST_OK;
  DeviceGuard g(ctx->device);
  (void)hipDeviceSynchronize();
  for (auto& kv : ctx->ws)
    if (kv.second.ptr) (void)hipFree(kv.second.ptr);
  if (ctx->ctl_host) (void)hipHostFree(ctx->ctl_host);
  if (ctx->err_host) (void)hipHostFree(ctx->err_host);
  if (ctx->err_dev) (void)hipFree(ctx->err_dev);
  if (ctx->rb_host) (void)hipHostFree(ctx->rb_host);
  if (ctx->mctl_host) (void)hipHostFree(ctx->mctl_host);
  if (ctx->gctl_host) (void)hipHostFree(ctx->gctl_host);
  if (ctx->gm_host) (void)hipHostFree(ctx->gm_host);
  for (auto e : ctx->gm_ev)
    if (e) (void)hipEventDestroy(e);
  for (auto g : ctx->graphs)
    if (g) (void)hipGraphExecDestroy(g);
  if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
  delete ctx;
  return DST_OK;
}

const char* dst_last_error(const dst_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int dst_synchronize(dst_ctx* ctx, void* stream) {
  if (!ctx) return DST_EINVAL;
  DeviceGuard g(ctx->device);
  return finish(ctx, nullptr, static_cast<hipStream_t>(stream));
}

int dst_pixel_setup(dst_ctx* ctx, const dst_problem* prob, int32_t* hits_out, double* blocks_out, uint8_t* valid_out,
                    void* stream) {
  View v{};
  DST_TRY(check_problem(ctx, prob, false, v));
  if (v.iqu) return fail(ctx, DST_EINVAL, "DST_IQU streams are not supported by this entry point");
  ctx->err.clear();
  DeviceGuard g(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  Setup S;
  S.v = v;
  DST_TRY(run_setup(ctx, prob, S, false, blocks_out, st));
  if (hits_out) HIP_TRY(hipMemcpyAsync(hits_out, S.hits, v.n_pix * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
  if (valid_out) HIP_TRY(hipMemcpyAsync(valid_out, S.valid, v.n_pix, hipMemcpyDeviceToDevice, st));
  return issued(ctx);
}

int dst_bin(dst_ctx* ctx, const dst_problem* prob, const double* baselines, uint32_t flags, double* map_out,
            int32_t* hits_out, void* stream) {
  View v{};
  DST_TRY(check_bin_args(ctx, prob, flags, map_out, v));
  ctx->err.clear();
  DeviceGuard g(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  Setup S;
  S.v = v;
  DST_TRY(run_setup(ctx, prob, S, false, nullptr, st));
  double* s4 = nullptr;
  DST_TRY(ws(ctx, "s4", 4 * v.n_pix, &s4));
  return bin_pass(ctx, prob, S, baselines, flags, s4, map_out, hits_out, st);
}

int dst_bin_noalloc(dst_ctx* ctx, const dst_problem* prob, const double* baselines, uint32_t flags, double* map_out,
                    int32_t* hits_out, void* stream) {
  View v{};
  DST_TRY(check_bin_args(ctx, prob, flags, map_out, v));
  if (v.n_pix > kNoAllocMaxPix)
    return fail(ctx, DST_EINVAL, "dst_bin_noalloc: n_pix %lld exceeds the fixed scratch limit of %lld pixels",
                (long long)v.n_pix, (long long)kNoAllocMaxPix);
  if (!ctx->scratch) return fail(ctx, DST_EHIP, "dst_bin_noalloc: the scratch array has no device address");
  ctx->err.clear();
  DeviceGuard g(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  Setup S;
  S.v = v;
  double* s4 = nullptr;
  carve_scratch(ctx->scratch, v.n_pix, S, &s4);
  DST_TRY(setup_pixels(ctx, prob, S, nullptr, st));
  return bin_pass(ctx, prob, S, baselines, flags, s4, map_out, hits_out, st);
}

int dst_unbin(dst_ctx* ctx, const dst_problem* prob, const double* map, double* tod_out, void* stream) {
  View v{};
  DST_TRY(check_problem(ctx, prob, false, v));
  if (v.iqu) return fail(ctx, DST_EINVAL, "DST_IQU streams are not supported by this entry point");
  if (!map || !tod_out) return fail(ctx, DST_EINVAL, "map and tod_out must not be NULL");
  ctx->err.clear();
  DeviceGuard g(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(dst::launch_scan(v, prob->psi_dtype == DST_F32, map, tod_out, ctx->err_dev, st));
  return issued(ctx);
}

int dst_baseline_reduce(dst_ctx* ctx, const dst_problem* prob, const void* x, double* out, void* stream) {
  View v{};
  DST_TRY(check_problem(ctx, prob, false, v));
  if (v.iqu) return fail(ctx, DST_EINVAL, "DST_IQU streams are not supported by this entry point");
  if (!x || !out) return fail(ctx, DST_EINVAL, "x and out must not be NULL");
  if (!is_dtype(prob->tod_dtype)) return fail(ctx, DST_EINVAL, "tod_dtype must be DST_F32 or DST_F64");
  ctx->err.clear();
  DeviceGuard g(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  Setup S;
  S.v = v;
  DST_TRY(run_setup(ctx, prob, S, false, nullptr, st));
  HIP_TRY(dst::launch_reduce(v, x, prob->tod_dtype == DST_F32, S.valid, out, st));
  return issued(ctx);
}

int dst_residual(dst_ctx* ctx, const dst_problem* prob, const double* a, double* out, void* stream) {
  View v{};
  DST_TRY(check_problem(ctx, prob, false, v));
  if (v.iqu) return fail(ctx, DST_EINVAL, "DST_IQU streams are not supported by this entry point");
  if (prob->tod && !is_dtype(prob->tod_dtype)) return fail(ctx, DST_EINVAL, "tod_dtype must be DST_F32 or DST_F64");
  if (!out) return fail(ctx, DST_EINVAL, "out is NULL");
  ctx->err.clear();
  DeviceGuard g(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  Setup S;
  S.v = v;
  DST_TRY(run_setup(ctx, prob, S, true, nullptr, st));
  DST_TRY(operator_pass(ctx, S, prob->tod, a, -1.0, out, st));
  return issued(ctx);
}

int dst_apply_operator(dst_ctx* ctx, const dst_problem* prob, const double* vin, double* out, void* stream) {
  View v{};
  DST_TRY(check_problem(ctx, prob, false, v));
  if (!vin || !out) return fail(ctx, DST_EINVAL, "v and out must not be NULL");
  ctx->err.clear();
  DeviceGuard g(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  Plan P;
  P.full = v;
  DST_TRY(build_plan(ctx, prob, P, nullptr, nullptr, nullptr, nullptr, st));
  DST_TRY(plan_operator(ctx, P, vin, out, st));
  return finish(ctx, &P.S, st);
}

int dst_solve(dst_ctx* ctx, const dst_problem* prob, const dst_solve_opts* opts_in, double* baselines_out,
              double* map_out, double* binned_out, int32_t* hits_out, dst_solve_info* info, void* stream) {
  View v{};
  DST_TRY(check_problem(ctx, prob, true, v));
  if (!baselines_out) return fail(ctx, DST_EINVAL, "baselines_out is NULL");
  dst_solve_opts opts{};
  if (opts_in) opts = *opts_in;
  const uint32_t known = DST_SOLVE_NO_CANON | DST_SOLVE_PROFILE | DST_SOLVE_NO_GRAPH | DST_SOLVE_PER_SAMPLE |
                         DST_SOLVE_AUTOTUNE | DST_SOLVE_GMRES;
  const bool use_gmres = opts.flags & DST_SOLVE_GMRES;
  if (!use_gmres && opts.restart != 0) return fail(ctx, DST_EINVAL, "opts.restart is for DST_SOLVE_GMRES only");
  if (v.iqu && (opts.flags & DST_SOLVE_PER_SAMPLE))
    return fail(ctx, DST_EINVAL, "DST_IQU streams need the run form (no DST_SOLVE_PER_SAMPLE)");
  if (opts.restart < 0 || opts.restart > dst::kMaxKrylov - 2)
    return fail(ctx, DST_EINVAL, "opts.restart must be in [0, %d]", dst::kMaxKrylov - 2);
  if (opts.flags & ~known) return fail(ctx, DST_EINVAL, "unknown solve flags %u", opts.flags);
  if (!(opts.tol > 0.0)) opts.tol = 1e-10;
  if (!std::isfinite(opts.tol)) return fail(ctx, DST_EINVAL, "tol must be finite");
  if (opts.max_iter <= 0) opts.max_iter = 1000;
  const int check_every = opts.check_every > 0 ? opts.check_every : 10;
  const bool profile = opts.flags & DST_SOLVE_PROFILE;
  ctx->err.clear();
  DeviceGuard g(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);

  hipEvent_t ev[4];
  for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
  std::vector<hipEvent_t> pev;
  struct EvGuard {
    hipEvent_t* e;
    std::vector<hipEvent_t>* more;
    ~EvGuard() {
      for (int i = 0; i < 4; ++i) (void)hipEventDestroy(e[i]);
      for (auto x : *more) (void)hipEventDestroy(x);
    }
  } evg{ev, &pev};
  HIP_TRY(hipEventRecord(ev[0], st));

  const int64_t N = (int64_t)v.n_streams * v.n_b;
  double *b, *a, *r, *z, *p, *q, *ka, *partials, *sd4 = nullptr, *md4 = nullptr, *rnorm;
  CgCtl* ctl;
  DST_TRY(ws(ctx, "cg_b", N, &b));
  // pointing setup, binned map and right-hand side b = F^T W (d - A m_d)
  Plan P;
  P.full = v;
  P.runs = !(opts.flags & DST_SOLVE_PER_SAMPLE);
  DST_TRY(build_plan(ctx, prob, P, prob->tod, &sd4, &md4, b, st));
  Setup& S = P.S;
  const View& vc = S.v;
  DST_TRY(ws(ctx, "cg_a", N, &a));
  DST_TRY(ws(ctx, "cg_r", N, &r));
  DST_TRY(ws(ctx, "cg_z", N, &z));
  DST_TRY(ws(ctx, "cg_p", N, &p));
  DST_TRY(ws(ctx, "cg_q", N, &q));
  DST_TRY(ws(ctx, "cg_ka", N, &ka));
  DST_TRY(ws(ctx, "cg_part", 3 * (size_t)std::max<int64_t>(v.n_b, 4096), &partials));
  DST_TRY(ws(ctx, "cg_rnorm", 1, &rnorm));
  DST_TRY(ws(ctx, "cg_ctl", 1, &ctl));
  HIP_TRY(dst::launch_fill_u32(reinterpret_cast<uint32_t*>(ctl), sizeof(CgCtl) / 4, 0u, st));

  // several components: b and K a0 lose their component means here (one
  // component: the global mean inside the start-up kernels)
  const dst::CompView cv = P.cv();
  HIP_TRY(dst::launch_comp_project(cv, b, 1, 1, st));
  const double* ka_ptr = nullptr;
  if (opts.a0) {
    DST_TRY(plan_operator(ctx, P, opts.a0, ka, st));
    HIP_TRY(dst::launch_comp_project(cv, ka, 1, 1, st));
    ka_ptr = ka;
  }
  HIP_TRY(dst::launch_cg_start(v, b, ka_ptr, opts.a0, a, r, z, p, S.J, ctl, partials, opts.tol, opts.max_iter, st));
  HIP_TRY(dst::launch_p_update4(v, p, nullptr, P.pw4, nullptr, 0, P.dense_t, st));
  if (opts.flags & DST_SOLVE_AUTOTUNE) DST_TRY(autotune(ctx, P, p, ka, st));

  // PCG iterations: pixel-major bin + inverse (m = M^-1 A^T W F p) -> rescan and
  // baseline sums (q = K p, alpha) -> a, r, z update (beta) -> p and its copy
  auto one_iteration = [&](hipStream_t s, bool timed) -> int {
    hipEvent_t e[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    if (timed) {
      for (auto& x : e) {
        HIP_TRY(hipEventCreate(&x));
        pev.push_back(x);
      }
      HIP_TRY(hipEventRecord(e[0], s));
    }
    DST_TRY(plan_bin(ctx, P, ctl, s));
    if (timed) HIP_TRY(hipEventRecord(e[1], s));
    if (timed) HIP_TRY(hipEventRecord(e[2], s));
    DST_TRY(plan_unbin(ctx, P, p, q, ctl, partials, s));
    HIP_TRY(dst::launch_cg_alpha(P.runs ? dst::unbin_runs_parts(vc, P.bpw) : vc.n_b, ctl, partials, cv, q, p, s));
    if (timed) HIP_TRY(hipEventRecord(e[3], s));
    HIP_TRY(dst::launch_cg_update(v, a, r, z, p, q, S.J, ctl, partials, s));
    HIP_TRY(dst::launch_cg_beta(dst::cg_update_blocks(v), ctl, partials, s));
    HIP_TRY(dst::launch_p_update4(v, p, z, P.pw4, ctl, 1, P.dense_t, s));
    if (timed) HIP_TRY(hipEventRecord(e[4], s));
    return DST_OK;
  };

  // check_every iterations are captured once and replayed, unless profiling
  // or asked not to; captured here, while the setup still runs on the GPU.
  struct {
    hipGraphExec_t exec = nullptr;  // kept by the context
  } gg;
  if (!use_gmres && !(opts.flags & (DST_SOLVE_NO_GRAPH | DST_SOLVE_PROFILE)))
    DST_TRY(capture_graph_kept(ctx, 0, check_every,
                               [&](hipStream_t s) { return one_iteration(s, false); }, &gg.exec));
  HIP_TRY(hipEventRecord(ev[1], st));
  HIP_TRY(hipMemcpyAsync(ctx->ctl_host, ctl, sizeof(CgCtl), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(ctx->rb_host->counts, S.counts, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                         st));
  ctx->rb_host->ncomp[0] = 0;
  if (P.C.ncomp) HIP_TRY(hipMemcpyAsync(ctx->rb_host->ncomp, P.C.ncomp, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  DST_TRY(finish(ctx, &S, st));
  const int ncomp = ctx->rb_host->ncomp[0];
  if (info) info->n_components = ncomp;
  {
    const unsigned long long* c = ctx->rb_host->counts;
    if (info) {
      info->n_valid_pix[0] = (int64_t)c[0];
      info->n_valid_pix[1] = (int64_t)c[1];
      info->n_valid_samples[0] = (int64_t)c[2];
      info->n_valid_samples[1] = (int64_t)c[3];
    }
    if (c[2] + c[3] == 0) {
      HIP_TRY(hipMemsetAsync(baselines_out, 0, N * sizeof(double), st));
      if (map_out) HIP_TRY(hipMemsetAsync(map_out, 0, 3 * v.n_pix * sizeof(double), st));
      if (binned_out) HIP_TRY(hipMemsetAsync(binned_out, 0, 3 * v.n_pix * sizeof(double), st));
      if (hits_out) HIP_TRY(dst::launch_scatter(v.n_pix, P.cid(), S.hits, hits_out, md4, nullptr, nullptr, st));
      HIP_TRY(hipStreamSynchronize(st));
      return fail(ctx, DST_EDEGENERATE, "no valid sample in the problem");
    }
  }

  CgCtl fin{};
  if (use_gmres) {
    // restarted GMRES from the projected residual of the start-up
    HIP_TRY(hipEventRecord(ev[2], st));
    DST_TRY(gmres_loop(ctx, P, v, b, a, r, q, partials, opts, ncomp > 1 ? cv : dst::CompView{}, &fin, st));
    HIP_TRY(hipEventRecord(ev[3], st));
  } else {
  // batches of check_every iterations between convergence checks
  CgCtl& h = *ctx->ctl_host;
  HIP_TRY(hipEventRecord(ev[2], st));
  int launched = 0;
  while (h.done == dst::DONE_RUNNING && launched < opts.max_iter) {
    const int k = std::min(check_every, opts.max_iter - launched);
    if (gg.exec) {
      HIP_TRY(hipGraphLaunch(gg.exec, st));  // check_every iterations (those past the stop return at once)
    } else {
      for (int i = 0; i < k; ++i) DST_TRY(one_iteration(st, profile));
    }
    launched += k;
    HIP_TRY(hipMemcpyAsync(ctx->ctl_host, ctl, sizeof(CgCtl), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  HIP_TRY(hipEventRecord(ev[3], st));
  fin = h;
  }

  // canonical baselines, true residual, maps (destriped = m_d - M^-1 A^T W F a)
  if (!(opts.flags & DST_SOLVE_NO_CANON)) {
    HIP_TRY(dst::launch_comp_project(cv, a, 1, 1, st));
    HIP_TRY(dst::launch_canonicalise(v, a, S.J, partials, ctl, st));
  }
  DST_TRY(plan_operator(ctx, P, a, ka, st));
  HIP_TRY(dst::launch_comp_project(cv, ka, 1, 1, st));
  HIP_TRY(dst::launch_residual_norm(v, b, ka, S.J, ctl, partials, rnorm, st));
  HIP_TRY(hipMemcpyAsync(baselines_out, a, N * sizeof(double), hipMemcpyDeviceToDevice, st));
  if (map_out) HIP_TRY(dst::launch_scatter(v.n_pix, P.cid(), nullptr, nullptr, md4, P.m4, map_out, st, P.dense_t));
  if (binned_out) HIP_TRY(dst::launch_scatter(v.n_pix, P.cid(), nullptr, nullptr, md4, nullptr, binned_out, st));
  if (hits_out) HIP_TRY(dst::launch_scatter(v.n_pix, P.cid(), S.hits, hits_out, md4, nullptr, nullptr, st));
  HIP_TRY(hipMemcpyAsync(&ctx->rb_host->rnorm, rnorm, sizeof(double), hipMemcpyDeviceToHost, st));
  DST_TRY(finish(ctx, &S, st));
  const double true_norm = ctx->rb_host->rnorm;

  if (info) {
    info->iterations = fin.iter;
    info->converged = fin.done == dst::DONE_CONVERGED;
    info->b_norm = fin.b_norm;
    info->rel_residual = fin.b_norm > 0.0 ? fin.r_norm / fin.b_norm : 0.0;
    info->true_rel_residual = fin.b_norm > 0.0 ? true_norm / fin.b_norm : 0.0;
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ev[0], ev[1]));
    info->t_setup_ms = ms;
    HIP_TRY(hipEventElapsedTime(&ms, ev[2], ev[3]));
    info->t_iter_ms = fin.iter > 0 ? ms / fin.iter : 0.0;
    HIP_TRY(hipEventElapsedTime(&ms, ev[0], ev[3]));
    info->t_total_ms = ms;
    info->t_bin_ms = info->t_apply_ms = info->t_unbin_ms = info->t_update_ms = 0.0;
    info->n_runs = P.runs ? P.W.R : 0;
    if (profile && !pev.empty()) {
      // only iterations that ran (not the launches after the stop) count
      const size_t n_it = pev.size() / 5;
      const size_t used = std::min<size_t>(n_it, (size_t)std::max(fin.iter, 0));
      double acc[4] = {0, 0, 0, 0};
      for (size_t i = 0; i < used; ++i) {
        for (int j = 0; j < 4; ++j) {
          float t = 0.f;
          HIP_TRY(hipEventElapsedTime(&t, pev[5 * i + j], pev[5 * i + j + 1]));
          acc[j] += t;
        }
      }
      if (used) {
        info->t_bin_ms = acc[0] / used;
        info->t_apply_ms = acc[1] / used;
        info->t_unbin_ms = acc[2] / used;
        info->t_update_ms = acc[3] / used;
      }
    }
  }
  switch (fin.done) {
    case dst::DONE_CONVERGED:
      return DST_OK;
    case dst::DONE_MAXITER:
    case dst::DONE_RUNNING:
      fail(ctx, DST_ENOCONV, "no convergence in %d iterations (rel residual %.3e)", fin.iter,
           fin.b_norm > 0 ? fin.r_norm / fin.b_norm : 0.0);
      return DST_ENOCONV;
    case dst::DONE_BREAKDOWN:
      return fail(ctx, DST_EBREAKDOWN, "CG breakdown after %d iterations", fin.iter);
    default:
      return fail(ctx, DST_ENAN, "non-finite value in the CG recurrences after %d iterations", fin.iter);
  }
}

int dst_solve_batched(dst_ctx* ctx, int32_t n_problems, const dst_problem* problems, const dst_solve_opts* opts_in,
                      double* const* baselines_out, double* const* map_out, double* const* binned_out,
                      int32_t* const* hits_out, dst_solve_info* infos, void* stream) {
  if (!ctx) return DST_EINVAL;
  if (n_problems < 1) return fail(ctx, DST_EINVAL, "n_problems must be >= 1 (got %d)", n_problems);
  if (!problems) return fail(ctx, DST_EINVAL, "problems is NULL");
  if (!baselines_out) return fail(ctx, DST_EINVAL, "baselines_out is NULL");
  dst_solve_opts opts{};
  if (opts_in) opts = *opts_in;
  if (opts.restart != 0) return fail(ctx, DST_EINVAL, "opts.restart must be 0 in the batched solve");
  if (opts.a0) return fail(ctx, DST_EINVAL, "opts.a0 is not supported by the batched solve");
  const uint32_t known = DST_SOLVE_NO_CANON | DST_SOLVE_PROFILE | DST_SOLVE_NO_GRAPH | DST_SOLVE_AUTOTUNE;
  if (opts.flags & ~known) return fail(ctx, DST_EINVAL, "unknown or unsupported solve flags %u", opts.flags);
  if (!(opts.tol > 0.0)) opts.tol = 1e-10;
  if (!std::isfinite(opts.tol)) return fail(ctx, DST_EINVAL, "tol must be finite");
  if (opts.max_iter <= 0) opts.max_iter = 1000;
  const int check_every = opts.check_every > 0 ? opts.check_every : 10;
  for (int i = 0; i < n_problems; ++i) {
    View v{};
    const int rc = check_problem(ctx, &problems[i], true, v);
    if (rc != DST_OK) {
      std::string msg = ctx->err;
      return fail(ctx, rc, "problem %d: %s", i, msg.c_str());
    }
    if (!baselines_out[i]) return fail(ctx, DST_EINVAL, "baselines_out[%d] is NULL", i);
  }
  ctx->err.clear();
  DeviceGuard g(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  // groups of problems that share the operator, in order of first appearance
  std::vector<std::vector<int>> groups;
  for (int i = 0; i < n_problems; ++i) {
    bool placed = false;
    for (auto& grp : groups) {
      if ((int)grp.size() < dst::kMaxRhs && same_operator(problems[grp[0]], problems[i])) {
        grp.push_back(i);
        placed = true;
        break;
      }
    }
    if (!placed) groups.push_back({i});
  }
  const BatchOut out{baselines_out, map_out, binned_out, hits_out, infos};
  int status = DST_OK;
  // problems that share the operator with no other: solved together as
  // groups of independent problems (one group per precision of the angle
  // sums; intensity-only problems have none and join any group)
  std::vector<int> solo32, solo64, soloT;
  for (const auto& grp : groups) {
    if (grp.size() != 1) continue;
    const dst_problem& pr = problems[grp[0]];
    if (pr.streams == DST_T)
      soloT.push_back(grp[0]);
    else if (pr.psi_dtype == DST_F32)
      solo32.push_back(grp[0]);
    else
      solo64.push_back(grp[0]);
  }
  std::vector<std::vector<int>> uneven;
  for (std::vector<int>* lst : {&solo32, &solo64}) {
    if (lst->empty()) continue;
    uneven.push_back(*lst);
  }
  if (!soloT.empty()) {
    if (uneven.empty()) uneven.emplace_back();
    uneven[0].insert(uneven[0].end(), soloT.begin(), soloT.end());
  }
  for (const auto& grp : groups) {
    if (grp.size() == 1) continue;
    const int rc = solve_group(ctx, problems, grp, opts, check_every, out, st, &status);
    if (rc != DST_OK) return rc;
  }
  for (const auto& lst : uneven) {
    for (size_t c0 = 0; c0 < lst.size(); c0 += kMaxGroup) {
      const std::vector<int> chunk(lst.begin() + c0, lst.begin() + std::min(lst.size(), c0 + kMaxGroup));
      if (chunk.size() == 1) {
        const int i = chunk[0];
        dst_solve_opts o = opts;
        const int rc = dst_solve(ctx, &problems[i], &o, baselines_out[i], map_out ? map_out[i] : nullptr,
                                 binned_out ? binned_out[i] : nullptr, hits_out ? hits_out[i] : nullptr,
                                 infos ? &infos[i] : nullptr, stream);
        if (rc < 0) return rc;
        status = worse(status, rc);
        continue;
      }
      const int rc = solve_uneven(ctx, problems, chunk, opts, check_every, out, st, &status);
      if (rc != DST_OK) return rc;
    }
  }
  if (status == DST_ENOCONV) fail(ctx, DST_ENOCONV, "at least one problem did not converge");
  return status;
}

int dst_pointing_expand(dst_ctx* ctx, const dst_scan* scan, int64_t nside, int64_t start, int64_t n_samples,
                        int32_t* pix_out, void* psi_out, int32_t psi_dtype, void* stream) {
  if (!ctx) return DST_EINVAL;
  if (!scan) return fail(ctx, DST_EINVAL, "scan is NULL");
  if (!pix_out) return fail(ctx, DST_EINVAL, "pix_out is NULL");
  if (nside < 1 || nside > 8192) return fail(ctx, DST_EINVAL, "nside must be in [1, 8192] (got %lld)", (long long)nside);
  if (n_samples < 1 || start < 0 || start > ((int64_t)1 << 53) - n_samples)
    return fail(ctx, DST_EINVAL, "need n_samples >= 1, start >= 0 and start + n_samples <= 2^53");
  if (psi_out && !is_dtype(psi_dtype)) return fail(ctx, DST_EINVAL, "psi_dtype must be DST_F32 or DST_F64");
  const dst_scan& s = *scan;
  const double vals[8] = {s.sample_rate_hz, s.spin_period_s, s.elevation_deg, s.latitude_deg,
                          s.az0_deg,        s.lst0_rad,      s.psi0_deg,      s.sidereal_day_s};
  for (double x : vals)
    if (!std::isfinite(x)) return fail(ctx, DST_EINVAL, "scan parameters must be finite");
  if (!(s.sample_rate_hz > 0.0) || !(s.spin_period_s > 0.0) || !(s.sidereal_day_s > 0.0))
    return fail(ctx, DST_EINVAL, "sample rate, spin period and sidereal day must be > 0");
  if (!(std::fabs(s.latitude_deg) < 90.0)) return fail(ctx, DST_EINVAL, "latitude must be in (-90, 90) degrees");
  const double per = s.sample_rate_hz * s.spin_period_s;
  if (!(per >= 1.0 && per <= (double)(1 << 24)) || std::fabs(per - std::nearbyint(per)) > 1e-9)
    return fail(ctx, DST_EINVAL, "a spin period must hold a whole number of samples in [1, 2^24]");
  const int64_t n_per = (int64_t)std::nearbyint(per);
  ctx->err.clear();
  DeviceGuard g(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<double> tab;
  dst::scan_period_table(s, n_per, tab);
  double* dtab = nullptr;
  DST_TRY(ws(ctx, "scan_tab", tab.size(), &dtab));
  HIP_TRY(hipMemcpyAsync(dtab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, st));
  HIP_TRY(dst::launch_expand(nside, start, n_samples, n_per, s, dtab, pix_out, psi_out, psi_dtype == DST_F32, st));
  HIP_TRY(hipStreamSynchronize(st));
  return DST_OK;
}

int dst_noise_generate(dst_ctx* ctx, uint64_t seed, uint64_t stream_id, int64_t n_samples, int64_t segment,
                       double sample_rate_hz, double sigma, double fknee_hz, double alpha, void* out,
                       int32_t out_dtype, uint32_t flags, void* stream) {
  if (!ctx) return DST_EINVAL;
  if (!out) return fail(ctx, DST_EINVAL, "out is NULL");
  if (!is_dtype(out_dtype)) return fail(ctx, DST_EINVAL, "out_dtype must be DST_F32 or DST_F64");
  if (n_samples < 1) return fail(ctx, DST_EINVAL, "n_samples must be >= 1");
  if (segment < 4 || segment > ((int64_t)1 << 26) || (segment & (segment - 1)))
    return fail(ctx, DST_EINVAL, "segment must be a power of two in [4, 2^26] (got %lld)", (long long)segment);
  if (!(sample_rate_hz > 0.0) || !std::isfinite(sample_rate_hz)) return fail(ctx, DST_EINVAL, "sample rate must be > 0");
  if (!(sigma >= 0.0) || !std::isfinite(sigma)) return fail(ctx, DST_EINVAL, "sigma must be >= 0 and finite");
  if (!(fknee_hz >= 0.0) || !std::isfinite(fknee_hz)) return fail(ctx, DST_EINVAL, "fknee must be >= 0 and finite");
  if (!std::isfinite(alpha)) return fail(ctx, DST_EINVAL, "alpha must be finite");
  if (flags & ~(uint32_t)DST_NOISE_ACCUMULATE) return fail(ctx, DST_EINVAL, "unknown flags %u", flags);
  ctx->err.clear();
  DeviceGuard g(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t nbuf = (size_t)dst::noise_pairs_per_chunk(segment) * (size_t)segment;
  double2 *b0 = nullptr, *b1 = nullptr;
  DST_TRY(ws(ctx, "noise_b0", nbuf, &b0));
  DST_TRY(ws(ctx, "noise_b1", nbuf, &b1));
  double2* tw = nullptr;
  DST_TRY(ws(ctx, "noise_tw", (size_t)dst::noise_twiddle_count(segment), &tw));
  HIP_TRY(dst::launch_noise(seed, stream_id, n_samples, segment, sample_rate_hz, sigma, fknee_hz, alpha, out,
                            out_dtype == DST_F32, (flags & DST_NOISE_ACCUMULATE) ? 1 : 0, b0, b1, tw, st));
  HIP_TRY(hipStreamSynchronize(st));
  return DST_OK;
}

}  // extern "C"
