/*
 * dst.h -- C ABI of the MI355X (gfx950) destriping library.
 *
 * The library computes the hot path of the polarimeter destriper of
 * Zonca, Williams, Meinhold & Lubin, "Destriping Cosmic Microwave Background
 * Polarimeter data" (Astronomy and Computing; arXiv:1309.5609):
 * the maximum-likelihood baselines a of the destriping equation (Eq. 13)
 *
 *       F^T Z F a = F^T Z d,        Z = W - W A M^-1 A^T W,
 *
 * by preconditioned conjugate gradient, where each operator application bins
 * timelines into per-pixel I/Q/U sums (A^T W), applies the inverted per-pixel
 * weight matrices (M^-1), scans the map back to the timeline (A) and sums
 * each fixed-length baseline (F^T).
 *
 * Notation (Algorithm section, Eqs. 2-9):
 *   streams k in {T, q, u} of one channel share the pixel p(t) and angle psi(t);
 *   pointing rows  A_T = (1, 0, 0), A_q = (0, cos2psi, sin2psi),
 *                  A_u = (0, -sin2psi, cos2psi)              (Eqs. 3-6);
 *   baseline of sample t: beta(t) = t / L, n_b = ceil(n_samples / L)
 *                  (fixed sample count per baseline, Polarimeters data section);
 *   white-noise weights w_k = 1/sigma_k^2, constant per stream;
 *   per-pixel matrix M_p = sum_t sum_k w_k A_k(t)^T A_k(t)  (block diagonal
 *                  T | QU; for equal q/u weights the QU block is w h I_2).
 *
 * Validity.  A pixel's T block is valid when it has hits; its QU block when
 * its smaller eigenvalue is positive and lambda_min/lambda_max >= rcond_cut.
 * A sample enters stream k only when pix >= 0 and the block stream k uses is
 * valid; other samples are left out of binning and of the baseline sums.
 *
 * Memory.  Every array argument is a device pointer owned by the caller
 * (hipMalloc'd memory or a torch tensor's data_ptr on the context's device),
 * in the layout stated at the argument.  Timelines are [n_streams][n_samples]
 * row-major with streams in the order T, q, u restricted to those present;
 * baseline vectors are [n_streams][n_b]; maps are [n_pix][3] in (I, Q, U)
 * order.  The library keeps no caller pointer after a call returns and owns
 * only the workspace inside its context (grown on demand, freed by
 * dst_destroy).
 *
 * Streams and synchrony.  Work is issued on the caller's `stream` (NULL = the
 * null stream).  dst_pixel_setup, dst_bin, dst_unbin, dst_baseline_reduce and
 * dst_residual are stream-ordered and asynchronous: they return once their
 * work is queued, and their outputs are ready when the stream reaches that
 * point.  Calls that need sizes or results on the host (dst_apply_operator,
 * dst_solve, dst_solve_batched, dst_pointing_expand, dst_noise_generate) wait
 * for their stream before returning.  The workspace of a context is shared by
 * its calls, so calls on one context must be ordered (one stream, or streams
 * synchronised in between); use one context per concurrent stream.
 *
 * Errors.  Functions return a dst_status.  Argument errors are found before
 * any launch and leave outputs untouched.  A pixel index >= n_pix found on
 * the device sets a flag in the context; the next call that waits for its
 * stream (or dst_synchronize) returns DST_EBOUNDS and clears it.
 * dst_last_error() gives a message for the context's most recent failure.  No
 * C++ exception crosses the ABI.
 *
 * Threads.  A context may be used by one host thread at a time.
 */
#ifndef DST_H
#define DST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DST_ABI_VERSION 2

typedef enum {
  DST_OK = 0,
  DST_ENOCONV = 1,        /* warning: max_iter reached; outputs hold the last iterate */
  DST_EINVAL = -1,        /* invalid argument (null pointer, size, dtype, stream set, weight) */
  DST_ENOMEM = -2,        /* device workspace allocation failed */
  DST_EHIP = -3,          /* HIP runtime error; message in dst_last_error */
  DST_ENAN = -4,          /* non-finite value in the CG recurrences */
  DST_EDEGENERATE = -5,   /* no valid sample in the problem */
  DST_EBOUNDS = -6,       /* a pixel index >= n_pix was found in the pointing */
  DST_EBREAKDOWN = -7     /* CG breakdown: p.Kp <= 0 before convergence */
} dst_status;

typedef enum { DST_F32 = 1, DST_F64 = 2 } dst_dtype;

/* Stream sets.  q and u always come together (the two channels of a
 * polarimeter, Algorithm section).  DST_IQU is one stream of a
 * polarisation-sensitive radiometer, d = I + Q cos 2psi + U sin 2psi, whose
 * pixels need the full 3x3 block (the remark after Eqs. 10-11); it is weighted
 * by weight[0] and its block cut by rcond_cut over all three eigenvalues.
 * DST_IQU is accepted by dst_solve (run form), dst_apply_operator and
 * dst_solve_batched (each such problem on its own); the other entry points
 * and DST_SOLVE_PER_SAMPLE return DST_EINVAL for it. */
enum { DST_T = 1u, DST_Q = 2u, DST_U = 4u, DST_QU = 6u, DST_TQU = 7u, DST_IQU = 8u };

typedef struct dst_ctx dst_ctx;

/* One channel's destriping problem (Algorithm section, Eqs. 2-8). */
typedef struct {
  int64_t n_samples;       /* n_t >= 1 */
  int64_t n_pix;           /* pixels of the map, >= 1 (12 nside^2 for HEALPix) */
  int64_t baseline_length; /* L >= 1 samples; the last baseline may be shorter */
  uint32_t streams;        /* DST_T, DST_QU, DST_TQU or DST_IQU */
  int32_t tod_dtype;       /* dst_dtype of `tod` */
  int32_t psi_dtype;       /* dst_dtype of `psi` (ignored for DST_T) */
  int32_t reserved;        /* must be 0 */
  const int32_t* pix;      /* device [n_samples]; pixel of each sample, < 0 masks the sample */
  const void* psi;         /* device [n_samples]; polarisation angle psi in radians (NULL for DST_T) */
  const void* tod;         /* device [n_streams][n_samples]; calibrated timelines in K (may be NULL
                              where a call states it is not read) */
  double weight[3];        /* w_T, w_q, w_u > 0 and finite (entries of absent streams ignored) */
  double rcond_cut;        /* eigenvalue-ratio cut of the QU block (IQU: of the 3x3 block) in [0, 1) */
} dst_problem;

/* Library ABI version (DST_ABI_VERSION of the build). */
int dst_version(void);

/* Create a context on HIP device `device`.  *ctx receives the handle.
 * Launch shapes of the run-form iteration kernels may be overridden by the
 * environment at creation: DST_BIN_LPP (lanes per pixel in the binning: 64,
 * 32 = default, 16, or -64 for 64 with a software pipeline over pixels) and
 * DST_UNBIN_BPW (baselines per wavefront in the rescan: 1, 2, 4 = default,
 * 8).  DST_RUN_SPLIT_BITS = k splits runs of consecutive samples on one
 * pixel at 2^k samples at most (runs are split anyway where a pixel id and a
 * run length would not fit one 32-bit key).  They change speed only, not
 * results beyond summation order. */
int dst_create(dst_ctx** ctx, int device);

/* Destroy a context and free its workspace (NULL is accepted). */
int dst_destroy(dst_ctx* ctx);

/* Message describing the context's most recent error ("" if none). */
const char* dst_last_error(const dst_ctx* ctx);

/* Wait for `stream` and report what the asynchronous calls of this context
 * found on the device: DST_EBOUNDS (flag then cleared) if a pixel index >=
 * n_pix was met since the last report, else DST_OK. */
int dst_synchronize(dst_ctx* ctx, void* stream);

/* Per-pixel setup (Eq. 9 and the per-pixel weight matrices after Eqs. 10-11).
 *   hits_out  [n_pix] int32   number of unmasked samples per pixel (NULL to skip)
 *   blocks_out[n_pix][4] f64  (M_II, M_QQ, M_QU, M_UU) (NULL to skip)
 *   valid_out [n_pix] uint8   bit 0: T block valid, bit 1: QU block valid (NULL to skip)
 * Reads pix and psi only. */
int dst_pixel_setup(dst_ctx* ctx, const dst_problem* prob, int32_t* hits_out, double* blocks_out,
                    uint8_t* valid_out, void* stream);

/* Binning, Eqs. 10-12 with weights: x = tod - F baselines (tod read when
 * flags has DST_BIN_USE_TOD, baselines when non-NULL), then
 *   s_p = sum over valid samples of sum_k w_k A_k(t)^T x_k(t)      (sum maps)
 * and, with DST_BIN_MAP, m_p = M_p^-1 s_p on valid blocks (0 elsewhere).
 *   baselines [n_streams][n_b] f64 or NULL
 *   map_out   [n_pix][3] f64: sums or map
 *   hits_out  [n_pix] int32 or NULL */
enum { DST_BIN_USE_TOD = 1u, DST_BIN_MAP = 2u };
int dst_bin(dst_ctx* ctx, const dst_problem* prob, const double* baselines, uint32_t flags, double* map_out,
            int32_t* hits_out, void* stream);

/* dst_bin without any device allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, results and asynchrony as dst_bin;
 * the per-pixel work arrays (hits, blocks, inverse, validity, sums: 101 bytes
 * per pixel) live in one fixed device array of the library, sized for
 * n_pix <= 786432 (12 * 256^2, a full N_side 256 sky; about 79 MB), which
 * each GPU the library runs on holds until the process ends.
 *   n_pix > 786432  -> DST_EINVAL (nothing launched).
 * Every call on one GPU shares that GPU's array (across contexts too) and
 * leaves its contents behind; the call clears what it accumulates into, but
 * calls that overlap in time on one GPU (different streams or contexts
 * without synchronisation in between) race on it. */
int dst_bin_noalloc(dst_ctx* ctx, const dst_problem* prob, const double* baselines, uint32_t flags, double* map_out,
                    int32_t* hits_out, void* stream);

/* Scan a map to timelines (the P and R matrices of Eqs. 2-6):
 *   tod_out_k(t) = A_k(t) . map[p(t)] for unmasked samples, 0 for masked ones.
 *   map [n_pix][3] f64, tod_out [n_streams][n_samples] f64.  Validity is not
 * applied (every unmasked sample is scanned).  Reads pix and psi only. */
int dst_unbin(dst_ctx* ctx, const dst_problem* prob, const double* map, double* tod_out, void* stream);

/* Weighted baseline sums F^T W x over valid samples (the F^T of Eq. 13):
 *   out_k[beta] = sum_{t in beta, valid_k(t)} w_k x_k(t)
 *   x [n_streams][n_samples] of dtype prob->tod_dtype (prob->tod is not read),
 *   out [n_streams][n_b] f64. */
int dst_baseline_reduce(dst_ctx* ctx, const dst_problem* prob, const void* x, double* out, void* stream);

/* Residual of the destriping equation (Eq. 13) for baselines a:
 *   out = F^T Z (d - F a)    (= b - K a)
 * with d = prob->tod (NULL: d = 0) and a [n_streams][n_b] (NULL: a = 0).
 * out [n_streams][n_b] f64.  No null-space projection is applied. */
int dst_residual(dst_ctx* ctx, const dst_problem* prob, const double* a, double* out, void* stream);

/* Operator of Eq. 13:  out = K v = F^T Z F v;  v, out [n_streams][n_b] f64. */
int dst_apply_operator(dst_ctx* ctx, const dst_problem* prob, const double* v, double* out, void* stream);

/* Solver options.  Zero-initialise and set what you need; tol <= 0 selects
 * 1e-10 and max_iter <= 0 selects 1000. */
enum {
  DST_SOLVE_NO_CANON = 1u,    /* return the raw CG iterate (skip the T mean removal) */
  DST_SOLVE_PROFILE = 2u,     /* time each kernel class with HIP events (into info) */
  DST_SOLVE_NO_GRAPH = 4u,    /* launch iterations one by one instead of a captured graph */
  DST_SOLVE_PER_SAMPLE = 8u,  /* iterate on per-sample pointing (recomputing cos 2psi, sin 2psi)
                                 instead of the default run-compressed pointing */
  DST_SOLVE_AUTOTUNE = 16u,   /* time the launch shapes of the run-form binning and rescan on this
                                 problem once (a few operator applications) and use the fastest;
                                 the choice is kept in the context per problem shape */
  DST_SOLVE_GMRES = 32u       /* restarted GMRES (Saad & Schultz 1986, the solver of the paper's
                                 implementation) with the same Jacobi diagonal as right
                                 preconditioner, instead of PCG; tol applies to the GMRES
                                 residual estimate ||b - K a|| / ||b|| */
};
typedef struct {
  double tol;               /* stop when ||r||_2 <= tol ||b||_2 (recurrence residual) */
  int32_t max_iter;
  int32_t check_every;      /* iterations per host convergence check and per captured graph
                               (<= 0: 10); iterations past the stop inside a graph do nothing */
  uint32_t flags;
  int32_t restart;          /* GMRES restart length in [1, 126] (0: 50); must be 0 without DST_SOLVE_GMRES */
  const double* a0;         /* device [n_streams][n_b] initial guess, or NULL for 0 */
} dst_solve_opts;

typedef struct {
  int32_t iterations;       /* CG iterations performed */
  int32_t converged;        /* 1 if the tolerance was met */
  double rel_residual;      /* recurrence ||r|| / ||b|| at exit */
  double true_rel_residual; /* ||b - P K a|| / ||b|| recomputed at exit */
  double b_norm;            /* ||b||_2 after the null-space projection */
  int64_t n_valid_pix[2];   /* pixels with a valid T block, with a valid QU block */
  int64_t n_valid_samples[2];
  double t_setup_ms;        /* pointing setup + right-hand side */
  double t_iter_ms;         /* CG loop wall time / iterations */
  double t_total_ms;
  /* with DST_SOLVE_PROFILE: mean device time per launch of each kernel class (ms) */
  double t_bin_ms, t_apply_ms, t_unbin_ms, t_update_ms;
  int64_t n_runs;           /* runs of the run-compressed pointing (0 in the per-sample form) */
  int64_t n_components;     /* connected components of the baseline-pixel graph over samples valid
                               for the T (or radiometer) stream: one null vector of Eq. 13 each
                               (0 without such a stream) */
} dst_solve_info;

/* Destripe one channel (Eq. 13 by PCG, then Eqs. 10-12 for the maps).
 *
 * Null space.  A constant added to the T baselines (DST_IQU: the radiometer
 * baselines) of one connected component of the bipartite graph baseline <->
 * pixel, linked by the valid samples of that stream, equals the same constant
 * added to the I map of the component's pixels (Eq. 8), so K has one null
 * vector per component.  The solver removes the component means from b and
 * from every K p, and reports the baselines with zero mean over each
 * component's baselines (baselines without valid samples are 0).
 *
 *   baselines_out [n_streams][n_b] f64   solution a (canonical as above
 *                 unless DST_SOLVE_NO_CANON)
 *   map_out       [n_pix][3] f64 or NULL  destriped map m = M^-1 A^T W (d - F a)
 *   binned_out    [n_pix][3] f64 or NULL  binned map   m = M^-1 A^T W d
 *   hits_out      [n_pix] int32 or NULL
 *   info          host struct or NULL
 * Returns DST_OK, DST_ENOCONV (outputs hold the last iterate) or an error. */
int dst_solve(dst_ctx* ctx, const dst_problem* prob, const dst_solve_opts* opts, double* baselines_out,
              double* map_out, double* binned_out, int32_t* hits_out, dst_solve_info* info, void* stream);

/* Scan strategy of a spinning ground telescope (input synthesis on the GPU).
 * The telescope turns about the vertical at constant elevation; sample i is
 * taken at t = i / sample_rate_hz, azimuth az0 + 2 pi t / spin_period_s, local
 * sidereal time lst0 + 2 pi t / sidereal_day_s.  The alt-az -> equatorial
 * transform gives declination, hour angle H and parallactic angle q; the
 * sample's direction is (colatitude 90 deg - dec, RA = LST - H) and its
 * polarisation angle psi = q + psi0 (the parallactic-angle footnote of the
 * Algorithm section). */
typedef struct {
  double sample_rate_hz;  /* > 0 */
  double spin_period_s;   /* > 0; sample_rate_hz * spin_period_s must be a whole number <= 2^24 */
  double elevation_deg;
  double latitude_deg;    /* in (-90, 90) */
  double az0_deg;
  double lst0_rad;
  double psi0_deg;
  double sidereal_day_s;  /* > 0 */
} dst_scan;

/* Pointing of samples start .. start + n_samples - 1 of the scan:
 *   pix_out [n_samples] int32   HEALPix RING index at resolution nside
 *   psi_out [n_samples] f64 or f32 (psi_dtype) polarisation angle, or NULL
 * nside in [1, 8192]; start >= 0 and start + n_samples <= 2^53.  The
 * per-period angles are tabulated on the host with the C library's sin, cos,
 * tan, asin and atan2; every per-sample step is a correctly rounded FP64
 * operation in a fixed order, so a host implementation evaluating the same
 * expressions reproduces the pixels bit for bit.  Stream-ordered; the call
 * waits for its stream before returning. */
int dst_pointing_expand(dst_ctx* ctx, const dst_scan* scan, int64_t nside, int64_t start, int64_t n_samples,
                        int32_t* pix_out, void* psi_out, int32_t psi_dtype, void* stream);

/* White + 1/f noise on the GPU (Eq. 1: P(f) = sigma^2 (1 + (f_k / f)^alpha)).
 * Timeline of n_samples made of segments of `segment` samples (a power of two
 * in [4, 2^26]; the last segment is drawn at full length and cut).  Segment j
 * is sigma times unit normals -- Box-Muller on Philox4x64-10 words, block b of
 * the segment from counter (b, j, 0, 0) and key (seed, stream_id), the four
 * words of a block giving samples 4b .. 4b+3 -- filtered by
 * sqrt(1 + (f_k / |f|)^alpha) in the Fourier domain of the segment with the
 * zero-frequency bin kept (fknee_hz = 0: white noise).
 *   out [n_samples] of out_dtype (DST_F32 or DST_F64); with flags
 *       DST_NOISE_ACCUMULATE the noise is added to what out holds.
 * Stream-ordered; the call waits for its stream before returning.  Work
 * memory: two buffers of up to 256 MiB in the context. */
enum { DST_NOISE_ACCUMULATE = 1u };
int dst_noise_generate(dst_ctx* ctx, uint64_t seed, uint64_t stream_id, int64_t n_samples, int64_t segment,
                       double sample_rate_hz, double sigma, double fknee_hz, double alpha, void* out,
                       int32_t out_dtype, uint32_t flags, void* stream);

/* Destripe several problems in one call.
 *
 * Problems that share the operator K of Eq. 13 -- the same pix and psi
 * pointers, n_samples, n_pix, baseline_length, streams, psi_dtype, weights and
 * rcond_cut, as Monte Carlo noise realizations of one channel do -- are solved
 * together (up to 64 per group): the pointing setup runs once, each iteration
 * applies K to every right-hand side in one pass over the pointing, and each
 * problem keeps its own CG scalars and stops when it meets the tolerance
 * (later iterations leave its solution unchanged).  Each problem has its own
 * tod (its tod_dtype may differ).  When every problem of such a group has
 * FP32 angles and timelines, the iterations gather p and the per-pixel map
 * from FP32 copies (sums, CG scalars and outputs stay FP64): the operator
 * then carries a relative error near 1e-8, so the true residual levels off
 * near 1e-9 while the recurrence residual meets tol.  Problems that share the operator with no
 * other are solved one after another as by dst_solve.
 *   n_problems     >= 1
 *   problems       host array [n_problems]
 *   opts           as for dst_solve, shared by every problem; a0 must be NULL
 *                  and DST_SOLVE_PER_SAMPLE is not accepted
 *   baselines_out  host array [n_problems] of device pointers, each
 *                  [n_streams][n_b] f64 (none may be NULL)
 *   map_out, binned_out, hits_out
 *                  host arrays [n_problems] of device pointers ([n_pix][3] f64,
 *                  [n_pix][3] f64, [n_pix] int32); the array or any entry may
 *                  be NULL to skip that output
 *   infos          host array [n_problems] or NULL; in a group the timings are
 *                  those of the group (t_iter_ms per iteration of the group)
 * Returns DST_OK when every problem converged, DST_ENOCONV when at least one
 * did not (its outputs hold the last iterate), else the first error met
 * (argument errors are reported before any launch, naming the problem). */
int dst_solve_batched(dst_ctx* ctx, int32_t n_problems, const dst_problem* problems, const dst_solve_opts* opts,
                      double* const* baselines_out, double* const* map_out, double* const* binned_out,
                      int32_t* const* hits_out, dst_solve_info* infos, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* DST_H */
