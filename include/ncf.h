/*
 * ncf.h -- C ABI of the MI355X kernel-weighted correlation library.
 *
 * The library computes the kernel-weighted auto- and cross-correlation
 * estimator for irregularly sampled series (eq. kernel_estimator, Sec. 2.3)
 * with the Gaussian kernel (eq. Gaussian_kernel, bandwidth h) or the
 * rectangle kernel (half-width h, closed window, as in Algorithm
 * "PairCount, rectangle"), together with the effective pair count b
 * (Appendix A.2, Algorithms "PairCount").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Series 1 is (t_i, x_i), series 2 is (s_j, y_j). Times must be finite and
 *    non-decreasing (ties allowed); values finite.
 *  - CCF lag +tau means series 2 lags series 1 by tau: pairs with
 *    s_j - t_i close to tau (Appendix A.1, sign convention).
 *    ACF pairs have t_i - t_j close to tau.
 *  - Gaussian window: t_i in [centre - 6h, centre + 6h) with
 *    centre = s_j + eps*tau (eps = +1 ACF, -1 CCF); weight
 *    exp(-d^2/2h^2)/(sqrt(2 pi) h) (Algorithm "PairCount, Gaussian").
 *    Rectangle window: t_i in [centre - h, centre + h], weight 1.
 *  - Values are standardized (mean 0, sd 1, ddof 0) before the pair sums
 *    (Algorithms "CCF via NUFFT" / "ACF via NUFFT", first step).
 *  - r(tau) = C(tau) / max(B(tau), 1e-16) where C is the kernel-weighted sum of
 *    value products and B the kernel-weighted pair sum.
 *    ACF: c_k = r(tau_k) / r(0)   (lag-0 normalization of "ACF via NUFFT").
 *    CCF: c_k = r(tau_k) / sqrt(scale_x * scale_y), scale_x = r_xx(0) of
 *    series 1 on itself, same for series 2 ("CCF via real-space ...").
 *  - b_k = max(effective pair count, 1e-16); count_k = raw number of pairs in
 *    the rectangle window (int64, exact). An empty window gives c_k = 0.
 *  - Optional per-sample errors err_i > 0 give weights w_i = 1/err_i^2: the
 *    mean and sd become weighted, and C and B weight each pair by w_i w_j.
 *    b and count stay unweighted. (An extension: the paper defines no
 *    weighted estimator.)
 *  - Lags may come in any order, repeat, or be negative; outputs are in the
 *    order of the request.
 *
 * Memory and ownership
 *  - By default every array argument is a HOST pointer; the call copies in,
 *    computes on the current HIP device and returns when the outputs are
 *    written.
 *  - With NCF_DEVICE_POINTERS in options->flags, every data array (times,
 *    values, errors, lags, outputs) is a DEVICE pointer on options->stream.
 *    Batch offset arrays and per-series bandwidths are always HOST arrays.
 *    The call still returns only after the outputs are written.
 *  - The caller owns all buffers; the library keeps no caller pointer after
 *    return. Device workspace is cached by the library per device and freed
 *    by ncf_release_workspace() or at process exit.
 *  - The environment variable NCF_WORKSPACE_LIMIT_MB (MiB, read once per
 *    process) bounds the device workspace arenas of a call or a plan: a call
 *    that would need more returns NCF_E_NOMEM with a message before
 *    allocating, and the library stays usable for smaller calls. Unset or
 *    not a positive number: no bound beyond the device's memory.
 *  - NCF_LOG (read at each call): 1 prints one line per call and per plan
 *    build on stderr (kind, sizes, kernel, precision, route, grids, window
 *    work, fallback lags, failed problems, status, host time); 2 adds each
 *    autotuner candidate; 3 the host time of each planning step.
 *  - NCF_AUTOTUNE_CACHE names the autotune cache file (see
 *    ncf_plan_info_t.tune_cached).
 *
 * Errors
 *  - Every entry point returns NCF_OK (0) or a negative NCF_E_* code; on an
 *    error the outputs are unspecified and ncf_last_error() returns a
 *    message (thread-local, valid until the next call on the thread).
 *    Batch calls also fill an optional per-series status array; the call
 *    itself then returns the first non-zero per-series status, if any.
 */
#ifndef NCF_H
#define NCF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NCF_OK 0
#define NCF_E_INVALID_ARG (-1) /* null pointer, n < 2, K < 0, h <= 0, non-finite input, err <= 0 */
#define NCF_E_UNSORTED (-2)    /* times not non-decreasing */
#define NCF_E_DEGENERATE (-3)  /* sd = 0, or lag-0 scale (ACF r(0), CCF scale product) <= 0 */
#define NCF_E_NOMEM (-4)       /* device or host allocation failed, or workspace bound reached */
#define NCF_E_DEVICE (-5)      /* HIP runtime error, or no GPU */
#define NCF_E_UNSUPPORTED (-6) /* option combination not implemented */

typedef enum { NCF_GAUSSIAN = 0, NCF_RECTANGLE = 1 } ncf_kernel_t;

/* NCF_MIXED: FP32 spreading / FFT / kernel weights with FP64 positions,
 * phases, moments, prefix sums and accumulators. c is divided by the lag-0
 * scale (ACF r(0), CCF sqrt(r_x(0) r_y(0)) of the standardized values), which
 * is of order 1 unless the kernel spans much of a short series and the lag-0
 * sums cancel; the FP32 weights and transforms leave a relative error of
 * about 1e-6 / r(0) on it. So a Gaussian problem whose smaller lag-0 scale
 * comes out below 0.1 is evaluated again in FP64 within the call (same
 * method) and reports the FP64 result; see the plans for their handling.
 * NCF_FP64: every step in FP64. */
typedef enum { NCF_MIXED = 0, NCF_FP64 = 1 } ncf_precision_t;

/* Every method: a problem with a series of fewer than 32 samples takes the
 * direct window sums (NCF_DIRECT), whatever the method and flags ask.
 * NCF_AUTO: Gaussian numerator by the spectral (Wiener-Khinchin + NUFFT)
 *   route (Sec. 2.6), unless the call is small enough that the direct window
 *   sums cost less (then as NCF_DIRECT; see NCF_SPECTRAL_ALWAYS). The Gaussian
 *   pair count b takes the same route with unit values (with errors: the
 *   weighted pair sum B with the weights, and b with unit values), and lags
 *   whose spectral b (B), times min(1, s) with s the lag-0 scale (ACF r(0),
 *   CCF sqrt(r_x(0) r_y(0)), below 1 when the lag-0 sums of the standardized
 *   values cancel), falls below a fraction beta of the reference (b(0) for
 *   the ACF, sqrt(b_xx(0) b_yy(0)) of the two series for the CCF: both bound
 *   b at every lag, requested or not; beta = 0.1 mixed, 0.01 FP64) are
 *   summed directly by the window scan. Rectangle:
 *   numerator by prefix sums over the window (Algorithm "CorrSum,
 *   rectangle") and exact pair counts from the window scan.
 * NCF_SPECTRAL: Gaussian numerator by the spectral route, pair counts by the
 *   window scan, and the direct numerator at lags where b min(1, s) is below
 *   beta times the same reference; for the rectangle kernel the spectral route with the box
 *   kernel's Fourier transform (diagnostic: its truncation error decays only
 *   as 1/f).
 * NCF_DIRECT: numerator and pair counts by the window scan (real-space
 *   estimator, Appendix B); with NCF_FP64 this is the plain FP64 GPU path. */
typedef enum { NCF_AUTO = 0, NCF_SPECTRAL = 1, NCF_DIRECT = 2 } ncf_method_t;

#define NCF_DEVICE_POINTERS 0x1u
/* Plans only: replay the recorded launches one by one instead of as one
 * captured HIP graph. */
#define NCF_PLAN_NO_GRAPH 0x2u
/* Scheduling: run the window scans as persistent workgroups that pull
 * (series, outer-sample tile, lag tile) work items from a device queue,
 * instead of one workgroup per item. Results are identical. Gaussian
 * window scans of 100,000 items or more use the queue without the flag
 * (except in the allocation-free entry point). */
#define NCF_WINDOW_QUEUE 0x4u
/* Plans only: build and time candidate scheduling settings (minimum grid
 * oversampling, FFT radix split and strided-pass tile, window tile scale,
 * window dispatch) by coordinate descent from the defaults, and keep the
 * fastest. Results may differ from an untuned plan at the rounding level
 * (another grid size or FFT order); building takes several plan builds. */
#define NCF_PLAN_AUTOTUNE 0x8u
/* NCF_AUTO with the Gaussian kernel normally picks, per call, the direct
 * window sums when their estimated work is below the spectral pipeline's
 * (small problems; the paper's K* crossover). With this flag it always takes
 * the spectral route. */
#define NCF_SPECTRAL_ALWAYS 0x10u

typedef struct {
    uint32_t struct_size; /* sizeof(ncf_options_t) */
    int32_t precision;    /* ncf_precision_t, default NCF_MIXED */
    int32_t method;       /* ncf_method_t, default NCF_AUTO */
    double tol;           /* spectral truncation target, 0 = default (1e-9 mixed, 1e-13 FP64) */
    double sigma;         /* minimum grid oversampling factor, 0 = default (1.5) */
    int64_t grid_size;    /* 0 = planned from h, L and tol; else a power of two to force */
    void* stream;         /* hipStream_t; NULL = the null stream */
    uint32_t flags;       /* NCF_DEVICE_POINTERS */
    uint32_t reserved;
} ncf_options_t;

/* Fill *opt with defaults. */
void ncf_options_init(ncf_options_t* opt);

/* Autocorrelation of one series.
 *   n       number of samples (>= 2)
 *   t, x    times (sorted) and values, n each; err optional (NULL or n)
 *   K       number of lags (>= 0); lags[K]
 *   kern, h kernel and bandwidth (Gaussian sd / rectangle half-width), h > 0
 *   c, b    outputs, K each; count optional output (K int64; rectangle pair
 *           counts, zeros for the Gaussian kernel)
 *   opt     NULL for defaults. */
int ncf_acf(int64_t n, const double* t, const double* x, const double* err, int64_t K,
            const double* lags, int kern, double h, double* c, double* b, int64_t* count,
            const ncf_options_t* opt);

/* Cross-correlation of series 1 (nx samples: tx, x, ex) and series 2 (ny
 * samples: ty, y, ey); arguments as in ncf_acf. */
int ncf_ccf(int64_t nx, const double* tx, const double* x, const double* ex, int64_t ny,
            const double* ty, const double* y, const double* ey, int64_t K, const double* lags,
            int kern, double h, double* c, double* b, int64_t* count, const ncf_options_t* opt);

/* Autocorrelation of nser independent series in one call (CSR layout).
 *   offs    HOST array of nser+1 offsets into t, x, err (offs[0] = 0)
 *   lags    K lags shared by every series
 *   h       HOST array of nser bandwidths
 *   c, b    nser*K outputs, series-major; count optional nser*K
 *   status  optional HOST array of nser per-series status codes. */
int ncf_acf_batch(int64_t nser, const int64_t* offs, const double* t, const double* x,
                  const double* err, int64_t K, const double* lags, int kern, const double* h,
                  double* c, double* b, int64_t* count, int* status, const ncf_options_t* opt);

/* Cross-correlation of npair series pairs in one call: series 1 of pair p
 * is tx/x/ex[offx[p] .. offx[p+1]), series 2 is ty/y/ey[offy[p] ..
 * offy[p+1]); other arguments as in ncf_acf_batch. */
int ncf_ccf_batch(int64_t npair, const int64_t* offx, const double* tx, const double* x,
                  const double* ex, const int64_t* offy, const double* ty, const double* y,
                  const double* ey, int64_t K, const double* lags, int kern, const double* h,
                  double* c, double* b, int64_t* count, int* status, const ncf_options_t* opt);

/* Allocation-free cross-correlation, for callers that cannot allocate device
 * memory during the call (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation). Arguments, outputs and errors as in
 * ncf_ccf; the estimate is that of ncf_ccf with method NCF_DIRECT (the
 * real-space window sums, exact rectangle counts; options->method and the
 * scheduling flags are ignored, NCF_DEVICE_POINTERS and the stream are
 * honoured).
 *  - The call allocates no device or pinned host memory and frees none: its
 *    workspace is a fixed 64 MiB array per device, held by the library from
 *    its load until the process ends, and its small tables go through a
 *    fixed 4 MiB host buffer. A call whose workspace would exceed them returns
 *    NCF_E_UNSUPPORTED with a message (roughly: 16 B per sample for the
 *    rectangle kernel, 8 B for the Gaussian, +16 B with host pointers, plus
 *    about K x ny / 8 B of window partial sums; a 1e6 + 1e6-sample rectangle
 *    CCF with 64 lags fits).
 *  - Every call on a device shares that device's workspace, which keeps the
 *    last call's contents; nothing in it needs to start at zero. Calls are
 *    serialized by the library's lock and each returns when its kernels are
 *    done, so two calls of one process do not overlap; work that overlapped
 *    them on the device (e.g. replayed captures of an earlier call) would
 *    race on the workspace.
 *  - In NCF_MIXED with the Gaussian kernel, a problem whose smaller lag-0
 *    scale is below 0.1 is not evaluated again in FP64 (that needs more
 *    workspace): it returns NCF_E_UNSUPPORTED with c = NaN, as plans do. */
int ncf_ccf_noalloc(int64_t nx, const double* tx, const double* x, const double* ex,
                    int64_t ny, const double* ty, const double* y, const double* ey, int64_t K,
                    const double* lags, int kern, double h, double* c, double* b,
                    int64_t* count, const ncf_options_t* opt);

/* ------------------------------------------------ regular-lattice family
 * Classic-FFT estimators for series sampled on a regular time lattice
 * (Sec. "Regularly-sampled data"; eq. wienerkhinchin of Sec. "Correlation
 * estimation on a regular grid"). They compute the same Gaussian/rectangle
 * kernel estimator (eq. kernel_estimator) as ncf_acf / ncf_ccf, at a cost
 * of O(N log N) with N ~ 2 x the lattice length, independent of K: one FP64
 * FFT correlation gives the raw lag correlations R(q) of the lattice grids
 * and the raw pair counts N(q) of the sample-count grids (the ramp n - |q|
 * without gaps), and every requested lag filters them with the kernel
 * weights (the pair count is the filtered N, as Sec. "Effective pair count"
 * describes for this family).
 *
 *  - Lattice: t_i = t_ref + m_i dt with integer m_i, where t_ref is the
 *    first time of the series (CCF: of either series, so both series must
 *    share one lattice). Gaps (missing m) and repeated times are allowed;
 *    times must be non-decreasing. A time farther than 1e-6 dt from its
 *    lattice point gives NCF_E_INVALID_ARG for its series (pair). dt > 0 is
 *    given by the caller (one per problem in the batch calls).
 *  - Reading of the estimator on the lattice: each sample sits exactly at
 *    its lattice point, so a pair's lag is q dt. Lattice lag q is in the
 *    window of lag tau when q lies between (tau - W)/dt and (tau + W)/dt
 *    (W = 6h Gaussian, h rectangle), each bound first rounded to the
 *    nearest integer when within 1e-9 (relative) of it, with the open and
 *    closed ends of the irregular estimator: Gaussian ACF [lo, hi), Gaussian
 *    CCF (lo, hi] (lag q = m_y - m_x), rectangle [lo, hi]. The weight is
 *    the kernel at q dt - tau. Where the times, lags, dt and h are exact
 *    binary fractions this is exactly the estimator of ncf_acf / ncf_ccf.
 *  - Always computed in FP64 (options->precision and ->method are
 *    ignored): the pair counts come out exact (count) and c agrees with the
 *    direct FP64 sums to ~1e-12.
 *  - Outputs, statuses, host/device pointers and streams as in the batch
 *    calls; lags may be any finite values (not only multiples of dt).
 *  - The lattice length (last time - t_ref)/dt + 1 plus the largest lag
 *    reach (max|tau| + W)/dt must stay below 2^31 (else NCF_E_UNSUPPORTED).
 */
int ncf_acf_regular(int64_t n, const double* t, const double* x, const double* err, double dt,
                    int64_t K, const double* lags, int kern, double h, double* c, double* b,
                    int64_t* count, const ncf_options_t* opt);

int ncf_ccf_regular(int64_t nx, const double* tx, const double* x, const double* ex, int64_t ny,
                    const double* ty, const double* y, const double* ey, double dt, int64_t K,
                    const double* lags, int kern, double h, double* c, double* b,
                    int64_t* count, const ncf_options_t* opt);

/* Batched forms (layout as in ncf_acf_batch / ncf_ccf_batch); dt is a HOST
 * array of one lattice step per series (pair). */
int ncf_acf_regular_batch(int64_t nser, const int64_t* offs, const double* t, const double* x,
                          const double* err, const double* dt, int64_t K, const double* lags,
                          int kern, const double* h, double* c, double* b, int64_t* count,
                          int* status, const ncf_options_t* opt);

int ncf_ccf_regular_batch(int64_t npair, const int64_t* offx, const double* tx, const double* x,
                          const double* ex, const int64_t* offy, const double* ty,
                          const double* y, const double* ey, const double* dt, int64_t K,
                          const double* lags, int kern, const double* h, double* c, double* b,
                          int64_t* count, int* status, const ncf_options_t* opt);

/* ------------------------------------------------- replicate error bars
 * Per-lag uncertainties by Monte-Carlo and bootstrap resampling, which the
 * paper leaves to the user (Sec. "Discussion": the estimator supplies no
 * per-lag error bars; they come from bootstrap or Monte-Carlo resampling of
 * the data, as pyZDCF does internally). R replicates of the series are
 * estimated as one batch over shared times; the call returns, per lag, the
 * mean and the sample standard deviation (R - 1 denominator) of c over the
 * replicates that succeed.
 *
 * Replicate r (0 <= r < R) of a series of n samples:
 *  - values x_i + sigma_i z[r*n + i] (flux randomization) when z is given;
 *    z holds caller-drawn deviates (normal for the usual scheme), sigma the
 *    per-sample scale (often the measurement errors). z and sigma go
 *    together; without them the values are x.
 *  - sample i counted mult[r*n + i] >= 0 times (bootstrap resampling with
 *    replacement: the multiplicities of n draws; 0 drops the sample) when
 *    mult is given. A sample counted k times is exactly the series with that
 *    sample repeated k times: the estimator runs with sample weights k
 *    (times 1/err_i^2 when err is given), which give the repeated series'
 *    mean, sd and pair sums.
 *  - err (nullable) weights the estimator as in ncf_acf; it is not used to
 *    perturb the values (pass it as sigma too for that).
 * The replicates use the precision and method of the options, as ncf_acf
 * does; with the default method their Gaussian pair sums (weighted by the
 * multiplicities) come from the spectral route, with the direct fallback
 * of NCF_AUTO for lags with few pairs. Arrays follow NCF_DEVICE_POINTERS (then t, x, err, sigma, z, mult,
 * lags, c_mean, c_sd and c_rep are device arrays); status is a HOST array.
 *   c_mean, c_sd  K outputs each (NaN where fewer than 1 / 2 replicates
 *                 succeed)
 *   c_rep         optional R*K output: every replicate's c (NaN for a
 *                 replicate that failed)
 *   status        optional R per-replicate statuses (a bootstrap draw that
 *                 leaves a constant series gives NCF_E_DEGENERATE)
 * Returns NCF_OK when at least one replicate succeeds, else the first
 * replicate's status; argument errors as in ncf_acf. n x R must stay below
 * 4e9 (NCF_E_UNSUPPORTED). */
int ncf_acf_resample(int64_t n, const double* t, const double* x, const double* err,
                     const double* sigma, int64_t R, const double* z, const int32_t* mult,
                     int64_t K, const double* lags, int kern, double h, double* c_mean,
                     double* c_sd, double* c_rep, int* status, const ncf_options_t* opt);

/* Cross-correlation replicates: series 1 (nx samples: tx, x, ex, sx, zx,
 * multx) and series 2 (ny samples: ty, y, ey, sy, zy, multy), each
 * resampled with its own deviates and multiplicities (R*nx and R*ny);
 * other arguments as in ncf_acf_resample. */
int ncf_ccf_resample(int64_t nx, const double* tx, const double* x, const double* ex,
                     const double* sx, const double* zx, const int32_t* multx, int64_t ny,
                     const double* ty, const double* y, const double* ey, const double* sy,
                     const double* zy, const int32_t* multy, int64_t R, int64_t K,
                     const double* lags, int kern, double h, double* c_mean, double* c_sd,
                     double* c_rep, int* status, const ncf_options_t* opt);

/* ----------------------------------------------------------------- plans
 * A plan fixes everything of a batch call except the values: times, errors,
 * lags, kernel, bandwidths and options. Building it runs the whole path once
 * on placeholder values, which fixes the grids, the window tiles and the
 * lags that the direct fallback sums (those depend on the times only), and
 * records every kernel launch; unless NCF_PLAN_NO_GRAPH is set the launches
 * are then captured into one HIP graph. Each execution takes new values
 * (series 1 and, for a CCF, series 2, laid out as at build time), writes
 * the same outputs as the batch call and needs no host-side planning. Use:
 * Monte-Carlo or bootstrap over values at fixed sampling, repeated
 * estimates in a serving loop (the batch scheduler of the paper's "batch
 * processing of large numbers of light curves" use, Sec. 1).
 *
 *  - Arrays given to ncf_plan_acf / ncf_plan_ccf follow the batch calls
 *    (host pointers, or device pointers with NCF_DEVICE_POINTERS; offsets
 *    and bandwidths on the host). The plan copies times and errors into its
 *    own device memory; the caller may free them after the call.
 *  - The plan owns all its device memory (released by ncf_plan_destroy).
 *    Series that fail the time checks (unsorted or non-finite times, bad h)
 *    do not fail the build: every execution reports them in `status`.
 *  - Executions run on options->stream of the build. Host-pointer plans
 *    return when the outputs are written, with the first failing per-series
 *    status. Device-pointer plans only enqueue: x, y, c, b, count and status
 *    are device arrays, status (nullable, int32 per series) is written on the
 *    stream, and the return value reports launch errors only.
 *  - Executions of one plan are ordered on its stream; a plan must not be
 *    executed from two threads at once. Pair counts and fallback lags are
 *    those of the build, so results can differ from a batch call on the
 *    same inputs at the rounding level of the spectral pair count.
 *  - A plan replays fixed launches, so it cannot evaluate a problem again in
 *    FP64 on its values: in NCF_MIXED with the Gaussian kernel, a problem
 *    whose smaller lag-0 scale is below 0.1 on the executed values reports
 *    NCF_E_UNSUPPORTED in `status` (c = NaN); build the plan with NCF_FP64
 *    for such series. */
typedef struct ncf_plan_s ncf_plan_t;

/* Build an ACF plan for nser series (arguments as in ncf_acf_batch, without
 * values and outputs). *out receives the plan, NULL on failure. */
int ncf_plan_acf(int64_t nser, const int64_t* offs, const double* t, const double* err,
                 int64_t K, const double* lags, int kern, const double* h,
                 const ncf_options_t* opt, ncf_plan_t** out);

/* Build a CCF plan for npair series pairs (arguments as in ncf_ccf_batch,
 * without values and outputs). */
int ncf_plan_ccf(int64_t npair, const int64_t* offx, const double* tx, const double* ex,
                 const int64_t* offy, const double* ty, const double* ey, int64_t K,
                 const double* lags, int kern, const double* h, const ncf_options_t* opt,
                 ncf_plan_t** out);

/* Plans of the regular-lattice estimators (arguments as in
 * ncf_acf_regular_batch / ncf_ccf_regular_batch, without values and
 * outputs; dt a HOST array of one lattice step per series or pair). The
 * lattice check of the times is part of every execution: a series off its
 * lattice reports NCF_E_INVALID_ARG in `status`. */
int ncf_plan_acf_regular(int64_t nser, const int64_t* offs, const double* t, const double* err,
                         const double* dt, int64_t K, const double* lags, int kern,
                         const double* h, const ncf_options_t* opt, ncf_plan_t** out);

int ncf_plan_ccf_regular(int64_t npair, const int64_t* offx, const double* tx, const double* ex,
                         const int64_t* offy, const double* ty, const double* ey,
                         const double* dt, int64_t K, const double* lags, int kern,
                         const double* h, const ncf_options_t* opt, ncf_plan_t** out);

/* Run a plan on values x (series 1, CSR as at build) and y (series 2 of a
 * CCF plan, NULL for an ACF plan); outputs as in the batch calls. */
int ncf_plan_execute(ncf_plan_t* plan, const double* x, const double* y, double* c, double* b,
                     int64_t* count, int* status);

/* Release a plan (NULL is ignored). Waits for the device to finish. */
void ncf_plan_destroy(ncf_plan_t* plan);

/* What a plan holds and how it was scheduled. Set struct_size first. */
typedef struct {
    uint32_t struct_size;      /* sizeof(ncf_plan_info_t) */
    int32_t autotuned;         /* 1 if built with NCF_PLAN_AUTOTUNE */
    int32_t candidates;        /* settings timed by the autotuner */
    int32_t spectral_grids;    /* spreading grids (spectral problems; regular plans: lattice problems) */
    int32_t window_launches;   /* window-scan launches per execution */
    int32_t graph;             /* 1 if executions replay a captured graph */
    int64_t grid_cells;        /* cells over all grids (transform length) */
    int64_t window_items;      /* window work items per execution */
    double sigma;              /* minimum grid oversampling chosen, 0 = default */
    int32_t fft_split;         /* 0 default radices, 1 swapped order, 2 three passes */
    int32_t fft_tile_log2;     /* strided-pass tile, 0 = default */
    int32_t window_tile_scale; /* log2 factor on the outer samples per workgroup */
    int32_t window_queue;      /* 1: work-queue dispatch of the window scans */
    double replay_ms;          /* autotuned: measured time of one execution */
    int32_t lattice_grids;     /* grids whose lags are read off the folded spectrum (lags on a
                                  lattice: Sec. "The Non-Uniform Fast Fourier Transform",
                                  type-2 step at equispaced points) */
    int32_t lattice_off;       /* 1: the autotuner chose inverse transform + interpolation
                                  although the lags sit on a lattice */
    int32_t tune_cached;       /* 1: NCF_PLAN_AUTOTUNE took its settings from the autotune
                                  cache (file named by the NCF_AUTOTUNE_CACHE environment
                                  variable, one JSON record per line; a plan tuned anew
                                  appends its record there) instead of timing candidates */
} ncf_plan_info_t;

int ncf_plan_info(const ncf_plan_t* plan, ncf_plan_info_t* info);

/* Message describing the last failure on the calling thread ("" if none). */
const char* ncf_last_error(void);

/* Free the cached device workspace of the current device. */
void ncf_release_workspace(void);

/* Library version, e.g. 100 for 0.1.0. */
int ncf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NCF_H */
