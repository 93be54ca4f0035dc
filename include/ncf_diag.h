/*
 * ncf_diag.h -- stage-level and profiling entry points of the ncf library.
 *
 * These expose single stages of the spectral route so that each can be
 * checked on its own against its textbook definition, and a per-kernel
 * event timer used for roofline accounting. Array conventions, error codes
 * and ownership are those of ncf.h; every array here is a HOST pointer.
 */
#ifndef NCF_DIAG_H
#define NCF_DIAG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Discrete Fourier transform of N complex values (N a power of two,
 * 4096 <= N <= 2^30), interleaved (re, im), FP32 (precision 0) or FP64
 * (precision 1), in place on the host array `data`, natural order in and out.
 *   sign = +1: X[k] = sum_n x[n] exp(+2 pi i n k / N)   (type-1 side,
 *              eq. nufft_type1 with the isign = +1 convention)
 *   sign = -1: X[k] = sum_n x[n] exp(-2 pi i n k / N)   (type-2 side)
 * No 1/N factor either way. Internally the forward (+1) transform leaves its
 * output in mixed-radix digit-reversed order and the -1 transform consumes
 * that order; this entry point applies the permutation so that callers see
 * natural order. */
int ncf_diag_fft(int64_t N, int precision, int sign, void* data);

/* Pass radices of the N-point transform (first pass first). Returns the
 * number of passes (<= max), or a negative NCF_E_* code. */
int ncf_diag_fft_radices(int64_t N, int* radices, int max);

/* Type-1 non-uniform transform of eq. nufft_type1 on a period L:
 *   X_m = sum_i v_i exp(+2 pi i m (t_i - t_ref) / L),  m = -M .. M
 * computed by Gaussian-kernel gridding on N cells, FFT and deconvolution
 * (Sec. 2.5), with the library's spreading parameters for `precision` and
 * grid size N (power of two, N >= 2M+1). The sample positions must satisfy
 * the library's no-wrap condition, checked here: every (t_i - t_ref) N / L
 * lies at least the spreading half-width inside (0, N).
 * out: 2*(2M+1) doubles, (re, im) for m = -M .. M. */
int ncf_diag_type1(int64_t n, const double* t, const double* v, double t_ref, double L,
                   int64_t N, int64_t M, int precision, double* out);

/* Spreading parameters the planner uses for a grid oversampling factor
 * sigma and tolerance eps: out[0] = Gaussian width s (cells), out[1] =
 * truncation half-width W (cells). */
int ncf_diag_spread_params(double sigma, double eps, double* out);

/* Grid geometry the planner picks for one Gaussian spectral problem (host
 * only; no device is needed), Sec. "From kernel-weighted estimators to
 * NUFFT" with the period and mode count of the type-1 / type-2 steps
 * (eq. nufft_type1, nufft_type2). Samples span [tmin, tmax]; `lags` holds
 * the K evaluation lags (with acf != 0 lag 0 is evaluated too); bandwidth h;
 * precision NCF_MIXED or NCF_FP64; `lattice` != 0 allows the lag-lattice
 * evaluation (lags read off the spectrum folded modulo P) where the lags sit
 * on a lattice. Outputs: out_f[0] = period L, out_f[1] = spreading width s
 * (cells); out_i[0] = cells N, out_i[1] = retained modes M, out_i[2] = P
 * (0: inverse transform and interpolation). Returns NCF_E_INVALID_ARG for
 * bad arguments, NCF_E_UNSUPPORTED when no grid of at most 2^31 cells fits. */
int ncf_diag_grid(double tmin, double tmax, int64_t K, const double* lags, int acf, double h,
                  int precision, int lattice, double* out_f, int64_t* out_i);

/* ------------------------------------------------------------ profiling */

/* Enable (1) or disable (0) per-kernel HIP-event timing on the stream each
 * kernel is launched on. Enabling clears the accumulated records. */
void ncf_profile_enable(int on);

/* Restrict the timing to launches of one kernel name (as reported by
 * ncf_profile_read); NULL or "" times every kernel. Each timed launch records
 * two events on its stream, from a pool the library keeps for reuse. */
void ncf_profile_filter(const char* name);

typedef struct {
    char name[48];     /* kernel name */
    int64_t launches;  /* number of timed launches */
    double total_ms;   /* summed event durations */
    double work;       /* summed algorithmic work of those launches */
    char work_unit[16];/* "bytes" (HBM-bound kernels) or "valu_ops" */
} ncf_profile_record_t;

/* Copy up to max records (one per kernel name) into out; returns the count.
 * Synchronizes the device first. */
int ncf_profile_read(ncf_profile_record_t* out, int max);

#ifdef __cplusplus
}
#endif

#endif /* NCF_DIAG_H */
