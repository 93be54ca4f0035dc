/*
 * ncf_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of the kernel-weighted
 * auto/cross-correlation estimator for irregularly sampled series
 * (the "real-space" estimator of the paper's Appendix B, Algorithms
 * "CorrSum" and "PairCount", assembled as in "ACF via real-space
 * kernel-weighted summation" and "CCF via real-space kernel-weighted
 * summation"; the estimator itself is eq. kernel_estimator of Sec. 2.3).
 *
 * It exists to check the GPU library. Only the test suite, the smoke
 * entry point and the benchmark's CPU-baseline leg may load it. It shares
 * no code, header or constant with the GPU library: the status codes below
 * are redefined here on purpose and only mirror the public interface.
 *
 * What it computes (series 1 = (t_i, x_i), series 2 = (s_j, y_j)):
 *   d = (t_i) - (s_j + eps*tau)       (eps = +1 ACF, -1 CCF; Appendix A.2)
 *   Gaussian kernel  (eq. Gaussian_kernel): weight phi(d) on the window
 *       t_i >= centre - 6h  and  t_i < centre + 6h   (PairCount, Gaussian)
 *   Rectangle kernel (PairCount, rectangle): weight 1 on the closed window
 *       t_i >= centre - h  and  t_i <= centre + h     (h = half-width)
 *   C(tau) = sum over window pairs of weight * v_i * v_j
 *   B(tau) = sum over window pairs of weight * w_i * w_j
 *   b(tau) = sum over window pairs of weight          (effective pair count)
 *   count  = number of window pairs                   (rectangle only)
 * with v = w * (x - mean)/sd the standardized values and w the per-sample
 * weight (1 without errors; 1/err^2 with errors, an extension the paper does
 * not define -- "parity unpinned" beyond the invariances the tests check).
 *
 *   r(tau) = C(tau) / max(B(tau), 1e-16)       (floor of PairCount)
 *   ACF: c_k = r(tau_k) / r(0)                 (lag-0 normalization, Alg. ACF via NUFFT)
 *   CCF: c_k = r_xy(tau_k) / sqrt(scale_x * scale_y),
 *        scale_x = C_xx(0)/max(B_xx(0),1e-16) on (t,x) with eps=+1, same for y
 *        (Algorithm "CCF via real-space kernel-weighted summation").
 *
 * The sums are taken straight from the definition: for each lag and each
 * outer sample j the window is the set of window samples i that satisfy the
 * predicate above. Since the window times are sorted that set is one run of
 * consecutive indices; its two ends are found by bisection on the predicate
 * and every pair in the run is summed directly (the rectangle numerator too,
 * never by prefix sums, so this file does not use the prefix-sum form the
 * GPU path relies on). A brute-force all-pairs mode tests the predicate on
 * every pair instead.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_E_INVALID_ARG (-1)
#define ORC_E_UNSORTED (-2)
#define ORC_E_DEGENERATE (-3)
#define ORC_E_NOMEM (-4)

#define ORC_GAUSSIAN 0
#define ORC_RECTANGLE 1

static const double ORC_FLOOR = 1e-16;
/* A lag-0 scale at or below this is degenerate. For standardized values r(0)
 * is of order 1; a kernel wide enough to hold every pair of a short series
 * makes the lag-0 sum (sum of z)^2 = 0 in exact arithmetic, and its rounded
 * value (~1e-16, either sign) must not decide the status. */
static const double ORC_MIN_SCALE = 1e-12;

/* ---------------------------------------------------------------- checks */

static int check_series(int64_t n, const double* t, const double* x, const double* err) {
    if (n < 2 || !t || !x) return ORC_E_INVALID_ARG;
    for (int64_t i = 0; i < n; ++i) {
        if (!isfinite(t[i]) || !isfinite(x[i])) return ORC_E_INVALID_ARG;
        if (err && (!isfinite(err[i]) || !(err[i] > 0.0))) return ORC_E_INVALID_ARG;
    }
    for (int64_t i = 1; i < n; ++i)
        if (t[i] < t[i - 1]) return ORC_E_UNSORTED;
    return ORC_OK;
}

static int check_lags(int64_t K, const double* lags, double h) {
    if (K < 0 || (K > 0 && !lags)) return ORC_E_INVALID_ARG;
    if (!isfinite(h) || !(h > 0.0)) return ORC_E_INVALID_ARG;
    for (int64_t k = 0; k < K; ++k)
        if (!isfinite(lags[k])) return ORC_E_INVALID_ARG;
    return ORC_OK;
}

/* ----------------------------------------------------- standardization */

/* Mean and standard deviation (ddof 0), weighted by w = 1/err^2 when err is
 * given; v = w * (x - mean) / sd, w written alongside (all ones without err).
 * Plain left-to-right FP64 sums. */
int oracle_standardize(int64_t n, const double* x, const double* err, double* v, double* w) {
    double sw = 0.0, swx = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double wi = err ? 1.0 / (err[i] * err[i]) : 1.0;
        w[i] = wi;
        sw += wi;
        swx += wi * x[i];
    }
    double mean = swx / sw;
    double swd = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double d = x[i] - mean;
        swd += w[i] * d * d;
    }
    double sd = sqrt(swd / sw);
    if (!(sd > 0.0) || !isfinite(sd)) return ORC_E_DEGENERATE;
    for (int64_t i = 0; i < n; ++i) v[i] = w[i] * ((x[i] - mean) / sd);
    return ORC_OK;
}

/* ------------------------------------------------------ kernel weights */

static double gauss_weight(double d, double h) {
    /* eq. Gaussian_kernel */
    return exp(-(d * d) / (2.0 * h * h)) / (h * sqrt(2.0 * M_PI));
}

/* ------------------------------------------------- scan over one lag */

typedef struct {
    int kernel, eps;
    int64_t n_out;
    const double *s, *v_out, *w_out;
    int64_t n_win;
    const double *t, *v_win, *w_win;
    double h;
    /* lattice reading (regular-lattice estimators): lattice indices of the
     * outer and window samples and the step; m_out == NULL for real times */
    const int64_t *m_out, *m_win;
    double dt;
} scan_args;

/* Bisection over a sorted array: the number of leading entries that satisfy
 * a predicate that holds for a prefix of the array (true, ..., true, false,
 * ..., false). `below(i)` is that predicate; `ctx` is passed through. */
typedef int (*prefix_pred)(const void* ctx, int64_t i);

static int64_t prefix_length(const void* ctx, int64_t n, prefix_pred below) {
    int64_t lo = 0, hi = n; /* below(i) for i < lo; !below(i) for i >= hi */
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (below(ctx, mid))
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

typedef struct {
    const double* t;
    double key;
} time_key;

static int time_lt(const void* c, int64_t i) {
    const time_key* k = (const time_key*)c;
    return k->t[i] < k->key;
}

static int time_le(const void* c, int64_t i) {
    const time_key* k = (const time_key*)c;
    return k->t[i] <= k->key;
}

/* Window sums for one lag from the definition (eq. kernel_estimator with
 * the window predicates of PairCount): for outer sample j with centre
 * s_j + eps*tau, the window samples are those with t_i >= centre - W and
 * t_i < centre + W (Gaussian, W = 6h) or t_i <= centre + h (rectangle).
 * With t sorted they are the indices [lo, hi): lo counts the t_i below
 * centre - W, hi those below centre + W (Gaussian) or at most centre + h
 * (rectangle). */
static void scan_one_lag(const scan_args* a, double tau, double* C, double* B, double* b,
                         int64_t* count) {
    double c_acc = 0.0, B_acc = 0.0, b_acc = 0.0;
    int64_t n_acc = 0;
    const double e = (double)a->eps;
    const int gauss = a->kernel == ORC_GAUSSIAN;
    const double W = gauss ? 6.0 * a->h : a->h;
    for (int64_t j = 0; j < a->n_out; ++j) {
        const double centre = a->s[j] + e * tau;
        time_key klo = {a->t, centre - W}, khi = {a->t, centre + W};
        const int64_t lo = prefix_length(&klo, a->n_win, time_lt);
        const int64_t hi = prefix_length(&khi, a->n_win, gauss ? time_lt : time_le);
        for (int64_t i = lo; i < hi; ++i) {
            const double wt = gauss ? gauss_weight(a->t[i] - centre, a->h) : 1.0;
            c_acc += wt * a->v_win[i] * a->v_out[j];
            B_acc += wt * a->w_win[i] * a->w_out[j];
            b_acc += wt;
            n_acc += 1;
        }
    }
    *C = c_acc;
    *B = B_acc;
    *b = b_acc;
    *count = n_acc;
}

/* ------------------------------------------- lattice reading of the scan */

/* Regular-lattice estimators (Sec. "Regularly-sampled data"): every sample
 * sits at its lattice point t_ref + m dt, so the pair (i, j) has lag
 * (m_i - m_j) dt and d = (m_i - m_j) dt - eps*tau. The window is decided in
 * lattice units: with lo = (eps*tau - W)/dt and hi = (eps*tau + W)/dt, each
 * rounded to the nearest integer when within 1e-9 (relative) of it, the pair
 * is in the window when lo <= m_i - m_j < hi (Gaussian, W = 6h) or
 * lo <= m_i - m_j <= hi (rectangle, W = h): the predicates above with the
 * times replaced by their lattice points. */
static double snap_edge(double e) {
    double r = nearbyint(e);
    return fabs(e - r) <= 1e-9 * fmax(1.0, fabs(e)) ? r : e;
}

typedef struct {
    const int64_t* m;
    int64_t mj;
    double edge;
} lattice_key;

static int lattice_lt(const void* c, int64_t i) {
    const lattice_key* k = (const lattice_key*)c;
    return (double)(k->m[i] - k->mj) < k->edge;
}

static int lattice_le(const void* c, int64_t i) {
    const lattice_key* k = (const lattice_key*)c;
    return (double)(k->m[i] - k->mj) <= k->edge;
}

static void lattice_one_lag(const scan_args* a, double tau, double* C, double* B, double* b,
                            int64_t* count) {
    double c_acc = 0.0, B_acc = 0.0, b_acc = 0.0;
    int64_t n_acc = 0;
    const double e = (double)a->eps;
    const int gauss = a->kernel == ORC_GAUSSIAN;
    const double W = gauss ? 6.0 * a->h : a->h;
    const double lo_edge = snap_edge((e * tau - W) / a->dt);
    const double hi_edge = snap_edge((e * tau + W) / a->dt);
    for (int64_t j = 0; j < a->n_out; ++j) {
        const int64_t mj = a->m_out[j];
        /* the lattice indices are sorted with the times: the window is
         * again one run [i_lo, i_hi) of window samples */
        lattice_key klo = {a->m_win, mj, lo_edge}, khi = {a->m_win, mj, hi_edge};
        const int64_t i_lo = prefix_length(&klo, a->n_win, lattice_lt);
        const int64_t i_hi = prefix_length(&khi, a->n_win, gauss ? lattice_lt : lattice_le);
        for (int64_t i = i_lo; i < i_hi; ++i) {
            const double q = (double)(a->m_win[i] - mj);
            const double wt = gauss ? gauss_weight(q * a->dt - e * tau, a->h) : 1.0;
            c_acc += wt * a->v_win[i] * a->v_out[j];
            B_acc += wt * a->w_win[i] * a->w_out[j];
            b_acc += wt;
            n_acc += 1;
        }
    }
    *C = c_acc;
    *B = B_acc;
    *b = b_acc;
    *count = n_acc;
}

/* All-pairs evaluation of the same window predicates (no scan). */
static void brute_one_lag(const scan_args* a, double tau, double* C, double* B, double* b,
                          int64_t* count) {
    double c_acc = 0.0, B_acc = 0.0, b_acc = 0.0;
    int64_t n_acc = 0;
    const double e = (double)a->eps;
    for (int64_t j = 0; j < a->n_out; ++j) {
        double centre = a->s[j] + e * tau;
        for (int64_t i = 0; i < a->n_win; ++i) {
            double ti = a->t[i];
            double wt;
            if (a->kernel == ORC_GAUSSIAN) {
                const double W = 6.0 * a->h;
                if (ti < centre - W || !(ti < centre + W)) continue;
                wt = gauss_weight(ti - centre, a->h);
            } else {
                if (ti < centre - a->h || !(ti <= centre + a->h)) continue;
                wt = 1.0;
            }
            c_acc += wt * a->v_win[i] * a->v_out[j];
            B_acc += wt * a->w_win[i] * a->w_out[j];
            b_acc += wt;
            n_acc += 1;
        }
    }
    *C = c_acc;
    *B = B_acc;
    *b = b_acc;
    *count = n_acc;
}

/* Window sums for every lag; the lags are independent and shared out over
 * threads. Outputs are raw (not floored). m_out/m_win: lattice
 * indices for the lattice reading, or NULL. */
static int window_sums(int kernel, int eps, int64_t n_out, const double* s, const double* v_out,
                       const double* w_out, int64_t n_win, const double* t, const double* v_win,
                       const double* w_win, const int64_t* m_out, const int64_t* m_win,
                       double dt, int64_t K, const double* lags, double h, double* C, double* B,
                       double* b, int64_t* count, int nthreads, int brute) {
    if (kernel != ORC_GAUSSIAN && kernel != ORC_RECTANGLE) return ORC_E_INVALID_ARG;
    if (eps != 1 && eps != -1) return ORC_E_INVALID_ARG;
    scan_args a = {kernel, eps, n_out, s, v_out, w_out, n_win, t, v_win, w_win, h,
                   m_out, m_win, dt};
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t k = 0; k < K; ++k) {
        if (m_out)
            lattice_one_lag(&a, lags[k], &C[k], &B[k], &b[k], &count[k]);
        else if (brute)
            brute_one_lag(&a, lags[k], &C[k], &B[k], &b[k], &count[k]);
        else
            scan_one_lag(&a, lags[k], &C[k], &B[k], &b[k], &count[k]);
    }
    (void)nthreads;
    return ORC_OK;
}

int oracle_window_sums(int kernel, int eps, int64_t n_out, const double* s, const double* v_out,
                       const double* w_out, int64_t n_win, const double* t, const double* v_win,
                       const double* w_win, int64_t K, const double* lags, double h, double* C,
                       double* B, double* b, int64_t* count, int nthreads, int brute) {
    return window_sums(kernel, eps, n_out, s, v_out, w_out, n_win, t, v_win, w_win, NULL, NULL,
                       0.0, K, lags, h, C, B, b, count, nthreads, brute);
}

/* Lattice indices m_i = round((t_i - t_ref)/dt); a time farther than
 * 1e-6 dt from its lattice point is rejected. */
static int lattice_indices(int64_t n, const double* t, double t_ref, double dt, int64_t* m) {
    for (int64_t i = 0; i < n; ++i) {
        double u = nearbyint((t[i] - t_ref) / dt);
        if (!(fabs(t[i] - (t_ref + u * dt)) <= 1e-6 * dt)) return ORC_E_INVALID_ARG;
        m[i] = (int64_t)u;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------ estimators */

static double floor_b(double v) { return v > ORC_FLOOR ? v : ORC_FLOOR; }

/* dt > 0: lattice reading with t_ref = t[0] (regular-lattice estimators) */
static int acf_impl(int64_t n, const double* t, const double* x, const double* err, int64_t K,
                    const double* lags, int kernel, double h, double* c, double* b_out,
                    int64_t* count_out, int nthreads, int brute, double dt) {
    int st = check_series(n, t, x, err);
    if (st) return st;
    st = check_lags(K, lags, h);
    if (st) return st;
    if (kernel != ORC_GAUSSIAN && kernel != ORC_RECTANGLE) return ORC_E_INVALID_ARG;
    if (dt != 0.0 && (!(dt > 0.0) || !isfinite(dt))) return ORC_E_INVALID_ARG;

    double* v = malloc(sizeof(double) * n);
    double* w = malloc(sizeof(double) * n);
    double* ev = malloc(sizeof(double) * (K + 1));
    double* C = malloc(sizeof(double) * (K + 1));
    double* B = malloc(sizeof(double) * (K + 1));
    double* bb = malloc(sizeof(double) * (K + 1));
    int64_t* cnt = malloc(sizeof(int64_t) * (K + 1));
    int64_t* m = dt > 0.0 ? malloc(sizeof(int64_t) * n) : NULL;
    if (!v || !w || !ev || !C || !B || !bb || !cnt || (dt > 0.0 && !m)) {
        st = ORC_E_NOMEM;
        goto done;
    }
    if (m) {
        st = lattice_indices(n, t, t[0], dt, m);
        if (st) goto done;
    }
    st = oracle_standardize(n, x, err, v, w);
    if (st) goto done;
    /* evaluation lags (0, tau_1, ..., tau_K): lag 0 is prepended */
    ev[0] = 0.0;
    for (int64_t k = 0; k < K; ++k) ev[k + 1] = lags[k];
    window_sums(kernel, +1, n, t, v, w, n, t, v, w, m, m, dt, K + 1, ev, h, C, B, bb, cnt,
                nthreads, brute);
    double r0 = C[0] / floor_b(B[0]);
    if (!(r0 > ORC_MIN_SCALE) || !isfinite(r0)) {
        for (int64_t k = 0; k < K; ++k) {
            c[k] = NAN;
            if (b_out) b_out[k] = floor_b(bb[k + 1]);
            if (count_out) count_out[k] = cnt[k + 1];
        }
        st = ORC_E_DEGENERATE;
        goto done;
    }
    for (int64_t k = 0; k < K; ++k) {
        double r = C[k + 1] / floor_b(B[k + 1]);
        c[k] = r / r0;
        if (b_out) b_out[k] = floor_b(bb[k + 1]);
        if (count_out) count_out[k] = cnt[k + 1];
    }
done:
    free(v);
    free(w);
    free(ev);
    free(C);
    free(B);
    free(bb);
    free(cnt);
    free(m);
    return st;
}

int oracle_acf(int64_t n, const double* t, const double* x, const double* err, int64_t K,
               const double* lags, int kernel, double h, double* c, double* b_out,
               int64_t* count_out, int nthreads, int brute) {
    return acf_impl(n, t, x, err, K, lags, kernel, h, c, b_out, count_out, nthreads, brute, 0.0);
}

int oracle_acf_regular(int64_t n, const double* t, const double* x, const double* err,
                       double dt, int64_t K, const double* lags, int kernel, double h, double* c,
                       double* b_out, int64_t* count_out, int nthreads) {
    if (!(dt > 0.0)) return ORC_E_INVALID_ARG;
    return acf_impl(n, t, x, err, K, lags, kernel, h, c, b_out, count_out, nthreads, 0, dt);
}

/* dt > 0: lattice reading with t_ref = min(t[0], s[0]) */
static int ccf_impl(int64_t nx, const double* t, const double* x, const double* ex, int64_t ny,
                    const double* s, const double* y, const double* ey, int64_t K,
                    const double* lags, int kernel, double h, double* c, double* b_out,
                    int64_t* count_out, int nthreads, int brute, double dt) {
    int st = check_series(nx, t, x, ex);
    if (st) return st;
    st = check_series(ny, s, y, ey);
    if (st) return st;
    st = check_lags(K, lags, h);
    if (st) return st;
    if (kernel != ORC_GAUSSIAN && kernel != ORC_RECTANGLE) return ORC_E_INVALID_ARG;
    if (dt != 0.0 && (!(dt > 0.0) || !isfinite(dt))) return ORC_E_INVALID_ARG;

    double *vx = malloc(sizeof(double) * nx), *wx = malloc(sizeof(double) * nx);
    double *vy = malloc(sizeof(double) * ny), *wy = malloc(sizeof(double) * ny);
    double* C = malloc(sizeof(double) * (K + 1));
    double* B = malloc(sizeof(double) * (K + 1));
    double* bb = malloc(sizeof(double) * (K + 1));
    int64_t* cnt = malloc(sizeof(int64_t) * (K + 1));
    int64_t* mx = dt > 0.0 ? malloc(sizeof(int64_t) * nx) : NULL;
    int64_t* my = dt > 0.0 ? malloc(sizeof(int64_t) * ny) : NULL;
    if (!vx || !wx || !vy || !wy || !C || !B || !bb || !cnt || (dt > 0.0 && (!mx || !my))) {
        st = ORC_E_NOMEM;
        goto done;
    }
    if (dt > 0.0) {
        const double t_ref = t[0] < s[0] ? t[0] : s[0];
        st = lattice_indices(nx, t, t_ref, dt, mx);
        if (st) goto done;
        st = lattice_indices(ny, s, t_ref, dt, my);
        if (st) goto done;
    }
    st = oracle_standardize(nx, x, ex, vx, wx);
    if (st) goto done;
    st = oracle_standardize(ny, y, ey, vy, wy);
    if (st) goto done;

    /* cross sums: outer array = series 2 (s), window array = series 1 (t), eps = -1 */
    if (K > 0)
        window_sums(kernel, -1, ny, s, vy, wy, nx, t, vx, wx, my, mx, dt, K, lags, h, C, B, bb,
                    cnt, nthreads, brute);
    /* lag-0 scales of each series on itself, eps = +1 */
    double zero = 0.0, Cs, Bs, bs;
    int64_t ns;
    window_sums(kernel, +1, nx, t, vx, wx, nx, t, vx, wx, mx, mx, dt, 1, &zero, h, &Cs, &Bs, &bs,
                &ns, nthreads, brute);
    double scale_x = Cs / floor_b(Bs);
    window_sums(kernel, +1, ny, s, vy, wy, ny, s, vy, wy, my, my, dt, 1, &zero, h, &Cs, &Bs, &bs,
                &ns, nthreads, brute);
    double scale_y = Cs / floor_b(Bs);
    double prod = scale_x * scale_y;
    int degenerate = !(fabs(scale_x) > ORC_MIN_SCALE) || !(fabs(scale_y) > ORC_MIN_SCALE) ||
                     !(prod > 0.0) || !isfinite(prod);
    double scale = degenerate ? NAN : sqrt(prod);
    for (int64_t k = 0; k < K; ++k) {
        double r = C[k] / floor_b(B[k]);
        c[k] = degenerate ? NAN : r / scale;
        if (b_out) b_out[k] = floor_b(bb[k]);
        if (count_out) count_out[k] = cnt[k];
    }
    if (degenerate) st = ORC_E_DEGENERATE;
done:
    free(vx);
    free(wx);
    free(vy);
    free(wy);
    free(C);
    free(B);
    free(bb);
    free(cnt);
    free(mx);
    free(my);
    return st;
}

int oracle_ccf(int64_t nx, const double* t, const double* x, const double* ex, int64_t ny,
               const double* s, const double* y, const double* ey, int64_t K, const double* lags,
               int kernel, double h, double* c, double* b_out, int64_t* count_out, int nthreads,
               int brute) {
    return ccf_impl(nx, t, x, ex, ny, s, y, ey, K, lags, kernel, h, c, b_out, count_out,
                    nthreads, brute, 0.0);
}

int oracle_ccf_regular(int64_t nx, const double* t, const double* x, const double* ex,
                       int64_t ny, const double* s, const double* y, const double* ey, double dt,
                       int64_t K, const double* lags, int kernel, double h, double* c,
                       double* b_out, int64_t* count_out, int nthreads) {
    if (!(dt > 0.0)) return ORC_E_INVALID_ARG;
    return ccf_impl(nx, t, x, ex, ny, s, y, ey, K, lags, kernel, h, c, b_out, count_out,
                    nthreads, 0, dt);
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
