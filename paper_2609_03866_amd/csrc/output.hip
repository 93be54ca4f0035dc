// output.hip -- normalization and reordering (step A8).
//
// r(tau) = C(tau) / max(B(tau), 1e-16) with the floor of the PairCount
// algorithms. ACF: c_k = r(tau_k) / r(0) (lag-0 normalization of "ACF via
// NUFFT"). CCF: c_k = r(tau_k) / sqrt(scale_x scale_y) with scale_x the lag-0
// ratio of series 1 on itself ("CCF via NUFFT" / "CCF via real-space").
// Outputs are written in the order of the request; a non-positive lag-0
// scale gives NaN and NCF_E_DEGENERATE.
#include "internal.h"

namespace ncf {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double fl(double v) { return v > kFloor ? v : kFloor; }

// Per requested lag the numerator C and pair sum B come from one of:
//  * the direct fallback sums (lags whose spectral b was small),
//  * the spectral route (N, and b when the unit-weight channel ran),
//  * the window sums (rectangle, direct method; and with the spectral
//    numerator but window b, the window's direct numerator at lags whose
//    b < beta * b_ref).
__global__ void __launch_bounds__(kThreads)
k_normalize(const NormTask* __restrict__ tasks, const IoBlock* __restrict__ io) {
    __shared__ double red[4][kThreads];
    __shared__ double sh_scale, sh_bref;
    const NormTask& T = tasks[blockIdx.x];
    const int tid = threadIdx.x;
    double* const out_c = io->c + T.out_off;
    double* const out_b = io->b + T.out_off;
    int64_t* const out_n = io->count ? io->count + T.out_off : nullptr;
    int32_t* const out_st = io->status + T.index;
    // failed host checks, or failed value checks of this call's moments
    int32_t fail = T.skip ? T.skip_status : NCF_OK;
    if (fail == NCF_OK && T.st0 && T.st0->status != NCF_OK) fail = T.st0->status;
    if (fail == NCF_OK && T.st1 && T.st1->status != NCF_OK) fail = T.st1->status;
    if (fail != NCF_OK) {
        for (int k = tid; k < T.K; k += kThreads) {
            out_c[k] = NAN;
            out_b[k] = 0.0;
            if (out_n) out_n[k] = 0;
        }
        if (tid == 0) {
            *out_st = fail;
            if (T.rmin) *T.rmin = INFINITY;
        }
        return;
    }
    const int bq = T.weighted ? 1 : 2;  // which window sum is the denominator B
    // lag-0 scale: from the direct window sums where the call has them (the
    // direct path, and the Gaussian spectral numerator with window pair
    // counts: there the lag-0 sums of a short series under a wide kernel can
    // cancel, and the transforms' rounding error would not), else from the
    // spectral lag-0 values (spectral pair counts; the rectangle kernel on
    // the spectral route, whose window pass sums no numerator)
    const bool spec_scale = T.spectral && (T.spec_b || T.is_rect);
    // spectral lag-0 sums (CCF): S_xx, S_yy and, with spectral b, B_xx, B_yy
    if (T.ccf && spec_scale) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int64_t i = tid; i < T.nscale_part; i += kThreads)
            for (int q = 0; q < 4; ++q) acc[q] += T.scale_part[4 * i + q];
        for (int q = 0; q < 4; ++q) red[q][tid] = acc[q];
        __syncthreads();
        for (int off = kThreads / 2; off > 0; off >>= 1) {
            if (tid < off)
                for (int q = 0; q < 4; ++q) red[q][tid] += red[q][tid + off];
            __syncthreads();
        }
    }
    // Gaussian spectral numerator with window pair counts: the direct
    // numerator where b is small
    const bool sel_window = T.spectral && !T.spec_b && !T.is_rect;
    if (tid == 0) {
        double scale, rmin;
        if (T.ccf) {
            double cx, cy, bx, by;
            if (T.spectral && T.spec_b) {
                cx = red[0][0];
                cy = red[1][0];
                bx = red[2][0];
                by = red[3][0];
            } else if (spec_scale) {
                cx = red[0][0];
                cy = red[1][0];
                bx = T.self_x[bq];
                by = T.self_y[bq];
            } else {
                cx = T.self_x[0];
                cy = T.self_y[0];
                bx = T.self_x[bq];
                by = T.self_y[bq];
            }
            const double sx = cx / fl(bx), sy = cy / fl(by), prod = sx * sy;
            scale = (fabs(sx) > kMinScale && fabs(sy) > kMinScale && prod > 0.0 &&
                     isfinite(prod))
                        ? sqrt(prod)
                        : NAN;
            rmin = fmin(sx, sy);
        } else {
            double c0, b0;
            if (T.spectral && T.spec_b) {
                c0 = T.numer[T.K];
                b0 = T.bspec[T.K];
            } else {
                c0 = spec_scale ? T.numer[T.K] : T.wsums[4 * T.row0 + 0];
                b0 = T.wsums[4 * T.row0 + bq];
            }
            const double r0 = c0 / fl(b0);
            scale = (r0 > kMinScale && isfinite(r0)) ? r0 : NAN;
            rmin = r0;
        }
        // a scale at or below kMinScale in mixed precision is also evaluated
        // again in FP64 (rmin is kept): FP32 rounding may have decided it
        int32_t st = (scale == scale) ? NCF_OK : NCF_E_DEGENERATE;
        if (rmin != rmin) rmin = INFINITY;
        if (st == NCF_OK && T.guard && rmin < kPromoteScale) {
            // a plan replays fixed launches and cannot evaluate this problem
            // again in FP64: its mixed-precision result is not reported
            scale = NAN;
            st = NCF_E_UNSUPPORTED;
        }
        if (T.rmin) *T.rmin = rmin;
        sh_scale = scale;
        *out_st = st;
        if (sel_window) {
            // reference pair count of the window-b spectral path, a bound of
            // the pair sum over every lag: ACF b(0); CCF sqrt(B_xx(0) B_yy(0))
            // from the two series' lag-0 window sums (Cauchy-Schwarz: the
            // Gaussian lag kernel is a self-convolution); it sets the scale of
            // the spectral numerator's rounding error, which the division by
            // a lag-0 scale below 1 amplifies: a lag takes the direct
            // numerator when b min(1, scale) < beta b_ref
            const double bref =
                T.ccf ? sqrt(T.self_x[bq] * T.self_y[bq]) : T.wsums[4 * T.row0 + bq];
            sh_bref = bref / (scale > 0.0 ? fmin(1.0, scale) : 1.0);
        }
    }
    __syncthreads();
    const double scale = sh_scale;
    for (int k = tid; k < T.K; k += kThreads) {
        const int fb = T.fb_row ? T.fb_row[k] : -1;
        double num, den, bout;
        int64_t cnt = 0;
        if (fb >= 0) {
            const double* w = T.fb_sums + 4 * (int64_t)fb;
            // empty: no pair, or (weights) a weighted pair sum of exactly 0,
            // a window of samples of weight 0 only (dropped bootstrap samples)
            const bool empty = __double_as_longlong(w[3]) == 0 || (T.weighted && w[bq] == 0.0);
            num = empty ? 0.0 : w[0];
            den = w[bq];
            bout = w[2];
        } else if (T.spectral && T.spec_b) {
            num = T.numer[k];
            den = T.bspec[k];
            bout = T.bunw ? T.bunw[k] : T.bspec[k];
        } else {
            const double* w = T.wsums + 4 * (int64_t)T.perm[k];
            cnt = __double_as_longlong(w[3]);
            // an empty window has numerator exactly 0: no pair, or (weights)
            // no pair of two nonzero weights, a window of samples of weight 0
            // only (dropped bootstrap samples). Gaussian: the weighted pair
            // sum is then exactly 0 (a direct sum of zero terms); rectangle:
            // the window pass counts those pairs exactly in w[2] (its weight
            // prefix differences can leave rounding residue). A window with
            // few pairs takes the direct numerator (the spectral value there
            // is rounding noise that a small denominator would amplify)
            const bool empty =
                cnt == 0 || (T.weighted && (T.is_rect ? w[2] == 0.0 : w[bq] == 0.0));
            const bool direct = !T.spectral || (sel_window && w[bq] < T.beta * sh_bref);
            num = empty ? 0.0 : (direct ? w[0] : T.numer[k]);
            den = w[bq];
            bout = T.is_rect ? (double)cnt : w[2];
        }
        out_c[k] = (num / fl(den)) / scale;
        out_b[k] = fl(bout);
        if (out_n) out_n[k] = T.is_rect ? cnt : 0;
    }
}

__global__ void k_set_io(IoBlock* __restrict__ dst, IoBlock v) {
    if (threadIdx.x == 0) *dst = v;
}

}  // namespace

int launch_normalize(const NormTask* d_tasks, int ntasks, const IoBlock* io, hipStream_t st) {
    if (ntasks <= 0) return NCF_OK;
    ProfScope p(st, "normalize", 0.0, "bytes");
    hipLaunchKernelGGL(k_normalize, dim3(ntasks), dim3(kThreads), 0, st, d_tasks, io);
    NCF_CHECK_LAUNCH();
    return NCF_OK;
}

int launch_set_io(IoBlock* dst, const IoBlock& v, hipStream_t st) {
    hipLaunchKernelGGL(k_set_io, dim3(1), dim3(64), 0, st, dst, v);
    NCF_CHECK_LAUNCH();
    return NCF_OK;
}

}  // namespace ncf
