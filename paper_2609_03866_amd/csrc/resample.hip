// resample.hip -- replicate series for Monte-Carlo and bootstrap error bars
// of the estimator (the per-lag uncertainty the paper leaves to external
// bootstrap or Monte-Carlo resampling, Sec. "Discussion" and "Summary and
// Conclusion"; pyZDCF-style flux randomization and sample resampling).
//
// Replicate r perturbs every value by its sigma times a given normal deviate
// (flux randomization) and repeats sample i mult_r[i] times (bootstrap
// resampling with replacement). A sample repeated k times enters every pair
// sum k_i k_j times, and the weighted mean and sd with weights k equal those
// of the repeated series, so the replicate is the weighted estimator with
// sample weights k (times 1/err^2 when errors weight the estimator). All R
// replicates then run as one batch that shares the times.
#include "internal.h"

namespace ncf {

namespace {

constexpr int kThreads = 256;

__global__ void __launch_bounds__(kThreads)
k_resample_prep(int64_t n, int64_t total, const double* __restrict__ x,
                const double* __restrict__ sigma, const double* __restrict__ z,
                const double* __restrict__ err, const int32_t* __restrict__ mult,
                double* __restrict__ xr, double* __restrict__ wr) {
    const int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (g >= total) return;
    const int64_t i = g % n;
    double v = gbl(x)[i];
    if (z) v += gbl(sigma)[i] * gbl(z)[g];
    gbl(xr)[g] = v;
    if (wr) {
        double w = mult ? (double)gbl(mult)[g] : 1.0;
        if (err) {
            const double e = gbl(err)[i];
            w *= 1.0 / (e * e);
        }
        gbl(wr)[g] = w;
    }
}

// One thread per lag: the replicates in order, mean first, then the sum of
// squared deviations (two passes, fixed order).
__global__ void __launch_bounds__(kThreads)
k_resample_stats(const double* __restrict__ c_rep, int64_t R, int64_t K,
                 double* __restrict__ c_mean, double* __restrict__ c_sd) {
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (k >= K) return;
    const gptr<const double> c = gbl(c_rep);
    double s = 0.0;
    int64_t m = 0;
    for (int64_t r = 0; r < R; ++r) {
        const double v = c[r * K + k];
        if (v == v) {
            s += v;
            ++m;
        }
    }
    const double mean = m > 0 ? s / (double)m : NAN;
    double ss = 0.0;
    for (int64_t r = 0; r < R; ++r) {
        const double v = c[r * K + k];
        if (v == v) ss += (v - mean) * (v - mean);
    }
    gbl(c_mean)[k] = mean;
    gbl(c_sd)[k] = m > 1 ? sqrt(ss / (double)(m - 1)) : NAN;
}

}  // namespace

int launch_resample_prep(int64_t n, int64_t R, const double* x, const double* sigma,
                         const double* z, const double* err, const int32_t* mult, double* xr,
                         double* wr, hipStream_t st) {
    const int64_t total = n * R;
    if (total <= 0) return NCF_OK;
    ProfScope p(st, "resample_prep", (double)total * 8.0 * (2.0 + (z ? 1 : 0) + (wr ? 1 : 0)),
                "bytes");
    hipLaunchKernelGGL(k_resample_prep, dim3((unsigned)ceil_div(total, kThreads)), dim3(kThreads),
                       0, st, n, total, x, sigma, z, err, mult, xr, wr);
    NCF_CHECK_LAUNCH();
    return NCF_OK;
}

int launch_resample_stats(const double* c_rep, int64_t R, int64_t K, double* c_mean,
                          double* c_sd, hipStream_t st) {
    if (K <= 0) return NCF_OK;
    ProfScope p(st, "resample_stats", 0.0, "bytes");
    hipLaunchKernelGGL(k_resample_stats, dim3((unsigned)ceil_div(K, kThreads)), dim3(kThreads), 0,
                       st, c_rep, R, K, c_mean, c_sd);
    NCF_CHECK_LAUNCH();
    return NCF_OK;
}

}  // namespace ncf
