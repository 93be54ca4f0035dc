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

__global__ void __launch_bounds__(kThreads)
k_normalize(const NormTask* __restrict__ tasks) {
    __shared__ double red[2][kThreads];
    __shared__ double sh_scale;
    const NormTask& T = tasks[blockIdx.x];
    const int tid = threadIdx.x;
    if (T.skip) {  // the problem failed validation
        for (int k = tid; k < T.K; k += kThreads) {
            T.c[k] = NAN;
            T.b[k] = 0.0;
            if (T.count) T.count[k] = 0;
        }
        return;
    }
    const int bq = T.weighted ? 1 : 2;  // which window sum is the denominator B
    // lag-0 scale
    if (T.ccf && T.spectral) {
        double sx = 0.0, sy = 0.0;
        for (int64_t i = tid; i < T.nscale_part; i += kThreads) {
            sx += T.scale_part[2 * i];
            sy += T.scale_part[2 * i + 1];
        }
        red[0][tid] = sx;
        red[1][tid] = sy;
        __syncthreads();
        for (int off = kThreads / 2; off > 0; off >>= 1) {
            if (tid < off) {
                red[0][tid] += red[0][tid + off];
                red[1][tid] += red[1][tid + off];
            }
            __syncthreads();
        }
    }
    if (tid == 0) {
        double scale;
        if (T.ccf) {
            double cx, cy;
            if (T.spectral) {
                cx = red[0][0];
                cy = red[1][0];
            } else {
                cx = T.self_x[0];
                cy = T.self_y[0];
            }
            const double sxv = cx / fl(T.self_x[bq]);
            const double syv = cy / fl(T.self_y[bq]);
            const double prod = sxv * syv;
            scale = (prod > 0.0 && isfinite(prod)) ? sqrt(prod) : NAN;
        } else {
            const double c0 = T.spectral ? T.numer[T.K] : T.wsums[4 * T.row0 + 0];
            const double r0 = c0 / fl(T.wsums[4 * T.row0 + bq]);
            scale = (r0 > 0.0 && isfinite(r0)) ? r0 : NAN;
        }
        sh_scale = scale;
        if (!(scale == scale)) *T.status = NCF_E_DEGENERATE;
    }
    __syncthreads();
    const double scale = sh_scale;
    for (int k = tid; k < T.K; k += kThreads) {
        const int row = T.perm[k];
        const double* w = T.wsums + 4 * (int64_t)row;
        // an empty window has numerator exactly 0 (the spectral value there is
        // rounding noise that the 1e-16 floor would amplify)
        const bool empty = __double_as_longlong(w[3]) == 0;
        const double num = empty ? 0.0 : (T.spectral ? T.numer[k] : w[0]);
        const double r = num / fl(w[bq]);
        T.c[k] = r / scale;
        T.b[k] = fl(w[2]);
        if (T.count) T.count[k] = T.is_rect ? (int64_t)__double_as_longlong(w[3]) : 0;
    }
}

}  // namespace

int launch_normalize(const NormTask* d_tasks, int ntasks, int64_t total_k, const int64_t* d_k0,
                     hipStream_t st) {
    (void)total_k;
    (void)d_k0;
    if (ntasks <= 0) return NCF_OK;
    ProfScope p(st, "normalize", 0.0, "bytes");
    hipLaunchKernelGGL(k_normalize, dim3(ntasks), dim3(kThreads), 0, st, d_tasks);
    NCF_CHECK_LAUNCH();
    return NCF_OK;
}

}  // namespace ncf
