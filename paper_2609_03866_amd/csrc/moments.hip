// moments.hip -- validation, FP64 moments and standardization (step A1).
//
// The estimator standardizes each series before any pair sum (first step
// of the paper's ACF/CCF algorithms); only the mean matters for c, the sd
// cancels, but it is computed for the degenerate-series check. Each series
// is split into chunks; a chunk produces (sum of weights, mean, M2) by a
// two-pass FP64 reduction in a fixed tree order, and the per-series result
// combines the chunks in order (pairwise update of mean and M2), so the
// result is deterministic and does not suffer from the cancellation of a
// one-pass sum of squares. The same chunks then write the standardized
// values and, for the rectangle kernel, the FP64 prefix sums used by the
// window scan (Algorithm "CorrSum, rectangle").
#include "internal.h"

namespace ncf {

namespace {

constexpr int kThreads = 256;

// Fixed-order block reduction of one double per thread.
__device__ double block_sum(double v, double* sh) {
    // wave-level tree via LDS (fixed order, independent of timing)
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int off = kThreads / 2; off > 0; off >>= 1) {
        if (tid < off) sh[tid] += sh[tid + off];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(kThreads)
k_chunk_moments(MomentsArgs a) {
    __shared__ double sh[kThreads];
    const Chunk ch = a.chunks[blockIdx.x];
    const SeriesDesc sd = a.series[ch.series];
    const double* X = a.io->x[sd.set] + sd.xoff;
    const int tid = threadIdx.x;
    double sw = 0.0, swx = 0.0;
    int bad = 0, unsorted = 0;
    for (int64_t i = ch.begin + tid; i < ch.end; i += kThreads) {
        double ti = sd.t[i], xi = X[i];
        double wi = 1.0;
        if (sd.err) {
            double e = sd.err[i];
            if (!(e > 0.0) || !isfinite(e)) bad = 1;
            wi = 1.0 / (e * e);
        }
        if (!isfinite(ti) || !isfinite(xi)) bad = 1;
        if (i > 0 && !(ti >= sd.t[i - 1])) unsorted = 1;
        sw += wi;
        swx += wi * xi;
    }
    double Sw = block_sum(sw, sh);
    double Swx = block_sum(swx, sh);
    double mean = Swx / Sw;
    double m2 = 0.0;
    for (int64_t i = ch.begin + tid; i < ch.end; i += kThreads) {
        double wi = 1.0;
        if (sd.err) {
            double e = sd.err[i];
            wi = 1.0 / (e * e);
        }
        double d = X[i] - mean;
        m2 += wi * d * d;
    }
    double M2 = block_sum(m2, sh);
    double nbad = block_sum((double)bad, sh);
    double nuns = block_sum((double)unsorted, sh);
    if (tid == 0) {
        double* p = a.chunk_part + 4 * (int64_t)blockIdx.x;
        p[0] = Sw;
        p[1] = mean;
        p[2] = M2;
        p[3] = (nbad > 0.0 ? 1.0 : 0.0) + (nuns > 0.0 ? 2.0 : 0.0);
    }
}

// Combine (sum of weights, mean, M2) of two disjoint parts (pairwise update).
__device__ __forceinline__ void merge_moments(double& sw, double& mean, double& m2, double swb,
                                              double mb, double m2b) {
    if (swb == 0.0) return;
    if (sw == 0.0) {
        sw = swb;
        mean = mb;
        m2 = m2b;
        return;
    }
    const double tot = sw + swb;
    const double dlt = mb - mean;
    mean = mean + dlt * (swb / tot);
    m2 = m2 + m2b + dlt * dlt * (sw * swb / tot);
    sw = tot;
}

// One workgroup per series: each thread merges a contiguous run of chunks in
// order, then the threads' results are merged pairwise in a fixed tree.
__global__ void __launch_bounds__(kThreads)
k_series_finalize(MomentsArgs a) {
    __shared__ double sh[3][kThreads];
    __shared__ int shf[kThreads];
    const int s = blockIdx.x;
    const int tid = threadIdx.x;
    const SeriesDesc sd = a.series[s];
    double sw = 0.0, mean = 0.0, m2 = 0.0;
    int fl = 0;
    const int per = (sd.nchunk + kThreads - 1) / kThreads;
    const int c0 = tid * per, c1 = min(sd.nchunk, c0 + per);
    for (int c = c0; c < c1; ++c) {
        const double* p = a.chunk_part + 4 * (int64_t)(sd.chunk0 + c);
        merge_moments(sw, mean, m2, p[0], p[1], p[2]);
        fl |= (int)p[3];
    }
    sh[0][tid] = sw;
    sh[1][tid] = mean;
    sh[2][tid] = m2;
    shf[tid] = fl;
    __syncthreads();
    for (int off = 1; off < kThreads; off <<= 1) {
        if ((tid & (2 * off - 1)) == 0 && tid + off < kThreads) {
            double w0 = sh[0][tid], m0 = sh[1][tid], q0 = sh[2][tid];
            merge_moments(w0, m0, q0, sh[0][tid + off], sh[1][tid + off], sh[2][tid + off]);
            sh[0][tid] = w0;
            sh[1][tid] = m0;
            sh[2][tid] = q0;
            shf[tid] |= shf[tid + off];
        }
        __syncthreads();
    }
    if (tid != 0) return;
    SeriesStat st;
    st.status = NCF_OK;
    st.pad = 0;
    const int flags = shf[0];
    const double swt = sh[0][0];
    const double sdv = sqrt(sh[2][0] / swt);
    st.mean = sh[1][0];
    st.sd = sdv;
    st.sw = swt;
    st.tmin = sd.t[0];
    st.tmax = sd.t[sd.n - 1];
    if (sd.n < 2 || (flags & 1))
        st.status = NCF_E_INVALID_ARG;
    else if (flags & 2)
        st.status = NCF_E_UNSORTED;
    else if (!(sdv > 0.0) || !isfinite(sdv))
        st.status = NCF_E_DEGENERATE;
    a.stats[s] = st;
}

// Standardize one chunk and write the chunk-local inclusive prefix sums.
__global__ void __launch_bounds__(kThreads)
k_standardize(MomentsArgs a) {
    __shared__ double shv[kThreads];
    __shared__ double shw[kThreads];
    const Chunk ch = a.chunks[blockIdx.x];
    const SeriesDesc sd = a.series[ch.series];
    const SeriesStat st = a.stats[ch.series];
    const double* X = a.io->x[sd.set] + sd.xoff;
    const int tid = threadIdx.x;
    const bool ok = st.status == NCF_OK;
    const double mean = st.mean;
    const double inv_sd = ok ? 1.0 / st.sd : 0.0;
    const bool do_prefix = sd.pv != nullptr;
    double carry_v = 0.0, carry_w = 0.0;
    // prefix index of sample i within the series' prefix array: i + 1
    for (int64_t base = ch.begin; base < ch.end; base += kThreads) {
        int64_t i = base + tid;
        double v = 0.0, w = 0.0;
        if (i < ch.end) {
            w = 1.0;
            if (sd.err) {
                double e = sd.err[i];
                w = 1.0 / (e * e);
            }
            v = ok ? w * ((X[i] - mean) * inv_sd) : 0.0;
            if (sd.v32) sd.v32[i] = (float)v;
            if (sd.v64) sd.v64[i] = v;
            if (sd.w64) sd.w64[i] = w;
        }
        if (do_prefix) {
            // inclusive Hillis-Steele scan over the block (fixed order)
            shv[tid] = v;
            shw[tid] = w;
            __syncthreads();
            for (int off = 1; off < kThreads; off <<= 1) {
                double av = tid >= off ? shv[tid - off] : 0.0;
                double aw = tid >= off ? shw[tid - off] : 0.0;
                __syncthreads();
                shv[tid] += av;
                shw[tid] += aw;
                __syncthreads();
            }
            if (i < ch.end) {
                sd.pv[i + 1] = carry_v + shv[tid];
                if (sd.pw) sd.pw[i + 1] = carry_w + shw[tid];
            }
            carry_v += shv[kThreads - 1];
            carry_w += shw[kThreads - 1];
            __syncthreads();
        }
    }
    if (do_prefix && tid == 0) {
        a.chunk_tot[2 * (int64_t)blockIdx.x] = carry_v;
        a.chunk_tot[2 * (int64_t)blockIdx.x + 1] = carry_w;
        if (ch.begin == 0) {
            sd.pv[0] = 0.0;
            if (sd.pw) sd.pw[0] = 0.0;
        }
    }
}

// Exclusive scan of chunk totals per series (in place: chunk_tot becomes the
// offset to add to each chunk). One workgroup per series: per-thread runs,
// then a fixed-order scan of the run totals.
__global__ void __launch_bounds__(kThreads)
k_chunk_offsets(MomentsArgs a) {
    __shared__ double shv[kThreads];
    __shared__ double shw[kThreads];
    const int s = blockIdx.x;
    const int tid = threadIdx.x;
    const SeriesDesc sd = a.series[s];
    if (!sd.pv) return;
    const int per = (sd.nchunk + kThreads - 1) / kThreads;
    const int c0 = tid * per, c1 = min(sd.nchunk, c0 + per);
    double tv = 0.0, tw = 0.0;
    for (int c = c0; c < c1; ++c) {
        const double* p = a.chunk_tot + 2 * (int64_t)(sd.chunk0 + c);
        tv += p[0];
        tw += p[1];
    }
    shv[tid] = tv;
    shw[tid] = tw;
    __syncthreads();
    if (tid == 0) {  // exclusive scan of 256 run totals, in order
        double cv = 0.0, cw = 0.0;
        for (int i = 0; i < kThreads; ++i) {
            const double v = shv[i], w = shw[i];
            shv[i] = cv;
            shw[i] = cw;
            cv += v;
            cw += w;
        }
    }
    __syncthreads();
    double cv = shv[tid], cw = shw[tid];
    for (int c = c0; c < c1; ++c) {
        double* p = a.chunk_tot + 2 * (int64_t)(sd.chunk0 + c);
        const double v = p[0], w = p[1];
        p[0] = cv;
        p[1] = cw;
        cv += v;
        cw += w;
    }
}

__global__ void __launch_bounds__(kThreads)
k_prefix_add(MomentsArgs a) {
    const Chunk ch = a.chunks[blockIdx.x];
    const SeriesDesc sd = a.series[ch.series];
    if (!sd.pv) return;
    const double ov = a.chunk_tot[2 * (int64_t)blockIdx.x];
    const double ow = a.chunk_tot[2 * (int64_t)blockIdx.x + 1];
    if (ch.begin == 0) return;  // first chunk: offset 0
    for (int64_t i = ch.begin + threadIdx.x; i < ch.end; i += kThreads) {
        sd.pv[i + 1] += ov;
        if (sd.pw) sd.pw[i + 1] += ow;
    }
}

__global__ void __launch_bounds__(kThreads)
k_fill_alternating(double* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) p[i] = (i & 1) ? -1.0 : 1.0;
}

}  // namespace

int launch_fill_alternating(double* p, int64_t n, hipStream_t st) {
    if (n <= 0) return NCF_OK;
    hipLaunchKernelGGL(k_fill_alternating, dim3((unsigned)ceil_div(n, kThreads)), dim3(kThreads),
                       0, st, p, n);
    NCF_CHECK_LAUNCH();
    return NCF_OK;
}

int launch_moments(const MomentsArgs& a, hipStream_t st) {
    if (a.nchunks > 0) {
        ProfScope p(st, "moments", 0.0, "bytes");
        hipLaunchKernelGGL(k_chunk_moments, dim3(a.nchunks), dim3(kThreads), 0, st, a);
        NCF_CHECK_LAUNCH();
    }
    {
        ProfScope p(st, "series_finalize", 0.0, "bytes");
        hipLaunchKernelGGL(k_series_finalize, dim3(a.nseries), dim3(kThreads), 0, st, a);
        NCF_CHECK_LAUNCH();
    }
    return NCF_OK;
}

int launch_standardize(const MomentsArgs& a, hipStream_t st) {
    if (a.nchunks == 0) return NCF_OK;
    {
        ProfScope p(st, "standardize", 0.0, "bytes");
        hipLaunchKernelGGL(k_standardize, dim3(a.nchunks), dim3(kThreads), 0, st, a);
        NCF_CHECK_LAUNCH();
    }
    if (a.prefix) {
        hipLaunchKernelGGL(k_chunk_offsets, dim3(a.nseries), dim3(kThreads), 0, st, a);
        NCF_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_prefix_add, dim3(a.nchunks), dim3(kThreads), 0, st, a);
        NCF_CHECK_LAUNCH();
    }
    return NCF_OK;
}

}  // namespace ncf
