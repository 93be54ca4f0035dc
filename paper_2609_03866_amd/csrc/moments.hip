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
    const int tid = threadIdx.x;
    double sw = 0.0, swx = 0.0;
    int bad = 0, unsorted = 0;
    for (int64_t i = ch.begin + tid; i < ch.end; i += kThreads) {
        double ti = a.t[i], xi = a.x[i];
        double wi = 1.0;
        if (a.err) {
            double e = a.err[i];
            if (!(e > 0.0) || !isfinite(e)) bad = 1;
            wi = 1.0 / (e * e);
        }
        if (!isfinite(ti) || !isfinite(xi)) bad = 1;
        if (i > sd.off && !(ti >= a.t[i - 1])) unsorted = 1;
        sw += wi;
        swx += wi * xi;
    }
    double Sw = block_sum(sw, sh);
    double Swx = block_sum(swx, sh);
    double mean = Swx / Sw;
    double m2 = 0.0;
    for (int64_t i = ch.begin + tid; i < ch.end; i += kThreads) {
        double wi = 1.0;
        if (a.err) {
            double e = a.err[i];
            wi = 1.0 / (e * e);
        }
        double d = a.x[i] - mean;
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

__global__ void k_series_finalize(MomentsArgs a) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.nseries) return;
    const SeriesDesc sd = a.series[s];
    SeriesStat st;
    st.status = NCF_OK;
    st.pad = 0;
    if (sd.n < 2) {
        st.status = NCF_E_INVALID_ARG;
        st.mean = st.sd = st.sw = st.tmin = st.tmax = 0.0;
        a.stats[s] = st;
        return;
    }
    double sw = 0.0, mean = 0.0, m2 = 0.0;
    int bad = 0, unsorted = 0;
    for (int c = 0; c < sd.nchunk; ++c) {
        const double* p = a.chunk_part + 4 * (int64_t)(sd.chunk0 + c);
        double swb = p[0], mb = p[1], m2b = p[2];
        int fl = (int)p[3];
        bad |= fl & 1;
        unsorted |= (fl >> 1) & 1;
        if (c == 0) {
            sw = swb;
            mean = mb;
            m2 = m2b;
        } else {
            double tot = sw + swb;
            double dlt = mb - mean;
            mean = mean + dlt * (swb / tot);
            m2 = m2 + m2b + dlt * dlt * (sw * swb / tot);
            sw = tot;
        }
    }
    double sdv = sqrt(m2 / sw);
    st.mean = mean;
    st.sd = sdv;
    st.sw = sw;
    st.tmin = a.t[sd.off];
    st.tmax = a.t[sd.off + sd.n - 1];
    if (bad)
        st.status = NCF_E_INVALID_ARG;
    else if (unsorted)
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
    const int tid = threadIdx.x;
    const bool ok = st.status == NCF_OK;
    const double mean = st.mean;
    const double inv_sd = ok ? 1.0 / st.sd : 0.0;
    const bool do_prefix = a.pv != nullptr;
    double carry_v = 0.0, carry_w = 0.0;
    // prefix index of sample i within the series' prefix array: i - off + 1
    for (int64_t base = ch.begin; base < ch.end; base += kThreads) {
        int64_t i = base + tid;
        double v = 0.0, w = 0.0;
        if (i < ch.end) {
            w = 1.0;
            if (a.err) {
                double e = a.err[i];
                w = 1.0 / (e * e);
            }
            v = ok ? w * ((a.x[i] - mean) * inv_sd) : 0.0;
            if (a.v32) a.v32[i] = (float)v;
            if (a.v64) a.v64[i] = v;
            if (a.w64) a.w64[i] = w;
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
                int64_t pidx = sd.pre_off + (i - sd.off) + 1;
                a.pv[pidx] = carry_v + shv[tid];
                if (a.pw) a.pw[pidx] = carry_w + shw[tid];
            }
            carry_v += shv[kThreads - 1];
            carry_w += shw[kThreads - 1];
            __syncthreads();
        }
    }
    if (do_prefix && tid == 0) {
        a.chunk_tot[2 * (int64_t)blockIdx.x] = carry_v;
        a.chunk_tot[2 * (int64_t)blockIdx.x + 1] = carry_w;
        if (ch.begin == sd.off) {
            a.pv[sd.pre_off] = 0.0;
            if (a.pw) a.pw[sd.pre_off] = 0.0;
        }
    }
}

// Exclusive scan of chunk totals per series (in place: chunk_tot becomes the
// offset to add to each chunk).
__global__ void k_chunk_offsets(MomentsArgs a) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.nseries) return;
    const SeriesDesc sd = a.series[s];
    double cv = 0.0, cw = 0.0;
    for (int c = 0; c < sd.nchunk; ++c) {
        double* p = a.chunk_tot + 2 * (int64_t)(sd.chunk0 + c);
        double tv = p[0], tw = p[1];
        p[0] = cv;
        p[1] = cw;
        cv += tv;
        cw += tw;
    }
}

__global__ void __launch_bounds__(kThreads)
k_prefix_add(MomentsArgs a) {
    const Chunk ch = a.chunks[blockIdx.x];
    const SeriesDesc sd = a.series[ch.series];
    const double ov = a.chunk_tot[2 * (int64_t)blockIdx.x];
    const double ow = a.chunk_tot[2 * (int64_t)blockIdx.x + 1];
    if (ch.begin == sd.off) return;  // first chunk: offset 0
    for (int64_t i = ch.begin + threadIdx.x; i < ch.end; i += kThreads) {
        int64_t pidx = sd.pre_off + (i - sd.off) + 1;
        a.pv[pidx] += ov;
        if (a.pw) a.pw[pidx] += ow;
    }
}

}  // namespace

int launch_moments(const MomentsArgs& a, hipStream_t st) {
    if (a.nchunks > 0) {
        ProfScope p(st, "moments", 0.0, "bytes");
        hipLaunchKernelGGL(k_chunk_moments, dim3(a.nchunks), dim3(kThreads), 0, st, a);
        NCF_CHECK_LAUNCH();
    }
    {
        ProfScope p(st, "series_finalize", 0.0, "bytes");
        hipLaunchKernelGGL(k_series_finalize, dim3((a.nseries + 127) / 128), dim3(128), 0, st, a);
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
    if (a.pv) {
        hipLaunchKernelGGL(k_chunk_offsets, dim3((a.nseries + 127) / 128), dim3(128), 0, st, a);
        NCF_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_prefix_add, dim3(a.nchunks), dim3(kThreads), 0, st, a);
        NCF_CHECK_LAUNCH();
    }
    return NCF_OK;
}

}  // namespace ncf
