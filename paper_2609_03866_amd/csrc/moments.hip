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
// values and, for the rectangle kernel, the chunk-local FP64 prefix sums
// used by the window scan (Algorithm "CorrSum, rectangle"), which adds the
// chunk offsets (the exclusive sums of the preceding chunks) as it reads
// them.
#include "internal.h"

namespace ncf {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kPer = (int)(kMomentChunk / kThreads);  // samples per thread in a chunk
static_assert(kPer * kThreads == kMomentChunk, "chunk must be a multiple of the block");

// Sum over a wave by a fixed butterfly (every lane ends with the same total:
// each step adds the same two values on both partners), then over the
// block's waves in index order: deterministic, one barrier.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

template <int Q>
__device__ __forceinline__ void block_sum(double (&v)[Q], double (*sh)[kWaves]) {
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < Q; ++q) v[q] = wave_sum(v[q]);
    __syncthreads();  // the exchange area may still be read by a previous call
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int q = 0; q < Q; ++q) sh[q][wave] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        double t = sh[q][0];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) t += sh[q][w];
        v[q] = t;
    }
}

__global__ void __launch_bounds__(kThreads)
k_chunk_moments(MomentsArgs a) {
    __shared__ double sh[3][kWaves];
    __shared__ int shf[kWaves];
    const Chunk ch = a.chunks[blockIdx.x];
    const SeriesDesc sd = a.series[ch.series];
    const gptr<const double> X = gbl(a.io->x[sd.set] + sd.xoff);
    const gptr<const double> t = gbl(sd.t);
    const gptr<const double> er = gbl(sd.err);
    const int tid = threadIdx.x;
    // the thread's samples stay in registers for the second pass
    double xs[kPer], ws[kPer];
    int bad = 0, unsorted = 0;
    double acc[3] = {0.0, 0.0, 0.0};  // sum w, sum w x, sum w^2
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int64_t i = ch.begin + tid + (int64_t)k * kThreads;
        xs[k] = 0.0;
        ws[k] = 0.0;
        if (i < ch.end) {
            const double ti = t[i], xi = X[i];
            double wi = 1.0;
            if (sd.err) {
                const double e = er[i];
                if (sd.wmode) {
                    if (!(e >= 0.0) || !isfinite(e)) bad = 1;
                    wi = e;
                } else {
                    if (!(e > 0.0) || !isfinite(e)) bad = 1;
                    wi = 1.0 / (e * e);
                }
            }
            if (!isfinite(ti) || !isfinite(xi)) bad = 1;
            if (i > 0 && !(ti >= t[i - 1])) unsorted = 1;
            xs[k] = xi;
            ws[k] = wi;
            acc[0] += wi;
            acc[1] += wi * xi;
            acc[2] += wi * wi;
        }
    }
    int fl = bad | (unsorted << 1);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) fl |= __shfl_xor(fl, off);
    if ((tid & 63) == 0) shf[tid >> 6] = fl;
    block_sum<3>(acc, sh);
    const double mean = acc[1] / acc[0];
    double m2[1] = {0.0};
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const double d = xs[k] - mean;
        m2[0] += ws[k] * d * d;  // zero weight outside the chunk
    }
    block_sum<1>(m2, sh);
    if (tid == 0) {
        int f = 0;
        for (int w = 0; w < kWaves; ++w) f |= shf[w];
        double* p = a.chunk_part + kChunkPart * (int64_t)blockIdx.x;
        p[0] = acc[0];
        p[1] = mean;
        p[2] = m2[0];
        p[3] = (double)f;
        p[4] = acc[2];
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
// order; then a fixed left-to-right pairwise tree over the lanes of each
// wave (shuffles) and over the waves in order.
__global__ void __launch_bounds__(kThreads)
k_series_finalize(MomentsArgs a) {
    __shared__ double sh[4][kWaves];
    __shared__ int shf[kWaves];
    const int s = blockIdx.x;
    const int tid = threadIdx.x;
    if (s == 0 && a.lag_src)
        for (int64_t i = tid; i < a.nlag; i += kThreads) gbl(a.lag_dst)[i] = gbl(a.lag_src)[i];
    const int lane = tid & 63, wave = tid >> 6;
    const SeriesDesc sd = a.series[s];
    double sw = 0.0, mean = 0.0, m2 = 0.0, sw2 = 0.0;
    int fl = 0;
    const int per = (sd.nchunk + kThreads - 1) / kThreads;
    const int c0 = tid * per, c1 = min(sd.nchunk, c0 + per);
    for (int c = c0; c < c1; ++c) {
        const double* p = a.chunk_part + kChunkPart * (int64_t)(sd.chunk0 + c);
        merge_moments(sw, mean, m2, p[0], p[1], p[2]);
        fl |= (int)p[3];
        sw2 += p[4];
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double w1 = __shfl_down(sw, off), m1 = __shfl_down(mean, off),
                     q1 = __shfl_down(m2, off), s1 = __shfl_down(sw2, off);
        const int f1 = __shfl_down(fl, off);
        if ((lane & (2 * off - 1)) == 0) {  // left operand of this level
            merge_moments(sw, mean, m2, w1, m1, q1);
            fl |= f1;
            sw2 += s1;
        }
    }
    if (lane == 0) {
        sh[0][wave] = sw;
        sh[1][wave] = mean;
        sh[2][wave] = m2;
        sh[3][wave] = sw2;
        shf[wave] = fl;
    }
    __syncthreads();
    if (tid != 0) return;
    sw = sh[0][0];
    mean = sh[1][0];
    m2 = sh[2][0];
    sw2 = sh[3][0];
    fl = shf[0];
    for (int w = 1; w < kWaves; ++w) {
        merge_moments(sw, mean, m2, sh[0][w], sh[1][w], sh[2][w]);
        fl |= shf[w];
        sw2 += sh[3][w];
    }
    SeriesStat st;
    st.status = NCF_OK;
    st.pad = 0;
    const double sdv = sqrt(m2 / sw);
    st.mean = mean;
    st.sd = sdv;
    st.sw = sw;
    st.sw2 = sw2;
    st.tmin = sd.t[0];
    st.tmax = sd.t[sd.n - 1];
    if (sd.n < 2 || (fl & 1))
        st.status = NCF_E_INVALID_ARG;
    else if (fl & 2)
        st.status = NCF_E_UNSORTED;
    else if (!(sdv > 0.0) || !isfinite(sdv))
        st.status = NCF_E_DEGENERATE;
    a.stats[s] = st;
}

// Inclusive sum over a wave by shuffles (fixed order per lane).
__device__ __forceinline__ double wave_scan(double v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double t = __shfl_up(v, off);
        if (lane >= off) v += t;
    }
    return v;
}

// Chunk-local inclusive prefix sums of x (x[k]: sample tid + k kThreads of
// the chunk), in place; returns the chunk total. The samples pass through
// LDS so that each thread holds a run of kPer consecutive samples and adds
// them in order; the run totals take one wave scan, and each run adds the
// totals of the preceding waves (in wave order) and of the preceding runs of
// its wave: one scan per run instead of one per row of samples. buf holds
// one chunk with a pad slot per run (kMomentChunk + kMomentChunk / kPer).
__device__ __forceinline__ double chunk_scan(double (&x)[kPer], double* buf, double* wsum) {
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    auto pad = [](int e) { return e + e / kPer; };
    __syncthreads();  // buf and wsum may still be read by a previous scan
#pragma unroll
    for (int k = 0; k < kPer; ++k) buf[pad(tid + k * kThreads)] = x[k];
    __syncthreads();
    double r[kPer];
#pragma unroll
    for (int m = 0; m < kPer; ++m) r[m] = buf[pad(tid * kPer + m)];
#pragma unroll
    for (int m = 1; m < kPer; ++m) r[m] += r[m - 1];
    const double incl = wave_scan(r[kPer - 1]);
    const double before = __shfl_up(incl, 1);  // runs of the wave before this one
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    double carry = 0.0, total = 0.0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) {
        if (q < wave) carry += wsum[q];
        total += wsum[q];
    }
    if (lane > 0) carry += before;
#pragma unroll
    for (int m = 0; m < kPer; ++m) buf[pad(tid * kPer + m)] = carry + r[m];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; ++k) x[k] = buf[pad(tid + k * kThreads)];
    return total;
}

// Standardize one chunk and write the chunk-local inclusive prefix sums.
// A thread holds the samples tid + k * kThreads (k < kPer) of its chunk: all
// loads are issued before any store; the prefix sums come from chunk_scan.
__global__ void __launch_bounds__(kThreads)
k_standardize(MomentsArgs a) {
    __shared__ double sbuf[kMomentChunk + kMomentChunk / kPer];
    __shared__ double swsum[kWaves];
    const Chunk ch = a.chunks[blockIdx.x];
    const SeriesDesc sd = a.series[ch.series];
    const SeriesStat st = a.stats[ch.series];
    const gptr<const double> X = gbl(a.io->x[sd.set] + sd.xoff);
    const gptr<const double> er = gbl(sd.err);
    const int tid = threadIdx.x;
    const bool ok = st.status == NCF_OK;
    const double mean = st.mean;
    const double inv_sd = ok ? 1.0 / st.sd : 0.0;
    // weights scaled to a mean within a factor 2 of 1 over the series: the
    // estimator is invariant (C, B and the series' lag-0 sums scale
    // together), and the spectral route packs two series' grids into one
    // FP32 transform, whose rounding is relative to the larger of the two
    // (weights of 1/err^2 with err = 0.05 against unit weights: 400 times
    // the error on the smaller one). The scale is a power of two, so
    // integer weights (bootstrap multiplicities) stay exact and so do the
    // sums of their prefix arrays: a window of samples of weight 0 has a
    // weighted pair sum of exactly 0
    const double wscale = (sd.err && ok && st.sw > 0.0)
                              ? ldexp(1.0, (int)lrint(log2((double)sd.n / st.sw)))
                              : 1.0;
    double v[kPer], w[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int64_t i = ch.begin + tid + (int64_t)k * kThreads;
        v[k] = 0.0;
        w[k] = 0.0;
        if (i < ch.end) {
            double wk = 1.0;
            if (sd.err) {
                const double e = er[i];
                wk = (sd.wmode ? e : 1.0 / (e * e)) * wscale;
            }
            w[k] = wk;
            v[k] = X[i];
        }
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int64_t i = ch.begin + tid + (int64_t)k * kThreads;
        if (i < ch.end) {
            v[k] = ok ? w[k] * ((v[k] - mean) * inv_sd) : 0.0;
            if (sd.v32) gbl(sd.v32)[i] = (float)v[k];
            if (sd.v64) gbl(sd.v64)[i] = v[k];
            if (sd.w64) gbl(sd.w64)[i] = w[k];
        }
    }
    if (sd.pv == nullptr) return;
    // prefix index of sample i within the series' prefix array: i + 1
    const bool scan_w = sd.pw != nullptr;  // weight prefix only with weights
    // count of samples with a nonzero weight (weighted series): exact in
    // FP64 whatever the weights are, so a window of zero-weight samples only
    // is recognized as empty even where the weight prefix differences leave
    // rounding residue
    const bool scan_z = sd.pz != nullptr;
    double z[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) z[k] = w[k] != 0.0 ? 1.0 : 0.0;
    const double tv = chunk_scan(v, sbuf, swsum);
    const double tw = scan_w ? chunk_scan(w, sbuf, swsum) : 0.0;
    const double tz = scan_z ? chunk_scan(z, sbuf, swsum) : 0.0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int64_t i = ch.begin + tid + (int64_t)k * kThreads;
        if (i < ch.end) {
            gbl(sd.pv)[i + 1] = v[k];
            if (scan_w) gbl(sd.pw)[i + 1] = w[k];
            if (scan_z) gbl(sd.pz)[i + 1] = z[k];
        }
    }
    if (tid == 0) {
        a.chunk_tot[3 * (int64_t)blockIdx.x] = tv;
        a.chunk_tot[3 * (int64_t)blockIdx.x + 1] = tw;
        a.chunk_tot[3 * (int64_t)blockIdx.x + 2] = tz;
        if (ch.begin == 0) {
            sd.pv[0] = 0.0;
            if (sd.pw) sd.pw[0] = 0.0;
            if (sd.pz) sd.pz[0] = 0.0;
        }
    }
}

// Exclusive scan of chunk totals per series (in place: chunk_tot becomes the
// offset to add to each chunk). One workgroup per series: per-thread runs in
// order, then a scan of the run totals (wave scans, then the totals of the
// preceding waves).
__global__ void __launch_bounds__(kThreads)
k_chunk_offsets(MomentsArgs a) {
    __shared__ double shv[3][kWaves];
    const int s = blockIdx.x;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const SeriesDesc sd = a.series[s];
    if (!sd.pv) return;
    const int per = (sd.nchunk + kThreads - 1) / kThreads;
    const int c0 = tid * per, c1 = min(sd.nchunk, c0 + per);
    double tv = 0.0, tw = 0.0, tz = 0.0;
    for (int c = c0; c < c1; ++c) {
        const double* p = a.chunk_tot + 3 * (int64_t)(sd.chunk0 + c);
        tv += p[0];
        tw += p[1];
        tz += p[2];
    }
    const double iv = wave_scan(tv), iw = wave_scan(tw), iz = wave_scan(tz);
    if (lane == 63) {
        shv[0][wave] = iv;
        shv[1][wave] = iw;
        shv[2][wave] = iz;
    }
    __syncthreads();
    // exclusive within the wave
    double ev = __shfl_up(iv, 1), ew = __shfl_up(iw, 1), ez = __shfl_up(iz, 1);
    double cv = 0.0, cw = 0.0, cz = 0.0;
    for (int q = 0; q < wave; ++q) {
        cv += shv[0][q];
        cw += shv[1][q];
        cz += shv[2][q];
    }
    if (lane > 0) {
        cv += ev;
        cw += ew;
        cz += ez;
    }
    for (int c = c0; c < c1; ++c) {
        double* p = a.chunk_tot + 3 * (int64_t)(sd.chunk0 + c);
        const double v = p[0], w = p[1], z = p[2];
        p[0] = cv;
        p[1] = cw;
        p[2] = cz;
        cv += v;
        cw += w;
        cz += z;
    }
}

__global__ void __launch_bounds__(kThreads)
k_fill_alternating(double* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) p[i] = (i & 1) ? -1.0 : 1.0;
}

// One workgroup per segment; up to three arrays share the segment table.
__global__ void __launch_bounds__(kThreads)
k_copy_segments(const CopySeg* __restrict__ segs, const double* __restrict__ s0,
                double* __restrict__ d0, const double* __restrict__ s1, double* __restrict__ d1,
                const double* __restrict__ s2, double* __restrict__ d2) {
    const CopySeg g = segs[blockIdx.x];
    for (int64_t i = threadIdx.x; i < g.len; i += kThreads) {
        if (s0) d0[g.dst_off + i] = s0[g.src_off + i];
        if (s1) d1[g.dst_off + i] = s1[g.src_off + i];
        if (s2) d2[g.dst_off + i] = s2[g.src_off + i];
    }
}

}  // namespace

int launch_copy_segments(const CopySeg* d_segs, int64_t nseg, const double* const s[3],
                         double* const d[3], hipStream_t st) {
    if (nseg <= 0 || (!s[0] && !s[1] && !s[2])) return NCF_OK;
    if (nseg > INT32_MAX) return NCF_E_INVALID_ARG;
    hipLaunchKernelGGL(k_copy_segments, dim3((unsigned)nseg), dim3(kThreads), 0, st, d_segs,
                       s[0], d[0], s[1], d[1], s[2], d[2]);
    NCF_CHECK_LAUNCH();
    return NCF_OK;
}

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
    // the prefix sums stay chunk-local: their reader (the window scan) adds
    // the chunk offsets computed here
    if (a.prefix) {
        hipLaunchKernelGGL(k_chunk_offsets, dim3(a.nseries), dim3(kThreads), 0, st, a);
        NCF_CHECK_LAUNCH();
    }
    return NCF_OK;
}

}  // namespace ncf
