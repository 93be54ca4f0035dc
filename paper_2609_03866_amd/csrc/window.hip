// window.hip -- per-lag window scan over sorted times (step A7).
//
// For every outer sample j and lag k the window of the PairCount / CorrSum
// algorithms (Appendix A.2 and B) is
//   Gaussian : t_i in [c - 6h, c + 6h)      weight exp(-d^2/2h^2)
//   rectangle: t_i in [c - h,  c + h]       weight 1
// with centre c = s_j + delta_k, delta_k = eps * tau_k (eps = +1 ACF,
// -1 CCF). The paper runs one two-pointer scan per lag over all j; here the
// (j, k) plane is tiled: a workgroup owns J consecutive outer samples and up
// to 64 consecutive sorted lag offsets, stages the window samples its tile
// can reach in LDS, and each lane runs the two-pointer scan for one lag over
// a contiguous run of j. Lane results are combined in a fixed order, tiles
// write partial sums, and a second kernel sums the partials over j-tiles in
// order, so every result is deterministic.
//
// Per (j, k) the rectangle kernel needs only the two window bounds: the
// count is hi - lo (exact int64) and the numerator uses the FP64 prefix sums
// of the window values (Algorithm "CorrSum, rectangle"). The Gaussian kernel
// sums its weights over the window: FP64 differences, scaled by 1/h, an FP32
// exp2 (or FP64 exp in the FP64 path) and FP64 accumulation.
//
// Window predicates are evaluated exactly as (s_j + delta_k) - W and
// (s_j + delta_k) + W in FP64 with W = 6h or h, so rectangle counts are
// bit-identical to a sequential scan.
#include "internal.h"

namespace ncf {

namespace {

constexpr int kThreads = 256;

// First index i in [0, n) with (upper ? a[i] > key : a[i] >= key), else n.
// Called by a whole wavefront: 64 probes per round.
template <typename T>
__device__ int64_t wave_search(const T* a, int64_t n, T key, bool upper) {
    const int lane = threadIdx.x & 63;
    int64_t lo = 0, hi = n;
    while (hi > lo) {
        const int64_t len = hi - lo;
        const int64_t stride = (len + 63) / 64;
        const int64_t p = lo + (int64_t)lane * stride;
        bool before = false;
        if (p < hi) {
            T v = a[p];
            before = upper ? (v <= key) : (v < key);
        }
        const uint64_t m = __ballot(before);
        const int q = __popcll(m);
        if (stride == 1 || q == 0) return lo + (stride == 1 ? q : 0);
        const int64_t nlo = lo + (int64_t)(q - 1) * stride + 1;
        const int64_t phq = lo + (int64_t)q * stride;
        hi = phq < hi ? phq : hi;
        lo = nlo;
    }
    return lo;
}

__device__ __forceinline__ int lower_idx(const double* a, int lo, int hi, double key) {
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int upper_idx(const double* a, int lo, int hi, double key) {
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] <= key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

struct Acc {
    double C, B, b;
    int64_t n;
};

// Two-pointer scan of one lane over outer samples [ja, jb) (indices relative
// to the tile's first outer sample) for one lag offset `delta`, on the window
// samples Tl[0, len) (relative to the tile's first window sample).
template <uint32_t F>
__device__ __forceinline__ void scan_lane(Acc& acc, const double* Tl, const double* A1,
                                          const double* A2, int len, const double* Sl,
                                          const double* VOl, const double* WOl, int ja, int jb,
                                          double delta, double W, double inv_h) {
    constexpr bool RECT = (F & WIN_RECT) != 0;
    constexpr bool NUMER = (F & WIN_NUMER) != 0;
    constexpr bool WTD = (F & WIN_WEIGHTED) != 0;
    constexpr bool E64 = (F & WIN_EXP64) != 0;
    if (ja >= jb) return;
    double c = Sl[ja] + delta;
    int lo = lower_idx(Tl, 0, len, c - W);
    int hi = RECT ? upper_idx(Tl, lo, len, c + W) : lower_idx(Tl, lo, len, c + W);
    // -0.5 * log2(e): exp(-z^2/2) = exp2(z^2 * kHalfLog2e)
    const float kHalfLog2e = -0.72134752044448170f;
    for (int j = ja; j < jb; ++j) {
        c = Sl[j] + delta;
        const double lk = c - W;
        const double hk = c + W;
        while (lo < len && Tl[lo] < lk) ++lo;
        if (RECT) {
            while (hi < len && Tl[hi] <= hk) ++hi;
            acc.n += hi - lo;
            if (NUMER) acc.C += VOl[j] * (A1[hi] - A1[lo]);
            if (WTD) acc.B += WOl[j] * (A2[hi] - A2[lo]);
        } else {
            while (hi < len && Tl[hi] < hk) ++hi;
            double bj = 0.0, Cj = 0.0, Bj = 0.0;
            for (int i = lo; i < hi; ++i) {
                const double z = (Tl[i] - c) * inv_h;
                double e;
                if (E64) {
                    e = exp(-0.5 * z * z);
                } else {
                    const float zf = (float)z;
                    e = (double)__builtin_amdgcn_exp2f(zf * zf * kHalfLog2e);
                }
                bj += e;
                if (NUMER) Cj += e * A1[i];
                if (WTD) Bj += e * A2[i];
            }
            acc.b += bj;
            acc.n += hi - lo;
            if (NUMER) acc.C += Cj * VOl[j];
            if (WTD) acc.B += Bj * WOl[j];
        }
    }
}

template <uint32_t F>
__global__ void __launch_bounds__(kThreads)
k_window(const WinTask* __restrict__ tasks, const int64_t* __restrict__ item0, int ntasks,
         int64_t nitems, int64_t nblocks, int cap, int jmax) {
    constexpr bool RECT = (F & WIN_RECT) != 0;
    constexpr bool NUMER = (F & WIN_NUMER) != 0;
    constexpr bool WTD = (F & WIN_WEIGHTED) != 0;
    // window-side auxiliary arrays: rectangle -> prefix sums (pv, pw);
    // Gaussian -> values / weights
    constexpr bool HAS_A1 = NUMER;
    constexpr bool HAS_A2 = WTD;
    extern __shared__ double lds[];
    __shared__ int64_t sh_rng[4];

    const int64_t item = xcd_remap(blockIdx.x, nblocks);
    if (item >= nitems) return;
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;

    // task of this item: last ti with item0[ti] <= item
    const int ti = (int)wave_search<int64_t>(item0, ntasks, item, true) - 1;
    const WinTask& T = tasks[ti];
    const int64_t local = item - T.item0;
    const int jt = (int)(local / T.n_kt);
    const int kt = (int)(local % T.n_kt);
    const int64_t j0 = (int64_t)jt * T.J;
    const int64_t j1 = min(j0 + (int64_t)T.J, T.n_out);
    const int k0 = kt * 64;
    const int nk = min(64, T.K - k0);
    const double W = T.W;

    if (wave == 0) {
        const double dmin = T.delta[k0];
        const double dmax = T.delta[k0 + nk - 1];
        const double lo_key = (T.s[j0] + dmin) - W;
        const double hi_key = (T.s[j1 - 1] + dmax) + W;
        int64_t tlo = wave_search<double>(T.t, T.n_win, lo_key, false);
        int64_t thi = wave_search<double>(T.t, T.n_win, hi_key, RECT);
        if (lane == 0) {
            sh_rng[0] = tlo;
            sh_rng[1] = thi;
        }
    }
    __syncthreads();
    const int64_t tlo = sh_rng[0];
    const int64_t thi = sh_rng[1];
    const int len = (int)(thi - tlo);
    const int nj = (int)(j1 - j0);
    const bool fits = (thi - tlo) <= cap && nj <= jmax;

    // LDS carve-up
    double* Ts = lds;
    double* A1s = Ts + cap;
    double* A2s = A1s + (HAS_A1 ? cap + 1 : 0);
    double* Ss = A2s + (HAS_A2 ? cap + 1 : 0);
    double* VOs = Ss + jmax;
    double* WOs = VOs + (NUMER ? jmax : 0);
    double* Red = lds;  // reused after the scan

    const double* A1g = RECT ? T.pv : T.v;
    const double* A2g = RECT ? T.pw : T.w;
    const int a_len = RECT ? len + 1 : len;  // prefix arrays need the entry at hi
    if (fits) {
        for (int i = tid; i < len; i += kThreads) Ts[i] = T.t[tlo + i];
        if (HAS_A1)
            for (int i = tid; i < a_len; i += kThreads) A1s[i] = A1g[tlo + i];
        if (HAS_A2)
            for (int i = tid; i < a_len; i += kThreads) A2s[i] = A2g[tlo + i];
        for (int i = tid; i < nj; i += kThreads) {
            Ss[i] = T.s[j0 + i];
            if (NUMER) VOs[i] = T.vo[j0 + i];
            if (WTD) WOs[i] = T.wo[j0 + i];
        }
    }
    __syncthreads();

    // lane -> (lag, j-stream)
    int KW = 1;
    while (KW < nk) KW <<= 1;
    const int streams = 64 / KW;
    const int kl = lane & (KW - 1);
    const int stream = lane / KW;
    const bool active = kl < nk;
    const int nseg = 4 * streams;
    const int seg = wave * streams + stream;
    const int ja = (int)((int64_t)nj * seg / nseg);
    const int jb = (int)((int64_t)nj * (seg + 1) / nseg);
    const double delta = active ? T.delta[k0 + kl] : 0.0;
    const double inv_h = 1.0 / T.h;

    Acc acc = {0.0, 0.0, 0.0, 0};
    if (active) {
        if (fits)
            scan_lane<F>(acc, Ts, A1s, A2s, len, Ss, VOs, WOs, ja, jb, delta, W, inv_h);
        else
            scan_lane<F>(acc, T.t + tlo, HAS_A1 ? A1g + tlo : nullptr,
                         HAS_A2 ? A2g + tlo : nullptr, len, T.s + j0,
                         NUMER ? T.vo + j0 : nullptr, WTD ? T.wo + j0 : nullptr, ja, jb, delta,
                         W, inv_h);
    }
    __syncthreads();  // staging area is reused for the reduction
    Red[4 * tid + 0] = acc.C;
    Red[4 * tid + 1] = acc.B;
    Red[4 * tid + 2] = acc.b;
    Red[4 * tid + 3] = __longlong_as_double((long long)acc.n);
    __syncthreads();
    if (tid < nk) {
        double C = 0.0, B = 0.0, b = 0.0;
        long long n = 0;
        for (int w = 0; w < 4; ++w)
            for (int st = 0; st < streams; ++st) {
                const int src = 4 * (w * 64 + st * KW + tid);
                C += Red[src + 0];
                B += Red[src + 1];
                b += Red[src + 2];
                n += __double_as_longlong(Red[src + 3]);
            }
        double* out = T.part + ((int64_t)jt * T.K + k0 + tid) * 4;
        out[0] = C;
        out[1] = B;
        out[2] = b;
        out[3] = __longlong_as_double(n);
    }
}

// Sum partials over j-tiles in order; scale the Gaussian weights by
// 1/(sqrt(2 pi) h) (eq. Gaussian_kernel).
__global__ void k_window_reduce(const WinTask* __restrict__ tasks, int ntasks,
                                const int64_t* __restrict__ k0s, int64_t total_k,
                                uint32_t flags) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total_k) return;
    // task: last ti with k0s[ti] <= g
    int lo = 0, hi = ntasks;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (k0s[mid] <= g)
            lo = mid;
        else
            hi = mid;
    }
    const WinTask& T = tasks[lo];
    const int k = (int)(g - k0s[lo]);
    double C = 0.0, B = 0.0, b = 0.0;
    long long n = 0;
    for (int jt = 0; jt < T.n_jt; ++jt) {
        const double* p = T.part + ((int64_t)jt * T.K + k) * 4;
        C += p[0];
        B += p[1];
        b += p[2];
        n += __double_as_longlong(p[3]);
    }
    if (!(flags & WIN_RECT)) {
        const double norm = 1.0 / (T.h * 2.5066282746310002);  // 1/(h sqrt(2 pi))
        C *= norm;
        B *= norm;
        b *= norm;
    } else {
        b = (double)n;
    }
    double* out = T.sums + (int64_t)k * 4;
    out[0] = C;
    out[1] = B;
    out[2] = b;
    out[3] = __longlong_as_double(n);
}

template <uint32_t F>
int launch_window_t(const WinTask* d_tasks, const int64_t* d_item0, int ntasks, int64_t nitems,
                    int cap, int jmax, hipStream_t st, double work) {
    constexpr bool RECT = (F & WIN_RECT) != 0;
    constexpr bool NUMER = (F & WIN_NUMER) != 0;
    constexpr bool WTD = (F & WIN_WEIGHTED) != 0;
    size_t stage = (size_t)cap + (NUMER ? cap + 1 : 0) + (WTD ? cap + 1 : 0) + jmax +
                   (NUMER ? jmax : 0) + (WTD ? jmax : 0);
    size_t red = 4 * kThreads;
    size_t bytes = (stage > red ? stage : red) * sizeof(double);
    (void)RECT;
    int64_t nblocks = round_up(nitems, kXcds);
    ProfScope p(st, RECT ? "window_rect" : "window_gauss", work, "valu_ops");
    hipLaunchKernelGGL(k_window<F>, dim3((unsigned)nblocks), dim3(kThreads), bytes, st, d_tasks,
                       d_item0, ntasks, nitems, nblocks, cap, jmax);
    NCF_CHECK_LAUNCH();
    return NCF_OK;
}

}  // namespace

int launch_window(const WinTask* d_tasks, const int64_t* d_item0, int ntasks, int64_t nitems,
                  uint32_t flags, int cap, int jmax, hipStream_t st, double work) {
    if (nitems <= 0) return NCF_OK;
    switch (flags) {
#define NCF_WIN_CASE(f) \
    case (f):           \
        return launch_window_t<(f)>(d_tasks, d_item0, ntasks, nitems, cap, jmax, st, work);
        NCF_WIN_CASE(0)
        NCF_WIN_CASE(WIN_NUMER)
        NCF_WIN_CASE(WIN_WEIGHTED)
        NCF_WIN_CASE(WIN_NUMER | WIN_WEIGHTED)
        NCF_WIN_CASE(WIN_EXP64)
        NCF_WIN_CASE(WIN_EXP64 | WIN_NUMER)
        NCF_WIN_CASE(WIN_EXP64 | WIN_WEIGHTED)
        NCF_WIN_CASE(WIN_EXP64 | WIN_NUMER | WIN_WEIGHTED)
        NCF_WIN_CASE(WIN_RECT)
        NCF_WIN_CASE(WIN_RECT | WIN_NUMER)
        NCF_WIN_CASE(WIN_RECT | WIN_WEIGHTED)
        NCF_WIN_CASE(WIN_RECT | WIN_NUMER | WIN_WEIGHTED)
#undef NCF_WIN_CASE
        default:
            set_error("window scan: unsupported flag set %u", flags);
            return NCF_E_UNSUPPORTED;
    }
}

int launch_window_reduce(const WinTask* d_tasks, int ntasks, int64_t total_k, const int64_t* d_k0,
                         uint32_t flags, hipStream_t st) {
    if (total_k <= 0) return NCF_OK;
    ProfScope p(st, "window_reduce", 0.0, "bytes");
    hipLaunchKernelGGL(k_window_reduce, dim3((unsigned)ceil_div(total_k, 128)), dim3(128), 0, st,
                       d_tasks, ntasks, d_k0, total_k, flags);
    NCF_CHECK_LAUNCH();
    return NCF_OK;
}

}  // namespace ncf
