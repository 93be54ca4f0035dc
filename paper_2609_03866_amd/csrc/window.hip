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
#include <algorithm>
#include <map>
#include <mutex>
#include <utility>

#include "internal.h"

namespace ncf {

namespace {

constexpr int kThreads = 256;

struct Acc {
    double C, B, b;
    int64_t n;
};

// Dynamic LDS of the window kernel, referenced by symbol so that reads
// through it are LDS instructions.
extern __shared__ double g_win_lds[];

typedef __attribute__((address_space(1))) const double* gdp;

constexpr double kInf = __builtin_huge_val();

// Window samples and outer samples staged in LDS; the staged window array
// is followed by +inf sentinels, so reads up to 8 past its end need no check.
struct LdsView {
    int t0, a10, a20, s0, vo0, wo0, len;
    __device__ __forceinline__ double T(int i) const { return g_win_lds[t0 + i]; }
    __device__ __forceinline__ double A1(int i) const { return g_win_lds[a10 + i]; }
    __device__ __forceinline__ double A2(int i) const { return g_win_lds[a20 + i]; }
    __device__ __forceinline__ double A3(int) const { return 0.0; }  // rectangle only, global path
    __device__ __forceinline__ double S(int j) const { return g_win_lds[s0 + j]; }
    __device__ __forceinline__ double VO(int j) const { return g_win_lds[vo0 + j]; }
    __device__ __forceinline__ double WO(int j) const { return g_win_lds[wo0 + j]; }
};

// Fallback when the window range does not fit in LDS: global memory with
// explicit bounds.
struct GlbView {
    gdp t, a1, a2, a3, s, vo, wo;
    int len;
    __device__ __forceinline__ double T(int i) const { return i < len ? t[i] : kInf; }
    __device__ __forceinline__ double A1(int i) const { return a1[i]; }
    __device__ __forceinline__ double A2(int i) const { return a2[i]; }
    __device__ __forceinline__ double A3(int i) const { return a3[i]; }
    __device__ __forceinline__ double S(int j) const { return s[j]; }
    __device__ __forceinline__ double VO(int j) const { return vo[j]; }
    __device__ __forceinline__ double WO(int j) const { return wo[j]; }
};

// Offset of chunk-local prefix entry j (q: 0 values, 1 weights, 2 counts).
__device__ __forceinline__ double prefix_off(gdp poff, int64_t j, int q) {
    return j > 0 ? poff[3 * ((j - 1) / kMomentChunk) + q] : 0.0;
}

// The same view of a rectangle task whose prefix arrays start at prefix
// entry base: each read adds its chunk offset.
struct GlbPrefixView : GlbView {
    gdp poff;
    int64_t base;
    __device__ __forceinline__ double A1(int i) const {
        return a1[i] + prefix_off(poff, base + i, 0);
    }
    __device__ __forceinline__ double A2(int i) const {
        return a2[i] + prefix_off(poff, base + i, 1);
    }
    __device__ __forceinline__ double A3(int i) const {
        return a3[i] + prefix_off(poff, base + i, 2);
    }
};

template <typename V>
__device__ __forceinline__ int lower_idx(const V& v, int lo, int hi, double key) {
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (v.T(mid) < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

template <typename V>
__device__ __forceinline__ int upper_idx(const V& v, int lo, int hi, double key) {
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (v.T(mid) <= key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Advance a pointer over sorted samples while T(p) < key (or <= key):
// kAdv independent reads per round; sorted order makes the passing samples a
// prefix of them.
constexpr int kAdv = 3;

template <bool LE, typename V>
__device__ __forceinline__ int advance(const V& v, int p, double key) {
    for (;;) {
        int a = 0;
#pragma unroll
        for (int q = 0; q < kAdv; ++q) a += LE ? (v.T(p + q) <= key) : (v.T(p + q) < key);
        p += a;
        if (a < kAdv) return p;
    }
}

// Two-pointer scan of one lane over outer samples [ja, jb) (relative to the
// tile's first outer sample) for one lag offset `delta`, on the window
// samples [0, len) (relative to the tile's first window sample).
template <uint32_t F, typename V>
__device__ __forceinline__ void scan_lane(Acc& acc, const V& v, int ja, int jb, double delta,
                                          double W, double inv_h) {
    constexpr bool RECT = (F & WIN_RECT) != 0;
    constexpr bool NUMER = (F & WIN_NUMER) != 0;
    constexpr bool WTD = (F & WIN_WEIGHTED) != 0;
    constexpr bool E64 = (F & WIN_EXP64) != 0;
    if (ja >= jb) return;
    const int len = v.len;
    double c = v.S(ja) + delta;
    int lo = lower_idx(v, 0, len, c - W);
    int hi = RECT ? upper_idx(v, lo, len, c + W) : lower_idx(v, lo, len, c + W);
    // exp(-d^2/2h^2) = exp2(d^2 * k2), k2 = -log2(e) / (2 h^2); the argument
    // is formed in FP64 and its integer part applied exactly, so the FP32
    // exp2 only sees the fraction (weights keep FP32 relative accuracy even
    // at the window edge)
    const double k2 = -0.72134752044448170 * inv_h * inv_h;
    double s_next = v.S(ja);
    for (int j = ja; j < jb; ++j) {
        c = s_next + delta;
        if (j + 1 < jb) s_next = v.S(j + 1);  // next centre's load overlaps this one
        const double lk = c - W;
        const double hk = c + W;
        lo = advance<false>(v, lo, lk);
        if (RECT) {
            hi = advance<true>(v, hi, hk);
            acc.n += hi - lo;
            if (NUMER) acc.C += v.VO(j) * (v.A1(hi) - v.A1(lo));
            if (WTD) {
                const double wo = v.WO(j);
                acc.B += wo * (v.A2(hi) - v.A2(lo));
                // pairs of two nonzero weights (exact integer count)
                if (wo != 0.0) acc.b += v.A3(hi) - v.A3(lo);
            }
        } else {
            hi = advance<false>(v, hi, hk);
            double bj = 0.0, Cj = 0.0, Bj = 0.0;
            // window points per round (reads past the window land on staged
            // samples or the sentinels); measured: one for the FP32
            // exponential, four for the FP64 one
            constexpr int kPts = E64 ? 4 : 1;
            for (int i = lo; i < hi; i += kPts) {
                double dd[kPts];
#pragma unroll
                for (int m = 0; m < kPts; ++m) dd[m] = v.T(i + m) - c;  // FP64 difference
#pragma unroll
                for (int m = 0; m < kPts; ++m) {
                    if (kPts == 1 || i + m < hi) {
                        if (E64) {
                            const double z = dd[m] * inv_h;
                            const double e = exp(-0.5 * z * z);
                            bj += e;
                            if (NUMER) Cj += e * v.A1(i + m);
                            if (WTD) Bj += e * v.A2(i + m);
                        } else {
                            const double a = dd[m] * dd[m] * k2;
                            const double n = floor(a);
                            const float e =
                                __builtin_amdgcn_ldexpf(__builtin_amdgcn_exp2f((float)(a - n)),
                                                        (int)n);
                            bj += (double)e;  // FP64 sum: windows of bursty
                                              // samples hold thousands of points
                            if (NUMER) Cj += (double)e * v.A1(i + m);
                            if (WTD) Bj += (double)e * v.A2(i + m);
                        }
                    }
                }
            }
            acc.b += bj;
            acc.n += hi - lo;
            if (NUMER) acc.C += Cj * v.VO(j);
            if (WTD) acc.B += Bj * v.WO(j);
        }
    }
}

// Rectangle scan over LDS. The window times are staged contiguously (then
// +inf sentinels), their prefix sums P (and PW, PZ) in parallel arrays `dp`
// doubles further on. The two bounds are LDS addresses into the time array
// and the times at them are kept in registers, so a bound is read again only
// after it moves; an outer sample whose window does not move costs two
// compares. Counts accumulate as address differences and a prefix value is
// read at a fixed distance from its bound. Same predicates and the same
// order of the numerator sums as scan_lane. The outer samples (s_j, vo_j,
// wo_j) are not staged: they come from global memory.
struct AccR {
    double C, B;
    double nz;  // weighted: pairs of two nonzero weights
    int bytes;  // sum over j of (hi - lo) * 8 S
};

// Window samples in LDS as records of S doubles: S = 2 interleaves each time
// with its value prefix (unweighted numerator scans: one paired read fetches
// both, the prefix at the final bounds is already in registers); S = 1 keeps
// the times alone, the prefix arrays at dp, 2 dp, ... doubles further on.
template <int S>
struct RectBounds {
    const double* plo;
    const double* phi;
    double tl, th;  // times at the bounds
    double pl, ph;  // (S = 2) value prefixes at the bounds
};

// bounds of the first outer sample of a run, by binary search
template <int S>
__device__ __forceinline__ void rect_init(RectBounds<S>& st, const double* win, int len, double c0,
                                          double W) {
    const double key = c0 - W;
    int a = 0, b = len;
    while (a < b) {
        const int m = (a + b) >> 1;
        if (win[S * m] < key)
            a = m + 1;
        else
            b = m;
    }
    st.plo = win + S * a;
    const double keyh = c0 + W;
    b = len;
    while (a < b) {
        const int m = (a + b) >> 1;
        if (win[S * m] <= keyh)
            a = m + 1;
        else
            b = m;
    }
    st.phi = win + S * a;
    st.tl = st.plo[0];
    st.th = st.phi[0];
    if (S == 2) {
        st.pl = st.plo[1];
        st.ph = st.phi[1];
    }
}

// One outer sample: move both bounds to its window, add its terms.
template <bool NUMER, bool WTD, int S>
__device__ __forceinline__ void rect_step(AccR& acc, RectBounds<S>& st, int dp, double s,
                                          double vo, double wo, double delta, double W) {
    constexpr int QW = NUMER ? 2 : 1;  // PW array follows P when both exist
    constexpr int QZ = QW + 1;         // then the nonzero-weight count prefix
    const double c = s + delta;
    const double lk = c - W;
    const double hk = c + W;
    // both bounds advance in one loop, one sample per round each, on the
    // lanes where one of them moves (reads past the staged times land on the
    // sentinels); measured faster than a loop per bound
    bool a = st.tl < lk, b = st.th <= hk;
    while (a || b) {
        st.plo += a ? S : 0;
        st.phi += b ? S : 0;
        st.tl = st.plo[0];
        st.th = st.phi[0];
        if (S == 2) {
            st.pl = st.plo[1];
            st.ph = st.phi[1];
        }
        a = st.tl < lk;
        b = st.th <= hk;
    }
    acc.bytes += (int)((const char*)st.phi - (const char*)st.plo);
    if (NUMER) acc.C += vo * (S == 2 ? st.ph - st.pl : st.phi[dp] - st.plo[dp]);
    if (WTD) {
        acc.B += wo * (st.phi[QW * dp] - st.plo[QW * dp]);
        if (wo != 0.0) acc.nz += st.phi[QZ * dp] - st.plo[QZ * dp];
    }
}

typedef const __attribute__((address_space(4))) double* cdp;

__device__ __forceinline__ cdp uniform_ptr(const double* p) {
    const uint64_t a = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    return (cdp)(((uint64_t)hi << 32) | lo);
}

// Every lane of the wave walks the same outer run [ja, jb) (one lag per
// lane): the outer samples come through scalar loads, eight at a time.
template <bool NUMER, bool WTD, int S>
__device__ __forceinline__ void scan_rect_wave(AccR& acc, const double* win, int dp, int len,
                                               int ja, int jb, double delta, double W,
                                               const double* gs, const double* gvo,
                                               const double* gwo) {
    ja = __builtin_amdgcn_readfirstlane(ja);
    jb = __builtin_amdgcn_readfirstlane(jb);
    if (ja >= jb) return;
    const cdp cs = uniform_ptr(gs);
    const cdp cvo = NUMER ? uniform_ptr(gvo) : cs;
    const cdp cwo = WTD ? uniform_ptr(gwo) : cs;
    RectBounds<S> st;
    rect_init(st, win, len, cs[ja] + delta, W);
    int j = ja;
    for (; j + 8 <= jb; j += 8) {
        double sb[8], vb[8], wb[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            sb[m] = cs[j + m];
            vb[m] = NUMER ? cvo[j + m] : 0.0;
            wb[m] = WTD ? cwo[j + m] : 0.0;
        }
#pragma unroll
        for (int m = 0; m < 8; ++m)
            rect_step<NUMER, WTD, S>(acc, st, dp, sb[m], vb[m], wb[m], delta, W);
    }
    for (; j < jb; ++j)
        rect_step<NUMER, WTD, S>(acc, st, dp, cs[j], NUMER ? cvo[j] : 0.0, WTD ? cwo[j] : 0.0,
                              delta, W);
}

// Each lane walks its own outer run (items of few lags): outer samples by
// vector loads, the next one's in flight while the current one is scanned.
template <bool NUMER, bool WTD, int S>
__device__ __forceinline__ void scan_rect_lane(AccR& acc, const double* win, int dp, int len,
                                               int ja, int jb, double delta, double W,
                                               gdp gs, gdp gvo, gdp gwo) {
    if (ja >= jb) return;
    RectBounds<S> st;
    rect_init(st, win, len, gs[ja] + delta, W);
    double s = gs[ja], vo = NUMER ? gvo[ja] : 0.0, wo = WTD ? gwo[ja] : 0.0;
    for (int j = ja; j < jb; ++j) {
        double s_n = 0.0, vo_n = 0.0, wo_n = 0.0;
        if (j + 1 < jb) {
            s_n = gs[j + 1];
            if (NUMER) vo_n = gvo[j + 1];
            if (WTD) wo_n = gwo[j + 1];
        }
        rect_step<NUMER, WTD, S>(acc, st, dp, s, vo, wo, delta, W);
        s = s_n;
        vo = vo_n;
        wo = wo_n;
    }
}

// One work item: (task, j-group, lag-tile) -> partial sums of the group. A
// j-group is up to G consecutive j-tiles; the workgroup stages and scans them
// in order, each lane keeping its sums across the tiles, so one partial per
// group and lag is written.
template <uint32_t F>
__device__ __forceinline__ void window_item(const WinTask* __restrict__ tasks,
                                            const int64_t* __restrict__ item0, int ntasks,
                                            int64_t item, int cap, int jmax) {
    constexpr bool RECT = (F & WIN_RECT) != 0;
    constexpr bool NUMER = (F & WIN_NUMER) != 0;
    constexpr bool WTD = (F & WIN_WEIGHTED) != 0;
    // window-side auxiliary arrays: rectangle -> prefix sums (pv, pw);
    // Gaussian -> values / weights
    constexpr bool HAS_A1 = NUMER;
    constexpr bool HAS_A2 = WTD;
    __shared__ int64_t sh_rng[4];
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;

    // task of this item: last ti with item0[ti] <= item
    const int ti = ntasks == 1 ? 0 : (int)wave_search<int64_t>(item0, ntasks, item, true) - 1;
    const WinTask& T = tasks[ti];
    const int64_t local = item - T.item0;
    const int jg = (int)(local / T.n_kt);
    const int kt = (int)(local % T.n_kt);
    const int jt_end = min(T.n_jt, (jg + 1) * T.G);
    const int k0 = kt * 64;
    const int nk = min(64, T.K - k0);
    const double W = T.W;

    // lane -> (lag, j-stream)
    int KW = 1;
    while (KW < nk) KW <<= 1;
    const int streams = 64 / KW;
    const int kl = lane & (KW - 1);
    const int stream = lane / KW;
    const bool active = kl < nk;
    const int nseg = 4 * streams;
    const int seg = wave * streams + stream;
    const double delta = active ? T.delta[k0 + kl] : 0.0;
    const double inv_h = 1.0 / T.h;

    // LDS carve-up (offsets in doubles)
    const int o_t = 0;
    const int o_a1 = o_t + cap + 8;
    const int o_a2 = o_a1 + (HAS_A1 ? cap + 8 : 0);
    const int o_s = o_a2 + (HAS_A2 ? cap + 8 : 0);
    const int o_vo = o_s + jmax;
    const int o_wo = o_vo + (NUMER ? jmax : 0);
    const double* A1g = RECT ? T.pv : T.v;
    const double* A2g = RECT ? T.pw : T.w;
    // rectangle: times, then the prefix arrays (each cap + 8 long: values,
    // weights and the nonzero-weight count), or with values only (no
    // weights) each time paired with its value prefix; the outer samples
    // stay in global memory
    constexpr int QW = NUMER ? 2 : 1;
    const int dp = cap + 8;
    // unweighted numerator: time and value prefix interleaved (records of 2)
    constexpr int RS = (RECT && NUMER && !WTD) ? 2 : 1;
    const gdp gt = (gdp)T.t, gs = (gdp)T.s, gvo = (gdp)T.vo, gwo = (gdp)T.wo;
    const gdp ga1 = (gdp)A1g, ga2 = (gdp)A2g, ga3 = (gdp)T.pz, gpo = (gdp)T.poff;

    // window range [tlo, thi) of j-tile jt for this item's lags, into slot
    // sl of sh_rng: wave 0 searches the low end, wave 1 the high end
    auto search_tile = [&](int jt_s, int sl) {
        const int64_t a0 = (int64_t)jt_s * T.J;
        const int64_t a1 = min(a0 + (int64_t)T.J, T.n_out);
        if (wave == 0) {
            const double lo_key = (T.s[a0] + T.delta[k0]) - W;
            const int64_t r = wave_search<double>(T.t, T.n_win, lo_key, false);
            if (lane == 0) sh_rng[2 * sl] = r;
        } else if (wave == 1) {
            const double hi_key = (T.s[a1 - 1] + T.delta[k0 + nk - 1]) + W;
            const int64_t r = wave_search<double>(T.t, T.n_win, hi_key, RECT);
            if (lane == 0) sh_rng[2 * sl + 1] = r;
        }
    };
    Acc acc = {0.0, 0.0, 0.0, 0};
    search_tile(jg * T.G, 0);
    for (int jt = jg * T.G; jt < jt_end; ++jt) {
        const int sl = (jt - jg * T.G) & 1;
        const int64_t j0 = (int64_t)jt * T.J;
        const int64_t j1 = min(j0 + (int64_t)T.J, T.n_out);
        __syncthreads();  // the tile's range is in slot sl; every wave is done with the previous tile
        const int64_t tlo = sh_rng[2 * sl];
        const int64_t thi = sh_rng[2 * sl + 1];
        const int len = (int)(thi - tlo);
        const int nj = (int)(j1 - j0);
        const bool fits = (thi - tlo) <= cap && (RECT || nj <= jmax);
        const int a_len = RECT ? len + 1 : len;  // prefix arrays need the entry at hi
        if (RECT && fits && RS == 2) {
            for (int i = tid; i < len + 8; i += kThreads) {
                double* r = g_win_lds + 2 * i;
                r[0] = i < len ? gt[tlo + i] : kInf;
                r[1] = i <= len ? ga1[tlo + i] + prefix_off(gpo, tlo + i, 0) : 0.0;
            }
        } else if (RECT && fits) {
            for (int i = tid; i < len + 8; i += kThreads) {
                double* r = g_win_lds + i;
                r[0] = i < len ? gt[tlo + i] : kInf;
                if (NUMER) r[dp] = i <= len ? ga1[tlo + i] + prefix_off(gpo, tlo + i, 0) : 0.0;
                if (WTD) {
                    r[QW * dp] = i <= len ? ga2[tlo + i] + prefix_off(gpo, tlo + i, 1) : 0.0;
                    r[(QW + 1) * dp] =
                        i <= len ? ga3[tlo + i] + prefix_off(gpo, tlo + i, 2) : 0.0;
                }
            }
        } else if (fits) {
            for (int i = tid; i < len + 8; i += kThreads)
                g_win_lds[o_t + i] = i < len ? gt[tlo + i] : kInf;
            if (HAS_A1)
                for (int i = tid; i < a_len; i += kThreads) g_win_lds[o_a1 + i] = ga1[tlo + i];
            if (HAS_A2)
                for (int i = tid; i < a_len; i += kThreads) g_win_lds[o_a2 + i] = ga2[tlo + i];
            for (int i = tid; i < nj; i += kThreads) {
                g_win_lds[o_s + i] = gs[j0 + i];
                if (NUMER) g_win_lds[o_vo + i] = gvo[j0 + i];
                if (WTD) g_win_lds[o_wo + i] = gwo[j0 + i];
            }
        }
        __syncthreads();
        // the next tile's range, searched while this one is scanned (its
        // slot was last read before the barrier above)
        if (jt + 1 < jt_end) search_tile(jt + 1, sl ^ 1);

        const int ja = (int)((int64_t)nj * seg / nseg);
        const int jb = (int)((int64_t)nj * (seg + 1) / nseg);
        if (RECT && fits) {
            AccR ar = {0.0, 0.0, 0.0, 0};
            if (streams == 1) {  // one outer run per wave
                if (active)
                    scan_rect_wave<NUMER, WTD, RS>(ar, g_win_lds, dp, len, ja, jb, delta, W,
                                               T.s + j0, NUMER ? T.vo + j0 : nullptr,
                                               WTD ? T.wo + j0 : nullptr);
            } else if (active) {
                scan_rect_lane<NUMER, WTD, RS>(ar, g_win_lds, dp, len, ja, jb, delta, W, gs + j0,
                                           NUMER ? gvo + j0 : nullptr,
                                           WTD ? gwo + j0 : nullptr);
            }
            acc.C += ar.C;
            acc.B += ar.B;
            acc.b += ar.nz;
            acc.n += ar.bytes / (int)(RS * sizeof(double));
        } else if (active) {
            if (fits) {
                LdsView v{o_t, o_a1, o_a2, o_s, o_vo, o_wo, len};
                scan_lane<F>(acc, v, ja, jb, delta, W, inv_h);
            } else {
                const GlbView g{(gdp)(T.t + tlo),
                                HAS_A1 ? (gdp)(A1g + tlo) : nullptr,
                                HAS_A2 ? (gdp)(A2g + tlo) : nullptr,
                                (RECT && WTD) ? (gdp)(T.pz + tlo) : nullptr,
                                (gdp)(T.s + j0),
                                NUMER ? (gdp)(T.vo + j0) : nullptr,
                                WTD ? (gdp)(T.wo + j0) : nullptr,
                                len};
                if constexpr (RECT) {  // chunk-local prefix sums: offsets on read
                    const GlbPrefixView v{g, gpo, tlo};
                    scan_lane<F>(acc, v, ja, jb, delta, W, inv_h);
                } else {
                    scan_lane<F>(acc, g, ja, jb, delta, W, inv_h);
                }
            }
        }
    }
    __syncthreads();  // staging area is reused for the reduction
    double* Red = g_win_lds;
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
        double* out = T.part + ((int64_t)jg * T.K + k0 + tid) * 4;
        out[0] = C;
        out[1] = B;
        out[2] = b;
        out[3] = __longlong_as_double(n);
    }
}

// Work items (series x j-group x lag-tile) of a whole batch in one launch.
// Flat dispatch: workgroup b runs item xcd_remap(b) (the hardware hands
// workgroups out in order, round robin over the XCDs). Queue dispatch: a grid of resident workgroups pulls items from
// a device counter until the items run out; the last workgroup to leave
// resets the counter pair for the next launch (no memset, so a captured
// graph can replay it). Every item writes its own partial sums, so results
// do not depend on which workgroup ran it.
template <uint32_t F>
__device__ __forceinline__ void window_dispatch(const WinTask* __restrict__ tasks,
                                                const int64_t* __restrict__ item0, int ntasks,
                                                int64_t nitems, int cap, int jmax,
                                                unsigned long long* __restrict__ queue) {
    if (!queue) {
        // XCD-aware order: each XCD takes a contiguous run of items, so the
        // lag tiles of one j-group (consecutive items, the same window
        // samples) meet in one L2
        const int64_t item = xcd_remap(blockIdx.x, gridDim.x);
        if (item < nitems) window_item<F>(tasks, item0, ntasks, item, cap, jmax);
        return;
    }
    __shared__ int64_t sh_item;
    for (;;) {
        if (threadIdx.x == 0) sh_item = (int64_t)atomicAdd(queue, 1ull);
        __syncthreads();
        const int64_t item = sh_item;
        __syncthreads();  // every thread has the item before the next pull
        if (item >= nitems) break;
        window_item<F>(tasks, item0, ntasks, item, cap, jmax);
    }
    if (threadIdx.x == 0) {
        const unsigned long long done = atomicAdd(queue + 1, 1ull);
        if (done == (unsigned long long)gridDim.x - 1) {  // all workgroups have left
            atomicExch(queue, 0ull);
            atomicExch(queue + 1, 0ull);
        }
    }
}

template <uint32_t F>
__global__ void __launch_bounds__(kThreads)
k_window(const WinTask* __restrict__ tasks, const int64_t* __restrict__ item0, int ntasks,
         int64_t nitems, int cap, int jmax, unsigned long long* __restrict__ queue) {
    window_dispatch<F>(tasks, item0, ntasks, nitems, cap, jmax, queue);
}

// The unweighted rectangle scans, register-allocated for eight waves per
// SIMD (scalar registers partly spilled to vector lanes): their wait on each
// dependent LDS read is covered by more waves (c5 window_rect 25.1 ->
// 22.8 ms). The weighted ones would spill vector registers to memory.
template <uint32_t F>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(8, 8)))
k_window_rect8(const WinTask* __restrict__ tasks, const int64_t* __restrict__ item0,
               int ntasks, int64_t nitems, int cap, int jmax,
               unsigned long long* __restrict__ queue) {
    window_dispatch<F>(tasks, item0, ntasks, nitems, cap, jmax, queue);
}

// the kernel that runs window flags F
template <uint32_t F>
constexpr auto window_kernel() {
    if constexpr (F == WIN_RECT || F == (WIN_RECT | WIN_NUMER))
        return k_window_rect8<F>;
    else
        return k_window<F>;
}

// Level 1: sum the partials of up to kJc consecutive j-tiles for 64 lags
// (one lane per lag, four waves over interleaved j-tiles, combined in a fixed
// order) into part2[chunk][k].
constexpr int kJc = 64;

__global__ void __launch_bounds__(kThreads)
k_window_reduce1(const WinTask* __restrict__ tasks, const int64_t* __restrict__ r0s, int ntasks,
                 int64_t nitems) {
    __shared__ double red[4][64][4];
    const int64_t item = blockIdx.x;
    if (item >= nitems) return;
    const int ti = (int)wave_search<int64_t>(r0s, ntasks, item, true) - 1;
    const WinTask& T = tasks[ti];
    const int64_t local = item - r0s[ti];
    const int n_jc = (T.n_jg + kJc - 1) / kJc;
    const int kt = (int)(local / n_jc);
    const int jc = (int)(local % n_jc);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int k = kt * 64 + lane;
    double C = 0.0, B = 0.0, b = 0.0;
    long long n = 0;
    if (k < T.K) {
        const int jt_end = min(T.n_jg, (jc + 1) * kJc);
        for (int jt = jc * kJc + wave; jt < jt_end; jt += 4) {
            const double* p = T.part + ((int64_t)jt * T.K + k) * 4;
            C += p[0];
            B += p[1];
            b += p[2];
            n += __double_as_longlong(p[3]);
        }
    }
    red[wave][lane][0] = C;
    red[wave][lane][1] = B;
    red[wave][lane][2] = b;
    red[wave][lane][3] = __longlong_as_double(n);
    __syncthreads();
    if (wave == 0 && k < T.K) {
        for (int w = 1; w < 4; ++w) {
            C += red[w][lane][0];
            B += red[w][lane][1];
            b += red[w][lane][2];
            n += __double_as_longlong(red[w][lane][3]);
        }
        double* o = T.part2 + ((int64_t)jc * T.K + k) * 4;
        o[0] = C;
        o[1] = B;
        o[2] = b;
        o[3] = __longlong_as_double(n);
    }
}

// Level 2: sum the chunk partials in order; scale the Gaussian weights by
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
    const int n_jc = (T.n_jg + kJc - 1) / kJc;
    double C = 0.0, B = 0.0, b = 0.0;
    long long n = 0;
    for (int jc = 0; jc < n_jc; ++jc) {
        const double* p = T.part2 + ((int64_t)jc * T.K + k) * 4;
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
    } else if (!(flags & WIN_WEIGHTED)) {
        b = (double)n;  // weighted: b holds the pairs of two nonzero weights
    }
    double* out = T.sums + (int64_t)k * 4;
    out[0] = C;
    out[1] = B;
    out[2] = b;
    out[3] = __longlong_as_double(n);
}

// Resident workgroups of a window kernel instance with `bytes` of LDS on the
// current device (cached: the first eager launch fills it, later launches,
// also under graph capture, only read it).
template <uint32_t F>
int resident_blocks(size_t bytes, int64_t* out) {
    static std::mutex mu;
    static std::map<std::pair<int, size_t>, int64_t> cache;
    int dev = 0;
    NCF_TRY_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    auto key = std::make_pair(dev, bytes);
    auto it = cache.find(key);
    if (it == cache.end()) {
        int per_cu = 0, cus = 0;
        NCF_TRY_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, window_kernel<F>(), kThreads,
                                                                 bytes));
        NCF_TRY_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        it = cache.emplace(key, (int64_t)std::max(per_cu, 1) * std::max(cus, 1)).first;
    }
    *out = it->second;
    return NCF_OK;
}

template <uint32_t F>
int launch_window_t(const WinTask* d_tasks, const int64_t* d_item0, int ntasks, int64_t nitems,
                    int cap, int jmax, unsigned long long* queue, hipStream_t st, double work) {
    constexpr bool RECT = (F & WIN_RECT) != 0;
    constexpr bool NUMER = (F & WIN_NUMER) != 0;
    constexpr bool WTD = (F & WIN_WEIGHTED) != 0;
    size_t stage = (size_t)(cap + 8) * (1 + (NUMER ? 1 : 0) + (WTD ? (RECT ? 2 : 1) : 0)) +
                   (RECT ? 0 : (size_t)(jmax + 2) * (1 + (NUMER ? 1 : 0) + (WTD ? 1 : 0)));
    size_t red = 4 * kThreads;
    size_t bytes = (stage > red ? stage : red) * sizeof(double);
    (void)RECT;
    int64_t nblocks = round_up(nitems, kXcds);
    if (queue) {
        int64_t res = 0;
        NCF_TRY(resident_blocks<F>(bytes, &res));
        nblocks = std::min(nitems, res);
    }
    ProfScope p(st, RECT ? "window_rect" : "window_gauss", work, "valu_ops");
    hipLaunchKernelGGL(window_kernel<F>(), dim3((unsigned)nblocks), dim3(kThreads), bytes, st, d_tasks,
                       d_item0, ntasks, nitems, cap, jmax, queue);
    NCF_CHECK_LAUNCH();
    return NCF_OK;
}

}  // namespace

int launch_window(const WinTask* d_tasks, const int64_t* d_item0, int ntasks, int64_t nitems,
                  uint32_t flags, int cap, int jmax, unsigned long long* queue, hipStream_t st,
                  double work) {
    if (nitems <= 0) return NCF_OK;
    switch (flags) {
#define NCF_WIN_CASE(f) \
    case (f):           \
        return launch_window_t<(f)>(d_tasks, d_item0, ntasks, nitems, cap, jmax, queue, st, work);
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
                         const int64_t* d_r0, int64_t nred1, uint32_t flags, hipStream_t st) {
    if (total_k <= 0) return NCF_OK;
    ProfScope p(st, "window_reduce", 0.0, "bytes");
    if (nred1 > 0) {
        hipLaunchKernelGGL(k_window_reduce1, dim3((unsigned)nred1), dim3(kThreads), 0, st,
                           d_tasks, d_r0, ntasks, nred1);
        NCF_CHECK_LAUNCH();
    }
    hipLaunchKernelGGL(k_window_reduce, dim3((unsigned)ceil_div(total_k, 128)), dim3(128), 0, st,
                       d_tasks, ntasks, d_k0, total_k, flags);
    NCF_CHECK_LAUNCH();
    return NCF_OK;
}

}  // namespace ncf
