// spectral.hip -- Wiener-Khinchin route for the Gaussian numerator (A2-A6).
//
// The numerator of eq. kernel_estimator with the Gaussian kernel is
//   N(tau) = sum_ij v_i v'_j phi_h(s_j - t_i - tau)
//          = (1/L) sum_m phihat(m/L) conj(X_m) Y_m exp(-2 pi i m tau / L)
// on a period L long enough that the periodic images of phi_h do not reach
// the data (Poisson summation), with X_m = sum_i v_i exp(+2 pi i m t_i / L)
// the type-1 transform of eq. nufft_type1 and phihat(f) = exp(-2 pi^2 h^2 f^2)
// the Fourier transform of eq. Gaussian_kernel. Sec. 2.6 evaluates the same
// identity with a type-1 NUFFT, a cross-spectrum product and a type-2 NUFFT at
// the lags; here the lag kernel's transform multiplies the cross-spectrum
// directly instead of smoothing along the lag axis afterwards.
//
// Both non-uniform transforms use Gaussian gridding (Sec. 2.5: spread, FFT,
// deconvolve): psi(d) = exp(-d^2 / 2 s^2) on a grid of N cells, truncated at
// |d| <= W cells, whose transform Psi(xi) = sqrt(2 pi) s exp(-2 pi^2 s^2 xi^2)
// is closed form. The product step therefore folds phihat, the forward
// deconvolution 1/Psi^2 and the type-2 pre-correction 1/Psi into one factor
//   exp(-2 pi^2 m^2 (h^2/L^2 - 3 s^2/N^2)) / (L (2 pi)^(3/2) s^3).
//
// Positions are split in FP64 into an integer cell and an FP32 (or FP64)
// fraction before any FP32 arithmetic, so long baselines keep their phase.
// Spreading gathers: each workgroup owns a tile of grid cells, stages the
// samples that can reach it (sorted times -> contiguous index range) in LDS,
// and every thread sums the samples near its own cells. No atomics; one
// coalesced write per cell; deterministic.
#include <algorithm>

#include "fft_tile.h"
#include "internal.h"

namespace ncf {

namespace {

constexpr int kThreads = 256;
constexpr int kCellsPerThread = 16;
constexpr int kTile = kThreads * kCellsPerThread;  // 4096 cells per workgroup
constexpr int kPtsChunk = 1024;  // staged samples per round (a tile holds a few hundred)

template <typename R>
struct Cplx;
template <>
struct Cplx<float> {
    using T = float2;
};
template <>
struct Cplx<double> {
    using T = double2;
};

__device__ __forceinline__ int64_t find_task(const int64_t* starts, int ntasks, int64_t g) {
    int lo = 0, hi = ntasks;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (starts[mid] <= g)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Sample index ranges [p0, p1) that reach each spreading tile, from one
// coalesced pass over the sorted samples instead of a search per tile. With
// u_i the FP64 grid coordinate of sample i, tile g (cells [gT, gT + T)) needs
// the samples with u in [gT - W - 2, gT + T + W + 2) (one cell of slack past
// the truncation radius). A(i) = floor((u_i + W + 2) / T) and
// B(i) = floor((u_i - W - 2) / T) are non-decreasing in i, so
// p0(g) = first i with A(i) >= g and p1(g) = first i with B(i) >= g + 1;
// sample i writes p0 of the tiles g in (A(i-1), A(i)] and p1 of those with
// g + 1 in (B(i-1), B(i)]. Every bound is written exactly once.
// Tiles reached by a sample at grid coordinate u: A = floor((u + W + 2) / T)
// is the last tile whose range starts at or before it, B = floor((u - W - 2)
// / T) the last tile + 1 it closes. One expression for both kernels below.
__device__ __forceinline__ void tile_reach(double u, double reach, int64_t& A, int64_t& B) {
    constexpr double inv_tile = 1.0 / kTile;  // exact: a power of two
    A = (int64_t)floor((u + reach) * inv_tile);
    B = (int64_t)floor((u - reach) * inv_tile);
}

__global__ void __launch_bounds__(kThreads)
k_tile_bounds(const SpecTask* __restrict__ tasks, const Chunk* __restrict__ chunks,
              const int32_t* __restrict__ series_map) {
    // one workgroup per chunk of one series; lanes take consecutive samples
    const Chunk ch = chunks[blockIdx.x];
    const int32_t code = series_map[ch.series];  // 2 * task + set, or -1
    if (code < 0) return;
    const int task = code >> 1;
    const SpecTask& T = tasks[task];
    const int set = code & 1;
    const gptr<const double> t = gbl(set ? T.t1 : T.t0);
    const int64_t n = set ? T.n1 : T.n0;
    const double sc = (double)T.N / T.L;
    const double reach = T.W + 2.0;
    const int64_t nt = T.ntiles;
    const gptr<int64_t> rec = gbl(T.tile_rng);  // [tile][kTileRec]
    const int lane = threadIdx.x & 63;
    // kUnroll rows of the chunk per round: their loads are issued together
    constexpr int kUnroll = 4;
    for (int64_t b = ch.begin; b < ch.end; b += kThreads * kUnroll) {
        double tv[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t i = b + u * kThreads + threadIdx.x;
            tv[u] = i < ch.end ? t[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t i = b + u * kThreads + threadIdx.x;
            const bool live = i < ch.end;
            int64_t a1 = 0, b1 = 0;
            if (live) tile_reach((tv[u] - T.t_ref) * sc, reach, a1, b1);
            // the previous sample's A, B from the neighbouring lane (same
            // chunk, consecutive samples), recomputed by the first lane of
            // each wave
            int64_t a0 = __shfl_up(a1, 1), b0 = __shfl_up(b1, 1);
            if (!live) continue;
            if (i == 0) {
                a0 = -1;
                b0 = -1;
            } else if (lane == 0) {
                tile_reach((t[i - 1] - T.t_ref) * sc, reach, a0, b0);
            }
            for (int64_t q = max(a0 + 1, (int64_t)0); q <= min(a1, nt - 1); ++q) {
                rec[kTileRec * q + 2 * set] = i;
                if (set == 0) rec[kTileRec * q + 4] = task;
            }
            for (int64_t q = max(b0, (int64_t)0); q <= min(b1 - 1, nt - 1); ++q)
                rec[kTileRec * q + 2 * set + 1] = i;
        }
    }
    // tiles past the last sample's reach: bound n, filled by the workgroup
    // that holds the last sample, all threads together
    if (ch.end == n) {
        int64_t A, B;
        tile_reach((t[n - 1] - T.t_ref) * sc, reach, A, B);
        for (int64_t q = max(A + 1, (int64_t)0) + threadIdx.x; q < nt; q += kThreads) {
            rec[kTileRec * q + 2 * set] = n;
            if (set == 0) rec[kTileRec * q + 4] = task;
        }
        for (int64_t q = max(B, (int64_t)0) + threadIdx.x; q < nt; q += kThreads)
            rec[kTileRec * q + 2 * set + 1] = n;
    }
}

// LDS of a spreading workgroup: the staged samples, later reused to stage
// half of the tile's cells for the coalesced write (one pad slot per 16).
template <typename R>
struct PtsLds {
    union {
        struct {
            int cell[kPtsChunk];  // cell index relative to the tile start
            R frac[kPtsChunk];    // fraction in [0, 1)
            R val[kPtsChunk];
            R wgt[kPtsChunk];     // sample weights (weighted pair-count channel)
        };
        typename Cplx<R>::T out[kTile / 2 + kTile / 32];
    };
};

// Accumulate one point set into the thread's 16 cells. UNIT: also the
// pair-count channel, with unit weights or (WGT) the sample weights wd;
// UNW (with WGT): a third channel with unit weights.
template <typename R, bool UNIT, bool WGT, bool UNW>
__device__ void gather_set(R (&acc)[kCellsPerThread], R (&accu)[kCellsPerThread],
                           R (&accn)[kCellsPerThread], PtsLds<R>& P, const double* t,
                           const float* vf, const double* vd, const double* wd, int64_t p0,
                           int64_t p1, int64_t c0, double t_ref, double scale, R W, R k2) {
    const int tid = threadIdx.x;
    const int cb = tid * kCellsPerThread;  // first own cell, relative to tile
    for (int64_t base = p0; base < p1; base += kPtsChunk) {
        const int np = (int)min((int64_t)kPtsChunk, p1 - base);
        __syncthreads();
        const gptr<const double> tg = gbl(t);
        for (int i = tid; i < np; i += kThreads) {
            const double u = (tg[base + i] - t_ref) * scale;  // FP64 grid coordinate
            const double cf = floor(u);
            P.cell[i] = (int)((int64_t)cf - c0);
            P.frac[i] = (R)(u - cf);
            P.val[i] = vd ? (R)gbl(vd)[base + i] : (R)gbl(vf)[base + i];
            if (WGT) P.wgt[i] = wd ? (R)gbl(wd)[base + i] : (R)1;
        }
        __syncthreads();
        // first staged point whose cell can reach cell cb: cell >= cb - W - 1
        const int need_lo = cb - (int)W - 2;
        const int need_hi = cb + kCellsPerThread + (int)W + 1;
        int lo = 0, hi = np;
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (P.cell[mid] < need_lo)
                lo = mid + 1;
            else
                hi = mid;
        }
        const R W2 = W * W;
        for (int i = lo; i < np; ++i) {
            const int ci = P.cell[i];
            if (ci > need_hi) break;
            const R fr = P.frac[i];
            const R vv = P.val[i];
            const R ww = WGT ? P.wgt[i] : (R)1;
            // offset of the point from the thread's first cell, as an exact
            // integer in R; cell q is at d = (m0 - q) + fr (m0 - q exact)
            const R m0 = (R)(ci - cb);
#pragma unroll
            for (int q = 0; q < kCellsPerThread; ++q) {
                const R d = (m0 - (R)q) + fr;
                const R d2 = d * d;
                R e;
                if constexpr (sizeof(R) == 4)
                    e = __builtin_amdgcn_exp2f(d2 * k2);
                else
                    e = exp(d2 * k2);
                e = d2 <= W2 ? e : (R)0;  // the kernel's support |d| <= W
                acc[q] += e * vv;
                if (UNIT) accu[q] += WGT ? e * ww : e;  // pair-count channel
                if (UNW) accn[q] += e;                  // unweighted pair count
            }
        }
    }
}

// MODE: bit 1 CCF (two point sets), bit 0 pair-count channel, bit 2 sample
// weights in that channel, bit 3 (with bits 0 and 2) one more channel with
// unit weights for the unweighted pair count; fixed per launch, so
// accumulators that a mode does not use cost no registers.
//   ACF: grid = values + i (weights or units); bit 3: gridb = units
//   CCF: grid = x values + i y values; gridb = pair-count channels of x and
//        y; bit 3: gridc = unit channels of x and y
template <typename R, int MODE>
__global__ void __launch_bounds__(kThreads)
k_spread(const SpecTask* __restrict__ tasks, const int64_t* __restrict__ tile0, int ntasks,
         int64_t ntiles, int64_t nblocks, const int64_t* __restrict__ tile_rec) {
    using C2 = typename Cplx<R>::T;
    constexpr bool CCF = (MODE & 2) != 0;
    constexpr bool WB = (MODE & 1) != 0;
    constexpr bool WGT = WB && (MODE & 4) != 0;
    constexpr bool UNW = WGT && (MODE & 8) != 0;
    // grids written: grid, gridb (CCF pair channels or ACF units), gridc
    constexpr int ngrids = CCF ? 1 + (WB ? 1 : 0) + (UNW ? 1 : 0) : 1 + (UNW ? 1 : 0);
    __shared__ PtsLds<R> P;
    const int64_t g = blockIdx.x;
    (void)nblocks;
    if (g >= ntiles) return;
    // task of this tile: from its bounds record (bounds pass), else by search
    int ti;
    int64_t rec[kTileRec];
    const bool have_rec = tile_rec != nullptr;
    if (have_rec) {
        const gptr<const int64_t> r = gbl(tile_rec) + kTileRec * g;
#pragma unroll
        for (int q = 0; q < 5; ++q) rec[q] = r[q];
        // one task: its descriptor loads need not wait for the record
        ti = ntasks == 1 ? 0 : (int)rec[4];
    } else {
        ti = ntasks == 1 ? 0 : (int)wave_search<int64_t>(tile0, ntasks, g, true) - 1;
    }
    const SpecTask& T = tasks[ti];
    const int64_t tile = g - T.tile0;
    const int64_t c0 = tile * kTile;
    // sample index ranges that reach this tile: from the bounds record, or
    // for calls with few tiles by wave searches in this workgroup
    __shared__ int64_t srng[4];
    int64_t rng[4];
    if (!have_rec) {
        const int wave = threadIdx.x >> 6;
        const double inv_scale = T.L / (double)T.N;  // time per cell
        const double lo_t = T.t_ref + ((double)c0 - T.W - 2.0) * inv_scale;
        const double hi_t = T.t_ref + ((double)c0 + kTile + T.W + 2.0) * inv_scale;
        int64_t r = 0;
        if (wave == 0) r = wave_search<double>(T.t0, T.n0, lo_t, false);
        if (wave == 1) r = wave_search<double>(T.t0, T.n0, hi_t, false);
        if (wave == 2) r = T.ccf ? wave_search<double>(T.t1, T.n1, lo_t, false) : 0;
        if (wave == 3) r = T.ccf ? wave_search<double>(T.t1, T.n1, hi_t, false) : 0;
        if ((threadIdx.x & 63) == 0) srng[wave] = r;
        __syncthreads();
        for (int q = 0; q < 4; ++q) rng[q] = srng[q];
    } else {
        rng[0] = rec[0];
        rng[1] = rec[1];
        rng[2] = CCF ? rec[2] : 0;
        rng[3] = CCF ? rec[3] : 0;
    }
    // a tile no sample reaches (lag padding, seasonal gaps): coalesced zeros,
    // no staging
    if (rng[0] >= rng[1] && rng[2] >= rng[3]) {
        for (int gsel = 0; gsel < ngrids; ++gsel) {
            void* gp = gsel == 0 ? T.grid : gsel == 1 ? T.gridb : T.gridc;
            const gptr<R> grid = gbl(reinterpret_cast<R*>(gp) + 2 * c0);
            for (int i = threadIdx.x; i < 2 * kTile; i += kThreads) grid[i] = (R)0;
        }
        return;
    }
    const double scale = (double)T.N / T.L;
    const R W = (R)T.W;
    // exp(-d^2 / 2 s^2): FP32 uses exp2 with log2(e) folded in
    const R k2 = sizeof(R) == 4 ? (R)(-0.72134752044448170 / (T.s * T.s))
                                : (R)(-0.5 / (T.s * T.s));
    R re[kCellsPerThread], im[kCellsPerThread], u0[kCellsPerThread], u1[kCellsPerThread];
    R n0[kCellsPerThread], n1[kCellsPerThread];
#pragma unroll
    for (int q = 0; q < kCellsPerThread; ++q) re[q] = im[q] = u0[q] = u1[q] = n0[q] = n1[q] = (R)0;
    if constexpr (!CCF) {
        // ACF: values in the real channel, pair-count weights (with_b) in the
        // imaginary one, units in n0 (UNW)
        gather_set<R, WB, WGT, UNW>(re, im, n0, P, T.t0, T.v0f, T.v0d, T.w0, rng[0], rng[1], c0,
                                    T.t_ref, scale, W, k2);
    } else if constexpr (WB) {
        // CCF: grid = series 1 values + i series 2 values; gridb = the same
        // with the pair-count weights; gridc = units (UNW)
        gather_set<R, true, WGT, UNW>(re, u0, n0, P, T.t0, T.v0f, T.v0d, T.w0, rng[0], rng[1],
                                      c0, T.t_ref, scale, W, k2);
        gather_set<R, true, WGT, UNW>(im, u1, n1, P, T.t1, T.v1f, T.v1d, T.w1, rng[2], rng[3],
                                      c0, T.t_ref, scale, W, k2);
    } else {
        gather_set<R, false, false, false>(re, u0, n0, P, T.t0, T.v0f, T.v0d, nullptr, rng[0],
                                           rng[1], c0, T.t_ref, scale, W, k2);
        gather_set<R, false, false, false>(im, u1, n1, P, T.t1, T.v1f, T.v1d, nullptr, rng[2],
                                           rng[3], c0, T.t_ref, scale, W, k2);
    }
    // stage the tile through LDS for a coalesced write (two halves, so the
    // staging fits the point buffer); one pad slot per 16 cells keeps the
    // threads' 16-cell runs on different banks
    static_assert(sizeof(PtsLds<R>) >= sizeof(C2) * (kTile / 2 + kTile / 32),
                  "LDS staging too small");
    C2* out = P.out;
    for (int gsel = 0; gsel < ngrids; ++gsel) {
        void* gp = gsel == 0 ? T.grid : gsel == 1 ? T.gridb : T.gridc;
        const gptr<R> grid = gbl(reinterpret_cast<R*>(gp) + 2 * c0);
        for (int half = 0; half < 2; ++half) {
            __syncthreads();
            const int hbase = half * (kTile / 2);
            const int tb = threadIdx.x * kCellsPerThread - hbase;
            if (tb >= 0 && tb < kTile / 2) {
#pragma unroll
                for (int q = 0; q < kCellsPerThread; ++q) {
                    C2 v;
                    if (gsel == 0) {
                        v.x = re[q];
                        v.y = im[q];
                    } else if (CCF && gsel == 1) {
                        v.x = u0[q];
                        v.y = u1[q];
                    } else {  // units: ACF gridb, CCF gridc
                        v.x = n0[q];
                        v.y = CCF ? n1[q] : (R)0;
                    }
                    out[tb + q + (tb >> 4)] = v;
                }
            }
            __syncthreads();
            for (int i = threadIdx.x; i < kTile / 2; i += kThreads) {
                const C2 v = out[i + (i >> 4)];
                grid[2 * (hbase + i)] = v.x;
                grid[2 * (hbase + i) + 1] = v.y;
            }
        }
    }
}

// ---------------------------------------------------------------- product


template <typename R>
__device__ __forceinline__ double lag_kernel_ft(int kern, double f, double h) {
    if (kern == NCF_GAUSSIAN) return exp(-2.0 * M_PI * M_PI * h * h * f * f);
    // box of half-width h: integral_{-h}^{h} exp(2 pi i f d) dd = sin(2 pi h f) / (pi f)
    if (f == 0.0) return 2.0 * h;
    return sinpi(2.0 * h * f) / (M_PI * f);
}

// complex element i of a global-memory grid of R pairs
template <typename C2, typename R>
__device__ __forceinline__ C2 cld(gptr<R> g, int64_t i) {
    C2 v;
    v.x = g[2 * i];
    v.y = g[2 * i + 1];
    return v;
}
template <typename C2, typename R>
__device__ __forceinline__ void cst(gptr<R> g, int64_t i, C2 v) {
    g[2 * i] = v.x;
    g[2 * i + 1] = v.y;
}

template <typename R>
struct ProductCtx {
    gptr<R> Z;
    gptr<R> U;
    gptr<R> C;  // unit channel of a weighted CCF (gridc)
    int64_t N, M;
    double L, h, s;
    int32_t kern;
    // per-mode factors f3 = phihat(m/L) / (L Psi^3) and f2 = phihat(m/L) /
    // (L Psi^2) with Psi(m/N) = sqrt(2 pi) s exp(-2 pi^2 s^2 m^2 / N^2):
    double c3, c2;  // 1 / (L (2 pi)^(3/2) s^3), 1 / (L 2 pi s^2)
    double psi;     // 2 pi^2 s^2 / N^2, the exponent of 1/Psi per m^2
    double e3, e2;  // Gaussian lag kernel: exponents of f3, f2 per m^2
                    // (base 2 for FP32 grids, base e for FP64 grids)
};

template <typename R>
__device__ __forceinline__ ProductCtx<R> product_ctx(gptr<R> Z, gptr<R> U, gptr<R> C,
                                                     const SpecTask& T) {
    ProductCtx<R> X{Z, U, C, T.N, T.M, T.L, T.h, T.s, T.kern, 0.0, 0.0, 0.0, 0.0, 0.0};
    const double s = T.s, L = T.L, Nd = (double)T.N, h = T.h;
    X.c3 = 1.0 / (L * 15.749609945722419 * s * s * s);
    X.c2 = 1.0 / (L * 6.283185307179586 * s * s);
    X.psi = 2.0 * M_PI * M_PI * s * s / (Nd * Nd);
    const double ker = 2.0 * M_PI * M_PI * h * h / (L * L);  // of phihat per m^2
    const double base = sizeof(R) == 4 ? 1.4426950408889634 : 1.0;
    X.e3 = (3.0 * X.psi - ker) * base;
    X.e2 = (2.0 * X.psi - ker) * base;
    return X;
}

// 2^y to ~1 FP32 ulp for any y in range: y is split in FP64 into an integer
// part (applied exactly) and a fraction in [0, 1) for the FP32 exp2.
__device__ __forceinline__ double exp2_split(double y) {
    const double n = floor(y);
    return ldexp((double)__builtin_amdgcn_exp2f((float)(y - n)), (int)n);
}

// The factors at signed mode m (|m| <= N/2); both zero beyond the retained
// modes.
// f3 is the factor of the evaluated spectrum: phihat / (L Psi^3) when the
// lags are read by interpolation (one more Psi for the interpolating
// kernel), phihat / (L Psi^2) = f2 when they are read off a lag lattice
// (`fold`: no interpolation).
template <typename R, bool CCF>
__device__ __forceinline__ void product_factors_m(const ProductCtx<R>& X, int64_t m, double& f3,
                                                  double& f2, bool fold = false) {
    f3 = 0.0;
    f2 = 0.0;
    if (m > X.M || m < -X.M) return;
    const double md = (double)m;
    const double m2 = md * md;
    if (X.kern == NCF_GAUSSIAN) {
        if (sizeof(R) == 4) {
            if (fold || CCF) f2 = X.c2 * exp2_split(X.e2 * m2);
            f3 = fold ? f2 : X.c3 * exp2_split(X.e3 * m2);
        } else {
            if (fold || CCF) f2 = X.c2 * exp(X.e2 * m2);
            f3 = fold ? f2 : X.c3 * exp(X.e3 * m2);
        }
    } else {
        const double ker = lag_kernel_ft<R>(X.kern, md / X.L, X.h);
        if (fold || CCF) f2 = X.c2 * ker * exp(2.0 * X.psi * m2);
        f3 = fold ? f2 : X.c3 * ker * exp(3.0 * X.psi * m2);
    }
}

// The factors at the frequency of digit-reversed position p.
template <typename R, bool CCF>
__device__ __forceinline__ void product_factors(const ProductCtx<R>& X, const RadixInfo& ri,
                                                int64_t p, double& f3, double& f2) {
    const int64_t k = freq_of_pos(p, ri);
    product_factors_m<R, CCF>(X, k <= X.N / 2 ? k : k - X.N, f3, f2);
}

template <typename R, bool CCF, bool WB>
__device__ __forceinline__ void product_math(const ProductCtx<R>& X, const RadixInfo& ri,
                                             int64_t p, int64_t pp, typename Cplx<R>::T a,
                                             typename Cplx<R>::T b, typename Cplx<R>::T va,
                                             typename Cplx<R>::T vb, double (&sacc)[4],
                                             typename Cplx<R>::T& o, typename Cplx<R>::T& oc) {
    double f3, f2;
    product_factors<R, CCF>(X, ri, p, f3, f2);
    if (!CCF && !WB) {  // each position on its own: f3 |Z|^2 (oc unused)
        const double pw = (double)a.x * a.x + (double)a.y * a.y;
        o.x = (R)(f3 * pw);
        o.y = (R)0;
        oc = o;
        return;
    }
    // the two real sequences packed in Z: A = (Z_m + conj Z_-m)/2,
    // B = (Z_m - conj Z_-m)/(2i)
    const double ar = 0.5 * ((double)a.x + b.x), ai = 0.5 * ((double)a.y - b.y);
    const double br = 0.5 * ((double)a.y + b.y), bi = -0.5 * ((double)a.x - b.x);
    const double mult = (pp != p) ? 2.0 : 1.0;
    if (!CCF) {
        // ACF with b: A = X (values), B = W (unit weights); G_N = |X|^2, G_B = |W|^2
        const double gn = ar * ar + ai * ai, gbb = br * br + bi * bi;
        o.x = (R)(f3 * gn);
        o.y = (R)(f3 * gbb);
        oc = o;
    } else {
        // CCF: G_N = conj(X) Y
        const double gr = ar * br + ai * bi;
        const double gi = ar * bi - ai * br;
        sacc[0] += mult * f2 * (ar * ar + ai * ai);
        sacc[1] += mult * f2 * (br * br + bi * bi);
        if (!WB) {
            o.x = (R)(f3 * gr);
            o.y = (R)(f3 * gi);
            oc.x = o.x;
            oc.y = -o.y;
        } else {
            // unit-weight grid: G_B = conj(U_x) U_y
            const double xr = 0.5 * ((double)va.x + vb.x), xi = 0.5 * ((double)va.y - vb.y);
            const double yr = 0.5 * ((double)va.y + vb.y), yi = -0.5 * ((double)va.x - vb.x);
            const double hr = xr * yr + xi * yi;
            const double hi = xr * yi - xi * yr;
            sacc[2] += mult * f2 * (xr * xr + xi * xi);
            sacc[3] += mult * f2 * (yr * yr + yi * yi);
            // G_N + i G_B at m, conj(G_N) + i conj(G_B) at -m
            o.x = (R)(f3 * (gr - hi));
            o.y = (R)(f3 * (gi + hr));
            oc.x = (R)(f3 * (gr + hi));
            oc.y = (R)(f3 * (hr - gi));
        }
    }
}

template <typename R, bool CCF, bool WB>
__device__ __forceinline__ void product_item(const ProductCtx<R>& X, const RadixInfo& ri,
                                             int64_t p, int64_t pp, typename Cplx<R>::T a,
                                             typename Cplx<R>::T b, typename Cplx<R>::T va,
                                             typename Cplx<R>::T vb, double (&sacc)[4]) {
    typename Cplx<R>::T o, oc;
    product_math<R, CCF, WB>(X, ri, p, pp, a, b, va, vb, sacc, o, oc);
    cst(X.Z, p, o);
    if ((CCF || WB) && pp != p) cst(X.Z, pp, oc);
}

// Unweighted pair-count spectrum of a weighted call from its unit channel
// (values c at p and d at pp): ACF gridb = units + i 0, |U|^2; CCF gridc =
// x units + i y units, conj(U_x) U_y. Written to gridb (X.U) as G_b at p
// and conj(G_b) at pp, after the thread's loads of gridb.
template <typename R, bool CCF>
__device__ __forceinline__ void unit_item(const ProductCtx<R>& X, const RadixInfo& ri, int64_t p,
                                          int64_t pp, typename Cplx<R>::T c,
                                          typename Cplx<R>::T d) {
    using C2 = typename Cplx<R>::T;
    double f3, f2;
    product_factors<R, false>(X, ri, p, f3, f2);
    C2 o, oc;
    if (!CCF) {
        const double ur = 0.5 * ((double)c.x + d.x), ui = 0.5 * ((double)c.y - d.y);
        o.x = (R)(f3 * (ur * ur + ui * ui));
        o.y = (R)0;
        oc = o;
    } else {
        const double xr = 0.5 * ((double)c.x + d.x), xi = 0.5 * ((double)c.y - d.y);
        const double yr = 0.5 * ((double)c.y + d.y), yi = -0.5 * ((double)c.x - d.x);
        o.x = (R)(f3 * (xr * yr + xi * yi));
        o.y = (R)(f3 * (xr * yi - xi * yr));
        oc.x = o.x;
        oc.y = -o.y;
    }
    cst(X.U, p, o);
    if (pp != p) cst(X.U, pp, oc);
}

// In-place product on the digit-reversed spectrum. Without the unit-weight
// channel: ACF -> phihat |X|^2 / (L Psi^3); CCF -> phihat conj(X) Y / (L Psi^3)
// after unpacking X, Y from the packed grid. With it (with_b) the same
// factor multiplies the numerator spectrum G_N and the pair-count spectrum
// G_B (from the unit weights), and the grid receives G_N + i G_B: both are
// Hermitian, so the inverse transform returns N(tau) in the real part and
// b(tau) in the imaginary part. CCF blocks also reduce the lag-0 sums
// S_xx, S_yy (and B_xx, B_yy) = sum_m phihat |.|^2 / (L Psi^2).
template <typename R, int MODE>
__global__ void __launch_bounds__(kThreads)
k_product(const SpecTask* __restrict__ tasks, const int64_t* __restrict__ pos0, int ntasks,
          int64_t total, const RadixInfo* __restrict__ rinfo) {
    using C2 = typename Cplx<R>::T;
    __shared__ double red[4][kThreads];
    // a block owns kTile consecutive positions of one grid (N >= kTile)
    const int64_t gb = (int64_t)blockIdx.x * kTile;
    const int ti = ntasks == 1 ? 0 : (int)wave_search<int64_t>(pos0, ntasks, gb, true) - 1;
    const SpecTask& T = tasks[ti];
    const RadixInfo ri = rinfo[ti];
    const int64_t N = T.N;
    const gptr<R> Z = gbl(reinterpret_cast<R*>(T.grid));
    const gptr<R> U = gbl(reinterpret_cast<R*>(T.gridb));
    const gptr<R> Cg = gbl(reinterpret_cast<R*>(T.gridc));
    double sacc[4] = {0.0, 0.0, 0.0, 0.0};
    // Each (m, -m) pair is handled by the thread that owns the position of
    // its frequency k in [0, N/2]. The top bit of k is bit 11 of the position
    // (the last pass has radix 4096), so the owned positions are the first
    // half of every 4096-position tile, plus k = N/2 at position 2048 of
    // tile 0. A thread issues the loads of its positions before any store:
    // pairs are disjoint, so nothing is read after being written.
    constexpr bool CCF = (MODE & 2) != 0;
    constexpr bool WB = (MODE & 1) != 0;
    constexpr bool UNW = WB && (MODE & 4) != 0;  // unweighted pair count of a weighted call
    constexpr bool two = CCF || WB;    // pairs (m, -m) needed
    constexpr bool unit = CCF && WB;   // second (pair-count) grid of a CCF
    const int64_t tb = gb - T.pos0;    // first position of the tile in its grid
    constexpr int kIt = kTile / 2 / kThreads;
    const ProductCtx<R> X = product_ctx<R>(Z, U, Cg, T);
    for (int half = 0; half < (two ? 1 : 2); ++half) {
        int64_t pb[kIt];
        C2 za[kIt], zb[kIt], ua[kIt], ub[kIt], na[kIt], nb[kIt];
        const int64_t p0 = tb + half * (kTile / 2) + threadIdx.x;
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int64_t p = p0 + it * kThreads;
            za[it] = cld<C2>(Z, p);
            if constexpr (two) {
                pb[it] = pos_of_freq((N - freq_of_pos(p, ri)) & (N - 1), ri);
                zb[it] = cld<C2>(Z, pb[it]);
            }
            if constexpr (unit) {
                ua[it] = cld<C2>(U, p);
                ub[it] = cld<C2>(U, pb[it]);
            }
            if constexpr (UNW) {  // unit channel: ACF gridb, CCF gridc
                na[it] = cld<C2>(CCF ? Cg : U, p);
                nb[it] = cld<C2>(CCF ? Cg : U, pb[it]);
            }
        }
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int64_t p = p0 + it * kThreads;
            product_item<R, CCF, WB>(X, ri, p, two ? pb[it] : p, za[it], two ? zb[it] : za[it],
                                     unit ? ua[it] : za[it], unit ? ub[it] : za[it], sacc);
            if constexpr (UNW) unit_item<R, CCF>(X, ri, p, pb[it], na[it], nb[it]);
        }
    }
    if (two && tb == 0 && threadIdx.x == 0) {  // k = N/2, its own partner
        const int64_t p = kTile / 2;
        const int64_t pp = pos_of_freq((N - freq_of_pos(p, ri)) & (N - 1), ri);
        const C2 a = cld<C2>(Z, p), b = cld<C2>(Z, pp);
        const C2 c = unit ? cld<C2>(U, p) : a, d = unit ? cld<C2>(U, pp) : a;
        C2 e = a, f = a;
        if (UNW) {
            e = cld<C2>(CCF ? Cg : U, p);
            f = cld<C2>(CCF ? Cg : U, pp);
        }
        product_item<R, CCF, WB>(X, ri, p, pp, a, b, c, d, sacc);
        if (UNW) unit_item<R, CCF>(X, ri, p, pp, e, f);
    }
    if (CCF) {
#pragma unroll
        for (int q = 0; q < 4; ++q) red[q][threadIdx.x] = sacc[q];
        __syncthreads();
        for (int off = kThreads / 2; off > 0; off >>= 1) {
            if (threadIdx.x < off) {
#pragma unroll
                for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + off];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const int64_t wg = (gb - T.pos0) / kTile;
#pragma unroll
            for (int q = 0; q < 4; ++q) T.scale_part[4 * wg + q] = red[q][0];
        }
    }
}

// --------------------------------------------------------- type-2 at lags

template <typename R>
__global__ void k_interp(const SpecTask* __restrict__ tasks, int ntasks, const int64_t* __restrict__ k0s,
                         int64_t total_k) {
    using C2 = typename Cplx<R>::T;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total_k) return;
    const int ti = (int)find_task(k0s, ntasks, g);
    const SpecTask& T = tasks[ti];
    if (T.P > 0) return;  // lag-lattice task: k_fold_eval
    const int k = (int)(g - k0s[ti]);
    const double tau = T.lags[k];
    const double Nd = (double)T.N;
    double u = tau * (Nd / T.L);
    u -= Nd * floor(u / Nd);  // wrap to [0, N)
    const double cf = floor(u);
    const double fr = u - cf;
    const int64_t cell = (int64_t)cf;
    const C2* G = reinterpret_cast<const C2*>(T.grid);
    const C2* Gb = reinterpret_cast<const C2*>(T.gridb);  // b spectrum (weighted calls)
    const int wi = (int)ceil(T.W);
    const double kk = -0.5 / (T.s * T.s);
    double acc = 0.0, accb = 0.0, accn = 0.0;
    for (int q = -wi - 1; q <= wi + 1; ++q) {
        const double d = fr - (double)q;  // u - (cell + q)
        if (d > T.W || d < -T.W) continue;
        const int64_t c = (cell + q) & (T.N - 1);
        const double wgt = exp(d * d * kk);
        const C2 gv = G[c];
        acc += (double)gv.x * wgt;
        accb += (double)gv.y * wgt;
        if (T.bunw) accn += (double)Gb[c].x * wgt;
    }
    T.numer[k] = acc;
    if (T.with_b) T.bspec[k] = accb;
    if (T.bunw) T.bunw[k] = accn;
}


// Lag-lattice evaluation, the sum over the tiles (after mid_fold): workgroup
// b of task i takes the evaluation lags [64 c, 64 c + 64) and the tiles
// [kFoldTiles q, kFoldTiles (q + 1)) of one chunk q (b - fe0[i] = c nmc + q).
// Lane l of wave w sums, for lag 64 c + l at lattice point n = tau P / L (a
// whole number for a lag on the lattice), the tiles k_low of its quarter of
// the chunk: sum exp(-2 pi i k_low n / P) Y[k_low][n mod P2], the
// exponential by FP64 recurrence in k_low, re-anchored every 64 terms with
// exact integer reduction of k_low n mod P. The quarters are added in a
// fixed order; a task of one chunk writes the result (real part: numerator
// N(tau); imaginary part: pair count), one of several writes the chunk's
// sum for k_fold_sum.
template <typename R>
__global__ void __launch_bounds__(256)
k_fold_eval(const SpecTask* __restrict__ tasks, int ntasks, const int64_t* __restrict__ fe0) {
    using C2 = typename Cplx<R>::T;
    __shared__ double red[2][4][64];
    const int64_t blk = blockIdx.x;
    const int ti = (int)find_task(fe0, ntasks, blk);
    const SpecTask& T = tasks[ti];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t local = blk - fe0[ti];
    const int nmc = T.nmc;
    const int q = (int)(local % nmc);
    const int k = (int)(local / nmc) * kFoldLags + lane;
    const bool live = k < T.K_eval;
    double ax = 0.0, ay = 0.0;
    if (live) {
        const int64_t P = T.P;
        const int64_t P2 = 1LL << T.lgP2;
        const int64_t N1 = T.N >> 12;
        int64_t n = llround(T.lags[k] * ((double)P / T.L)) % P;
        if (n < 0) n += P;
        const int64_t n2 = n & (P2 - 1);
        const int64_t c0 = (int64_t)q * kFoldTiles;
        const int64_t c1 = c0 + kFoldTiles < N1 ? c0 + kFoldTiles : N1;
        const int64_t quarter = (c1 - c0 + 3) / 4;
        const int64_t m0 = c0 + wave * quarter;
        const int64_t m1 = m0 + quarter < c1 ? m0 + quarter : c1;
        const C2* Y = reinterpret_cast<const C2*>(T.ybuf);
        double sr, cr;
        sincospi(-2.0 * (double)n / (double)P, &sr, &cr);  // ratio exp(-2 pi i n / P)
        double tc = 1.0, ts = 0.0;
        for (int64_t m = m0; m < m1; ++m) {
            if (((m - m0) & 63) == 0) {
                const int64_t e = (m * n) % P;  // m n < 2^50 (N <= 2^31)
                sincospi(-2.0 * (double)e / (double)P, &ts, &tc);
            }
            const C2 y = Y[m * P2 + n2];
            ax += tc * (double)y.x - ts * (double)y.y;
            ay += tc * (double)y.y + ts * (double)y.x;
            const double nc = tc * cr - ts * sr;
            ts = tc * sr + ts * cr;
            tc = nc;
        }
    }
    red[0][wave][lane] = ax;
    red[1][wave][lane] = ay;
    __syncthreads();
    if (wave == 0 && live) {
        double x = 0.0, y = 0.0;
        for (int w = 0; w < 4; ++w) {
            x += red[0][w][lane];
            y += red[1][w][lane];
        }
        if (nmc == 1) {
            T.numer[k] = x;
            if (T.with_b) T.bspec[k] = y;
        } else {
            double* o = T.fpart + ((int64_t)q * T.K_eval + k) * 2;
            o[0] = x;
            o[1] = y;
        }
    }
}

// The chunk sums of the tasks with several chunks, in chunk order; one
// thread per task and evaluation lag.
__global__ void k_fold_sum(const SpecTask* __restrict__ tasks, int ntasks,
                           const int64_t* __restrict__ k0s, int64_t total_k) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total_k) return;
    const int ti = (int)find_task(k0s, ntasks, g);
    const SpecTask& T = tasks[ti];
    if (T.P <= 0 || T.nmc <= 1) return;
    const int k = (int)(g - k0s[ti]);
    double x = 0.0, y = 0.0;
    for (int q = 0; q < T.nmc; ++q) {
        const double* o = T.fpart + ((int64_t)q * T.K_eval + k) * 2;
        x += o[0];
        y += o[1];
    }
    T.numer[k] = x;
    if (T.with_b) T.bspec[k] = y;
}

// ------------------------------------------- fused last pass + product

// The forward transform's last pass (radix 4096) works on contiguous
// 4096-position tiles, and so does the inverse transform's first pass. All
// positions of one tile share the frequency bits below the last digit,
// k_low, and the partners -k of its frequencies all lie in the tile of
// -k_low. A workgroup therefore takes such a pair of tiles (one tile when
// k_low = -k_low: k_low = 0 or half the range), runs the forward last pass
// of both into LDS, forms the products there, and runs the inverse first
// pass of both back to HBM: two sweeps over the grids fewer than separate
// passes and a product kernel.
//
// Pair q of a grid with 2^m tiles: q = 0 -> k_low = 0; q = 1 -> k_low =
// 2^(m-1); q >= 2 -> k_low = q - 1 with partner 2^m - k_low.
__device__ __forceinline__ void mid_pair(int64_t q, const RadixInfo& ri, int64_t& tA,
                                         int64_t& tB, int64_t& klow, int64_t& kpart) {
    const int m = ri.lgN - 12;
    int64_t kl = 0, kp = 0;
    if (m > 0 && q == 1) {
        kl = 1LL << (m - 1);
        kp = kl;
    } else if (m > 0 && q >= 2) {
        kl = q - 1;
        kp = (1LL << m) - kl;
    }
    tA = pos_of_freq(kl, ri) >> 12;
    tB = pos_of_freq(kp, ri) >> 12;
    klow = kl;
    kpart = kp;
}

// The product of the fused kernel in the grid's precision R. The factors
// (FP64) are rounded to R once per position, with the 1/2 of each unpacked
// spectrum folded in; the lag-0 partial sums accumulate in FP64. `paired`:
// the partner is another position (each term counts twice in the sums).
template <typename R, bool CCF, bool WB, typename C2>
__device__ __forceinline__ void mid_math(double f3d, double f2d, bool paired, C2 a, C2 b, C2 va,
                                         C2 vb, double (&sacc)[4], C2& o, C2& oc) {
    if (!CCF && !WB) {  // f3 |Z|^2
        o.x = (R)f3d * (a.x * a.x + a.y * a.y);
        o.y = (R)0;
        oc = o;
        return;
    }
    const R q = (R)(0.25 * f3d);
    // twice the unpacked spectra: 2A = Z_m + conj Z_-m, 2B = (Z_m - conj Z_-m)/i
    const R ar = a.x + b.x, ai = a.y - b.y;
    const R br = a.y + b.y, bi = b.x - a.x;
    if (!CCF) {  // |X|^2 + i |W|^2
        o.x = q * (ar * ar + ai * ai);
        o.y = q * (br * br + bi * bi);
        oc = o;
        return;
    }
    const double w = (paired ? 0.5 : 0.25) * f2d;
    sacc[0] += w * (double)(ar * ar + ai * ai);
    sacc[1] += w * (double)(br * br + bi * bi);
    const R gr = ar * br + ai * bi, gi = ar * bi - ai * br;  // 4 conj(X) Y
    if (!WB) {
        o.x = q * gr;
        o.y = q * gi;
        oc.x = o.x;
        oc.y = -o.y;
        return;
    }
    const R xr = va.x + vb.x, xi = va.y - vb.y;
    const R yr = va.y + vb.y, yi = vb.x - va.x;
    const R hr = xr * yr + xi * yi, hi = xr * yi - xi * yr;  // 4 conj(U_x) U_y
    sacc[2] += w * (double)(xr * xr + xi * xi);
    sacc[3] += w * (double)(yr * yr + yi * yi);
    // G_N + i G_B at m, conj(G_N) + i conj(G_B) at -m
    o.x = q * (gr - hi);
    o.y = q * (gi + hr);
    oc.x = q * (gr + hi);
    oc.y = q * (hr - gi);
}

constexpr int kMidPad = 4096 + 4096 / 16;  // one padded LDS tile (fftk::lds_pad)
constexpr int kMidThreads = 512;            // threads of the fused kernel

extern __shared__ char g_mid_lds[];

// Lag-lattice evaluation, the tile part. Position r of a tile holds frequency
// k_low + r N1 (N1 = N / 4096). With P = N1 P2 (P2 a power of two <= 4096) the
// frequency's residue mod P is k_low + N1 (r mod P2), so the tile folds on
// its own: F[r2] = sum_j G[r2 + P2 j]. The lag sum at lattice point n,
// sum over the residues p of F_p exp(-2 pi i p n / P), splits with
// p = k_low + N1 r2 into the P2-point inverse DFT of the tile's F at
// n mod P2, times exp(-2 pi i k_low n / P), summed over the N1 tiles; this
// function leaves Y[n2] = that inverse DFT in ybuf[k_low P2 + n2]. The DFT
// runs as Stockham stages in LDS with the twiddle progressions of the FFT
// passes: 8 entries per thread for P2 = 2048 (radix 8, 8, 8, 4 over all 256
// threads of the half), 4 below (radix-4 stages, then one of 2; P2 / 4
// threads). The planner keeps 16 <= P2 <= 2048 (2 <= N / P <= 256). Each
// half of the workgroup (256 threads) takes its own tile; every thread
// meets the same barriers.
template <int LG, typename C2>
__device__ __forceinline__ void fold_dft(const fftk::PassArgs& a, C2* tile, bool act, int lt) {
    // one column of 2^LG entries; threads past 2^LG / EPT only keep the barriers
    constexpr int EPT = LG >= 11 ? 8 : 4;
    fftk::run_stages_io<LG, 0, 1, LG, false, false, EPT>(a, tile, tile, 0, lt,
                                                         act && lt < (1 << LG) / EPT);
}

template <typename R>
__device__ __forceinline__ void mid_fold(const SpecTask& T, typename Cplx<R>::T* tile, bool act,
                                         int64_t k_low, int lt, const void* wsmall) {
    using C2 = typename Cplx<R>::T;
    const int lg = T.lgP2;
    const int P2 = 1 << lg;
    const int nf = 4096 >> lg;  // terms per folded entry
    C2 f[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int r2 = lt + 256 * i;
        C2 acc;
        acc.x = (R)0;
        acc.y = (R)0;
        if (act && r2 < P2)
            for (int j = 0; j < nf; ++j) acc = fftk::cadd(acc, tile[fftk::lds_pad(r2 + P2 * j)]);
        f[i] = acc;
    }
    __syncthreads();  // every read of the product tile is done
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int r2 = lt + 256 * i;
        if (act && r2 < P2) tile[fftk::lds_pad(r2)] = f[i];
    }
    __syncthreads();
    fftk::PassArgs a{};
    a.N = P2;
    a.S = 1;
    a.B = P2;
    a.sign = -1;
    a.wsmall = wsmall;
    switch (lg) {  // uniform over the workgroup (one task)
        case 4: fold_dft<4>(a, tile, act, lt); break;
        case 5: fold_dft<5>(a, tile, act, lt); break;
        case 6: fold_dft<6>(a, tile, act, lt); break;
        case 7: fold_dft<7>(a, tile, act, lt); break;
        case 8: fold_dft<8>(a, tile, act, lt); break;
        case 9: fold_dft<9>(a, tile, act, lt); break;
        case 10: fold_dft<10>(a, tile, act, lt); break;
        default: fold_dft<11>(a, tile, act, lt); break;
    }
    if (act) {
        C2* Y = reinterpret_cast<C2*>(T.ybuf) + k_low * P2;
        for (int n = lt; n < P2; n += 256) Y[n] = tile[fftk::lds_pad(n)];
    }
}

// MODE: bit 1 CCF, bit 0 pair-count channel (gridb for the CCF); as k_product
// without the unit channel. 512 threads: the two halves transform the two
// tiles at the same time (in a one-tile pair the second half only keeps the
// barriers); all threads share the products.
template <typename R, int MODE>
__global__ void __launch_bounds__(kMidThreads)
k_mid(const SpecTask* __restrict__ tasks, const int64_t* __restrict__ pair0, int ntasks,
      const RadixInfo* __restrict__ rinfo, const void* wsmall) {
    using C2 = typename Cplx<R>::T;
    constexpr bool CCF = (MODE & 2) != 0;
    constexpr bool WB = (MODE & 1) != 0;
    constexpr bool TWO = CCF && WB;  // the CCF pair-count grid is read too
    constexpr int kWaves = kMidThreads / 64;
    __shared__ double red[4][kWaves];
    C2* A = reinterpret_cast<C2*>(g_mid_lds);  // grid tile tA
    C2* Bt = A + kMidPad;                       // grid tile tB
    C2* UA = Bt + kMidPad;                      // (TWO) gridb tile tA
    C2* UB = UA + kMidPad;                      // (TWO) gridb tile tB
    const int64_t blk = blockIdx.x;
    const int ti = ntasks == 1 ? 0 : (int)wave_search<int64_t>(pair0, ntasks, blk, true) - 1;
    const SpecTask& T = tasks[ti];
    const RadixInfo ri = rinfo[ti];
    const int64_t N = T.N;
    int64_t tA, tB, kl, kp;
    mid_pair(blk - pair0[ti], ri, tA, tB, kl, kp);
    const bool self = tA == tB;
    const bool fold = T.P > 0;  // lag-lattice evaluation
    C2* const Z = reinterpret_cast<C2*>(T.grid);
    C2* const U = reinterpret_cast<C2*>(T.gridb);
    const int half = threadIdx.x >> 8;  // wave-uniform
    const int lt = threadIdx.x & 255;
    const bool act = half == 0 || !self;
    C2* const myZ = half ? Bt : A;
    C2* const myU = half ? UB : UA;
    const int64_t myT = half ? tB : tA;
    fftk::PassArgs a{};
    a.N = N;
    a.S = 1;
    a.B = 4096;
    a.sign = +1;
    a.wsmall = wsmall;
    // forward last pass of the tiles, into LDS
    if (act)
        fftk::run_stages_io<12, 0, 1, 12, true, false>(a, myZ, Z + myT * 4096, 0, lt);
    else
        fftk::run_stages_idle<12, 0, true, false>();
    if (TWO) {
        if (act)
            fftk::run_stages_io<12, 0, 1, 12, true, false>(a, myU, U + myT * 4096, 0, lt);
        else
            fftk::run_stages_idle<12, 0, true, false>();
    }
    C2* const PB = self ? A : Bt;
    C2* const PUB = self ? UA : UB;
    // products: position r of tile tA pairs with r' of tile tB (k_low = 0:
    // r' = -r mod 4096; else r' = 4095 - r)
    const ProductCtx<R> X =
        product_ctx<R>(gbl(reinterpret_cast<R*>(T.grid)), gbl(reinterpret_cast<R*>(T.gridb)),
                       gbl(reinterpret_cast<R*>(T.gridc)), T);
    double sacc[4] = {0.0, 0.0, 0.0, 0.0};
    constexpr bool pairs = CCF || WB;
    // position r of a tile holds frequency k_low + r 2^(lgN - 12)
    const int lgs = ri.lgN - 12;
    auto mode_of = [&](int64_t k) { return k <= N / 2 ? k : k - N; };
    // a pair of distinct tiles: every r of tA; one tile: r in [0, 2048)
    // (partners in the upper half), plus r = 2048 when it is its own partner
    const int nown = (!pairs || !self) ? 4096 : 2048;
    for (int r = threadIdx.x; r < nown; r += kMidThreads) {
        const int rp = kl == 0 ? ((4096 - r) & 4095) : (4095 - r);
        const bool paired = pairs && (tA != tB || rp != r);
        const C2 za = A[fftk::lds_pad(r)];
        const C2 zb = PB[fftk::lds_pad(rp)];
        C2 ua = za, ub = za;
        if (TWO) {
            ua = UA[fftk::lds_pad(r)];
            ub = PUB[fftk::lds_pad(rp)];
        }
        double f3, f2;
        product_factors_m<R, CCF>(X, mode_of(kl + ((int64_t)r << lgs)), f3, f2, fold);
        C2 o, oc;
        mid_math<R, CCF, WB>(f3, f2, paired, za, pairs ? zb : za, ua, ub, sacc, o, oc);
        A[fftk::lds_pad(r)] = o;
        if (paired) PB[fftk::lds_pad(rp)] = oc;
    }
    if (!pairs && !self) {  // each position on its own: the second tile too
        for (int r = threadIdx.x; r < 4096; r += kMidThreads) {
            const C2 za = Bt[fftk::lds_pad(r)];
            double f3, f2;
            product_factors_m<R, CCF>(X, mode_of(kp + ((int64_t)r << lgs)), f3, f2, fold);
            C2 o, oc;
            mid_math<R, CCF, WB>(f3, f2, false, za, za, za, za, sacc, o, oc);
            Bt[fftk::lds_pad(r)] = o;
        }
    }
    if (pairs && self && kl == 0 && threadIdx.x == 0) {  // k = N/2 at r = 2048
        const int r = 2048;
        const C2 za = A[fftk::lds_pad(r)];
        const C2 ua = TWO ? UA[fftk::lds_pad(r)] : za;
        double f3, f2;
        product_factors_m<R, CCF>(X, mode_of((int64_t)r << lgs), f3, f2, fold);
        C2 o, oc;
        mid_math<R, CCF, WB>(f3, f2, false, za, za, ua, ua, sacc, o, oc);
        A[fftk::lds_pad(r)] = o;
    }
    __syncthreads();
    if (fold) {
        // lag lattice: fold each product tile modulo P and inverse-transform
        // the P2 folded entries in LDS (see mid_fold)
        mid_fold<R>(T, myZ, act, half ? kp : kl, lt, wsmall);
    } else {
        // inverse first pass of the product tiles, to HBM
        a.sign = -1;
        if (act)
            fftk::run_stages_io<12, 0, 1, 12, false, true>(a, myZ, Z + myT * 4096, 0, lt);
        else
            fftk::run_stages_idle<12, 0, false, true>();
    }
    if (CCF) {  // lag-0 partial sums: the pair's in the slot of tile tA, 0 in tB's
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            double v = sacc[q];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
            if (lane == 0) red[q][wave] = v;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                double v = 0.0;
                for (int w = 0; w < kWaves; ++w) v += red[q][w];
                T.scale_part[4 * tA + q] = v;
                if (!self) T.scale_part[4 * tB + q] = 0.0;
            }
        }
    }
}

// Fallback flags of the spectral pair counts; workgroup b = i chunks + g
// takes rows [256 g, 256 g + 256) of problem i: window row r is flagged when its
// spectral b (evaluation index rowk[r]; -1: no requested lag) is below beta
// times the reference, or when the reference is not positive. Bit r % 64 of
// mask[i * words + r / 64].
//
// The reference bounds the pair sum at every lag and sets the scale of the
// transforms' rounding error. ACF: b(0), the lag-0 entry. CCF:
// sqrt(B_xx(0) B_yy(0)), the two series' lag-0 pair sums, which the product
// kernel leaves as Parseval partials (entries 2 and 3 of each of the task's
// N / 4096 records; each workgroup adds them in a fixed order). The Gaussian
// lag kernel is the self-convolution of a narrower Gaussian, so by
// Cauchy-Schwarz no lag of the CCF exceeds that bound, whether requested or
// not; the largest requested b would miss a peak between or beyond the
// requested lags.
//
// The output divides by the lag-0 scale s (ACF r(0) = N(0) / b(0); CCF
// sqrt(r_x(0) r_y(0)) from the partials' S and B entries), which for
// standardized values is near 1 unless the lag kernel spans much of a short
// series and the lag-0 sums cancel; then the rounding error, which does not
// cancel, is amplified by 1 / s. A row is therefore compared as
// b min(1, s) against beta times the reference (s not positive or NaN: the
// output is NaN with a status, and the factor is taken as 1). Plans fix
// their fallback lags when built, on placeholder values, so they must not
// depend on values: with use_scale = 0 the factor is 1.
constexpr int kFlagThreads = 256;

__global__ void __launch_bounds__(kFlagThreads)
k_fallback_flags(const SpecTask* __restrict__ tasks, const double* __restrict__ bspec, int Keval,
                 int K, int ccf, int use_scale, const int32_t* __restrict__ rowk, int Krow,
                 double beta, int words, uint64_t* __restrict__ mask) {
    const int chunks = (Krow + kFlagThreads - 1) / kFlagThreads;
    const int64_t i = (int64_t)blockIdx.x / chunks;
    const int g = (int)((int64_t)blockIdx.x % chunks);
    const gptr<const double> bb = gbl(bspec) + i * Keval;
    __shared__ double red[4][kFlagThreads / 64];
    double bref, scale;
    if (ccf) {
        const int64_t nrec = tasks[i].N / 4096;
        const gptr<const double> sp = gbl(tasks[i].scale_part);
        double v[4] = {0.0, 0.0, 0.0, 0.0};  // S_xx, S_yy, B_xx, B_yy
        for (int64_t r = threadIdx.x; r < nrec; r += kFlagThreads)
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] += sp[4 * r + q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] += __shfl_xor(v[q], off);
        if ((threadIdx.x & 63) == 0)
#pragma unroll
            for (int q = 0; q < 4; ++q) red[q][threadIdx.x >> 6] = v[q];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            v[q] = red[q][0];
#pragma unroll
            for (int w = 1; w < kFlagThreads / 64; ++w) v[q] += red[q][w];
        }
        bref = sqrt(v[2] * v[3]);
        scale = sqrt((v[0] / v[2]) * (v[1] / v[3]));
    } else {
        bref = bb[K];
        scale = gbl(tasks[i].numer)[K] / bref;
    }
    const double gs = (use_scale && scale > 0.0) ? fmin(1.0, scale) : 1.0;
    {
        const int r = g * kFlagThreads + (int)threadIdx.x;
        bool f = false;
        if (r < Krow) {
            const int k = gbl(rowk)[r];
            if (k >= 0) f = !(bb[k] * gs >= beta * bref) || !(bref > 0.0);
        }
        const unsigned long long bits = __ballot(f);
        if ((threadIdx.x & 63) == 0 && r < Krow) gbl(mask)[i * words + r / 64] = bits;
    }
}

}  // namespace

SpreadParams spread_params(double sigma, double eps) {
    // aliasing exp(-2 pi^2 s^2 (1 - 1/sigma)) and truncation exp(-W^2/2s^2)
    // both set to eps
    const double Le = -log(eps);
    SpreadParams p;
    p.s = sqrt(Le / (2.0 * M_PI * M_PI * (1.0 - 1.0 / sigma)));
    p.W = p.s * sqrt(2.0 * Le);
    return p;
}

int launch_tile_bounds(const SpecTask* d_tasks, const Chunk* d_chunks, int nchunks,
                       const int32_t* d_series_map, hipStream_t st, double bytes) {
    if (nchunks <= 0) return NCF_OK;
    ProfScope p(st, "tile_bounds", bytes, "bytes");
    hipLaunchKernelGGL(k_tile_bounds, dim3((unsigned)nchunks), dim3(kThreads), 0, st, d_tasks,
                       d_chunks, d_series_map);
    NCF_CHECK_LAUNCH();
    return NCF_OK;
}

template <typename R>
void (*spread_kernel(int mode))(const SpecTask*, const int64_t*, int, int64_t, int64_t,
                                const int64_t*) {
    switch (mode & 15) {
        case 0: return k_spread<R, 0>;
        case 1: return k_spread<R, 1>;
        case 2: return k_spread<R, 2>;
        case 3: return k_spread<R, 3>;
        case 5: return k_spread<R, 5>;
        case 7: return k_spread<R, 7>;
        case 13: return k_spread<R, 13>;
        case 15: return k_spread<R, 15>;
        default: return nullptr;  // weights or units without the pair-count channel
    }
}

int launch_spread(const SpecTask* d_tasks, const int64_t* d_tile0, int ntasks, int64_t ntiles,
                  const int64_t* d_tile_rec, int tile, bool ccf, bool with_b, bool weighted,
                  bool unw, bool fp64, hipStream_t st, double bytes) {
    if (tile != kTile || (weighted && !with_b) || (unw && !weighted)) {
        set_error("spread tile mismatch");
        return NCF_E_UNSUPPORTED;
    }
    if (ntiles <= 0) return NCF_OK;
    const int64_t nblocks = round_up(ntiles, kXcds);
    const int mode = (ccf ? 2 : 0) | (with_b ? 1 : 0) | (weighted ? 4 : 0) | (unw ? 8 : 0);
    ProfScope p(st, fp64 ? "spread_f64" : "spread_f32", bytes, "bytes");
    if (fp64)
        hipLaunchKernelGGL(spread_kernel<double>(mode), dim3((unsigned)nblocks), dim3(kThreads),
                           0, st, d_tasks, d_tile0, ntasks, ntiles, nblocks, d_tile_rec);
    else
        hipLaunchKernelGGL(spread_kernel<float>(mode), dim3((unsigned)nblocks), dim3(kThreads),
                           0, st, d_tasks, d_tile0, ntasks, ntiles, nblocks, d_tile_rec);
    NCF_CHECK_LAUNCH();
    return NCF_OK;
}

template <typename R>
void (*product_kernel(int mode))(const SpecTask*, const int64_t*, int, int64_t,
                                  const RadixInfo*) {
    switch (mode & 7) {
        case 0: return k_product<R, 0>;
        case 1: return k_product<R, 1>;
        case 2: return k_product<R, 2>;
        case 3: return k_product<R, 3>;
        case 5: return k_product<R, 5>;
        case 7: return k_product<R, 7>;
        default: return nullptr;  // a unit channel needs the pair-count channel
    }
}

int launch_product(const SpecTask* d_tasks, const int64_t* d_pos0, int ntasks, int64_t total,
                   const int64_t* d_radix_info, bool ccf, bool with_b, bool unw, bool fp64,
                   hipStream_t st, double bytes) {
    if (total <= 0) return NCF_OK;
    if (unw && !with_b) {
        set_error("product: unit channel without the pair-count channel");
        return NCF_E_UNSUPPORTED;
    }
    const RadixInfo* ri = reinterpret_cast<const RadixInfo*>(d_radix_info);
    const int mode = (ccf ? 2 : 0) | (with_b ? 1 : 0) | (unw ? 4 : 0);
    ProfScope p(st, fp64 ? "product_f64" : "product_f32", bytes, "bytes");
    if (fp64)
        hipLaunchKernelGGL(product_kernel<double>(mode), dim3((unsigned)ceil_div(total, kTile)),
                           dim3(kThreads), 0, st, d_tasks, d_pos0, ntasks, total, ri);
    else
        hipLaunchKernelGGL(product_kernel<float>(mode), dim3((unsigned)ceil_div(total, kTile)),
                           dim3(kThreads), 0, st, d_tasks, d_pos0, ntasks, total, ri);
    NCF_CHECK_LAUNCH();
    return NCF_OK;
}

int launch_fallback_flags(const SpecTask* d_tasks, const double* bspec, int64_t nprob,
                          int Keval, int K, bool ccf, bool use_scale, const int32_t* rowk,
                          int Krow, double beta, uint64_t* mask, hipStream_t st) {
    if (nprob <= 0 || Krow <= 0) return NCF_OK;
    const int64_t blocks = nprob * ceil_div(Krow, kFlagThreads);
    if (blocks > INT32_MAX) {
        set_error("fallback flags: %lld workgroups", (long long)blocks);
        return NCF_E_UNSUPPORTED;
    }
    ProfScope p(st, "fallback_flags", 0.0, "bytes");
    hipLaunchKernelGGL(k_fallback_flags, dim3((unsigned)blocks), dim3(kFlagThreads), 0, st,
                       d_tasks, bspec, Keval, K, ccf ? 1 : 0, use_scale ? 1 : 0, rowk, Krow,
                       beta, (int)ceil_div(Krow, 64), mask);
    NCF_CHECK_LAUNCH();
    return NCF_OK;
}

int launch_interp(const SpecTask* d_tasks, int ntasks, const int64_t* d_k0, int64_t total_k,
                  bool fp64, hipStream_t st) {
    if (total_k <= 0) return NCF_OK;
    ProfScope p(st, "interp", 0.0, "bytes");
    if (fp64)
        hipLaunchKernelGGL(k_interp<double>, dim3((unsigned)ceil_div(total_k, 128)), dim3(128), 0,
                           st, d_tasks, ntasks, d_k0, total_k);
    else
        hipLaunchKernelGGL(k_interp<float>, dim3((unsigned)ceil_div(total_k, 128)), dim3(128), 0,
                           st, d_tasks, ntasks, d_k0, total_k);
    NCF_CHECK_LAUNCH();
    return NCF_OK;
}

int launch_fold_eval(const SpecTask* d_tasks, int ntasks, const int64_t* d_fe0, int64_t nblocks,
                     const int64_t* d_k0, int64_t total_k, bool chunk_sums, bool fp64,
                     hipStream_t st) {
    if (nblocks <= 0) return NCF_OK;
    {
        ProfScope p(st, "fold_eval", 0.0, "bytes");
        if (fp64)
            hipLaunchKernelGGL(k_fold_eval<double>, dim3((unsigned)nblocks), dim3(256), 0, st,
                               d_tasks, ntasks, d_fe0);
        else
            hipLaunchKernelGGL(k_fold_eval<float>, dim3((unsigned)nblocks), dim3(256), 0, st,
                               d_tasks, ntasks, d_fe0);
        NCF_CHECK_LAUNCH();
    }
    if (chunk_sums && total_k > 0) {
        ProfScope p(st, "fold_sum", 0.0, "bytes");
        hipLaunchKernelGGL(k_fold_sum, dim3((unsigned)ceil_div(total_k, 128)), dim3(128), 0, st,
                           d_tasks, ntasks, d_k0, total_k);
        NCF_CHECK_LAUNCH();
    }
    return NCF_OK;
}

}  // namespace ncf

namespace ncf {

bool mid_supported(bool ccf, bool with_b, bool unw, bool fp64) {
    if (unw) return false;
    const int tiles = (ccf && with_b) ? 4 : 2;
    const size_t csz = fp64 ? 16 : 8;
    return (size_t)tiles * kMidPad * csz <= 160 * 1024;
}

int64_t mid_pairs(int64_t N) { return N <= 4096 ? 1 : N / 8192 + 1; }

template <typename R, int MODE>
static int launch_mid_t(const SpecTask* d_tasks, const int64_t* d_pair0, int ntasks,
                        int64_t npairs, const RadixInfo* ri, const void* wsmall, hipStream_t st) {
    constexpr bool TWO = (MODE & 3) == 3;
    const size_t lds = (size_t)(TWO ? 4 : 2) * kMidPad * sizeof(typename Cplx<R>::T);
    static bool attr_set = false;
    if (!attr_set) {
        NCF_TRY_HIP(hipFuncSetAttribute((const void*)k_mid<R, MODE>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        attr_set = true;
    }
    hipLaunchKernelGGL((k_mid<R, MODE>), dim3((unsigned)npairs), dim3(kMidThreads), lds, st,
                       d_tasks, d_pair0, ntasks, ri, wsmall);
    NCF_CHECK_LAUNCH();
    return NCF_OK;
}

int launch_mid(const SpecTask* d_tasks, const int64_t* d_pair0, int ntasks, int64_t npairs,
               const int64_t* d_radix_info, const void* wsmall, bool ccf, bool with_b, bool fp64,
               hipStream_t st, double bytes) {
    if (npairs <= 0) return NCF_OK;
    if (!mid_supported(ccf, with_b, false, fp64)) {
        set_error("fused last pass: mode not covered");
        return NCF_E_UNSUPPORTED;
    }
    const RadixInfo* ri = reinterpret_cast<const RadixInfo*>(d_radix_info);
    const int mode = (ccf ? 2 : 0) | (with_b ? 1 : 0);
    ProfScope p(st, fp64 ? "mid_f64" : "mid_f32", bytes, "bytes");
    if (fp64) {
        switch (mode) {
            case 0: return launch_mid_t<double, 0>(d_tasks, d_pair0, ntasks, npairs, ri, wsmall, st);
            case 1: return launch_mid_t<double, 1>(d_tasks, d_pair0, ntasks, npairs, ri, wsmall, st);
            default: return launch_mid_t<double, 2>(d_tasks, d_pair0, ntasks, npairs, ri, wsmall, st);
        }
    }
    switch (mode) {
        case 0: return launch_mid_t<float, 0>(d_tasks, d_pair0, ntasks, npairs, ri, wsmall, st);
        case 1: return launch_mid_t<float, 1>(d_tasks, d_pair0, ntasks, npairs, ri, wsmall, st);
        case 2: return launch_mid_t<float, 2>(d_tasks, d_pair0, ntasks, npairs, ri, wsmall, st);
        default: return launch_mid_t<float, 3>(d_tasks, d_pair0, ntasks, npairs, ri, wsmall, st);
    }
}

}  // namespace ncf
