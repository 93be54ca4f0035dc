// regular.hip -- the classic-FFT estimators for series on a regular time
// lattice (Sec. "Regularly-sampled data"; the Wiener-Khinchin correlation of
// Sec. "Correlation estimation on a regular grid", eq. wienerkhinchin).
//
// With times t_i = t_ref + m_i dt every pair sits at a whole lattice lag q,
// so the kernel estimator (eq. kernel_estimator) at lag tau is a filter over
// q (Sec. "Effective pair count": the pair count comes from filtering the
// raw pair-count sequence with the numerator's filter):
//   C(tau) = sum_q omega(q dt - tau) R(q),  R(q) = sum over pairs at q of v_i v_j
//   B(tau), b(tau), count(tau): the same filter over the weight and count
//   correlations (on a gapless lattice N(q) is the ramp n - |q|).
// R and N come from one zero-padded FFT correlation of the lattice grids. In
// FP64 the transforms leave N(q) far closer than 1/2 to its integer value, so
// it is rounded: rectangle counts are exact and a lag with no pairs has a
// numerator of exactly zero.
//
// Window membership is decided in lattice units: q is in the window of tau
// when it lies between (tau -+ W)/dt, each edge snapped to an integer when
// within 1e-9 (relative) of one, with the same open/closed ends as the
// irregular estimator (Gaussian: W = 6h, half-open; rectangle: W = h,
// closed). The weight is evaluated at q dt - tau.
#include "internal.h"

namespace ncf {

namespace {

constexpr int kThreads = 256;

// one complex128 grid value
struct C64 {
    double x, y;
};
__device__ __forceinline__ C64 ld(gptr<const double> g, int64_t i) {
    return C64{g[2 * i], g[2 * i + 1]};
}
__device__ __forceinline__ void st(gptr<double> g, int64_t i, const C64& v) {
    g[2 * i] = v.x;
    g[2 * i + 1] = v.y;
}

__device__ __forceinline__ double fl(double v) { return v > kFloor ? v : kFloor; }

// ------------------------------------------------------------------ fill

__global__ void k_reg_clear(const RegTask* __restrict__ tasks, int ntasks) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ntasks) *gbl(tasks[i].bad) = 0;
}

// One workgroup fills kRegCells lattice cells of every input grid of one
// task. The samples of the tile are those with times in
// [t_ref + (a0 - 1/2) dt, t_ref + (a0 + kRegCells - 1/2) dt): adjacent tiles
// use the same boundary expression, so every sample belongs to one tile.
// Samples of one cell are consecutive (sorted times); the first of them sums
// the run in sample order, so the grid values are deterministic.
template <int MODE>
__global__ void __launch_bounds__(kThreads)
k_reg_fill(const RegTask* __restrict__ tasks, const int64_t* __restrict__ blk0, int ntasks) {
    constexpr bool CCF = MODE >= 2;
    constexpr bool WT = (MODE & 1) != 0;
    constexpr int NG = reg_in_grids(MODE);
    constexpr int NCH = 2 * NG;
    __shared__ double cell[NCH][kRegCells];
    __shared__ int64_t rng[2][2];
    const int64_t b = blockIdx.x;
    const int ti = ntasks == 1 ? 0 : (int)wave_search<int64_t>(blk0, ntasks, b, true) - 1;
    const RegTask& T = tasks[ti];
    const int64_t a0 = (b - T.blk0) * kRegCells;
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    if (wave < (CCF ? 4 : 2)) {
        const int s = wave >> 1;
        const int64_t a = a0 + (wave & 1) * kRegCells;
        int64_t r = 0;
        if (a0 < T.G) {
            const double thr = T.t_ref + ((double)a - 0.5) * T.dt;
            r = wave_search<double>(T.t[s], T.n[s], thr, false);
        }
        if ((tid & 63) == 0) rng[s][wave & 1] = r;
    }
    for (int c = tid; c < kRegCells; c += kThreads)
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) cell[ch][c] = 0.0;
    __syncthreads();
    bool bad = false;
    // lattice index of a time: rint((t - t_ref) / dt), formed with the
    // reciprocal; an accepted time lies within tol = 1e-6 dt of its lattice
    // point, so the quotient is never near a half-integer and both forms give
    // the same index (a time near a half-point is rejected either way)
    const double inv_dt = 1.0 / T.dt;
    auto lat = [&](double tv) { return rint((tv - T.t_ref) * inv_dt); };
#pragma unroll
    for (int s = 0; s < (CCF ? 2 : 1); ++s) {
        const gptr<const double> t = gbl(T.t[s]);
        const gptr<const double> v = gbl(T.v[s]);
        const double* wp = WT ? T.w[s] : nullptr;
        const gptr<const double> w = gbl(wp);
        const int64_t i0 = rng[s][0], i1 = rng[s][1];
        // channels of this set: value, weight, count
        const int chv = CCF ? s : 0;
        const int chw = CCF ? 2 + s : 1;
        const int chn = CCF ? (WT ? 4 + s : 2 + s) : (WT ? 2 : 1);
        for (int64_t i = i0 + tid; i < i1; i += kThreads) {
            const double tv = t[i];
            const double mr = lat(tv);
            const double cd = mr - (double)a0;
            if (!(fabs(tv - (T.t_ref + mr * T.dt)) <= T.tol) || !(cd >= 0.0) ||
                !(cd < (double)kRegCells)) {
                bad = true;
                continue;
            }
            if (i > i0 && lat(t[i - 1]) == mr) continue;  // not first
            double sv = 0.0, sw = 0.0, sn = 0.0;
            for (int64_t j = i; j < i1; ++j) {
                if (j > i && lat(t[j]) != mr) break;
                sv += v[j];
                if (WT) sw += wp ? w[j] : 1.0;
                sn += 1.0;
            }
            const int c = (int)cd;
            cell[chv][c] = sv;
            if (WT) cell[chw][c] = sw;
            cell[chn][c] = sn;
        }
    }
    if (bad) *gbl(T.bad) = 1;
    __syncthreads();
    const gptr<double> g = gbl(T.grids);
    for (int c = tid; c < kRegCells; c += kThreads) {
#pragma unroll
        for (int q = 0; q < NG; ++q) {
            st(g, q * T.N + a0 + c, C64{cell[2 * q][c], cell[2 * q + 1][c]});
        }
    }
}

// --------------------------------------------------------------- product

struct Spec {
    double r, i;
};

// conj(A) B
__device__ __forceinline__ Spec cross(const Spec& a, const Spec& b) {
    return Spec{a.r * b.r + a.i * b.i, a.r * b.i - a.i * b.r};
}
__device__ __forceinline__ Spec power(const Spec& a) { return Spec{a.r * a.r + a.i * a.i, 0.0}; }

// Spectra of one (k, -k) pair: unpack the channels of every input grid from
// the values at p (frequency k) and pp (frequency -k), form the products and
// store S1 + i S2 of every output grid at p and conj(S1) + i conj(S2) at pp.
// The packed grid Z = A + iB of two real channels gives
// A_k = (Z_k + conj Z_-k)/2 and B_k = (Z_k - conj Z_-k)/(2i); the inverse
// transform of S1 + i S2 returns both real lag sequences (real and imaginary
// parts).
template <int MODE>
__device__ __forceinline__ void reg_pair(gptr<double> Z, int64_t N, int64_t p, int64_t pp,
                                         const C64 (&za)[reg_in_grids(MODE)],
                                         const C64 (&zb)[reg_in_grids(MODE)]) {
    constexpr int NG = reg_in_grids(MODE);
    constexpr int NO = reg_out_grids(MODE);
    Spec ch[2 * NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        const C64 a = za[g], b = zb[g];
        ch[2 * g] = Spec{0.5 * (a.x + b.x), 0.5 * (a.y - b.y)};
        ch[2 * g + 1] = Spec{0.5 * (a.y + b.y), -0.5 * (a.x - b.x)};
    }
    Spec s1[NO], s2[NO];
    const Spec zero{0.0, 0.0};
    if constexpr (MODE == 0) {
        s1[0] = power(ch[0]);
        s2[0] = power(ch[1]);
    } else if constexpr (MODE == 1) {
        s1[0] = power(ch[0]);
        s2[0] = power(ch[1]);
        s1[1] = power(ch[2]);
        s2[1] = zero;
    } else if constexpr (MODE == 2) {
        s1[0] = cross(ch[0], ch[1]);
        s2[0] = cross(ch[2], ch[3]);
        s1[1] = power(ch[0]);
        s2[1] = power(ch[1]);
        s1[2] = power(ch[2]);
        s2[2] = power(ch[3]);
    } else {
        s1[0] = cross(ch[0], ch[1]);
        s2[0] = cross(ch[2], ch[3]);
        s1[1] = cross(ch[4], ch[5]);
        s2[1] = zero;
        s1[2] = power(ch[0]);
        s2[2] = power(ch[1]);
        s1[3] = power(ch[2]);
        s2[3] = power(ch[3]);
    }
    const double inv = 1.0 / (double)N;
#pragma unroll
    for (int o = 0; o < NO; ++o) {
        const C64 at{inv * (s1[o].r - s2[o].i), inv * (s1[o].i + s2[o].r)};
        const C64 am{inv * (s1[o].r + s2[o].i), inv * (s2[o].r - s1[o].i)};
        st(Z, o * N + p, at);
        if (pp != p) st(Z, o * N + pp, am);
    }
}

// A workgroup owns kProdTile consecutive positions of one task. The last
// transform pass has radix 4096, so the top bit of the frequency k is bit 11
// of the position: positions with that bit clear hold k < N/2 and own the
// pair (k, -k); k = N/2 (position 2048 of the first tile) is its own
// partner and is handled there. Each thread issues the loads of its
// positions before any store (pairs are disjoint, so nothing is read after
// being written).
constexpr int kProdTile = 4096;
// pairs per thread (fewer with more input grids, to bound registers) and
// threads per workgroup
__host__ __device__ constexpr int prod_it(int mode) { return reg_in_grids(mode) == 1 ? 8 : reg_in_grids(mode) == 2 ? 4 : 2; }
__host__ __device__ constexpr int prod_threads(int mode) { return kProdTile / 2 / prod_it(mode); }

template <int MODE>
__global__ void __launch_bounds__(prod_threads(MODE))
k_reg_product(const RegTask* __restrict__ tasks, const int64_t* __restrict__ pos0, int ntasks) {
    constexpr int NG = reg_in_grids(MODE);
    constexpr int kProdIt = prod_it(MODE);
    constexpr int kTh = prod_threads(MODE);
    const int64_t gb = (int64_t)blockIdx.x * kProdTile;
    const int ti = ntasks == 1 ? 0 : (int)wave_search<int64_t>(pos0, ntasks, gb, true) - 1;
    const RegTask& T = tasks[ti];
    const int64_t N = T.N;
    const int64_t tb = gb - T.pos0;  // first position of the tile in its grid
    const RadixInfo ri = T.ri;
    const gptr<double> Z = gbl(T.grids);
    int64_t pb[kProdIt];
    C64 za[kProdIt][NG], zb[kProdIt][NG];
#pragma unroll
    for (int it = 0; it < kProdIt; ++it) {
        const int64_t p = tb + threadIdx.x + it * kTh;
        pb[it] = pos_of_freq((N - freq_of_pos(p, ri)) & (N - 1), ri);
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            za[it][g] = ld(Z, g * N + p);
            zb[it][g] = ld(Z, g * N + pb[it]);
        }
    }
#pragma unroll
    for (int it = 0; it < kProdIt; ++it)
        reg_pair<MODE>(Z, N, tb + threadIdx.x + it * kTh, pb[it], za[it], zb[it]);
    if (tb == 0 && threadIdx.x == 0) {  // k = N/2
        const int64_t p = kProdTile / 2;
        const int64_t pp = pos_of_freq((N - freq_of_pos(p, ri)) & (N - 1), ri);
        C64 a[NG], b[NG];
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            a[g] = ld(Z, g * N + p);
            b[g] = ld(Z, g * N + pp);
        }
        reg_pair<MODE>(Z, N, p, pp, a, b);
    }
}

// ---------------------------------------------------------------- finish

__device__ __forceinline__ double snap(double e) {
    const double r = rint(e);
    return fabs(e - r) <= 1e-9 * fmax(1.0, fabs(e)) ? r : e;
}

// Lattice lags [q0, q1] in the window of lag tau. ccf_open: the window is
// open at its lower lattice end (the Gaussian CCF predicate seen from the
// lag q = m_y - m_x); otherwise the Gaussian window is open at the top.
template <int KERN>
__device__ __forceinline__ void reg_window(double tau, const RegTask& T, bool ccf_open,
                                           int64_t* q0, int64_t* q1) {
    const double W = KERN == NCF_GAUSSIAN ? 6.0 * T.h : T.h;
    const double lo = snap((tau - W) / T.dt);
    const double hi = snap((tau + W) / T.dt);
    double a, b;
    if (KERN == NCF_RECTANGLE) {
        a = ceil(lo);
        b = floor(hi);
    } else if (ccf_open) {
        a = floor(lo) + 1.0;
        b = floor(hi);
    } else {
        a = ceil(lo);
        b = ceil(hi) - 1.0;
    }
    const double Qd = (double)T.Q;
    a = fmax(a, -Qd);
    b = fmin(b, Qd);
    *q0 = (int64_t)a;
    *q1 = b >= a ? (int64_t)b : (int64_t)a - 1;
}

__device__ __forceinline__ double gauss_w(double d, double h) {
    return exp(-(d * d) / (2.0 * h * h)) * (0.3989422804014327 / h);
}

// Sums over one window: numerator C, denominator B, pair sum b, count.
struct Acc {
    double C, B, b;
    int64_t n;
};

// Lag quantities of output grid o (real or imaginary part) at lattice lag q.
__device__ __forceinline__ double lagval(const RegTask& T, int o, bool im, int64_t q) {
    const int64_t idx = q >= 0 ? q : T.N + q;
    const gptr<const double> g = gbl(reinterpret_cast<const double*>(T.grids));
    return g[2 * (o * T.N + idx) + (im ? 1 : 0)];
}

// Where each quantity lives, as (grid, imaginary part): the numerator, the
// weighted denominator and the sample-count correlation (hc: present).
struct Slots {
    int on, dn, cn;
    bool in, id, ic, hc;
};
template <int MODE>
__device__ __forceinline__ Slots main_slots() {
    if (MODE == 0) return Slots{0, 0, 0, false, true, true, true};
    if (MODE == 1) return Slots{0, 0, 1, false, true, false, true};
    if (MODE == 2) return Slots{0, 0, 0, false, true, true, true};
    return Slots{0, 0, 1, false, true, false, true};
}
// CCF lag-0 terms of series 1 (y = false) or series 2 (y = true) on itself;
// weighted, only the numerator and the weighted denominator are needed
template <int MODE>
__device__ __forceinline__ Slots self_slots(bool y) {
    if (MODE == 2) return Slots{1, 2, 2, y, y, y, true};
    return Slots{2, 3, 3, y, y, y, false};
}

template <int MODE, int KERN>
__device__ __forceinline__ void acc_q(const RegTask& T, const Slots& S, int64_t q, double tau,
                                      Acc& a) {
    constexpr bool WT = (MODE & 1) != 0;
    double cnt = 0.0;
    if (S.hc) {
        cnt = rint(lagval(T, S.cn, S.ic, q));
        if (cnt == 0.0) return;  // no pair at this lag: every sum is exactly 0
    }
    const double om = KERN == NCF_GAUSSIAN ? gauss_w((double)q * T.dt - tau, T.h) : 1.0;
    a.C += om * lagval(T, S.on, S.in, q);
    a.B += om * (WT ? lagval(T, S.dn, S.id, q) : cnt);
    a.b += om * cnt;
    a.n += (int64_t)cnt;
}

// Block-wide window sums (fixed order: strided per thread, then a tree).
template <int MODE, int KERN>
__device__ void block_window(const RegTask& T, const Slots& S, double tau, bool ccf_open,
                             double (&red)[2][kThreads], double* outC, double* outB) {
    int64_t q0, q1;
    reg_window<KERN>(tau, T, ccf_open, &q0, &q1);
    Acc a{0.0, 0.0, 0.0, 0};
    for (int64_t q = q0 + threadIdx.x; q <= q1; q += kThreads) acc_q<MODE, KERN>(T, S, q, tau, a);
    red[0][threadIdx.x] = a.C;
    red[1][threadIdx.x] = a.B;
    __syncthreads();
    for (int off = kThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            red[0][threadIdx.x] += red[0][threadIdx.x + off];
            red[1][threadIdx.x] += red[1][threadIdx.x + off];
        }
        __syncthreads();
    }
    *outC = red[0][0];
    *outB = red[1][0];
    __syncthreads();
}

template <int MODE, int KERN>
__global__ void __launch_bounds__(kThreads)
k_reg_finish(const RegTask* __restrict__ tasks, int nkb, const double* __restrict__ lags,
             int64_t K, const IoBlock* __restrict__ io) {
    constexpr bool CCF = MODE >= 2;
    __shared__ double red[2][kThreads];
    const RegTask& T = tasks[blockIdx.x / nkb];
    const int kb = blockIdx.x % nkb;
    const int tid = threadIdx.x;
    double* const out_c = io->c + T.out_off;
    double* const out_b = io->b + T.out_off;
    int64_t* const out_n = io->count ? io->count + T.out_off : nullptr;
    int32_t fail = T.skip ? T.skip_status : NCF_OK;
    if (fail == NCF_OK && T.st0 && T.st0->status != NCF_OK) fail = T.st0->status;
    if (fail == NCF_OK && T.st1 && T.st1->status != NCF_OK) fail = T.st1->status;
    if (fail == NCF_OK && *gbl(T.bad) != 0) fail = NCF_E_INVALID_ARG;
    const int64_t k = (int64_t)kb * kThreads + tid;
    if (fail != NCF_OK) {
        if (k < K) {
            out_c[k] = NAN;
            out_b[k] = 0.0;
            if (out_n) out_n[k] = 0;
        }
        if (kb == 0 && tid == 0) io->status[T.index] = fail;
        return;
    }
    // lag-0 scale: ACF r(0); CCF sqrt(scale_x scale_y), each series on itself
    double scale;
    if (!CCF) {
        double c0, b0;
        block_window<MODE, KERN>(T, main_slots<MODE>(), 0.0, false, red, &c0, &b0);
        const double r0 = c0 / fl(b0);
        scale = (r0 > kMinScale && isfinite(r0)) ? r0 : NAN;
    } else {
        double cx, bx, cy, by;
        block_window<MODE, KERN>(T, self_slots<MODE>(false), 0.0, false, red, &cx, &bx);
        block_window<MODE, KERN>(T, self_slots<MODE>(true), 0.0, false, red, &cy, &by);
        const double sx = cx / fl(bx), sy = cy / fl(by), prod = sx * sy;
        scale = (fabs(sx) > kMinScale && fabs(sy) > kMinScale && prod > 0.0 && isfinite(prod))
                    ? sqrt(prod)
                    : NAN;
    }
    if (kb == 0 && tid == 0) io->status[T.index] = (scale == scale) ? NCF_OK : NCF_E_DEGENERATE;
    if (k >= K) return;
    const double tau = lags[k];
    int64_t q0, q1;
    reg_window<KERN>(tau, T, CCF, &q0, &q1);
    const Slots S = main_slots<MODE>();
    Acc a{0.0, 0.0, 0.0, 0};
    for (int64_t q = q0; q <= q1; ++q) acc_q<MODE, KERN>(T, S, q, tau, a);
    out_c[k] = (a.C / fl(a.B)) / scale;
    out_b[k] = fl(a.b);
    if (out_n) out_n[k] = KERN == NCF_RECTANGLE ? a.n : 0;
}

template <int MODE>
void (*fill_kernel())(const RegTask*, const int64_t*, int) {
    return k_reg_fill<MODE>;
}

}  // namespace

int launch_reg_clear(const RegTask* d_tasks, int ntasks, hipStream_t st) {
    if (ntasks <= 0) return NCF_OK;
    hipLaunchKernelGGL(k_reg_clear, dim3((unsigned)ceil_div(ntasks, kThreads)), dim3(kThreads), 0,
                       st, d_tasks, ntasks);
    NCF_CHECK_LAUNCH();
    return NCF_OK;
}

int launch_reg_fill(const RegTask* d_tasks, const int64_t* d_blk0, int ntasks, int64_t nblocks,
                    int mode, hipStream_t st, double bytes) {
    if (ntasks <= 0 || nblocks <= 0) return NCF_OK;
    ProfScope p(st, "reg_fill", bytes, "bytes");
    void (*k)(const RegTask*, const int64_t*, int) =
        mode == 0 ? fill_kernel<0>() : mode == 1 ? fill_kernel<1>() : mode == 2 ? fill_kernel<2>()
                                                                                 : fill_kernel<3>();
    hipLaunchKernelGGL(k, dim3((unsigned)nblocks), dim3(kThreads), 0, st, d_tasks, d_blk0, ntasks);
    NCF_CHECK_LAUNCH();
    return NCF_OK;
}

int launch_reg_product(const RegTask* d_tasks, const int64_t* d_pos0, int ntasks, int64_t total,
                       int mode, hipStream_t st, double bytes) {
    if (ntasks <= 0 || total <= 0) return NCF_OK;
    ProfScope p(st, "reg_product", bytes, "bytes");
    const dim3 grid((unsigned)ceil_div(total, kProdTile));
    switch (mode) {
        case 0: hipLaunchKernelGGL(k_reg_product<0>, grid, dim3(prod_threads(0)), 0, st, d_tasks, d_pos0, ntasks); break;
        case 1: hipLaunchKernelGGL(k_reg_product<1>, grid, dim3(prod_threads(1)), 0, st, d_tasks, d_pos0, ntasks); break;
        case 2: hipLaunchKernelGGL(k_reg_product<2>, grid, dim3(prod_threads(2)), 0, st, d_tasks, d_pos0, ntasks); break;
        default: hipLaunchKernelGGL(k_reg_product<3>, grid, dim3(prod_threads(3)), 0, st, d_tasks, d_pos0, ntasks); break;
    }
    NCF_CHECK_LAUNCH();
    return NCF_OK;
}

template <int MODE>
static void launch_finish_mode(int kern, dim3 grid, hipStream_t st, const RegTask* d_tasks, int nkb,
                               const double* d_lags, int64_t K, const IoBlock* io) {
    if (kern == NCF_GAUSSIAN)
        hipLaunchKernelGGL((k_reg_finish<MODE, NCF_GAUSSIAN>), grid, dim3(kThreads), 0, st,
                           d_tasks, nkb, d_lags, K, io);
    else
        hipLaunchKernelGGL((k_reg_finish<MODE, NCF_RECTANGLE>), grid, dim3(kThreads), 0, st,
                           d_tasks, nkb, d_lags, K, io);
}

int launch_reg_finish(const RegTask* d_tasks, int ntasks, const double* d_lags, int64_t K,
                      int mode, int kern, const IoBlock* io, hipStream_t st) {
    if (ntasks <= 0) return NCF_OK;
    ProfScope p(st, "reg_finish", 0.0, "bytes");
    const int nkb = (int)std::max<int64_t>(1, ceil_div(K, kThreads));
    const dim3 grid((unsigned)((int64_t)ntasks * nkb));
    switch (mode) {
        case 0: launch_finish_mode<0>(kern, grid, st, d_tasks, nkb, d_lags, K, io); break;
        case 1: launch_finish_mode<1>(kern, grid, st, d_tasks, nkb, d_lags, K, io); break;
        case 2: launch_finish_mode<2>(kern, grid, st, d_tasks, nkb, d_lags, K, io); break;
        default: launch_finish_mode<3>(kern, grid, st, d_tasks, nkb, d_lags, K, io); break;
    }
    NCF_CHECK_LAUNCH();
    return NCF_OK;
}

}  // namespace ncf
