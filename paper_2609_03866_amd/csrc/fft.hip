// fft.hip -- power-of-two complex FFT for the spreading grid (step A4).
//
// N = R_1 * R_2 * ... * R_P with R_P = 4096 and the other radices <= 1024.
// Pass i treats the grid as blocks of B_i = N / (R_1 ... R_{i-1}) elements,
// each a R_i x S_i matrix (S_i = B_i / R_i), and performs the four-step
// decomposition of that block: length-R_i DFTs down the columns, then the
// twiddles w_{B_i}^(s k). With the +1 sign (type-1 side) the passes run in
// order and leave the spectrum in mixed-radix digit-reversed order; the -1
// sign (type-2 side) runs the adjoint passes in reverse order, consuming that
// order and producing natural order. The spectral product works in the
// digit-reversed order directly, so no transpose pass is ever made.
//
// A workgroup transforms one tile of T = 4096 or 8192 elements: R_i rows by
// C_i = T / R_i adjacent columns (C_i * element size contiguous bytes per
// row in HBM; the strided passes use the larger tile for longer runs). Each column's DFT is a Stockham autosort sequence of radix-16
// stages (and one radix-8/4/2 stage for the remainder) with 16 elements per
// thread in registers: the first stage reads HBM directly, the last writes
// HBM directly, and the stages in between exchange through padded LDS.
// Twiddles: the factors a thread applies to its 16 elements form geometric
// progressions (w^(e0 + i d), i = 0, 1, ...). The thread looks up the start and
// the ratio in FP64 tables (computed on the host with exact integer range
// reduction), forms the powers by FP64 recurrence (relative error ~i 2^-53)
// and rounds each once to the working precision: two table lookups per
// progression instead of one per element.
#include <cmath>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "internal.h"

namespace ncf {

namespace {

constexpr int kTileElems = 4096;  // last pass (radix 4096) and the w_4096 table

template <typename R>
struct C2T;
template <>
struct C2T<float> {
    using T = float2;
};
template <>
struct C2T<double> {
    using T = double2;
};

template <typename C2>
__device__ __forceinline__ C2 cmul(C2 a, C2 b) {
    C2 r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}

template <typename C2>
__device__ __forceinline__ C2 cconj(C2 a) {
    a.y = -a.y;
    return a;
}

template <typename C2>
__device__ __forceinline__ C2 cadd(C2 a, C2 b) {
    a.x += b.x;
    a.y += b.y;
    return a;
}

template <typename C2>
__device__ __forceinline__ C2 csub(C2 a, C2 b) {
    a.x -= b.x;
    a.y -= b.y;
    return a;
}

// multiply by sign * i
template <typename C2>
__device__ __forceinline__ C2 cmul_si(C2 a, int sign) {
    C2 r;
    if (sign > 0) {
        r.x = -a.y;
        r.y = a.x;
    } else {
        r.x = a.y;
        r.y = -a.x;
    }
    return r;
}

struct PassArgs {
    void* data;          // grids: base pointer of grid 0
    int64_t grid_stride; // elements between consecutive grids (batched)
    const void* const* grids;  // optional per-grid pointers (nullptr: base + g * stride)
    int64_t N;
    int lgR;             // log2 radix of this pass
    int64_t S;           // column stride (elements)
    int64_t B;           // block size R * S
    int lgC;             // log2 columns per tile (T / R)
    int lgT;             // log2 tile elements (12 or 13)
    int64_t tiles_per_grid;  // N / T
    int64_t ntiles;          // tiles over all grids
    int64_t nblocks;         // launched workgroups (multiple of 8)
    int sign;            // +1 forward (DIF, twiddle after), -1 inverse (DIT, twiddle before)
    int lobits;
    const void* wlo;     // FP64 w_N^e, e < 2^lobits     (sign +1)
    const void* whi;     // FP64 w_N^(e << lobits)
    const void* wsmall;  // FP64 w_4096^e
};

// Global-memory element access through address-space-1 scalar pointers
// (global loads and stores rather than flat ones).
template <typename C2>
__device__ __forceinline__ C2 gld(const void* base, int64_t idx) {
    typedef decltype(C2{}.x) R;
    typedef __attribute__((address_space(1))) const R* P;
    P p = (P)base;
    C2 v;
    v.x = p[2 * idx];
    v.y = p[2 * idx + 1];
    return v;
}

template <typename C2>
__device__ __forceinline__ void gst(void* base, int64_t idx, C2 v) {
    typedef decltype(C2{}.x) R;
    typedef __attribute__((address_space(1))) R* P;
    P p = (P)base;
    p[2 * idx] = v.x;
    p[2 * idx + 1] = v.y;
}

// w_N^e (any e >= 0, reduced mod N), FP64, with the sign of the pass
__device__ __forceinline__ double2 tw_big(const PassArgs& a, int64_t e) {
    e &= a.N - 1;
    double2 w = cmul(gld<double2>(a.whi, e >> a.lobits),
                     gld<double2>(a.wlo, e & ((1LL << a.lobits) - 1)));
    return a.sign > 0 ? w : cconj(w);
}

// w_4096^e, FP64, with the sign of the pass
__device__ __forceinline__ double2 tw_small(const PassArgs& a, int e) {
    double2 w = gld<double2>(a.wsmall, e & (kTileElems - 1));
    return a.sign > 0 ? w : cconj(w);
}

template <typename C2>
__device__ __forceinline__ C2 round_tw(double2 w) {
    typedef decltype(C2{}.x) R;
    C2 r;
    r.x = (R)w.x;
    r.y = (R)w.y;
    return r;
}

// ------------------------------------------------ small DFTs in registers
// X[k] = sum_n x[n] w_r^(n k), w_r = exp(sign 2 pi i / r), in place.

template <typename C2>
__device__ __forceinline__ void dft2(C2& a0, C2& a1) {
    const C2 t = a0;
    a0 = cadd(t, a1);
    a1 = csub(t, a1);
}

template <typename C2>
__device__ __forceinline__ void dft4(C2& a0, C2& a1, C2& a2, C2& a3, int sign) {
    const C2 t0 = cadd(a0, a2);
    const C2 t1 = csub(a0, a2);
    const C2 t2 = cadd(a1, a3);
    const C2 t3 = cmul_si(csub(a1, a3), sign);
    a0 = cadd(t0, t2);
    a1 = cadd(t1, t3);
    a2 = csub(t0, t2);
    a3 = csub(t1, t3);
}

// multiply by w_16^m (m in 0..15) for the given sign; constants fold
template <typename C2>
__device__ __forceinline__ C2 mul_w16(C2 a, int m, int sign) {
    typedef decltype(a.x) R;
    const R c1 = (R)0.92387953251128674, s1 = (R)0.38268343236508978;  // pi/8
    const R c2 = (R)0.70710678118654752;                                // pi/4
    R wr, wi;
    switch (m & 15) {
        case 0: return a;
        case 1: wr = c1; wi = s1; break;
        case 2: wr = c2; wi = c2; break;
        case 3: wr = s1; wi = c1; break;
        case 4: wr = 0; wi = 1; break;
        case 5: wr = -s1; wi = c1; break;
        case 6: wr = -c2; wi = c2; break;
        case 7: wr = -c1; wi = s1; break;
        case 8: wr = -1; wi = 0; break;
        case 9: wr = -c1; wi = -s1; break;
        default: wr = -c2; wi = -c2; break;  // 10 (larger m do not occur)
    }
    if (sign < 0) wi = -wi;
    C2 w;
    w.x = wr;
    w.y = wi;
    return cmul(a, w);
}

// DFT of size 8: n = 4 n1 + n2, k = k1 + 2 k2
template <typename C2>
__device__ __forceinline__ void dft8(C2* a, int sign) {
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft2(a[n2], a[4 + n2]);
    // twiddle w_8^(n2 k1) = w_16^(2 n2 k1); k1 = 1 lives at a[4 + n2]
#pragma unroll
    for (int n2 = 1; n2 < 4; ++n2) a[4 + n2] = mul_w16(a[4 + n2], 2 * n2, sign);
    dft4(a[0], a[1], a[2], a[3], sign);  // k1 = 0 -> X[2 k2]
    dft4(a[4], a[5], a[6], a[7], sign);  // k1 = 1 -> X[1 + 2 k2]
    C2 o[8];
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) {
        o[2 * k2] = a[k2];
        o[2 * k2 + 1] = a[4 + k2];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = o[i];
}

// DFT of size 16: n = 4 n1 + n2, k = k1 + 4 k2
template <typename C2>
__device__ __forceinline__ void dft16(C2* a, int sign) {
    // inner DFT4 over n1 for each n2: inputs a[4 n1 + n2]
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4(a[n2], a[4 + n2], a[8 + n2], a[12 + n2], sign);
    // now a[4 k1 + n2] holds y[n2][k1]; twiddle w_16^(n2 k1)
#pragma unroll
    for (int k1 = 1; k1 < 4; ++k1)
#pragma unroll
        for (int n2 = 1; n2 < 4; ++n2) a[4 * k1 + n2] = mul_w16(a[4 * k1 + n2], n2 * k1, sign);
    // outer DFT4 over n2 for each k1: X[k1 + 4 k2]
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4(a[4 * k1], a[4 * k1 + 1], a[4 * k1 + 2], a[4 * k1 + 3], sign);
    // a[4 k1 + k2] = X[k1 + 4 k2]
    C2 o[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) o[k1 + 4 * k2] = a[4 * k1 + k2];
#pragma unroll
    for (int i = 0; i < 16; ++i) a[i] = o[i];
}

template <int RADIX, typename C2>
__device__ __forceinline__ void dft_r(C2* a, int sign) {
    if constexpr (RADIX == 16) {
        dft16(a, sign);
    } else if constexpr (RADIX == 8) {
        dft8(a, sign);
    } else if constexpr (RADIX == 4) {
        dft4(a[0], a[1], a[2], a[3], sign);
    } else {
        dft2(a[0], a[1]);
    }
}

__device__ __forceinline__ int lds_pad(int e) { return e + (e >> 4); }

// One Stockham stage of radix RADIX over the tile's C columns of length R.
// Each thread owns 16 / RADIX butterflies (16 elements). Inputs come from
// `src` (global or LDS view), outputs go to `dst`.
template <int RADIX, bool FROM_GLOBAL, bool TO_GLOBAL, int LGR, int NS, int LGT, typename C2>
__device__ __forceinline__ void stockham_stage(const PassArgs& a, C2* lds, C2* gbase,
                                               int64_t s0) {
    constexpr int kThreads = 1 << (LGT - 4);  // 16 elements per thread
    constexpr int NB = 16 / RADIX;  // butterflies per thread
    constexpr int lgC = LGT - LGR;
    constexpr int R = 1 << LGR;
    constexpr int C = 1 << lgC;
    constexpr int Rr = R / RADIX;
    constexpr int Ns = NS;
    const int tid = threadIdx.x;
    C2 v[16];
    int jj[NB], cc[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int beta = tid + u * kThreads;
        const int c = beta & (C - 1);
        const int j = beta >> lgC;
        jj[u] = j;
        cc[u] = c;
#pragma unroll
        for (int i = 0; i < RADIX; ++i) {
            const int row = j + i * Rr;
            v[u * RADIX + i] = FROM_GLOBAL ? gld<C2>(gbase, (int64_t)row * a.S + c)
                                           : lds[lds_pad(row * C + c)];
        }
        if (FROM_GLOBAL && a.sign < 0) {
            // adjoint of the forward pass twiddle, applied before the DFT:
            // w^(E row), rows j + i Rr, E = (s0 + c) N / B
            const int64_t E = (s0 + c) * (a.N / a.B);
            double2 t = tw_big(a, E * j);
            const double2 d = tw_big(a, E * Rr);
#pragma unroll
            for (int i = 0; i < RADIX; ++i) {
                if (i) t = cmul(t, d);
                v[u * RADIX + i] = cmul(v[u * RADIX + i], round_tw<C2>(t));
            }
        }
        // stage twiddles w_{Ns r}^(i k), k = j mod Ns: powers of w_4096^(k step)
        const int k = j & (Ns - 1);
        if (Ns > 1 && k) {
            const int step = kTileElems / (Ns * RADIX);
            const double2 d = tw_small(a, k * step);
            double2 t = d;
#pragma unroll
            for (int i = 1; i < RADIX; ++i) {
                if (i > 1) t = cmul(t, d);
                v[u * RADIX + i] = cmul(v[u * RADIX + i], round_tw<C2>(t));
            }
        }
        dft_r<RADIX>(v + u * RADIX, a.sign);
    }
    // all reads of this stage are done before any write (the tile is
    // transformed in place, in LDS or in HBM)
    if (!FROM_GLOBAL || TO_GLOBAL) __syncthreads();
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int j = jj[u], c = cc[u];
        const int k = j & (Ns - 1);
        const int obase = (j / Ns) * Ns * RADIX + k;
        if (TO_GLOBAL && a.sign > 0) {
            // pass twiddle w^(E row), rows obase + i Ns, E = (s0 + c) N / B
            const int64_t E = (s0 + c) * (a.N / a.B);
            double2 t = tw_big(a, E * obase);
            const double2 d = tw_big(a, E * Ns);
#pragma unroll
            for (int i = 0; i < RADIX; ++i) {
                if (i) t = cmul(t, d);
                v[u * RADIX + i] = cmul(v[u * RADIX + i], round_tw<C2>(t));
            }
        }
#pragma unroll
        for (int i = 0; i < RADIX; ++i) {
            const int row = obase + i * Ns;
            if (TO_GLOBAL)
                gst<C2>(gbase, (int64_t)row * a.S + c, v[u * RADIX + i]);
            else
                lds[lds_pad(row * C + c)] = v[u * RADIX + i];
        }
    }
    if (!TO_GLOBAL) __syncthreads();  // outputs visible to the next stage
}

// Radix schedule of a column of length R = 2^LGR: radix-16 stages first, then
// one stage of 8, 4 or 2 for the remainder; fixed at compile time.
template <int LGR, int ST, int NS, int LGT, typename C2>
__device__ __forceinline__ void run_stages(const PassArgs& a, C2* lds, C2* gbase,
                                           int64_t s0) {
    constexpr int n16 = LGR / 4;
    constexpr int rem = LGR % 4;
    constexpr int nst = n16 + (rem ? 1 : 0);
    if constexpr (ST < nst) {
        constexpr int RX = ST < n16 ? 16 : (1 << rem);
        stockham_stage<RX, ST == 0, ST == nst - 1, LGR, NS, LGT>(a, lds, gbase, s0);
        run_stages<LGR, ST + 1, NS * RX, LGT>(a, lds, gbase, s0);
    }
}

template <typename Real, int LGR, int LGT>
__global__ void __launch_bounds__(1 << (LGT - 4))
k_fft_pass(PassArgs a) {
    using C2 = typename C2T<Real>::T;
    constexpr int lgC = LGT - LGR;
    constexpr int kElems = 1 << LGT;
    __shared__ C2 buf[kElems + kElems / 16];
    const int64_t wg = blockIdx.x;
    if (wg >= a.ntiles) return;
    const int64_t gidx = wg / a.tiles_per_grid;
    const int64_t tile = wg % a.tiles_per_grid;
    C2* data = a.grids ? reinterpret_cast<C2*>(const_cast<void*>(a.grids[gidx]))
                       : reinterpret_cast<C2*>(a.data) + gidx * a.grid_stride;
    // tile -> (block, first column)
    const int64_t chunks_per_block = a.S >> lgC;  // S / C
    const int64_t blk = tile / chunks_per_block;
    const int64_t s0 = (tile % chunks_per_block) << lgC;
    C2* base = data + blk * a.B + s0;
    run_stages<LGR, 0, 1, LGT>(a, buf, base, s0);
}

template <typename Real>
using PassKernel = void (*)(PassArgs);

template <typename Real, int LGT>
PassKernel<Real> pass_kernel_t(int lgR) {
    switch (lgR) {
        case 1: return k_fft_pass<Real, 1, LGT>;
        case 2: return k_fft_pass<Real, 2, LGT>;
        case 3: return k_fft_pass<Real, 3, LGT>;
        case 4: return k_fft_pass<Real, 4, LGT>;
        case 5: return k_fft_pass<Real, 5, LGT>;
        case 6: return k_fft_pass<Real, 6, LGT>;
        case 7: return k_fft_pass<Real, 7, LGT>;
        case 8: return k_fft_pass<Real, 8, LGT>;
        case 9: return k_fft_pass<Real, 9, LGT>;
        case 10: return k_fft_pass<Real, 10, LGT>;
        case 11: return k_fft_pass<Real, 11, LGT>;
        default: return k_fft_pass<Real, 12, LGT>;
    }
}

// radix 2^lgR on tiles of 2^lgT elements (lgT = 13 only for strided passes)
template <typename Real>
PassKernel<Real> pass_kernel(int lgR, int lgT) {
    if constexpr (sizeof(Real) == 4) {
        if (lgT == 13 && lgR <= 11) return pass_kernel_t<Real, 13>(lgR);
    }
    return pass_kernel_t<Real, 12>(lgR);
}

struct TwKey {
    int64_t N;
    bool fp64;
    int device;
    bool operator<(const TwKey& o) const {
        if (N != o.N) return N < o.N;
        if (fp64 != o.fp64) return fp64 < o.fp64;
        return device < o.device;
    }
};
struct TwVal {
    void* lo;
    void* hi;
    void* small;
    int lobits;
};
std::mutex g_tw_mu;
std::map<TwKey, TwVal> g_tw;

int ilog2(int64_t n) {
    int l = 0;
    while ((1LL << l) < n) ++l;
    return l;
}

template <typename R>
int upload_table(const std::vector<double>& re_im, void** out, hipStream_t st) {
    size_t n = re_im.size() / 2;
    std::vector<R> h(re_im.size());
    for (size_t i = 0; i < re_im.size(); ++i) h[i] = (R)re_im[i];
    void* d = nullptr;
    NCF_TRY_HIP(hipMalloc(&d, sizeof(R) * 2 * n));
    NCF_TRY_HIP(hipMemcpyAsync(d, h.data(), sizeof(R) * 2 * n, hipMemcpyHostToDevice, st));
    NCF_TRY_HIP(hipStreamSynchronize(st));
    *out = d;
    return NCF_OK;
}

// w_M^(e * mult) for e < count, FP64: exp(+2 pi i e mult / M) with exact
// integer range reduction of the exponent.
std::vector<double> twiddles(int64_t M, int64_t count, int64_t mult) {
    std::vector<double> v(2 * count);
    for (int64_t e = 0; e < count; ++e) {
        const int64_t ex = (int64_t)(((__int128)e * mult) % M);
        const double ang = 2.0 * M_PI * (double)ex / (double)M;
        v[2 * e] = std::cos(ang);
        v[2 * e + 1] = std::sin(ang);
    }
    return v;
}

}  // namespace

int fft_plan(int64_t N, bool fp64, FftPlan* plan, hipStream_t st, const FftVariant& var) {
    if (N < kTileElems || (N & (N - 1)) || N > (1LL << 31)) {
        set_error("fft: N = %lld must be a power of two in [4096, 2^31]", (long long)N);
        return NCF_E_INVALID_ARG;
    }
    const int p = ilog2(N);
    const int r = p - 12;  // log2 of the strided part
    plan->N = N;
    if (p == 12) {
        plan->npass = 1;
        plan->radix[0] = 4096;
    } else if (p <= 22 && !(var.split == 2 && r >= 2)) {
        plan->npass = 2;
        plan->radix[0] = 1 << r;
        plan->radix[1] = 4096;
    } else {
        plan->npass = 3;
        int a = (r + 1) / 2, b = r / 2;  // larger strided radix first
        if (var.split == 1) std::swap(a, b);
        plan->radix[0] = 1 << a;
        plan->radix[1] = 1 << b;
        plan->radix[2] = 4096;
    }
    int64_t B = N;
    for (int i = 0; i < plan->npass; ++i) {
        plan->stride[i] = B / plan->radix[i];
        B = plan->stride[i];
        // strided passes of the FP32 transform move 8192-element tiles
        int lgt = (i < plan->npass - 1 && !fp64) ? 13 : 12;
        if (i < plan->npass - 1 && var.lgt_strided == 12) lgt = 12;
        if (i < plan->npass - 1 && var.lgt_strided == 13 && !fp64) lgt = 13;
        plan->lgt[i] = lgt;
    }
    int dev = 0;
    NCF_TRY_HIP(hipGetDevice(&dev));
    TwKey key{N, fp64, dev};
    std::lock_guard<std::mutex> lock(g_tw_mu);
    auto it = g_tw.find(key);
    if (it == g_tw.end()) {
        TwVal v;
        v.lobits = (p + 1) / 2;
        const int64_t nlo = 1LL << v.lobits;
        const int64_t nhi = N >> v.lobits;
        auto lo = twiddles(N, nlo, 1);
        auto hi = twiddles(N, nhi, nlo);
        auto sm = twiddles(kTileElems, kTileElems, 1);
        NCF_TRY(upload_table<double>(lo, &v.lo, st));
        NCF_TRY(upload_table<double>(hi, &v.hi, st));
        NCF_TRY(upload_table<double>(sm, &v.small, st));
        it = g_tw.emplace(key, v).first;
    }
    plan->lobits = it->second.lobits;
    plan->wlo = it->second.lo;
    plan->whi = it->second.hi;
    plan->small = it->second.small;
    return NCF_OK;
}

int64_t fft_position(const FftPlan& plan, int64_t k) {
    // k = sum_i d_i * (R_1..R_{i-1}),  p = sum_i d_i * (N / (R_1..R_i))
    int64_t p = 0, below = 1, above = plan.N;
    for (int i = 0; i < plan.npass; ++i) {
        const int64_t d = (k / below) % plan.radix[i];
        above /= plan.radix[i];
        p += d * above;
        below *= plan.radix[i];
    }
    return p;
}

int fft_exec(const FftPlan& plan, void* const* d_grids, int count, int sign, bool fp64,
             hipStream_t st) {
    if (count <= 0) return NCF_OK;
    PassArgs a{};
    a.data = nullptr;
    a.grid_stride = 0;
    a.grids = reinterpret_cast<const void* const*>(d_grids);
    a.N = plan.N;
    a.sign = sign;
    a.lobits = plan.lobits;
    a.wlo = plan.wlo;
    a.whi = plan.whi;
    a.wsmall = plan.small;
    const double bytes = 2.0 * (fp64 ? 16.0 : 8.0) * (double)plan.N * count;
    for (int q = 0; q < plan.npass; ++q) {
        const int i = sign > 0 ? q : plan.npass - 1 - q;
        a.lgR = ilog2(plan.radix[i]);
        a.lgT = plan.lgt[i];
        a.lgC = a.lgT - a.lgR;
        a.S = plan.stride[i];
        a.B = a.S * plan.radix[i];
        a.tiles_per_grid = plan.N >> a.lgT;
        a.ntiles = a.tiles_per_grid * count;
        a.nblocks = round_up(a.ntiles, kXcds);
        const unsigned threads = 1u << (a.lgT - 4);
        ProfScope p(st, fp64 ? "fft_pass_f64" : "fft_pass_f32", bytes, "bytes");
        if (fp64)
            hipLaunchKernelGGL(pass_kernel<double>(a.lgR, a.lgT), dim3((unsigned)a.nblocks),
                               dim3(threads), 0, st, a);
        else
            hipLaunchKernelGGL(pass_kernel<float>(a.lgR, a.lgT), dim3((unsigned)a.nblocks),
                               dim3(threads), 0, st, a);
        NCF_CHECK_LAUNCH();
    }
    return NCF_OK;
}

}  // namespace ncf
