// fft_tile.h -- tile-level building blocks of the power-of-two FFT: complex
// helpers, pass arguments and twiddle tables, register DFTs of size 2-16 and
// the Stockham stages that transform one 4096- or 8192-element tile through
// registers and padded LDS. Used by the FFT passes and by the fused
// last-pass / product / first-inverse-pass kernel of the spectral route.
#pragma once

#include "internal.h"

namespace ncf {
namespace fftk {

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
// Each thread owns EPT / RADIX butterflies (EPT elements, 16 unless a
// caller asks for fewer). Inputs come from `src` (global or LDS view),
// outputs go to `dst`.
// tid: the thread's index among the 2^LGT / EPT threads of the tile. `on`
// false: the thread does no work and only meets the stage's barriers, which
// lie outside the work it skips.
template <int RADIX, bool FROM_GLOBAL, bool TO_GLOBAL, int LGR, int NS, int LGT, int EPT = 16,
          typename C2>
__device__ __forceinline__ void stockham_stage(const PassArgs& a, C2* lds, C2* gbase, int64_t s0,
                                               int tid, bool on = true) {
    static_assert(RADIX <= EPT && EPT <= 16, "a thread holds whole butterflies");
    constexpr int kThreads = (1 << LGT) / EPT;  // EPT elements per thread
    constexpr int NB = EPT / RADIX;             // butterflies per thread
    constexpr int lgC = LGT - LGR;
    constexpr int R = 1 << LGR;
    constexpr int C = 1 << lgC;
    constexpr int Rr = R / RADIX;
    constexpr int Ns = NS;
    C2 v[EPT];
    int jj[NB], cc[NB];
#pragma unroll
    for (int u = 0; u < NB && on; ++u) {
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
    for (int u = 0; u < NB && on; ++u) {
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
        stockham_stage<RX, ST == 0, ST == nst - 1, LGR, NS, LGT>(a, lds, gbase, s0,
                                                                  (int)threadIdx.x);
        run_stages<LGR, ST + 1, NS * RX, LGT>(a, lds, gbase, s0);
    }
}

// Stages of one tile column of length 2^LGR, as run_stages, with the source
// of the first stage (global memory or LDS) and the destination of the last
// (global memory or LDS) chosen at compile time; EPT elements per thread
// (radix-EPT stages, then one for the remainder).
template <int LGR, int ST, int NS, int LGT, bool G_IN, bool G_OUT, int EPT = 16, typename C2>
__device__ __forceinline__ void run_stages_io(const PassArgs& a, C2* lds, C2* gbase, int64_t s0,
                                              int tid, bool on = true) {
    constexpr int lgE = __builtin_ctz(EPT);
    constexpr int nbig = LGR / lgE;
    constexpr int rem = LGR % lgE;
    constexpr int nst = nbig + (rem ? 1 : 0);
    if constexpr (ST < nst) {
        constexpr int RX = ST < nbig ? EPT : (1 << rem);
        stockham_stage<RX, G_IN && ST == 0, G_OUT && ST == nst - 1, LGR, NS, LGT, EPT>(
            a, lds, gbase, s0, tid, on);
        run_stages_io<LGR, ST + 1, NS * RX, LGT, G_IN, G_OUT, EPT>(a, lds, gbase, s0, tid, on);
    }
}

// The workgroup barriers of run_stages_io without its work: threads with no
// tile to transform call this so that the barriers stay matched.
template <int LGR, int ST, bool G_IN, bool G_OUT>
__device__ __forceinline__ void run_stages_idle() {
    constexpr int n16 = LGR / 4;
    constexpr int rem = LGR % 4;
    constexpr int nst = n16 + (rem ? 1 : 0);
    if constexpr (ST < nst) {
        constexpr bool from_g = G_IN && ST == 0, to_g = G_OUT && ST == nst - 1;
        if (!from_g || to_g) __syncthreads();
        if (!to_g) __syncthreads();
        run_stages_idle<LGR, ST + 1, G_IN, G_OUT>();
    }
}

}  // namespace fftk
}  // namespace ncf
