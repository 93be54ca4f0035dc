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
// A workgroup transforms one tile of 4096 elements: R_i rows by
// C_i = 4096 / R_i adjacent columns (C_i * element size contiguous bytes per
// row in HBM), held in LDS; each column's DFT is a Stockham autosort
// sequence of radix-4 (and one radix-2) stages. Twiddles come from tables
// computed in FP64 on the host and rounded once to the working precision.
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "internal.h"

namespace ncf {

namespace {

constexpr int kThreads = 256;
constexpr int kTileElems = 4096;

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
    int lgC;             // log2 columns per tile (4096 / R)
    int64_t tiles_per_grid;  // N / 4096
    int64_t ntiles;          // tiles over all grids
    int64_t nblocks;         // launched workgroups (multiple of 8)
    int sign;            // +1 forward (DIF, twiddle after), -1 inverse (DIT, twiddle before)
    int lobits;
    const void* wlo;     // w_N^e, e < 2^lobits     (sign +1)
    const void* whi;     // w_N^(e << lobits)
    const void* wsmall;  // w_4096^e
};

template <typename C2>
__device__ __forceinline__ C2 tw_big(const PassArgs& a, int64_t e) {
    // w_N^e for 0 <= e < N, with the sign of the pass
    const C2* lo = reinterpret_cast<const C2*>(a.wlo);
    const C2* hi = reinterpret_cast<const C2*>(a.whi);
    C2 w = cmul(hi[e >> a.lobits], lo[e & ((1LL << a.lobits) - 1)]);
    return a.sign > 0 ? w : cconj(w);
}

template <typename C2>
__device__ __forceinline__ C2 tw_small(const PassArgs& a, int e) {
    const C2* sm = reinterpret_cast<const C2*>(a.wsmall);
    C2 w = sm[e & (kTileElems - 1)];
    return a.sign > 0 ? w : cconj(w);
}

template <typename Real>
__global__ void __launch_bounds__(kThreads)
k_fft_pass(PassArgs a) {
    using C2 = typename C2T<Real>::T;
    __shared__ C2 buf[kTileElems];
    const int64_t wg = xcd_remap(blockIdx.x, a.nblocks);
    if (wg >= a.ntiles) return;
    const int tid = threadIdx.x;
    const int64_t gidx = wg / a.tiles_per_grid;
    const int64_t tile = wg % a.tiles_per_grid;
    C2* data = a.grids ? reinterpret_cast<C2*>(const_cast<void*>(a.grids[gidx]))
                       : reinterpret_cast<C2*>(a.data) + gidx * a.grid_stride;
    const int R = 1 << a.lgR;
    const int C = 1 << a.lgC;
    // tile -> (block, first column)
    const int64_t chunks_per_block = a.S >> a.lgC;  // S / C
    const int64_t blk = tile / chunks_per_block;
    const int64_t s0 = (tile % chunks_per_block) << a.lgC;
    C2* base = data + blk * a.B + s0;

    // load: element (r, c) at base + r*S + c  ->  buf[c*R + r]
    for (int e = tid; e < kTileElems; e += kThreads) {
        const int r = e >> a.lgC;
        const int c = e & (C - 1);
        C2 v = base[(int64_t)r * a.S + c];
        if (a.sign < 0) {
            // DIT: input index r is the frequency digit k of the forward pass
            const int64_t ex = (s0 + c) * (int64_t)r * (a.N / a.B);
            if (ex) v = cmul(v, tw_big<C2>(a, ex));
        }
        buf[c * R + r] = v;
    }
    __syncthreads();

    // Stockham stages on each column (length R): radix-2 first if lgR is odd
    int Ns = 1;
    if (a.lgR & 1) {
        // radix-2: C*R/2 = 2048 butterflies, 8 per thread
        C2 va[8][2];
        int dst[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int beta = tid + u * kThreads;
            const int c = beta >> (a.lgR - 1);
            const int j = beta & ((R >> 1) - 1);
            C2* col = buf + c * R;
            C2 x0 = col[j];
            C2 x1 = col[j + (R >> 1)];
            // Ns = 1: no twiddle
            va[u][0] = cadd(x0, x1);
            va[u][1] = csub(x0, x1);
            dst[u] = c * R + j * 2;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            buf[dst[u]] = va[u][0];
            buf[dst[u] + 1] = va[u][1];
        }
        __syncthreads();
        Ns = 2;
    }
    const int lgR4 = a.lgR - 2;  // log2(R/4)
    for (; Ns < R; Ns <<= 2) {
        C2 va[4][4];
        int dst[4];
        // twiddle step in units of w_4096: w_{4 Ns}^1 = w_4096^(4096 / (4 Ns))
        const int step = kTileElems / (4 * Ns);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int beta = tid + u * kThreads;
            const int c = beta >> lgR4;
            const int j = beta & ((R >> 2) - 1);
            C2* col = buf + c * R;
            const int k = j & (Ns - 1);
            const int q = R >> 2;
            C2 x0 = col[j];
            C2 x1 = col[j + q];
            C2 x2 = col[j + 2 * q];
            C2 x3 = col[j + 3 * q];
            if (k) {
                x1 = cmul(x1, tw_small<C2>(a, k * step));
                x2 = cmul(x2, tw_small<C2>(a, 2 * k * step));
                x3 = cmul(x3, tw_small<C2>(a, 3 * k * step));
            }
            const C2 t0 = cadd(x0, x2);
            const C2 t1 = csub(x0, x2);
            const C2 t2 = cadd(x1, x3);
            const C2 t3 = cmul_si(csub(x1, x3), a.sign);
            va[u][0] = cadd(t0, t2);
            va[u][1] = cadd(t1, t3);
            va[u][2] = csub(t0, t2);
            va[u][3] = csub(t1, t3);
            dst[u] = c * R + (j / Ns) * Ns * 4 + k;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            buf[dst[u]] = va[u][0];
            buf[dst[u] + Ns] = va[u][1];
            buf[dst[u] + 2 * Ns] = va[u][2];
            buf[dst[u] + 3 * Ns] = va[u][3];
        }
        __syncthreads();
    }

    // store: buf[c*R + k] -> base + k*S + c (DIF: twiddle w_B^(s k) first)
    for (int e = tid; e < kTileElems; e += kThreads) {
        const int k = e >> a.lgC;
        const int c = e & (C - 1);
        C2 v = buf[c * R + k];
        if (a.sign > 0) {
            const int64_t ex = (s0 + c) * (int64_t)k * (a.N / a.B);
            if (ex) v = cmul(v, tw_big<C2>(a, ex));
        }
        base[(int64_t)k * a.S + c] = v;
    }
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

int fft_plan(int64_t N, bool fp64, FftPlan* plan, hipStream_t st) {
    if (N < kTileElems || (N & (N - 1)) || N > (1LL << 31)) {
        set_error("fft: N = %lld must be a power of two in [4096, 2^31]", (long long)N);
        return NCF_E_INVALID_ARG;
    }
    const int p = ilog2(N);
    plan->N = N;
    if (p == 12) {
        plan->npass = 1;
        plan->radix[0] = 4096;
    } else if (p <= 22) {
        plan->npass = 2;
        plan->radix[0] = 1 << (p - 12);
        plan->radix[1] = 4096;
    } else {
        plan->npass = 3;
        const int r = p - 12;
        plan->radix[0] = 1 << ((r + 1) / 2);
        plan->radix[1] = 1 << (r / 2);
        plan->radix[2] = 4096;
    }
    int64_t B = N;
    for (int i = 0; i < plan->npass; ++i) {
        plan->stride[i] = B / plan->radix[i];
        B = plan->stride[i];
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
        if (fp64) {
            NCF_TRY(upload_table<double>(lo, &v.lo, st));
            NCF_TRY(upload_table<double>(hi, &v.hi, st));
            NCF_TRY(upload_table<double>(sm, &v.small, st));
        } else {
            NCF_TRY(upload_table<float>(lo, &v.lo, st));
            NCF_TRY(upload_table<float>(hi, &v.hi, st));
            NCF_TRY(upload_table<float>(sm, &v.small, st));
        }
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
    a.tiles_per_grid = plan.N / kTileElems;
    a.ntiles = a.tiles_per_grid * count;
    a.nblocks = round_up(a.ntiles, kXcds);
    a.sign = sign;
    a.lobits = plan.lobits;
    a.wlo = plan.wlo;
    a.whi = plan.whi;
    a.wsmall = plan.small;
    const double bytes = 2.0 * (fp64 ? 16.0 : 8.0) * (double)plan.N * count;
    for (int q = 0; q < plan.npass; ++q) {
        const int i = sign > 0 ? q : plan.npass - 1 - q;
        a.lgR = ilog2(plan.radix[i]);
        a.lgC = 12 - a.lgR;
        a.S = plan.stride[i];
        a.B = a.S * plan.radix[i];
        ProfScope p(st, fp64 ? "fft_pass_f64" : "fft_pass_f32", bytes, "bytes");
        if (fp64)
            hipLaunchKernelGGL(k_fft_pass<double>, dim3((unsigned)a.nblocks), dim3(kThreads), 0,
                               st, a);
        else
            hipLaunchKernelGGL(k_fft_pass<float>, dim3((unsigned)a.nblocks), dim3(kThreads), 0,
                               st, a);
        NCF_CHECK_LAUNCH();
    }
    return NCF_OK;
}

}  // namespace ncf
