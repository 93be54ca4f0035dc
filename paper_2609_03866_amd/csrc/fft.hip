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

#include "fft_tile.h"

namespace ncf {

namespace {

using namespace fftk;

template <typename Real, int LGR, int LGT>
__global__ void __launch_bounds__(1 << (LGT - 4))
k_fft_pass(PassArgs a) {
    using C2 = typename C2T<Real>::T;
    constexpr int lgC = LGT - LGR;
    constexpr int kElems = 1 << LGT;
    __shared__ C2 buf[kElems + kElems / 16];
    // XCD-aware order: each XCD takes a contiguous run of tiles (adjacent
    // column chunks of the same rows)
    const int64_t wg = xcd_remap(blockIdx.x, a.nblocks);
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
             hipStream_t st, bool skip_tile_pass) {
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
        if (skip_tile_pass && i == plan.npass - 1) continue;
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
