// internal.h -- shared declarations of the ncf HIP library (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstddef>

#include "ncf.h"

namespace ncf {

// ----------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
void clear_error();

#define NCF_TRY_HIP(call)                                                              \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            ::ncf::set_error("%s:%d %s: %s", __FILE__, __LINE__, #call,                \
                             hipGetErrorString(e_));                                   \
            return NCF_E_DEVICE;                                                       \
        }                                                                              \
    } while (0)

#define NCF_TRY(expr)              \
    do {                           \
        int st_ = (expr);          \
        if (st_ != NCF_OK) return st_; \
    } while (0)

// Check the launch that was just enqueued.
#define NCF_CHECK_LAUNCH() NCF_TRY_HIP(hipGetLastError())

// -------------------------------------------------------------- profiling
// Bracket a kernel launch with HIP events on `stream` when profiling is on.
struct ProfScope {
    ProfScope(hipStream_t stream, const char* name, double work, const char* unit);
    ~ProfScope();
    hipStream_t stream;
    const char* name;
    double work;
    const char* unit;
    void* ev0;
};

// ------------------------------------------------------------ constants
constexpr double kFloor = 1e-16;        // pair-count floor (PairCount algorithms)
constexpr int kWarp = 64;               // CDNA wavefront
constexpr int kXcds = 8;                // MI355X accelerator complex dies

// XCD-aware block index: consecutive logical tiles land on the same XCD
// (hardware dispatches workgroup b to XCD b % 8). `nblocks` is the launched
// grid (a multiple of 8); the result is a bijection of [0, nblocks).
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nblocks) {
    int64_t per = nblocks / kXcds;
    return (b % kXcds) * per + b / kXcds;
}

// Global-memory views of device pointers: accesses through them compile to
// global (not flat) memory instructions, which do not wait on LDS traffic.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> gbl(T* p) {
    return (gptr<T>)p;
}

// First index i in [0, n) with (upper ? a[i] > key : a[i] >= key), else n.
// Called by a whole wavefront: 64 probes per round. `a` is in global memory.
template <typename T>
__device__ __forceinline__ int64_t wave_search(const T* a_, int64_t n, T key, bool upper) {
    const gptr<const T> a = gbl(a_);
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

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ------------------------------------------- digit-reversed positions
// Radices of a transform plan (first pass first): the forward transform
// leaves frequency k at position p with p = sum_i d_i 2^(lgN - B_i) where
// k = sum_i d_i 2^(B_{i-1}) and B_i is the bit count of the first i radices.
struct RadixInfo {
    int npass;
    int lg[4];  // log2 radix of each pass (first pass first)
    int lgN;
};

__device__ __forceinline__ int64_t freq_of_pos(int64_t p, const RadixInfo& ri) {
    // p = sum_i d_i * 2^(lgN - B_i), k = sum_i d_i * 2^(B_{i-1}); at most four
    // passes, unrolled so that the radix table stays in registers
    int64_t k = 0;
    int B = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (i < ri.npass) {
            const int lg = ri.lg[i];
            const int64_t d = (p >> (ri.lgN - B - lg)) & ((1LL << lg) - 1);
            k |= d << B;
            B += lg;
        }
    }
    return k;
}

__device__ __forceinline__ int64_t pos_of_freq(int64_t k, const RadixInfo& ri) {
    int64_t p = 0;
    int B = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (i < ri.npass) {
            const int lg = ri.lg[i];
            const int64_t d = (k >> B) & ((1LL << lg) - 1);
            p |= d << (ri.lgN - B - lg);
            B += lg;
        }
    }
    return p;
}

// ------------------------------------------------------------- call I/O
// The caller's value arrays and output arrays of one call. Kernels reach
// them through this device block, so a recorded launch sequence (a plan) can
// run again on other buffers once the block is rewritten.
struct IoBlock {
    const double* x[2];  // values of set 0 and set 1, concatenated over series
    double* c;           // [problems][K]
    double* b;           // [problems][K]
    int64_t* count;      // [problems][K] or null
    int32_t* status;     // [problems]
};
// Write `v` into the device block `dst` on `st` (a one-thread kernel, so the
// values are taken at enqueue time).
int launch_set_io(IoBlock* dst, const IoBlock& v, hipStream_t st);

// ----------------------------------------------------------- A1 moments
struct SeriesDesc {
    const double* t;  // times and optional errors of this series
    int64_t xoff;     // first value of this series in IoBlock::x[set]
    const double* err;
    float* v32;       // outputs, each may be null: w (x - mean)/sd in FP32 / FP64,
    double* v64;      // weights, and FP64 prefix sums of v and w (n + 1 entries),
    double* w64;      // and the prefix count of samples with a nonzero weight
    double* pv;       // (exact integers in FP64: a window holding no sample of
    double* pw;       // nonzero weight is empty whatever its weight prefix says)
    double* pz;
    int64_t n;        // samples
    int32_t chunk0;   // first chunk of the series
    int32_t nchunk;   // chunks of the series
    int32_t set;      // value array of the series (IoBlock::x index)
    int32_t wmode;    // 1: err holds sample weights w >= 0 directly (else errors, w = 1/err^2)
};

// Smallest lag-0 scale that is not degenerate: r(0) of standardized values
// is of order 1, and when a kernel holds every pair of a short series the
// lag-0 sum (sum of z)^2 is 0 exactly, so its rounding (either sign) must not
// decide the status. CCF: each series' r(0) in magnitude, and the product > 0.
constexpr double kMinScale = 1e-12;
// Mixed precision, Gaussian kernel: a problem whose smallest lag-0 scale is
// below this value is evaluated again in FP64. The FP32 kernel weights and
// transforms leave an error of about 1e-6 relative on the lag-0 sums, and c
// divides by the scale, so its error grows as 1/r(0) when the lag-0 sums
// cancel (a kernel wide against the series).
constexpr double kPromoteScale = 0.1;
// Series shorter than this take the direct window sums on any route: with a
// few samples under a wide kernel, the rounding of the transforms, measured
// against the lag-0 pair sums, is far above its usual size.
constexpr int64_t kMinSpectralSamples = 32;
constexpr int64_t kMomentChunk = 2048;  // samples per moments chunk (8 per thread)
constexpr int kChunkPart = 5;           // partial moments per chunk (MomentsArgs)
constexpr int64_t kQueueAutoItems = 100000;  // Gaussian window launches this large pull items from a queue

struct Chunk {
    int64_t begin, end;  // sample range [begin, end) within the series
    int32_t series;
    int32_t pad;
};

struct SeriesStat {
    double mean, sd, sw;  // weighted mean, sd (ddof 0), sum of weights
    double sw2;           // sum of squared weights
    double tmin, tmax;
    int32_t status;       // NCF_OK or a negative NCF_E_* code
    int32_t pad;
};

struct MomentsArgs {
    const SeriesDesc* series;
    const Chunk* chunks;
    int32_t nseries, nchunks;
    double* chunk_part;      // kChunkPart doubles per chunk: sw, mean, M2, flags, sum w^2
    double* chunk_tot;       // 3 doubles per chunk (v, w, nonzero-weight count): chunk totals,
                             // then (chunk-offset pass) the exclusive sums of the preceding
                             // chunks of the series, which readers of the chunk-local prefix
                             // sums add
    SeriesStat* stats;       // nseries
    const IoBlock* io;       // value arrays
    int32_t prefix;          // any series has prefix outputs
    int32_t pad;
    const double* lag_src;   // optional: lags copied to lag_dst by the finalize
    double* lag_dst;         // kernel (next to the statistics, one readback)
    int64_t nlag;
};

int launch_moments(const MomentsArgs& a, hipStream_t st);
int launch_standardize(const MomentsArgs& a, hipStream_t st);
// Fill p[0..n) with alternating +1, -1 (finite values of unit variance).
int launch_fill_alternating(double* p, int64_t n, hipStream_t st);
// One segment of a gather or scatter: len values from src + src_off to
// dst + dst_off.
struct CopySeg {
    int64_t src_off, dst_off, len;
};
// Copy the segments (device table, nseg entries) of up to three arrays that
// share them: s[a] -> d[a] for every a whose s[a] is not null.
int launch_copy_segments(const CopySeg* d_segs, int64_t nseg, const double* const s[3],
                         double* const d[3], hipStream_t st);

// --------------------------------------------------- replicate statistics
// Replicate r of a series of n samples: values x + sigma z_r (z_r: R x n,
// row-major) and weights mult_r (x 1/err^2 when err is given). Either part
// may be absent (sigma/z null: the values are copied; mult and err null: no
// weights are written).
int launch_resample_prep(int64_t n, int64_t R, const double* x, const double* sigma,
                         const double* z, const double* err, const int32_t* mult, double* xr,
                         double* wr, hipStream_t st);
// Per lag, the mean and sample standard deviation (n - 1) of the replicate
// estimates c_rep[R][K] over the replicates whose estimate is a number.
int launch_resample_stats(const double* c_rep, int64_t R, int64_t K, double* c_mean,
                          double* c_sd, hipStream_t st);

// ------------------------------------------------------- A7 window scan
enum WinFlags : uint32_t {
    WIN_RECT = 1u,       // rectangle kernel (else Gaussian)
    WIN_NUMER = 2u,      // also accumulate the numerator C (Gaussian: direct sum)
    WIN_WEIGHTED = 4u,   // accumulate the weighted pair sum B separately
    WIN_EXP64 = 8u,      // Gaussian weights in FP64 (else FP32 exp of FP64 differences)
};

struct WinTask {
    // window array (series 1 of a CCF, the series itself for an ACF)
    const double* t;
    const double* v;     // FP64 values (Gaussian numerator) or null
    const double* w;     // FP64 weights or null
    const double* pv;    // prefix of v (n_win + 1) or null
    const double* pw;    // prefix of w (n_win + 1) or null
    const double* pz;    // prefix count of nonzero weights (n_win + 1), weighted rectangle
    // prefix sums above are chunk-local (kMomentChunk samples): entry j >= 1
    // adds poff[3 c + q] (q = 0 values, 1 weights, 2 counts) of chunk
    // c = (j - 1) / kMomentChunk, the exclusive sum of the preceding chunks
    const double* poff;
    int64_t n_win;
    // outer array (series 2 of a CCF)
    const double* s;
    const double* vo;
    const double* wo;
    int64_t n_out;
    const double* delta; // K sorted lag offsets eps * tau
    int32_t K;
    int32_t J;           // outer samples per workgroup
    int32_t n_jt, n_kt;  // tiles
    int32_t G;           // j-tiles per work item (a j-group)
    int32_t n_jg;        // j-groups: ceil(n_jt / G)
    double h;            // bandwidth
    double W;            // window half-width: 6h (Gaussian) or h (rectangle)
    double* part;        // [n_jg][K][4] partial sums: C, B, b, count (count as bits);
                         // weighted rectangle: b holds the count of pairs of two
                         // nonzero weights (the window is empty when it is 0)
    double* part2;       // [ceil(n_jg / 64)][K][4] first-level sums of part
    double* sums;        // [K][4] final sums
    int64_t item0;       // first work item of this task
};

// queue: null for flat dispatch, else a zeroed device counter pair (reset by
// the launch itself when it ends) for queue dispatch over resident workgroups.
int launch_window(const WinTask* d_tasks, const int64_t* d_item0, int ntasks, int64_t nitems,
                  uint32_t flags, int cap, int jmax, unsigned long long* queue, hipStream_t st,
                  double work_units);
int launch_window_reduce(const WinTask* d_tasks, int ntasks, int64_t total_k, const int64_t* d_k0,
                         const int64_t* d_r0, int64_t nred1, uint32_t flags, hipStream_t st);
constexpr int kWinJc = 64;          // j-groups per first-level reduction block
constexpr int kWinGroupMax = 16;    // most j-tiles per window work item
constexpr int kWinItemsMin = 16384; // items a launch keeps before grouping j-tiles

// --------------------------------------------------- A2-A6 spectral route
struct SpreadParams {
    double s;     // Gaussian spreading width (cells)
    double W;     // truncation half-width (cells)
};
SpreadParams spread_params(double sigma, double eps);

// One spectral problem: grid of N cells over period L.
struct SpecTask {
    // point sets: set 0 -> real channel, set 1 -> imaginary channel (CCF)
    const double* t0; const float* v0f; const double* v0d; int64_t n0;
    const double* t1; const float* v1f; const double* v1d; int64_t n1;
    double t_ref;          // grid origin
    double L;              // period
    int64_t N;             // grid cells (power of two)
    int64_t M;             // retained modes |m| <= M
    double s, W;           // spreading kernel
    double h;              // lag-kernel bandwidth
    int32_t kern;          // NCF_GAUSSIAN / NCF_RECTANGLE (diagnostic)
    int32_t ccf;           // 1: packed two-series grid
    void* grid;            // N complex (float2 or double2)
    int64_t tile0;         // first spreading tile of this task
    int64_t ntiles;
    int64_t* tile_rng;     // [ntiles][kTileRec] bounds records of this task's tiles
    double* lags;          // K_eval lags to evaluate (device)
    int32_t K_eval;
    int32_t pad;
    double* numer;         // K_eval results N(tau)
    double* scale_part;    // per-workgroup partial sums of the product kernel (4 per block:
                           // S_xx, S_yy, and with with_b the lag-0 pair sums B_xx, B_yy)
    int64_t pos0;          // first element offset of this task in the flattened product launch
    int32_t with_b;        // also carry the unit-weight channel: pair count b(tau) spectrally
    int32_t pad2;
    void* gridb;           // CCF with_b: unit-weight grid (series 1 real, series 2 imaginary)
    double* bspec;         // with_b: K_eval results b(tau)
    const double* w0;      // with_b, weighted calls: sample weights of set 0 / set 1 spread
    const double* w1;      //   into the pair-count channel (null: unit weights)
    // weighted calls that also need the unweighted pair count b: one more
    // channel with unit weights (ACF: gridb; CCF: gridc); after the product
    // gridb holds the spectrum of b and bunw receives b(tau) at the lags
    void* gridc;
    double* bunw;
    // lag-lattice evaluation (P > 0): every evaluation lag is a whole number of
    // lattice units L / P, so the lag sum is a P-point DFT of the spectrum
    // folded modulo P. The fused kernel folds each 4096-position tile to
    // P2 = 4096 P / N entries, inverse-transforms them and writes them to
    // ybuf[k_low * P2 + n2] (k_low: the tile's frequency residue mod N / 4096);
    // the evaluation kernel finishes the sum at each lag. P = 0: the inverse
    // transform and the interpolation at the lags.
    int64_t P;
    int32_t lgP2;
    int32_t nmc;           // chunks of kFoldTiles tiles summed by separate workgroups
    void* ybuf;
    double* fpart;         // nmc > 1: [nmc][K_eval][2] partial lag sums of the chunks
};

// Spreading tile records: p0, p1 of set 0, p0, p1 of set 1, task index,
// padding (kTileRec int64 per tile, one cache line).
constexpr int kTileRec = 8;

// Fill every task's tile records (tile_rng) for the spread, one workgroup
// per chunk of samples (the moments chunks);
// d_series_map[chunk.series] = 2 * task + set, or -1 for a series without a
// spectral task.
int launch_tile_bounds(const SpecTask* d_tasks, const Chunk* d_chunks, int nchunks,
                       const int32_t* d_series_map, hipStream_t st, double bytes);
// All tasks of one launch share the mode (ACF/CCF, unit-weight channel).
// d_tile_rec: the tile records of all tasks (contiguous, in tile order) from
// launch_tile_bounds, or null to search the ranges in each workgroup.
// weighted: the pair-count channel (with_b) carries the sample weights, so
// it yields the weighted pair sum B instead of the unweighted b; unw: one
// more channel with unit weights for b (SpecTask::gridc / gridb).
int launch_spread(const SpecTask* d_tasks, const int64_t* d_tile0, int ntasks, int64_t ntiles,
                  const int64_t* d_tile_rec, int tile, bool ccf, bool with_b, bool weighted,
                  bool unw, bool fp64, hipStream_t st, double bytes);
// Bit masks of the window rows whose spectral pair count falls back to the
// direct sums (b below beta times the problem's reference: b(0) for the ACF,
// sqrt(B_xx(0) B_yy(0)) from the tasks' product partials for the CCF): bspec
// holds the problems' Keval evaluations contiguously (problem i is task i),
// rowk the evaluation index of each of the Krow window rows (-1: none); mask
// gets ceil(Krow / 64) words per problem. use_scale: compare b times
// min(1, lag-0 scale) (one-shot calls); plans, whose fallback lags are fixed
// on placeholder values, pass false.
int launch_fallback_flags(const SpecTask* d_tasks, const double* bspec, int64_t nprob,
                          int Keval, int K, bool ccf, bool use_scale, const int32_t* rowk,
                          int Krow, double beta, uint64_t* mask, hipStream_t st);
int launch_interp(const SpecTask* d_tasks, int ntasks, const int64_t* d_k0, int64_t total_k,
                  bool fp64, hipStream_t st);
// Lag-lattice evaluation of the tasks with P > 0: workgroup b of
// [d_fe0[i], d_fe0[i + 1]) takes 64 evaluation lags and one chunk of
// kFoldTiles tiles of task i (nmc chunks); tasks of several chunks add their
// chunk sums in a second kernel (one thread per task and lag, indexed like
// the interpolation: d_k0).
constexpr int kFoldLags = 64;
constexpr int kFoldTiles = 1024;
int launch_fold_eval(const SpecTask* d_tasks, int ntasks, const int64_t* d_fe0, int64_t nblocks,
                     const int64_t* d_k0, int64_t total_k, bool chunk_sums, bool fp64,
                     hipStream_t st);

// FFT (A4)
struct FftPlan {
    int64_t N;
    int npass;
    int radix[4];       // first pass first
    int64_t stride[4];  // S of each pass
    int lgt[4];         // log2 tile elements of each pass (12 or 13)
    // twiddles: wlo[e] = w_N^e (e < 2^b), whi[e] = w_N^(e << b); small[e] = w_4096^e
    int lobits;
    void* wlo;  // float2 or double2
    void* whi;
    void* small;
};
// Plan variants (chosen by the autotuner): split 0 = default radices (larger
// strided radix first), 1 = strided radices in the other order, 2 = three
// passes where the default has two; lgt_strided 0 = default tile of the
// strided passes (8192 elements in FP32, 4096 in FP64), else 12 or 13.
struct FftVariant {
    int split = 0;
    int lgt_strided = 0;
};
// Twiddle tables are cached per (N, fp64, device).
int fft_plan(int64_t N, bool fp64, FftPlan* plan, hipStream_t st,
             const FftVariant& v = FftVariant{});
// Batched transform of `count` grids of the same N laid out at `grids[i]`.
// sign +1: natural -> digit-reversed; sign -1: digit-reversed -> natural.
// skip_tile_pass: leave out the radix-4096 pass (the last of sign +1, the
// first of sign -1), which launch_mid performs.
int fft_exec(const FftPlan& plan, void* const* d_grids, int count, int sign, bool fp64,
             hipStream_t st, bool skip_tile_pass = false);
// storage position of frequency k after the sign +1 transform
int64_t fft_position(const FftPlan& plan, int64_t k);

// A5 spectral product (in place, digit-reversed order)
// All tasks of one launch share the mode: ACF or CCF, with or without the
// unit-weight (pair-count) channel.
// unw: the unit channel (gridb for the ACF, gridc for the CCF) also gives the
// spectrum of the unweighted pair count, written to gridb.
int launch_product(const SpecTask* d_tasks, const int64_t* d_pos0, int ntasks, int64_t total,
                   const int64_t* d_radix_info, bool ccf, bool with_b, bool unw, bool fp64,
                   hipStream_t st, double bytes);

// ------------------------------------------- regular-lattice estimators
// Series whose times sit on a common lattice t_ref + m dt: the pair lags are
// whole multiples of dt, so the raw lag correlations R(q) = sum_c a_c b_(c+q)
// of the lattice grids (values, weights, sample counts) come from one
// zero-padded FFT correlation, and every lag tau is a filter over q.
//
// Channel modes (all tasks of a launch share one):
//   0 ACF       grids (v, n)               outputs (R_vv, R_nn)
//   1 ACF + w   grids (v, w), (n, 0)       outputs (R_vv, R_ww), (R_nn, 0)
//   2 CCF       grids (vx, vy), (nx, ny)   outputs (R_xy, N_xy), (R_xx, R_yy), (N_xx, N_yy)
//   3 CCF + w   grids (vx, vy), (wx, wy), (nx, ny)
//               outputs (R_xy, W_xy), (N_xy, 0), (R_xx, R_yy), (W_xx, W_yy)
// with v = w (x - mean)/sd, w the sample weights and n the sample counts per
// lattice cell. Input grids are transformed in place and the products
// overwrite them (the extra output grids follow the inputs).
constexpr int kRegCells = 1024;  // lattice cells per fill workgroup
__host__ __device__ constexpr int reg_in_grids(int mode) { return mode == 3 ? 3 : mode == 0 ? 1 : 2; }
__host__ __device__ constexpr int reg_out_grids(int mode) { return mode == 0 ? 1 : mode == 1 ? 2 : mode == 2 ? 3 : 4; }
__host__ __device__ constexpr int reg_grids(int mode) {
    return reg_in_grids(mode) > reg_out_grids(mode) ? reg_in_grids(mode) : reg_out_grids(mode);
}

struct RegTask {
    const double* t[2];   // times of series 1 and (CCF) series 2
    const double* v[2];   // FP64 standardized weighted values
    const double* w[2];   // FP64 weights, or null (unit weights)
    int64_t n[2];
    double t_ref;         // lattice origin (first time of either series)
    double dt;            // lattice step
    double tol;           // accepted distance of a time from its lattice point
    double h;             // lag-kernel bandwidth
    int64_t G;            // lattice cells from t_ref to the last time
    int64_t N;            // transform length (power of two >= G + Q)
    int64_t Q;            // largest |q| any requested window reaches (<= G - 1)
    double* grids;        // reg_grids(mode) grids of N complex128 values
    int32_t* bad;         // set to 1 when a time is off the lattice
    int64_t blk0;         // first fill workgroup of this task
    int64_t pos0;         // first position of this task in the product launch
    RadixInfo ri;         // transform radices (digit-reversed positions)
    // normalization
    const SeriesStat* st0;
    const SeriesStat* st1;
    int32_t skip;         // failed the host checks: outputs NaN / 0 / 0
    int32_t skip_status;
    int64_t out_off;      // first output of this problem in IoBlock::c, b, count
    int64_t index;        // problem index (IoBlock::status)
};
// Zero the lattice flags of `n` tasks.
int launch_reg_clear(const RegTask* d_tasks, int ntasks, hipStream_t st);
// Lattice grids of every task (natural order, zero-padded to N cells).
int launch_reg_fill(const RegTask* d_tasks, const int64_t* d_blk0, int ntasks, int64_t nblocks,
                    int mode, hipStream_t st, double bytes);
// Correlation spectra from the forward-transformed grids (digit-reversed
// order, in place), scaled by 1/N for the inverse transform.
int launch_reg_product(const RegTask* d_tasks, const int64_t* d_pos0, int ntasks, int64_t total,
                       int mode, hipStream_t st, double bytes);
// Lag filter, normalization and outputs (request order) of every task.
int launch_reg_finish(const RegTask* d_tasks, int ntasks, const double* d_lags, int64_t K,
                      int mode, int kern, const IoBlock* io, hipStream_t st);

// Fused forward last FFT pass (radix 4096), product and inverse first pass
// over pairs of 4096-position tiles (the tiles of frequencies k and -k), all
// tasks in one launch; replaces the last forward pass, launch_product and
// the first inverse pass for the modes mid_supported accepts (no unit
// channel; LDS for two or four tiles within 160 KB). d_pair0: prefix of
// mid_pairs(N) over the tasks; wsmall: the FFT's w_4096 table.
bool mid_supported(bool ccf, bool with_b, bool unw, bool fp64);
int64_t mid_pairs(int64_t N);
int launch_mid(const SpecTask* d_tasks, const int64_t* d_pair0, int ntasks, int64_t npairs,
               const int64_t* d_radix_info, const void* wsmall, bool ccf, bool with_b, bool fp64,
               hipStream_t st, double bytes);

// ------------------------------------------------------------ A8 output
struct NormTask {
    int32_t ccf;          // 0 ACF, 1 CCF
    int32_t K;            // requested lags
    const int32_t* perm;  // requested lag k -> row of the window sums
    int32_t row0;         // ACF: row of lag 0 in the window sums
    int32_t spectral;     // numerator from the spectral route
    int32_t spec_b;       // pair counts from the spectral route too (else window sums)
    int32_t guard;        // plan execution in mixed precision (Gaussian): a lag-0 scale
                          // below kPromoteScale reports NCF_E_UNSUPPORTED
    double* rmin;         // or null: receives the problem's smallest lag-0 scale (ACF
                          // r(0); CCF min(r_x(0), r_y(0))), +inf when it failed
    const double* bspec;  // spectral b per requested lag (+ lag 0 last for ACF); with
                          // weights the weighted pair sum B
    const double* bunw;   // weighted calls: spectral unweighted b per lag, or null
    const int32_t* fb_row;  // requested lag -> row of the direct fallback sums, -1 if none
    const double* fb_sums;  // direct window sums [rows][4] of the fallback lags
    double beta;          // fallback threshold (window-b path): b < beta * b_ref
    const double* wsums;  // window sums [K_rows][4]
    const double* numer;  // spectral numerator per requested lag (+ lag 0 last for ACF)
    const double* self_x; // CCF: window sums of series 1 on itself at lag 0 ([4])
    const double* self_y; // CCF: window sums of series 2 on itself at lag 0
    const double* scale_part; // CCF spectral: partial (S_xx, S_yy) pairs
    int64_t nscale_part;
    int32_t weighted;
    int32_t is_rect;
    int32_t skip;         // problem failed the host checks: outputs NaN / 0 / 0
    int32_t skip_status;  // its status
    const SeriesStat* st0;  // device statistics of the problem's series (a failed
    const SeriesStat* st1;  // value check there also gives NaN / 0 / 0); st1 CCF only
    int64_t out_off;      // first output of this problem in IoBlock::c, b, count
    int64_t index;        // problem index (IoBlock::status)
};
// Every task writes its outputs and its status through `io`.
int launch_normalize(const NormTask* d_tasks, int ntasks, const IoBlock* io, hipStream_t st);

}  // namespace ncf
