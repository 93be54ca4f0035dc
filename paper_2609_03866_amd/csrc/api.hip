// api.hip -- C ABI, planner and batch scheduler of the ncf library.
//
// A call runs in two phases on one stream:
//   1. inputs on the device -> per-series validation and FP64 moments (A1);
//      the per-series statistics (status, mean, sd, time span) come back to
//      the host, which plans the rest from them;
//   2. standardization (+ FP64 prefix sums for the rectangle kernel), the
//      window scan over every (series, j-tile, lag-tile) work item of the
//      whole batch in one launch (A7), the spectral route for the Gaussian
//      numerator (A2-A6: spreading tiles of every series in one launch, the
//      FFT passes of all grids of one size in one launch per pass, the
//      product, the lag evaluation), and the normalization (A8).
// Work items of a batch are flattened across series so that a single
// launch covers thousands of uneven series.
#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include <unistd.h>

#include "internal.h"
#include "ncf_diag.h"

namespace ncf {

// ------------------------------------------------------------------ errors

namespace {
thread_local std::string g_err;
}

// Verbosity of the call log on stderr, from NCF_LOG (0 when unset): 1, one
// line per call (route, grids, window work, fallback lags, statuses, host
// time) and per plan build; 2, also every autotuner candidate.
int log_level() {
    const char* v = std::getenv("NCF_LOG");
    return v ? std::atoi(v) : 0;
}

void set_error(const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}

void clear_error() { g_err.clear(); }

// ------------------------------------------------------- host worker pool
// The per-problem planning loops of large batches (grid geometry, window
// task tiling) run on a few host threads: workers created on first use and
// kept for the process (never joined: they only ever wait on the pool's
// condition variable), one job at a time; a call that finds the pool busy
// (another host thread's call, or a loop nested in a job) runs its loop
// alone, and so does a forked child, which has no workers. f(i) for i in
// [0, n) must touch only its own outputs and must not throw.
class HostPool {
   public:
    static HostPool& get() {
        static HostPool* pool = new HostPool();  // never destroyed (see above)
        return *pool;
    }
    template <typename F>
    void run(int64_t n, const F& f) {
        constexpr int64_t kMinItems = 1024;  // below this the hand-off costs more
        std::unique_lock<std::mutex> busy(job_mu_, std::try_to_lock);
        if (n < kMinItems || nthreads_ == 0 || !busy.owns_lock() || getpid() != pid_) {
            for (int64_t i = 0; i < n; ++i) f(i);
            return;
        }
        std::function<void(int64_t)> fn = [&f](int64_t i) { f(i); };
        const int64_t nblk = (int64_t)(nthreads_ + 1) * 4;
        {
            std::lock_guard<std::mutex> lk(mu_);
            job_ = &fn;
            n_ = n;
            nblk_ = nblk;
            next_.store(0);
            left_ = nthreads_;
            ++gen_;
        }
        cv_.notify_all();
        work();
        std::unique_lock<std::mutex> lk(mu_);
        done_cv_.wait(lk, [&] { return left_ == 0; });
        job_ = nullptr;
    }

   private:
    HostPool() : pid_(getpid()) {
        const unsigned hw = std::thread::hardware_concurrency();
        nthreads_ = (int)std::min(7u, hw > 1 ? hw - 1 : 0u);
        for (int i = 0; i < nthreads_; ++i) std::thread([this] { loop(); }).detach();
    }
    void work() {  // blocks of the current job until none is left
        for (;;) {
            const int64_t b = next_.fetch_add(1);
            if (b >= nblk_) return;
            const int64_t i0 = n_ * b / nblk_, i1 = n_ * (b + 1) / nblk_;
            for (int64_t i = i0; i < i1; ++i) (*job_)(i);
        }
    }
    void loop() {
        uint64_t seen = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return gen_ != seen; });
                seen = gen_;
            }
            work();
            std::lock_guard<std::mutex> lk(mu_);
            if (--left_ == 0) done_cv_.notify_one();
        }
    }
    pid_t pid_;  // the process whose threads these are
    int nthreads_ = 0;
    std::mutex job_mu_;  // one job at a time
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    const std::function<void(int64_t)>* job_ = nullptr;
    int64_t n_ = 0, nblk_ = 0;
    std::atomic<int64_t> next_{0};
    int left_ = 0;
    uint64_t gen_ = 0;
};

template <typename F>
void host_parallel_for(int64_t n, const F& f) {
    HostPool::get().run(n, f);
}

// --------------------------------------------------------------- profiling

namespace {

struct ProfRec {
    int64_t launches = 0;
    double ms = 0.0;
    double work = 0.0;
    std::string unit;
};
struct Pending {
    std::string name;
    hipEvent_t e0, e1;
    double work;
    std::string unit;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::string g_prof_only;            // empty: every kernel; else only this name
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_ev_free;  // events kept for reuse (no create per launch)
std::map<std::string, ProfRec> g_prof;

void prof_flush_locked() {
    for (auto& p : g_pending) {
        float ms = 0.f;
        (void)hipEventSynchronize(p.e1);
        (void)hipEventElapsedTime(&ms, p.e0, p.e1);
        auto& r = g_prof[p.name];
        r.launches += 1;
        r.ms += ms;
        r.work += p.work;
        r.unit = p.unit;
        g_ev_free.push_back(p.e0);
        g_ev_free.push_back(p.e1);
    }
    g_pending.clear();
}

hipEvent_t prof_event_locked() {
    if (!g_ev_free.empty()) {
        hipEvent_t e = g_ev_free.back();
        g_ev_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

}  // namespace

namespace {
thread_local bool g_capturing = false;  // a plan's launches are being captured
}

ProfScope::ProfScope(hipStream_t s, const char* n, double w, const char* u)
    : stream(s), name(n), work(w), unit(u), ev0(nullptr) {
    if (!g_prof_on || g_capturing) return;
    hipEvent_t e;
    {
        std::lock_guard<std::mutex> lock(g_prof_mu);
        if (!g_prof_only.empty() && g_prof_only != n) return;
        e = prof_event_locked();
    }
    if (!e) return;
    (void)hipEventRecord(e, stream);
    ev0 = e;
}

ProfScope::~ProfScope() {
    if (!ev0) return;
    std::lock_guard<std::mutex> lock(g_prof_mu);
    hipEvent_t e1 = prof_event_locked();
    if (!e1) {
        g_ev_free.push_back((hipEvent_t)ev0);
        return;
    }
    (void)hipEventRecord(e1, stream);
    g_pending.push_back({name, (hipEvent_t)ev0, e1, work, unit});
}

// --------------------------------------------------------------- workspace

namespace {

struct DevBuf {
    void* ptr = nullptr;
    size_t cap = 0;
};

// Small tables (descriptors, offsets, lag lists) of one phase are laid out
// in a pinned host buffer mirrored by a device buffer and uploaded with a
// single copy.
struct Staging {
    char* h = nullptr;
    char* d = nullptr;
    size_t cap = 0;
};

// Device memory of a call: workspace arenas (moments, main phase, fallback,
// and the replicate series of the resampling calls) and three table stagings. One-shot calls share one set per
// device (grown on demand, kept until ncf_release_workspace); a plan owns
// its own set for its lifetime.
struct Resources {
    DevBuf ws[4];  // moments, main phase, fallback, replicate inputs
    Staging stage[3];
    unsigned long long* queue = nullptr;  // work-queue counter pairs, zeroed once
    bool exact = false;  // plan: allocate what is asked, no growth slack
    // allocation-free calls: every arena and staging buffer is carved, in
    // order, from a fixed device region and a fixed host region; a request
    // beyond them fails (nothing is allocated or freed)
    char* fixed_dev = nullptr;
    size_t fixed_cap = 0, fixed_off = 0;
    char* fixed_host = nullptr;
    size_t fixed_host_cap = 0, fixed_host_off = 0;
};

// Next `bytes` of a fixed region (256-byte aligned), or null when it is full.
char* carve(char* base, size_t cap, size_t* off, size_t bytes) {
    const size_t a = (*off + 255) & ~(size_t)255;
    if (a > cap || bytes > cap - a) return nullptr;
    *off = a + bytes;
    return base + a;
}

constexpr int kQueuePairs = 4;

// Counter pairs of the queue-dispatched launches (zeroed once at allocation;
// each launch leaves its pair zeroed).
int ensure_queue(Resources& R, unsigned long long** out) {
    if (!R.queue) {
        if (hipMalloc((void**)&R.queue, sizeof(unsigned long long) * 2 * kQueuePairs) !=
            hipSuccess) {
            (void)hipGetLastError();
            R.queue = nullptr;
            set_error("work-queue counter allocation failed");
            return NCF_E_NOMEM;
        }
        NCF_TRY_HIP(hipMemset(R.queue, 0, sizeof(unsigned long long) * 2 * kQueuePairs));
    }
    *out = R.queue;
    return NCF_OK;
}
std::mutex g_ws_mu;
std::map<int, Resources> g_res;  // one-shot calls, per device

// Bound on the device workspace arenas of one call or plan, in bytes, from
// the environment variable NCF_WORKSPACE_LIMIT_MB (MiB, read once; unset or
// not a positive number: no bound). A call whose arenas would exceed it
// fails with NCF_E_NOMEM before allocating.
size_t workspace_limit() {
    static const size_t lim = [] {
        const char* e = std::getenv("NCF_WORKSPACE_LIMIT_MB");
        if (!e || !*e) return (size_t)0;
        char* end = nullptr;
        const double v = std::strtod(e, &end);
        if (end == e || !(v > 0.0) || !(v < 1e12)) return (size_t)0;
        return (size_t)(v * 1048576.0);
    }();
    return lim;
}

int ensure_ws(Resources& R, int which, size_t bytes, void** out) {
    DevBuf& b = R.ws[which];
    if (R.fixed_dev) {
        char* p = carve(R.fixed_dev, R.fixed_cap, &R.fixed_off, bytes);
        if (!p) {
            set_error("the call needs more device workspace than the allocation-free "
                      "entry point's fixed %zu bytes (%zu in use, %zu more asked)",
                      R.fixed_cap, R.fixed_off, bytes);
            return NCF_E_UNSUPPORTED;
        }
        b.ptr = p;
        b.cap = bytes;
        *out = p;
        return NCF_OK;
    }
    if (b.cap < bytes) {
        if (b.ptr) {
            NCF_TRY_HIP(hipDeviceSynchronize());
            NCF_TRY_HIP(hipFree(b.ptr));
            b.ptr = nullptr;
            b.cap = 0;
        }
        size_t want = R.exact ? bytes : bytes + bytes / 8 + (1 << 20);
        if (const size_t lim = workspace_limit()) {
            size_t others = 0;
            for (int i = 0; i < 4; ++i)
                if (i != which) others += R.ws[i].cap;
            if (others > lim || bytes > lim - others) {
                set_error("device workspace limit of %zu bytes (NCF_WORKSPACE_LIMIT_MB) "
                          "reached: %zu bytes held, %zu more asked",
                          lim, others, bytes);
                return NCF_E_NOMEM;
            }
            want = std::min(want, lim - others);
        }
        hipError_t e = hipMalloc(&b.ptr, want);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            b.ptr = nullptr;
            set_error("device workspace allocation of %zu bytes failed", want);
            return NCF_E_NOMEM;
        }
        b.cap = want;
    }
    *out = b.ptr;
    return NCF_OK;
}

int ensure_stage(Resources& R, int phase, size_t bytes, Staging** out) {
    Staging& S = R.stage[phase];
    if (R.fixed_dev) {
        char* d = carve(R.fixed_dev, R.fixed_cap, &R.fixed_off, bytes);
        char* h = carve(R.fixed_host, R.fixed_host_cap, &R.fixed_host_off, bytes);
        if (!d || !h) {
            set_error("the call's tables (%zu bytes) do not fit the allocation-free entry "
                      "point's fixed workspace",
                      bytes);
            return NCF_E_UNSUPPORTED;
        }
        S.h = h;
        S.d = d;
        S.cap = bytes;
        *out = &S;
        return NCF_OK;
    }
    if (S.cap < bytes) {
        if (S.h) {
            NCF_TRY_HIP(hipDeviceSynchronize());
            NCF_TRY_HIP(hipHostFree(S.h));
            NCF_TRY_HIP(hipFree(S.d));
            S = Staging{};
        }
        const size_t want = R.exact ? bytes + 256 : 2 * bytes + 65536;
        if (hipHostMalloc((void**)&S.h, want) != hipSuccess ||
            hipMalloc((void**)&S.d, want) != hipSuccess) {
            (void)hipGetLastError();
            set_error("staging allocation of %zu bytes failed", want);
            return NCF_E_NOMEM;
        }
        S.cap = want;
    }
    *out = &S;
    return NCF_OK;
}

void free_resources(Resources& R) {
    if (R.queue) (void)hipFree(R.queue);
    R.queue = nullptr;
    for (auto& b : R.ws) {
        if (b.ptr) (void)hipFree(b.ptr);
        b = DevBuf{};
    }
    for (auto& S : R.stage) {
        if (S.h) (void)hipHostFree(S.h);
        if (S.d) (void)hipFree(S.d);
        S = Staging{};
    }
}

// Bump allocator over a workspace: first a sizing pass (base == nullptr),
// then the same sequence of takes on the real buffer.
struct Arena {
    char* base = nullptr;
    size_t off = 0;
    template <typename T>
    T* take(size_t count) {
        size_t a = (off + 255) & ~(size_t)255;
        off = a + sizeof(T) * count;
        return base ? reinterpret_cast<T*>(base + a) : reinterpret_cast<T*>(a + 1);
    }
};

// -------------------------------------------------------------- the job

constexpr int64_t kChunk = kMomentChunk;  // samples per moments chunk

// Reserve table slots: device address for kernels, host address for filling.
struct Tables {
    char* h = nullptr;  // null during the sizing pass
    char* d = nullptr;
    size_t off = 0;
    template <typename T>
    T* take(size_t n, T** host) {
        const size_t a = (off + 15) & ~(size_t)15;
        off = a + sizeof(T) * std::max<size_t>(n, 1);
        *host = h ? reinterpret_cast<T*>(h + a) : nullptr;
        return d ? reinterpret_cast<T*>(d + a) : nullptr;
    }
};

struct SeriesSet {
    const double* t = nullptr;  // device inputs
    const double* x = nullptr;
    const double* err = nullptr;
    int64_t ntot = 0;
    std::vector<int64_t> offs;  // host, nser + 1
    int nser = 0;
    // derived device arrays (concatenated over the set's series)
    float* v32 = nullptr;
    double* v64 = nullptr;
    double* w64 = nullptr;
    double* pv = nullptr;  // ntot + nser entries (n + 1 per series)
    double* pw = nullptr;
    double* pz = nullptr;  // prefix count of nonzero weights (weighted rectangle)
    int sd0 = 0;           // first descriptor of this set in the moments table
    bool shared_t = false; // every series of the set has the same times (t holds one copy)
    bool wmode = false;    // err holds sample weights (w >= 0) instead of errors
};

// Scheduling settings that change speed, not the estimator (results differ
// at most at the rounding level): chosen by the plan autotuner.
struct Tune {
    double sigma = 0.0;  // minimum grid oversampling (0: options or 1.5)
    FftVariant fft;      // radix split and strided-pass tile of the FFTs
    int jscale = 0;      // window tiles (outer samples per workgroup) times 2^jscale
    bool queue = false;  // window scans by work-queue dispatch
    bool no_mid = false; // separate last FFT pass, product and first inverse pass
    bool eval_interp = false;  // lags by inverse transform and interpolation even on a lattice
};

struct Job {
    double lag_unit = 0.0;  // lattice unit of the evaluation lags (0: not on a lattice)
    bool ccf = false;
    int64_t nprob = 0;
    int kern = NCF_GAUSSIAN;
    std::vector<double> h;     // per problem
    std::vector<double> lags;  // host copy, K
    const double* lags_dev = nullptr;  // device lags still to be copied (phase 1)
    int64_t K = 0;
    double* c = nullptr;       // user outputs
    double* b = nullptr;
    int64_t* count = nullptr;
    int* status = nullptr;     // host, nprob (may be null)
    ncf_options_t opt;
    bool dev_ptrs = false;
    hipStream_t st = nullptr;
    SeriesSet set[2];          // ACF: set[0]; CCF: set[0] = series 1, set[1] = series 2
    Resources* res = nullptr;  // device memory of this call
    // plan construction: every launch reads and writes the caller arrays
    // through this device block (else through blocks in the call's tables),
    // and is appended to `rec` for replay
    IoBlock* io_fixed = nullptr;
    int32_t* io_status = nullptr;  // device status array the block points at
    std::vector<std::function<int(hipStream_t)>>* rec = nullptr;
    bool plan_build = false;   // statuses are those of the host checks only
    Tune tune;
    // the caller does not read b (replicates): weighted Gaussian calls may take
    // the weighted pair sum B from the spectral route
    bool no_b = false;
    // allocation-free call: no FP64 re-evaluation (it needs workspace); a
    // near-degenerate mixed-precision problem is reported as plans do
    bool no_alloc = false;
    // regular-lattice estimators: lattice step per problem
    bool regular = false;
    std::vector<double> dt;
    // filled by run_job: what the call planned
    int64_t info_grid_cells = 0, info_window_items = 0;
    int info_grids = 0, info_window_launches = 0;
    int info_fold_grids = 0;  // grids read off a lag lattice
};

int check_lags(const Job& J) {
    for (double v : J.lags)
        if (!std::isfinite(v)) {
            set_error("non-finite lag");
            return NCF_E_INVALID_ARG;
        }
    return NCF_OK;
}

// Enqueue a launch now and, when a plan is being built, keep it for replay.
template <class F>
int emit(Job& J, F f) {
    NCF_TRY(f(J.st));
    if (J.rec) J.rec->emplace_back(std::move(f));
    return NCF_OK;
}

bool use_spectral(const Job& J) {
    if (J.opt.method == NCF_DIRECT) return false;
    if (J.kern == NCF_GAUSSIAN) return true;
    return J.opt.method == NCF_SPECTRAL;  // rectangle: diagnostic only
}

// log2 of a power of two (0 to 63)
int ilog2_exact(int64_t n) { return n > 0 ? 63 - __builtin_clzll((unsigned long long)n) : 0; }

int64_t pow2_at_least(double v) {
    if (!(v > 1.0)) return 1;
    int e = 0;
    const double m = std::frexp(v, &e);  // v = m 2^e, m in [0.5, 1)
    const int k = m == 0.5 ? e - 1 : e;
    return k >= 62 ? (int64_t)1 << 62 : (int64_t)1 << k;
}

// One spectral problem's geometry.
struct SpecGeom {
    double L, t_ref, s, W;
    int64_t N, M;
    int64_t P = 0;  // lag-lattice evaluation: L = P lattice units (0: interpolation)
};

// A unit D > 0 of which every evaluation lag (and 0) is a whole multiple, to
// 1e-9 relative, with fewer than 2^30 units to the farthest lag: the finest
// of gap / q, q = 1..8, over the smallest gap between distinct lags. 0 when
// the lags are not on such a lattice (then they are read by interpolation).
double lag_lattice_unit(const std::vector<double>& lags, bool with_zero) {
    std::vector<double> v(lags);
    if (with_zero) v.push_back(0.0);
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    if (v.size() < 2) return 0.0;
    double gap = HUGE_VAL;
    for (size_t i = 1; i < v.size(); ++i) gap = std::min(gap, v[i] - v[i - 1]);
    if (!(gap > 0.0) || !std::isfinite(gap)) return 0.0;
    const double far = std::max(std::fabs(v.front()), std::fabs(v.back()));
    for (int q = 1; q <= 8; ++q) {
        const double D = gap / q;
        if (far / D >= 1073741824.0) break;
        bool ok = true;
        for (double x : v) {
            const double u = x / D;
            if (std::fabs(u - std::nearbyint(u)) > 1e-9 * std::max(1.0, std::fabs(u))) {
                ok = false;
                break;
            }
        }
        if (ok) return D;
    }
    return 0.0;
}

int plan_grid(const Job& J, double tmin, double tmax, double maxlag, double h, SpecGeom* g) {
    const bool fp64 = J.opt.precision == NCF_FP64;
    const double tol = J.opt.tol > 0 ? J.opt.tol : (fp64 ? 1e-13 : 1e-9);
    const double eps_s = fp64 ? 1e-13 : 1e-7;  // spreading accuracy
    const double sig_min = J.tune.sigma > 1.0 ? J.tune.sigma : J.opt.sigma > 1.0 ? J.opt.sigma : 1.5;
    const double span = tmax - tmin;
    double Wh, fcut;
    if (J.kern == NCF_GAUSSIAN) {
        Wh = 9.0 * h;  // phi_h(9h)/phi_h(0) = e^-40.5
        fcut = std::sqrt(std::log(1.0 / tol) / (2.0 * M_PI * M_PI)) / h;
    } else {
        Wh = h;
        fcut = 16.0 / h;
    }
    // modes, cells and spreading kernel for period L; the evaluated factor
    // phihat / Psi^q (q = 3 with interpolation at the lags, 2 on a lag
    // lattice) must decay with |m|
    auto cells = [&](double L, double q, double sig, int64_t* Nout, int64_t* Mout,
                     SpreadParams* spo) {
        int64_t M = (int64_t)std::ceil(fcut * L);
        int64_t N;
        if (J.opt.grid_size > 0) {
            N = J.opt.grid_size;
            M = std::min<int64_t>(M, (int64_t)std::floor((N / sig - 1.0) / 2.0));
        } else {
            N = std::max<int64_t>(4096, pow2_at_least(sig * (2.0 * M + 1.0)));
        }
        SpreadParams sp{};
        for (;;) {
            const double sigma = (double)N / (2.0 * M + 1.0);
            sp = spread_params(sigma, eps_s);
            const double h_cells = h * (double)N / L;
            if (J.kern != NCF_GAUSSIAN || h_cells >= std::sqrt(q) * sp.s || J.opt.grid_size > 0)
                break;
            N *= 2;
        }
        *Nout = N;
        *Mout = M;
        *spo = sp;
    };
    double L = span + maxlag + Wh;
    bool done = false;
    for (int iter = 0; iter < 8 && !done; ++iter) {
        int64_t M, N;
        SpreadParams sp;
        cells(L, 3.0, sig_min, &N, &M, &sp);
        if (N > (1LL << 31)) {
            set_error("spectral grid of %lld cells exceeds the supported maximum (2^31)",
                      (long long)N);
            return NCF_E_UNSUPPORTED;
        }
        const double cell = L / (double)N;
        const double margin = (sp.W + 2.0) * cell;
        if (span + 2.0 * margin <= L) {
            g->L = L;
            g->N = N;
            g->M = M;
            g->s = sp.s;
            g->W = sp.W;
            g->t_ref = tmin - margin;
            g->P = 0;
            done = true;
        } else {
            L = span + 2.0 * margin + cell;
        }
    }
    if (!done) {
        set_error("grid planning did not converge");
        return NCF_E_UNSUPPORTED;
    }
    // Lag lattice of unit D: with L = P D / d for a
    // whole d, every lag is a whole number of units L / P and the lag sum is
    // a P-point DFT of the spectrum folded modulo P. P = 2^j >= d Lmin / D,
    // so L lies in [Lmin, 2 Lmin); over d = 1..32 the geometry with the
    // fewest cells wins (then the smallest P), taken when it has no more
    // cells than the interpolating one. P must divide N with 2 <= N / P <= 256
    // (16 to 2048 folded entries per 4096-position tile).
    // (Lmin: the interpolating period before its margin adjustment.)
    if (J.lag_unit > 0.0 && J.kern == NCF_GAUSSIAN && J.opt.grid_size <= 0) {
        const double Lmin = span + maxlag + Wh;
        // L = P D / d lies in [Lmin, 2 Lmin), so the cell count at the
        // minimum oversampling takes at most two values, N_a (that of Lmin)
        // and 2 N_a. For a target count Nt the admissible periods are
        // L <= L_t (the longest whose modes fit Nt); the smallest P among them
        // comes from the smallest d that has a power of two in
        // [d Lmin / D, d L_t / D] (P grows with d). The lattice period may
        // take the oversampling down to 1.25 (a wider spreading kernel) where
        // the interpolating grid keeps the default 1.5.
        const double sig_fold = std::min(sig_min, 1.25);
        const int64_t Na = std::max<int64_t>(
            4096, pow2_at_least(sig_fold * (2.0 * std::ceil(fcut * Lmin) + 1.0)));
        for (int64_t Nt = Na; Nt <= g->N && Nt <= Na * 2; Nt *= 2) {
            const double Lt = std::floor((Nt / sig_fold - 1.0) / 2.0) / fcut;
            int64_t P = 0;
            double Lf = 0.0;
            for (int d = 1; d <= 32; ++d) {
                const double u = J.lag_unit / d;
                const int64_t Pd = pow2_at_least(Lmin / u);
                if (2 * Pd > Nt) break;        // larger d only makes P larger
                if (Nt / Pd > 256) continue;   // too few folded entries per tile
                if ((double)Pd * u <= Lt) {
                    P = Pd;
                    Lf = (double)Pd * u;
                    break;
                }
            }
            if (P == 0) continue;
            int64_t M, N;
            SpreadParams sp;
            cells(Lf, 2.0, sig_fold, &N, &M, &sp);
            if (N > g->N || 2 * P > N || N / P > 256) continue;
            const double cell = Lf / (double)N;
            const double margin = (sp.W + 2.0) * cell;
            if (span + 2.0 * margin > Lf) continue;
            *g = SpecGeom{Lf, tmin - margin, sp.s, sp.W, N, M, P};
            break;
        }
    }
    return NCF_OK;
}

// Per-problem statuses of a finished call (h_fstat: device statuses read
// back); the call returns the first failure.
int finish_status(Job& J, const std::vector<int>& pstat, const int32_t* h_fstat) {
    if (J.plan_build) {  // placeholder values: only the host checks count
        if (J.status)
            for (int64_t p = 0; p < J.nprob; ++p) J.status[p] = pstat[p];
        return NCF_OK;
    }
    int first = NCF_OK;
    for (int64_t p = 0; p < J.nprob; ++p) {
        if (J.status) J.status[p] = h_fstat[p];
        if (h_fstat[p] != NCF_OK && first == NCF_OK) first = h_fstat[p];
    }
    if (first != NCF_OK) {
        static const char* names[] = {"ok", "invalid argument", "unsorted times",
                                      "degenerate series", "out of memory", "device error",
                                      "unsupported"};
        int idx = -first;
        set_error("series failed: %s", (idx >= 0 && idx <= 6) ? names[idx] : "error");
    }
    return first;
}

// ------------------------------------------------------------ regular lattice

// The classic-FFT route for series on a common time lattice (after the
// moments and the standardization of run_job): lattice grids, FP64
// transforms, correlation products, inverse transforms and the lag filter.
int run_regular(Job& J, const std::vector<SeriesDesc>& sdesc,
                const std::vector<SeriesStat>& stats, std::vector<int>& pstat,
                const SeriesStat* d_stats) {
    const int64_t K = J.K;
    const bool rect = J.kern == NCF_RECTANGLE;
    const int nsets = J.ccf ? 2 : 1;
    bool weighted = false;
    for (int si = 0; si < nsets; ++si) weighted |= (J.set[si].err != nullptr);
    const int mode = (J.ccf ? 2 : 0) + (weighted ? 1 : 0);
    const int ng = reg_in_grids(mode), no = reg_out_grids(mode), ngr = reg_grids(mode);
    double maxlag = 0.0;
    for (double v : J.lags) maxlag = std::max(maxlag, std::fabs(v));
    auto stat_of = [&](int si, int64_t s) -> const SeriesStat& {
        return stats[J.set[si].sd0 + s];
    };

    // lattice geometry of every problem that passed the host checks
    struct RegPlan {
        int64_t prob;
        double t_ref;
        int64_t G, Q, N;
    };
    std::vector<RegPlan> rps;
    for (int64_t p = 0; p < J.nprob; ++p) {
        if (pstat[p] != NCF_OK) continue;
        const double dt = J.dt[p];
        if (!(dt > 0.0) || !std::isfinite(dt)) {
            pstat[p] = NCF_E_INVALID_ARG;
            continue;
        }
        double t0 = stat_of(0, p).tmin, t1 = stat_of(0, p).tmax;
        if (J.ccf) {
            t0 = std::min(t0, stat_of(1, p).tmin);
            t1 = std::max(t1, stat_of(1, p).tmax);
        }
        const double W = rect ? J.h[p] : 6.0 * J.h[p];
        const double cells = std::rint((t1 - t0) / dt) + 1.0;
        const double qreach = std::ceil((maxlag + W) / dt) + 2.0;
        if (!(cells < 2147483648.0)) {
            pstat[p] = NCF_E_UNSUPPORTED;  // lattice longer than the largest transform
            continue;
        }
        RegPlan rp;
        rp.prob = p;
        rp.t_ref = t0;
        rp.G = (int64_t)cells;
        rp.Q = (int64_t)std::min((double)(rp.G - 1), qreach);
        rp.N = std::max<int64_t>(4096, pow2_at_least((double)(rp.G + rp.Q)));
        if (rp.N > (1LL << 31)) {
            pstat[p] = NCF_E_UNSUPPORTED;
            continue;
        }
        rps.push_back(rp);
    }
    std::stable_sort(rps.begin(), rps.end(),
                     [](const RegPlan& a, const RegPlan& b) { return a.N < b.N; });
    const int nreg = (int)rps.size();
    J.info_grids = nreg;
    J.info_grid_cells = 0;
    for (auto& rp : rps) J.info_grid_cells += rp.N;
    J.info_window_items = 0;
    J.info_window_launches = 0;

    // device workspace: grids, lattice flags, outputs (host mode)
    Resources& R = *J.res;
    std::vector<double*> grids(nreg);
    int32_t* d_bad = nullptr;
    double *d_c = nullptr, *d_b = nullptr;
    int64_t* d_cnt = nullptr;
    auto layout = [&](Arena& ar) {
        for (int i = 0; i < nreg; ++i) grids[i] = ar.take<double>(2 * (size_t)rps[i].N * ngr);
        d_bad = ar.take<int32_t>(std::max(nreg, 1));
        if (J.dev_ptrs) {
            d_c = J.c;
            d_b = J.b;
            d_cnt = J.count;
        } else {
            d_c = ar.take<double>(std::max<int64_t>(J.nprob * K, 1));
            d_b = ar.take<double>(std::max<int64_t>(J.nprob * K, 1));
            d_cnt = J.count ? ar.take<int64_t>(std::max<int64_t>(J.nprob * K, 1)) : nullptr;
        }
    };
    Arena a2;
    layout(a2);
    void* ws2 = nullptr;
    NCF_TRY(ensure_ws(R, 1, a2.off + 256, &ws2));
    a2 = Arena{(char*)ws2, 0};
    layout(a2);

    // transform plans and size groups
    std::map<int64_t, FftPlan> plans;
    std::vector<std::pair<int, int>> groups;  // first task, tasks
    for (int i = 0; i < nreg; ++i) {
        if (!plans.count(rps[i].N)) {
            FftPlan fp;
            NCF_TRY(fft_plan(rps[i].N, true, &fp, J.st, J.tune.fft));
            plans[rps[i].N] = fp;
        }
        if (i == 0 || rps[i].N != rps[i - 1].N)
            groups.push_back({i, 1});
        else
            groups.back().second++;
    }

    // tables: tasks (lattice problems first, then the failed ones), prefix
    // arrays, lags, grid pointers, outputs block, statuses
    const int ntask = (int)J.nprob;
    struct TT {
        RegTask* task;
        int64_t *blk0, *pos0;
        double* lags;
        void** gfwd;
        void** ginv;
        IoBlock* io;
        int32_t* status;
    } dU{}, hU{};
    auto take = [&](Tables& tb) {
        dU.task = tb.take<RegTask>(ntask, &hU.task);
        dU.blk0 = tb.take<int64_t>(nreg + 1, &hU.blk0);
        dU.pos0 = tb.take<int64_t>(nreg + 1, &hU.pos0);
        dU.lags = tb.take<double>(std::max<int64_t>(K, 1), &hU.lags);
        dU.gfwd = tb.take<void*>((size_t)nreg * ng, &hU.gfwd);
        dU.ginv = tb.take<void*>((size_t)nreg * no, &hU.ginv);
        dU.io = tb.take<IoBlock>(1, &hU.io);
        dU.status = tb.take<int32_t>(J.nprob, &hU.status);
    };
    Tables tb;
    take(tb);
    Staging* stg = nullptr;
    NCF_TRY(ensure_stage(R, 1, tb.off, &stg));
    tb = Tables{stg->h, stg->d, 0};
    take(tb);
    int64_t nblocks = 0, total_pos = 0, nsamp = 0;
    double cells_all = 0.0;
    std::vector<bool> has_task(J.nprob, false);
    for (int i = 0; i < nreg; ++i) {
        const RegPlan& rp = rps[i];
        const int64_t p = rp.prob;
        has_task[p] = true;
        RegTask T{};
        for (int si = 0; si < nsets; ++si) {
            const SeriesDesc& d = sdesc[J.set[si].sd0 + p];
            T.t[si] = d.t;
            T.v[si] = d.v64;
            T.w[si] = d.w64;
            T.n[si] = d.n;
            nsamp += d.n;
        }
        T.t_ref = rp.t_ref;
        T.dt = J.dt[p];
        T.tol = 1e-6 * J.dt[p];
        T.h = J.h[p];
        T.G = rp.G;
        T.N = rp.N;
        T.Q = rp.Q;
        T.grids = grids[i];
        T.bad = d_bad + i;
        T.blk0 = nblocks;
        T.pos0 = total_pos;
        const FftPlan& fp = plans[rp.N];
        T.ri.npass = fp.npass;
        for (int q = 0; q < 4; ++q) {
            int lg = 0;
            if (q < fp.npass)
                while ((1 << lg) < fp.radix[q]) ++lg;
            T.ri.lg[q] = lg;
        }
        int lgN = 0;
        while ((1LL << lgN) < rp.N) ++lgN;
        T.ri.lgN = lgN;
        T.st0 = d_stats + J.set[0].sd0 + p;
        T.st1 = J.ccf ? d_stats + J.set[1].sd0 + p : nullptr;
        T.out_off = p * K;
        T.index = p;
        hU.task[i] = T;
        hU.blk0[i] = nblocks;
        hU.pos0[i] = total_pos;
        nblocks += rp.N / kRegCells;
        total_pos += rp.N;
        cells_all += (double)rp.N;
    }
    hU.blk0[nreg] = nblocks;
    hU.pos0[nreg] = total_pos;
    {
        int o = nreg;
        for (int64_t p = 0; p < J.nprob; ++p) {
            hU.status[p] = pstat[p];
            if (has_task[p]) continue;
            RegTask T{};
            T.skip = 1;
            T.skip_status = pstat[p];
            T.out_off = p * K;
            T.index = p;
            hU.task[o++] = T;
        }
    }
    for (int64_t k = 0; k < K; ++k) hU.lags[k] = J.lags[k];
    {
        int of = 0, oi = 0;
        for (auto& gq : groups)
            for (int i = gq.first; i < gq.first + gq.second; ++i) {
                for (int g = 0; g < ng; ++g)
                    hU.gfwd[of + (i - gq.first) + (int64_t)g * gq.second] =
                        grids[i] + 2 * (size_t)rps[i].N * g;
                for (int g = 0; g < no; ++g)
                    hU.ginv[oi + (i - gq.first) + (int64_t)g * gq.second] =
                        grids[i] + 2 * (size_t)rps[i].N * g;
                if (i == gq.first + gq.second - 1) {
                    of += ng * gq.second;
                    oi += no * gq.second;
                }
            }
    }
    *hU.io = IoBlock{};
    hU.io->x[0] = J.set[0].x;
    hU.io->x[1] = J.ccf ? J.set[1].x : nullptr;
    hU.io->c = d_c;
    hU.io->b = d_b;
    hU.io->count = d_cnt;
    hU.io->status = dU.status;
    NCF_TRY_HIP(hipMemcpyAsync(stg->d, stg->h, tb.off, hipMemcpyHostToDevice, J.st));

    // launches
    const RegTask* tasks = dU.task;
    const int64_t* blk0 = dU.blk0;
    const int64_t* pos0 = dU.pos0;
    const double fill_bytes =
        (double)nsamp * (weighted ? 24.0 : 16.0) + cells_all * 16.0 * ng;
    const double prod_bytes = cells_all * 16.0 * (ng + no);
    if (nreg > 0) {
        NCF_TRY(emit(J, [=](hipStream_t s) { return launch_reg_clear(tasks, nreg, s); }));
        NCF_TRY(emit(J, [=](hipStream_t s) {
            return launch_reg_fill(tasks, blk0, nreg, nblocks, mode, s, fill_bytes);
        }));
        int of = 0;
        for (auto& gq : groups) {
            const FftPlan fp = plans[rps[gq.first].N];
            void* const* gp = dU.gfwd + of;
            const int cnt = ng * gq.second;
            NCF_TRY(emit(J, [=](hipStream_t s) { return fft_exec(fp, gp, cnt, +1, true, s); }));
            of += cnt;
        }
        NCF_TRY(emit(J, [=](hipStream_t s) {
            return launch_reg_product(tasks, pos0, nreg, total_pos, mode, s, prod_bytes);
        }));
        int oi = 0;
        for (auto& gq : groups) {
            const FftPlan fp = plans[rps[gq.first].N];
            void* const* gp = dU.ginv + oi;
            const int cnt = no * gq.second;
            NCF_TRY(emit(J, [=](hipStream_t s) { return fft_exec(fp, gp, cnt, -1, true, s); }));
            oi += cnt;
        }
    }
    {
        const double* lg = dU.lags;
        const IoBlock* io = J.io_fixed ? J.io_fixed : dU.io;
        const int kern = J.kern;
        NCF_TRY(emit(J, [=](hipStream_t s) {
            return launch_reg_finish(tasks, ntask, lg, K, mode, kern, io, s);
        }));
    }
    int32_t* h_fstat = hU.status;
    NCF_TRY_HIP(hipMemcpyAsync(h_fstat, J.io_fixed ? J.io_status : dU.status,
                               sizeof(int32_t) * J.nprob, hipMemcpyDeviceToHost, J.st));
    if (!J.dev_ptrs && K > 0) {
        NCF_TRY_HIP(hipMemcpyAsync(J.c, d_c, sizeof(double) * J.nprob * K, hipMemcpyDeviceToHost,
                                   J.st));
        NCF_TRY_HIP(hipMemcpyAsync(J.b, d_b, sizeof(double) * J.nprob * K, hipMemcpyDeviceToHost,
                                   J.st));
        if (J.count)
            NCF_TRY_HIP(hipMemcpyAsync(J.count, d_cnt, sizeof(int64_t) * J.nprob * K,
                                       hipMemcpyDeviceToHost, J.st));
    }
    NCF_TRY_HIP(hipStreamSynchronize(J.st));
    if (g_prof_on) {
        std::lock_guard<std::mutex> lock(g_prof_mu);
        prof_flush_locked();
    }
    const int rc = finish_status(J, pstat, h_fstat);
    if (log_level() > 0) {
        int64_t nbad = 0;
        for (int64_t p = 0; p < J.nprob; ++p)
            nbad += J.plan_build ? pstat[p] != NCF_OK : (h_fstat && h_fstat[p] != NCF_OK);
        std::fprintf(stderr,
                     "ncf: %s%s n=%lld K=%lld %s regular route=lattice grids=%d cells=%lld "
                     "failed=%lld rc=%d\n",
                     J.plan_build ? "plan-build " : "", J.ccf ? "ccf" : "acf",
                     (long long)J.nprob, (long long)J.K,
                     J.kern == NCF_RECTANGLE ? "rectangle" : "gaussian", J.info_grids,
                     (long long)J.info_grid_cells, (long long)nbad, rc);
    }
    return rc;
}

int run_job(Job& J, const double* const* tin, const double* const* xin,
            const double* const* ein);

// Problems of a finished mixed-precision call whose smallest lag-0 scale is
// below kPromoteScale are evaluated again in FP64 (same estimator), and
// their outputs and statuses replace the mixed ones. Each problem takes the
// direct window sums (the real-space estimator itself) unless their work
// (windows x (8 + 8 x samples per window) lane-ops) would take more than
// about 10 ms; then the call's method in FP64. The problems of each choice
// run as one batch call on the call's stream: their series are gathered
// into a workspace of their own (the call's arenas still hold the inputs:
// device copies in host-pointer mode, replicate series of the resampling
// calls), and the batch's rows are scattered back into the outputs.
int promote_batch(Job& J, const std::vector<int64_t>& probs, int method, int32_t* h_fstat);

int promote_fp64(Job& J, const std::vector<int64_t>& probs, int32_t* h_fstat,
                 const std::vector<SeriesStat>& stats) {
    const int64_t K = J.K;
    std::vector<int64_t> direct, other;
    for (int64_t p : probs) {
        const SeriesStat& sw = stats[J.set[0].sd0 + p];
        const int so = J.ccf ? 1 : 0;
        const double nw = (double)(J.set[0].offs[p + 1] - J.set[0].offs[p]);
        const double no = (double)(J.set[so].offs[p + 1] - J.set[so].offs[p]);
        const double dens = (nw - 1.0) / std::max(sw.tmax - sw.tmin, 1e-300);
        const double pts = std::min(dens * 12.0 * J.h[p], nw);
        const double windows = no * (double)(K + 1) + (J.ccf ? nw + no : 0.0);
        (windows * (8.0 + 8.0 * pts) <= 2e10 ? direct : other).push_back(p);
    }
    if (!direct.empty()) NCF_TRY(promote_batch(J, direct, NCF_DIRECT, h_fstat));
    if (!other.empty()) NCF_TRY(promote_batch(J, other, J.opt.method, h_fstat));
    return NCF_OK;
}

int promote_batch(Job& J, const std::vector<int64_t>& probs, int method, int32_t* h_fstat) {
    const int nsets = J.ccf ? 2 : 1;
    const int64_t K = J.K, nb = (int64_t)probs.size();
    const int64_t Kr = std::max<int64_t>(K, 1);
    // workspace: segment tables (per set: values, then times; outputs), the
    // gathered series (per set: t, x and err when present), the batch outputs
    std::vector<CopySeg> segs;
    segs.reserve((size_t)(2 * nsets + 1) * nb);
    int64_t nser[2] = {0, 0};
    size_t seg0[2][2] = {{0, 0}, {0, 0}};
    for (int si = 0; si < nsets; ++si) {
        const SeriesSet& S = J.set[si];
        for (int part = 0; part < 2; ++part) {  // 0: values and errors, 1: times
            seg0[si][part] = segs.size();
            int64_t at = 0;
            for (int64_t p : probs) {
                const int64_t o = S.offs[p], n = S.offs[p + 1] - o;
                segs.push_back({part == 1 && S.shared_t ? 0 : o, at, n});
                at += n;
            }
            nser[si] = at;
        }
    }
    const size_t segout = segs.size();
    for (int64_t i = 0; i < nb; ++i) segs.push_back({i * Kr, probs[i] * K, K});
    size_t bytes = sizeof(CopySeg) * segs.size();
    bytes = (bytes + 255) & ~(size_t)255;
    const size_t data0 = bytes;
    for (int si = 0; si < nsets; ++si)
        bytes += sizeof(double) * (size_t)nser[si] * (J.set[si].err ? 3 : 2);
    const size_t out0 = bytes;
    bytes += sizeof(double) * 2 * (size_t)(nb * Kr);
    char* ws = nullptr;
    if (hipMalloc((void**)&ws, bytes) != hipSuccess) {
        (void)hipGetLastError();
        set_error("workspace allocation for the FP64 re-evaluation failed");
        return NCF_E_NOMEM;
    }
    std::unique_ptr<char, void (*)(char*)> ws_guard(ws, [](char* q) { (void)hipFree(q); });
    CopySeg* d_segs = (CopySeg*)ws;
    NCF_TRY_HIP(hipMemcpyAsync(d_segs, segs.data(), sizeof(CopySeg) * segs.size(),
                               hipMemcpyHostToDevice, J.st));
    Job P;
    P.ccf = J.ccf;
    P.nprob = nb;
    P.kern = J.kern;
    P.h.resize((size_t)nb);
    for (int64_t i = 0; i < nb; ++i) P.h[(size_t)i] = J.h[probs[(size_t)i]];
    P.lags = J.lags;
    P.K = K;
    P.c = (double*)(ws + out0);
    P.b = P.c + nb * Kr;
    P.count = nullptr;
    // a status left at kUnset after the call means the call itself failed
    constexpr int kUnset = 1;
    std::vector<int> pst((size_t)nb, kUnset);
    P.status = pst.data();
    P.opt = J.opt;
    P.opt.precision = NCF_FP64;
    P.opt.method = method;
    P.opt.flags = (J.opt.flags & (NCF_SPECTRAL_ALWAYS | NCF_WINDOW_QUEUE)) | NCF_DEVICE_POINTERS;
    P.dev_ptrs = true;
    P.st = J.st;
    Resources R2;
    R2.exact = true;
    P.res = &R2;
    P.no_b = J.no_b;
    const double* tin[2] = {nullptr, nullptr};
    const double* xin[2] = {nullptr, nullptr};
    const double* ein[2] = {nullptr, nullptr};
    double* at = (double*)(ws + data0);
    for (int si = 0; si < nsets; ++si) {
        const SeriesSet& S = J.set[si];
        const int64_t n = nser[si];
        double* gt = at;
        double* gx = gt + n;
        double* ge = S.err ? gx + n : nullptr;
        at += n * (S.err ? 3 : 2);
        const double* sv[3] = {S.x, S.err, nullptr};
        double* dv[3] = {gx, ge, nullptr};
        NCF_TRY(launch_copy_segments(d_segs + seg0[si][0], nb, sv, dv, J.st));
        const double* st3[3] = {S.t, nullptr, nullptr};
        double* dt3[3] = {gt, nullptr, nullptr};
        NCF_TRY(launch_copy_segments(d_segs + seg0[si][1], nb, st3, dt3, J.st));
        SeriesSet& Q = P.set[si];
        Q.ntot = n;
        Q.nser = (int)nb;
        Q.offs.resize((size_t)nb + 1);
        Q.offs[0] = 0;
        for (int64_t i = 0; i < nb; ++i)
            Q.offs[(size_t)i + 1] = Q.offs[(size_t)i] + segs[seg0[si][0] + (size_t)i].len;
        Q.wmode = S.wmode;
        tin[si] = gt;
        xin[si] = gx;
        ein[si] = ge;
    }
    int rc = run_job(P, tin, xin, ein);
    for (int v : pst)
        if (v == kUnset) {  // the batch call failed before reporting statuses
            (void)hipStreamSynchronize(J.st);
            free_resources(R2);
            return rc != NCF_OK ? rc : NCF_E_DEVICE;
        }
    rc = NCF_OK;
    for (int64_t i = 0; i < nb; ++i) h_fstat[probs[(size_t)i]] = pst[(size_t)i];
    if (K > 0) {
        if (J.dev_ptrs) {
            const double* so[3] = {P.c, J.b ? P.b : nullptr, nullptr};
            double* dso[3] = {J.c, J.b, nullptr};
            rc = launch_copy_segments(d_segs + segout, nb, so, dso, J.st);
        } else {
            std::vector<double> hout((size_t)(2 * nb * Kr));
            if (hipMemcpyAsync(hout.data(), P.c, sizeof(double) * hout.size(),
                               hipMemcpyDeviceToHost, J.st) != hipSuccess ||
                hipStreamSynchronize(J.st) != hipSuccess) {
                set_error("copy of the FP64 re-evaluation failed");
                rc = NCF_E_DEVICE;
            } else {
                for (int64_t i = 0; i < nb; ++i) {
                    const int64_t p = probs[(size_t)i];
                    std::memcpy(J.c + p * K, hout.data() + i * Kr, sizeof(double) * K);
                    if (J.b)
                        std::memcpy(J.b + p * K, hout.data() + (nb + i) * Kr, sizeof(double) * K);
                }
            }
        }
    }
    if (hipStreamSynchronize(J.st) != hipSuccess && rc == NCF_OK) {
        set_error("FP64 re-evaluation failed on the device");
        rc = NCF_E_DEVICE;
    }
    free_resources(R2);
    return rc;
}

// The state and steps of one call of the irregular-sampling estimators
// (run_job). A window task of one window launch (the main pass, or the
// fallback pass of the spectral pair counts):
struct WinPlan {
    int wi_set, wo_set;  // window set, outer set (series index = problem)
    int64_t prob;
    int role;            // 0 main, 1 self x, 2 self y, 3 fallback
    // sorted lag offsets of this task (tasks with the same offsets share one
    // list, and one copy of it in the tables)
    std::shared_ptr<const std::vector<double>> dl;
};

// Offsets of the distinct lag-offset lists of a launch's tasks in one table
// (first[i]: task i is the first holder of its list); returns the length.
size_t dl_layout(const std::vector<WinPlan>& plans, std::vector<size_t>* off,
                 std::vector<char>* first) {
    off->assign(plans.size(), 0);
    first->assign(plans.size(), 0);
    std::unordered_map<const std::vector<double>*, size_t> seen;
    seen.reserve(plans.size());
    size_t n = 0;
    for (size_t i = 0; i < plans.size(); ++i) {
        auto it = seen.find(plans[i].dl.get());
        if (it == seen.end()) {
            it = seen.emplace(plans[i].dl.get(), n).first;
            n += plans[i].dl->size();
            (*first)[i] = 1;
        }
        (*off)[i] = it->second;
    }
    return n;
}
// Window tasks of one launch: tile sizes, LDS size, work items.
struct WinLaunch {
    std::vector<WinPlan> plans;
    std::vector<WinTask> wt;
    std::vector<int64_t> item0, wk0, r0;
    int64_t nitems = 0, total_rows = 0, nred1 = 0;
    int cap = 256, jmax = 64;
    double work = 0.0;
};

// A spectral problem and its grid geometry.
struct SpecPlan {
    int64_t prob;
    SpecGeom g;
};

struct Phase2Tables {  // phase-2 tables (device views, host staging)
    WinTask* wt;
    int64_t *item0, *wk0, *r0;
    double* dl;
    SpecTask* st;
    int64_t *tile0, *pos0, *sk0, *pair0, *fe0;
    int32_t* smap;
    int32_t* rinfo;
    double* ev;
    void** gfwd;
    void** ginv;
    int32_t* rowk;   // evaluation index of each window row (-1: none)
    uint64_t* mask;  // fallback flags, written on the device and read back
};

struct Phase3Tables {  // phase-3 tables
    int32_t* status;  // first: right after the flag masks when merged
    double* rmin;     // smallest lag-0 scale per problem (comes back with the statuses)
    WinTask* wt;
    int64_t *item0, *wk0, *r0;
    double* dl;
    int32_t* fbrow;
    int32_t* perm;
    NormTask* nt;
    IoBlock* io;
};

// The steps of one call, in order (run): the moments and the standardization
// (A1), the route choice and the lag rows, the window tasks (A7), the grid
// geometry of the spectral problems (A2), the device workspace, the phase-2
// tables and their upload, the launches of the window scan and of the
// spectral route (A3-A6), the fallback flags of the spectral pair counts,
// then phase 3 (fallback window scans, normalization A8, outputs) and the
// statuses. State that crosses steps lives in the members; every window
// launch checks its tasks' input arrays in check_win.
class CallRun {
   public:
    CallRun(Job& job, const double* const* t, const double* const* x, const double* const* e)
        : J(job), tin(t), xin(x), ein(e), R(*job.res) {}
    int run();

   private:
    void init_flags();
    int moments();
    int plan_route();
    bool weights_fall_back(int64_t p) const;
    void plan_window(WinLaunch& W);
    int check_win(const WinLaunch& W, uint32_t f) const;
    void plan_windows();
    int plan_spectral();
    int alloc_phase2();
    void take2(Tables& tb);
    void take3(Tables& tb, int ntw2, size_t ndl2, bool any_fb);
    int tables_phase2();
    void fill3(int ntw2, bool any_fb);
    int record_window();
    int record_spectral();
    int record_flags();
    void read_flags();
    int launch3(int ntw2, bool with_masks);
    int separate3();
    int done();
    const SeriesStat& stat_of(int si, int64_t s) const { return stats[J.set[si].sd0 + s]; }

    Job& J;
    const double* const* tin;
    const double* const* xin;
    const double* const* ein;
    Resources& R;
    // route and arrays (init_flags)
    bool fp64 = false, spectral = false, rect = false, weighted = false;
    int nsets = 1;
    std::vector<char> short_p;  // problems with a series too short for the spectral route
    bool any_short = false, numer_in_window = false, need_v32 = false, need_v64 = false,
         need_prefix = false, v32_needed = false, v64_needed = false;
    // phase 1
    std::vector<SeriesDesc> sdesc;
    std::vector<Chunk> chunks;
    int nsd = 0, nch = 0;
    double *d_cpart = nullptr, *d_ctot = nullptr, *d_lagc = nullptr;
    SeriesStat* d_stats = nullptr;
    Chunk* d_ch = nullptr;
    MomentsArgs ma{};
    std::vector<SeriesStat> stats;
    std::vector<int> pstat;
    // route choice, lag rows, window flags
    int64_t K = 0;
    double maxlag = 0.0;
    std::vector<SpecGeom> geom;
    std::vector<char> have_geom, direct_p;
    std::vector<char> fb_direct;  // weighted problems sent to the direct sums (every lag falls back)
    bool any_direct = false, spec_b = false, spec_w = false, spec_unw = false;
    double beta = 0.1;
    std::vector<std::pair<double, int>> rows;
    int Krow = 0;
    std::vector<double> delta;
    std::vector<int32_t> perm;
    int row0 = -1;
    uint32_t wflags = 0;
    // window launches: main pass, fallback pass
    WinLaunch W1, W2;
    int ntw = 0;
    // spectral problems and their device arrays
    std::vector<SpecPlan> splans;
    int nts = 0, Keval = 0;
    size_t csz = 8;
    bool two_grids = false, three_grids = false;
    int nfwd = 1;
    std::vector<void*> grids, gridbs, gridcs, ybufs;
    std::vector<double*> fparts, numer, bspec, spart, bunw;
    int64_t ntiles_all = 0;
    bool bounds_pass = false;
    int64_t* d_rng = nullptr;
    double *d_c = nullptr, *d_b = nullptr;
    int64_t* d_cnt = nullptr;
    // tables
    Phase2Tables dT{}, hT{};
    Phase3Tables dU{}, hU{};
    int fwords = 1;
    bool flag_pass = false, speculate = false, merge3 = false, combine = false;
    size_t ndl = 0;
    Tables t2;
    Staging* stg2 = nullptr;
    std::map<int64_t, FftPlan> plans;
    int64_t total_pos = 0, ntiles = 0, total_samp = 0, total_pairs = 0, fold_blocks = 0,
            mid_out = 0;
    bool fold_chunks = false;
    double spread_bytes = 0.0;
    std::vector<std::pair<int, int>> groups, fwd_groups, inv_groups;
    std::vector<int> spec_of;
    std::vector<std::vector<int>> flagged;
    std::vector<size_t> dl2_off;  // fallback tasks' lag offsets in the phase-3 table
    std::vector<char> dl2_first;
    unsigned long long* qbase = nullptr;
    int32_t* h_fstat = nullptr;
    double* h_rmin = nullptr;
    std::chrono::steady_clock::time_point t_start = std::chrono::steady_clock::now();
    void log_call(int rc) const;
    // NCF_LOG >= 3: host time of each step, in the call's log line
    int log = 0;
    std::chrono::steady_clock::time_point t_mark = t_start;
    std::string steps;
    void mark(const char* name) {
        if (log < 3) return;
        const auto now = std::chrono::steady_clock::now();
        char b[64];
        std::snprintf(b, sizeof(b), " %s=%.3f", name,
                      std::chrono::duration<double, std::milli>(now - t_mark).count());
        steps += b;
        t_mark = now;
    }
};

// Route flags and the derived arrays the call needs.
void CallRun::init_flags() {
    fp64 = J.opt.precision == NCF_FP64;
    spectral = use_spectral(J);  // may turn to the window route after phase 1
    rect = J.kern == NCF_RECTANGLE;
    nsets = J.ccf ? 2 : 1;
    weighted = false;
    for (int si = 0; si < nsets; ++si) weighted |= (ein[si] != nullptr);
    // problems with a series shorter than kMinSpectralSamples take the direct
    // window sums on every route (the spectral route makes no accuracy claim
    // for them); the lengths are known from the offsets
    short_p.assign((size_t)J.nprob, 0);
    any_short = false;
    for (int64_t p = 0; p < J.nprob; ++p) {
        for (int si = 0; si < nsets; ++si)
            if (J.set[si].offs[p + 1] - J.set[si].offs[p] < kMinSpectralSamples) short_p[p] = 1;
        any_short |= short_p[p] != 0;
    }
    numer_in_window = !spectral;  // C from the window scan
    need_v32 = spectral && !fp64;
    // FP64 values: FP64 spreading, and every Gaussian window pass (its direct
    // numerator backs up the spectral one at lags with few pairs), and the
    // rectangle window numerator of the direct problems
    need_v64 = (spectral && fp64) || numer_in_window || !rect || any_short;
    // prefix sums for the rectangle window pass: values (numerator in the
    // window), weights and the nonzero-weight count (weighted calls)
    need_prefix = rect && !J.regular;
    v32_needed = need_v32 && !J.regular;
    v64_needed = need_v64 || J.regular;
}

// Phase 1 (A1): per-chunk moments of every series, the statistics and the
// per-problem statuses back on the host, then the standardization (and the
// prefix sums) of all series in one launch.
int CallRun::moments() {
    // ------------------------------------------------ phase 1: A1 moments
    // chunks of every series of every set, one launch for all of them
    sdesc.clear();
    chunks.clear();
    for (int si = 0; si < nsets; ++si) {
        SeriesSet& S = J.set[si];
        S.sd0 = (int)sdesc.size();
        for (int s = 0; s < S.nser; ++s) {
            SeriesDesc d{};
            d.n = S.offs[s + 1] - S.offs[s];
            d.set = si;
            d.chunk0 = (int32_t)chunks.size();
            int32_t nc = 0;
            for (int64_t b = 0; b < d.n; b += kChunk) {
                chunks.push_back(Chunk{b, std::min(b + kChunk, d.n), (int32_t)sdesc.size(), 0});
                ++nc;
            }
            d.nchunk = nc;
            sdesc.push_back(d);
        }
    }
    nsd = (int)sdesc.size();
    nch = (int)chunks.size();

    // device workspace of phase 1: inputs (host mode), derived arrays, partials
    const bool lags_with_stats = J.lags_dev && !J.rec;
    auto layout1 = [&](Arena& ar, double** o_cpart, double** o_ctot, SeriesStat** o_stats,
                       double** o_lagc) {
        for (int si = 0; si < nsets; ++si) {
            SeriesSet& S = J.set[si];
            if (J.dev_ptrs) {
                S.t = tin[si];
                S.x = xin[si];
                S.err = ein[si];
            } else {
                S.t = ar.take<double>(S.shared_t ? S.offs[1] : S.ntot);
                S.x = ar.take<double>(S.ntot);
                S.err = ein[si] ? ar.take<double>(S.ntot) : nullptr;
            }
            S.v32 = v32_needed ? ar.take<float>(S.ntot) : nullptr;
            S.v64 = v64_needed ? ar.take<double>(S.ntot) : nullptr;
            // weights (and their prefix sums) for every set of a weighted
            // call: a set without errors gets unit weights, since the pair
            // weight w_i w_j of a CCF with errors on one side only needs
            // both (the window passes read both arrays)
            S.w64 = weighted ? ar.take<double>(S.ntot) : nullptr;
            S.pv = need_prefix ? ar.take<double>(S.ntot + S.nser) : nullptr;
            S.pw = (need_prefix && weighted) ? ar.take<double>(S.ntot + S.nser) : nullptr;
            S.pz = (need_prefix && weighted) ? ar.take<double>(S.ntot + S.nser) : nullptr;
        }
        *o_cpart = ar.take<double>(kChunkPart * (size_t)nch);
        *o_ctot = ar.take<double>(3 * (size_t)nch);
        *o_stats = ar.take<SeriesStat>(nsd);
        // device lags of a one-shot call: copied next to the statistics by
        // the moments launch, so one readback brings both (recorded launches
        // must not keep the caller's lag pointer: they copy them apart)
        *o_lagc = ar.take<double>(lags_with_stats ? J.K : 0);
    };
    Arena a1;
    layout1(a1, &d_cpart, &d_ctot, &d_stats, &d_lagc);
    void* ws1 = nullptr;
    NCF_TRY(ensure_ws(R, 0, a1.off + 256, &ws1));
    a1 = Arena{(char*)ws1, 0};
    layout1(a1, &d_cpart, &d_ctot, &d_stats, &d_lagc);
    // bytes from the statistics to the end of the lag copy (the readback)
    const size_t stat_span = lags_with_stats
                                 ? (size_t)((char*)(d_lagc + J.K) - (char*)d_stats)
                                 : sizeof(SeriesStat) * nsd;
    if (!J.dev_ptrs) {
        for (int si = 0; si < nsets; ++si) {
            SeriesSet& S = J.set[si];
            const size_t by = sizeof(double) * S.ntot;
            const size_t byt = sizeof(double) * (S.shared_t ? S.offs[1] : S.ntot);
            NCF_TRY_HIP(hipMemcpyAsync((void*)S.t, tin[si], byt, hipMemcpyHostToDevice, J.st));
            NCF_TRY_HIP(hipMemcpyAsync((void*)S.x, xin[si], by, hipMemcpyHostToDevice, J.st));
            if (ein[si])
                NCF_TRY_HIP(
                    hipMemcpyAsync((void*)S.err, ein[si], by, hipMemcpyHostToDevice, J.st));
        }
    }
    for (int si = 0; si < nsets; ++si) {
        const SeriesSet& S = J.set[si];
        for (int s = 0; s < S.nser; ++s) {
            SeriesDesc& d = sdesc[S.sd0 + s];
            const int64_t o = S.offs[s];
            d.t = S.shared_t ? S.t : S.t + o;
            d.wmode = S.wmode ? 1 : 0;
            d.xoff = o;
            d.err = S.err ? S.err + o : nullptr;
            d.v32 = S.v32 ? S.v32 + o : nullptr;
            d.v64 = S.v64 ? S.v64 + o : nullptr;
            d.w64 = S.w64 ? S.w64 + o : nullptr;
            d.pv = S.pv ? S.pv + o + s : nullptr;
            d.pw = S.pw ? S.pw + o + s : nullptr;
            d.pz = S.pz ? S.pz + o + s : nullptr;
        }
    }
    Staging* stg1 = nullptr;
    Tables t1;
    {
        SeriesDesc* hs;
        Chunk* hc;
        IoBlock* hio;
        char* hst;
        t1.take<SeriesDesc>(nsd, &hs);
        t1.take<Chunk>(nch, &hc);
        t1.take<IoBlock>(1, &hio);
        t1.take<char>(stat_span, &hst);
        double* hl;
        t1.take<double>(J.lags_dev && !lags_with_stats ? J.K : 0, &hl);
    }
    NCF_TRY(ensure_stage(R, 0, t1.off, &stg1));
    t1 = Tables{stg1->h, stg1->d, 0};
    SeriesDesc* h_sd;
    Chunk* h_ch;
    IoBlock* h_io1;
    SeriesStat* h_stats;
    SeriesDesc* d_sd = t1.take<SeriesDesc>(nsd, &h_sd);
    d_ch = t1.take<Chunk>(nch, &h_ch);
    IoBlock* d_io1 = t1.take<IoBlock>(1, &h_io1);
    // host landing area of the statistics (and of the lag copy behind them,
    // laid out as on the device)
    char* h_span;
    t1.take<char>(stat_span, &h_span);
    h_stats = reinterpret_cast<SeriesStat*>(h_span);
    double* h_lags;
    t1.take<double>(J.lags_dev && !lags_with_stats ? J.K : 0, &h_lags);  // device lags apart
    if (lags_with_stats) h_lags = reinterpret_cast<double*>(h_span + ((char*)d_lagc - (char*)d_stats));
    std::memcpy(h_sd, sdesc.data(), sizeof(SeriesDesc) * nsd);
    std::memcpy(h_ch, chunks.data(), sizeof(Chunk) * nch);
    *h_io1 = IoBlock{};
    for (int si = 0; si < nsets; ++si) h_io1->x[si] = J.set[si].x;
    const size_t up1 = (size_t)((char*)h_stats - stg1->h);
    NCF_TRY_HIP(hipMemcpyAsync(stg1->d, stg1->h, up1, hipMemcpyHostToDevice, J.st));
    ma = MomentsArgs{};
    ma.series = d_sd;
    ma.chunks = d_ch;
    ma.nseries = nsd;
    ma.nchunks = nch;
    ma.chunk_part = d_cpart;
    ma.chunk_tot = d_ctot;
    ma.stats = d_stats;
    ma.io = J.io_fixed ? J.io_fixed : d_io1;
    ma.prefix = need_prefix ? 1 : 0;
    if (lags_with_stats) {
        ma.lag_src = J.lags_dev;
        ma.lag_dst = d_lagc;
        ma.nlag = J.K;
    }
    NCF_TRY(emit(J, [m = ma](hipStream_t s) { return launch_moments(m, s); }));
    NCF_TRY_HIP(hipMemcpyAsync(h_span, d_stats, stat_span, hipMemcpyDeviceToHost, J.st));
    if (J.lags_dev && !lags_with_stats)
        NCF_TRY_HIP(hipMemcpyAsync(h_lags, J.lags_dev, sizeof(double) * J.K,
                                   hipMemcpyDeviceToHost, J.st));
    NCF_TRY_HIP(hipStreamSynchronize(J.st));
    if (J.lags_dev) {
        std::memcpy(J.lags.data(), h_lags, sizeof(double) * J.K);
        J.lags_dev = nullptr;
        NCF_TRY(check_lags(J));
    }
    stats.assign(h_stats, h_stats + nsd);

    // per-problem status from its series
    pstat.assign(J.nprob, NCF_OK);
    for (int64_t p = 0; p < J.nprob; ++p) {
        for (int si = 0; si < nsets; ++si) {
            int s = stat_of(si, p).status;
            if (s != NCF_OK && pstat[p] == NCF_OK) pstat[p] = s;
        }
        if (pstat[p] == NCF_OK && !(J.h[p] > 0.0 && std::isfinite(J.h[p])))
            pstat[p] = NCF_E_INVALID_ARG;
    }

    // standardization (+ prefix sums), all series in one launch
    NCF_TRY(emit(J, [m = ma](hipStream_t s) { return launch_standardize(m, s); }));
    return NCF_OK;
}

// Route choice (the K* crossover of NCF_AUTO), the sorted lag rows of the
// window scans and the window flags.
// Weighted Gaussian problem of the spectral route: would every lag fall back
// to the direct window sums? The spectral weighted pair sums B serve the lags
// with B(tau) >= beta B_ref (B_ref: B(0), CCF sqrt(B_xx(0) B_yy(0))). B(0)
// holds the self-pairs, sum w^2, which weights spread over decades make
// dominant. With the samples spread evenly over their span T, a sample's
// neighbours at any lag carry weight sw / T per unit time, so B(tau) is at
// most about sw_x sw_y h sqrt(2 pi) / T and B(0) is sum w^2 + sw^2 h
// sqrt(2 pi) / T. The estimate leaves out two factors that lower the tested
// B(tau) further (the overlap 1 - |tau| / T of the spans, and for the ACF
// the lag-0 scale min(1, r(0)) that the test applies) and one that raises
// it (samples clustered in seasons or bursts put more pairs at small lags);
// measured on light curves with errors over four decades, problems whose
// estimate lay between a quarter of the threshold and the threshold still
// sent 94-97 % of their lags to the fallback.
bool CallRun::weights_fall_back(int64_t p) const {
    const double beta_p = fp64 ? 1e-2 : 0.1;  // the fallback threshold below
    const double kint = J.h[p] * 2.5066282746310002;  // integral of the kernel
    const SeriesStat& a = stat_of(0, p);
    const SeriesStat& b = stat_of(J.ccf ? 1 : 0, p);
    const double ta = std::max(a.tmax - a.tmin, 1e-300);
    const double tb = std::max(b.tmax - b.tmin, 1e-300);
    const double b0a = a.sw2 + a.sw * a.sw * kint / ta;
    const double b0b = b.sw2 + b.sw * b.sw * kint / tb;
    const double bref = std::sqrt(b0a * b0b);
    const double btau = a.sw * b.sw * kint / std::max(ta, tb);
    return bref > 0.0 && btau < beta_p * bref;
}

int CallRun::plan_route() {
    // ------------------------------------------------ phase 2 planning (host)
    K = J.K;
    maxlag = 0.0;
    for (double v : J.lags) maxlag = std::max(maxlag, std::fabs(v));
    // NCF_AUTO, Gaussian: the real-space route (direct window sums) when its
    // work is below the spectral pipeline's, the paper's K* crossover
    // (Sec. "Choosing an estimator"). Window cost: windows x (8 + 8 x samples
    // per window) lane-ops at the scan's measured rate (5e12/s mixed, 2e12/s
    // FP64); spectral cost: about 11 passes over the grids at 4 TB/s plus
    // 30 us for its extra launches and the fallback round trip.
    // grid geometry per problem, planned once (the route choice and the
    // spectral planning below both use it)
    // Lag lattice: Gaussian spectral problems through the fused kernel (the
    // fold needs the product tiles in LDS) read lags that sit on a lattice off
    // a folded spectrum instead of an inverse transform and interpolation.
    {
        const bool sb = spectral && !rect && J.opt.method == NCF_AUTO;
        const bool su = sb && weighted && !J.no_b;
        J.lag_unit = 0.0;
        if (spectral && J.kern == NCF_GAUSSIAN && J.opt.grid_size <= 0 && !J.tune.no_mid &&
            !J.tune.eval_interp && mid_supported(J.ccf, sb, su, fp64))
            J.lag_unit = lag_lattice_unit(J.lags, !J.ccf);
    }
    geom.assign((size_t)J.nprob, SpecGeom{});
    have_geom.assign((size_t)J.nprob, 0);
    fb_direct.assign((size_t)J.nprob, 0);
    if (spectral && J.opt.method == NCF_AUTO && J.kern == NCF_GAUSSIAN &&
        !(J.opt.flags & NCF_SPECTRAL_ALWAYS)) {
        const double nrows = (double)(J.ccf ? K : K + 1);
        const double rate = fp64 ? 2e12 : 5e12;
        const double csz_b = fp64 ? 16.0 : 8.0;
        double direct_s = 0.0, spec_s = 30e-6;
        // grid geometry of every problem (independent: host threads for
        // large batches), then the costs in problem order
        std::vector<int> grc((size_t)J.nprob, NCF_OK);
        host_parallel_for(J.nprob, [&](int64_t p) {
            if (pstat[p] != NCF_OK) return;
            double tmin = stat_of(0, p).tmin, tmax = stat_of(0, p).tmax;
            if (J.ccf) {
                tmin = std::min(tmin, stat_of(1, p).tmin);
                tmax = std::max(tmax, stat_of(1, p).tmax);
            }
            grc[p] = plan_grid(J, tmin, tmax, maxlag, J.h[p], &geom[p]);
        });
        for (int64_t p = 0; p < J.nprob; ++p) {
            if (pstat[p] != NCF_OK) continue;
            const SeriesStat& s0 = stat_of(0, p);
            const double n0 = (double)(J.set[0].offs[p + 1] - J.set[0].offs[p]);
            const double n1 = J.ccf ? (double)(J.set[1].offs[p + 1] - J.set[1].offs[p]) : n0;
            const double dens = (n0 - 1.0) / std::max(s0.tmax - s0.tmin, 1e-300);
            const double pts = dens * 12.0 * J.h[p];
            const double windows = n1 * nrows + (J.ccf ? n0 + n1 : 0.0);
            const double dcost = windows * (8.0 + 8.0 * pts) / rate;
            direct_s += dcost;
            const SpecGeom& g = geom[p];
            if (grc[p] != NCF_OK) {
                clear_error();
                direct_s = 0.0;  // no grid fits: the window route
                break;
            }
            have_geom[p] = 1;
            if (weighted && weights_fall_back(p)) {
                fb_direct[p] = 1;
                spec_s += dcost;
                continue;
            }
            spec_s += (g.P > 0 ? 7.0 : 11.0) * (double)g.N * csz_b * (J.ccf ? 2.0 : 1.0) / 4e12 +
                      (n0 + (J.ccf ? n1 : 0.0)) * 12.0 / 4e12;
        }
        if (direct_s < spec_s) spectral = false;
    }
    // per problem: the direct window sums (no spectral grid)
    direct_p.assign((size_t)J.nprob, 0);
    any_direct = false;
    for (int64_t p = 0; p < J.nprob; ++p) {
        direct_p[p] = (!spectral || short_p[p] || fb_direct[p]) ? 1 : 0;
        any_direct |= direct_p[p] != 0;
    }
    // Gaussian default: numerator and pair count both by the spectral route
    // (unit-weight channel); lags whose spectral b is small against the
    // reference are re-evaluated by the direct window scan.
    // Weighted calls: the pair-count channel carries the weights and yields
    // B; one more channel with unit weights yields the unweighted b, unless
    // the caller does not read b (then b is reported equal to B).
    spec_b = spectral && !rect && J.opt.method == NCF_AUTO;
    spec_w = spec_b && weighted;
    spec_unw = spec_w && !J.no_b;
    // Mixed: the FP32 transforms leave |dN|, |db| ~ 7e-7 b_ref on every lag, so
    // |dc| ~ 2 * 7e-7 b_ref / b stays below 1e-5 for b >= 0.1 b_ref. FP64: the
    // limit is the 6h truncation of the window scan, whose effect is
    // relatively large where a lag has few pairs.
    beta = fp64 ? 1e-2 : 0.1;
    // window lag rows: sorted offsets delta = eps * tau (ACF: plus lag 0)
    const double epsv = J.ccf ? -1.0 : 1.0;
    rows.clear();
    for (int64_t k = 0; k < K; ++k) rows.push_back({epsv * J.lags[k], (int)k});
    bool have0 = false;
    for (double v : J.lags) have0 |= (v == 0.0);
    if (!J.ccf && !have0) rows.push_back({0.0, -1});
    std::stable_sort(rows.begin(), rows.end(),
                     [](const std::pair<double, int>& a, const std::pair<double, int>& b) {
                         return a.first < b.first;
                     });
    Krow = (int)rows.size();
    delta.assign(std::max(Krow, 1), 0.0);
    perm.assign(std::max<int64_t>(K, 1), 0);
    row0 = -1;
    for (int r = 0; r < Krow; ++r) {
        delta[r] = rows[r].first;
        if (rows[r].second >= 0) perm[rows[r].second] = r;
        if (rows[r].first == 0.0 && row0 < 0) row0 = r;
    }

    // window flags: the rectangle numerator is always the prefix form; the
    // Gaussian window pass also sums the direct numerator (its weights are
    // already computed), used where the window b is small
    wflags = 0;
    if (rect) wflags |= WIN_RECT;
    if (!rect || numer_in_window) wflags |= WIN_NUMER;
    if (weighted) wflags |= WIN_WEIGHTED;
    if (fp64 && !rect) wflags |= WIN_EXP64;

    // the rectangle window numerator is needed only by the direct problems
    if (rect && !numer_in_window && !any_direct) wflags &= ~(uint32_t)WIN_NUMER;
    return NCF_OK;
}

// Tile sizes, LDS size and work items of the window tasks in W.
void CallRun::plan_window(WinLaunch& W) {
    // staged window arrays: times, values (or their prefix), weights (or
    // their prefix and, rectangle, the nonzero-weight count prefix)
    const int arrays = 1 + ((W.plans.empty() ? false : ((wflags & WIN_NUMER) != 0)) ? 1 : 0) +
                       (weighted ? (rect ? 2 : 1) : 0);
    const int jmax = 1024;
    // LDS per workgroup (doubles): Gaussian items stage the window arrays
    // and their outer samples; rectangle items stage only the window
    // arrays and keep a smaller footprint, for more resident workgroups
    const int budget = (rect ? 24 : 40) * 1024 / 8;
    int cap = rect ? budget / arrays - 8 : (budget - jmax * arrays) / arrays - 8;
    cap = std::max(256, std::min(4096, cap));
    const int ntask = (int)W.plans.size();
    W.wt.assign(ntask, WinTask{});
    W.item0.assign(ntask + 1, 0);
    W.wk0.assign(ntask + 1, 0);
    W.r0.assign(ntask + 1, 0);
    std::vector<std::array<double, 3>> dens(ntask);  // window / outer density, extent
    for (int i = 0; i < ntask; ++i) {
        const WinPlan& P = W.plans[i];
        const SeriesSet& SW = J.set[P.wi_set];
        const SeriesSet& SO = J.set[P.wo_set];
        const SeriesDesc& dw = sdesc[SW.sd0 + P.prob];
        const SeriesDesc& dO = sdesc[SO.sd0 + P.prob];
        const SeriesStat& sw = stat_of(P.wi_set, P.prob);
        const SeriesStat& so = stat_of(P.wo_set, P.prob);
        const double h = J.h[P.prob];
        WinTask T{};
        T.t = dw.t;
        T.n_win = dw.n;
        T.s = dO.t;
        T.n_out = dO.n;
        if (wflags & WIN_NUMER) {
            if (rect)
                T.pv = dw.pv;
            else
                T.v = dw.v64;
            T.vo = dO.v64;
        }
        if (weighted) {
            if (rect) {
                T.pw = dw.pw;
                T.pz = dw.pz;
            } else {
                T.w = dw.w64;
            }
            T.wo = dO.w64;
        }
        // chunk offsets of the window series' (chunk-local) prefix sums
        if (rect) T.poff = d_ctot + 3 * (int64_t)dw.chunk0;
        const std::vector<double>& dl = *P.dl;
        T.K = (int32_t)dl.size();
        T.h = h;
        T.W = rect ? h : 6.0 * h;
        double lext = 0.0;
        for (size_t r = 0; r < dl.size(); r += 64) {
            const size_t r1 = std::min(dl.size(), r + 64) - 1;
            lext = std::max(lext, dl[r1] - dl[r]);
        }
        const double span_w = std::max(sw.tmax - sw.tmin, 1e-300);
        const double span_o = std::max(so.tmax - so.tmin, 1e-300);
        const double dens_w = (double)(dw.n - 1) / span_w;
        const double dens_o = (double)(dO.n - 1) / span_o;
        const int n_kt = (int)ceil_div(T.K, 64);
        const double ext = lext + 2.0 * T.W;
        auto est = [&](int64_t j) { return dens_w * ((double)j / dens_o + ext) + 2.0; };
        // outer samples per workgroup: as many as keep the window range in
        // LDS (half the capacity, for clustering) while leaving at least
        // 2048 work items (eight per CU) when the problem is big enough
        int64_t Jt = 64;
        while (Jt * 2 <= jmax && est(Jt * 2) <= 0.5 * cap &&
               (double)dO.n * n_kt / (double)(Jt * 2) >= 2048.0)
            Jt *= 2;
        while (Jt > 16 && est(Jt) > 0.5 * cap) Jt /= 2;
        if (J.tune.jscale > 0) Jt = std::min<int64_t>(Jt << J.tune.jscale, jmax);
        if (J.tune.jscale < 0) Jt = std::max<int64_t>(Jt >> -J.tune.jscale, 16);
        T.J = (int32_t)Jt;
        T.n_kt = n_kt;
        dens[i] = {dens_w, dens_o, ext};
        // algorithmic work: per (j, k) window, searches + per-point weight ops
        const double pts = rect ? 0.0 : dens_w * 2.0 * T.W;
        W.work += (double)dO.n * T.K * (8.0 + (rect ? 4.0 : 8.0 * pts));
        W.wt[i] = T;
    }
    // the launch has one LDS size, set by the largest footprint
    double need = 0.0;
    int jneed = 16;
    auto est_of = [&](int i, int64_t j) {
        return dens[i][0] * ((double)j / dens[i][1] + dens[i][2]) + 2.0;
    };
    for (int i = 0; i < ntask; ++i) {
        need = std::max(need, est_of(i, W.wt[i].J));
        jneed = std::max(jneed, (int)W.wt[i].J);
    }
    // LDS: twice the estimated window range (clustering margin), rounded up
    const int want = (int)std::min<double>(cap, round_up((int64_t)(2.0 * need) + 64, 64));
    W.cap = std::max(256, want);
    W.jmax = (int)round_up(jneed, 64);
    // items of few lags (e.g. the lag-0 scale tasks) grow within that
    // footprint until they hold ~8192 windows: a workgroup's searches and
    // staging cost the same for any size
    for (int i = 0; i < ntask; ++i) {
        WinTask& T = W.wt[i];
        const int64_t kin = std::min<int64_t>(T.K, 64);
        int64_t Jt = T.J;
        while (Jt * 2 <= W.jmax && est_of(i, Jt * 2) <= 0.5 * W.cap && Jt * 2 * kin <= 8192)
            Jt *= 2;
        T.J = (int32_t)Jt;
    }
    // j-tiles per work item: one item per tile while that leaves the
    // launch few items; more tiles per item (one partial per group of
    // tiles) when the launch has many
    int64_t tiles = 0;
    for (int i = 0; i < ntask; ++i) {
        WinTask& T = W.wt[i];
        T.n_jt = (int32_t)ceil_div(T.n_out, T.J);
        tiles += (int64_t)T.n_jt * T.n_kt;
    }
    const int G = (int)std::max<int64_t>(1, std::min<int64_t>(kWinGroupMax,
                                                              tiles / kWinItemsMin));
    for (int i = 0; i < ntask; ++i) {
        WinTask& T = W.wt[i];
        T.G = G;
        T.n_jg = (int32_t)ceil_div(T.n_jt, G);
        T.item0 = W.nitems;
        W.item0[i] = W.nitems;
        W.wk0[i] = W.total_rows;
        W.r0[i] = W.nred1;
        W.nitems += (int64_t)T.n_jg * T.n_kt;
        W.nred1 += (int64_t)T.n_kt * ceil_div(T.n_jg, kWinJc);
        W.total_rows += T.K;
    }
    W.item0[ntask] = W.nitems;
    W.wk0[ntask] = W.total_rows;
    W.r0[ntask] = W.nred1;
}

// every array that a window pass reads must exist: checked on the host
// before the launch, since a missing one would be read on the device
int CallRun::check_win(const WinLaunch& W, uint32_t f) const {
    const bool need_num = (f & WIN_NUMER) != 0, wtd = (f & WIN_WEIGHTED) != 0;
    for (const WinTask& T : W.wt) {
        bool ok = T.t != nullptr && T.s != nullptr && (!rect || T.poff != nullptr);
        if (need_num) ok = ok && (rect ? T.pv != nullptr : T.v != nullptr) && T.vo != nullptr;
        if (wtd)
            ok = ok && (rect ? (T.pw != nullptr && T.pz != nullptr) : T.w != nullptr) &&
                 T.wo != nullptr;
        if (!ok) {
            set_error("window pass: a task lacks one of its input arrays");
            return NCF_E_INVALID_ARG;
        }
    }
    return NCF_OK;
}

// The main window launch: every problem that the spectral route does not
// take whole (its numerator and pair counts, or the CCF lag-0 scales).
void CallRun::plan_windows() {
    W1 = WinLaunch{};
    const auto dall = std::make_shared<const std::vector<double>>(delta);
    const auto dzero = std::make_shared<const std::vector<double>>(1, 0.0);
    for (int64_t p = 0; p < J.nprob; ++p) {
        if (pstat[p] != NCF_OK || (spec_b && !direct_p[p])) continue;
        if (!J.ccf) {
            W1.plans.push_back({0, 0, p, 0, dall});
        } else {
            if (Krow > 0) W1.plans.push_back({0, 1, p, 0, dall});
            W1.plans.push_back({0, 0, p, 1, dzero});
            W1.plans.push_back({1, 1, p, 2, dzero});
        }
    }
    if (Krow == 0) delta.assign(1, 0.0);
    plan_window(W1);
    ntw = (int)W1.plans.size();
}

// Spectral problems (A2), sorted by grid size so grids of one size are
// contiguous, and the grids each needs.
int CallRun::plan_spectral() {
    splans.clear();
    if (spectral) {
        auto range = [&](int64_t p, double* tmin, double* tmax) {
            *tmin = stat_of(0, p).tmin;
            *tmax = stat_of(0, p).tmax;
            if (J.ccf) {
                *tmin = std::min(*tmin, stat_of(1, p).tmin);
                *tmax = std::max(*tmax, stat_of(1, p).tmax);
            }
        };
        // geometry of the problems the route choice did not plan (host
        // threads for large batches)
        std::vector<int> grc((size_t)J.nprob, NCF_OK);
        host_parallel_for(J.nprob, [&](int64_t p) {
            if (pstat[p] != NCF_OK || direct_p[p] || have_geom[p]) return;
            double tmin, tmax;
            range(p, &tmin, &tmax);
            grc[p] = plan_grid(J, tmin, tmax, maxlag, J.h[p], &geom[p]);
        });
        // problems by grid size, stable (counting sort on log2 N)
        int64_t cnt[65] = {0};
        for (int64_t p = 0; p < J.nprob; ++p) {
            if (pstat[p] != NCF_OK || direct_p[p]) continue;
            if (grc[p] != NCF_OK) {
                // the first failure in problem order; planned again here so
                // that its message is this thread's
                double tmin, tmax;
                range(p, &tmin, &tmax);
                NCF_TRY(plan_grid(J, tmin, tmax, maxlag, J.h[p], &geom[p]));
            }
            cnt[1 + ilog2_exact(geom[p].N)]++;
        }
        for (int b = 1; b < 65; ++b) cnt[b] += cnt[b - 1];
        splans.resize((size_t)cnt[64]);
        for (int64_t p = 0; p < J.nprob; ++p) {
            if (pstat[p] != NCF_OK || direct_p[p]) continue;
            splans[(size_t)cnt[ilog2_exact(geom[p].N)]++] = SpecPlan{p, geom[p]};
        }
    }
    nts = (int)splans.size();
    Keval = (int)(J.ccf ? K : K + 1);
    J.info_grids = nts;
    J.info_grid_cells = 0;
    J.info_fold_grids = 0;
    for (auto& sp : splans) {
        J.info_grid_cells += sp.g.N;
        J.info_fold_grids += sp.g.P > 0 ? 1 : 0;
    }
    J.info_window_items = W1.nitems;
    J.info_window_launches = ntw > 0 ? 1 : 0;
    csz = fp64 ? 16 : 8;
    // second grid: the CCF pair-count channels, or the ACF unit channel of a
    // weighted call; third grid: the CCF unit channels of a weighted call
    two_grids = (spec_b && J.ccf) || spec_unw;
    three_grids = spec_unw && J.ccf;
    nfwd = 1 + (two_grids ? 1 : 0) + (three_grids ? 1 : 0);
    return NCF_OK;
}

// Phase-2 device workspace: window partials and sums, grids, per-lag
// spectral results, spreading-tile ranges and (host-pointer calls) outputs.
int CallRun::alloc_phase2() {
    grids.assign(nts, nullptr);
    gridbs.assign(nts, nullptr);
    gridcs.assign(nts, nullptr);
    ybufs.assign(nts, nullptr);
    fparts.assign(nts, nullptr);
    numer.assign(nts, nullptr);
    bspec.assign(nts, nullptr);
    spart.assign(nts, nullptr);
    bunw.assign(nts, nullptr);
    ntiles_all = 0;
    for (int i = 0; i < nts; ++i) ntiles_all += splans[i].g.N / 4096;
    // sample ranges of the spreading tiles: one pass over the samples when
    // there are many tiles; with a few, each spreading workgroup searches
    bounds_pass = ntiles_all > 4096;
    d_rng = nullptr;  // [tiles][4] sample ranges of every spreading tile
    d_c = d_b = nullptr;
    d_cnt = nullptr;
    auto layout2 = [&](Arena& ar) {
        for (int i = 0; i < ntw; ++i) {
            WinTask& T = W1.wt[i];
            T.part = ar.take<double>((size_t)T.n_jg * T.K * 4);
            T.part2 = ar.take<double>((size_t)ceil_div(T.n_jg, kWinJc) * T.K * 4);
            T.sums = ar.take<double>((size_t)T.K * 4);
        }
        // per-lag spectral results of all problems are contiguous (one readback)
        double* numer_all = ar.take<double>((size_t)std::max(nts, 1) * std::max(Keval, 1));
        double* bspec_all =
            spec_b ? ar.take<double>((size_t)std::max(nts, 1) * std::max(Keval, 1)) : nullptr;
        double* bunw_all =
            spec_unw ? ar.take<double>((size_t)std::max(nts, 1) * std::max(Keval, 1)) : nullptr;
        d_rng = (nts > 0 && bounds_pass) ? ar.take<int64_t>(kTileRec * (size_t)ntiles_all)
                                         : nullptr;
        for (int i = 0; i < nts; ++i) {
            grids[i] = ar.take<char>((size_t)splans[i].g.N * csz);
            if (two_grids) gridbs[i] = ar.take<char>((size_t)splans[i].g.N * csz);
            if (three_grids) gridcs[i] = ar.take<char>((size_t)splans[i].g.N * csz);
            if (splans[i].g.P > 0) {
                ybufs[i] = ar.take<char>((size_t)splans[i].g.P * csz);
                const int64_t nmc = ceil_div(splans[i].g.N / 4096, kFoldTiles);
                if (nmc > 1) fparts[i] = ar.take<double>((size_t)nmc * std::max(Keval, 1) * 2);
            }
            numer[i] = numer_all + (size_t)i * std::max(Keval, 1);
            if (spec_b) bspec[i] = bspec_all + (size_t)i * std::max(Keval, 1);
            if (spec_unw) bunw[i] = bunw_all + (size_t)i * std::max(Keval, 1);
            if (J.ccf) spart[i] = ar.take<double>(4 * (splans[i].g.N / 4096));
        }
        if (J.dev_ptrs) {
            d_c = J.c;
            d_b = J.b;
            d_cnt = J.count;
        } else {
            d_c = ar.take<double>(std::max<int64_t>(J.nprob * K, 1));
            d_b = ar.take<double>(std::max<int64_t>(J.nprob * K, 1));
            d_cnt = J.count ? ar.take<int64_t>(std::max<int64_t>(J.nprob * K, 1)) : nullptr;
        }
    };
    Arena a2;
    layout2(a2);
    void* ws2 = nullptr;
    NCF_TRY(ensure_ws(R, 1, a2.off + 256, &ws2));
    a2 = Arena{(char*)ws2, 0};
    layout2(a2);
    return NCF_OK;
}

// Layout of the phase-3 tables in tb (ntw2 fallback window tasks).
void CallRun::take3(Tables& tb, int ntw2, size_t ndl2, bool any_fb) {
    dU.status = tb.take<int32_t>(J.nprob, &hU.status);
    dU.rmin = tb.take<double>(J.nprob, &hU.rmin);
    dU.wt = tb.take<WinTask>(ntw2, &hU.wt);
    dU.item0 = tb.take<int64_t>(ntw2 + 1, &hU.item0);
    dU.wk0 = tb.take<int64_t>(ntw2 + 1, &hU.wk0);
    dU.r0 = tb.take<int64_t>(ntw2 + 1, &hU.r0);
    dU.dl = tb.take<double>(ndl2, &hU.dl);
    // fallback rows: K entries per problem with fallback lags
    dU.fbrow = tb.take<int32_t>(any_fb ? (size_t)ntw2 * K : 1, &hU.fbrow);
    dU.perm = tb.take<int32_t>(K, &hU.perm);
    dU.nt = tb.take<NormTask>(J.nprob, &hU.nt);
    dU.io = tb.take<IoBlock>(1, &hU.io);
}

// Layout of the phase-2 tables in tb (with phase 3 behind them when merged).
void CallRun::take2(Tables& tb) {
    dT.wt = tb.take<WinTask>(ntw, &hT.wt);
    dT.item0 = tb.take<int64_t>(ntw + 1, &hT.item0);
    dT.wk0 = tb.take<int64_t>(ntw + 1, &hT.wk0);
    dT.r0 = tb.take<int64_t>(ntw + 1, &hT.r0);
    dT.dl = tb.take<double>(ndl, &hT.dl);
    dT.st = tb.take<SpecTask>(nts, &hT.st);
    dT.tile0 = tb.take<int64_t>(nts + 1, &hT.tile0);
    dT.pos0 = tb.take<int64_t>(nts + 1, &hT.pos0);
    dT.pair0 = tb.take<int64_t>(nts + 1, &hT.pair0);
    dT.sk0 = tb.take<int64_t>(nts + 1, &hT.sk0);
    dT.fe0 = tb.take<int64_t>(nts + 1, &hT.fe0);
    dT.smap = tb.take<int32_t>(nsd, &hT.smap);
    dT.rinfo = tb.take<int32_t>(6 * (size_t)nts, &hT.rinfo);
    dT.ev = tb.take<double>(Keval, &hT.ev);
    dT.gfwd = tb.take<void*>(3 * (size_t)nts, &hT.gfwd);
    dT.ginv = tb.take<void*>(2 * (size_t)nts, &hT.ginv);
    dT.rowk = tb.take<int32_t>(flag_pass ? Krow : 0, &hT.rowk);
    dT.mask = tb.take<uint64_t>(flag_pass ? (size_t)nts * fwords : 0, &hT.mask);
    if (merge3) take3(tb, 0, 0, false);  // phase 3 without fallback lags
}

// Phase-2 tables: window tasks and their lag offsets, spectral tasks, FFT
// plans and grid groups, the fallback-flag rows; phase 3 travels with them
// when it does not wait for the flags. One upload.
int CallRun::tables_phase2() {
    fwords = (int)ceil_div(std::max(Krow, 1), 64);
    flag_pass = spec_b && nts > 0 && K > 0;
    // Phase 3 (fallback window scans, normalization, outputs). For the
    // spectral pair counts of a one-shot call it is first enqueued
    // speculatively with no fallback lags, behind the fallback flags: when no
    // lag is flagged (the common case) those outputs are final and the call
    // ends on one round trip; otherwise phase 3 runs again with the flagged
    // lags and rewrites every output. Only calls of a few problems
    // speculate: in large batches some series nearly always has a flagged
    // lag, and phase 3 would be planned and uploaded twice. Recorded launch
    // sequences (plans) take the final path only. When phase 3 does not wait
    // for the flags (no spectral pair counts, or speculation) its tables
    // travel in the phase-2 upload (merge3), and with speculation the flag
    // masks and the statuses, adjacent in the staging, come back in one copy
    // (combine).
    constexpr int64_t kSpeculateMaxProblems = 8;
    speculate = flag_pass && !J.rec && J.nprob <= kSpeculateMaxProblems;
    merge3 = !flag_pass || speculate;
    combine = speculate && !J.io_fixed;
    ndl = 0;
    std::vector<size_t> dl_off;
    std::vector<char> dl_first;
    ndl = dl_layout(W1.plans, &dl_off, &dl_first);
    t2 = Tables{};
    take2(t2);
    stg2 = nullptr;
    NCF_TRY(ensure_stage(R, 1, t2.off, &stg2));
    t2 = Tables{stg2->h, stg2->d, 0};
    take2(t2);

    // window tables: each task's sorted lag offsets
    {
        for (int i = 0; i < ntw; ++i) {
            if (dl_first[i])
                std::memcpy(hT.dl + dl_off[i], W1.plans[i].dl->data(),
                            sizeof(double) * W1.plans[i].dl->size());
            W1.wt[i].delta = dT.dl + dl_off[i];
        }
    }
    if (ntw) {
        std::memcpy(hT.wt, W1.wt.data(), sizeof(WinTask) * ntw);
        std::memcpy(hT.item0, W1.item0.data(), sizeof(int64_t) * (ntw + 1));
        std::memcpy(hT.wk0, W1.wk0.data(), sizeof(int64_t) * (ntw + 1));
        std::memcpy(hT.r0, W1.r0.data(), sizeof(int64_t) * (ntw + 1));
    }

    // spectral tables
    plans.clear();
    total_pos = ntiles = total_samp = total_pairs = fold_blocks = mid_out = 0;
    fold_chunks = false;  // a lattice task sums its tiles in several chunks
    for (int q = 0; q < nsd; ++q) hT.smap[q] = -1;
    spread_bytes = 0.0;
    groups.clear();  // (first task, count) per grid size
    for (int i = 0; i < nts; ++i) {
        const SpecPlan& P = splans[i];
        const SeriesDesc& d0 = sdesc[J.set[0].sd0 + P.prob];
        SpecTask T{};
        T.t0 = d0.t;
        T.v0f = d0.v32;
        T.v0d = d0.v32 ? nullptr : d0.v64;
        T.n0 = d0.n;
        if (J.ccf) {
            const SeriesDesc& d1 = sdesc[J.set[1].sd0 + P.prob];
            T.t1 = d1.t;
            T.v1f = d1.v32;
            T.v1d = d1.v32 ? nullptr : d1.v64;
            T.n1 = d1.n;
        }
        T.t_ref = P.g.t_ref;
        T.L = P.g.L;
        T.N = P.g.N;
        T.M = P.g.M;
        T.s = P.g.s;
        T.W = P.g.W;
        T.h = J.h[P.prob];
        T.kern = J.kern;
        T.ccf = J.ccf ? 1 : 0;
        T.grid = grids[i];
        T.gridb = gridbs[i];
        T.gridc = gridcs[i];
        T.bunw = bunw[i];
        T.with_b = spec_b ? 1 : 0;
        T.bspec = bspec[i];
        if (spec_w) {
            T.w0 = d0.w64;
            T.w1 = J.ccf ? sdesc[J.set[1].sd0 + P.prob].w64 : nullptr;
        }
        T.tile0 = ntiles;
        T.ntiles = P.g.N / 4096;
        T.tile_rng = d_rng ? d_rng + kTileRec * ntiles : nullptr;
        ntiles += T.ntiles;
        total_samp += T.n0 + T.n1;
        hT.smap[J.set[0].sd0 + P.prob] = 2 * i;
        if (J.ccf) hT.smap[J.set[1].sd0 + P.prob] = 2 * i + 1;
        T.lags = dT.ev;
        T.K_eval = Keval;
        T.P = P.g.P;
        T.ybuf = ybufs[i];
        T.fpart = fparts[i];
        T.nmc = T.P > 0 ? (int32_t)ceil_div(T.N / 4096, kFoldTiles) : 0;
        fold_chunks |= T.nmc > 1;
        if (T.P > 0) {
            int lg = 0;
            while ((T.N >> lg) > T.P) ++lg;  // N / P = 2^lg
            T.lgP2 = 12 - lg;
        }
        T.numer = numer[i];
        T.scale_part = spart[i];
        T.pos0 = total_pos;
        total_pos += P.g.N;
        hT.st[i] = T;
        hT.tile0[i] = T.tile0;
        hT.pos0[i] = T.pos0;
        hT.pair0[i] = total_pairs;
        total_pairs += mid_pairs(T.N);
        hT.sk0[i] = (int64_t)i * Keval;
        hT.fe0[i] = fold_blocks;
        if (T.P > 0) fold_blocks += ceil_div(Keval, kFoldLags) * T.nmc;
        mid_out += T.P > 0 ? T.P : T.N;
        if (i == 0 || splans[i].g.N != splans[i - 1].g.N)
            groups.push_back({i, 1});
        else
            groups.back().second++;
        // tasks are sorted by grid size: the plan and radix record of the
        // previous task serve while the size repeats
        if (i == 0 || T.N != splans[i - 1].g.N) {
            auto it = plans.find(T.N);
            if (it == plans.end()) {
                FftPlan fp;
                NCF_TRY(fft_plan(T.N, fp64, &fp, J.st, J.tune.fft));
                it = plans.emplace(T.N, fp).first;
            }
            const FftPlan& fp = it->second;
            int lgN = 0;
            while ((1LL << lgN) < T.N) ++lgN;
            hT.rinfo[6 * i + 0] = fp.npass;
            for (int q = 0; q < 4; ++q) {
                int lg = 0;
                if (q < fp.npass)
                    while ((1 << lg) < fp.radix[q]) ++lg;
                hT.rinfo[6 * i + 1 + q] = lg;
            }
            hT.rinfo[6 * i + 5] = lgN;
        } else {
            std::memcpy(hT.rinfo + 6 * i, hT.rinfo + 6 * (i - 1), 6 * sizeof(int32_t));
        }
        spread_bytes += (double)(T.n0 + T.n1) * (spec_w ? 20.0 : 12.0) +
                        (double)T.N * csz * nfwd;
    }
    // forward table: per size group, its grids, then its second grids (CCF
    // pair-count channels, or the ACF unit channels of a weighted call), then
    // its third grids (CCF unit channels of a weighted call)
    fwd_groups.clear();
    inv_groups.clear();
    {
        int o = 0;
        for (auto& gq : groups) {
            fwd_groups.push_back({o, gq.second * nfwd});
            for (int i = gq.first; i < gq.first + gq.second; ++i) hT.gfwd[o++] = grids[i];
            if (two_grids)
                for (int i = gq.first; i < gq.first + gq.second; ++i) hT.gfwd[o++] = gridbs[i];
            if (three_grids)
                for (int i = gq.first; i < gq.first + gq.second; ++i) hT.gfwd[o++] = gridcs[i];
        }
        // inverse table: per size group, its grids then (weighted with b) the
        // b spectra in gridb
        // (grids read off a lag lattice have no inverse transform)
        int oi = 0;
        for (auto& gq : groups) {
            const int o0 = oi;
            for (int i = gq.first; i < gq.first + gq.second; ++i)
                if (splans[i].g.P == 0) hT.ginv[oi++] = grids[i];
            if (spec_unw)
                for (int i = gq.first; i < gq.first + gq.second; ++i)
                    if (splans[i].g.P == 0) hT.ginv[oi++] = gridbs[i];
            inv_groups.push_back({o0, oi - o0});
        }
    }
    if (nts > 0) {
        hT.tile0[nts] = ntiles;
        hT.pos0[nts] = total_pos;
        hT.pair0[nts] = total_pairs;
        hT.sk0[nts] = (int64_t)nts * Keval;
        hT.fe0[nts] = fold_blocks;
        for (int64_t k = 0; k < K; ++k) hT.ev[k] = J.lags[k];
        if (!J.ccf) hT.ev[K] = 0.0;
    }
    if (flag_pass)
        for (int r = 0; r < Krow; ++r) hT.rowk[r] = rows[r].second;
    // lags whose spectral pair count is below beta times the reference
    // (b(0) for the ACF, sqrt(B_xx(0) B_yy(0)) for the CCF) are summed
    // directly: their spectral value is dominated by rounding noise
    spec_of.assign(J.nprob, -1);
    for (int i = 0; i < nts; ++i) spec_of[splans[i].prob] = i;
    flagged.assign(J.nprob, std::vector<int>());  // requested lag indices
    W2 = WinLaunch{};
    if (merge3) fill3(0, false);
    NCF_TRY_HIP(hipMemcpyAsync(stg2->d, stg2->h, t2.off, hipMemcpyHostToDevice, J.st));
    return NCF_OK;
}

// phase-3 tables (laid out in dU / hU): the fallback window tasks of W2
// (ntw2 of them), the normalization tasks, statuses and the I/O block
void CallRun::fill3(int ntw2, bool any_fb) {
    std::vector<int> fb_task(J.nprob, -1);
    {
        for (int i = 0; i < ntw2; ++i) {
            if (dl2_first[i])
                std::memcpy(hU.dl + dl2_off[i], W2.plans[i].dl->data(),
                            sizeof(double) * W2.plans[i].dl->size());
            W2.wt[i].delta = dU.dl + dl2_off[i];
            fb_task[W2.plans[i].prob] = i;
        }
        if (ntw2) {
            std::memcpy(hU.wt, W2.wt.data(), sizeof(WinTask) * ntw2);
            std::memcpy(hU.item0, W2.item0.data(), sizeof(int64_t) * (ntw2 + 1));
            std::memcpy(hU.wk0, W2.wk0.data(), sizeof(int64_t) * (ntw2 + 1));
            std::memcpy(hU.r0, W2.r0.data(), sizeof(int64_t) * (ntw2 + 1));
        }
        if (any_fb) {
            for (int64_t i = 0; i < (int64_t)ntw2 * K; ++i) hU.fbrow[i] = -1;
            // flagged lags are in sorted-row order; their fallback row is their rank
            for (int i = 0; i < ntw2; ++i) {
                const int64_t p = W2.plans[i].prob;
                for (size_t q = 0; q < flagged[p].size(); ++q)
                    hU.fbrow[(int64_t)i * K + flagged[p][q]] = (int32_t)q;
            }
        }
    }
    // normalization tables
    std::memcpy(hU.perm, perm.data(), sizeof(int32_t) * K);
    {
        std::vector<int> main_t(J.nprob, -1), selfx(J.nprob, -1), selfy(J.nprob, -1);
        for (int i = 0; i < ntw; ++i) {
            const WinPlan& P = W1.plans[i];
            (P.role == 0 ? main_t : P.role == 1 ? selfx : selfy)[P.prob] = i;
        }
        for (int64_t p = 0; p < J.nprob; ++p) {
            const bool sp = spectral && !direct_p[p];
            NormTask T{};
            T.ccf = J.ccf ? 1 : 0;
            T.K = (int32_t)K;
            T.perm = dU.perm;
            T.row0 = row0;
            T.spectral = sp ? 1 : 0;
            T.spec_b = (spec_b && sp) ? 1 : 0;
            // mixed-precision Gaussian: the lag-0 scale decides whether the
            // problem is evaluated again in FP64 (one-shot calls) or, in a
            // plan execution, reported as unsupported
            const bool promotable = !fp64 && !rect;
            const bool fixed_launches = J.rec != nullptr || J.no_alloc;
            T.guard = (promotable && fixed_launches) ? 1 : 0;
            T.rmin = (promotable && !fixed_launches) ? dU.rmin + p : nullptr;
            T.weighted = weighted ? 1 : 0;
            T.is_rect = rect ? 1 : 0;
            T.beta = beta;
            T.out_off = p * K;
            T.index = p;
            T.st0 = d_stats + J.set[0].sd0 + p;
            T.st1 = J.ccf ? d_stats + J.set[1].sd0 + p : nullptr;
            hU.status[p] = pstat[p];
            if (pstat[p] == NCF_OK) {
                if (main_t[p] >= 0) T.wsums = W1.wt[main_t[p]].sums;
                if (J.ccf && selfx[p] >= 0) {
                    T.self_x = W1.wt[selfx[p]].sums;
                    T.self_y = W1.wt[selfy[p]].sums;
                }
                if (sp) {
                    const int i = spec_of[p];
                    T.numer = numer[i];
                    T.bspec = bspec[i];
                    T.bunw = bunw[i];
                    T.scale_part = spart[i];
                    T.nscale_part = splans[i].g.N / 4096;
                }
                if (fb_task[p] >= 0) {
                    T.fb_row = dU.fbrow + (int64_t)fb_task[p] * K;
                    T.fb_sums = W2.wt[fb_task[p]].sums;
                }
            } else {
                T.skip = 1;  // outputs: c = NaN, b = 0, count = 0
                T.skip_status = pstat[p];
            }
            hU.nt[p] = T;
        }
    }
    // caller arrays of the normalization (one-shot calls)
    hU.io->x[0] = J.set[0].x;
    hU.io->x[1] = J.ccf ? J.set[1].x : nullptr;
    hU.io->c = d_c;
    hU.io->b = d_b;
    hU.io->count = d_cnt;
    hU.io->status = dU.status;
}

// A7: the main window launch and its reduction.
int CallRun::record_window() {
    // ------------------------------------------------ A7 window scan
    // work-queue dispatch of the window scans (scheduling option; also the
    // default for Gaussian launches of many items, whose costs vary with the
    // density of each series: 101.3 -> 95.7 ms on 10,000 weighted curves)
    qbase = nullptr;
    const bool auto_queue = !rect && !J.no_alloc && W1.nitems >= kQueueAutoItems;
    if ((J.opt.flags & NCF_WINDOW_QUEUE) || J.tune.queue || auto_queue)
        NCF_TRY(ensure_queue(R, &qbase));
    // the launch lambdas capture copies only: recorded launches (plans) are
    // replayed after this object is gone
    {
        const WinTask* wt = dT.wt;
        const int64_t *it0 = dT.item0, *wk0 = dT.wk0, *r0 = dT.r0;
        const int64_t nitems = W1.nitems, nrows = W1.total_rows, nred1 = W1.nred1;
        const int cap = W1.cap, jmax = W1.jmax, nt = ntw;
        const double work = W1.work;
        const uint32_t wf = wflags;
        unsigned long long* q = qbase;
        if (nt > 0) {
            NCF_TRY(check_win(W1, wf));
            NCF_TRY(emit(J, [=](hipStream_t s) {
                return launch_window(wt, it0, nt, nitems, wf, cap, jmax, q, s, work);
            }));
            NCF_TRY(emit(J, [=](hipStream_t s) {
                return launch_window_reduce(wt, nt, nrows, wk0, r0, nred1, wf, s);
            }));
        }
    }
    return NCF_OK;
}

// A2-A6: tile ranges, spreading, forward passes, the fused middle (or the
// product), inverse passes, and the evaluation at the lags.
int CallRun::record_spectral() {
    // ------------------------------------------------ A2-A6 spectral route
    if (nts > 0) {
        const SpecTask* stk = dT.st;
        const int64_t *tile0 = dT.tile0, *pos0 = dT.pos0, *sk0 = dT.sk0;
        const int64_t* rinfo = (const int64_t*)dT.rinfo;
        const double pbytes = (nfwd + 1.0 + (spec_unw ? 1.0 : 0.0)) * total_pos * csz;
        const int64_t nkeval = (int64_t)nts * Keval;
        const bool ccf = J.ccf;
        const int32_t* smap = dT.smap;
        const int64_t* rec_all = d_rng;
        const Chunk* dch = d_ch;
        const double tb_bytes = 8.0 * (double)total_samp;
        // the launch lambdas capture copies only (see record_window)
        const int nc = nch, nt = nts;
        const int64_t ntl = ntiles, tpos = total_pos;
        const bool sb = spec_b, sw = spec_w, su = spec_unw, f64 = fp64;
        const double sbytes = spread_bytes;
        if (bounds_pass)
            NCF_TRY(emit(J, [=](hipStream_t s) {
                return launch_tile_bounds(stk, dch, nc, smap, s, tb_bytes);
            }));
        NCF_TRY(emit(J, [=](hipStream_t s) {
            return launch_spread(stk, tile0, nt, ntl, rec_all, 4096, ccf, sb, sw, su, f64, s,
                                 sbytes);
        }));
        // the forward last pass, the product and the inverse first pass run
        // fused over tile pairs where the mode fits the LDS of one workgroup
        const bool fuse = !J.tune.no_mid && mid_supported(J.ccf, spec_b, spec_unw, fp64);
        for (size_t q = 0; q < groups.size(); ++q) {
            const FftPlan fp = plans[splans[groups[q].first].g.N];
            void* const* gp = dT.gfwd + fwd_groups[q].first;
            const int cnt = fwd_groups[q].second;
            NCF_TRY(emit(J, [=](hipStream_t s) {
                return fft_exec(fp, gp, cnt, +1, f64, s, fuse);
            }));
        }
        if (fuse) {
            const int64_t* pair0 = dT.pair0;
            const int64_t npairs = total_pairs;
            const void* wsmall = plans.begin()->second.small;
            // reads every grid it transforms, writes the product grids (or
            // the folded spectra of the grids on a lag lattice)
            const double mbytes = ((double)nfwd * total_pos + (double)mid_out) * csz;
            NCF_TRY(emit(J, [=](hipStream_t s) {
                return launch_mid(stk, pair0, nt, npairs, rinfo, wsmall, ccf, sb, f64, s,
                                  mbytes);
            }));
        } else {
            NCF_TRY(emit(J, [=](hipStream_t s) {
                return launch_product(stk, pos0, nt, tpos, rinfo, ccf, sb, su, f64, s, pbytes);
            }));
        }
        for (size_t q = 0; q < groups.size(); ++q) {
            const FftPlan fp = plans[splans[groups[q].first].g.N];
            void* const* gp = dT.ginv + inv_groups[q].first;
            const int cnt = inv_groups[q].second;
            if (cnt == 0) continue;  // every grid of the size is on a lag lattice
            NCF_TRY(emit(J, [=](hipStream_t s) {
                return fft_exec(fp, gp, cnt, -1, f64, s, fuse);
            }));
        }
        if (J.info_fold_grids < nts)
            NCF_TRY(emit(J, [=](hipStream_t s) {
                return launch_interp(stk, nt, sk0, nkeval, f64, s);
            }));
        if (fold_blocks > 0) {
            const int64_t* fe0 = dT.fe0;
            const int64_t nfb = fold_blocks;
            const bool fch = fold_chunks;
            NCF_TRY(emit(J, [=](hipStream_t s) {
                return launch_fold_eval(stk, nt, fe0, nfb, sk0, nkeval, fch, f64, s);
            }));
        }
    }
    return NCF_OK;
}

// Fallback flags of the spectral pair counts.
int CallRun::record_flags() {
    // ------------------------------------------------ direct fallback (spectral b)
    h_fstat = nullptr;
    h_rmin = nullptr;
    if (flag_pass) {
        // flags computed on the device from the spectral b values (contiguous
        // over the problems); only the bit masks come back
        // a plan's fallback lags must not depend on the placeholder values
        NCF_TRY(launch_fallback_flags(dT.st, bspec[0], nts, Keval, (int)K, J.ccf, !J.rec,
                                      dT.rowk, Krow, beta, dT.mask, J.st));
        if (!combine)
            NCF_TRY_HIP(hipMemcpyAsync(hT.mask, dT.mask, sizeof(uint64_t) * (size_t)nts * fwords,
                                       hipMemcpyDeviceToHost, J.st));
    }
    return NCF_OK;
}

// Flagged lags of each spectral problem -> fallback window tasks in W2.
void CallRun::read_flags() {
    for (int i = 0; i < nts; ++i) {
        const int64_t p = splans[i].prob;
        const uint64_t* mw = hT.mask + (size_t)i * fwords;
        std::vector<double> dl;
        for (int w = 0; w < fwords; ++w)
            for (uint64_t m = mw[w]; m; m &= m - 1) {
                const int r = w * 64 + __builtin_ctzll(m);
                flagged[p].push_back(rows[r].second);
                dl.push_back(delta[r]);
            }
        if (!dl.empty())
            W2.plans.push_back(
                {0, J.ccf ? 1 : 0, p, 3, std::make_shared<const std::vector<double>>(std::move(dl))});
    }
}

// phase-3 launches on the tables in dU: the fallback window scans, the
// normalization, and the copies of the statuses (with the flag masks in
// front when with_masks) and of host-memory outputs
int CallRun::launch3(int ntw2, bool with_masks) {
    const uint32_t wflags2 = (fp64 ? (uint32_t)WIN_EXP64 : 0u) | (uint32_t)WIN_NUMER |
                             (weighted ? (uint32_t)WIN_WEIGHTED : 0u);
    if (ntw2 > 0) {
        const WinTask* wt = dU.wt;
        const int64_t *it0 = dU.item0, *wk0 = dU.wk0, *r0 = dU.r0;
        const int64_t nitems = W2.nitems, nrows = W2.total_rows, nred1 = W2.nred1;
        const int cap = W2.cap, jmax = W2.jmax;
        const double work = W2.work;
        unsigned long long* q = qbase ? qbase + 2 : nullptr;
        NCF_TRY(check_win(W2, wflags2));
        NCF_TRY(emit(J, [=](hipStream_t s) {
            return launch_window(wt, it0, ntw2, nitems, wflags2, cap, jmax, q, s, work);
        }));
        NCF_TRY(emit(J, [=](hipStream_t s) {
            return launch_window_reduce(wt, ntw2, nrows, wk0, r0, nred1, wflags2, s);
        }));
    }

    // ------------------------------------------------ A8 normalization, outputs
    {
        const NormTask* nt = dU.nt;
        const int np = (int)J.nprob;
        const IoBlock* io = J.io_fixed ? J.io_fixed : dU.io;
        NCF_TRY(emit(J, [=](hipStream_t s) { return launch_normalize(nt, np, io, s); }));
    }
    h_fstat = hU.status;  // pinned
    // written by promotable tasks only
    h_rmin = (J.rec || J.no_alloc || fp64 || rect) ? nullptr : hU.rmin;
    if (with_masks) {
        const size_t bytes =
            (size_t)((const char*)(dU.rmin + J.nprob) - (const char*)dT.mask);
        NCF_TRY_HIP(hipMemcpyAsync(hT.mask, dT.mask, bytes, hipMemcpyDeviceToHost, J.st));
    } else if (J.io_fixed) {
        NCF_TRY_HIP(hipMemcpyAsync(h_fstat, J.io_status, sizeof(int32_t) * J.nprob,
                                   hipMemcpyDeviceToHost, J.st));
    } else {
        // statuses and the lag-0 scales behind them
        const size_t bytes = (size_t)((const char*)(dU.rmin + J.nprob) -
                                      (const char*)dU.status);
        NCF_TRY_HIP(hipMemcpyAsync(h_fstat, dU.status, bytes, hipMemcpyDeviceToHost, J.st));
    }
    if (!J.dev_ptrs && K > 0) {
        NCF_TRY_HIP(hipMemcpyAsync(J.c, d_c, sizeof(double) * J.nprob * K, hipMemcpyDeviceToHost,
                                   J.st));
        NCF_TRY_HIP(hipMemcpyAsync(J.b, d_b, sizeof(double) * J.nprob * K, hipMemcpyDeviceToHost,
                                   J.st));
        if (J.count)
            NCF_TRY_HIP(hipMemcpyAsync(J.count, d_cnt, sizeof(int64_t) * J.nprob * K,
                                       hipMemcpyDeviceToHost, J.st));
    }
    return NCF_OK;
}

// Phase 3 with its own tables and upload (the fallback tasks of W2).
int CallRun::separate3() {
    const int ntw2 = (int)W2.plans.size();
    // fallback workspace and the output tables
    auto layout3 = [&](Arena& ar) {
        for (int i = 0; i < ntw2; ++i) {
            WinTask& T = W2.wt[i];
            T.part = ar.take<double>((size_t)T.n_jg * T.K * 4);
            T.part2 = ar.take<double>((size_t)ceil_div(T.n_jg, kWinJc) * T.K * 4);
            T.sums = ar.take<double>((size_t)T.K * 4);
        }
    };
    Arena a3;
    layout3(a3);
    if (ntw2 > 0) {
        void* ws3 = nullptr;
        NCF_TRY(ensure_ws(R, 2, a3.off + 256, &ws3));
        a3 = Arena{(char*)ws3, 0};
        layout3(a3);
    }
    const size_t ndl2 = dl_layout(W2.plans, &dl2_off, &dl2_first);
    const bool any_fb = ntw2 > 0;
    Tables t3;
    take3(t3, ntw2, ndl2, any_fb);
    Staging* stg3 = nullptr;
    NCF_TRY(ensure_stage(R, 2, t3.off, &stg3));
    t3 = Tables{stg3->h, stg3->d, 0};
    take3(t3, ntw2, ndl2, any_fb);
    fill3(ntw2, any_fb);
    NCF_TRY_HIP(hipMemcpyAsync(stg3->d, stg3->h, t3.off, hipMemcpyHostToDevice, J.st));
    return launch3(ntw2, false);
}

// Wait for the call, re-evaluate problems of small lag-0 scale in FP64,
// report the statuses.
int CallRun::done() {
    NCF_TRY_HIP(hipStreamSynchronize(J.st));
    if (g_prof_on) {
        std::lock_guard<std::mutex> lock(g_prof_mu);
        prof_flush_locked();
    }
    if (h_rmin && !J.plan_build) {
        // problems whose lag-0 scale is small in mixed precision: again in FP64
        std::vector<int64_t> again;
        for (int64_t p = 0; p < J.nprob; ++p)
            if ((h_fstat[p] == NCF_OK || h_fstat[p] == NCF_E_DEGENERATE) &&
                h_rmin[p] < kPromoteScale)
                again.push_back(p);
        if (!again.empty()) NCF_TRY(promote_fp64(J, again, h_fstat, stats));
    }
    mark("wait_end");
    const int rc = finish_status(J, pstat, h_fstat);
    if (log > 0) log_call(rc);
    return rc;
}

// One NCF_LOG line for a finished call.
void CallRun::log_call(int rc) const {
    // a plan build reports the statuses of the host checks (its device pass
    // ran on placeholder values)
    int64_t ndirect = 0, nbad = 0;
    for (int64_t p = 0; p < J.nprob; ++p) {
        ndirect += direct_p.empty() ? 0 : direct_p[p];
        nbad += J.plan_build ? pstat[p] != NCF_OK : (h_fstat && h_fstat[p] != NCF_OK);
    }
    const double ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start)
            .count();
    std::fprintf(stderr,
                 "ncf: %s%s n=%lld K=%lld %s %s%s route=%s direct_problems=%lld grids=%d "
                 "cells=%lld lattice_grids=%d window_items=%lld window_launches=%d "
                 "fallback_rows=%lld failed=%lld rc=%d host_ms=%.3f%s%s\n",
                 J.plan_build ? "plan-build " : "", J.ccf ? "ccf" : "acf", (long long)J.nprob,
                 (long long)J.K, rect ? "rectangle" : "gaussian", fp64 ? "fp64" : "mixed",
                 weighted ? " weighted" : "", spectral ? "spectral" : "direct",
                 (long long)ndirect, J.info_grids, (long long)J.info_grid_cells,
                 J.info_fold_grids, (long long)J.info_window_items, J.info_window_launches,
                 (long long)W2.total_rows, (long long)nbad, rc, ms, steps.empty() ? "" : " steps:",
                 steps.c_str());
}

int CallRun::run() {
    log = log_level();
    init_flags();
    NCF_TRY(moments());
    mark("moments");
    if (J.regular) return run_regular(J, sdesc, stats, pstat, d_stats);
    NCF_TRY(plan_route());
    mark("route");
    plan_windows();
    mark("windows");
    NCF_TRY(plan_spectral());
    mark("spectral");
    NCF_TRY(alloc_phase2());
    mark("alloc");
    NCF_TRY(tables_phase2());
    mark("tables");
    NCF_TRY(record_window());
    NCF_TRY(record_spectral());
    NCF_TRY(record_flags());
    mark("launch");
    if (!flag_pass) {  // tables uploaded with phase 2
        NCF_TRY(launch3(0, false));
        return done();
    }
    if (speculate) {
        NCF_TRY(launch3(0, combine));
        NCF_TRY_HIP(hipStreamSynchronize(J.st));
        mark("wait_flags");
        read_flags();
        if (W2.plans.empty()) return done();
    } else {
        NCF_TRY_HIP(hipStreamSynchronize(J.st));
        mark("wait_flags");
        read_flags();
    }
    if (!W2.plans.empty()) plan_window(W2);
    J.info_window_items += W2.nitems;
    J.info_window_launches += W2.plans.empty() ? 0 : 1;
    mark("fallback_plan");
    NCF_TRY(separate3());
    mark("phase3");
    return done();
}

int run_job(Job& J, const double* const* tin, const double* const* xin,
            const double* const* ein) {
    CallRun run(J, tin, xin, ein);
    return run.run();
}

// ---------------------------------------------------------- entry helpers

int common_checks(const ncf_options_t* opt, ncf_options_t* o, int kern) {
    ncf_options_init(o);
    if (opt) {
        if (opt->struct_size != sizeof(ncf_options_t)) {
            set_error("ncf_options_t.struct_size mismatch");
            return NCF_E_INVALID_ARG;
        }
        *o = *opt;
    }
    if (kern != NCF_GAUSSIAN && kern != NCF_RECTANGLE) {
        set_error("unknown kernel %d", kern);
        return NCF_E_INVALID_ARG;
    }
    if (o->precision != NCF_MIXED && o->precision != NCF_FP64) {
        set_error("unknown precision %d", o->precision);
        return NCF_E_INVALID_ARG;
    }
    if (o->method != NCF_AUTO && o->method != NCF_SPECTRAL && o->method != NCF_DIRECT) {
        set_error("unknown method %d", o->method);
        return NCF_E_INVALID_ARG;
    }
    if (o->grid_size > 0 && (o->grid_size < 4096 || (o->grid_size & (o->grid_size - 1)))) {
        set_error("grid_size must be a power of two >= 4096");
        return NCF_E_INVALID_ARG;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        set_error("no HIP device available");
        return NCF_E_DEVICE;
    }
    return NCF_OK;
}

int load_lags(Job& J, int64_t K, const double* lags) {
    if (K < 0 || (K > 0 && !lags)) {
        set_error("invalid lag array");
        return NCF_E_INVALID_ARG;
    }
    J.K = K;
    J.lags.resize(K);
    if (K > 0) {
        if (J.dev_ptrs) {
            // copied with the phase-1 statistics (one synchronization)
            J.lags_dev = lags;
            return NCF_OK;
        }
        std::memcpy(J.lags.data(), lags, sizeof(double) * K);
    }
    return check_lags(J);
}

int check_offs(const int64_t* offs, int64_t n, int64_t* total) {
    if (!offs || offs[0] != 0) {
        set_error("offset array must start at 0");
        return NCF_E_INVALID_ARG;
    }
    for (int64_t i = 0; i < n; ++i)
        if (offs[i + 1] < offs[i] + 2) {
            set_error("series %lld has fewer than 2 samples", (long long)i);
            return NCF_E_INVALID_ARG;
        }
    *total = offs[n];
    return NCF_OK;
}

}  // namespace

}  // namespace ncf

using namespace ncf;

extern "C" {

void ncf_options_init(ncf_options_t* opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof *opt);
    opt->struct_size = sizeof(ncf_options_t);
    opt->precision = NCF_MIXED;
    opt->method = NCF_AUTO;
}

const char* ncf_last_error(void) { return g_err.c_str(); }

int ncf_version(void) { return 100; }

void ncf_release_workspace(void) {
    std::lock_guard<std::mutex> lock(g_ws_mu);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    (void)hipDeviceSynchronize();
    auto it = g_res.find(dev);
    if (it != g_res.end()) free_resources(it->second);
}

}  // extern "C"

namespace ncf {
namespace {

// Common set-up of an ACF or CCF job (arguments already checked).
int setup_job(Job& J, bool ccf, int64_t nprob, const int64_t* off0, const int64_t* off1,
              int64_t tot0, int64_t tot1, int kern, const double* h, int64_t K,
              const double* lags) {
    J.ccf = ccf;
    J.nprob = nprob;
    J.kern = kern;
    J.h.assign(h, h + nprob);
    J.dev_ptrs = (J.opt.flags & NCF_DEVICE_POINTERS) != 0;
    J.st = (hipStream_t)J.opt.stream;
    NCF_TRY(load_lags(J, K, lags));
    J.set[0].ntot = tot0;
    J.set[0].nser = (int)nprob;
    J.set[0].offs.assign(off0, off0 + nprob + 1);
    if (ccf) {
        J.set[1].ntot = tot1;
        J.set[1].nser = (int)nprob;
        J.set[1].offs.assign(off1, off1 + nprob + 1);
    }
    return NCF_OK;
}

Resources* device_resources() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return &g_res[dev];
}

}  // namespace
}  // namespace ncf

namespace ncf {
namespace {

// ACF and CCF batches; dt (per problem) selects the regular-lattice route.
int acf_batch_impl(int64_t nser, const int64_t* offs, const double* t, const double* x,
                   const double* err, const double* dt, bool regular, int64_t K,
                   const double* lags, int kern, const double* h, double* c, double* b,
                   int64_t* count, int* status, const ncf_options_t* opt) {
    clear_error();
    Job J;
    NCF_TRY(common_checks(opt, &J.opt, kern));
    if (nser <= 0 || !t || !x || !h || (regular && !dt) || (K > 0 && (!c || !b))) {
        set_error("null argument or nser <= 0");
        return NCF_E_INVALID_ARG;
    }
    int64_t total = 0;
    NCF_TRY(check_offs(offs, nser, &total));
    std::lock_guard<std::mutex> lock(g_ws_mu);
    J.c = c;
    J.b = b;
    J.count = count;
    J.status = status;
    J.regular = regular;
    if (regular) J.dt.assign(dt, dt + nser);
    NCF_TRY(setup_job(J, false, nser, offs, nullptr, total, 0, kern, h, K, lags));
    J.res = device_resources();
    if (!J.res) {
        set_error("no current HIP device");
        return NCF_E_DEVICE;
    }
    const double* tin[2] = {t, nullptr};
    const double* xin[2] = {x, nullptr};
    const double* ein[2] = {err, nullptr};
    return run_job(J, tin, xin, ein);
}

int ccf_batch_impl(int64_t npair, const int64_t* offx, const double* tx, const double* x,
                   const double* ex, const int64_t* offy, const double* ty, const double* y,
                   const double* ey, const double* dt, bool regular, int64_t K,
                   const double* lags, int kern, const double* h, double* c, double* b,
                   int64_t* count, int* status, const ncf_options_t* opt) {
    clear_error();
    Job J;
    NCF_TRY(common_checks(opt, &J.opt, kern));
    if (npair <= 0 || !tx || !x || !ty || !y || !h || (regular && !dt) ||
        (K > 0 && (!c || !b))) {
        set_error("null argument or npair <= 0");
        return NCF_E_INVALID_ARG;
    }
    int64_t totx = 0, toty = 0;
    NCF_TRY(check_offs(offx, npair, &totx));
    NCF_TRY(check_offs(offy, npair, &toty));
    std::lock_guard<std::mutex> lock(g_ws_mu);
    J.c = c;
    J.b = b;
    J.count = count;
    J.status = status;
    J.regular = regular;
    if (regular) J.dt.assign(dt, dt + npair);
    NCF_TRY(setup_job(J, true, npair, offx, offy, totx, toty, kern, h, K, lags));
    J.res = device_resources();
    if (!J.res) {
        set_error("no current HIP device");
        return NCF_E_DEVICE;
    }
    const double* tin[2] = {tx, ty};
    const double* xin[2] = {x, y};
    const double* ein[2] = {ex, ey};
    return run_job(J, tin, xin, ein);
}

}  // namespace
}  // namespace ncf

extern "C" {

int ncf_acf_batch(int64_t nser, const int64_t* offs, const double* t, const double* x,
                  const double* err, int64_t K, const double* lags, int kern, const double* h,
                  double* c, double* b, int64_t* count, int* status, const ncf_options_t* opt) {
    return acf_batch_impl(nser, offs, t, x, err, nullptr, false, K, lags, kern, h, c, b, count,
                          status, opt);
}

int ncf_ccf_batch(int64_t npair, const int64_t* offx, const double* tx, const double* x,
                  const double* ex, const int64_t* offy, const double* ty, const double* y,
                  const double* ey, int64_t K, const double* lags, int kern, const double* h,
                  double* c, double* b, int64_t* count, int* status, const ncf_options_t* opt) {
    return ccf_batch_impl(npair, offx, tx, x, ex, offy, ty, y, ey, nullptr, false, K, lags, kern,
                          h, c, b, count, status, opt);
}

int ncf_acf_regular_batch(int64_t nser, const int64_t* offs, const double* t, const double* x,
                          const double* err, const double* dt, int64_t K, const double* lags,
                          int kern, const double* h, double* c, double* b, int64_t* count,
                          int* status, const ncf_options_t* opt) {
    return acf_batch_impl(nser, offs, t, x, err, dt, true, K, lags, kern, h, c, b, count, status,
                          opt);
}

int ncf_ccf_regular_batch(int64_t npair, const int64_t* offx, const double* tx, const double* x,
                          const double* ex, const int64_t* offy, const double* ty,
                          const double* y, const double* ey, const double* dt, int64_t K,
                          const double* lags, int kern, const double* h, double* c, double* b,
                          int64_t* count, int* status, const ncf_options_t* opt) {
    return ccf_batch_impl(npair, offx, tx, x, ex, offy, ty, y, ey, dt, true, K, lags, kern, h, c,
                          b, count, status, opt);
}

int ncf_acf_regular(int64_t n, const double* t, const double* x, const double* err, double dt,
                    int64_t K, const double* lags, int kern, double h, double* c, double* b,
                    int64_t* count, const ncf_options_t* opt) {
    if (n < 2) {
        set_error("n must be >= 2");
        return NCF_E_INVALID_ARG;
    }
    int64_t offs[2] = {0, n};
    return ncf_acf_regular_batch(1, offs, t, x, err, &dt, K, lags, kern, &h, c, b, count,
                                 nullptr, opt);
}

int ncf_ccf_regular(int64_t nx, const double* tx, const double* x, const double* ex, int64_t ny,
                    const double* ty, const double* y, const double* ey, double dt, int64_t K,
                    const double* lags, int kern, double h, double* c, double* b,
                    int64_t* count, const ncf_options_t* opt) {
    if (nx < 2 || ny < 2) {
        set_error("nx and ny must be >= 2");
        return NCF_E_INVALID_ARG;
    }
    int64_t ox[2] = {0, nx}, oy[2] = {0, ny};
    return ncf_ccf_regular_batch(1, ox, tx, x, ex, oy, ty, y, ey, &dt, K, lags, kern, &h, c, b,
                                 count, nullptr, opt);
}

int ncf_acf(int64_t n, const double* t, const double* x, const double* err, int64_t K,
            const double* lags, int kern, double h, double* c, double* b, int64_t* count,
            const ncf_options_t* opt) {
    if (n < 2) {
        set_error("n must be >= 2");
        return NCF_E_INVALID_ARG;
    }
    int64_t offs[2] = {0, n};
    return ncf_acf_batch(1, offs, t, x, err, K, lags, kern, &h, c, b, count, nullptr, opt);
}

int ncf_ccf(int64_t nx, const double* tx, const double* x, const double* ex, int64_t ny,
            const double* ty, const double* y, const double* ey, int64_t K, const double* lags,
            int kern, double h, double* c, double* b, int64_t* count, const ncf_options_t* opt) {
    if (nx < 2 || ny < 2) {
        set_error("nx and ny must be >= 2");
        return NCF_E_INVALID_ARG;
    }
    int64_t ox[2] = {0, nx}, oy[2] = {0, ny};
    return ncf_ccf_batch(1, ox, tx, x, ex, oy, ty, y, ey, K, lags, kern, &h, c, b, count,
                         nullptr, opt);
}

}  // extern "C"

// ------------------------------------------------ allocation-free entry point

namespace ncf {
namespace {

// Device workspace of ncf_ccf_noalloc: one array per device, held by the
// loaded code object until the process ends. Host code never passes its name
// to a kernel or a copy: it takes the array's device address, per device,
// from hipGetSymbolAddress and carves the call's arenas from that address.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];
// host side of the call's table staging (uploads and readbacks of small
// tables), shared by every device: calls hold the workspace lock
constexpr size_t kScratchHostBytes = (size_t)4 << 20;
alignas(256) char g_scratch_host[kScratchHostBytes];
constexpr int kScratchDevices = 64;
char* g_scratch_dev[kScratchDevices] = {};  // device address of `scratch`, per device

// The device address of this device's `scratch` array (looked up once per
// device, with that device current).
int scratch_of_device(char** out) {
    int dev = 0;
    NCF_TRY_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kScratchDevices) {
        set_error("device %d: the allocation-free entry point supports devices 0..%d", dev,
                  kScratchDevices - 1);
        return NCF_E_UNSUPPORTED;
    }
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        NCF_TRY_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            set_error("no device address for the allocation-free workspace");
            return NCF_E_DEVICE;
        }
        g_scratch_dev[dev] = (char*)p;
    }
    *out = g_scratch_dev[dev];
    return NCF_OK;
}

}  // namespace
}  // namespace ncf

extern "C" {

int ncf_ccf_noalloc(int64_t nx, const double* tx, const double* x, const double* ex,
                    int64_t ny, const double* ty, const double* y, const double* ey, int64_t K,
                    const double* lags, int kern, double h, double* c, double* b,
                    int64_t* count, const ncf_options_t* opt) {
    clear_error();
    Job J;
    NCF_TRY(common_checks(opt, &J.opt, kern));
    if (nx < 2 || ny < 2 || !tx || !x || !ty || !y || (K > 0 && (!c || !b))) {
        set_error("null argument, or nx or ny below 2");
        return NCF_E_INVALID_ARG;
    }
    // the direct window sums, one launch per step, no queue counters
    J.opt.method = NCF_DIRECT;
    J.opt.flags &= NCF_DEVICE_POINTERS;
    std::lock_guard<std::mutex> lock(g_ws_mu);
    Resources R;
    NCF_TRY(scratch_of_device(&R.fixed_dev));
    R.fixed_cap = kScratchBytes;
    R.fixed_host = g_scratch_host;
    R.fixed_host_cap = kScratchHostBytes;
    R.exact = true;
    J.c = c;
    J.b = b;
    J.count = count;
    J.no_alloc = true;
    int64_t ox[2] = {0, nx}, oy[2] = {0, ny};
    NCF_TRY(setup_job(J, true, 1, ox, oy, nx, ny, kern, &h, K, lags));
    J.res = &R;
    const double* tin[2] = {tx, ty};
    const double* xin[2] = {x, y};
    const double* ein[2] = {ex, ey};
    const int rc = run_job(J, tin, xin, ein);
    // a call that stopped early may still have work in flight on the
    // workspace that the next call reuses
    if (rc != NCF_OK) (void)hipStreamSynchronize(J.st);
    return rc;
}

}  // extern "C"

// ------------------------------------------------------------ resampling

namespace ncf {
namespace {

struct ResampleSet {
    int64_t n;
    const double* t;
    const double* x;
    const double* err;
    const double* sigma;
    const double* z;
    const int32_t* mult;
};

// R replicates of an ACF (one set) or CCF (two sets) as one batch over
// shared times; per-lag mean and standard deviation of c over the
// replicates that succeed.
int resample_impl(bool ccf, const ResampleSet* in, int64_t R, int64_t K, const double* lags,
                  int kern, double h, double* c_mean, double* c_sd, double* c_rep, int* status,
                  const ncf_options_t* opt) {
    clear_error();
    ncf_options_t o;
    NCF_TRY(common_checks(opt, &o, kern));
    const int nsets = ccf ? 2 : 1;
    if (R < 1 || K < 0 || (K > 0 && (!lags || !c_mean || !c_sd))) {
        set_error("invalid replicate count, lags or outputs");
        return NCF_E_INVALID_ARG;
    }
    for (int si = 0; si < nsets; ++si) {
        const ResampleSet& S = in[si];
        if (S.n < 2 || !S.t || !S.x) {
            set_error("series %d: fewer than 2 samples or null arrays", si + 1);
            return NCF_E_INVALID_ARG;
        }
        if ((S.z == nullptr) != (S.sigma == nullptr)) {
            set_error("series %d: deviates z and their scale sigma go together", si + 1);
            return NCF_E_INVALID_ARG;
        }
        if ((double)S.n * (double)R > 4.0e9) {
            set_error("series %d: n x R above 4e9 samples", si + 1);
            return NCF_E_UNSUPPORTED;
        }
    }
    const bool dev = (o.flags & NCF_DEVICE_POINTERS) != 0;
    hipStream_t st = (hipStream_t)o.stream;
    std::lock_guard<std::mutex> lock(g_ws_mu);
    Resources* res = device_resources();
    if (!res) {
        set_error("no current HIP device");
        return NCF_E_DEVICE;
    }

    // replicate workspace: device copies of host inputs, replicate values
    // and weights, replicate estimates and (host mode) the statistics
    struct Dev {
        const double *t, *x, *err, *sigma, *z;
        const int32_t* mult;
        double *xr, *wr;
    } D[2] = {};
    double *crep = nullptr, *brep = nullptr, *cm = nullptr, *cs = nullptr;
    const double* dlags = lags;
    auto layout = [&](Arena& ar) {
        for (int si = 0; si < nsets; ++si) {
            const ResampleSet& S = in[si];
            Dev& d = D[si];
            const size_t nr = (size_t)S.n * R;
            if (dev) {
                d.t = S.t;
                d.x = S.x;
                d.err = S.err;
                d.sigma = S.sigma;
                d.z = S.z;
                d.mult = S.mult;
            } else {
                d.t = ar.take<double>(S.n);
                d.x = ar.take<double>(S.n);
                d.err = S.err ? ar.take<double>(S.n) : nullptr;
                d.sigma = S.sigma ? ar.take<double>(S.n) : nullptr;
                d.z = S.z ? ar.take<double>(nr) : nullptr;
                d.mult = S.mult ? ar.take<int32_t>(nr) : nullptr;
            }
            d.xr = ar.take<double>(nr);
            d.wr = (S.mult || S.err) ? ar.take<double>(nr) : nullptr;
        }
        if (!dev) dlags = ar.take<double>(std::max<int64_t>(K, 1));
        crep = (dev && c_rep) ? c_rep : ar.take<double>(std::max<int64_t>(R * K, 1));
        brep = ar.take<double>(std::max<int64_t>(R * K, 1));
        cm = dev ? c_mean : ar.take<double>(std::max<int64_t>(K, 1));
        cs = dev ? c_sd : ar.take<double>(std::max<int64_t>(K, 1));
    };
    Arena a;
    layout(a);
    void* ws = nullptr;
    NCF_TRY(ensure_ws(*res, 3, a.off + 256, &ws));
    a = Arena{(char*)ws, 0};
    layout(a);
    if (!dev) {
        auto up = [&](const void* dst, const void* src, size_t by) -> int {
            if (src && by)
                NCF_TRY_HIP(hipMemcpyAsync((void*)dst, src, by, hipMemcpyHostToDevice, st));
            return NCF_OK;
        };
        for (int si = 0; si < nsets; ++si) {
            const ResampleSet& S = in[si];
            const size_t nr = (size_t)S.n * R;
            NCF_TRY(up(D[si].t, S.t, sizeof(double) * S.n));
            NCF_TRY(up(D[si].x, S.x, sizeof(double) * S.n));
            NCF_TRY(up(D[si].err, S.err, sizeof(double) * S.n));
            NCF_TRY(up(D[si].sigma, S.sigma, sizeof(double) * S.n));
            NCF_TRY(up(D[si].z, S.z, sizeof(double) * nr));
            NCF_TRY(up(D[si].mult, S.mult, sizeof(int32_t) * nr));
        }
        NCF_TRY(up(dlags, lags, sizeof(double) * K));
    }
    for (int si = 0; si < nsets; ++si)
        NCF_TRY(launch_resample_prep(in[si].n, R, D[si].x, D[si].sigma, D[si].z, D[si].err,
                                     D[si].mult, D[si].xr, D[si].wr, st));

    // the replicates as one batch over shared times
    Job J;
    J.opt = o;
    J.opt.flags |= NCF_DEVICE_POINTERS;
    J.res = res;
    std::vector<double> hs((size_t)R, h);
    // statuses are written only when the batch runs to its end; the sentinel
    // marks a call that failed before (invalid lags, a device error)
    constexpr int kNotRun = -1000;
    std::vector<int> rstat((size_t)R, kNotRun);
    std::vector<int64_t> offs[2];
    for (int si = 0; si < nsets; ++si) {
        offs[si].resize((size_t)R + 1);
        for (int64_t r = 0; r <= R; ++r) offs[si][r] = r * in[si].n;
    }
    J.c = crep;
    J.b = brep;
    J.count = nullptr;
    J.status = rstat.data();
    J.no_b = true;
    NCF_TRY(setup_job(J, ccf, R, offs[0].data(), ccf ? offs[1].data() : nullptr, R * in[0].n,
                      ccf ? R * in[1].n : 0, kern, hs.data(), K, dlags));
    const double* tin[2] = {D[0].t, ccf ? D[1].t : nullptr};
    const double* xin[2] = {D[0].xr, ccf ? D[1].xr : nullptr};
    const double* ein[2] = {D[0].wr, ccf ? D[1].wr : nullptr};
    for (int si = 0; si < nsets; ++si) {
        J.set[si].shared_t = true;
        J.set[si].wmode = D[si].wr != nullptr;
    }
    const int rc = run_job(J, tin, xin, ein);
    if (rstat[0] == kNotRun) return rc != NCF_OK ? rc : NCF_E_DEVICE;
    clear_error();
    NCF_TRY(launch_resample_stats(crep, R, K, cm, cs, st));
    if (!dev && K > 0) {
        NCF_TRY_HIP(hipMemcpyAsync(c_mean, cm, sizeof(double) * K, hipMemcpyDeviceToHost, st));
        NCF_TRY_HIP(hipMemcpyAsync(c_sd, cs, sizeof(double) * K, hipMemcpyDeviceToHost, st));
        if (c_rep)
            NCF_TRY_HIP(hipMemcpyAsync(c_rep, crep, sizeof(double) * R * K, hipMemcpyDeviceToHost,
                                       st));
    }
    NCF_TRY_HIP(hipStreamSynchronize(st));
    int first = NCF_OK, ok = 0;
    for (int64_t r = 0; r < R; ++r) {
        if (status) status[r] = rstat[r];
        if (rstat[r] == NCF_OK)
            ++ok;
        else if (first == NCF_OK)
            first = rstat[r];
    }
    if (ok == 0) {
        set_error("no replicate succeeded (first status %d)", first);
        return first;
    }
    return NCF_OK;
}

}  // namespace
}  // namespace ncf

extern "C" {

int ncf_acf_resample(int64_t n, const double* t, const double* x, const double* err,
                     const double* sigma, int64_t R, const double* z, const int32_t* mult,
                     int64_t K, const double* lags, int kern, double h, double* c_mean,
                     double* c_sd, double* c_rep, int* status, const ncf_options_t* opt) {
    ResampleSet S{n, t, x, err, sigma, z, mult};
    return resample_impl(false, &S, R, K, lags, kern, h, c_mean, c_sd, c_rep, status, opt);
}

int ncf_ccf_resample(int64_t nx, const double* tx, const double* x, const double* ex,
                     const double* sx, const double* zx, const int32_t* multx, int64_t ny,
                     const double* ty, const double* y, const double* ey, const double* sy,
                     const double* zy, const int32_t* multy, int64_t R, int64_t K,
                     const double* lags, int kern, double h, double* c_mean, double* c_sd,
                     double* c_rep, int* status, const ncf_options_t* opt) {
    ResampleSet S[2] = {{nx, tx, x, ex, sx, zx, multx}, {ny, ty, y, ey, sy, zy, multy}};
    return resample_impl(true, S, R, K, lags, kern, h, c_mean, c_sd, c_rep, status, opt);
}

}  // extern "C"

// ------------------------------------------------------------------ plans

struct ncf_plan_s {
    int device = 0;
    bool ccf = false, dev_ptrs = false, use_graph = true;
    int64_t nprob = 0, K = 0;
    int64_t ntot[2] = {0, 0};
    hipStream_t st = nullptr;
    ncf::Resources res;
    std::vector<std::function<int(hipStream_t)>> rec;  // the recorded launches
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // plan-owned device memory
    ncf::IoBlock* io = nullptr;
    int32_t* status = nullptr;           // [nprob]
    double* tcopy[2] = {nullptr, nullptr};
    double* ecopy[2] = {nullptr, nullptr};
    double* xbuf[2] = {nullptr, nullptr};  // values (host-pointer plans)
    double* cbuf = nullptr;               // outputs (host-pointer plans, and the build)
    double* bbuf = nullptr;
    int64_t* nbuf = nullptr;
    std::vector<int32_t> hstatus;          // host statuses (host-pointer plans)
    // what was planned, and how (ncf_plan_info)
    ncf::Tune tune;
    int grids = 0, window_launches = 0, fold_grids = 0;
    int64_t grid_cells = 0, window_items = 0;
    int autotuned = 0, candidates = 0;
    int tune_cached = 0;  // autotuned settings read from the autotune cache
    double replay_ms = 0.0;
};

namespace ncf {
namespace {

void plan_free(ncf_plan_s* P) {
    if (!P) return;
    (void)hipDeviceSynchronize();
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    free_resources(P->res);
    void* bufs[] = {P->io,       P->status,   P->tcopy[0], P->tcopy[1], P->ecopy[0],
                    P->ecopy[1], P->xbuf[0], P->xbuf[1], P->cbuf,     P->bbuf,
                    P->nbuf};
    for (void* q : bufs)
        if (q) (void)hipFree(q);
    delete P;
}

template <typename T>
int dev_alloc(T** p, size_t n) {
    if (hipMalloc((void**)p, sizeof(T) * std::max<size_t>(n, 1)) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        set_error("plan allocation of %zu bytes failed", sizeof(T) * n);
        return NCF_E_NOMEM;
    }
    return NCF_OK;
}

// Build a plan: copy times and errors, run the whole path once on
// placeholder values (recording every launch), then capture the launches
// into a graph.
int plan_build(ncf_plan_s* P, Job& J, const double* const* tin, const double* const* ein,
               const Tune& tune, double* dummy) {
    const int nsets = J.ccf ? 2 : 1;
    NCF_TRY_HIP(hipGetDevice(&P->device));
    P->ccf = J.ccf;
    P->dev_ptrs = J.dev_ptrs;
    P->use_graph = (J.opt.flags & NCF_PLAN_NO_GRAPH) == 0;
    P->nprob = J.nprob;
    P->K = J.K;
    P->st = J.st;
    P->res.exact = true;
    const hipMemcpyKind kind = J.dev_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    int64_t nmax = 0;
    for (int si = 0; si < nsets; ++si) {
        const int64_t n = J.set[si].ntot;
        P->ntot[si] = n;
        nmax = std::max(nmax, n);
        NCF_TRY(dev_alloc(&P->tcopy[si], n));
        NCF_TRY_HIP(hipMemcpyAsync(P->tcopy[si], tin[si], sizeof(double) * n, kind, J.st));
        if (ein[si]) {
            NCF_TRY(dev_alloc(&P->ecopy[si], n));
            NCF_TRY_HIP(hipMemcpyAsync(P->ecopy[si], ein[si], sizeof(double) * n, kind, J.st));
        }
        if (!J.dev_ptrs) NCF_TRY(dev_alloc(&P->xbuf[si], n));
    }
    const int64_t nout = std::max<int64_t>(J.nprob * J.K, 1);
    NCF_TRY(dev_alloc(&P->io, 1));
    NCF_TRY(dev_alloc(&P->status, J.nprob));
    NCF_TRY(dev_alloc(&P->cbuf, nout));
    NCF_TRY(dev_alloc(&P->bbuf, nout));
    NCF_TRY(dev_alloc(&P->nbuf, nout));
    P->hstatus.assign(J.nprob, NCF_OK);

    (void)nmax;
    IoBlock io{};
    io.x[0] = dummy;
    io.x[1] = J.ccf ? dummy : nullptr;
    io.c = P->cbuf;
    io.b = P->bbuf;
    io.count = P->nbuf;
    io.status = P->status;
    NCF_TRY(launch_set_io(P->io, io, J.st));

    Job B = J;  // the build run: device pointers throughout
    B.dev_ptrs = true;
    B.c = P->cbuf;
    B.b = P->bbuf;
    B.count = P->nbuf;
    B.status = nullptr;
    B.res = &P->res;
    B.io_fixed = P->io;
    B.io_status = P->status;
    B.rec = &P->rec;
    B.plan_build = true;
    B.tune = tune;
    const double* tdev[2] = {P->tcopy[0], P->tcopy[1]};
    const double* xdev[2] = {dummy, J.ccf ? dummy : nullptr};
    const double* edev[2] = {P->ecopy[0], P->ecopy[1]};
    NCF_TRY(run_job(B, tdev, xdev, edev));
    P->tune = tune;
    P->grids = B.info_grids;
    P->fold_grids = B.info_fold_grids;
    P->grid_cells = B.info_grid_cells;
    P->window_items = B.info_window_items;
    P->window_launches = B.info_window_launches;

    if (P->use_graph) {
        hipStream_t cs = nullptr;
        NCF_TRY_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        int rc = NCF_OK;
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            g_capturing = true;
            for (auto& f : P->rec) {
                rc = f(cs);
                if (rc != NCF_OK) break;
            }
            g_capturing = false;
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(cs, &g);
            if (e == hipSuccess && rc == NCF_OK) {
                P->graph = g;
                e = hipGraphInstantiate(&P->exec, g, nullptr, nullptr, 0);
            } else if (g) {
                (void)hipGraphDestroy(g);
            }
        }
        (void)hipStreamDestroy(cs);
        if (rc != NCF_OK) return rc;
        if (e != hipSuccess) {
            set_error("graph capture of the plan failed: %s", hipGetErrorString(e));
            (void)hipGetLastError();
            return NCF_E_DEVICE;
        }
    }
    return NCF_OK;
}

// Mean time of one execution of a built plan on the placeholder values
// (one warm-up execution, then `reps` timed with events on the plan stream).
int plan_time(ncf_plan_s* P, double* dummy, int reps, double* ms) {
    IoBlock io{};
    io.x[0] = dummy;
    io.x[1] = P->ccf ? dummy : nullptr;
    io.c = P->cbuf;
    io.b = P->bbuf;
    io.count = P->nbuf;
    io.status = P->status;
    NCF_TRY(launch_set_io(P->io, io, P->st));
    auto run = [&]() -> int {
        if (P->exec) {
            NCF_TRY_HIP(hipGraphLaunch(P->exec, P->st));
        } else {
            for (auto& f : P->rec) NCF_TRY(f(P->st));
        }
        return NCF_OK;
    };
    NCF_TRY(run());
    hipEvent_t e0, e1;
    NCF_TRY_HIP(hipEventCreate(&e0));
    NCF_TRY_HIP(hipEventCreate(&e1));
    int rc = NCF_OK;
    if (hipEventRecord(e0, P->st) != hipSuccess) rc = NCF_E_DEVICE;
    for (int r = 0; r < reps && rc == NCF_OK; ++r) rc = run();
    float el = 0.f;
    if (rc == NCF_OK && (hipEventRecord(e1, P->st) != hipSuccess ||
                         hipEventSynchronize(e1) != hipSuccess ||
                         hipEventElapsedTime(&el, e0, e1) != hipSuccess))
        rc = NCF_E_DEVICE;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = el / std::max(reps, 1);
    return rc;
}

// ------------------------------------------------------------ autotune cache
// The autotuner's choice persists in the text file that NCF_AUTOTUNE_CACHE
// names: one JSON record per line, {"key": "...", "sigma": ..., ...}, keyed
// by the device (architecture, compute units) and the call's shape: kind,
// kernel, precision, method, flags, weights, options, and power-of-two
// buckets of the problem count, total samples, lag count and the first
// problem's h. The settings change speed only (results differ at the
// rounding level), so calls of one bucket share them. The last record of a
// key wins; a line that does not parse, or holds a value out of range, is
// skipped. Appends are serialized within the process.
std::mutex g_tune_mu;

std::string tune_key(const Job& J, int device, bool weighted) {
    hipDeviceProp_t prop{};
    char arch[64] = "unknown";
    int cus = 0;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        std::snprintf(arch, sizeof(arch), "%s", prop.gcnArchName);
        cus = prop.multiProcessorCount;
    }
    for (char* c = arch; *c; ++c)
        if (*c == '"' || *c == '\\') *c = '_';
    auto lg2 = [](double v) { return v > 0.0 ? (int)std::floor(std::log2(v)) : -999; };
    const int64_t ntot = J.set[0].ntot + (J.ccf ? J.set[1].ntot : 0);
    const unsigned fl = J.opt.flags & (NCF_SPECTRAL_ALWAYS | NCF_WINDOW_QUEUE | NCF_PLAN_NO_GRAPH |
                                       NCF_DEVICE_POINTERS);
    char buf[320];
    std::snprintf(buf, sizeof(buf),
                  "%s/%dcu %s %s %s prec%d method%d flags%u w%d tol%.3g sigma%.3g grid%lld "
                  "n%d N%d K%d h%d",
                  arch, cus, J.ccf ? "ccf" : "acf", J.regular ? "regular" : "irregular",
                  J.kern == NCF_RECTANGLE ? "rect" : "gauss", (int)J.opt.precision,
                  (int)J.opt.method, fl, weighted ? 1 : 0, J.opt.tol, J.opt.sigma,
                  (long long)J.opt.grid_size, lg2((double)J.nprob), lg2((double)ntot),
                  lg2((double)J.K + 1.0), lg2(J.h.empty() ? 0.0 : J.h[0]));
    return buf;
}

bool tune_cache_find(const char* path, const std::string& key, Tune* out) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    static const char* const names[8] = {"sigma", "fft_split", "fft_tile_log2",
                                         "window_tile_scale", "window_queue", "no_mid",
                                         "eval_interp", "replay_ms"};
    const std::string kq = "\"key\": \"" + key + "\"";
    char line[2048];
    bool found = false;
    while (std::fgets(line, sizeof(line), f)) {
        if (!std::strstr(line, kq.c_str())) continue;
        double v[8];
        bool ok = true;
        for (int i = 0; i < 8 && ok; ++i) {
            char pat[48];
            std::snprintf(pat, sizeof(pat), "\"%s\": ", names[i]);
            const char* q = std::strstr(line, pat);
            char* end = nullptr;
            if (q) v[i] = std::strtod(q + std::strlen(pat), &end);
            ok = q && end != q + std::strlen(pat) && std::isfinite(v[i]);
        }
        if (!ok) continue;
        ok = (v[0] == 0.0 || (v[0] >= 1.25 && v[0] <= 2.0)) && (v[1] >= 0 && v[1] <= 2) &&
             (v[2] == 0 || v[2] == 12 || v[2] == 13) && (v[3] >= -2 && v[3] <= 2) &&
             (v[4] == 0 || v[4] == 1) && (v[5] == 0 || v[5] == 1) && (v[6] == 0 || v[6] == 1);
        if (!ok) continue;
        Tune t;
        t.sigma = v[0];
        t.fft.split = (int)v[1];
        t.fft.lgt_strided = (int)v[2];
        t.jscale = (int)v[3];
        t.queue = v[4] != 0.0;
        t.no_mid = v[5] != 0.0;
        t.eval_interp = v[6] != 0.0;
        *out = t;
        found = true;
    }
    std::fclose(f);
    return found;
}

void tune_cache_store(const char* path, const std::string& key, const Tune& t, double ms) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    FILE* f = std::fopen(path, "a");
    if (!f) {
        if (log_level() > 0) std::fprintf(stderr, "ncf: autotune cache %s: cannot append\n", path);
        return;
    }
    std::fprintf(f,
                 "{\"key\": \"%s\", \"sigma\": %.17g, \"fft_split\": %d, \"fft_tile_log2\": %d, "
                 "\"window_tile_scale\": %d, \"window_queue\": %d, \"no_mid\": %d, "
                 "\"eval_interp\": %d, \"replay_ms\": %.6g}\n",
                 key.c_str(), t.sigma, t.fft.split, t.fft.lgt_strided, t.jscale, t.queue ? 1 : 0,
                 t.no_mid ? 1 : 0, t.eval_interp ? 1 : 0, ms);
    std::fclose(f);
}

// Build a plan; with NCF_PLAN_AUTOTUNE, build and time candidate settings by
// coordinate descent from the defaults (minimum oversampling, FFT radix split
// and strided tile, window tile scale, window dispatch) and keep the fastest.
int plan_create(Job& J, const double* const* tin, const double* const* ein, ncf_plan_t** out) {
    int64_t nmax = J.set[0].ntot;
    if (J.ccf) nmax = std::max(nmax, J.set[1].ntot);
    // placeholder values: finite, unit variance (the plan's pair counts and
    // fallback lags depend on the times only)
    double* dummy = nullptr;
    NCF_TRY(dev_alloc(&dummy, nmax));
    struct Guard {
        double* p;
        ~Guard() {
            (void)hipDeviceSynchronize();
            (void)hipFree(p);
        }
    } guard{dummy};
    NCF_TRY(launch_fill_alternating(dummy, nmax, J.st));

    // autotune cache: a plan whose key is there takes the recorded settings
    const char* cpath =
        (J.opt.flags & NCF_PLAN_AUTOTUNE) ? std::getenv("NCF_AUTOTUNE_CACHE") : nullptr;
    if (cpath && !*cpath) cpath = nullptr;
    std::string ckey;
    if (cpath) {
        int dev = 0;
        NCF_TRY_HIP(hipGetDevice(&dev));
        ckey = tune_key(J, dev, ein[0] != nullptr || (J.ccf && ein[1] != nullptr));
        Tune ct;
        if (tune_cache_find(cpath, ckey, &ct)) {
            ncf_plan_s* P = new ncf_plan_s;
            const int r = plan_build(P, J, tin, ein, ct, dummy);
            if (r == NCF_OK) {
                P->autotuned = 1;
                P->tune_cached = 1;
                if (log_level() > 0)
                    std::fprintf(stderr, "ncf: plan settings from the autotune cache [%s]\n",
                                 ckey.c_str());
                *out = P;
                return NCF_OK;
            }
            plan_free(P);  // e.g. a grid that no longer fits: tune again
            clear_error();
        }
    }

    ncf_plan_s* best = new ncf_plan_s;
    int rc = plan_build(best, J, tin, ein, Tune{}, dummy);
    if (rc != NCF_OK) {
        plan_free(best);
        return rc;
    }
    if (J.opt.flags & NCF_PLAN_AUTOTUNE) {
        constexpr int kReps = 3;
        double tb = 0.0;
        rc = plan_time(best, dummy, kReps, &tb);
        if (rc != NCF_OK) {
            plan_free(best);
            return rc;
        }
        int ncand = 1;
        auto attempt = [&](const Tune& t) -> int {
            ncf_plan_s* P = new ncf_plan_s;
            double tp = 0.0;
            int r = plan_build(P, J, tin, ein, t, dummy);
            if (r == NCF_OK) r = plan_time(P, dummy, kReps, &tp);
            if (r != NCF_OK) {  // e.g. a larger grid that does not fit: skip it
                plan_free(P);
                clear_error();
                return r == NCF_E_DEVICE ? r : NCF_OK;
            }
            ++ncand;
            if (log_level() > 1)
                std::fprintf(stderr,
                             "ncf: autotune candidate sigma=%g fft_split=%d fft_tile_log2=%d "
                             "window_tile_scale=%d window_queue=%d no_mid=%d eval_interp=%d: "
                             "%.3f ms (best %.3f ms)\n",
                             t.sigma, t.fft.split, t.fft.lgt_strided, t.jscale, t.queue ? 1 : 0,
                             t.no_mid ? 1 : 0, t.eval_interp ? 1 : 0, tp, tb);
            if (tp < 0.97 * tb) {
                plan_free(best);
                best = P;
                tb = tp;
            } else {
                plan_free(P);
            }
            return NCF_OK;
        };
        const bool fp64 = J.opt.precision == NCF_FP64;
        if (best->grids > 0 && !J.regular) {
            for (double sg : {1.25, 2.0}) {
                Tune t = best->tune;
                t.sigma = sg;
                rc = attempt(t);
                if (rc != NCF_OK) break;
            }
        }
        if (best->grids > 0) {
            for (int sp : {1, 2}) {
                if (rc != NCF_OK) break;
                Tune t = best->tune;
                t.fft.split = sp;
                rc = attempt(t);
            }
            if (rc == NCF_OK && !fp64 && !J.regular) {
                Tune t = best->tune;
                t.fft.lgt_strided = 12;
                rc = attempt(t);
            }
            if (rc == NCF_OK && !J.regular) {  // separate last pass and product
                Tune t = best->tune;
                t.no_mid = true;
                rc = attempt(t);
            }
            if (rc == NCF_OK && !J.regular && best->fold_grids > 0) {
                // lags by inverse transform and interpolation although they
                // sit on a lattice
                Tune t = best->tune;
                t.eval_interp = true;
                rc = attempt(t);
            }
        }
        if (rc == NCF_OK && best->window_items > 0) {
            for (int js : {-1, 1}) {
                Tune t = best->tune;
                t.jscale = js;
                rc = attempt(t);
                if (rc != NCF_OK) break;
            }
            if (rc == NCF_OK) {
                Tune t = best->tune;
                t.queue = true;
                rc = attempt(t);
            }
        }
        if (rc != NCF_OK) {
            plan_free(best);
            return rc;
        }
        best->autotuned = 1;
        best->candidates = ncand;
        best->replay_ms = tb;
        if (cpath) tune_cache_store(cpath, ckey, best->tune, tb);
        if (log_level() > 0)
            std::fprintf(stderr, "ncf: plan autotuned over %d candidates: %.3f ms per execution\n",
                         ncand, tb);
    }
    *out = best;
    return NCF_OK;
}

int plan_acf_impl(int64_t nser, const int64_t* offs, const double* t, const double* err,
                  const double* dt, bool regular, int64_t K, const double* lags, int kern,
                  const double* h, const ncf_options_t* opt, ncf_plan_t** out) {
    clear_error();
    if (!out) {
        set_error("null plan pointer");
        return NCF_E_INVALID_ARG;
    }
    *out = nullptr;
    Job J;
    NCF_TRY(common_checks(opt, &J.opt, kern));
    if (nser <= 0 || !t || !h || (regular && !dt)) {
        set_error("null argument or nser <= 0");
        return NCF_E_INVALID_ARG;
    }
    int64_t total = 0;
    NCF_TRY(check_offs(offs, nser, &total));
    std::lock_guard<std::mutex> lock(g_ws_mu);
    J.regular = regular;
    if (regular) J.dt.assign(dt, dt + nser);
    NCF_TRY(setup_job(J, false, nser, offs, nullptr, total, 0, kern, h, K, lags));
    const double* tin[2] = {t, nullptr};
    const double* ein[2] = {err, nullptr};
    return plan_create(J, tin, ein, out);
}

int plan_ccf_impl(int64_t npair, const int64_t* offx, const double* tx, const double* ex,
                  const int64_t* offy, const double* ty, const double* ey, const double* dt,
                  bool regular, int64_t K, const double* lags, int kern, const double* h,
                  const ncf_options_t* opt, ncf_plan_t** out) {
    clear_error();
    if (!out) {
        set_error("null plan pointer");
        return NCF_E_INVALID_ARG;
    }
    *out = nullptr;
    Job J;
    NCF_TRY(common_checks(opt, &J.opt, kern));
    if (npair <= 0 || !tx || !ty || !h || (regular && !dt)) {
        set_error("null argument or npair <= 0");
        return NCF_E_INVALID_ARG;
    }
    int64_t totx = 0, toty = 0;
    NCF_TRY(check_offs(offx, npair, &totx));
    NCF_TRY(check_offs(offy, npair, &toty));
    std::lock_guard<std::mutex> lock(g_ws_mu);
    J.regular = regular;
    if (regular) J.dt.assign(dt, dt + npair);
    NCF_TRY(setup_job(J, true, npair, offx, offy, totx, toty, kern, h, K, lags));
    const double* tin[2] = {tx, ty};
    const double* ein[2] = {ex, ey};
    return plan_create(J, tin, ein, out);
}

int plan_status_error(const int32_t* st, int64_t n) {
    for (int64_t p = 0; p < n; ++p)
        if (st[p] != NCF_OK) {
            set_error("series %lld failed with status %d", (long long)p, st[p]);
            return st[p];
        }
    return NCF_OK;
}

}  // namespace
}  // namespace ncf

extern "C" {

int ncf_plan_acf(int64_t nser, const int64_t* offs, const double* t, const double* err,
                 int64_t K, const double* lags, int kern, const double* h,
                 const ncf_options_t* opt, ncf_plan_t** out) {
    return plan_acf_impl(nser, offs, t, err, nullptr, false, K, lags, kern, h, opt, out);
}

int ncf_plan_ccf(int64_t npair, const int64_t* offx, const double* tx, const double* ex,
                 const int64_t* offy, const double* ty, const double* ey, int64_t K,
                 const double* lags, int kern, const double* h, const ncf_options_t* opt,
                 ncf_plan_t** out) {
    return plan_ccf_impl(npair, offx, tx, ex, offy, ty, ey, nullptr, false, K, lags, kern, h, opt,
                         out);
}

int ncf_plan_acf_regular(int64_t nser, const int64_t* offs, const double* t, const double* err,
                         const double* dt, int64_t K, const double* lags, int kern,
                         const double* h, const ncf_options_t* opt, ncf_plan_t** out) {
    return plan_acf_impl(nser, offs, t, err, dt, true, K, lags, kern, h, opt, out);
}

int ncf_plan_ccf_regular(int64_t npair, const int64_t* offx, const double* tx, const double* ex,
                         const int64_t* offy, const double* ty, const double* ey,
                         const double* dt, int64_t K, const double* lags, int kern,
                         const double* h, const ncf_options_t* opt, ncf_plan_t** out) {
    return plan_ccf_impl(npair, offx, tx, ex, offy, ty, ey, dt, true, K, lags, kern, h, opt,
                         out);
}

int ncf_plan_execute(ncf_plan_t* P, const double* x, const double* y, double* c, double* b,
                     int64_t* count, int* status) {
    clear_error();
    if (!P || !x || (P->ccf && !y) || (P->K > 0 && (!c || !b))) {
        set_error("null argument");
        return NCF_E_INVALID_ARG;
    }
    int dev = 0;
    NCF_TRY_HIP(hipGetDevice(&dev));
    if (dev != P->device) {
        set_error("plan belongs to device %d, current device is %d", P->device, dev);
        return NCF_E_INVALID_ARG;
    }
    const hipStream_t st = P->st;
    IoBlock io{};
    if (P->dev_ptrs) {
        io.x[0] = x;
        io.x[1] = P->ccf ? y : nullptr;
        io.c = c;
        io.b = b;
        io.count = count;
        io.status = status ? (int32_t*)status : P->status;
    } else {
        NCF_TRY_HIP(hipMemcpyAsync(P->xbuf[0], x, sizeof(double) * P->ntot[0],
                                   hipMemcpyHostToDevice, st));
        if (P->ccf)
            NCF_TRY_HIP(hipMemcpyAsync(P->xbuf[1], y, sizeof(double) * P->ntot[1],
                                       hipMemcpyHostToDevice, st));
        io.x[0] = P->xbuf[0];
        io.x[1] = P->xbuf[1];
        io.c = P->cbuf;
        io.b = P->bbuf;
        io.count = count ? P->nbuf : nullptr;
        io.status = P->status;
    }
    NCF_TRY(launch_set_io(P->io, io, st));
    if (P->exec) {
        ProfScope ps(st, "plan_graph", 0.0, "launches");
        NCF_TRY_HIP(hipGraphLaunch(P->exec, st));
    } else {
        for (auto& f : P->rec) NCF_TRY(f(st));
    }
    if (P->dev_ptrs) return NCF_OK;
    const int64_t nout = P->nprob * P->K;
    if (nout > 0) {
        NCF_TRY_HIP(hipMemcpyAsync(c, P->cbuf, sizeof(double) * nout, hipMemcpyDeviceToHost, st));
        NCF_TRY_HIP(hipMemcpyAsync(b, P->bbuf, sizeof(double) * nout, hipMemcpyDeviceToHost, st));
        if (count)
            NCF_TRY_HIP(
                hipMemcpyAsync(count, P->nbuf, sizeof(int64_t) * nout, hipMemcpyDeviceToHost, st));
    }
    NCF_TRY_HIP(hipMemcpyAsync(P->hstatus.data(), P->status, sizeof(int32_t) * P->nprob,
                               hipMemcpyDeviceToHost, st));
    NCF_TRY_HIP(hipStreamSynchronize(st));
    if (status)
        for (int64_t p = 0; p < P->nprob; ++p) status[p] = P->hstatus[p];
    return plan_status_error(P->hstatus.data(), P->nprob);
}

void ncf_plan_destroy(ncf_plan_t* P) { plan_free(P); }

int ncf_plan_info(const ncf_plan_t* P, ncf_plan_info_t* info) {
    clear_error();
    if (!P || !info || info->struct_size != sizeof(ncf_plan_info_t)) {
        set_error("null plan or info, or info.struct_size mismatch");
        return NCF_E_INVALID_ARG;
    }
    info->autotuned = P->autotuned;
    info->candidates = P->candidates;
    info->spectral_grids = P->grids;
    info->window_launches = P->window_launches;
    info->grid_cells = P->grid_cells;
    info->window_items = P->window_items;
    info->sigma = P->tune.sigma > 1.0 ? P->tune.sigma : 0.0;
    info->fft_split = P->tune.fft.split;
    info->fft_tile_log2 = P->tune.fft.lgt_strided;
    info->window_tile_scale = P->tune.jscale;
    info->window_queue = P->tune.queue ? 1 : 0;
    info->graph = P->exec ? 1 : 0;
    info->replay_ms = P->replay_ms;
    info->lattice_grids = P->fold_grids;
    info->lattice_off = P->tune.eval_interp ? 1 : 0;
    info->tune_cached = P->tune_cached;
    return NCF_OK;
}

// ------------------------------------------------------------- diagnostics

int ncf_diag_fft_radices(int64_t N, int* radices, int max) {
    clear_error();
    if (N < 4096 || (N & (N - 1))) {
        set_error("N must be a power of two >= 4096");
        return NCF_E_INVALID_ARG;
    }
    int p = 0;
    while ((1LL << p) < N) ++p;
    int r[3], np;
    if (p == 12) {
        np = 1;
        r[0] = 4096;
    } else if (p <= 22) {
        np = 2;
        r[0] = 1 << (p - 12);
        r[1] = 4096;
    } else {
        np = 3;
        r[0] = 1 << ((p - 11) / 2);
        r[1] = 1 << ((p - 12) / 2);
        r[2] = 4096;
    }
    for (int i = 0; i < np && i < max; ++i) radices[i] = r[i];
    return np;
}

int ncf_diag_fft(int64_t N, int precision, int sign, void* data) {
    clear_error();
    if (!data || (sign != 1 && sign != -1)) {
        set_error("invalid argument");
        return NCF_E_INVALID_ARG;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        set_error("no HIP device available");
        return NCF_E_DEVICE;
    }
    const bool fp64 = precision == NCF_FP64;
    const size_t esz = fp64 ? 16 : 8;
    FftPlan plan;
    hipStream_t st = nullptr;
    NCF_TRY(fft_plan(N, fp64, &plan, st));
    std::vector<char> h((size_t)N * esz);
    // the -1 transform consumes digit-reversed order: permute on the host
    if (sign < 0) {
        for (int64_t k = 0; k < N; ++k)
            std::memcpy(&h[fft_position(plan, k) * esz], (char*)data + k * esz, esz);
    } else {
        std::memcpy(h.data(), data, (size_t)N * esz);
    }
    void* d = nullptr;
    NCF_TRY_HIP(hipMalloc(&d, (size_t)N * esz));
    void** dg = nullptr;
    NCF_TRY_HIP(hipMalloc((void**)&dg, sizeof(void*)));
    NCF_TRY_HIP(hipMemcpy(dg, &d, sizeof(void*), hipMemcpyHostToDevice));
    NCF_TRY_HIP(hipMemcpy(d, h.data(), (size_t)N * esz, hipMemcpyHostToDevice));
    int rc = fft_exec(plan, dg, 1, sign, fp64, st);
    if (rc == NCF_OK) {
        NCF_TRY_HIP(hipMemcpy(h.data(), d, (size_t)N * esz, hipMemcpyDeviceToHost));
        if (sign > 0) {
            for (int64_t k = 0; k < N; ++k)
                std::memcpy((char*)data + k * esz, &h[fft_position(plan, k) * esz], esz);
        } else {
            std::memcpy(data, h.data(), (size_t)N * esz);
        }
    }
    (void)hipFree(d);
    (void)hipFree(dg);
    return rc;
}

int ncf_diag_spread_params(double sigma, double eps, double* out) {
    if (!out || !(sigma > 1.0) || !(eps > 0.0 && eps < 1.0)) return NCF_E_INVALID_ARG;
    SpreadParams p = spread_params(sigma, eps);
    out[0] = p.s;
    out[1] = p.W;
    return NCF_OK;
}

int ncf_diag_grid(double tmin, double tmax, int64_t K, const double* lags, int acf, double h,
                  int precision, int lattice, double* out_f, int64_t* out_i) {
    clear_error();
    if (K < 0 || (K > 0 && !lags) || !out_f || !out_i || !(h > 0.0) || !std::isfinite(h) ||
        !(tmax >= tmin) || !std::isfinite(tmin) || !std::isfinite(tmax) ||
        (precision != NCF_MIXED && precision != NCF_FP64)) {
        set_error("ncf_diag_grid: invalid argument");
        return NCF_E_INVALID_ARG;
    }
    Job J;
    ncf_options_init(&J.opt);
    J.opt.precision = precision;
    J.kern = NCF_GAUSSIAN;
    J.ccf = acf == 0;
    J.lags.assign(lags, lags + K);
    double maxlag = 0.0;
    for (double v : J.lags) {
        if (!std::isfinite(v)) {
            set_error("ncf_diag_grid: non-finite lag");
            return NCF_E_INVALID_ARG;
        }
        maxlag = std::max(maxlag, std::fabs(v));
    }
    J.lag_unit = lattice ? lag_lattice_unit(J.lags, acf != 0) : 0.0;
    SpecGeom g;
    NCF_TRY(plan_grid(J, tmin, tmax, maxlag, h, &g));
    out_f[0] = g.L;
    out_f[1] = g.s;
    out_i[0] = g.N;
    out_i[1] = g.M;
    out_i[2] = g.P;
    return NCF_OK;
}

int ncf_diag_type1(int64_t n, const double* t, const double* v, double t_ref, double L,
                   int64_t N, int64_t M, int precision, double* out) {
    clear_error();
    if (n < 1 || !t || !v || !out || !(L > 0) || N < 4096 || (N & (N - 1)) || M < 0 ||
        2 * M + 1 > N) {
        set_error("invalid argument");
        return NCF_E_INVALID_ARG;
    }
    const bool fp64 = precision == NCF_FP64;
    const double sigma = (double)N / (2.0 * M + 1.0);
    if (sigma <= 1.0) return NCF_E_INVALID_ARG;
    SpreadParams sp = spread_params(sigma, fp64 ? 1e-13 : 1e-7);
    for (int64_t i = 0; i < n; ++i) {
        const double u = (t[i] - t_ref) * ((double)N / L);
        if (!(u >= sp.W + 2.0 && u <= (double)N - sp.W - 2.0) || (i && t[i] < t[i - 1])) {
            set_error("sample %lld outside the no-wrap band or unsorted", (long long)i);
            return NCF_E_INVALID_ARG;
        }
    }
    hipStream_t st = nullptr;
    const size_t esz = fp64 ? 16 : 8;
    double* dt;
    void* dv;
    void* grid;
    int64_t* rng;
    SpecTask* dtask;
    int64_t* dtile0;
    Chunk* dch;
    int32_t* dmap;
    void** dg;
    NCF_TRY_HIP(hipMalloc((void**)&dt, sizeof(double) * n));
    NCF_TRY_HIP(hipMalloc(&dv, (fp64 ? 8 : 4) * n));
    NCF_TRY_HIP(hipMalloc(&grid, esz * N));
    NCF_TRY_HIP(hipMalloc((void**)&rng, sizeof(int64_t) * kTileRec * (N / 4096)));
    NCF_TRY_HIP(hipMalloc((void**)&dtask, sizeof(SpecTask)));
    NCF_TRY_HIP(hipMalloc((void**)&dtile0, sizeof(int64_t) * 2));
    std::vector<Chunk> hch;
    for (int64_t b = 0; b < n; b += kChunk) hch.push_back(Chunk{b, std::min(b + kChunk, n), 0, 0});
    const int32_t hmap = 0;  // series 0 -> task 0, set 0
    NCF_TRY_HIP(hipMalloc((void**)&dch, sizeof(Chunk) * hch.size()));
    NCF_TRY_HIP(hipMalloc((void**)&dmap, sizeof(int32_t)));
    NCF_TRY_HIP(hipMalloc((void**)&dg, sizeof(void*)));
    NCF_TRY_HIP(hipMemcpy(dt, t, sizeof(double) * n, hipMemcpyHostToDevice));
    if (fp64) {
        NCF_TRY_HIP(hipMemcpy(dv, v, sizeof(double) * n, hipMemcpyHostToDevice));
    } else {
        std::vector<float> vf(v, v + n);
        NCF_TRY_HIP(hipMemcpy(dv, vf.data(), sizeof(float) * n, hipMemcpyHostToDevice));
    }
    SpecTask T{};
    T.t0 = dt;
    T.v0f = fp64 ? nullptr : (const float*)dv;
    T.v0d = fp64 ? (const double*)dv : nullptr;
    T.n0 = n;
    T.t_ref = t_ref;
    T.L = L;
    T.N = N;
    T.M = M;
    T.s = sp.s;
    T.W = sp.W;
    T.grid = grid;
    T.tile0 = 0;
    T.ntiles = N / 4096;
    T.tile_rng = rng;
    int64_t t0h[2] = {0, T.ntiles};
    NCF_TRY_HIP(hipMemcpy(dtask, &T, sizeof T, hipMemcpyHostToDevice));
    NCF_TRY_HIP(hipMemcpy(dtile0, t0h, sizeof t0h, hipMemcpyHostToDevice));
    NCF_TRY_HIP(hipMemcpy(dch, hch.data(), sizeof(Chunk) * hch.size(), hipMemcpyHostToDevice));
    NCF_TRY_HIP(hipMemcpy(dmap, &hmap, sizeof hmap, hipMemcpyHostToDevice));
    NCF_TRY_HIP(hipMemcpy(dg, &grid, sizeof(void*), hipMemcpyHostToDevice));
    int rc = launch_tile_bounds(dtask, dch, (int)hch.size(), dmap, st, 8.0 * n);
    if (rc == NCF_OK)
        rc = launch_spread(dtask, dtile0, 1, T.ntiles, rng, 4096, false, false, false, false, fp64,
                           st, 0.0);
    FftPlan plan;
    if (rc == NCF_OK) rc = fft_plan(N, fp64, &plan, st);
    if (rc == NCF_OK) rc = fft_exec(plan, dg, 1, +1, fp64, st);
    if (rc == NCF_OK) {
        std::vector<char> h(esz * N);
        NCF_TRY_HIP(hipMemcpy(h.data(), grid, esz * N, hipMemcpyDeviceToHost));
        const double twopi = 2.0 * M_PI;
        for (int64_t m = -M; m <= M; ++m) {
            const int64_t k = m >= 0 ? m : m + N;
            const int64_t p = fft_position(plan, k);
            double re, im;
            if (fp64) {
                re = ((double*)h.data())[2 * p];
                im = ((double*)h.data())[2 * p + 1];
            } else {
                re = ((float*)h.data())[2 * p];
                im = ((float*)h.data())[2 * p + 1];
            }
            // deconvolve: divide by Psi(m/N) = sqrt(2 pi) s exp(-2 pi^2 s^2 (m/N)^2)
            const double xi = (double)m / (double)N;
            const double psi = std::sqrt(twopi) * sp.s * std::exp(-2.0 * M_PI * M_PI * sp.s * sp.s * xi * xi);
            out[2 * (m + M)] = re / psi;
            out[2 * (m + M) + 1] = im / psi;
        }
    }
    (void)hipFree(dt);
    (void)hipFree(dv);
    (void)hipFree(grid);
    (void)hipFree(rng);
    (void)hipFree(dtask);
    (void)hipFree(dtile0);
    (void)hipFree(dch);
    (void)hipFree(dmap);
    (void)hipFree(dg);
    return rc;
}

void ncf_profile_enable(int on) {
    std::lock_guard<std::mutex> lock(g_prof_mu);
    if (on) {
        prof_flush_locked();
        g_prof.clear();
    }
    g_prof_on = on != 0;
}

void ncf_profile_filter(const char* name) {
    std::lock_guard<std::mutex> lock(g_prof_mu);
    g_prof_only = name ? name : "";
}

int ncf_profile_read(ncf_profile_record_t* out, int max) {
    (void)hipDeviceSynchronize();
    std::lock_guard<std::mutex> lock(g_prof_mu);
    prof_flush_locked();
    int i = 0;
    for (auto& kv : g_prof) {
        if (i >= max) break;
        ncf_profile_record_t& r = out[i++];
        std::memset(&r, 0, sizeof r);
        std::snprintf(r.name, sizeof r.name, "%s", kv.first.c_str());
        r.launches = kv.second.launches;
        r.total_ms = kv.second.ms;
        r.work = kv.second.work;
        std::snprintf(r.work_unit, sizeof r.work_unit, "%s", kv.second.unit.c_str());
    }
    return i;
}

}  // extern "C"
