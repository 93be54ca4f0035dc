"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds only input generation (sampling patterns and signals): no
part of the correlation estimator. Both the GPU path's tests and the CPU
oracle's tests draw their inputs from here.

Workloads (all seeded with numpy's PCG64):

* ``c1`` -- single-series ACF, n = 2000, i.i.d. exponential gaps of mean 1 d
  from t = 0; x = Ornstein-Uhlenbeck / damped random walk, time scale 20 d,
  unit variance, exact transition (the footnote of Sec. 3.1 on the OU
  discretisation), plus white noise sd 0.1. Gaussian kernel,
  h = 0.25 x realized mean gap, lags 0..100 d.
* ``c2`` -- CCF of two independent irregular series, n = 1e5 each, nightly
  epochs within an 8-month (243-night) season per 365.25-d year, 30 % of
  nights dropped, +-0.1 d jitter. x = DRW (50 d) on a 0.05-d grid, y = x
  smoothed by a centred 10-d top-hat and delayed by 40 d, plus noise sd 0.05;
  each series read at its own epochs by linear interpolation. Lags -200..200 d,
  h = 0.5 d, Gaussian and rectangle kernels.
* ``c3`` -- ACF of n = 1e7 samples on a unit grid with 5 % dropouts and
  +-0.3 jitter; x = three unit sinusoids (periods 7, 31, 365) plus unit white
  noise; lags 0..4095, Gaussian, h = 0.25 x realized mean gap.
* ``c4`` -- 10,000 light curves, lengths log-uniform in [100, 5e4], seasonal
  sampling as c2; quasi-periodic rotation signal of eq. astro_model with
  period U[5, 50] d, OU amplitude (A0 = 1, sd 0.35, time scale U[2, 5]
  periods), flicker = 5 OU components with time scales log-spaced over
  0.5-50 d whose variances sum to 0.55^2, heteroscedastic errors
  sd_i = 0.01 * 10^(0.5 N(0,1)). Lags 0..255 d, Gaussian, h = 0.5 d.
* ``c5`` -- 2,048 CCF pairs, each length log-uniform in [1e3, 2e5]; DRW driver
  (50 d, 0.5-d latent grid) and its 10-d top-hat smoothed response delayed by
  U[5, 100] d plus noise sd 0.05; 512 lags over [-300, 300] d, rectangle,
  h = 0.5 d.

* ``r1`` -- regular-lattice ACF (the paper's benchmark on regularly sampled
  data, Sec. "Regularly-sampled data"): white noise N(0, 1) on t = m dt,
  dt = 1 d, n = 2.56e5 samples without gaps, integer lags 0..365 d
  (K = 366), Gaussian and rectangle kernels with h = 0.5 d.
* ``m1`` -- Monte-Carlo error bars of a c2-shaped CCF: n = 2e4 samples per
  series, errors sd 0.05, R = 100 replicates, each with flux randomization
  (standard normal deviates) and a bootstrap resampling (multiplicities of
  n draws with replacement); lags -200..200 d, Gaussian, h = 0.5 d.
* ``r2`` -- batched regular-lattice ACF: 4,096 series on 1-d lattices,
  lengths log-uniform in [1e3, 1e5], 10 % of lattice points dropped, white
  noise; lags 0..365 d, rectangle, h = 0.5 d.

Scaled-down variants (``scale`` < 1) keep the sampling pattern and signal and
shrink only the lengths / counts; tests use them at sizes the oracle finishes
in seconds.
"""
from __future__ import annotations

import math

import numpy as np

YEAR = 365.25
SEASON_NIGHTS = 243


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------- sampling

def exp_gap_times(rng, n, mean_gap=1.0):
    gaps = rng.exponential(mean_gap, size=n - 1)
    return np.concatenate([[0.0], np.cumsum(gaps)])


def seasonal_epochs(rng, n, keep=0.7, jitter=0.1, phase=0.0, start=0.0):
    """Nightly epochs in a 243-night season per 365.25-d year, each night kept
    with probability ``keep``, jittered by U(-jitter, jitter). Returns n sorted
    epochs."""
    frac_in = SEASON_NIGHTS / YEAR * keep
    out = []
    got = 0
    night0 = 0
    while got < n:
        m = int((n - got) / frac_in * 1.2) + 64
        d = np.arange(night0, night0 + m, dtype=np.float64)
        night0 += m
        inseason = np.mod(d + phase, YEAR) < SEASON_NIGHTS
        kept = inseason & (rng.random(m) < keep)
        e = d[kept] + rng.uniform(-jitter, jitter, size=int(kept.sum()))
        out.append(e)
        got += e.size
    t = np.concatenate(out)[:n] + start
    return t


def jittered_grid_times(rng, n, keep=0.95, jitter=0.3):
    """Unit grid with random dropouts (each point kept with ``keep``), extended
    until exactly n are kept, then jittered by U(-jitter, jitter)."""
    G = int(math.ceil(n / keep))
    parts = []
    got = 0
    g0 = 0
    while got < n:
        g = np.arange(g0, g0 + G, dtype=np.float64)
        g0 += G
        k = g[rng.random(G) < keep]
        parts.append(k)
        got += k.size
        G = max(1024, int((n - got) / keep * 1.1) + 64)
    g = np.concatenate(parts)[:n]
    return g + rng.uniform(-jitter, jitter, size=n)


# ----------------------------------------------------------------- signals

def ou_at_times(rng, t, tau, sd=1.0):
    """Stationary OU process at sorted times t via the exact transition
    x_{i+1} = a x_i + sqrt(1 - a^2) sd N(0,1), a = exp(-dt/tau)."""
    n = t.size
    z = rng.standard_normal(n)
    a = np.exp(-np.diff(t) / tau)
    e = np.empty(n)
    e[0] = sd * z[0]
    e[1:] = sd * np.sqrt(1.0 - a * a) * z[1:]
    return _ar1_scan(np.concatenate([[0.0], a]), e)


def _ar1_scan(a, e):
    """x_i = a_i x_{i-1} + e_i (a_0 ignored), by a doubling scan."""
    A = a.copy()
    A[0] = 0.0
    X = e.copy()
    d = 1
    n = X.size
    while d < n:
        Xn = X.copy()
        Xn[d:] = X[d:] + A[d:] * X[:-d]
        An = A.copy()
        An[d:] = A[d:] * A[:-d]
        X, A = Xn, An
        if not A[d:].any():
            break
        d *= 2
    return X


def drw_grid(rng, n_grid, dt, tau):
    """Unit-variance DRW (AR(1) with a = exp(-dt/tau)) on a regular grid."""
    from scipy.signal import lfilter
    a = math.exp(-dt / tau)
    z = rng.standard_normal(n_grid)
    z[1:] *= math.sqrt(1.0 - a * a)
    zi = np.array([0.0])
    out, _ = lfilter([1.0], [1.0, -a], z, zi=zi)
    return out


def tophat_smooth(x, width_pts):
    """Centred moving average over ``width_pts`` grid points (edges shrink)."""
    c = np.concatenate([[0.0], np.cumsum(x)])
    n = x.size
    half = width_pts // 2
    lo = np.clip(np.arange(n) - half, 0, n)
    hi = np.clip(np.arange(n) - half + width_pts, 0, n)
    return (c[hi] - c[lo]) / (hi - lo)


# -------------------------------------------------------------- workloads

def c1(seed=1, n=2000):
    rng = rng_for(seed)
    t = exp_gap_times(rng, n, 1.0)
    x = ou_at_times(rng, t, 20.0) + rng.normal(0.0, 0.1, size=n)
    mean_gap = (t[-1] - t[0]) / (n - 1)
    return dict(kind="acf", name="c1", t=t, x=x, err=None, lags=np.arange(101.0),
                kernel="gaussian", h=0.25 * mean_gap)


def _c2_pair(rng, nx, ny, delay, dt_grid, noise=0.05, tau=50.0, tophat=10.0, phase=None):
    if phase is None:
        phase = rng.uniform(0.0, YEAR)
    tx = seasonal_epochs(rng, nx, phase=phase)
    ty = seasonal_epochs(rng, ny, phase=phase)
    tmax = max(tx[-1], ty[-1])
    pad = tophat + delay + 5.0
    g0 = -pad
    ng = int((tmax + 2 * pad) / dt_grid) + 2
    grid = g0 + dt_grid * np.arange(ng)
    lat = drw_grid(rng, ng, dt_grid, tau)
    resp = tophat_smooth(lat, max(1, int(round(tophat / dt_grid))))
    x = np.interp(tx, grid, lat)
    # y(t) = smoothed latent at t - delay
    y = np.interp(ty - delay, grid, resp) + rng.normal(0.0, noise, size=ny)
    return tx, x, ty, y


def c2(seed=2, n=100_000, kernel="gaussian"):
    rng = rng_for(seed)
    tx, x, ty, y = _c2_pair(rng, n, n, 40.0, 0.05)
    lags = -200.0 + np.arange(401.0)
    return dict(kind="ccf", name="c2", t=tx, x=x, s=ty, y=y, ex=None, ey=None, lags=lags,
                kernel=kernel, h=0.5)


def c3(seed=3, n=10_000_000, K=4096):
    rng = rng_for(seed)
    t = jittered_grid_times(rng, n, 0.95, 0.3)
    x = rng.standard_normal(n)
    for P in (7.0, 31.0, 365.0):
        x += np.sin(2.0 * np.pi * t / P + rng.uniform(0.0, 2.0 * np.pi))
    mean_gap = (t[-1] - t[0]) / (n - 1)
    return dict(kind="acf", name="c3", t=t, x=x, err=None, lags=np.arange(float(K)),
                kernel="gaussian", h=0.25 * mean_gap)


def _ou_batch(rng, t, offs, taus, sds):
    """Independent stationary OU processes for every series of a CSR batch and
    every (tau, sd) column: exact transitions, advanced one sample index at a
    time across all series (all columns at once)."""
    ns = np.diff(offs)
    order = np.argsort(-ns, kind="stable")  # longest first: active set is a prefix
    ns_sorted = ns[order]
    starts = offs[:-1][order]
    taus = np.asarray(taus, dtype=np.float64)
    sds = np.asarray(sds, dtype=np.float64)
    ncol = taus.shape[-1]
    out = np.empty((t.size, ncol))
    first = starts
    out[first] = sds[order] * rng.standard_normal((first.size, ncol))
    for i in range(1, int(ns_sorted[0])):
        m = int(np.searchsorted(-ns_sorted, -i, side="left"))  # series with n > i
        idx = starts[:m] + i
        a = np.exp(-(t[idx] - t[idx - 1])[:, None] / taus[order[:m]])
        z = rng.standard_normal((m, ncol))
        out[idx] = a * out[idx - 1] + sds[order[:m]] * np.sqrt(1.0 - a * a) * z
    return out


def c4(seed=4, n_series=10_000, nmin=100, nmax=50_000, K=256, with_err=False):
    rng = rng_for(seed)
    ns = np.round(np.exp(rng.uniform(math.log(nmin), math.log(nmax), size=n_series))).astype(
        np.int64)
    offs = np.concatenate([[0], np.cumsum(ns)])
    tot = int(offs[-1])
    t = np.empty(tot)
    for c in range(n_series):
        t[offs[c]:offs[c + 1]] = seasonal_epochs(rng, int(ns[c]), phase=rng.uniform(0.0, YEAR))
    P = rng.uniform(5.0, 50.0, size=n_series)
    tauA = rng.uniform(2.0, 5.0, size=n_series) * P
    phase = rng.uniform(0.0, 2.0 * np.pi, size=n_series)
    flick_tau = np.exp(np.linspace(math.log(0.5), math.log(50.0), 5))
    flick_sd = math.sqrt(0.55 ** 2 / 5.0)
    # columns: amplitude OU (tau_A, 0.35) and 5 flicker components
    taus = np.column_stack([tauA] + [np.full(n_series, tf) for tf in flick_tau])
    sds = np.column_stack([np.full(n_series, 0.35)] + [np.full(n_series, flick_sd)] * 5)
    ou = _ou_batch(rng, t, offs, taus, sds)
    sid = np.repeat(np.arange(n_series), ns)
    A = 1.0 + ou[:, 0]
    x = A * np.cos(2.0 * np.pi * t / P[sid] + phase[sid]) + ou[:, 1:].sum(axis=1)
    err = 0.01 * 10.0 ** (0.5 * rng.standard_normal(tot))
    x += rng.standard_normal(tot) * err
    return dict(kind="acf_batch", name="c4", offs=offs, t=t, x=x,
                err=err if with_err else None, err_values=err, lags=np.arange(float(K)),
                kernel="gaussian", h=np.full(n_series, 0.5))


def c5(seed=5, n_pairs=2048, nmin=1000, nmax=200_000, K=512):
    rng = rng_for(seed)
    nx = np.round(np.exp(rng.uniform(math.log(nmin), math.log(nmax), size=n_pairs))).astype(
        np.int64)
    ny = np.round(np.exp(rng.uniform(math.log(nmin), math.log(nmax), size=n_pairs))).astype(
        np.int64)
    offx = np.concatenate([[0], np.cumsum(nx)])
    offy = np.concatenate([[0], np.cumsum(ny)])
    tx = np.empty(int(offx[-1]))
    x = np.empty_like(tx)
    ty = np.empty(int(offy[-1]))
    y = np.empty_like(ty)
    delays = rng.uniform(5.0, 100.0, size=n_pairs)
    for p in range(n_pairs):
        a, b, c, d = _c2_pair(rng, int(nx[p]), int(ny[p]), delays[p], 0.5)
        sx, sy = slice(offx[p], offx[p + 1]), slice(offy[p], offy[p + 1])
        tx[sx], x[sx], ty[sy], y[sy] = a, b, c, d
    lags = np.linspace(-300.0, 300.0, K)
    return dict(kind="ccf_batch", name="c5", offx=offx, t=tx, x=x, offy=offy, s=ty, y=y,
                lags=lags, kernel="rectangle", h=np.full(n_pairs, 0.5), delays=delays)


# --------------------------------------------------------- regular lattice

def lattice_times(rng, n, dt=1.0, keep=1.0, t0=0.0, dup_frac=0.0):
    """n times on the lattice t0 + m dt (m increasing from 0); each lattice
    point kept with probability `keep`, and a fraction `dup_frac` of the
    samples repeated at the previous sample's time."""
    if keep >= 1.0:
        m = np.arange(n, dtype=np.int64)
    else:
        gaps = rng.geometric(keep, size=n - 1)
        m = np.concatenate([[0], np.cumsum(gaps)]).astype(np.int64)
    if dup_frac > 0.0:
        k = int(dup_frac * n)
        idx = np.sort(rng.integers(1, n, size=k))
        m[idx] = m[idx - 1]
        m = np.sort(m)
    return t0 + m * dt


def r1(seed=11, n=256_000, kernel="gaussian", K=366):
    rng = rng_for(seed)
    t = lattice_times(rng, n, dt=1.0)
    x = rng.normal(size=n)
    return dict(kind="acf", name="r1", t=t, x=x, err=None, dt=1.0,
                lags=np.arange(K, dtype=np.float64), kernel=kernel, h=0.5)


def r2(seed=12, n_series=4096, nmin=1000, nmax=100_000, K=366, kernel="rectangle"):
    rng = rng_for(seed)
    ns = np.round(np.exp(rng.uniform(math.log(nmin), math.log(nmax), n_series))).astype(np.int64)
    offs = np.concatenate([[0], np.cumsum(ns)])
    t = np.empty(offs[-1])
    for i in range(n_series):
        t[offs[i]:offs[i + 1]] = lattice_times(rng, int(ns[i]), dt=1.0, keep=0.9)
    x = rng.normal(size=offs[-1])
    return dict(kind="acf_batch", name="r2", offs=offs, t=t, x=x, err=None, dt=np.ones(n_series),
                lags=np.arange(K, dtype=np.float64), kernel=kernel, h=np.full(n_series, 0.5))


# ------------------------------------------------------- replicate draws

def resample_draws(rng, n, R, flux=True, bootstrap=True):
    """Random inputs of R replicates of an n-sample series: z (R, n) standard
    normal deviates for flux randomization, and mult (R, n) int32 bootstrap
    multiplicities (the counts of n draws with replacement). Either may be
    None."""
    z = rng.normal(size=(R, n)) if flux else None
    mult = None
    if bootstrap:
        mult = np.stack([np.bincount(rng.integers(0, n, size=n), minlength=n)
                         for _ in range(R)]).astype(np.int32)
    return z, mult


def m1(seed=13, n=20_000, R=100, K=401):
    """Monte-Carlo error bars of a c2-shaped CCF: two seasonal series of n
    samples (DRW driver, delayed top-hat response), measurement errors sd
    0.05 on both (ex, ey: the flux-randomization scale); R replicates with
    flux randomization and bootstrap resampling; lags -200..200 d, Gaussian,
    h = 0.5 d."""
    d = c2(seed, n=n, kernel="gaussian")
    rng = rng_for(seed + 1000)
    nx, ny = d["t"].size, d["s"].size
    d["ex"] = np.full(nx, 0.05)
    d["ey"] = np.full(ny, 0.05)
    d["zx"], d["multx"] = resample_draws(rng, nx, R)
    d["zy"], d["multy"] = resample_draws(rng, ny, R)
    d.update(kind="ccf_resample", name="m1", R=R)
    return d


WORKLOADS = {"c1": c1, "c2": c2, "c3": c3, "c4": c4, "c5": c5, "r1": r1, "r2": r2, "m1": m1}


def small(name, seed=0):
    """Scaled-down version of a workload: same sampling pattern and signal,
    sizes the oracle finishes in well under a second."""
    if name == "c1":
        return c1(seed, n=2000)
    if name == "c2":
        return c2(seed, n=3000)
    if name == "c3":
        return c3(seed, n=20_000, K=300)
    if name == "c4":
        return c4(seed, n_series=24, nmin=100, nmax=3000, K=64)
    if name == "c5":
        return c5(seed, n_pairs=12, nmin=300, nmax=4000, K=96)
    if name == "r1":
        return r1(seed, n=20_000, K=366)
    if name == "r2":
        return r2(seed, n_series=16, nmin=200, nmax=6000, K=120)
    if name == "m1":
        return m1(seed, n=1500, R=12, K=101)
    raise KeyError(name)
