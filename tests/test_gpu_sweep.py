"""Seeded random sweep of the GPU path against the FP64 oracle.

Each case draws an ACF or CCF call (or a batch), the kernel, the precision
and the method, the series lengths (2 to 4,000 samples, log-uniform), the
sampling pattern, the lag set (sorted, unsorted with repeats, beyond the
data) and h (0.2 to 20 mean spacings), and compares every output with the
oracle. Statuses must be equal; c and b are compared at the single-call
parity tolerances, plus the terms that the data of a random case can call
for (each derived in the design notes, each named where it is applied):

  * rectangle: counts bit-exact, c within 1e-9;
  * Gaussian, mixed precision: c within 1e-5; b within 1e-5 of the largest
    pair count of the call (spectral pair count) or 1e-6 relative (window
    scan pair count);
  * Gaussian, FP64 direct: c within 1e-11 and b 1e-12 relative, or the
    recursive-summation bound 4e-16 n when larger, n the largest pair count
    of the lags and of the lag-0 scale sums (bursts put 1e5 to 1e6 pairs
    under one lag);
  * Gaussian, FP64 spectral: the oracle truncates the kernel at 6h and the
    transforms do not; the mass beyond 6h is ~2e-9 of a window's at even
    density (the only pattern FP64 spectral calls are drawn with), and lags
    down to beta = 1e-2 of the reference are served spectrally, so c within
    4e-7 and b 2e-7 relative (the parity tests' 5e-8 holds on the
    benchmark workloads, whose lags stay far above the threshold).

Near-degenerate lag-0 scales: c = r(tau) / s with s the lag-0 scale (ACF
r(0), CCF sqrt(r_x(0) r_y(0))). When a kernel wide against a short series
makes a lag-0 sum of standardized values cancel (r(0) << 1), the absolute
error u of r(tau) and the relative error u / r_min of s (r_min the smaller
r(0); u = 1e-15 in FP64 sums, prefix sums included) both reach c divided by
r_min: FP64 and rectangle tolerances add u (1 + |c|) / g with g = min(1,
r_min). In mixed precision (u = 1e-6 with FP32 kernel weights or
transforms) the library evaluates a Gaussian problem again in FP64 when its
lag-0 scale is below 0.1, so the mixed tolerance is the plain 1e-5 and the
statuses equal the oracle's. r_min is computed here from the standardized
values under the case's window. Plan executions cannot re-evaluate: below
0.1 (a band of +-10 % around it accepts either outcome) a mixed Gaussian
problem reports NCF_E_UNSUPPORTED, or degenerate where the FP32 lag-0 sum
rounds to zero.

Series of fewer than 32 samples take the direct window sums on every route
(the spectral route forced onto them, method "spectral" or the forced route
of "auto", left transform rounding far above its usual size: up to 1e-1 at
2 to 6 samples); they are checked at the parity tolerances.

Sampling patterns: evenly random; seasonal (observable part of a 365-day
cycle only); bursts (a few tight clusters holding most samples, so some
work items take the global-memory window path); a quarter-day grid with
ties.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_03866_amd import ncf, synth

pytestmark = pytest.mark.gpu

PATTERNS = ("even", "seasonal", "bursts", "ties")


def _times(rng, n, span, pattern):
    if pattern == "even":
        t = rng.uniform(0.0, span, n)
    elif pattern == "seasonal":
        t = np.empty(0)
        while t.size < n:
            u = rng.uniform(0.0, span, 2 * n)
            t = np.concatenate([t, u[(u % 365.0) < 150.0]])
        t = t[:n]
    elif pattern == "bursts":
        nb = int(rng.integers(1, 4))
        centres = rng.uniform(0.0, span, nb)
        k = rng.integers(0, nb + 1, n)  # index nb: the sparse background
        width = span * 1e-3
        t = np.where(k < nb, centres[np.minimum(k, nb - 1)] + rng.normal(0.0, width, n),
                     rng.uniform(0.0, span, n))
    else:
        t = np.round(rng.uniform(0.0, span, n) * 4.0) / 4.0
    return np.sort(t)


def _series(rng, n, span, pattern):
    t = _times(rng, n, span, pattern)
    x = rng.normal(size=n).cumsum() * 0.1 + rng.normal(size=n)
    return t, x


def _lags(rng, span):
    K = int(np.exp(rng.uniform(0.0, np.log(256.0))))
    L = rng.uniform(0.05, 1.2) * span
    kind = rng.integers(0, 3)
    if kind == 0:
        lags = np.linspace(-L, L, K)
    elif kind == 1:
        lags = rng.uniform(-L, L, K)
        if K > 3:
            lags[rng.integers(0, K, K // 4)] = lags[0]  # repeats
    else:
        lags = np.sort(rng.uniform(0.0, L, K))
    return lags


def _mode(rng, kernel, pattern):
    prec = ("mixed", "fp64")[int(rng.integers(0, 2))]
    if kernel == "rectangle":
        return prec, ("auto", "direct")[int(rng.integers(0, 2))], bool(rng.integers(0, 2))
    method = ("auto", "direct", "spectral")[int(rng.integers(0, 3))]
    if prec == "fp64" and pattern != "even":
        method = "direct"
    return prec, method, bool(rng.integers(0, 2))


def _lag0_r(t, x, h, kernel, err=None):
    """(r(0) of the standardized values under the case's window (Gaussian
    |d| < 6h, rectangle |d| <= h, as the oracle), its pair count)."""
    w = np.ones_like(x) if err is None else 1.0 / (err * err)
    m = np.sum(w * x) / np.sum(w)
    z = (x - m) / np.sqrt(np.sum(w * (x - m) ** 2) / np.sum(w))
    d = t[:, None] - t[None, :]
    if kernel == "gaussian":
        phi = np.where(np.abs(d) < 6.0 * h, np.exp(-0.5 * (d / h) ** 2), 0.0)
    else:
        phi = (np.abs(d) <= h).astype(float)
    npairs = int(np.sum(phi > 0.0))
    phi = phi * np.outer(w, w)
    return float(np.sum(phi * np.outer(z, z)) / np.sum(phi)), npairs


def _tols(kernel, prec, method, spec_always, oc, on, r_min, n_min, n0):
    """(c tolerance per lag, b tolerance) of one case."""
    oc = np.abs(np.asarray(oc))
    g = min(1.0, r_min)
    if kernel == "rectangle":
        return 1e-9 + 1e-15 * (1.0 + oc) / g, None
    if prec == "mixed":
        btol = ("ref", 2e-6) if method == "auto" else 1e-6
        return np.full(oc.shape, 1e-5), btol
    nsum = max(int(np.max(on)) if np.size(on) else 0, n0)
    if method == "direct":
        return max(1e-11, 4e-16 * nsum) + 1e-15 * (1.0 + oc) / g, max(1e-12, 4e-16 * nsum)
    return 4e-7 + 4e-16 * nsum + 1e-15 * (1.0 + oc) / g, 2e-7


def _status_ok(gst, ost, kernel, prec, r_min, plan=False):
    if gst == ost:
        return True
    # plan execution, mixed Gaussian, small lag-0 scale: not re-evaluated in
    # FP64 but reported (or degenerate where the FP32 lag-0 sum rounds to 0)
    return (plan and kernel == "gaussian" and prec == "mixed" and ost == 0 and
            r_min < 0.11 and gst in (ncf.E_UNSUPPORTED, ncf.E_DEGENERATE))


def _check(what, c, b, n, oc, ob, on, kernel, ctol, btol):
    c, b = np.asarray(c), np.asarray(b)
    assert np.all(np.isfinite(c)), what
    dc = np.abs(c - oc)
    ok = dc <= ctol
    assert np.all(ok), f"{what}: max |dc| = {np.max(dc):.3e} (over the tolerance at {np.sum(~ok)} lags)"
    if kernel == "rectangle":
        np.testing.assert_array_equal(np.asarray(n), on, err_msg=what)
        np.testing.assert_array_equal(b, np.maximum(on.astype(float), 1e-16), err_msg=what)
    elif isinstance(btol, tuple):
        np.testing.assert_allclose(b, ob, rtol=0, atol=btol[1] * np.max(ob), err_msg=what)
    else:
        np.testing.assert_allclose(b, ob, rtol=btol, atol=0, err_msg=what)


def _compare(what, kernel, prec, method, spec_always, got, want, sides, plan=False):
    """got = (c, b, count, status), want = the oracle's (status, c, b, count);
    sides = [(t, x, err), ...] the case's series."""
    c, b, cnt, gst = got
    ost, oc, ob, on = want
    lag0 = [_lag0_r(t, x, h, kernel, e) for (t, x, e, h) in sides]
    r_min = min(r for r, _ in lag0)
    n0 = max(n for _, n in lag0)
    n_min = min(t.size for (t, _, _, _) in sides)
    assert _status_ok(gst, ost, kernel, prec, r_min, plan), (
        f"{what}: status {gst}, oracle {ost} (r_min {r_min:.3e})")
    if plan and kernel == "gaussian" and prec == "mixed" and ost == 0:
        # away from the band around 0.1 the plan's choice is fixed
        if r_min < 0.09:
            assert gst != 0, f"{what}: small lag-0 scale {r_min:.3e} reported as OK"
    if gst == 0 and ost == 0:
        ctol, btol = _tols(kernel, prec, method, spec_always, oc, on, r_min, n_min, n0)
        _check(what, c, b, cnt, oc, ob, on, kernel, ctol, btol)


def _length(rng):
    return int(np.exp(rng.uniform(np.log(2.0), np.log(4000.0))))


@pytest.mark.parametrize("seed", range(40))
def test_random_single_call(seed):
    rng = synth.rng_for(7000 + seed)
    is_ccf = bool(rng.integers(0, 2))
    kernel = ("gaussian", "rectangle")[int(rng.integers(0, 2))]
    pattern = PATTERNS[int(rng.integers(0, len(PATTERNS)))]
    span = rng.uniform(50.0, 5000.0)
    n = _length(rng)
    t, x = _series(rng, n, span, pattern)
    h = span / n * np.exp(rng.uniform(np.log(0.2), np.log(20.0)))
    lags = _lags(rng, span)
    weighted = rng.uniform() < 0.3
    prec, method, spec_always = _mode(rng, kernel, pattern)
    what = (f"seed {seed}: {'ccf' if is_ccf else 'acf'} {kernel} {prec} {method} "
            f"spectral_always={spec_always} {pattern} n={n} K={lags.size} h={h:.4g} "
            f"span={span:.4g} weighted={weighted}")
    print(what, flush=True)
    if is_ccf:
        m = _length(rng)
        s, y = _series(rng, m, span, pattern)
        # errors on both series, or on one only (the other takes unit weights)
        side = ("both", "x", "y")[int(rng.integers(0, 3))] if weighted else None
        ex = rng.uniform(0.5, 2.0, n) if side in ("both", "x") else None
        ey = rng.uniform(0.5, 2.0, m) if side in ("both", "y") else None
        want = O.ccf(t, x, s, y, lags, kernel, h, ex=ex, ey=ey)
        got = ncf.ccf(t, x, s, y, lags, kernel, h, ex=ex, ey=ey, precision=prec, method=method,
                      spectral_always=spec_always, raise_on_error=False)
        sides = [(t, x, ex, h), (s, y, ey, h)]
    else:
        err = rng.uniform(0.5, 2.0, n) if weighted else None
        want = O.acf(t, x, lags, kernel, h, err=err)
        got = ncf.acf(t, x, lags, kernel, h, err=err, precision=prec, method=method,
                      spectral_always=spec_always, raise_on_error=False)
        sides = [(t, x, err, h)]
    # a degenerate draw (e.g. two samples whose standardized values cancel at
    # lag 0) must give the oracle's status
    _compare(what, kernel, prec, method, spec_always, got, want, sides)


def _batch_case(seed):
    rng = synth.rng_for(seed)
    is_ccf = bool(rng.integers(0, 2))
    kernel = ("gaussian", "rectangle")[int(rng.integers(0, 2))]
    pattern = PATTERNS[int(rng.integers(0, len(PATTERNS)))]
    span = rng.uniform(50.0, 2000.0)
    nser = int(rng.integers(1, 17))
    lags = _lags(rng, span)
    prec, method, spec_always = _mode(rng, kernel, pattern)
    sx = [_series(rng, _length(rng), span, pattern) for _ in range(nser)]
    sy = [_series(rng, _length(rng), span, pattern) for _ in range(nser)] if is_ccf else None
    nx = np.array([a[0].size for a in sx])
    h = span / nx * np.exp(rng.uniform(np.log(0.2), np.log(20.0), nser))
    offx = np.concatenate([[0], np.cumsum(nx)]).astype(np.int64)
    d = dict(rng=rng, is_ccf=is_ccf, kernel=kernel, pattern=pattern, nser=nser, lags=lags,
             prec=prec, method=method, spec_always=spec_always, sx=sx, sy=sy, h=h, offx=offx,
             t=np.concatenate([a[0] for a in sx]), x=np.concatenate([a[1] for a in sx]))
    if is_ccf:
        ny = np.array([a[0].size for a in sy])
        d["offy"] = np.concatenate([[0], np.cumsum(ny)]).astype(np.int64)
        d["s"] = np.concatenate([a[0] for a in sy])
        d["y"] = np.concatenate([a[1] for a in sy])
    d["what"] = (f"{'ccf' if is_ccf else 'acf'} batch of {nser} {kernel} {prec} {method} "
                 f"spectral_always={spec_always} {pattern} K={lags.size} "
                 f"lengths={nx.tolist()}")
    return d


def _compare_batch(what, d, out, sx, sy, plan=False):
    """out = (c, b, count, status, rc) of a batch call or plan execution whose
    values are those of sx (and sy)."""
    c, b, cnt, st, rc = out
    st = np.asarray(st)
    # the call's code is the first failing series' status
    bad = np.flatnonzero(st != 0)
    assert rc == (st[bad[0]] if bad.size else 0), what
    kernel, lags, h = d["kernel"], d["lags"], d["h"]
    for i in range(d["nser"]):
        if d["is_ccf"]:
            ost, oc, ob, on = O.ccf(sx[i][0], sx[i][1], sy[i][0], sy[i][1], lags, kernel, h[i])
        else:
            ost, oc, ob, on = O.acf(sx[i][0], sx[i][1], lags, kernel, h[i])
        sides = [(sx[i][0], sx[i][1], None, h[i])]
        if d["is_ccf"]:
            sides.append((sy[i][0], sy[i][1], None, h[i]))
        _compare(f"{what} [series {i}]", kernel, d["prec"], d["method"], d["spec_always"],
                 (c[i], b[i], cnt[i], st[i]), (ost, oc, ob, on), sides, plan)


@pytest.mark.parametrize("seed", range(10))
def test_random_batch(seed):
    d = _batch_case(7100 + seed)
    what = f"seed {seed}: {d['what']}"
    print(what, flush=True)
    kw = dict(precision=d["prec"], method=d["method"], spectral_always=d["spec_always"],
              raise_on_error=False)
    if d["is_ccf"]:
        out = ncf.ccf_batch(d["offx"], d["t"], d["x"], d["offy"], d["s"], d["y"], d["lags"],
                            d["kernel"], d["h"], **kw)
    else:
        out = ncf.acf_batch(d["offx"], d["t"], d["x"], d["lags"], d["kernel"], d["h"], **kw)
    _compare_batch(what, d, out, d["sx"], d["sy"])


@pytest.mark.parametrize("seed", range(10))
def test_random_plan(seed):
    # a plan fixes the times (and the fallback lags); it is executed on the
    # case's values and then on fresh values of the same lengths
    d = _batch_case(7200 + seed)
    graph = bool(d["rng"].integers(0, 2))
    what = f"seed {seed}: plan (graph={graph}) of {d['what']}"
    print(what, flush=True)
    kw = dict(precision=d["prec"], method=d["method"], spectral_always=d["spec_always"],
              graph=graph)
    if d["is_ccf"]:
        plan = ncf.plan_ccf(d["offx"], d["t"], d["offy"], d["s"], d["lags"], d["kernel"],
                            d["h"], **kw)
    else:
        plan = ncf.plan_acf(d["offx"], d["t"], d["lags"], d["kernel"], d["h"], **kw)
    try:
        sx, sy = d["sx"], d["sy"]
        for rep in range(2):
            x = np.concatenate([a[1] for a in sx])
            y = np.concatenate([a[1] for a in sy]) if d["is_ccf"] else None
            out = plan.execute(x, y, raise_on_error=False)
            _compare_batch(f"{what} [execution {rep}]", d, out, sx, sy, plan=True)
            rng = d["rng"]
            sx = [(a[0], rng.normal(size=a[0].size).cumsum() * 0.1 + rng.normal(size=a[0].size))
                  for a in sx]
            if d["is_ccf"]:
                sy = [(a[0], rng.normal(size=a[0].size)) for a in sy]
    finally:
        plan.close()


def _regular_case(seed):
    rng = synth.rng_for(seed)
    is_ccf = bool(rng.integers(0, 2))
    kernel = ("gaussian", "rectangle")[int(rng.integers(0, 2))]
    dt = (1.0, 0.5, 0.1, 0.25, 1.0 / 3.0, 0.01)[int(rng.integers(0, 6))]
    keep = rng.uniform(0.05, 1.0)
    dup = (0.0, 0.05, 0.2)[int(rng.integers(0, 3))]
    t0 = rng.uniform(-100.0, 100.0)
    nser = int(rng.integers(1, 9))
    series = []
    for _ in range(nser * (2 if is_ccf else 1)):
        n = _length(rng)
        t = synth.lattice_times(rng, n, dt=dt, keep=keep, t0=t0, dup_frac=dup)
        t = t + int(rng.integers(0, 50)) * dt  # both series of a pair on one lattice
        series.append((t, rng.normal(size=n).cumsum() * 0.1 + rng.normal(size=n)))
    sx = series[:nser]
    sy = series[nser:] if is_ccf else None
    span = max(max(a[0][-1] - a[0][0] for a in series), dt)
    lags = _lags(rng, span)
    h = dt * np.exp(rng.uniform(np.log(0.3), np.log(20.0), nser))
    return is_ccf, kernel, dt, keep, dup, sx, sy, lags, h


@pytest.mark.parametrize("seed", range(20))
def test_random_regular(seed):
    # lattice family (classic FFT in FP64): c within 1e-9, counts exact,
    # Gaussian b within 1e-10 relative (or the summation bound), plus the
    # near-degenerate scale term; single calls for one series, batches
    # otherwise
    is_ccf, kernel, dt, keep, dup, sx, sy, lags, h = _regular_case(7300 + seed)
    nser = len(sx)
    what = (f"seed {seed}: regular {'ccf' if is_ccf else 'acf'} x{nser} {kernel} dt={dt:.4g} "
            f"keep={keep:.2f} dup={dup} K={lags.size} lengths={[a[0].size for a in sx]}")
    print(what, flush=True)
    if nser == 1:
        if is_ccf:
            c, b, cnt, rc = ncf.ccf_regular(sx[0][0], sx[0][1], sy[0][0], sy[0][1], lags, dt,
                                            kernel, h[0], raise_on_error=False)
        else:
            c, b, cnt, rc = ncf.acf_regular(sx[0][0], sx[0][1], lags, dt, kernel, h[0],
                                            raise_on_error=False)
        c, b, cnt, st = [c], [b], [cnt], [rc]
    else:
        offx = np.concatenate([[0], np.cumsum([a[0].size for a in sx])]).astype(np.int64)
        t = np.concatenate([a[0] for a in sx])
        x = np.concatenate([a[1] for a in sx])
        if is_ccf:
            offy = np.concatenate([[0], np.cumsum([a[0].size for a in sy])]).astype(np.int64)
            c, b, cnt, st, rc = ncf.ccf_regular_batch(
                offx, t, x, offy, np.concatenate([a[0] for a in sy]),
                np.concatenate([a[1] for a in sy]), lags, dt, kernel, h, raise_on_error=False)
        else:
            c, b, cnt, st, rc = ncf.acf_regular_batch(offx, t, x, lags, dt, kernel, h,
                                                      raise_on_error=False)
    for i in range(nser):
        if is_ccf:
            ost, oc, ob, on = O.ccf_regular(sx[i][0], sx[i][1], sy[i][0], sy[i][1], lags, dt,
                                            kernel, h[i])
            sides = [sx[i], sy[i]]
        else:
            ost, oc, ob, on = O.acf_regular(sx[i][0], sx[i][1], lags, dt, kernel, h[i])
            sides = [sx[i]]
        w = f"{what} [series {i}]"
        assert st[i] == ost, f"{w}: status {st[i]}, oracle {ost}"
        if ost != 0:
            continue
        lag0 = [_lag0_r(tt, xx, h[i], kernel) for (tt, xx) in sides]
        g = min(1.0, min(r for r, _ in lag0))
        nsum = max(int(np.max(on)) if on.size else 0, max(n for _, n in lag0))
        ctol = 1e-9 + 1e-15 * (1.0 + np.abs(oc)) / g
        _check(w, c[i], b[i], cnt[i], oc, ob, on, kernel, ctol, max(1e-10, 4e-16 * nsum))


@pytest.mark.parametrize("seed", range(15))
def test_random_resample(seed):
    # replicate family: flux randomization, bootstrap multiplicities or both;
    # every replicate against the oracle's replicate at the tolerances above
    # (the replicate's own lag-0 scale), the returned per-lag mean and sd
    # against those of the returned replicates
    rng = synth.rng_for(7400 + seed)
    is_ccf = bool(rng.integers(0, 2))
    kernel = ("gaussian", "rectangle")[int(rng.integers(0, 2))]
    pattern = PATTERNS[int(rng.integers(0, len(PATTERNS)))]
    span = rng.uniform(50.0, 2000.0)
    scheme = ("flux", "bootstrap", "both")[int(rng.integers(0, 3))]
    prec, method = (("mixed", "auto"), ("fp64", "direct"))[int(rng.integers(0, 2))]
    R = int(rng.integers(2, 25))
    lags = _lags(rng, span)
    sides = []
    for _ in range(2 if is_ccf else 1):
        n = int(np.exp(rng.uniform(np.log(8.0), np.log(2000.0))))
        t, x = _series(rng, n, span, pattern)
        z, mult = synth.resample_draws(rng, n, R, flux=scheme != "bootstrap",
                                       bootstrap=scheme != "flux")
        sigma = rng.uniform(0.1, 0.5, n) if z is not None else None
        err = rng.uniform(0.5, 2.0, n) if rng.uniform() < 0.3 else None
        sides.append(dict(t=t, x=x, z=z, mult=mult, sigma=sigma, err=err))
    h = span / sides[0]["t"].size * np.exp(rng.uniform(np.log(0.5), np.log(20.0)))
    what = (f"seed {seed}: resample {'ccf' if is_ccf else 'acf'} {kernel} {prec} {method} "
            f"{scheme} {pattern} R={R} K={lags.size} n={[d['t'].size for d in sides]}")
    print(what, flush=True)
    X = sides[0]
    if is_ccf:
        Y = sides[1]
        ost, orep, _, _ = O.ccf_resample(X["t"], X["x"], Y["t"], Y["x"], lags, kernel, h,
                                         ex=X["err"], ey=Y["err"], sx=X["sigma"],
                                         sy=Y["sigma"], zx=X["z"], zy=Y["z"],
                                         multx=X["mult"], multy=Y["mult"])
        cm, cs, crep, st, rc = ncf.ccf_resample(
            X["t"], X["x"], Y["t"], Y["x"], lags, kernel, h, ex=X["err"], ey=Y["err"],
            sx=X["sigma"], sy=Y["sigma"], zx=X["z"], zy=Y["z"], multx=X["mult"],
            multy=Y["mult"], R=R, with_reps=True, precision=prec, method=method,
            raise_on_error=False)
    else:
        ost, orep, _, _ = O.acf_resample(X["t"], X["x"], lags, kernel, h, err=X["err"],
                                         sigma=X["sigma"], z=X["z"], mult=X["mult"])
        cm, cs, crep, st, rc = ncf.acf_resample(
            X["t"], X["x"], lags, kernel, h, err=X["err"], sigma=X["sigma"], z=X["z"],
            mult=X["mult"], R=R, with_reps=True, precision=prec, method=method,
            raise_on_error=False)
    st = np.asarray(st)
    if np.all(st == 0):
        assert rc == 0, what
    for r in range(R):
        reps = [O._replicate(d["t"], d["x"], d["err"], d["sigma"], d["z"], d["mult"], r)
                for d in sides]
        lag0 = [_lag0_r(tr, xr, h, kernel, er) for (tr, xr, er) in reps]
        r_min = min(v for v, _ in lag0)
        w = f"{what} [replicate {r}]"
        assert _status_ok(st[r], ost[r], kernel, prec, r_min), (
            f"{w}: status {st[r]}, oracle {ost[r]} (r_min {r_min:.3e})")
        if st[r] != 0 or ost[r] != 0:
            continue
        g = min(1.0, r_min)
        oc = np.abs(orep[r])
        n0 = max(n for _, n in lag0)
        if kernel == "rectangle":
            ctol = 1e-9 + 1e-15 * (1.0 + oc) / g
        elif prec == "mixed":
            ctol = np.full(oc.shape, 1e-5)
        else:
            ctol = max(1e-11, 4e-16 * n0) + 1e-15 * (1.0 + oc) / g
        dc = np.abs(crep[r] - orep[r])
        assert np.all(dc <= ctol), f"{w}: max |dc| = {np.max(dc):.3e}"
        # windows that hold no pair of the replicate (only dropped samples,
        # multiplicity 0): c is exactly 0 on both sides
        assert np.all(crep[r][orep[r] == 0.0] == 0.0), f"{w}: empty window not 0"
    # returned statistics: those of the returned replicates (finite ones)
    ok = np.isfinite(crep)
    for k in range(lags.size):
        col = crep[ok[:, k], k]
        if col.size:
            assert abs(cm[k] - col.mean()) <= 1e-12 * max(1.0, np.max(np.abs(col))), what
        if col.size > 1:
            assert abs(cs[k] - col.std(ddof=1)) <= 1e-12 * max(1.0, np.max(np.abs(col))), what


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
@pytest.mark.parametrize("method", ["auto", "direct"])
def test_window_holding_every_pair_is_degenerate(prec, method):
    # rectangle window wider than a short series: the lag-0 sum (sum of z)^2
    # is 0 up to rounding of either sign; the status is degenerate as in the
    # oracle, for the ACF and for a CCF with such a series on either side
    rng = synth.rng_for(950)
    for n in (2, 3, 7, 40):
        t = np.sort(rng.uniform(0.0, 100.0, n))
        x = rng.normal(size=n)
        s = np.sort(rng.uniform(0.0, 100.0, 50))
        y = rng.normal(size=50)
        lags = np.array([0.0, 5.0])
        c, b, cnt, st = ncf.acf(t, x, lags, "rectangle", 1000.0, precision=prec,
                                method=method, raise_on_error=False)
        assert st == O.E_DEGENERATE and np.all(np.isnan(c)), n
        for a in ((t, x, s, y), (s, y, t, x)):
            c, b, cnt, st = ncf.ccf(*a, lags, "rectangle", 1000.0, precision=prec,
                                    method=method, raise_on_error=False)
            assert st == O.E_DEGENERATE and np.all(np.isnan(c)), n
