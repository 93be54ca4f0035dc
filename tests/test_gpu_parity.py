"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle.

Tolerances (|delta c| absolute per lag, b relative):
  * mixed precision, Gaussian, spectral numerator and pair count: c 1e-5,
    |delta b| <= 1e-5 b_ref (b_ref = the largest pair count of the call;
    the fallback rule's own reference is b(0) for the ACF and
    sqrt(b_xx(0) b_yy(0)) for the CCF, both at least as large):
    the FP32 transforms leave an absolute error of about log2(N) eps32 b_ref
    on every lag, and lags with b < 0.1 b_ref are summed directly (FP64:
    b < 1e-2 b_ref);
  * mixed precision with the window-scan pair count: c 1e-5, b 1e-6;
  * FP64 spectral numerator and pair count: c 5e-8, b 2e-8 -- the spectral
    sums have no 6h window truncation, the oracle's do; the Gaussian mass
    beyond 6h is erfc(3 sqrt 2) ~ 2e-9 of the total (x10 margin for uneven
    sampling density);
  * FP64 direct window sums: c 1e-11, b 1e-12;
  * rectangle: counts bit-exact, c 1e-9 (FP64 prefix sums).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_03866_amd import ncf, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _spectral_route(monkeypatch):
    """NCF_AUTO here always takes the spectral route (NCF_SPECTRAL_ALWAYS), so
    these small cases test it; the automatic choice of the direct window sums
    for small calls is tested in test_gpu_route.py."""
    orig = ncf._options

    def opts(*a, **k):
        o = orig(*a, **k)
        o.flags |= ncf.SPECTRAL_ALWAYS
        return o

    monkeypatch.setattr(ncf, "_options", opts)



def _orc_acf(d, lags=None, kernel=None, err=None, h=None):
    lags = d["lags"] if lags is None else lags
    st, c, b, n = O.acf(d["t"], d["x"], lags, kernel or d["kernel"], d["h"] if h is None else h,
                        err=err if err is not None else d.get("err"))
    assert st == 0
    return c, b, n


def _orc_ccf(d, lags=None, kernel=None):
    lags = d["lags"] if lags is None else lags
    st, c, b, n = O.ccf(d["t"], d["x"], d["s"], d["y"], lags, kernel or d["kernel"], d["h"],
                        ex=d.get("ex"), ey=d.get("ey"))
    assert st == 0
    return c, b, n


def _check(c, b, n, oc, ob, on, kernel, ctol, btol):
    c, b = np.asarray(c), np.asarray(b)
    assert np.all(np.isfinite(c))
    err = np.max(np.abs(c - oc))
    assert err <= ctol, f"max |dc| = {err:.3e} > {ctol:.1e}"
    if kernel == "rectangle":
        np.testing.assert_array_equal(np.asarray(n), on)
        np.testing.assert_array_equal(b, np.maximum(on.astype(float), 1e-16))
    elif isinstance(btol, tuple):  # ("ref", tol): relative to the largest pair count
        np.testing.assert_allclose(b, ob, rtol=0, atol=btol[1] * np.max(ob))
    else:
        np.testing.assert_allclose(b, ob, rtol=btol, atol=0)


MODES = [
    ("mixed", "auto", 1e-5, ("ref", 2e-6)),
    ("fp64", "auto", 5e-8, 2e-8),
    ("fp64", "direct", 1e-11, 1e-12),
    ("mixed", "direct", 1e-5, 1e-6),
    ("mixed", "spectral", 1e-5, 1e-6),   # spectral numerator, window-scan pair count
    ("fp64", "spectral", 5e-8, 1e-12),
]


@pytest.mark.parametrize("prec,method,ctol,btol", MODES)
@pytest.mark.parametrize("name", ["c1", "c3"])
def test_acf_gaussian_small(name, prec, method, ctol, btol):
    d = synth.small(name, seed=7)
    oc, ob, on = _orc_acf(d)
    c, b, n, _ = ncf.acf(d["t"], d["x"], d["lags"], "gaussian", d["h"], precision=prec,
                         method=method)
    _check(c, b, n, oc, ob, on, "gaussian", ctol, btol)


@pytest.mark.parametrize("prec,method,ctol,btol", MODES)
def test_ccf_gaussian_small(prec, method, ctol, btol):
    d = synth.small("c2", seed=3)
    oc, ob, on = _orc_ccf(d, kernel="gaussian")
    c, b, n, _ = ncf.ccf(d["t"], d["x"], d["s"], d["y"], d["lags"], "gaussian", d["h"],
                         precision=prec, method=method)
    _check(c, b, n, oc, ob, on, "gaussian", ctol, btol)


@pytest.mark.parametrize("method", ["auto", "direct"])
def test_rectangle_acf_ccf_small(method):
    d = synth.small("c2", seed=4)
    oc, ob, on = _orc_ccf(d, kernel="rectangle")
    c, b, n, _ = ncf.ccf(d["t"], d["x"], d["s"], d["y"], d["lags"], "rectangle", d["h"],
                         method=method)
    _check(c, b, n, oc, ob, on, "rectangle", 1e-9, 0)
    d1 = synth.small("c1", seed=5)
    lags = np.linspace(-30.0, 30.0, 97)
    oc, ob, on = _orc_acf(d1, lags=lags, kernel="rectangle", h=0.5)
    c, b, n, _ = ncf.acf(d1["t"], d1["x"], lags, "rectangle", 0.5, method=method)
    _check(c, b, n, oc, ob, on, "rectangle", 1e-9, 0)


def test_ties_negative_repeated_unsorted_lags():
    rng = np.random.default_rng(17)
    t = np.sort(np.round(rng.uniform(0, 500, 1500) * 4) / 4)  # quarter-day grid: many ties
    x = rng.normal(size=t.size).cumsum()
    lags = np.array([3.25, -7.5, 0.0, 3.25, 100.0, -0.25, 12.0, 480.0, 900.0])
    for kern, h in (("rectangle", 0.5), ("gaussian", 0.4)):
        st, oc, ob, on = O.acf(t, x, lags, kern, h)
        for prec in ("mixed", "fp64"):
            c, b, n, _ = ncf.acf(t, x, lags, kern, h, precision=prec)
            _check(c, b, n, oc, ob, on, kern, 1e-5 if prec == "mixed" else 5e-8, 1e-6)
        # lag 900 is beyond the data: empty window -> c = 0, b = 1e-16
        assert b[-1] == 1e-16 and c[-1] == 0.0


def test_weighted_mode_matches_oracle():
    # Gaussian with errors: spectral numerator, weighted pair sum B (weights
    # channel) and unweighted b (unit channel), direct fallback where B is
    # small; tolerances of the unweighted auto path
    d = synth.small("c4", seed=2)
    i0, i1 = d["offs"][3], d["offs"][4]
    t, x, e = d["t"][i0:i1], d["x"][i0:i1], d["err_values"][i0:i1]
    lags = np.arange(40.0)
    for kern in ("gaussian", "rectangle"):
        st, oc, ob, on = O.acf(t, x, lags, kern, 0.5, err=e)
        assert st == 0
        for prec, ctol, btol in (("mixed", 1e-5, ("ref", 2e-6)), ("fp64", 5e-8, 2e-8)):
            c, b, n, _ = ncf.acf(t, x, lags, kern, 0.5, err=e, precision=prec)
            if kern == "rectangle":
                ctol = 1e-9
            _check(c, b, n, oc, ob, on, kern, ctol, btol)


@pytest.mark.parametrize("prec,ctol,btol", [("mixed", 1e-5, ("ref", 2e-6)),
                                            ("fp64", 5e-8, 2e-8)])
@pytest.mark.parametrize("which", ["both", "x", "y"])
def test_weighted_ccf_gaussian(which, prec, ctol, btol):
    d = synth.small("c2", seed=5)
    rng = synth.rng_for(6)
    ex = rng.uniform(0.5, 2.0, d["t"].size) if which in ("both", "x") else None
    ey = rng.uniform(0.5, 2.0, d["s"].size) if which in ("both", "y") else None
    st, oc, ob, on = O.ccf(d["t"], d["x"], d["s"], d["y"], d["lags"], "gaussian", d["h"],
                           ex=ex, ey=ey)
    assert st == 0
    c, b, n, _ = ncf.ccf(d["t"], d["x"], d["s"], d["y"], d["lags"], "gaussian", d["h"], ex=ex,
                         ey=ey, precision=prec)
    _check(c, b, n, oc, ob, on, "gaussian", ctol, btol)


def test_weighted_batch_gaussian():
    d = synth.small("c4", seed=3)
    offs, t, x, e = d["offs"], d["t"], d["x"], d["err_values"]
    lags = d["lags"]
    c, b, n, st, rc = ncf.acf_batch(offs, t, x, lags, "gaussian", d["h"], err=e)
    assert rc == 0
    for i in range(offs.size - 1):
        sl = slice(offs[i], offs[i + 1])
        s_, oc, ob, on = O.acf(t[sl], x[sl], lags, "gaussian", d["h"][i], err=e[sl])
        assert s_ == 0
        _check(c[i], b[i], n[i], oc, ob, on, "gaussian", 1e-5, ("ref", 2e-6))


def test_status_codes_on_gpu():
    t = np.arange(50.0)
    x = np.sin(t)
    lags = np.arange(5.0)
    assert ncf.acf(t[::-1].copy(), x, lags, "g", 0.5, raise_on_error=False)[3] == ncf.E_UNSORTED
    xb = x.copy()
    xb[7] = np.inf
    assert ncf.acf(t, xb, lags, "g", 0.5, raise_on_error=False)[3] == ncf.E_INVALID_ARG
    assert ncf.acf(t, np.ones(50), lags, "g", 0.5, raise_on_error=False)[3] == ncf.E_DEGENERATE
    assert ncf.acf(t, x, lags, "g", -1.0, raise_on_error=False)[3] == ncf.E_INVALID_ARG
    c, b, n, rc = ncf.acf(t, x, np.zeros(0), "g", 0.5)
    assert rc == 0 and c.size == 0


def test_batch_acf_small_matches_per_series_oracle():
    d = synth.small("c4", seed=9)
    offs = d["offs"]
    c, b, n, st, rc = ncf.acf_batch(offs, d["t"], d["x"], d["lags"], "gaussian", d["h"])
    assert rc == 0 and np.all(st == 0)
    for i in range(len(offs) - 1):
        sl = slice(offs[i], offs[i + 1])
        s2, oc, ob, on = O.acf(d["t"][sl], d["x"][sl], d["lags"], "gaussian", d["h"][i])
        _check(c[i], b[i], n[i], oc, ob, on, "gaussian", 1e-5, 1e-6)


def test_batch_ccf_small_rectangle_exact_counts():
    d = synth.small("c5", seed=9)
    c, b, n, st, rc = ncf.ccf_batch(d["offx"], d["t"], d["x"], d["offy"], d["s"], d["y"],
                                    d["lags"], "rectangle", d["h"])
    assert rc == 0 and np.all(st == 0)
    for p in range(len(d["offx"]) - 1):
        sx = slice(d["offx"][p], d["offx"][p + 1])
        sy = slice(d["offy"][p], d["offy"][p + 1])
        s2, oc, ob, on = O.ccf(d["t"][sx], d["x"][sx], d["s"][sy], d["y"][sy], d["lags"],
                               "rectangle", d["h"][p])
        _check(c[p], b[p], n[p], oc, ob, on, "rectangle", 1e-9, 0)


def test_batch_with_a_bad_series_reports_per_series_status():
    d = synth.small("c4", seed=11)
    x = d["x"].copy()
    x[d["offs"][2]:d["offs"][3]] = 1.0  # constant series
    c, b, n, st, rc = ncf.acf_batch(d["offs"], d["t"], x, d["lags"], "gaussian", d["h"],
                                    raise_on_error=False)
    assert rc == ncf.E_DEGENERATE and st[2] == ncf.E_DEGENERATE
    assert np.all(np.isnan(c[2])) and np.sum(st != 0) == 1
    i0, i1 = d["offs"][0], d["offs"][1]
    s2, oc, ob, on = O.acf(d["t"][i0:i1], x[i0:i1], d["lags"], "gaussian", d["h"][0])
    _check(c[0], b[0], n[0], oc, ob, on, "gaussian", 1e-5, 1e-6)


def test_device_pointer_mode_with_torch_tensors():
    import torch
    d = synth.small("c2", seed=5)
    dev = torch.device("cuda:0")
    tt = {k: torch.as_tensor(d[k], device=dev) for k in ("t", "x", "s", "y", "lags")}
    c, b, n, _ = ncf.ccf(tt["t"], tt["x"], tt["s"], tt["y"], tt["lags"], "gaussian", d["h"])
    torch.cuda.synchronize()
    oc, ob, on = _orc_ccf(d, kernel="gaussian")
    _check(c.cpu().numpy(), b.cpu().numpy(), n.cpu().numpy(), oc, ob, on, "gaussian", 1e-5, 1e-6)


@pytest.mark.parametrize("prec,method,ctol,btol", MODES)
def test_sparse_lags_take_the_direct_fallback(prec, method, ctol, btol):
    # a short seasonal light curve whose lag grid reaches its span: some lags
    # hold only a few far-tail pairs (b/b0 down to ~1e-6), where a spectral
    # value alone would be dominated by rounding noise
    rng = synth.rng_for(35)
    t = synth.seasonal_epochs(rng, 130, phase=0.0)
    x = synth.ou_at_times(rng, t, 8.0) + 0.3 * rng.standard_normal(t.size)
    lags = np.arange(0.0, 256.0)
    st, oc, ob, on = O.acf(t, x, lags, "gaussian", 0.5)
    nonempty = ob > 1e-16
    assert st == 0 and np.min(ob[nonempty] / ob[0]) < 1e-9 and not np.all(nonempty)
    c, b, n, _ = ncf.acf(t, x, lags, "gaussian", 0.5, precision=prec, method=method)
    _check(c, b, n, oc, ob, on, "gaussian", ctol, btol)


@pytest.mark.parametrize("prec,method,ctol,btol", MODES)
def test_batch_fallback_sets_differ_per_series(prec, method, ctol, btol):
    # the fallback lags are flagged per series on the device (one bit per
    # lag row, 64 rows to a word): series of different spans flag different
    # lag sets, among them sets that start and end inside a word and span
    # several words (200 lags: 4 words)
    rng = synth.rng_for(36)
    ts, xs = [], []
    for span_frac in (0.25, 0.6, 1.0, 0.4):
        t = np.sort(rng.uniform(0.0, 200.0 * span_frac, int(300 * span_frac) + 40))
        ts.append(t)
        xs.append(synth.ou_at_times(rng, t, 6.0) + 0.2 * rng.standard_normal(t.size))
    offs = np.concatenate([[0], np.cumsum([t.size for t in ts])])
    lags = np.arange(0.0, 200.0)
    c, b, n, st, rc = ncf.acf_batch(offs, np.concatenate(ts), np.concatenate(xs), lags,
                                    "gaussian", 0.5, precision=prec, method=method)
    assert rc == 0 and np.all(st == 0)
    for i, (t, x) in enumerate(zip(ts, xs)):
        ost, oc, ob, on = O.acf(t, x, lags, "gaussian", 0.5)
        assert ost == 0
        _check(c[i], b[i], n[i], oc, ob, on, "gaussian", ctol, btol)


@pytest.mark.parametrize("prec,method,ctol,btol", MODES)
def test_ccf_with_partly_empty_lags(prec, method, ctol, btol):
    # series 2 covers only part of series 1's span: lags beyond the overlap
    # have no pairs at all, lags at its edge only a few
    rng = synth.rng_for(77)
    t = np.sort(rng.uniform(0.0, 300.0, 900))
    x = rng.standard_normal(t.size).cumsum()
    s_ = np.sort(rng.uniform(200.0, 260.0, 250))
    y = rng.standard_normal(s_.size).cumsum()
    lags = np.linspace(-320.0, 120.0, 177)
    st, oc, ob, on = O.ccf(t, x, s_, y, lags, "gaussian", 0.6)
    assert st == 0 and np.any(ob == 1e-16)
    c, b, n, _ = ncf.ccf(t, x, s_, y, lags, "gaussian", 0.6, precision=prec, method=method)
    _check(c, b, n, oc, ob, on, "gaussian", ctol, btol)


def test_results_are_deterministic():
    d = synth.small("c3", seed=1)
    r1 = ncf.acf(d["t"], d["x"], d["lags"], "gaussian", d["h"])
    r2 = ncf.acf(d["t"], d["x"], d["lags"], "gaussian", d["h"])
    np.testing.assert_array_equal(r1[0], r2[0])
    np.testing.assert_array_equal(r1[1], r2[1])


# ------------------------------------------------------- stage-level pins

@pytest.mark.parametrize("p", [12, 15, 21, 23])
@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_fft_against_numpy(p, prec):
    N = 2 ** p
    rng = np.random.default_rng(p)
    x = rng.normal(size=N) + 1j * rng.normal(size=N)
    want_p = np.fft.ifft(x) * N  # sum x exp(+2 pi i n k / N)
    want_m = np.fft.fft(x)       # sum x exp(-2 pi i n k / N)
    # relative L2 error, and every element against the RMS of the output (a
    # wrong twiddle or index shows in a few elements before the norm)
    tol, tol_el = (5e-7, 4e-6) if prec == "mixed" else (1e-14, 5e-14)
    for sign, want in ((+1, want_p), (-1, want_m)):
        got = ncf.diag_fft(x, sign, prec)
        rel = np.linalg.norm(got - want) / np.linalg.norm(want)
        assert rel < tol, (sign, rel)
        el = np.max(np.abs(got - want)) / (np.linalg.norm(want) / np.sqrt(N))
        assert el < tol_el, (sign, el)


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_type1_against_direct_dft(prec):
    rng = np.random.default_rng(3)
    n, L, N, M = 700, 1000.0, 8192, 2600
    t = np.sort(rng.uniform(20.0, 980.0, n))
    v = rng.normal(size=n)
    got = ncf.diag_type1(t, v, 0.0, L, N, M, prec)
    m = np.arange(-M, M + 1)
    want = np.exp(2j * np.pi * np.outer(m, t) / L) @ v
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert rel < (2e-6 if prec == "mixed" else 1e-11), rel
    el = np.max(np.abs(got - want)) / (np.linalg.norm(want) / np.sqrt(want.size))
    assert el < (3e-5 if prec == "mixed" else 3e-10), el


# ------------------------------------------- full-size, bench configuration

def test_c2_full_size_ccf_both_kernels():
    for kern in ("gaussian", "rectangle"):
        d = synth.c2(kernel=kern)
        oc, ob, on = _orc_ccf(d)
        c, b, n, _ = ncf.ccf(d["t"], d["x"], d["s"], d["y"], d["lags"], kern, d["h"])
        _check(c, b, n, oc, ob, on, kern, 1e-5 if kern == "gaussian" else 1e-9, 1e-6)
        # the delay of the response (40 d) is recovered
        assert abs(d["lags"][np.argmax(c)] - 40.0) <= 3.0


def test_c1_full_size_both_precisions():
    d = synth.c1()
    oc, ob, on = _orc_acf(d)
    for prec, method, ctol, btol in MODES:
        c, b, n, _ = ncf.acf(d["t"], d["x"], d["lags"], "gaussian", d["h"], precision=prec,
                             method=method)
        _check(c, b, n, oc, ob, on, "gaussian", ctol, btol)


def test_c3_full_size_sampled_lags():
    # 1e7 samples, 4,096 lags: the mixed-precision product path and the
    # all-FP64 spectral path (complex128 grids), each on 64 evenly spaced
    # lags plus the sinusoids' periods, in one call over all 4,096 lags
    d = synth.c3()
    pick = np.unique(np.concatenate([np.linspace(0, 4095, 64).round().astype(int),
                                     [1, 2, 7, 31, 365]]))
    oc, ob, on = _orc_acf(d, lags=d["lags"][pick])
    c, b, n, _ = ncf.acf(d["t"], d["x"], d["lags"], "gaussian", d["h"])
    _check(c[pick], b[pick], n[pick], oc, ob, on, "gaussian", 1e-5, 1e-6)
    c, b, n, _ = ncf.acf(d["t"], d["x"], d["lags"], "gaussian", d["h"], precision="fp64")
    _check(c[pick], b[pick], n[pick], oc, ob, on, "gaussian", 5e-8, 2e-8)


@pytest.mark.parametrize("side", ["x", "y"])
@pytest.mark.parametrize("kernel,prec,method,ctol,btol", [
    ("rectangle", "mixed", "auto", 1e-9, 0),
    ("rectangle", "fp64", "direct", 1e-9, 0),
    ("gaussian", "mixed", "direct", 1e-5, 1e-6),
    ("gaussian", "fp64", "direct", 1e-11, 1e-12),
    ("gaussian", "mixed", "auto", 1e-5, ("ref", 2e-6)),
])
def test_ccf_weights_on_one_side(side, kernel, prec, method, ctol, btol):
    # errors on one series only: the other takes unit weights in the pair
    # weight w_i w_j, on every route (the window passes read both series'
    # weights and weight prefix sums)
    d = synth.small("c2", seed=8)
    rng = synth.rng_for(9)
    ex = rng.uniform(0.5, 2.0, d["t"].size) if side == "x" else None
    ey = rng.uniform(0.5, 2.0, d["s"].size) if side == "y" else None
    h = d["h"] if kernel == "gaussian" else 0.5
    st, oc, ob, on = O.ccf(d["t"], d["x"], d["s"], d["y"], d["lags"], kernel, h, ex=ex, ey=ey)
    assert st == 0
    c, b, n, s = ncf.ccf(d["t"], d["x"], d["s"], d["y"], d["lags"], kernel, h, ex=ex, ey=ey,
                         precision=prec, method=method)
    assert s == 0
    _check(c, b, n, oc, ob, on, kernel, ctol, btol)


@pytest.mark.parametrize("weighted", [False, True])
def test_rectangle_dense_burst_global_window_path(weighted):
    # a burst of 4,000 samples within one day in a 7,000-sample series: the
    # windows of the outer samples near it hold more samples than the LDS
    # stage, so the scan reads the window arrays from global memory, and the
    # burst spans several prefix chunks (2,048 samples each) whose offsets
    # are added on that path too; exact counts against the oracle
    rng = np.random.default_rng(77)
    t = np.sort(np.concatenate([rng.uniform(0.0, 1000.0, 3000), rng.uniform(500.0, 501.0, 4000)]))
    s = np.sort(rng.uniform(0.0, 1000.0, 2000))
    x = rng.standard_normal(t.size)
    y = rng.standard_normal(s.size)
    lags = np.linspace(-20.0, 20.0, 81)
    ex = 10.0 ** rng.uniform(-1.5, 0.0, t.size) if weighted else None
    ey = 10.0 ** rng.uniform(-1.5, 0.0, s.size) if weighted else None
    print(f"case: rectangle burst CCF/ACF, weighted={weighted}", flush=True)
    st, oc, ob, on = O.ccf(t, x, s, y, lags, "rectangle", 0.5, ex=ex, ey=ey)
    assert st == 0
    c, b, n, _ = ncf.ccf(t, x, s, y, lags, "rectangle", 0.5, ex=ex, ey=ey)
    _check(c, b, n, oc, ob, on, "rectangle", 1e-9, 0)
    st, oc, ob, on = O.acf(t, x, lags[40:], "rectangle", 0.5, err=ex)
    assert st == 0
    c, b, n, _ = ncf.acf(t, x, lags[40:], "rectangle", 0.5, err=ex)
    _check(c, b, n, oc, ob, on, "rectangle", 1e-9, 0)
