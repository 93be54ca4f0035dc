"""GPU parity of the regular-lattice (classic-FFT) estimators against the
oracle's lattice reading.

The GPU route correlates lattice grids with FP64 transforms and filters the
lag sequences; the oracle sums the pairs directly. Tolerances:
  * rectangle counts bit-exact (the count correlation is rounded to integers)
    and b equal to them;
  * Gaussian b relative 1e-10: the GPU multiplies exact integer counts by one
    weight per lattice lag, the oracle adds every pair's weight one at a
    time, so its rounding grows to ~n eps (1e-11 at n = 1e5);
  * c absolute 1e-9: a transform leaves an absolute error of about
    log2(N) eps64 sum(v^2) on every lag correlation, i.e. ~1e-15 n, which a
    lag holding at least one pair divides by its pair sum (>= 1 for the
    rectangle).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_03866_amd import ncf, synth

pytestmark = pytest.mark.gpu

CTOL = 1e-9


def _check(c, b, n, oc, ob, on, kernel):
    c, b = np.asarray(c), np.asarray(b)
    assert np.all(np.isfinite(c))
    err = np.max(np.abs(c - oc)) if c.size else 0.0
    assert err <= CTOL, f"max |dc| = {err:.3e}"
    if kernel == "rectangle":
        np.testing.assert_array_equal(np.asarray(n), on)
        np.testing.assert_array_equal(b, np.maximum(on.astype(float), 1e-16))
    else:
        np.testing.assert_allclose(b, ob, rtol=1e-10, atol=0)


def _lattice_case(seed, n, dt, keep, dup, t0=0.0):
    rng = synth.rng_for(seed)
    t = synth.lattice_times(rng, n, dt=dt, keep=keep, t0=t0, dup_frac=dup)
    x = np.sin(2 * np.pi * t / (37.0 * dt)) + rng.normal(size=n)
    err = rng.uniform(0.5, 2.0, n)
    return rng, t, x, err


LATTICES = [
    # n, dt, keep, duplicates: several fill tiles, a ragged tail, 1- and 2-pass transforms
    (20_000, 0.1, 0.8, 0.05),
    (9_000, 0.25, 1.0, 0.0),
    (700, 1.0 / 3.0, 0.5, 0.1),
]


@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("kernel", ["gaussian", "rectangle"])
@pytest.mark.parametrize("case", range(len(LATTICES)))
def test_acf_regular_parity(case, kernel, weighted):
    n, dt, keep, dup = LATTICES[case]
    rng, t, x, err = _lattice_case(10 + case, n, dt, keep, dup, t0=12.5)
    e = err if weighted else None
    h = 0.6 * dt if kernel == "gaussian" else 1.5 * dt
    span = t[-1] - t[0]
    lags = np.concatenate([np.arange(0, 200) * dt, np.arange(-30, 30) * 0.37 * dt,
                           [span * 0.99, span + 10 * dt, -span - 4 * dt]])
    st, oc, ob, on = O.acf_regular(t, x, lags, dt, kernel, h, err=e)
    assert st == 0
    c, b, cnt, rc = ncf.acf_regular(t, x, lags, dt, kernel, h, err=e)
    assert rc == 0
    _check(c, b, cnt, oc, ob, on, kernel)
    # lags beyond the span hold no pair
    assert c[-2] == 0.0 and b[-2] == 1e-16 and cnt[-2] == 0


@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("kernel", ["gaussian", "rectangle"])
def test_ccf_regular_parity(kernel, weighted):
    dt = 0.1
    rng, t, x, ex = _lattice_case(21, 12_000, dt, 0.85, 0.02, t0=5.0)
    s = synth.lattice_times(rng, 15_000, dt=dt, keep=0.9, t0=3.0, dup_frac=0.02)
    y = np.interp(s - 4.0, t, x) + 0.2 * rng.normal(size=s.size)
    ey = rng.uniform(0.5, 2.0, s.size)
    h = 0.55 * dt if kernel == "gaussian" else 2.0 * dt
    lags = np.concatenate([np.arange(-150, 150) * dt, [0.033, -7.77, 1e4]])
    ex_, ey_ = (ex, ey) if weighted else (None, None)
    st, oc, ob, on = O.ccf_regular(t, x, s, y, lags, dt, kernel, h, ex=ex_, ey=ey_)
    assert st == 0
    c, b, cnt, rc = ncf.ccf_regular(t, x, s, y, lags, dt, kernel, h, ex=ex_, ey=ey_)
    assert rc == 0
    _check(c, b, cnt, oc, ob, on, kernel)
    # the peak of the delayed copy sits at +4 (series 2 lags series 1)
    assert abs(lags[np.argmax(c[:300])] - 4.0) < 0.25


def test_ccf_regular_one_series_weighted():
    dt = 0.25
    rng, t, x, ex = _lattice_case(22, 3000, dt, 0.9, 0.0)
    s = synth.lattice_times(rng, 2500, dt=dt, keep=0.9, t0=1.0)
    y = rng.normal(size=s.size)
    lags = np.arange(-50, 50) * dt
    st, oc, ob, on = O.ccf_regular(t, x, s, y, lags, dt, "rectangle", dt, ex=ex)
    assert st == 0
    c, b, cnt, rc = ncf.ccf_regular(t, x, s, y, lags, dt, "rectangle", dt, ex=ex)
    assert rc == 0
    _check(c, b, cnt, oc, ob, on, "rectangle")


@pytest.mark.parametrize("kernel", ["gaussian", "rectangle"])
def test_acf_regular_batch(kernel):
    d = synth.small("r2", seed=4)
    d["kernel"] = kernel
    offs, t, x, lags = d["offs"], d["t"], d["x"], d["lags"]
    nser = offs.size - 1
    dts = np.where(np.arange(nser) % 3 == 0, 0.5, 1.0)  # two lattice steps in one batch
    tt = t.copy()
    for i in range(nser):
        seg = slice(offs[i], offs[i + 1])
        tt[seg] = t[seg] * dts[i] + 100.0 * i
    hs = 0.5 * dts if kernel == "gaussian" else 1.0 * dts
    c, b, cnt, st, rc = ncf.acf_regular_batch(offs, tt, x, lags, dts, kernel, hs)
    assert rc == 0 and np.all(st == 0)
    for i in range(nser):
        seg = slice(offs[i], offs[i + 1])
        s_, oc, ob, on = O.acf_regular(tt[seg], x[seg], lags, dts[i], kernel, hs[i])
        assert s_ == 0
        _check(c[i], b[i], cnt[i], oc, ob, on, kernel)
        c1, b1, n1, _ = ncf.acf_regular(tt[seg], x[seg], lags, dts[i], kernel, hs[i])
        np.testing.assert_allclose(c1, c[i], rtol=0, atol=1e-14)
        np.testing.assert_array_equal(n1, cnt[i])


def test_ccf_regular_batch_status():
    rng = synth.rng_for(30)
    offx, offy, tx, ty, xs, ys = [0], [0], [], [], [], []
    for i in range(4):
        t = synth.lattice_times(rng, 800 + 300 * i, dt=0.5, keep=0.9)
        s = synth.lattice_times(rng, 900, dt=0.5, keep=0.9, t0=2.0)
        if i == 2:
            s = s + 0.1  # off the common lattice
        tx.append(t)
        ty.append(s)
        xs.append(rng.normal(size=t.size))
        ys.append(rng.normal(size=s.size))
        offx.append(offx[-1] + t.size)
        offy.append(offy[-1] + s.size)
    lags = np.arange(-20, 21) * 0.5
    c, b, cnt, st, rc = ncf.ccf_regular_batch(offx, np.concatenate(tx), np.concatenate(xs), offy,
                                              np.concatenate(ty), np.concatenate(ys), lags, 0.5,
                                              "rectangle", 0.5, raise_on_error=False)
    assert rc == ncf.E_INVALID_ARG
    assert list(st) == [0, 0, ncf.E_INVALID_ARG, 0]
    assert np.all(np.isnan(c[2])) and np.all(cnt[2] == 0)
    for i in (0, 1, 3):
        s_, oc, ob, on = O.ccf_regular(tx[i], xs[i], ty[i], ys[i], lags, 0.5, "rectangle", 0.5)
        _check(c[i], b[i], cnt[i], oc, ob, on, "rectangle")


def test_regular_device_pointers():
    import torch
    rng, t, x, err = _lattice_case(40, 5000, 0.2, 0.9, 0.0)
    lags = np.arange(0, 120) * 0.1
    st, oc, ob, on = O.acf_regular(t, x, lags, 0.2, "gaussian", 0.13)
    dev = torch.device("cuda:0")
    tt = torch.tensor(t, device=dev)
    xt = torch.tensor(x, device=dev)
    lt = torch.tensor(lags, device=dev)
    c, b, cnt, rc = ncf.acf_regular(tt, xt, lt, 0.2, "gaussian", 0.13)
    torch.cuda.synchronize()
    assert rc == 0
    _check(c.cpu().numpy(), b.cpu().numpy(), cnt.cpu().numpy(), oc, ob, on, "gaussian")


def test_regular_edge_cases():
    # two samples; K = 0; four lattice cells holding 40 samples; wide kernel
    t = np.array([0.0, 0.5])
    x = np.array([1.0, -1.0])
    lags = np.array([0.0, 0.5, -0.5, 1.0])
    st, oc, ob, on = O.acf_regular(t, x, lags, 0.5, "rectangle", 0.25)
    c, b, cnt, rc = ncf.acf_regular(t, x, lags, 0.5, "rectangle", 0.25)
    assert rc == 0
    _check(c, b, cnt, oc, ob, on, "rectangle")
    c, b, cnt, rc = ncf.acf_regular(t, x, np.zeros(0), 0.5, "rectangle", 0.25)
    assert rc == 0 and c.size == 0
    t = 3.0 + 0.5 * np.sort(synth.rng_for(2).integers(0, 4, size=40))
    x = synth.rng_for(2).normal(size=40)
    st, oc, ob, on = O.acf_regular(t, x, lags, 0.5, "gaussian", 0.2)
    c, b, cnt, rc = ncf.acf_regular(t, x, lags, 0.5, "gaussian", 0.2)
    assert rc == 0
    _check(c, b, cnt, oc, ob, on, "gaussian")
    rng, t, x, _ = _lattice_case(41, 3000, 0.1, 0.7, 0.0)
    lags = np.linspace(-20, 20, 77)
    st, oc, ob, on = O.acf_regular(t, x, lags, 0.1, "gaussian", 3.0)  # 361 lattice lags
    c, b, cnt, rc = ncf.acf_regular(t, x, lags, 0.1, "gaussian", 3.0)
    assert rc == 0
    _check(c, b, cnt, oc, ob, on, "gaussian")


def test_regular_invalid_args():
    t = np.arange(10) * 0.5
    x = synth.rng_for(3).normal(size=10)
    for dt in (0.0, -0.5, np.inf):
        rc = ncf.acf_regular(t, x, [0.0], dt, "rectangle", 0.5, raise_on_error=False)[3]
        assert rc == ncf.E_INVALID_ARG
    t2 = t.copy()
    t2[3] += 0.1
    rc = ncf.acf_regular(t2, x, [0.0], 0.5, "rectangle", 0.5, raise_on_error=False)[3]
    assert rc == ncf.E_INVALID_ARG
    rc = ncf.acf_regular(t[::-1].copy(), x, [0.0], 0.5, "rectangle", 0.5,
                         raise_on_error=False)[3]
    assert rc == ncf.E_UNSORTED


@pytest.mark.parametrize("kernel", ["gaussian", "rectangle"])
def test_r1_full_size(kernel):
    d = synth.r1(kernel=kernel)
    st, oc, ob, on = O.acf_regular(d["t"], d["x"], d["lags"], d["dt"], kernel, d["h"])
    assert st == 0
    c, b, cnt, rc = ncf.acf_regular(d["t"], d["x"], d["lags"], d["dt"], kernel, d["h"])
    assert rc == 0
    _check(c, b, cnt, oc, ob, on, kernel)


# ------------------------------------------------------------------ plans

@pytest.mark.parametrize("graph", [True, False])
@pytest.mark.parametrize("kernel", ["gaussian", "rectangle"])
def test_regular_plan_replays(kernel, graph):
    d = synth.small("r2", seed=9)
    offs, t, lags = d["offs"], d["t"], d["lags"]
    hs = 0.5 if kernel == "gaussian" else 1.0
    plan = ncf.plan_acf_regular(offs, t, lags, 1.0, kernel, hs, graph=graph)
    try:
        info = plan.info()
        assert info["graph"] == (1 if graph else 0) and info["spectral_grids"] == offs.size - 1
        rng = synth.rng_for(1)
        for rep in range(3):  # new values each execution
            x = rng.normal(size=t.size)
            c, b, cnt, st, rc = plan.execute(x)
            assert rc == 0 and np.all(st == 0)
            c1, b1, n1, st1, _ = ncf.acf_regular_batch(offs, t, x, lags, 1.0, kernel, hs)
            np.testing.assert_allclose(c, c1, rtol=0, atol=1e-14)
            np.testing.assert_array_equal(b, b1)
            np.testing.assert_array_equal(cnt, n1)
            if rep == 0:
                for i in (0, offs.size - 2):
                    seg = slice(offs[i], offs[i + 1])
                    _, oc, ob, on = O.acf_regular(t[seg], x[seg], lags, 1.0, kernel, hs)
                    _check(c[i], b[i], cnt[i], oc, ob, on, kernel)
    finally:
        plan.close()


def test_regular_ccf_plan_status_and_autotune():
    rng = synth.rng_for(31)
    offx, offy, tx, ty = [0], [0], [], []
    for i in range(3):
        t = synth.lattice_times(rng, 3000 + 2000 * i, dt=0.5, keep=0.9)
        s = synth.lattice_times(rng, 4000, dt=0.5, keep=0.9, t0=1.5)
        if i == 1:
            s = s + 0.2  # off the common lattice
        tx.append(t)
        ty.append(s)
        offx.append(offx[-1] + t.size)
        offy.append(offy[-1] + s.size)
    TX, TY = np.concatenate(tx), np.concatenate(ty)
    lags = np.arange(-100, 101) * 0.5
    plan = ncf.plan_ccf_regular(offx, TX, offy, TY, lags, 0.5, "gaussian", 0.3, autotune=True)
    try:
        assert plan.info()["autotuned"] == 1
        x = rng.normal(size=TX.size)
        y = rng.normal(size=TY.size)
        c, b, cnt, st, rc = plan.execute(x, y, raise_on_error=False)
        assert rc == ncf.E_INVALID_ARG and list(st) == [0, ncf.E_INVALID_ARG, 0]
        for i in (0, 2):
            xs = x[offx[i]:offx[i + 1]]
            ys = y[offy[i]:offy[i + 1]]
            _, oc, ob, on = O.ccf_regular(tx[i], xs, ty[i], ys, lags, 0.5, "gaussian", 0.3)
            _check(c[i], b[i], cnt[i], oc, ob, on, "gaussian")
    finally:
        plan.close()
