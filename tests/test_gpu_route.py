"""NCF_AUTO's choice between the spectral route and the direct window sums
(the paper's K* crossover): small calls take the window sums, large ones the
spectral route, and NCF_SPECTRAL_ALWAYS keeps the spectral route. Whatever
the route, results match the oracle within the mixed-precision tolerance."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_03866_amd import ncf, synth

pytestmark = pytest.mark.gpu


def _route(d, **kw):
    offs = np.array([0, d["t"].size])
    if "s" in d:
        plan = ncf.plan_ccf(offs, d["t"], np.array([0, d["s"].size]), d["s"], d["lags"],
                            "gaussian", d["h"], **kw)
    else:
        plan = ncf.plan_acf(offs, d["t"], d["lags"], "gaussian", d["h"], **kw)
    try:
        return plan.info()["spectral_grids"]
    finally:
        plan.close()


def test_small_acf_takes_the_window_sums():
    d = synth.c1()  # 2000 samples, 101 lags: 2e5 windows
    assert _route(d) == 0
    assert _route(d, spectral_always=True) == 1
    st, oc, ob, on = O.acf(d["t"], d["x"], d["lags"], "gaussian", d["h"])
    c, b, n, _ = ncf.acf(d["t"], d["x"], d["lags"], "gaussian", d["h"])
    assert np.max(np.abs(c - oc)) <= 1e-5
    np.testing.assert_allclose(b, ob, rtol=1e-6)


def test_large_ccf_takes_the_spectral_route():
    d = synth.c2(n=30_000)  # 1.2e7 windows of ~3 samples
    assert _route(d) == 1
    st, oc, ob, on = O.ccf(d["t"], d["x"], d["s"], d["y"], d["lags"][::20], "gaussian", d["h"])
    c, b, n, _ = ncf.ccf(d["t"], d["x"], d["s"], d["y"], d["lags"][::20], "gaussian", d["h"])
    assert np.max(np.abs(c - oc)) <= 1e-5


def _batch_route(d, err, **kw):
    plan = ncf.plan_acf(d["offs"], d["t"], d["lags"], "gaussian", d["h"], err=err, **kw)
    try:
        return plan.info()["spectral_grids"]
    finally:
        plan.close()


def test_weights_over_decades_take_the_window_sums():
    # errors 0.01 x 10^(N(0, 0.5)): weights 1/err^2 over about four decades,
    # whose self-pairs dominate the weighted lag-0 sum B(0); B(tau) < 0.1
    # B(0) at every lag sends the spectral B of such curves to the direct
    # window sums, so they take them from the start. Narrow errors (a factor
    # 4 in weight) keep the spectral route.
    d = synth.c4(seed=41, n_series=32, nmin=2000, nmax=12_000, K=256, with_err=True)
    nser = d["offs"].size - 1
    wide = d["err_values"]
    narrow = np.random.default_rng(42).uniform(0.5, 1.0, wide.size)
    print(f"case: c4 batch of {nser} curves, K=256, wide and narrow error spreads", flush=True)
    assert _batch_route(d, narrow) == nser
    assert _batch_route(d, wide) == 0
    assert _batch_route(d, wide, spectral_always=True) == nser
    c, b, n, st, rc = ncf.acf_batch(d["offs"], d["t"], d["x"], d["lags"], "gaussian", d["h"],
                                    err=wide)
    assert rc == 0
    for i in (0, nser // 2, nser - 1):
        a, e = d["offs"][i], d["offs"][i + 1]
        ost, oc, ob, _ = O.acf(d["t"][a:e], d["x"][a:e], d["lags"], "gaussian", d["h"][i],
                               err=wide[a:e])
        assert ost == st[i] == 0
        assert np.max(np.abs(c[i] - oc)) <= 1e-5, f"curve {i}"
        np.testing.assert_allclose(b[i], ob, rtol=1e-6, err_msg=f"curve {i}")
