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
