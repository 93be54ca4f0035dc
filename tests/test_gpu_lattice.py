"""Lags on a lattice: the lag sum read off the spectrum folded modulo P.

When every evaluation lag is a whole multiple of one unit, the period L is
chosen as P units and the type-2 step (eq. nufft_type2) at the lags becomes
a P-point DFT of the spectrum folded modulo P, with no inverse transform of
the full grid and no interpolation. These tests check that route against
the oracle and against the interpolating route on the same inputs (a lag
list that breaks the lattice forces interpolation), in both precisions, for
single calls, batches and plans, and that plan_info reports which route ran.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_03866_amd import ncf, synth

pytestmark = pytest.mark.gpu

OFF = math.sqrt(2.0) * 0.37  # not a rational multiple of the lattice unit


def _lattice_grids(d, lags, **kw):
    offs = np.array([0, d["t"].size])
    if "s" in d:
        plan = ncf.plan_ccf(offs, d["t"], np.array([0, d["s"].size]), d["s"], lags,
                            "gaussian", d["h"], **kw)
    else:
        plan = ncf.plan_acf(offs, d["t"], lags, "gaussian", d["h"], **kw)
    try:
        info = plan.info()
        return info["lattice_grids"], info["spectral_grids"]
    finally:
        plan.close()


def _check_b(b, ob, precision):
    if precision == "mixed":  # spectral pair count: relative to the largest
        np.testing.assert_allclose(b, ob, rtol=0, atol=2e-6 * np.max(ob))
    else:
        np.testing.assert_allclose(b, ob, rtol=2e-8, atol=0)


def test_ccf_lattice_matches_oracle_and_interpolation():
    d = synth.c2(seed=21, n=20_000)
    lags = d["lags"][::4]  # -200 .. 200 step 4 d
    print(f"case: c2 n=2e4 CCF, {lags.size} lattice lags, mixed", flush=True)
    assert _lattice_grids(d, lags, spectral_always=True) == (1, 1)
    odd = np.concatenate([lags, [OFF]])
    assert _lattice_grids(d, odd, spectral_always=True) == (0, 1)
    c, b, _, _ = ncf.ccf(d["t"], d["x"], d["s"], d["y"], lags, "gaussian", d["h"],
                         spectral_always=True)
    ci, bi, _, _ = ncf.ccf(d["t"], d["x"], d["s"], d["y"], odd, "gaussian", d["h"],
                           spectral_always=True)
    st, oc, ob, _ = O.ccf(d["t"], d["x"], d["s"], d["y"], lags, "gaussian", d["h"])
    assert st == 0
    assert np.max(np.abs(c - oc)) <= 1e-5
    assert np.max(np.abs(ci[:-1] - oc)) <= 1e-5
    # the two evaluations of the same spectral sums agree to the transforms' rounding
    assert np.max(np.abs(c - ci[:-1])) <= 1e-5
    _check_b(b, ob, "mixed")
    _check_b(bi[:-1], ob, "mixed")


@pytest.mark.parametrize("precision,tol_c", [("mixed", 1e-5), ("fp64", 5e-8)])
def test_acf_lattice_matches_oracle_and_interpolation(precision, tol_c):
    d = synth.c2(seed=25, n=20_000)
    d = {"t": d["t"], "x": d["x"], "h": 0.5}
    lags = np.arange(0.0, 201.0, 2.0)
    print(f"case: ACF n=2e4, {lags.size} lattice lags, {precision}", flush=True)
    assert _lattice_grids(d, lags, spectral_always=True, precision=precision) == (1, 1)
    odd = np.concatenate([lags, [OFF]])
    assert _lattice_grids(d, odd, spectral_always=True, precision=precision) == (0, 1)
    c, b, _, _ = ncf.acf(d["t"], d["x"], lags, "gaussian", 0.5, precision=precision,
                         spectral_always=True)
    ci, bi, _, _ = ncf.acf(d["t"], d["x"], odd, "gaussian", 0.5, precision=precision,
                           spectral_always=True)
    st, oc, ob, _ = O.acf(d["t"], d["x"], lags, "gaussian", 0.5)
    assert st == 0
    assert np.max(np.abs(c - oc)) <= tol_c
    assert np.max(np.abs(c - ci[:-1])) <= tol_c
    _check_b(b, ob, precision)


def test_acf_lattice_negative_unsorted_and_repeated_lags():
    d = synth.c2(seed=22, n=12_000)
    d = {"t": d["t"], "x": d["x"], "h": 0.5}
    rng = np.random.default_rng(5)
    lags = rng.integers(-150, 151, size=90).astype(np.float64)
    lags[:3] = [7.0, 7.0, -7.0]
    print("case: ACF n=1.2e4, 90 random integer lags (repeats, negatives), mixed", flush=True)
    assert _lattice_grids(d, lags, spectral_always=True)[0] == 1
    c, b, _, _ = ncf.acf(d["t"], d["x"], lags, "gaussian", 0.5, spectral_always=True)
    st, oc, ob, _ = O.acf(d["t"], d["x"], lags, "gaussian", 0.5)
    assert st == 0
    assert np.max(np.abs(c - oc)) <= 1e-5
    assert c[0] == c[1] and abs(c[0] - c[2]) <= 1e-6  # acf is even
    _check_b(b, ob, "mixed")


def test_half_unit_lattice_of_an_even_symmetric_linspace():
    # linspace(-300, 300, 128): lags are odd multiples of half the spacing
    d = synth.c2(seed=23, n=15_000)
    lags = np.linspace(-300.0, 300.0, 128)
    print("case: c2 n=1.5e4 CCF, linspace(-300, 300, 128), mixed", flush=True)
    assert _lattice_grids(d, lags, spectral_always=True)[0] == 1
    c, b, _, _ = ncf.ccf(d["t"], d["x"], d["s"], d["y"], lags, "gaussian", d["h"],
                         spectral_always=True)
    st, oc, ob, _ = O.ccf(d["t"], d["x"], d["s"], d["y"], lags, "gaussian", d["h"])
    assert st == 0
    assert np.max(np.abs(c - oc)) <= 1e-5
    _check_b(b, ob, "mixed")


def test_single_tile_grid_and_batch_with_plans():
    # short curves (grids of one 4096-cell tile) and long ones in one batch
    d = synth.small("c4", seed=24)
    offs, lags, h = d["offs"], d["lags"], d["h"]
    print(f"case: c4-small batch of {offs.size - 1} curves, {lags.size} lags, mixed", flush=True)
    c, b, _, st, _ = ncf.acf_batch(offs, d["t"], d["x"], lags, "gaussian", h,
                                   spectral_always=True)
    assert np.all(st == 0)
    plan = ncf.plan_acf(offs, d["t"], lags, "gaussian", h, spectral_always=True)
    try:
        assert plan.info()["lattice_grids"] > 0
        cp, bp, _, stp = plan.execute(d["x"])[:4]
    finally:
        plan.close()
    assert np.max(np.abs(cp - c)) <= 1e-6
    for i in range(offs.size - 1):
        sl = slice(offs[i], offs[i + 1])
        so, oc, ob, _ = O.acf(d["t"][sl], d["x"][sl], lags, "gaussian", h[i])
        assert so == 0
        assert np.max(np.abs(c[i] - oc)) <= 1e-5, i
        _check_b(b[i], ob, "mixed")
