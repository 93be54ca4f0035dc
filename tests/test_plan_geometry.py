"""Host logic of the grid planner (no device): the period, cell count and lag
lattice it picks for one Gaussian spectral problem (ncf_diag_grid).

The period L must cover the samples, the largest lag and the kernel's reach
(L >= span + max|tau| + 9h, the padding reading of the paper's period); the
retained modes reach the cut-off frequency; with lags on a lattice of unit
D the period is P D / d for a whole d, so every lag is a whole number of
units L / P, and the lattice grid never has more cells than the
interpolating one."""
import math

import numpy as np
import pytest

from paper_2609_03866_amd import ncf


def _geom(tmin, tmax, lags, h, **kw):
    L, s, N, M, P = ncf.diag_grid(tmin, tmax, lags, h, **kw)
    return dict(L=L, s=s, N=N, M=M, P=P)


def _check_common(g, span, lags, h):
    assert g["L"] >= span + np.max(np.abs(lags)) + 9 * h - 1e-9
    assert g["N"] >= 4096 and g["N"] & (g["N"] - 1) == 0
    fcut = math.sqrt(math.log(1e9) / (2 * math.pi ** 2)) / h  # mixed default tol 1e-9
    assert g["M"] >= fcut * g["L"] - 1
    assert 2 * g["M"] + 1 <= g["N"]


@pytest.mark.parametrize("span", [300.0, 2065.0, 7.5e4, 1.05e7])
def test_lattice_geometry_on_integer_lags(span):
    lags = np.arange(0.0, 256.0)
    h = 0.5 if span < 1e6 else 0.263
    g = _geom(0.0, span, lags, h)
    gi = _geom(0.0, span, lags, h, lattice=False)
    _check_common(g, span, lags, h)
    _check_common(gi, span, lags, h)
    assert gi["P"] == 0
    assert g["P"] > 0, g
    assert 2 <= g["N"] // g["P"] <= 256 and g["N"] % g["P"] == 0
    assert g["N"] <= gi["N"]
    # L = P D / d with D = 1 and a whole d: every lag is a whole number of L / P
    d = g["P"] / g["L"]
    assert abs(d - round(d)) < 1e-9 and round(d) >= 1
    u = lags * (g["P"] / g["L"])
    assert np.all(np.abs(u - np.round(u)) < 1e-6)


def test_half_unit_lattice_and_negative_lags():
    lags = np.linspace(-300.0, 300.0, 128)  # odd multiples of half the spacing
    g = _geom(0.0, 4.0e4, lags, 0.5, acf=False)
    assert g["P"] > 0
    u = lags * (g["P"] / g["L"])
    assert np.all(np.abs(u - np.round(u)) < 1e-6)


@pytest.mark.parametrize("lags", [np.array([0.0, 1.0, math.sqrt(2.0)]), np.array([3.0]),
                                  np.array([], dtype=np.float64)])
def test_lags_off_a_lattice_are_interpolated(lags):
    g = _geom(0.0, 5.0e3, lags, 0.5, acf=False)
    assert g["P"] == 0


def test_geometry_is_invariant_to_the_lag_order():
    rng = np.random.default_rng(3)
    lags = np.arange(-100.0, 101.0)
    a = _geom(10.0, 9.0e3, lags, 0.5)
    b = _geom(10.0, 9.0e3, rng.permutation(lags), 0.5)
    assert a == b


def test_invalid_arguments_are_reported():
    with pytest.raises(ncf.NcfError):
        ncf.diag_grid(0.0, 100.0, np.arange(3.0), -1.0)
    with pytest.raises(ncf.NcfError):
        ncf.diag_grid(10.0, 0.0, np.arange(3.0), 0.5)
    with pytest.raises(ncf.NcfError):
        ncf.diag_grid(0.0, 100.0, np.array([np.nan]), 0.5)
