"""Pins for the oracle's lattice reading (no GPU).

The regular-lattice estimators (Sec. "Regularly-sampled data") place every
sample at its lattice point t_ref + m dt and decide window membership in
lattice units. These tests fix that reading against things other than
itself:

* on lattices whose times, lags, dt and h are exact binary fractions it is
  the real-space estimator itself (the oracle's direct scan, which the
  brute-force and textbook pins of test_oracle_pins.py already fix);
* on a decimal lattice (dt = 0.1, where the direct predicates suffer
  rounding at the window edges) the rectangle counts are the closed form
  sum over the window's lattice lags q of the ramp n - |q|, and the Gaussian
  pair sums are sum_q (n - |q|) phi_h(q dt - tau);
* the textbook estimator of eq. acf_regular on a gapless lattice;
* the CCF of a series with itself equals its ACF; lattice mismatches are
  rejected.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_03866_amd import synth


def _phi(d, h):
    return math.exp(-d * d / (2 * h * h)) / (h * math.sqrt(2 * math.pi))


@pytest.mark.parametrize("kernel,h", [("gaussian", 0.1875), ("gaussian", 0.75),
                                      ("rectangle", 0.25), ("rectangle", 0.625)])
@pytest.mark.parametrize("seed", [0, 1])
def test_dyadic_lattice_equals_direct_acf(kernel, h, seed):
    rng = synth.rng_for(seed)
    t = synth.lattice_times(rng, 400, dt=0.25, keep=0.6, t0=3.5, dup_frac=0.1)
    x = rng.normal(size=t.size)
    err = rng.uniform(0.5, 2.0, t.size)
    lags = np.concatenate([np.arange(-60, 61) * 0.125, [0.3125, -7.0625, 200.0]])
    for e in (None, err):
        st1, c1, b1, n1 = O.acf(t, x, lags, kernel, h, err=e)
        st2, c2, b2, n2 = O.acf_regular(t, x, lags, 0.25, kernel, h, err=e)
        assert st1 == st2 == 0
        np.testing.assert_array_equal(n1, n2)
        np.testing.assert_allclose(b2, b1, rtol=1e-14, atol=0)
        np.testing.assert_allclose(c2, c1, rtol=0, atol=1e-13)


@pytest.mark.parametrize("kernel,h", [("gaussian", 0.1875), ("rectangle", 0.25)])
def test_dyadic_lattice_equals_direct_ccf(kernel, h):
    rng = synth.rng_for(5)
    t = synth.lattice_times(rng, 300, dt=0.25, keep=0.7, t0=1.0)
    s = synth.lattice_times(rng, 350, dt=0.25, keep=0.8, t0=0.5, dup_frac=0.05)
    x = rng.normal(size=t.size)
    y = np.interp(s - 2.0, t, x) + 0.3 * rng.normal(size=s.size)
    ey = rng.uniform(0.5, 2.0, s.size)
    lags = np.arange(-40, 41) * 0.125
    for e in (None, ey):
        st1, c1, b1, n1 = O.ccf(t, x, s, y, lags, kernel, h, ey=e)
        st2, c2, b2, n2 = O.ccf_regular(t, x, s, y, lags, 0.25, kernel, h, ey=e)
        assert st1 == st2 == 0
        np.testing.assert_array_equal(n1, n2)
        np.testing.assert_allclose(b2, b1, rtol=1e-14, atol=0)
        np.testing.assert_allclose(c2, c1, rtol=0, atol=1e-13)


def _ramp_window(n, lo_q, hi_q):
    return [q for q in range(lo_q, hi_q + 1) if abs(q) < n]


@pytest.mark.parametrize("dt", [0.1, 0.3, 1.0 / 3.0])
def test_decimal_lattice_rectangle_counts_are_the_ramp(dt):
    # gapless lattice, h = dt, lags j dt: window lattice lags j-1..j+1
    n = 150
    t = np.arange(n) * dt
    x = synth.rng_for(2).normal(size=n)
    lags = np.arange(-20, 40) * dt
    st, c, b, cnt = O.acf_regular(t, x, lags, dt, "rectangle", dt)
    assert st == 0
    want = [sum(n - abs(q) for q in _ramp_window(n, j - 1, j + 1)) for j in range(-20, 40)]
    np.testing.assert_array_equal(cnt, want)
    np.testing.assert_array_equal(b, np.asarray(want, float))


def test_decimal_lattice_gaussian_pair_sum_closed_form():
    n, dt, h = 120, 0.1, 0.07
    t = np.arange(n) * dt
    x = synth.rng_for(3).normal(size=n)
    lags = np.array([0.0, 0.1, 0.25, 0.73, 2.0, -0.35])
    st, c, b, _ = O.acf_regular(t, x, lags, dt, "gaussian", h)
    assert st == 0
    for k, tau in enumerate(lags):
        qs = [q for q in range(-n + 1, n) if -6 * h <= q * dt - tau < 6 * h]
        want = sum((n - abs(q)) * _phi(q * dt - tau, h) for q in qs)
        assert b[k] == pytest.approx(max(want, 1e-16), rel=1e-13)


def test_textbook_estimator_on_gapless_lattice():
    # eq. acf_regular: with h < dt/2 (rectangle) each window holds one lattice
    # lag, c(k) = [sum_t x_t x_(t+k) / (n - k)] / [sum_t x_t^2 / n]
    n, dt = 300, 0.1
    t = 7.0 + np.arange(n) * dt
    x = synth.rng_for(4).normal(size=n)
    xs = (x - x.mean()) / x.std()
    ks = np.arange(0, 50)
    st, c, _, cnt = O.acf_regular(t, x, ks * dt, dt, "rectangle", 0.4 * dt)
    assert st == 0
    np.testing.assert_array_equal(cnt, n - ks)
    r0 = np.sum(xs * xs) / n
    want = np.array([np.sum(xs[:n - k] * xs[k:]) / (n - k) for k in ks]) / r0
    np.testing.assert_allclose(c, want, rtol=0, atol=1e-13)


def test_ccf_with_itself_is_acf():
    rng = synth.rng_for(6)
    t = synth.lattice_times(rng, 500, dt=0.1, keep=0.8)
    x = rng.normal(size=t.size)
    lags = np.arange(0, 80) * 0.05
    for kernel, h in (("gaussian", 0.06), ("rectangle", 0.1)):
        _, ca, ba, na = O.acf_regular(t, x, lags, 0.1, kernel, h)
        _, cc, bc, nc = O.ccf_regular(t, x, t, x, lags, 0.1, kernel, h)
        np.testing.assert_array_equal(na, nc)
        np.testing.assert_allclose(bc, ba, rtol=1e-13)
        np.testing.assert_allclose(cc, ca, rtol=0, atol=1e-12)


def test_off_lattice_times_are_rejected():
    t = np.arange(50) * 0.5
    x = synth.rng_for(7).normal(size=50)
    t2 = t.copy()
    t2[10] += 0.01
    assert O.acf_regular(t2, x, [0.0, 1.0], 0.5, "rectangle", 0.5)[0] == O.E_INVALID_ARG
    # second series on a shifted lattice
    assert O.ccf_regular(t, x, t + 0.2, x, [0.0], 0.5, "rectangle", 0.5)[0] == O.E_INVALID_ARG
    assert O.acf_regular(t, x, [0.0], 0.0, "rectangle", 0.5)[0] == O.E_INVALID_ARG
