"""Pins for the oracle's replicate definition (no GPU).

A replicate perturbs the values by sigma * z and writes sample i out mult[i]
times; the oracle builds exactly that series and runs its estimator on it.
The pins fix the definition against other facts:

* zero deviates and unit multiplicities reproduce the point estimate, with
  zero spread;
* a bootstrap replicate (multiplicities >= 1) equals the weighted estimator
  with weights k (errors 1/sqrt(k)): repeating a sample k times is weighting
  it by k (the duplicated-samples identity of the weighted mode);
* flux randomization of a constant series by unit normal deviates gives, on
  a regular grid with the rectangle kernel (one lattice lag per window), an
  ACF whose replicate spread at lag k is 1/sqrt(n - k) (a mean of n - k
  products of independent unit normals, over the lag-0 variance);
* a replicate that keeps one distinct time is degenerate and is left out of
  the statistics.
"""
import numpy as np

from oracle import oracle as O
from paper_2609_03866_amd import synth


def test_identity_replicates_reproduce_the_point_estimate():
    d = synth.small("c1", seed=3)
    t, x, lags = d["t"][:600], d["x"][:600], d["lags"][:40]
    R, n = 5, t.size
    z = np.zeros((R, n))
    mult = np.ones((R, n), dtype=np.int32)
    st, c0, _, _ = O.acf(t, x, lags, "gaussian", d["h"])
    sts, crep, cm, cs = O.acf_resample(t, x, lags, "gaussian", d["h"], sigma=np.ones(n), z=z,
                                       mult=mult)
    assert st == 0 and np.all(sts == 0)
    for r in range(R):
        np.testing.assert_array_equal(crep[r], c0)
    np.testing.assert_allclose(cm, c0, rtol=0, atol=1e-15)
    assert np.all(cs <= 1e-15)


def test_bootstrap_replicate_is_the_weighted_estimator():
    rng = synth.rng_for(4)
    d = synth.small("c1", seed=4)
    t, x, lags = d["t"][:400], d["x"][:400], d["lags"][:30]
    n = t.size
    mult = rng.integers(1, 4, size=(1, n)).astype(np.int32)
    for kernel, h in (("gaussian", d["h"]), ("rectangle", 0.5)):
        sts, crep, _, _ = O.acf_resample(t, x, lags, kernel, h, mult=mult)
        st, cw, _, _ = O.acf(t, x, lags, kernel, h, err=1.0 / np.sqrt(mult[0].astype(float)))
        assert sts[0] == 0 and st == 0
        np.testing.assert_allclose(crep[0], cw, rtol=0, atol=1e-12)


def test_flux_randomization_spread_of_white_noise():
    n, R = 300, 400
    t = np.arange(n, dtype=float)
    x = np.zeros(n)
    rng = synth.rng_for(5)
    z, _ = synth.resample_draws(rng, n, R, flux=True, bootstrap=False)
    lags = np.array([1.0, 2.0, 10.0, 50.0, 150.0])
    sts, crep, cm, cs = O.acf_resample(t, x, lags, "rectangle", 0.5, sigma=np.full(n, 2.0), z=z)
    assert np.all(sts == 0)
    want = 1.0 / np.sqrt(n - lags)
    np.testing.assert_allclose(cs, want, rtol=0.15)
    assert np.all(np.abs(cm) < 4 * want / np.sqrt(R))


def test_degenerate_bootstrap_replicate_is_left_out():
    d = synth.small("c1", seed=6)
    t, x, lags = d["t"][:200], d["x"][:200], d["lags"][:10]
    n = t.size
    mult = np.ones((3, n), dtype=np.int32)
    mult[1] = 0
    mult[1, 17] = 2  # one sample twice: a constant series (mean and sd exact)
    sts, crep, cm, cs = O.acf_resample(t, x, lags, "gaussian", d["h"], mult=mult)
    assert list(sts) == [0, O.E_DEGENERATE, 0]
    assert np.all(np.isnan(crep[1]))
    np.testing.assert_allclose(cm, 0.5 * (crep[0] + crep[2]), rtol=0, atol=1e-15)
