"""GPU parity of the replicate (Monte-Carlo / bootstrap) error bars against
the oracle, which builds every replicate series by its definition (values
perturbed, samples written out mult times) and runs its estimator on it.

The GPU runs the replicates as one weighted batch over shared times. Each
replicate is an ordinary estimate, so the per-replicate tolerances are those
of the single calls (mixed precision 1e-5 on c; FP64 direct sums 1e-11), and
the mean and standard deviation over replicates inherit them.
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


MODES = [("mixed", "auto", 1e-5), ("fp64", "direct", 1e-11)]


def _cmp(crep, cm, cs, o_st, o_crep, o_cm, o_cs, st, tol):
    np.testing.assert_array_equal(st, o_st)
    ok = o_st == 0
    assert np.all(np.isnan(crep[~ok]))
    assert np.max(np.abs(crep[ok] - o_crep[ok])) <= tol
    assert np.max(np.abs(cm - o_cm)) <= tol
    assert np.max(np.abs(cs - o_cs)) <= 2 * tol


@pytest.mark.parametrize("prec,method,tol", MODES)
def test_ccf_resample_m1_small(prec, method, tol):
    d = synth.small("m1", seed=2)
    args = dict(ex=d["ex"], ey=d["ey"], sx=d["ex"], sy=d["ey"], zx=d["zx"], zy=d["zy"],
                multx=d["multx"], multy=d["multy"])
    o_st, o_crep, o_cm, o_cs = O.ccf_resample(d["t"], d["x"], d["s"], d["y"], d["lags"],
                                              "gaussian", d["h"], **args)
    cm, cs, crep, st, rc = ncf.ccf_resample(d["t"], d["x"], d["s"], d["y"], d["lags"],
                                            "gaussian", d["h"], with_reps=True, precision=prec,
                                            method=method, **args)
    assert rc == 0
    _cmp(crep, cm, cs, o_st, o_crep, o_cm, o_cs, st, tol)


@pytest.mark.parametrize("kernel", ["gaussian", "rectangle"])
@pytest.mark.parametrize("scheme", ["flux", "bootstrap", "both"])
def test_acf_resample_schemes(kernel, scheme):
    d = synth.small("c1", seed=11)
    t, x = d["t"], d["x"]
    n, R = t.size, 9
    rng = synth.rng_for(12)
    z, mult = synth.resample_draws(rng, n, R, flux=scheme != "bootstrap",
                                   bootstrap=scheme != "flux")
    sigma = np.full(n, 0.3) if z is not None else None
    err = rng.uniform(0.5, 1.5, n) if scheme == "both" else None
    h = d["h"] if kernel == "gaussian" else 0.5
    o = O.acf_resample(t, x, d["lags"], kernel, h, err=err, sigma=sigma, z=z, mult=mult)
    for prec, method, tol in MODES:
        cm, cs, crep, st, rc = ncf.acf_resample(t, x, d["lags"], kernel, h, err=err, sigma=sigma,
                                                z=z, mult=mult, with_reps=True, precision=prec,
                                                method=method)
        assert rc == 0
        _cmp(crep, cm, cs, *o, st, 1e-9 if kernel == "rectangle" else tol)


def test_resample_degenerate_and_invalid_replicates():
    d = synth.small("c1", seed=13)
    t, x, lags = d["t"][:500], d["x"][:500], d["lags"][:20]
    n = t.size
    mult = np.ones((4, n), dtype=np.int32)
    mult[1] = 0
    mult[1, 17] = 2      # one sample twice: a constant series
    mult[2, 5] = -1      # a negative multiplicity: invalid weights
    o_st, o_crep, o_cm, o_cs = O.acf_resample(t, x, lags, "gaussian", d["h"],
                                              mult=np.where(mult < 0, 0, mult))
    cm, cs, crep, st, rc = ncf.acf_resample(t, x, lags, "gaussian", d["h"], mult=mult,
                                            with_reps=True, precision="fp64", method="direct")
    assert rc == 0
    assert list(st) == [0, ncf.E_DEGENERATE, ncf.E_INVALID_ARG, 0]
    assert np.all(np.isnan(crep[1])) and np.all(np.isnan(crep[2]))
    np.testing.assert_allclose(crep[[0, 3]], o_crep[[0, 3]], rtol=0, atol=1e-11)
    np.testing.assert_allclose(cm, 0.5 * (o_crep[0] + o_crep[3]), rtol=0, atol=1e-11)
    # every replicate failing: the call fails with the first status
    bad = np.zeros((2, n), dtype=np.int32)
    bad[:, 3] = 2
    rc = ncf.acf_resample(t, x, lags, "gaussian", d["h"], mult=bad, raise_on_error=False)[4]
    assert rc == ncf.E_DEGENERATE
    # deviates without their scale
    z = np.zeros((2, n))
    rc = ncf.acf_resample(t, x, lags, "gaussian", d["h"], z=z, raise_on_error=False)[4]
    assert rc == ncf.E_INVALID_ARG


def test_resample_device_pointers():
    import torch
    d = synth.small("c1", seed=14)
    t, x, lags = d["t"], d["x"], d["lags"]
    n, R = t.size, 6
    z, mult = synth.resample_draws(synth.rng_for(15), n, R)
    sigma = np.full(n, 0.2)
    o = O.acf_resample(t, x, lags, "gaussian", d["h"], sigma=sigma, z=z, mult=mult)
    dv = torch.device("cuda:0")
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=dv)
    cm, cs, crep, st, rc = ncf.acf_resample(T(t), T(x), T(lags), "gaussian", d["h"],
                                            sigma=T(sigma), z=T(z), mult=T(mult),
                                            with_reps=True)
    torch.cuda.synchronize()
    assert rc == 0
    _cmp(crep.cpu().numpy(), cm.cpu().numpy(), cs.cpu().numpy(), *o, st, 1e-5)


@pytest.mark.parametrize("kernel", ["rectangle", "gaussian"])
@pytest.mark.parametrize("prec,method,tol", MODES)
def test_ccf_resample_errors_on_one_side(kernel, prec, method, tol):
    # flux randomization of both series, weights from errors on series 2
    # only: series 1 takes unit weights in the pair weight (the window passes
    # read both series' weights)
    d = synth.small("m1", seed=3)
    args = dict(ex=None, ey=d["ey"], sx=d["ex"], sy=d["ey"], zx=d["zx"], zy=d["zy"])
    h = d["h"] if kernel == "gaussian" else 0.5
    o_st, o_crep, o_cm, o_cs = O.ccf_resample(d["t"], d["x"], d["s"], d["y"], d["lags"], kernel,
                                              h, **args)
    cm, cs, crep, st, rc = ncf.ccf_resample(d["t"], d["x"], d["s"], d["y"], d["lags"], kernel,
                                            h, with_reps=True, precision=prec, method=method,
                                            **args)
    assert rc == 0
    _cmp(crep, cm, cs, o_st, o_crep, o_cm, o_cs, st, 1e-9 if kernel == "rectangle" else tol)


def _dropped_run_series(rng, n, R, with_err, flux):
    """A series on [0, 400] whose samples in [100, 300] have multiplicity 0 in
    every replicate (the others 1..3): pairs of kept samples have lags in
    [-100, 100] or 200 and more apart, so lags between about 101 and 199 hold
    only dropped samples."""
    t = np.sort(rng.uniform(0.0, 400.0, n))
    x = rng.normal(size=n)
    mult = rng.integers(1, 4, size=(R, n)).astype(np.int32)
    mult[:, (t > 100.0) & (t < 300.0)] = 0
    err = rng.uniform(0.5, 2.0, n) if with_err else None
    z = rng.normal(size=(R, n)) if flux else None
    sigma = np.full(n, 0.3) if flux else None
    return t, x, err, sigma, z, mult


@pytest.mark.parametrize("kernel", ["rectangle", "gaussian"])
@pytest.mark.parametrize("with_err", [False, True])
@pytest.mark.parametrize("flux", [False, True])
@pytest.mark.parametrize("is_ccf", [False, True])
def test_windows_of_dropped_samples_are_empty(kernel, with_err, flux, is_ccf):
    # a window holding only samples of multiplicity 0 holds no pair of the
    # replicate series: c = 0 exactly, whatever the weights (integer
    # multiplicities, or multiplicities times 1/err^2, whose weight prefix
    # differences leave rounding residue); the other lags match the oracle
    rng = synth.rng_for(960 + 8 * is_ccf + 4 * flux + 2 * with_err + (kernel == "gaussian"))
    R = 3
    lags = np.arange(-20.0, 400.0, 5.0)
    h = 0.5
    X = _dropped_run_series(rng, 400, R, with_err, flux)
    if is_ccf:
        Y = _dropped_run_series(rng, 350, R, with_err, flux)
        args = dict(ex=X[2], ey=Y[2], sx=X[3], sy=Y[3], zx=X[4], zy=Y[4], multx=X[5],
                    multy=Y[5])
        o_st, o_crep, _, _ = O.ccf_resample(X[0], X[1], Y[0], Y[1], lags, kernel, h, **args)
    else:
        args = dict(err=X[2], sigma=X[3], z=X[4], mult=X[5])
        o_st, o_crep, _, _ = O.acf_resample(X[0], X[1], lags, kernel, h, **args)
    assert np.all(o_st == 0)
    gap = (lags > 101.0) & (lags < 199.0)
    assert np.all(o_crep[:, gap] == 0.0)  # the oracle's replicates: empty windows
    for prec, method, tol in MODES:
        if is_ccf:
            cm, cs, crep, st, rc = ncf.ccf_resample(X[0], X[1], Y[0], Y[1], lags, kernel, h,
                                                    with_reps=True, precision=prec,
                                                    method=method, **args)
        else:
            cm, cs, crep, st, rc = ncf.acf_resample(X[0], X[1], lags, kernel, h,
                                                    with_reps=True, precision=prec,
                                                    method=method, **args)
        what = f"{kernel} {prec} {method} err={with_err} flux={flux} ccf={is_ccf}"
        assert rc == 0 and np.all(np.asarray(st) == 0), what
        assert np.all(crep[:, gap] == 0.0), f"{what}: |c| = {np.max(np.abs(crep[:, gap]))}"
        np.testing.assert_array_equal(crep == 0.0, o_crep == 0.0, err_msg=what)
        dc = np.max(np.abs(crep - o_crep))
        assert dc <= (1e-9 if kernel == "rectangle" else tol), f"{what}: {dc}"
