"""Batches whose mixed-precision problems are partly re-evaluated in FP64.

c = r(tau) / s with s the lag-0 scale: when a kernel wide against a short
series of uncorrelated values makes r(0) cancel to a few hundredths, the
FP32 kernel weights' rounding (~1e-6 of the window sums) reaches 1e-4 in c.
The library evaluates such problems (lag-0 scale below 0.1) again in FP64
by the direct window sums, gathered from anywhere in the batch into one
FP64 batch call, and writes their rows back. Here a few such curves sit
between ordinary ones (first, middle, last): every row must meet the mixed
tolerance against the oracle, and the re-evaluated rows must equal an FP64
direct call of the whole batch to 1e-11 in c (a mixed evaluation misses by
orders of magnitude more), for ACF and CCF batches, with and without
errors, from host and from device arrays.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_03866_amd import ncf, synth

pytestmark = pytest.mark.gpu

WIDE_AT = (0, 5, 6, 27)  # positions of the near-degenerate curves


def _lag0_r(t, x, h, err=None):
    """r(0) of the standardized values under the Gaussian window |d| < 6h."""
    w = np.ones_like(x) if err is None else 1.0 / (err * err)
    m = np.sum(w * x) / np.sum(w)
    z = (x - m) / np.sqrt(np.sum(w * (x - m) ** 2) / np.sum(w))
    d = t[:, None] - t[None, :]
    phi = np.where(np.abs(d) < 6.0 * h, np.exp(-0.5 * (d / h) ** 2), 0.0) * np.outer(w, w)
    return float(np.sum(phi * np.outer(z, z)) / np.sum(phi))


def _wide_curve(rng, t0):
    """40 white-noise samples over 60 days, kernel width 12 days."""
    t = np.sort(t0 + rng.uniform(0.0, 60.0, 40))
    return t, rng.standard_normal(40), rng.uniform(0.5, 2.0, 40), 12.0


def _mix(seed, with_err):
    """ACF batch: the c4 sampling and signal (scaled down) with wide curves
    put at WIDE_AT. Returns (offs, t, x, err, h, wide mask, lags)."""
    d = synth.small("c4", seed=seed)
    rng = np.random.default_rng(seed + 1000)
    src = [(d["t"][a:b], d["x"][a:b], d["err_values"][a:b], float(d["h"][i]))
           for i, (a, b) in enumerate(zip(d["offs"][:-1], d["offs"][1:]))]
    curves, wide = [], []
    for i in range(len(src) + len(WIDE_AT)):
        if i in WIDE_AT:
            curves.append(_wide_curve(rng, rng.uniform(0.0, 300.0)))
            wide.append(True)
        else:
            curves.append(src.pop(0))
            wide.append(False)
    offs = np.concatenate([[0], np.cumsum([c[0].size for c in curves])]).astype(np.int64)
    t = np.concatenate([c[0] for c in curves])
    x = np.concatenate([c[1] for c in curves])
    err = np.concatenate([c[2] for c in curves]) if with_err else None
    h = np.array([c[3] for c in curves])
    return offs, t, x, err, h, np.array(wide), d["lags"]


def _np(a):
    return a.cpu().numpy() if hasattr(a, "cpu") else np.asarray(a)


def _dev(*arrs):
    import torch
    return [None if a is None else torch.from_numpy(np.ascontiguousarray(a)).cuda()
            for a in arrs]


@pytest.mark.parametrize("with_err", [False, True])
@pytest.mark.parametrize("device", [False, True])
def test_acf_batch_reevaluates_small_lag0_scales(with_err, device):
    offs, t, x, err, h, wide, lags = _mix(61 + int(with_err), with_err)
    nser = offs.size - 1
    print(f"case: ACF batch of {nser} curves, wide at {WIDE_AT}, err={with_err}, "
          f"device={device}", flush=True)
    for i in np.flatnonzero(wide):
        a, b = offs[i], offs[i + 1]
        r0 = _lag0_r(t[a:b], x[a:b], h[i], None if err is None else err[a:b])
        assert r0 < 0.09, f"curve {i}: lag-0 scale {r0:.3e} not small"
    args = (_dev(t, x, lags) if device else (t, x, lags))
    e_in = _dev(err)[0] if device and err is not None else err
    c, b, n, st, rc = ncf.acf_batch(offs, args[0], args[1], args[2], "gaussian", h, err=e_in)
    c, b, st = _np(c), _np(b), np.asarray(st)
    c64, b64, _, st64, _ = ncf.acf_batch(offs, t, x, lags, "gaussian", h, err=err,
                                         precision="fp64", method="direct")
    assert rc == 0 and np.all(st == 0) and np.all(st64 == 0)
    for i in range(nser):
        a, e = offs[i], offs[i + 1]
        ost, oc, ob, _ = O.acf(t[a:e], x[a:e], lags, "gaussian", h[i],
                               err=None if err is None else err[a:e])
        assert ost == 0
        dc = np.max(np.abs(c[i] - oc))
        assert dc <= 1e-5, f"curve {i} (wide={wide[i]}): max |dc| {dc:.3e}"
        if wide[i]:
            np.testing.assert_allclose(c[i], c64[i], rtol=0, atol=1e-11,
                                       err_msg=f"curve {i}: not the FP64 evaluation")
            np.testing.assert_allclose(b[i], b64[i], rtol=1e-12, atol=0,
                                       err_msg=f"curve {i}: b")


@pytest.mark.parametrize("with_err", [False, True])
@pytest.mark.parametrize("device", [False, True])
def test_ccf_batch_reevaluates_small_lag0_scales(with_err, device):
    offs, t, x, err, h, wide, lags = _mix(71 + int(with_err), with_err)
    rng = np.random.default_rng(81)
    # y: the same times, values and errors perturbed (wide pairs stay white noise)
    y = x + 0.3 * rng.standard_normal(x.size)
    ey = None if err is None else err * rng.uniform(0.8, 1.25, x.size)
    npair = offs.size - 1
    print(f"case: CCF batch of {npair} pairs, wide at {WIDE_AT}, err={with_err}, "
          f"device={device}", flush=True)
    if device:
        td, xd, yd, ld = _dev(t, x, y, lags)
        exd, eyd = _dev(err, ey)
        c, b, n, st, rc = ncf.ccf_batch(offs, td, xd, offs, td, yd, ld, "gaussian", h,
                                        ex=exd, ey=eyd)
    else:
        c, b, n, st, rc = ncf.ccf_batch(offs, t, x, offs, t, y, lags, "gaussian", h,
                                        ex=err, ey=ey)
    c, b, st = _np(c), _np(b), np.asarray(st)
    c64, b64, _, st64, _ = ncf.ccf_batch(offs, t, x, offs, t, y, lags, "gaussian", h,
                                         ex=err, ey=ey, precision="fp64", method="direct")
    assert rc == 0 and np.all(st == 0) and np.all(st64 == 0)
    for i in range(npair):
        a, e = offs[i], offs[i + 1]
        ost, oc, ob, _ = O.ccf(t[a:e], x[a:e], t[a:e], y[a:e], lags, "gaussian", h[i],
                               ex=None if err is None else err[a:e],
                               ey=None if ey is None else ey[a:e])
        assert ost == 0
        dc = np.max(np.abs(c[i] - oc))
        assert dc <= 1e-5, f"pair {i} (wide={wide[i]}): max |dc| {dc:.3e}"
        if wide[i]:
            np.testing.assert_allclose(c[i], c64[i], rtol=0, atol=1e-11,
                                       err_msg=f"pair {i}: not the FP64 evaluation")
            np.testing.assert_allclose(b[i], b64[i], rtol=1e-12, atol=0,
                                       err_msg=f"pair {i}: b")
