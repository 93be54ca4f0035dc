"""The allocation-free cross-correlation (ncf_ccf_noalloc) against the
entry point it is a variant of (ncf_ccf with the direct window sums), through
the C ABI: the same kernels on the same plan, so every output is bitwise
equal, and both match the oracle. Two calls in a row, the second on a
smaller input, reuse the library's fixed workspace; a call too large for it
is refused with a message."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_03866_amd import ncf, synth

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device=torch.device("cuda:0"))


def _host(a):
    if hasattr(a, "cpu"):
        import torch
        torch.cuda.synchronize()
        return a.cpu().numpy()
    return np.asarray(a)


def _cases():
    big = synth.small("c2", seed=31)      # 3,000 + 3,000 samples, 401 lags
    small = synth.small("c2", seed=32)    # then a smaller call
    n = 700
    small = dict(small, t=small["t"][:n], x=small["x"][:n], s=small["s"][:n // 2],
                 y=small["y"][:n // 2], lags=small["lags"][::3])
    return big, small


@pytest.mark.parametrize("kernel,prec", [("rectangle", "mixed"), ("rectangle", "fp64"),
                                         ("gaussian", "mixed"), ("gaussian", "fp64")])
@pytest.mark.parametrize("device", [False, True])
@pytest.mark.parametrize("weighted", [False, True])
def test_noalloc_equals_ccf_direct(kernel, prec, device, weighted):
    rng = synth.rng_for(33)
    for d in _cases():
        h = d["h"] if kernel == "gaussian" else 0.5
        ex = rng.uniform(0.5, 2.0, d["t"].size) if weighted else None
        ey = rng.uniform(0.5, 2.0, d["s"].size) if weighted else None
        args = [d["t"], d["x"], d["s"], d["y"], d["lags"]]
        wargs = dict(ex=ex, ey=ey)
        if device:
            args = [_dev(a) for a in args]
            wargs = {k: (None if v is None else _dev(v)) for k, v in wargs.items()}
        ref = ncf.ccf(*args, kernel, h, precision=prec, method="direct", **wargs)
        got = ncf.ccf_noalloc(*args, kernel, h, precision=prec, **wargs)
        assert ref[3] == 0 and got[3] == 0
        for a, b_ in zip(ref[:3], got[:3]):
            np.testing.assert_array_equal(_host(a), _host(b_))
        st, oc, ob, on = O.ccf(d["t"], d["x"], d["s"], d["y"], d["lags"], kernel, h, ex=ex,
                               ey=ey)
        assert st == 0
        c = _host(got[0])
        tol = 1e-9 if kernel == "rectangle" else (1e-5 if prec == "mixed" else 1e-11)
        assert np.max(np.abs(c - oc)) <= tol
        if kernel == "rectangle":
            np.testing.assert_array_equal(_host(got[2]), on)


def test_noalloc_refuses_a_call_beyond_its_workspace():
    # 2 x 3e6 samples: the derived arrays alone exceed the fixed workspace
    rng = synth.rng_for(34)
    n = 3_000_000
    t = _dev(np.sort(rng.uniform(0.0, 1e6, n)))
    x = _dev(rng.normal(size=n))
    lags = _dev(np.linspace(-10.0, 10.0, 21))
    c, b, cnt, rc = ncf.ccf_noalloc(t, x, t, x, lags, "rectangle", 0.5, raise_on_error=False)
    assert rc == ncf.E_UNSUPPORTED
    assert "allocation-free" in ncf.lib().ncf_last_error().decode()
    # the workspace is usable again afterwards
    d = synth.small("c2", seed=35)
    ref = ncf.ccf(d["t"], d["x"], d["s"], d["y"], d["lags"], "rectangle", 0.5, method="direct")
    got = ncf.ccf_noalloc(d["t"], d["x"], d["s"], d["y"], d["lags"], "rectangle", 0.5)
    for a, b_ in zip(ref[:3], got[:3]):
        np.testing.assert_array_equal(a, b_)
