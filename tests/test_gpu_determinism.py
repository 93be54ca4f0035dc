"""Determinism: every entry point, run again on the same inputs, returns
bitwise-identical outputs (c, b, pair counts, statuses).

No kernel accumulates into an output with floating-point atomics: window
items write per-item partials that fixed-order reductions add, spreading is
a gather, the FFT passes and the fused kernel own their cells, and the lag
evaluation sums tiles in a fixed order. So the scheduling of workgroups
(flat XCD-ordered dispatch or the work queue, whose item order depends on
timing) cannot change a result. These tests run each path three times, and
the window scans under both dispatch modes, and compare the raw bits.
"""
import numpy as np
import pytest

from paper_2609_03866_amd import ncf, synth

pytestmark = pytest.mark.gpu


def _bits(*arrs):
    out = []
    for a in arrs:
        a = np.ascontiguousarray(np.asarray(a))
        out.append(a.view(np.uint8).tobytes() if a.dtype != object else repr(a))
    return out


def _same(runs):
    first = _bits(*runs[0])
    for r in runs[1:]:
        assert _bits(*r) == first


@pytest.mark.parametrize("prec,method", [("mixed", "auto"), ("fp64", "auto"),
                                         ("mixed", "direct")])
def test_acf_batch_repeats_and_dispatch_modes(prec, method):
    d = synth.small("c4", seed=31)
    print(f"case: c4-small ACF batch {prec} {method}", flush=True)
    runs = []
    for q in (False, False, True, True):
        c, b, n, st, rc = ncf.acf_batch(d["offs"], d["t"], d["x"], d["lags"], "gaussian",
                                        d["h"], precision=prec, method=method,
                                        window_queue=q, spectral_always=True)
        assert rc == 0
        runs.append((c, b, n, st))
    _same(runs)


def test_weighted_acf_batch_repeats():
    d = synth.c4(seed=32, n_series=16, nmin=200, nmax=4000, K=64, with_err=True)
    print("case: weighted ACF batch (16 curves), mixed", flush=True)
    runs = []
    for q in (False, True, False):
        c, b, n, st, rc = ncf.acf_batch(d["offs"], d["t"], d["x"], d["lags"], "gaussian",
                                        d["h"], err=d["err_values"], window_queue=q,
                                        spectral_always=True)
        assert rc == 0
        runs.append((c, b, n, st))
    _same(runs)


@pytest.mark.parametrize("kernel", ["rectangle", "gaussian"])
def test_ccf_batch_repeats_and_dispatch_modes(kernel):
    d = synth.small("c5", seed=33)
    print(f"case: c5-small CCF batch, {kernel}", flush=True)
    runs = []
    for q in (False, False, True):
        c, b, n, st, rc = ncf.ccf_batch(d["offx"], d["t"], d["x"], d["offy"], d["s"], d["y"],
                                        d["lags"], kernel, d["h"], window_queue=q)
        assert rc == 0
        runs.append((c, b, n, st))
    _same(runs)


def test_single_calls_repeat():
    d = synth.small("c2", seed=34)
    print("case: c2-small single ACF and CCF, both kernels and precisions", flush=True)
    for kern in ("gaussian", "rectangle"):
        for prec in ("mixed", "fp64"):
            _same([ncf.acf(d["t"], d["x"], d["lags"], kern, d["h"], precision=prec,
                           spectral_always=True)[:3] for _ in range(3)])
            _same([ncf.ccf(d["t"], d["x"], d["s"], d["y"], d["lags"], kern, d["h"],
                           precision=prec, spectral_always=True)[:3] for _ in range(3)])


def test_noalloc_entry_repeats():
    d = synth.small("c2", seed=35)
    print("case: c2-small through the allocation-free entry point", flush=True)
    _same([ncf.ccf_noalloc(d["t"], d["x"], d["s"], d["y"], d["lags"], "rectangle",
                           d["h"])[:3] for _ in range(3)])


@pytest.mark.parametrize("kernel", ["gaussian", "rectangle"])
def test_regular_batch_repeats(kernel):
    d = synth.small("r2", seed=36)
    nser = d["offs"].size - 1
    dts = np.ones(nser)
    hs = (0.5 if kernel == "gaussian" else 1.0) * dts
    print(f"case: r2-small regular batch, {kernel}", flush=True)
    runs = []
    for _ in range(3):
        c, b, n, st, rc = ncf.acf_regular_batch(d["offs"], d["t"], d["x"], d["lags"], dts,
                                                kernel, hs)
        assert rc == 0
        runs.append((c, b, n, st))
    _same(runs)


def test_resample_repeats():
    d = synth.small("m1", seed=37)
    args = dict(ex=d["ex"], ey=d["ey"], sx=d["ex"], sy=d["ey"], zx=d["zx"], zy=d["zy"],
                multx=d["multx"], multy=d["multy"])
    print("case: m1-small replicate CCF", flush=True)
    runs = []
    for _ in range(3):
        cm, cs, crep, st, rc = ncf.ccf_resample(d["t"], d["x"], d["s"], d["y"], d["lags"],
                                                "gaussian", d["h"], with_reps=True, **args)
        assert rc == 0
        runs.append((cm, cs, crep, st))
    _same(runs)


@pytest.mark.parametrize("graph", [True, False])
def test_plan_replays_repeat(graph):
    d = synth.small("c4", seed=38)
    print(f"case: c4-small plan, graph={graph}", flush=True)
    plan = ncf.plan_acf(d["offs"], d["t"], d["lags"], "gaussian", d["h"], graph=graph,
                        spectral_always=True)
    try:
        _same([plan.execute(d["x"])[:4] for _ in range(4)])
    finally:
        plan.close()
