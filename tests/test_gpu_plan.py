"""GPU tests of plans (ncf_plan_acf / ncf_plan_ccf / ncf_plan_execute).

A plan is built once from the times and replayed on new values, as one
captured HIP graph or as a replay of the recorded launches. Every replay is
checked against the one-shot batch call on the same values (run eagerly in
between, with host synchronizations) and against the FP64 oracle.
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



def _values_acf(d, seed):
    """New values at the plan's times: an OU series per curve plus noise."""
    rng = synth.rng_for(1000 + seed)
    offs = d["offs"]
    out = np.empty_like(d["x"])
    for i in range(len(offs) - 1):
        sl = slice(offs[i], offs[i + 1])
        out[sl] = synth.ou_at_times(rng, d["t"][sl], 10.0) + 0.2 * rng.standard_normal(
            offs[i + 1] - offs[i])
    return out


def _values_ccf(d, seed):
    rng = synth.rng_for(2000 + seed)
    x = np.empty_like(d["x"])
    y = np.empty_like(d["y"])
    for p in range(len(d["offx"]) - 1):
        sx = slice(d["offx"][p], d["offx"][p + 1])
        sy = slice(d["offy"][p], d["offy"][p + 1])
        x[sx] = synth.ou_at_times(rng, d["t"][sx], 30.0)
        y[sy] = synth.ou_at_times(rng, d["s"][sy], 30.0) + 0.1 * rng.standard_normal(
            d["offy"][p + 1] - d["offy"][p])
    return x, y


def _close_b(b, ob, rel_ref):
    np.testing.assert_allclose(b, ob, rtol=0, atol=rel_ref * np.max(ob))


@pytest.mark.parametrize("graph", [True, False])
@pytest.mark.parametrize("prec,method,ctol,bref", [
    ("mixed", "auto", 1e-5, 2e-6),
    ("fp64", "auto", 5e-8, 2e-8),
    ("mixed", "direct", 1e-5, 1e-6),
])
def test_acf_plan_replays_match_batch_and_oracle(graph, prec, method, ctol, bref):
    d = synth.small("c4", seed=21)
    offs = d["offs"]
    plan = ncf.plan_acf(offs, d["t"], d["lags"], "gaussian", d["h"], precision=prec,
                        method=method, graph=graph)
    try:
        for r in range(4):
            x = _values_acf(d, r)
            c, b, n, st, rc = plan.execute(x)
            assert rc == 0 and np.all(st == 0)
            # eager one-shot call on the same values between replays
            c1, b1, n1, st1, rc1 = ncf.acf_batch(offs, d["t"], x, d["lags"], "gaussian",
                                                 d["h"], precision=prec, method=method)
            assert rc1 == 0
            assert np.max(np.abs(c - c1)) <= ctol
            _close_b(b, b1, bref)
            for i in (0, r + 3, len(offs) - 2):
                sl = slice(offs[i], offs[i + 1])
                s2, oc, ob, on = O.acf(d["t"][sl], x[sl], d["lags"], "gaussian", d["h"][i])
                assert s2 == 0
                assert np.max(np.abs(c[i] - oc)) <= ctol
                _close_b(b[i], ob, bref)
    finally:
        plan.close()


def test_graph_and_launch_replay_are_identical():
    d = synth.small("c4", seed=22)
    pg = ncf.plan_acf(d["offs"], d["t"], d["lags"], "gaussian", d["h"], graph=True)
    pe = ncf.plan_acf(d["offs"], d["t"], d["lags"], "gaussian", d["h"], graph=False)
    try:
        for r in range(3):
            x = _values_acf(d, 10 + r)
            cg, bg = pg.execute(x)[:2]
            ce, be = pe.execute(x)[:2]
            np.testing.assert_array_equal(cg, ce)
            np.testing.assert_array_equal(bg, be)
    finally:
        pg.close()
        pe.close()


@pytest.mark.parametrize("graph", [True, False])
def test_ccf_rectangle_plan_exact_counts(graph):
    d = synth.small("c5", seed=23)
    plan = ncf.plan_ccf(d["offx"], d["t"], d["offy"], d["s"], d["lags"], "rectangle", d["h"],
                        graph=graph)
    try:
        for r in range(3):
            x, y = _values_ccf(d, r)
            c, b, n, st, rc = plan.execute(x, y)
            assert rc == 0 and np.all(st == 0)
            c1, b1, n1, st1, rc1 = ncf.ccf_batch(d["offx"], d["t"], x, d["offy"], d["s"], y,
                                                 d["lags"], "rectangle", d["h"])
            np.testing.assert_array_equal(n, n1)
            np.testing.assert_array_equal(c, c1)
            for p in (0, len(d["offx"]) - 2):
                sx = slice(d["offx"][p], d["offx"][p + 1])
                sy = slice(d["offy"][p], d["offy"][p + 1])
                s2, oc, ob, on = O.ccf(d["t"][sx], x[sx], d["s"][sy], y[sy], d["lags"],
                                       "rectangle", d["h"][p])
                np.testing.assert_array_equal(n[p], on)
                assert np.max(np.abs(c[p] - oc)) <= 1e-9
    finally:
        plan.close()


def test_ccf_gaussian_plan_matches_oracle():
    d = synth.small("c2", seed=24)
    offx = np.array([0, d["t"].size])
    offy = np.array([0, d["s"].size])
    plan = ncf.plan_ccf(offx, d["t"], offy, d["s"], d["lags"], "gaussian", d["h"])
    try:
        for r in range(3):
            rng = synth.rng_for(3000 + r)
            x = d["x"] + 0.3 * rng.standard_normal(d["x"].size)
            y = d["y"] + 0.3 * rng.standard_normal(d["y"].size)
            c, b, n, st, rc = plan.execute(x, y)
            st2, oc, ob, on = O.ccf(d["t"], x, d["s"], y, d["lags"], "gaussian", d["h"])
            assert rc == 0 and st2 == 0
            assert np.max(np.abs(c[0] - oc)) <= 1e-5
            _close_b(b[0], ob, 2e-6)
    finally:
        plan.close()


def test_plan_reports_value_and_time_failures_per_series():
    d = synth.small("c4", seed=25)
    offs = d["offs"]
    t = d["t"].copy()
    t[offs[4]:offs[5]] = t[offs[4]:offs[5]][::-1].copy()  # unsorted times: series 4
    plan = ncf.plan_acf(offs, t, d["lags"], "gaussian", d["h"])
    try:
        for r in range(2):
            x = _values_acf(d, 20 + r)
            x[offs[1] + 3] = np.nan          # series 1: non-finite value
            x[offs[2]:offs[3]] = 2.5         # series 2: constant
            c, b, n, st, rc = plan.execute(x, raise_on_error=False)
            assert rc == ncf.E_INVALID_ARG
            assert st[1] == ncf.E_INVALID_ARG and st[2] == ncf.E_DEGENERATE
            assert st[4] == ncf.E_UNSORTED
            assert np.sum(st != 0) == 3
            for i in (1, 2, 4):
                assert np.all(np.isnan(c[i])) and np.all(b[i] == 0)
            sl = slice(offs[0], offs[1])
            s2, oc, ob, on = O.acf(t[sl], x[sl], d["lags"], "gaussian", d["h"][0])
            assert np.max(np.abs(c[0] - oc)) <= 1e-5
        # a clean execution afterwards reports only the time failure
        x = _values_acf(d, 30)
        st = plan.execute(x, raise_on_error=False)[3]
        assert st[4] == ncf.E_UNSORTED and np.sum(st != 0) == 1
    finally:
        plan.close()


def test_device_pointer_plan_with_torch_tensors():
    import torch
    d = synth.small("c4", seed=26)
    dev = torch.device("cuda:0")
    offs = d["offs"]
    tt = torch.as_tensor(d["t"], device=dev)
    lg = torch.as_tensor(d["lags"], device=dev)
    plan = ncf.plan_acf(offs, tt, lg, "gaussian", d["h"])
    try:
        del tt  # the plan keeps its own copy of the times
        torch.cuda.synchronize()
        outs = []
        xs = [_values_acf(d, 40 + r) for r in range(3)]
        for x in xs:  # enqueue three executions back to back
            outs.append(plan.execute(torch.as_tensor(x, device=dev)))
        torch.cuda.synchronize()
        for x, (c, b, n, st, rc) in zip(xs, outs):
            assert rc == 0 and int(st.abs().sum()) == 0
            c1, b1 = ncf.acf_batch(offs, d["t"], x, d["lags"], "gaussian", d["h"])[:2]
            assert np.max(np.abs(c.cpu().numpy() - c1)) <= 1e-5
    finally:
        plan.close()


def test_queue_dispatch_matches_flat_dispatch():
    # the window scans pull work items from a device queue when asked; every
    # item writes its own partial sums, so results are bitwise those of the
    # one-workgroup-per-item dispatch. Two calls in a row check that each
    # launch leaves its counters reset.
    d = synth.small("c5", seed=31)
    args = (d["offx"], d["t"], d["x"], d["offy"], d["s"], d["y"], d["lags"], "rectangle", d["h"])
    ref = ncf.ccf_batch(*args)
    for _ in range(2):
        q = ncf.ccf_batch(*args, window_queue=True)
        for a, b in zip(ref[:3], q[:3]):
            np.testing.assert_array_equal(a, b)
    g = synth.small("c4", seed=32)
    for prec in ("mixed", "fp64"):
        ref = ncf.acf_batch(g["offs"], g["t"], g["x"], g["lags"], "gaussian", g["h"],
                            precision=prec, method="direct")
        for _ in range(2):
            q = ncf.acf_batch(g["offs"], g["t"], g["x"], g["lags"], "gaussian", g["h"],
                              precision=prec, method="direct", window_queue=True)
            np.testing.assert_array_equal(ref[0], q[0])
            np.testing.assert_array_equal(ref[1], q[1])


def test_queue_dispatch_in_graph_replays():
    d = synth.small("c5", seed=33)
    pq = ncf.plan_ccf(d["offx"], d["t"], d["offy"], d["s"], d["lags"], "rectangle", d["h"],
                      window_queue=True)
    try:
        for r in range(3):
            x, y = _values_ccf(d, 50 + r)
            c, b, n, st, rc = pq.execute(x, y)
            c1, b1, n1 = ncf.ccf_batch(d["offx"], d["t"], x, d["offy"], d["s"], y, d["lags"],
                                       "rectangle", d["h"])[:3]
            np.testing.assert_array_equal(n, n1)
            np.testing.assert_array_equal(c, c1)
    finally:
        pq.close()


@pytest.mark.parametrize("kind", ["acf_gauss", "ccf_rect", "ccf_gauss"])
def test_autotuned_plans_match_oracle_and_default_plan(kind):
    # the autotuner may pick another grid oversampling, FFT radix split or
    # tile, window tiling and dispatch: results stay within the parity
    # tolerances (rectangle counts exact)
    if kind == "acf_gauss":
        d = synth.small("c4", seed=41)
        pa = ncf.plan_acf(d["offs"], d["t"], d["lags"], "gaussian", d["h"], autotune=True)
        pd = ncf.plan_acf(d["offs"], d["t"], d["lags"], "gaussian", d["h"])
        vals = (_values_acf(d, 60),)
    else:
        d = synth.small("c5" if kind == "ccf_rect" else "c2", seed=42)
        if kind == "ccf_gauss":
            d = dict(d, offx=np.array([0, d["t"].size]), offy=np.array([0, d["s"].size]),
                     h=np.array([d["h"]]))
        kern = "rectangle" if kind == "ccf_rect" else "gaussian"
        pa = ncf.plan_ccf(d["offx"], d["t"], d["offy"], d["s"], d["lags"], kern, d["h"],
                          autotune=True)
        pd = ncf.plan_ccf(d["offx"], d["t"], d["offy"], d["s"], d["lags"], kern, d["h"])
        vals = (d["x"], d["y"])
    try:
        info = pa.info()
        assert info["autotuned"] == 1 and info["candidates"] >= 2 and info["replay_ms"] > 0
        assert pd.info()["autotuned"] == 0
        ca, ba, na = pa.execute(*vals)[:3]
        cd, bd, nd = pd.execute(*vals)[:3]
        if kind == "ccf_rect":
            np.testing.assert_array_equal(na, nd)
            assert np.max(np.abs(ca - cd)) <= 1e-9
            sx = slice(d["offx"][0], d["offx"][1])
            sy = slice(d["offy"][0], d["offy"][1])
            st, oc, ob, on = O.ccf(d["t"][sx], vals[0][sx], d["s"][sy], vals[1][sy], d["lags"],
                                   "rectangle", d["h"][0])
            np.testing.assert_array_equal(na[0], on)
        else:
            assert np.max(np.abs(ca - cd)) <= 1e-5
            if kind == "acf_gauss":
                sl = slice(d["offs"][0], d["offs"][1])
                st, oc, ob, on = O.acf(d["t"][sl], vals[0][sl], d["lags"], "gaussian",
                                       d["h"][0])
            else:
                st, oc, ob, on = O.ccf(d["t"], vals[0], d["s"], vals[1], d["lags"], "gaussian",
                                       d["h"][0])
            assert np.max(np.abs(ca[0] - oc)) <= 1e-5
            _close_b(ba[0], ob, 2e-6)
    finally:
        pa.close()
        pd.close()


def test_autotune_cache(tmp_path, monkeypatch):
    # NCF_AUTOTUNE_CACHE names a file of JSON records (one per line): a tuned
    # plan appends its settings; a later plan of the same key takes them
    # without timing candidates and runs the same kernels (bitwise equal
    # outputs); lines that do not parse or hold values out of range are skipped
    import json

    path = tmp_path / "tune.jsonl"
    monkeypatch.setenv("NCF_AUTOTUNE_CACHE", str(path))
    d = synth.small("c4", seed=41)
    args = (d["offs"], d["t"], d["lags"], "gaussian", d["h"])
    keys = ("sigma", "fft_split", "fft_tile_log2", "window_tile_scale", "window_queue",
            "lattice_off")
    print("case: c4-small autotuned plan through the autotune cache", flush=True)
    p1 = ncf.plan_acf(*args, autotune=True)
    try:
        i1 = p1.info()
        assert i1["autotuned"] == 1 and i1["tune_cached"] == 0 and i1["candidates"] >= 2
        r1 = p1.execute(d["x"])[:4]
    finally:
        p1.close()
    lines = path.read_text().splitlines()
    assert len(lines) == 1
    rec = json.loads(lines[0])
    assert set(rec) == {"key", "sigma", "fft_split", "fft_tile_log2", "window_tile_scale",
                        "window_queue", "no_mid", "eval_interp", "replay_ms"}
    p2 = ncf.plan_acf(*args, autotune=True)
    try:
        i2 = p2.info()
        assert i2["autotuned"] == 1 and i2["tune_cached"] == 1 and i2["candidates"] == 0
        assert all(i2[k] == i1[k] for k in keys)
        r2 = p2.execute(d["x"])[:4]
    finally:
        p2.close()
    for a, b in zip(r1, r2):
        assert np.asarray(a).tobytes() == np.asarray(b).tobytes()
    assert len(path.read_text().splitlines()) == 1  # nothing appended
    # another key (other lags) is tuned anew and appended
    p3 = ncf.plan_acf(d["offs"], d["t"], d["lags"][:8], "gaussian", d["h"], autotune=True)
    try:
        assert p3.info()["tune_cached"] == 0
    finally:
        p3.close()
    assert len(path.read_text().splitlines()) == 2
    # a broken line and an out-of-range record of the first key are skipped:
    # the first plan's key is tuned again
    bad = dict(rec, sigma=7.0)
    path.write_text("not json at all\n" + json.dumps(bad) + "\n")
    p4 = ncf.plan_acf(*args, autotune=True)
    try:
        assert p4.info()["tune_cached"] == 0
    finally:
        p4.close()
    assert len(path.read_text().splitlines()) == 3


def test_call_log(tmp_path):
    # NCF_LOG=1: one line per call on stderr (route, grids, window work,
    # fallback rows, statuses, host time); 2 adds the autotune candidates
    import subprocess
    import sys

    code = (
        "import numpy as np\n"
        "from paper_2609_03866_amd import ncf, synth\n"
        "d = synth.small('c2', seed=3)\n"
        "ncf.acf(d['t'], d['x'], d['lags'], 'gaussian', d['h'], spectral_always=True)\n"
        "ncf.ccf(d['t'], d['x'], d['s'], d['y'], d['lags'], 'rectangle', d['h'])\n"
        "e = synth.small('c4', seed=5)\n"
        "p = ncf.plan_acf(e['offs'], e['t'], e['lags'], 'gaussian', e['h'], autotune=True)\n"
        "p.close()\n")
    import os
    env = dict(os.environ, NCF_LOG="2")
    env.pop("NCF_AUTOTUNE_CACHE", None)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    print("case: NCF_LOG=2 in a child process", flush=True)
    r = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True,
                       text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stderr.splitlines() if ln.startswith("ncf: ")]
    assert any(ln.startswith("ncf: acf n=1 ") and "route=spectral" in ln and "rc=0" in ln
               for ln in lines), lines
    assert any(ln.startswith("ncf: ccf n=1 ") and "rectangle" in ln and "route=direct" in ln
               for ln in lines), lines
    assert any(ln.startswith("ncf: plan-build acf n=") for ln in lines), lines
    assert any(ln.startswith("ncf: autotune candidate ") for ln in lines), lines
    assert any(ln.startswith("ncf: plan autotuned over ") for ln in lines), lines
