"""Benchmark of the kernel-weighted correlation hot path on one MI355X.

Default workload (``--workload c45``): the two batched workloads in one
step, mixed precision (FP32 spreading / FFT / kernel weights with FP64
positions, phases, moments, prefix sums and accumulators):
  * the ACF of 10,000 light curves (lengths log-uniform in [100, 5e4],
    seasonal sampling), 256 lags, Gaussian kernel, one batch call;
  * the CCF of 2,048 series pairs (lengths log-uniform in [1e3, 2e5]),
    512 lags over [-300, 300] d, rectangle kernel with exact pair counts,
    one batch call.
Inputs are resident in HBM. The metric is n*K lag-pairs per second (n = nx +
ny per CCF: the paper's O((n1 + n2) K) unit of work) and series (pairs)
completed per second.

Other workloads (``--workload c1|c2|c3|c4|c5``) are reported the same way. ``r1`` and ``r2`` are regular-lattice
ACFs (the paper's regular-data benchmark: white noise on a 1-d lattice,
366 integer lags) through the classic-FFT route in FP64, with the general
NUFFT route (``nufft_gpu_path``) and the FP64 direct window sums timed on the
same data.

``m1`` times Monte-Carlo error bars: 100 flux-randomized and bootstrap-
resampled replicates of a c2-shaped CCF (2e4 samples per series) in one
call; lag-pairs count every replicate.

Prints one JSON line. ``roofline`` describes the kernel with the largest
share of GPU time (found in untimed profiled steps before the timed ones),
timed with HIP events on the stream the library launches on, around each of
its launches inside the timed steps; ``kernels`` lists every kernel's mean
duration from the profiled steps. ``cpu_baseline`` times the FP64 CPU
oracle on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("n·K lag-pairs/s + batched series/s, mixed vs FP64 GPU path at "
          "|ΔACF|≤1e-5")
HBM_PEAK = 8.0e12            # B/s, MI355X
VALU_PEAK = 256 * 64 * 2.4e9  # lane-ops/s: 256 CUs x 4 SIMD16 x 2.4 GHz (non-packed issue)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_workload(name):
    from paper_2609_03866_amd import synth
    if name == "c1":
        return [synth.c1()]
    if name == "c2":
        return [synth.c2(kernel="gaussian"), synth.c2(kernel="rectangle")]
    if name == "c3":
        return [synth.c3()]
    if name == "c4":
        return [synth.c4()]
    if name == "c4w":
        return [synth.c4(with_err=True)]
    if name == "c5":
        return [synth.c5()]
    if name == "c45":
        return [synth.c4(), synth.c5()]
    if name == "r1":
        return [synth.r1(kernel="gaussian"), synth.r1(kernel="rectangle")]
    if name == "r2":
        return [synth.r2()]
    if name == "m1":
        return [synth.m1()]
    raise SystemExit(f"unknown workload {name}")


def lag_pairs(d):
    K = d["lags"].size
    if d["kind"] == "ccf_resample":
        return d["R"] * (d["t"].size + d["s"].size) * K
    if d["kind"] == "acf":
        return d["t"].size * K
    if d["kind"] == "ccf":
        return (d["t"].size + d["s"].size) * K
    if d["kind"] == "acf_batch":
        return d["t"].size * K
    return (d["t"].size + d["s"].size) * K


def n_series(d):
    if d["kind"] == "ccf_resample":
        return d["R"]
    if d["kind"] == "acf_batch":
        return d["offs"].size - 1
    if d["kind"] == "ccf_batch":
        return d["offx"].size - 1
    return 1


def to_dev(d):
    import torch
    dev = torch.device("cuda:0")
    out = dict(d)
    for k in ("t", "x", "s", "y", "lags", "err", "ex", "ey", "zx", "zy"):
        if d.get(k) is not None:
            out[k] = torch.as_tensor(np.ascontiguousarray(d[k], dtype=np.float64), device=dev)
    for k in ("multx", "multy"):
        if d.get(k) is not None:
            out[k] = torch.as_tensor(np.ascontiguousarray(d[k], dtype=np.int32), device=dev)
    return out


WINDOW_QUEUE = False  # --window-queue: queue dispatch of the window scans


def run_one(d, precision="mixed", method="auto"):
    """One call of the workload. Regular-lattice workloads (with "dt") take the
    classic-FFT route unless method names another ("spectral", "direct")."""
    from paper_2609_03866_amd import ncf
    if d["kind"] == "ccf_resample":
        return ncf.ccf_resample(d["t"], d["x"], d["s"], d["y"], d["lags"], d["kernel"], d["h"],
                                sx=d["ex"], sy=d["ey"], zx=d["zx"],
                                zy=d["zy"], multx=d["multx"], multy=d["multy"], with_reps=True,
                                precision=precision, method=method)
    if d.get("dt") is not None and method == "auto":
        if d["kind"] == "acf":
            return ncf.acf_regular(d["t"], d["x"], d["lags"], d["dt"], d["kernel"], d["h"])
        return ncf.acf_regular_batch(d["offs"], d["t"], d["x"], d["lags"], d["dt"], d["kernel"],
                                     d["h"])
    if d.get("dt") is not None and method == "nufft":
        method = "auto"
    kw = dict(precision=precision, method=method, with_count=True, window_queue=WINDOW_QUEUE)
    if d["kind"] == "acf":
        return ncf.acf(d["t"], d["x"], d["lags"], d["kernel"], d["h"], err=d.get("err"), **kw)
    if d["kind"] == "ccf":
        return ncf.ccf(d["t"], d["x"], d["s"], d["y"], d["lags"], d["kernel"], d["h"], **kw)
    if d["kind"] == "acf_batch":
        return ncf.acf_batch(d["offs"], d["t"], d["x"], d["lags"], d["kernel"], d["h"],
                             err=d.get("err"), **kw)
    return ncf.ccf_batch(d["offx"], d["t"], d["x"], d["offy"], d["s"], d["y"], d["lags"],
                         d["kernel"], d["h"], **kw)


def make_plan(d, precision="mixed", method="auto", autotune=False):
    """A plan over the workload's times (device tensors), replayed as a graph."""
    from paper_2609_03866_amd import ncf
    if d.get("dt") is not None:
        offs = d["offs"] if d["kind"] == "acf_batch" else np.array([0, d["t"].numel()])
        return ncf.plan_acf_regular(offs, d["t"], d["lags"], d["dt"], d["kernel"], d["h"],
                                    autotune=autotune)
    kw = dict(precision=precision, method=method, window_queue=WINDOW_QUEUE, autotune=autotune)
    if d["kind"] == "acf":
        return ncf.plan_acf(np.array([0, d["t"].numel()]), d["t"], d["lags"], d["kernel"],
                            d["h"], err=d.get("err"), **kw)
    if d["kind"] == "ccf":
        return ncf.plan_ccf(np.array([0, d["t"].numel()]), d["t"], np.array([0, d["s"].numel()]),
                            d["s"], d["lags"], d["kernel"], d["h"], **kw)
    if d["kind"] == "acf_batch":
        return ncf.plan_acf(d["offs"], d["t"], d["lags"], d["kernel"], d["h"], err=d.get("err"),
                            **kw)
    return ncf.plan_ccf(d["offx"], d["t"], d["offy"], d["s"], d["lags"], d["kernel"], d["h"],
                        **kw)


def run_plan(plan, d):
    if d["kind"] in ("acf", "acf_batch"):
        return plan.execute(d["x"])
    return plan.execute(d["x"], d["y"])


def lag_subset(d, max_windows=2.5e9):
    """Indices of an evenly spaced subset of the lags that bounds the oracle's
    work on a single large problem to about ``max_windows`` (j, k) windows."""
    n_out = d["s"].size if d["kind"] == "ccf" else d["t"].size
    K = d["lags"].size
    keep = int(min(K, max(8, max_windows // max(n_out, 1))))
    return np.unique(np.linspace(0, K - 1, keep).round().astype(int))


def oracle_subset(d, max_series):
    """The oracle on the whole workload (single problems; an evenly spaced
    subset of lags when the whole would take minutes) or on its first
    ``max_series`` series (batches). Returns (c list, count list, lag-pairs,
    seconds, lag indices)."""
    from oracle import oracle as O
    t0 = time.perf_counter()
    cs, ns, work = [], [], 0
    pick = None
    regular = d.get("dt") is not None
    if d["kind"] == "ccf_resample":
        m = min(max_series, d["R"])
        st, crep, _, _ = O.ccf_resample(d["t"], d["x"], d["s"], d["y"], d["lags"], d["kernel"],
                                        d["h"], sx=d["ex"], sy=d["ey"],
                                        zx=d["zx"][:m], zy=d["zy"][:m], multx=d["multx"][:m],
                                        multy=d["multy"][:m])
        cs, ns = list(crep), [None] * m
        work = m * (d["t"].size + d["s"].size) * d["lags"].size
    elif d["kind"] == "acf" and regular:
        pick = np.arange(d["lags"].size)
        st, c, b, n = O.acf_regular(d["t"], d["x"], d["lags"], d["dt"], d["kernel"], d["h"])
        cs, ns, work = [c], [n], d["t"].size * pick.size
    elif d["kind"] == "acf":
        pick = lag_subset(d)
        st, c, b, n = O.acf(d["t"], d["x"], d["lags"][pick], d["kernel"], d["h"],
                            err=d.get("err"))
        cs, ns, work = [c], [n], d["t"].size * pick.size
    elif d["kind"] == "ccf":
        pick = lag_subset(d)
        st, c, b, n = O.ccf(d["t"], d["x"], d["s"], d["y"], d["lags"][pick], d["kernel"],
                            d["h"])
        cs, ns, work = [c], [n], (d["t"].size + d["s"].size) * pick.size
    elif d["kind"] == "acf_batch":
        o = d["offs"]
        for i in range(min(max_series, o.size - 1)):
            sl = slice(o[i], o[i + 1])
            if regular:
                st, c, b, n = O.acf_regular(d["t"][sl], d["x"][sl], d["lags"], d["dt"][i],
                                            d["kernel"], d["h"][i])
            else:
                st, c, b, n = O.acf(d["t"][sl], d["x"][sl], d["lags"], d["kernel"], d["h"][i],
                                    err=None if d.get("err") is None else d["err"][sl])
            cs.append(c)
            ns.append(n)
            work += (o[i + 1] - o[i]) * d["lags"].size
    else:
        ox, oy = d["offx"], d["offy"]
        for i in range(min(max_series, ox.size - 1)):
            sx, sy = slice(ox[i], ox[i + 1]), slice(oy[i], oy[i + 1])
            st, c, b, n = O.ccf(d["t"][sx], d["x"][sx], d["s"][sy], d["y"][sy], d["lags"],
                                d["kernel"], d["h"][i])
            cs.append(c)
            ns.append(n)
            work += (ox[i + 1] - ox[i] + oy[i + 1] - oy[i]) * d["lags"].size
    return cs, ns, work, time.perf_counter() - t0, pick


def sample_of(d, pick, max_series):
    """What the oracle ran of one workload part."""
    if d["kind"] in ("acf", "ccf"):
        npick = pick.size
        return (f"{d['name']}: whole problem" if npick == d["lags"].size else
                f"{d['name']}: all samples, {npick} of {d['lags'].size} lags (evenly spaced)")
    if d["kind"] == "ccf_resample":
        return f"{d['name']}: first {min(max_series, d['R'])} replicates"
    if d["kind"] == "acf_batch":
        return f"{d['name']}: first {min(max_series, d['offs'].size - 1)} series of the batch"
    return f"{d['name']}: first {min(max_series, d['offx'].size - 1)} pairs of the batch"


def _host(a):
    return np.asarray(a.cpu() if hasattr(a, "cpu") else a)


def max_dc(gpu_c, orc_cs, pick=None):
    g = _host(gpu_c)
    K = g.shape[-1] if g.ndim > 1 else g.size // max(len(orc_cs), 1)
    g = g.reshape(-1, K)
    if pick is not None:
        g = g[:, pick]
    return float(max(np.max(np.abs(g[i] - orc_cs[i])) for i in range(len(orc_cs))))


def counts_equal(gpu_n, orc_ns, pick=None):
    g = _host(gpu_n)
    K = g.shape[-1] if g.ndim > 1 else g.size // max(len(orc_ns), 1)
    g = g.reshape(-1, K)
    if pick is not None:
        g = g[:, pick]
    return bool(all(np.array_equal(g[i], orc_ns[i]) for i in range(len(orc_ns))))


def measure_copy_bandwidth(torch):
    """HBM bandwidth of a plain device copy on this GPU (1 GiB read + 1 GiB
    written per copy, best of 5, HIP events), to set beside the published
    8 TB/s that the roofline uses as its peak."""
    n = 256 * 1024 * 1024  # float32 elements: 1 GiB
    src = torch.ones(n, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(5):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    nbytes = 2 * 4 * n
    del src, dst
    torch.cuda.empty_cache()
    return {"GB_per_s": nbytes / best / 1e9, "bytes_per_copy": nbytes,
            "frac_of_published": nbytes / best / HBM_PEAK}


def measured_traffic(workload, kernel):
    """HBM bytes per dispatch of `kernel` from the committed rocprofv3 counter
    summary (calibrated FETCH_SIZE + WRITE_SIZE), or None when no summary
    exists for this workload or the kernel's source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        tab = json.load(open(path))["workloads"][workload]
    except (OSError, KeyError, ValueError):
        return None
    hits = [v for k, v in tab.items() if k == kernel or k.startswith(kernel + "_r")]
    if not hits:
        return None
    for v in hits:
        src = v.get("source")
        if not src:
            return None
        cur = hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest()[:16]
        if cur != v.get("source_sha"):
            return None
    # variants of one kernel (FFT passes of several radices): per-dispatch
    # mean weighted by their dispatch counts
    n = sum(v.get("dispatches", 1) for v in hits)
    return sum(v["bytes_per_dispatch"] * v.get("dispatches", 1) for v in hits) / n


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c45")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 GPU path")
    ap.add_argument("--no-plan", action="store_true", help="skip the plan replay timing")
    ap.add_argument("--no-nufft", action="store_true",
                    help="regular-lattice workloads: skip the NUFFT-route comparison")
    ap.add_argument("--window-queue", action="store_true",
                    help="window scans as persistent workgroups on a device work queue")
    ap.add_argument("--oracle-series", type=int, default=64)
    ap.add_argument("--oracle-seconds", type=float, default=10.0,
                    help="repeat the oracle sample until it has run this long (>= 3 runs)")
    ap.add_argument("--calibrate", action="store_true",
                    help="first run a 256 MiB device fill and three 256 MiB device copies "
                         "(known byte counts for HBM counter calibration)")
    args = ap.parse_args()
    global WINDOW_QUEUE
    WINDOW_QUEUE = args.window_queue
    if args.gpus != 1:
        print(json.dumps({"error": "ncf runs on one GPU; --gpus must be 1 "
                          "(sharding across GPUs is not implemented)"}))
        sys.exit(2)

    import torch
    from paper_2609_03866_amd import ncf
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    ncf.lib()

    if args.calibrate:
        cal_src = torch.ones(64 * 1024 * 1024, device="cuda:0")
        cal_dst = torch.empty_like(cal_src)
        for _ in range(3):
            cal_dst.copy_(cal_src)
        torch.cuda.synchronize()
        del cal_src, cal_dst
    # a counter-calibration run holds only the known-size copies above
    copy_bw = None if args.calibrate else measure_copy_bandwidth(torch)
    if copy_bw:
        log(f"[bench] device copy: {copy_bw['GB_per_s']:.0f} GB/s (read + write)")
    log(f"[bench] generating workload {args.workload}")
    host = make_workload(args.workload)
    devs = [to_dev(d) for d in host]
    work = sum(lag_pairs(d) for d in host)
    nser = sum(n_series(d) for d in host)

    def step(precision="mixed", method="auto"):
        return [run_one(d, precision, method) for d in devs]

    log("[bench] warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # untimed steps with every kernel timed: the dominant kernel (largest
    # share of GPU time) and the per-kernel table
    ncf.profile_filter(None)
    ncf.profile_enable(True)
    nprof = max(2, min(5, args.steps))
    for _ in range(nprof):
        step()
    prof = ncf.profile_read()
    ncf.profile_enable(False)
    dom_name = max(prof.items(), key=lambda kv: kv[1]["total_ms"])[0]
    kernels = {}
    for k, v in prof.items():
        avg = v["total_ms"] / v["launches"]
        kernels[k] = {"avg_ms": avg, "launches_per_step": v["launches"] / nprof}
        if v["work"] > 0 and avg > 0:  # algorithmic rate of the kernel's launches
            rate = v["work"] / v["launches"] / (avg * 1e-3)
            if v["unit"] == "bytes":
                kernels[k]["GB_per_s"] = rate / 1e9
                kernels[k]["frac_hbm"] = rate / HBM_PEAK
            else:
                kernels[k]["Tlane_op_per_s"] = rate / 1e12
                kernels[k]["frac_valu"] = rate / VALU_PEAK
    # the timed steps; HIP events bracket the dominant kernel's launches only
    # (two event records per launch), so its duration is that of these steps
    ncf.profile_filter(dom_name)
    ncf.profile_enable(True)
    log(f"[bench] timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    dom_rec = ncf.profile_read()[dom_name]
    ncf.profile_enable(False)
    ncf.profile_filter(None)
    value = work / dt
    log(f"[bench] {dt * 1e3:.3f} ms/step, {value:.4e} lag-pairs/s")

    # FP64 plain GPU path (direct window sums, FP64 exp)
    fp64 = None
    if not args.no_fp64:
        step("fp64", "direct")
        torch.cuda.synchronize()
        n64 = max(2, args.steps // 4)
        t1 = time.perf_counter()
        for _ in range(n64):
            res64 = step("fp64", "direct")
        torch.cuda.synchronize()
        dt64 = (time.perf_counter() - t1) / n64
        fp64 = {"value": work / dt64, "ms_per_step": dt64 * 1e3, "path": "fp64 direct window sums"}
        log(f"[bench] fp64 direct: {dt64 * 1e3:.3f} ms/step")

    # all-FP64 spectral path (complex128 grids and transforms, FP64 weights)
    # on the same step: Gaussian workloads only (the rectangle numerator is
    # the same FP64 window scan in every precision)
    n64 = None
    has_gauss = any(d["kernel"] == "gaussian" and d.get("dt") is None for d in host)
    if not args.no_fp64 and has_gauss:
        step("fp64", "auto")
        torch.cuda.synchronize()
        nn = max(2, args.steps // 4)
        t1 = time.perf_counter()
        for _ in range(nn):
            resn64 = step("fp64", "auto")
        torch.cuda.synchronize()
        dtn64 = (time.perf_counter() - t1) / nn
        n64 = {"value": work / dtn64, "ms_per_step": dtn64 * 1e3,
               "path": "fp64 spectral (complex128 NUFFT numerator and pair counts, FP64 "
                       "direct fallback lags)"}
        log(f"[bench] fp64 spectral: {dtn64 * 1e3:.3f} ms/step")

    # regular-lattice workloads: the general (NUFFT, mixed precision) route on
    # the same data, the comparison of the paper's regular-data benchmark
    nufft = None
    regular = host[0].get("dt") is not None
    if regular and not args.no_nufft:
        step("mixed", "nufft")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(max(2, args.steps // 4)):
            resn = step("mixed", "nufft")
        torch.cuda.synchronize()
        dtn = (time.perf_counter() - t1) / max(2, args.steps // 4)
        nufft = {"value": work / dtn, "ms_per_step": dtn * 1e3,
                 "path": "general route (NUFFT numerator, spectral/window pair counts), mixed"}
        log(f"[bench] nufft mixed: {dtn * 1e3:.3f} ms/step")

    # the same step through plans built beforehand (graph replay on the values)
    plan_rep = None
    if not args.no_plan and host[0]["kind"] != "ccf_resample":
        plans = [make_plan(d) for d in devs]
        for pl, d in zip(plans, devs):
            run_plan(pl, d)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for _ in range(args.steps):
            pres = [run_plan(pl, d) for pl, d in zip(plans, devs)]
        torch.cuda.synchronize()
        dtp = (time.perf_counter() - t2) / args.steps
        dcp = max(float((pr[0].reshape(-1) - r[0].reshape(-1)).abs().max().item())
                  for pr, r in zip(pres, res))
        plan_rep = {"value": work / dtp, "ms_per_step": dtp * 1e3,
                    "max_abs_dc_vs_call": dcp,
                    "path": "ncf_plan_execute, captured HIP graph, plans built before timing"}
        for pl in plans:
            pl.close()
        log(f"[bench] plan replay: {dtp * 1e3:.3f} ms/step")
        # the same with autotuned plans (settings chosen by timing candidates)
        t3 = time.perf_counter()
        plans = [make_plan(d, autotune=True) for d in devs]
        torch.cuda.synchronize()
        tune_s = time.perf_counter() - t3
        for pl, d in zip(plans, devs):
            run_plan(pl, d)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        for _ in range(args.steps):
            pres = [run_plan(pl, d) for pl, d in zip(plans, devs)]
        torch.cuda.synchronize()
        dta = (time.perf_counter() - t4) / args.steps
        dca = max(float((pr[0].reshape(-1) - r[0].reshape(-1)).abs().max().item())
                  for pr, r in zip(pres, res))
        keys = ("candidates", "sigma", "fft_split", "fft_tile_log2", "window_tile_scale",
                "window_queue", "grid_cells", "window_items")
        plan_rep["autotuned"] = {"value": work / dta, "ms_per_step": dta * 1e3,
                                 "max_abs_dc_vs_call": dca, "tuning_seconds": tune_s,
                                 "settings": [{k: pl.info()[k] for k in keys} for pl in plans]}
        for pl in plans:
            pl.close()
        log(f"[bench] autotuned plan replay: {dta * 1e3:.3f} ms/step (tuning {tune_s:.2f} s)")

    # roofline of the dominant kernel, HIP events on the library's stream
    # over the timed steps
    name, rec = dom_name, dom_rec
    avg_s = rec["total_ms"] / rec["launches"] / 1e3
    work_per_launch = rec["work"] / rec["launches"]
    if rec["unit"] == "bytes":
        roof = {"bound": "hbm", "achieved": work_per_launch / avg_s / 1e9,
                "peak": HBM_PEAK / 1e9, "unit": "GB/s"}
    else:
        roof = {"bound": "alu", "achieved": work_per_launch / avg_s / 1e12,
                "peak": VALU_PEAK / 1e12, "unit": "Tlane-op/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(args.workload, name)
    roof["kernel"] = name
    roof["avg_launch_ms"] = avg_s * 1e3

    # accuracy against the oracle, CPU baseline
    acc = {}
    cpu = None
    if not args.no_cpu:
        from oracle import oracle as O
        cores = O.max_threads()
        log(f"[bench] oracle on {cores} threads")
        orc_work, orc_time = 0, 0.0
        picks = []
        rates = []
        for i, (d, r) in enumerate(zip(host, res)):
            cs, ns, w, sec, pick = oracle_subset(d, args.oracle_series)
            # repeat the same sample (>= 3 runs, about --oracle-seconds in
            # total); the median run gives the rate
            secs = [sec]
            while len(secs) < 3 or sum(secs) < args.oracle_seconds / len(host):
                secs.append(oracle_subset(d, args.oracle_series)[3])
                if len(secs) >= 200:
                    break
            picks.append(pick)
            orc_work += w
            orc_time += float(np.median(secs))
            rates.append(len(secs))
            key = f"{d['name']}_{d['kernel']}"
            rc_ = r[2] if d["kind"] == "ccf_resample" else r[0]
            acc[key] = {("max_abs_dc_regular_fp64" if regular else "max_abs_dc_mixed"):
                        max_dc(rc_, cs, pick)}
            if d["kernel"] == "rectangle":
                acc[key]["counts_bit_exact"] = counts_equal(r[2], ns, pick)
            if fp64 is not None:
                r64 = res64[i][2] if d["kind"] == "ccf_resample" else res64[i][0]
                acc[key]["max_abs_dc_fp64_direct"] = max_dc(r64, cs, pick)
            if n64 is not None and d["kernel"] == "gaussian":
                acc[key]["max_abs_dc_fp64_spectral"] = max_dc(resn64[i][0], cs, pick)
            acc[key]["oracle_sample"] = sample_of(d, pick, args.oracle_series)
        sample = "; ".join(sample_of(d, p, args.oracle_series) for d, p in zip(host, picks))
        cpu = {"value": orc_work / orc_time, "unit": "lag-pairs/s", "cores": cores,
               "kind": "oracle", "sample": sample, "seconds": orc_time,
               "runs": min(rates), "statistic": "median run"}

    d0 = host[0]
    cfg = {"workload": {"c1": "acf_n2000_K101_gauss_fp64plain_vs_mixed",
                        "c2": "ccf_n1e5x2_K401_gauss+rect_mixed",
                        "c3": "acf_n1e7_K4096_gauss_mixed",
                        "c4": "acf_batch_10000_curves_K256_gauss_mixed",
                        "c4w": "acf_batch_10000_curves_K256_gauss_mixed_weighted_by_errors",
                        "c5": "ccf_batch_2048_pairs_K512_rect_mixed",
                        "c45": "acf_batch_10000_curves_K256_gauss_mixed"
                               "+ccf_batch_2048_pairs_K512_rect_exact_counts",
                        "r1": "acf_regular_n256000_K366_gauss+rect_fp64",
                        "r2": "acf_regular_batch_4096_K366_rect_fp64",
                        "m1": "ccf_resample_R100_n2e4x2_K401_gauss_mixed"}[args.workload],
           "lag_pairs_per_step": int(work), "series_per_step": int(nser)}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "lag-pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if regular else "f32+f64 (mixed)",
        "data": "synthetic",
        "config": cfg,
        "series_per_s": nser / dt,
        "fp64_gpu_path": fp64,
        "fp64_spectral_gpu_path": n64,
        "nufft_gpu_path": nufft,
        "plan_replay": plan_rep,
        "accuracy_vs_oracle": acc,
        "roofline": roof,
        "hbm_copy_measured": copy_bw,
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
