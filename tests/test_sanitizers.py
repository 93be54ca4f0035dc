"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The FP64 oracle is rebuilt with gcc ``-fsanitize=address,undefined`` and
  every oracle pin test runs against that build.
* The HIP library is rebuilt with only its host pass instrumented (hipcc
  ``-Xarch_host``) and the host-side error paths of the C ABI run against it:
  argument validation, the no-device report, the plan calls on null plans,
  the option and diagnostic helpers.

Each run is a subprocess with the sanitizer runtime preloaded and recovery
off, so any report fails the test. No GPU is used: on a machine with a GPU
the library run is skipped (its entry points would reach the device).
"""
from __future__ import annotations

import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_SRC = os.path.join(ROOT, "oracle", "ncf_oracle.c")
CSRC = os.path.join(ROOT, "paper_2609_03866_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SAN_ENV = {
    "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=1",
    "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
}


def _runtime(cmd):
    try:
        p = subprocess.run(cmd, capture_output=True, text=True, check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _run(code, args, preload, timeout):
    env = dict(os.environ, LD_PRELOAD=preload, **SAN_ENV)
    r = subprocess.run([sys.executable, "-c", code, *args], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=timeout)
    assert r.returncode == 0, (r.stdout[-4000:] + "\n" + r.stderr[-6000:])
    return r.stdout


def test_oracle_pins_under_sanitizers(tmp_path):
    asan = _runtime(["gcc", "-print-file-name=libasan.so"])
    if asan is None:
        pytest.skip("gcc AddressSanitizer runtime not found")
    lib = str(tmp_path / "libncf_oracle_san.so")
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off",
                    "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", ORACLE_SRC, "-o", lib, "-lm"], check=True)
    code = textwrap.dedent("""
        import sys
        sys.path.insert(0, ".")
        from oracle import oracle as O
        O._LIB = sys.argv[1]
        import pytest
        sys.exit(pytest.main(["-q", "-x", "-p", "no:cacheprovider", "--noconftest",
                              "tests/test_oracle_pins.py", "tests/test_oracle_regular.py",
                              "tests/test_oracle_resample.py"]))
    """)
    out = _run(code, [lib], asan, 900)
    assert "passed" in out and "failed" not in out


def _has_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def _build_host_sanitized(out_dir):
    import concurrent.futures as cf
    import glob
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC,
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
             "-w"]

    def one(src):
        obj = os.path.join(out_dir, os.path.basename(src) + ".o")
        subprocess.run([HIPCC, *flags, "-c", src, "-o", obj], check=True, capture_output=True)
        return obj

    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(one, srcs))
    lib = os.path.join(out_dir, "libncf_san.so")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-shared-libsan",
                    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    *objs, "-o", lib], check=True, capture_output=True)
    return lib


HOST_PATHS = textwrap.dedent("""
    import ctypes, sys
    sys.path.insert(0, ".")
    import numpy as np
    from paper_2609_03866_amd import ncf
    ncf.LIB_PATH = sys.argv[1]
    L = ncf.lib()
    t = np.arange(10.0)
    x = t % 3
    lags = np.arange(3.0)
    checks = 0

    def rc_of(f, *a, **k):
        r = f(*a, raise_on_error=False, **k)
        return r[3]

    P = ctypes.c_void_p
    dp = lambda a: a.ctypes.data_as(P)
    c = np.zeros(3)
    b = np.zeros(3)

    def raw_acf(n, kern, opt):
        return L.ncf_acf(n, dp(t), dp(x), None, 3, dp(lags), kern, ctypes.c_double(0.5),
                         dp(c), dp(b), None, ctypes.byref(opt) if opt is not None else None)

    # argument errors found on the host before any device work
    opt = ncf.Options()
    L.ncf_options_init(ctypes.byref(opt))
    assert raw_acf(1, 0, None) == ncf.E_INVALID_ARG
    assert raw_acf(10, 7, None) == ncf.E_INVALID_ARG
    assert b"kernel" in L.ncf_last_error()
    bad = ncf.Options.from_buffer_copy(opt)
    bad.struct_size = 3
    assert raw_acf(10, 0, bad) == ncf.E_INVALID_ARG
    bad = ncf.Options.from_buffer_copy(opt)
    bad.precision = 9
    assert raw_acf(10, 0, bad) == ncf.E_INVALID_ARG
    bad = ncf.Options.from_buffer_copy(opt)
    bad.method = 9
    assert raw_acf(10, 1, bad) == ncf.E_INVALID_ARG
    bad = ncf.Options.from_buffer_copy(opt)
    bad.grid_size = 5000
    assert raw_acf(10, 0, bad) == ncf.E_INVALID_ARG
    assert L.ncf_ccf(1, None, None, None, 1, None, None, None, 0, None, 0,
                     ctypes.c_double(0.5), None, None, None, None) == ncf.E_INVALID_ARG
    assert len(L.ncf_last_error()) > 0
    checks += 8
    # valid calls reach the device check and report its absence
    assert raw_acf(10, 0, opt) == ncf.E_DEVICE
    assert rc_of(ncf.ccf, t, x, t + 0.25, x, lags, "r", 0.5) == ncf.E_DEVICE
    assert ncf.acf_regular(t, x, lags, 1.0, "r", 0.5, raise_on_error=False)[3] == ncf.E_DEVICE
    mult = np.ones((3, 10), dtype=np.int32)
    assert ncf.acf_resample(t, x, lags, "g", 0.5, mult=mult,
                            raise_on_error=False)[4] == ncf.E_DEVICE
    assert b"no HIP device" in L.ncf_last_error()
    checks += 5
    # null plans, helpers
    L.ncf_plan_destroy(None)
    assert L.ncf_plan_execute(None, None, None, None, None, None, None) == ncf.E_INVALID_ARG
    assert ncf.diag_fft_radices(4096) == [4096]
    for p in range(13, 31):
        assert int(np.prod(ncf.diag_fft_radices(2 ** p))) == 2 ** p
    checks += 3
    print("host paths ok", checks)
""")


def test_library_host_code_under_sanitizers(tmp_path):
    if _has_gpu():
        pytest.skip("a GPU is visible: the host-only paths are checked on CPU machines")
    asan = _runtime([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"])
    if asan is None:
        pytest.skip("clang AddressSanitizer runtime not found")
    lib = _build_host_sanitized(str(tmp_path))
    out = _run(HOST_PATHS, [lib], asan, 600)
    assert "host paths ok" in out
