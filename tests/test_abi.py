"""CPU checks of the C ABI: the library builds, loads, and exports every
function that include/*.h declares (no compute call without a GPU)."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

from paper_2609_03866_amd import ncf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"\b(ncf_[a-z0-9_]+)\s*\(", src):
            names.add(m.group(1))
    return names


def test_headers_declare_entry_points():
    names = _declared()
    for required in ("ncf_acf", "ncf_ccf", "ncf_acf_batch", "ncf_ccf_batch", "ncf_last_error",
                     "ncf_diag_fft", "ncf_diag_type1", "ncf_profile_read", "ncf_profile_filter",
                     "ncf_acf_regular", "ncf_ccf_regular", "ncf_acf_regular_batch", "ncf_ccf_regular_batch",
                     "ncf_acf_resample", "ncf_ccf_resample"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ncf.lib()
    missing = [n for n in sorted(_declared()) if not hasattr(lib, n)]
    assert not missing, missing


def test_version_and_options_struct():
    lib = ncf.lib()
    assert lib.ncf_version() == 100
    o = ncf.Options()
    lib.ncf_options_init(ctypes.byref(o))
    assert o.struct_size == ctypes.sizeof(ncf.Options)
    assert o.precision == ncf.MIXED and o.method == ncf.AUTO


def test_spread_parameters_meet_tolerance():
    # truncation exp(-W^2/2s^2) and aliasing exp(-2 pi^2 s^2 (1 - 1/sigma)) at eps
    for sigma in (1.5, 2.0, 2.9):
        for eps in (1e-7, 1e-13):
            s, W = ncf.diag_spread_params(sigma, eps)
            assert np.exp(-W * W / (2 * s * s)) == pytest.approx(eps, rel=1e-9)
            assert np.exp(-2 * np.pi ** 2 * s * s * (1 - 1 / sigma)) == pytest.approx(eps,
                                                                                       rel=1e-9)


def test_fft_radix_plans():
    assert ncf.diag_fft_radices(4096) == [4096]
    for p in range(13, 31):
        r = ncf.diag_fft_radices(2 ** p)
        assert int(np.prod(r)) == 2 ** p
        assert r[-1] == 4096 and all(x <= 1024 for x in r[:-1])


def test_no_device_is_reported_not_crashed():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("GPU present")
    except Exception:
        pass
    c, b, cnt, rc = ncf.acf(np.arange(10.0), np.arange(10.0) % 3, np.arange(3.0), "g", 0.5,
                            raise_on_error=False)
    assert rc == ncf.E_DEVICE
    assert b"no HIP device" in ncf.lib().ncf_last_error()


def test_regular_entry_points_report_no_device():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("GPU present")
    except Exception:
        pass
    t = np.arange(10.0)
    rc = ncf.acf_regular(t, t % 3, np.arange(3.0), 1.0, "r", 0.5, raise_on_error=False)[3]
    assert rc == ncf.E_DEVICE
    rc = ncf.ccf_regular(t, t % 3, t, t % 2, np.arange(3.0), 1.0, "g", 0.5,
                         raise_on_error=False)[3]
    assert rc == ncf.E_DEVICE


def test_resample_entry_points_report_no_device():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("GPU present")
    except Exception:
        pass
    t = np.arange(10.0)
    mult = np.ones((3, 10), dtype=np.int32)
    rc = ncf.acf_resample(t, t % 3, np.arange(3.0), "g", 0.5, mult=mult,
                          raise_on_error=False)[4]
    assert rc == ncf.E_DEVICE
    rc = ncf.ccf_resample(t, t % 3, t, t % 2, np.arange(3.0), "r", 0.5, multx=mult,
                          raise_on_error=False)[4]
    assert rc == ncf.E_DEVICE


def test_plan_entry_points_declared_and_report_no_device():
    names = _declared()
    for required in ("ncf_plan_acf", "ncf_plan_ccf", "ncf_plan_execute", "ncf_plan_destroy"):
        assert required in names
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("GPU present")
    except Exception:
        pass
    with pytest.raises(ncf.NcfError) as ei:
        ncf.plan_acf(np.array([0, 10]), np.arange(10.0), np.arange(3.0), "g", 0.5)
    assert ei.value.code == ncf.E_DEVICE
    lib = ncf.lib()
    lib.ncf_plan_destroy(None)  # NULL is ignored
    assert lib.ncf_plan_execute(None, None, None, None, None, None, None) == ncf.E_INVALID_ARG
