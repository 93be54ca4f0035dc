"""Thin ctypes binding of the ncf C ABI (include/ncf.h, include/ncf_diag.h).

Argument marshalling only: every step of the computation runs in the HIP
library. Host arrays (numpy) are passed as host pointers; torch CUDA tensors
are passed as device pointers on torch's current stream
(NCF_DEVICE_POINTERS). Loading fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libncf.so")

GAUSSIAN, RECTANGLE = 0, 1
MIXED, FP64 = 0, 1
AUTO, SPECTRAL, DIRECT = 0, 1, 2
DEVICE_POINTERS = 0x1
PLAN_NO_GRAPH = 0x2
WINDOW_QUEUE = 0x4
PLAN_AUTOTUNE = 0x8
SPECTRAL_ALWAYS = 0x10

OK = 0
E_INVALID_ARG = -1
E_UNSORTED = -2
E_DEGENERATE = -3
E_NOMEM = -4
E_DEVICE = -5
E_UNSUPPORTED = -6


class NcfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ncf error {code}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("precision", ctypes.c_int32),
                ("method", ctypes.c_int32), ("tol", ctypes.c_double),
                ("sigma", ctypes.c_double), ("grid_size", ctypes.c_int64),
                ("stream", ctypes.c_void_p), ("flags", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("autotuned", ctypes.c_int32),
                ("candidates", ctypes.c_int32), ("spectral_grids", ctypes.c_int32),
                ("window_launches", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("grid_cells", ctypes.c_int64), ("window_items", ctypes.c_int64),
                ("sigma", ctypes.c_double), ("fft_split", ctypes.c_int32),
                ("fft_tile_log2", ctypes.c_int32), ("window_tile_scale", ctypes.c_int32),
                ("window_queue", ctypes.c_int32), ("replay_ms", ctypes.c_double),
                ("lattice_grids", ctypes.c_int32), ("lattice_off", ctypes.c_int32),
                ("tune_cached", ctypes.c_int32)]


class ProfileRecord(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double), ("work", ctypes.c_double),
                ("work_unit", ctypes.c_char * 16)]


_lib = None
_P = ctypes.c_void_p
_I64 = ctypes.c_int64


def lib():
    """Load libncf.so (built by paper_2609_03866_amd.build). Raises if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2609_03866_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        L.ncf_acf.argtypes = [_I64, _P, _P, _P, _I64, _P, ctypes.c_int, ctypes.c_double, _P, _P,
                              _P, _P]
        L.ncf_ccf.argtypes = [_I64, _P, _P, _P, _I64, _P, _P, _P, _I64, _P, ctypes.c_int,
                              ctypes.c_double, _P, _P, _P, _P]
        L.ncf_ccf_noalloc.argtypes = [_I64, _P, _P, _P, _I64, _P, _P, _P, _I64, _P,
                                      ctypes.c_int, ctypes.c_double, _P, _P, _P, _P]
        L.ncf_acf_batch.argtypes = [_I64, _P, _P, _P, _P, _I64, _P, ctypes.c_int, _P, _P, _P, _P,
                                    _P, _P]
        L.ncf_ccf_batch.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _P, _P, _I64, _P,
                                    ctypes.c_int, _P, _P, _P, _P, _P, _P]
        L.ncf_acf_regular.argtypes = [_I64, _P, _P, _P, ctypes.c_double, _I64, _P, ctypes.c_int,
                                      ctypes.c_double, _P, _P, _P, _P]
        L.ncf_ccf_regular.argtypes = [_I64, _P, _P, _P, _I64, _P, _P, _P, ctypes.c_double, _I64,
                                      _P, ctypes.c_int, ctypes.c_double, _P, _P, _P, _P]
        L.ncf_acf_regular_batch.argtypes = [_I64, _P, _P, _P, _P, _P, _I64, _P, ctypes.c_int,
                                            _P, _P, _P, _P, _P, _P]
        L.ncf_ccf_regular_batch.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _I64, _P,
                                            ctypes.c_int, _P, _P, _P, _P, _P, _P]
        L.ncf_acf_resample.argtypes = [_I64, _P, _P, _P, _P, _I64, _P, _P, _I64, _P, ctypes.c_int,
                                       ctypes.c_double, _P, _P, _P, _P, _P]
        L.ncf_ccf_resample.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _I64, _P, _P, _P, _P, _P, _P,
                                       _I64, _I64, _P, ctypes.c_int, ctypes.c_double, _P, _P, _P,
                                       _P, _P]
        L.ncf_last_error.restype = ctypes.c_char_p
        L.ncf_options_init.argtypes = [_P]
        L.ncf_diag_fft.argtypes = [_I64, ctypes.c_int, ctypes.c_int, _P]
        L.ncf_diag_fft_radices.argtypes = [_I64, _P, ctypes.c_int]
        L.ncf_diag_type1.argtypes = [_I64, _P, _P, ctypes.c_double, ctypes.c_double, _I64, _I64,
                                     ctypes.c_int, _P]
        L.ncf_diag_spread_params.argtypes = [ctypes.c_double, ctypes.c_double, _P]
        L.ncf_diag_grid.argtypes = [ctypes.c_double, ctypes.c_double, _I64, _P, ctypes.c_int,
                                    ctypes.c_double, ctypes.c_int, ctypes.c_int, _P, _P]
        L.ncf_plan_acf.argtypes = [_I64, _P, _P, _P, _I64, _P, ctypes.c_int, _P, _P, _P]
        L.ncf_plan_ccf.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _I64, _P, ctypes.c_int, _P, _P,
                                   _P]
        L.ncf_plan_acf_regular.argtypes = [_I64, _P, _P, _P, _P, _I64, _P, ctypes.c_int, _P, _P,
                                           _P]
        L.ncf_plan_ccf_regular.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _P, _I64, _P,
                                           ctypes.c_int, _P, _P, _P]
        L.ncf_plan_execute.argtypes = [_P, _P, _P, _P, _P, _P, _P]
        L.ncf_plan_destroy.argtypes = [_P]
        L.ncf_plan_info.argtypes = [_P, _P]
        L.ncf_profile_enable.argtypes = [ctypes.c_int]
        L.ncf_profile_filter.argtypes = [ctypes.c_char_p]
        L.ncf_profile_read.argtypes = [_P, ctypes.c_int]
        _lib = L
    return _lib


def _kern(k):
    if isinstance(k, str):
        return {"gaussian": GAUSSIAN, "g": GAUSSIAN, "rectangle": RECTANGLE, "r": RECTANGLE}[
            k.lower()]
    return int(k)


def _is_torch(a):
    return type(a).__module__.startswith("torch")


class _Marshal:
    """Collects pointers for one call; keeps host copies alive."""

    def __init__(self, device):
        self.device = device
        self.keep = []

    def inp(self, a, dtype=np.float64):
        if a is None:
            return None
        if self.device:
            import torch
            tdt = {np.float64: torch.float64, np.int32: torch.int32}[dtype]
            assert a.is_cuda and a.dtype == tdt and a.is_contiguous(), \
                f"device arrays must be contiguous {tdt} CUDA tensors"
            return a.data_ptr()
        a = np.ascontiguousarray(a, dtype=dtype)
        self.keep.append(a)
        return a.ctypes.data

    def out(self, n, dtype):
        if self.device:
            import torch
            tdt = {np.float64: torch.float64, np.int64: torch.int64}[dtype]
            t = torch.empty(n, dtype=tdt, device=self.device)
            self.keep.append(t)
            return t, t.data_ptr()
        a = np.empty(n, dtype=dtype)
        self.keep.append(a)
        return a, a.ctypes.data

    def outs(self, n, with_count):
        """The c, b (float64) and count (int64, optional) outputs of n
        entries each; on the device one allocation holds all three."""
        if not self.device:
            c, pc = self.out(n, np.float64)
            b, pb = self.out(n, np.float64)
            cnt, pn = self.out(n, np.int64) if with_count else (None, None)
            return c, pc, b, pb, cnt, pn
        import torch
        buf = torch.empty((3 if with_count else 2) * n, dtype=torch.float64, device=self.device)
        self.keep.append(buf)
        c, b = buf[:n], buf[n:2 * n]
        cnt = buf[2 * n:].view(torch.int64) if with_count else None
        return (c, c.data_ptr(), b, b.data_ptr(), cnt,
                cnt.data_ptr() if with_count else None)


def _options(precision, method, tol, sigma, grid_size, device, stream, window_queue=False,
             spectral_always=False):
    o = Options()
    lib().ncf_options_init(ctypes.byref(o))
    o.precision = {"mixed": MIXED, "fp64": FP64}.get(precision, precision) \
        if isinstance(precision, str) else int(precision)
    o.method = {"auto": AUTO, "spectral": SPECTRAL, "direct": DIRECT}.get(method, method) \
        if isinstance(method, str) else int(method)
    o.tol = float(tol or 0.0)
    o.sigma = float(sigma or 0.0)
    o.grid_size = int(grid_size or 0)
    if device:
        import torch
        o.flags = DEVICE_POINTERS
        o.stream = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    if window_queue:
        o.flags |= WINDOW_QUEUE
    if spectral_always:
        o.flags |= SPECTRAL_ALWAYS
    return o


def _check(rc, allow=()):
    if rc != OK and rc not in allow:
        raise NcfError(rc, lib().ncf_last_error().decode())
    return rc


def acf(t, x, lags, kernel="gaussian", h=1.0, err=None, precision="mixed", method="auto",
        tol=0.0, sigma=0.0, grid_size=0, with_count=True, raise_on_error=True, stream=None,
        window_queue=False, spectral_always=False):
    """ncf_acf. Returns (c, b, count, status). numpy in -> numpy out; torch CUDA
    tensors in -> torch CUDA tensors out (stream-ordered on `stream`)."""
    dev = t.device if _is_torch(t) else None
    m = _Marshal(dev)
    K = int(lags.numel() if _is_torch(lags) else np.asarray(lags).size)
    c, pc, b, pb, cnt, pn = m.outs(K, with_count)
    n = int(t.numel() if _is_torch(t) else np.asarray(t).size)
    o = _options(precision, method, tol, sigma, grid_size, dev, stream, window_queue,
                 spectral_always)
    rc = lib().ncf_acf(n, m.inp(t), m.inp(x), m.inp(err), K, m.inp(lags), _kern(kernel),
                       float(h), pc, pb, pn, ctypes.byref(o))
    if raise_on_error:
        _check(rc)
    return c, b, cnt, rc


def ccf(t, x, s, y, lags, kernel="gaussian", h=1.0, ex=None, ey=None, precision="mixed",
        method="auto", tol=0.0, sigma=0.0, grid_size=0, with_count=True, raise_on_error=True,
        stream=None, window_queue=False, spectral_always=False):
    """ncf_ccf (lag +tau: series 2 (s, y) lags series 1 (t, x) by tau)."""
    dev = t.device if _is_torch(t) else None
    m = _Marshal(dev)
    K = int(lags.numel() if _is_torch(lags) else np.asarray(lags).size)
    c, pc, b, pb, cnt, pn = m.outs(K, with_count)
    nx = int(t.numel() if _is_torch(t) else np.asarray(t).size)
    ny = int(s.numel() if _is_torch(s) else np.asarray(s).size)
    o = _options(precision, method, tol, sigma, grid_size, dev, stream, window_queue,
                 spectral_always)
    rc = lib().ncf_ccf(nx, m.inp(t), m.inp(x), m.inp(ex), ny, m.inp(s), m.inp(y), m.inp(ey), K,
                       m.inp(lags), _kern(kernel), float(h), pc, pb, pn, ctypes.byref(o))
    if raise_on_error:
        _check(rc)
    return c, b, cnt, rc


def ccf_noalloc(t, x, s, y, lags, kernel="gaussian", h=1.0, ex=None, ey=None,
                precision="mixed", with_count=True, raise_on_error=True, stream=None):
    """ncf_ccf_noalloc: the direct window sums in the library's fixed
    workspace (no device allocation by the library during the call)."""
    dev = t.device if _is_torch(t) else None
    m = _Marshal(dev)
    K = int(lags.numel() if _is_torch(lags) else np.asarray(lags).size)
    c, pc, b, pb, cnt, pn = m.outs(K, with_count)
    nx = int(t.numel() if _is_torch(t) else np.asarray(t).size)
    ny = int(s.numel() if _is_torch(s) else np.asarray(s).size)
    o = _options(precision, "direct", 0.0, 0.0, 0, dev, stream)
    rc = lib().ncf_ccf_noalloc(nx, m.inp(t), m.inp(x), m.inp(ex), ny, m.inp(s), m.inp(y),
                               m.inp(ey), K, m.inp(lags), _kern(kernel), float(h), pc, pb, pn,
                               ctypes.byref(o))
    if raise_on_error:
        _check(rc)
    return c, b, cnt, rc


def acf_batch(offs, t, x, lags, kernel="gaussian", h=1.0, err=None, precision="mixed",
              method="auto", tol=0.0, sigma=0.0, grid_size=0, with_count=True,
              raise_on_error=True, stream=None, window_queue=False, spectral_always=False):
    """ncf_acf_batch over CSR series. Returns (c[nser, K], b, count, status[nser], rc)."""
    offs = np.ascontiguousarray(offs, dtype=np.int64)
    nser = offs.size - 1
    hs = np.ascontiguousarray(np.broadcast_to(np.asarray(h, dtype=np.float64), (nser,)))
    dev = t.device if _is_torch(t) else None
    m = _Marshal(dev)
    K = int(lags.numel() if _is_torch(lags) else np.asarray(lags).size)
    c, pc, b, pb, cnt, pn = m.outs(nser * K, with_count)
    st = np.zeros(nser, dtype=np.int32)
    o = _options(precision, method, tol, sigma, grid_size, dev, stream, window_queue,
                 spectral_always)
    rc = lib().ncf_acf_batch(nser, offs.ctypes.data, m.inp(t), m.inp(x), m.inp(err), K,
                             m.inp(lags), _kern(kernel), hs.ctypes.data, pc, pb, pn,
                             st.ctypes.data, ctypes.byref(o))
    if raise_on_error:
        _check(rc)
    rs = (lambda a: a.reshape(nser, K) if a is not None else None)
    return rs(c), rs(b), rs(cnt), st, rc


def ccf_batch(offx, t, x, offy, s, y, lags, kernel="gaussian", h=1.0, ex=None, ey=None,
              precision="mixed", method="auto", tol=0.0, sigma=0.0, grid_size=0,
              with_count=True, raise_on_error=True, stream=None, window_queue=False,
              spectral_always=False):
    """ncf_ccf_batch over CSR series pairs."""
    offx = np.ascontiguousarray(offx, dtype=np.int64)
    offy = np.ascontiguousarray(offy, dtype=np.int64)
    npair = offx.size - 1
    hs = np.ascontiguousarray(np.broadcast_to(np.asarray(h, dtype=np.float64), (npair,)))
    dev = t.device if _is_torch(t) else None
    m = _Marshal(dev)
    K = int(lags.numel() if _is_torch(lags) else np.asarray(lags).size)
    c, pc, b, pb, cnt, pn = m.outs(npair * K, with_count)
    st = np.zeros(npair, dtype=np.int32)
    o = _options(precision, method, tol, sigma, grid_size, dev, stream, window_queue,
                 spectral_always)
    rc = lib().ncf_ccf_batch(npair, offx.ctypes.data, m.inp(t), m.inp(x), m.inp(ex),
                             offy.ctypes.data, m.inp(s), m.inp(y), m.inp(ey), K, m.inp(lags),
                             _kern(kernel), hs.ctypes.data, pc, pb, pn, st.ctypes.data,
                             ctypes.byref(o))
    if raise_on_error:
        _check(rc)
    rs = (lambda a: a.reshape(npair, K) if a is not None else None)
    return rs(c), rs(b), rs(cnt), st, rc


# ------------------------------------------------- regular-lattice family

def acf_regular(t, x, lags, dt, kernel="gaussian", h=1.0, err=None, with_count=True,
                raise_on_error=True, stream=None):
    """ncf_acf_regular: times on the lattice t_ref + m dt (classic-FFT route).
    Returns (c, b, count, status); numpy or torch CUDA as in acf."""
    dev = t.device if _is_torch(t) else None
    m = _Marshal(dev)
    K = int(lags.numel() if _is_torch(lags) else np.asarray(lags).size)
    c, pc, b, pb, cnt, pn = m.outs(K, with_count)
    n = int(t.numel() if _is_torch(t) else np.asarray(t).size)
    o = _options("fp64", "auto", 0.0, 0.0, 0, dev, stream)
    rc = lib().ncf_acf_regular(n, m.inp(t), m.inp(x), m.inp(err), float(dt), K, m.inp(lags),
                               _kern(kernel), float(h), pc, pb, pn, ctypes.byref(o))
    if raise_on_error:
        _check(rc)
    return c, b, cnt, rc


def ccf_regular(t, x, s, y, lags, dt, kernel="gaussian", h=1.0, ex=None, ey=None,
                with_count=True, raise_on_error=True, stream=None):
    """ncf_ccf_regular: both series on one lattice (lag +tau: series 2 lags series 1)."""
    dev = t.device if _is_torch(t) else None
    m = _Marshal(dev)
    K = int(lags.numel() if _is_torch(lags) else np.asarray(lags).size)
    c, pc, b, pb, cnt, pn = m.outs(K, with_count)
    nx = int(t.numel() if _is_torch(t) else np.asarray(t).size)
    ny = int(s.numel() if _is_torch(s) else np.asarray(s).size)
    o = _options("fp64", "auto", 0.0, 0.0, 0, dev, stream)
    rc = lib().ncf_ccf_regular(nx, m.inp(t), m.inp(x), m.inp(ex), ny, m.inp(s), m.inp(y),
                               m.inp(ey), float(dt), K, m.inp(lags), _kern(kernel), float(h),
                               pc, pb, pn, ctypes.byref(o))
    if raise_on_error:
        _check(rc)
    return c, b, cnt, rc


def acf_regular_batch(offs, t, x, lags, dt, kernel="gaussian", h=1.0, err=None,
                      with_count=True, raise_on_error=True, stream=None):
    """ncf_acf_regular_batch over CSR series; dt and h scalars or one per series."""
    offs = np.ascontiguousarray(offs, dtype=np.int64)
    nser = offs.size - 1
    hs = np.ascontiguousarray(np.broadcast_to(np.asarray(h, dtype=np.float64), (nser,)))
    dts = np.ascontiguousarray(np.broadcast_to(np.asarray(dt, dtype=np.float64), (nser,)))
    dev = t.device if _is_torch(t) else None
    m = _Marshal(dev)
    K = int(lags.numel() if _is_torch(lags) else np.asarray(lags).size)
    c, pc, b, pb, cnt, pn = m.outs(nser * K, with_count)
    st = np.zeros(nser, dtype=np.int32)
    o = _options("fp64", "auto", 0.0, 0.0, 0, dev, stream)
    rc = lib().ncf_acf_regular_batch(nser, offs.ctypes.data, m.inp(t), m.inp(x), m.inp(err),
                                     dts.ctypes.data, K, m.inp(lags), _kern(kernel),
                                     hs.ctypes.data, pc, pb, pn, st.ctypes.data, ctypes.byref(o))
    if raise_on_error:
        _check(rc)
    rs = (lambda a: a.reshape(nser, K) if a is not None else None)
    return rs(c), rs(b), rs(cnt), st, rc


def ccf_regular_batch(offx, t, x, offy, s, y, lags, dt, kernel="gaussian", h=1.0, ex=None,
                      ey=None, with_count=True, raise_on_error=True, stream=None):
    """ncf_ccf_regular_batch over CSR series pairs."""
    offx = np.ascontiguousarray(offx, dtype=np.int64)
    offy = np.ascontiguousarray(offy, dtype=np.int64)
    npair = offx.size - 1
    hs = np.ascontiguousarray(np.broadcast_to(np.asarray(h, dtype=np.float64), (npair,)))
    dts = np.ascontiguousarray(np.broadcast_to(np.asarray(dt, dtype=np.float64), (npair,)))
    dev = t.device if _is_torch(t) else None
    m = _Marshal(dev)
    K = int(lags.numel() if _is_torch(lags) else np.asarray(lags).size)
    c, pc, b, pb, cnt, pn = m.outs(npair * K, with_count)
    st = np.zeros(npair, dtype=np.int32)
    o = _options("fp64", "auto", 0.0, 0.0, 0, dev, stream)
    rc = lib().ncf_ccf_regular_batch(npair, offx.ctypes.data, m.inp(t), m.inp(x), m.inp(ex),
                                     offy.ctypes.data, m.inp(s), m.inp(y), m.inp(ey),
                                     dts.ctypes.data, K, m.inp(lags), _kern(kernel),
                                     hs.ctypes.data, pc, pb, pn, st.ctypes.data,
                                     ctypes.byref(o))
    if raise_on_error:
        _check(rc)
    rs = (lambda a: a.reshape(npair, K) if a is not None else None)
    return rs(c), rs(b), rs(cnt), st, rc


# ------------------------------------------------ replicate error bars

def _numel(a):
    return int(a.numel() if _is_torch(a) else np.asarray(a).size)


def acf_resample(t, x, lags, kernel="gaussian", h=1.0, err=None, sigma=None, z=None, mult=None,
                 R=None, with_reps=False, precision="mixed", method="auto", raise_on_error=True,
                 stream=None):
    """ncf_acf_resample: R replicates (flux randomization x + sigma z[r],
    bootstrap multiplicities mult[r]); z and mult are (R, n) arrays drawn by
    the caller. Returns (c_mean, c_sd, c_rep or None, status[R], rc)."""
    n = _numel(t)
    if R is None:
        R = (_numel(z) if z is not None else _numel(mult)) // n
    dev = t.device if _is_torch(t) else None
    m = _Marshal(dev)
    K = _numel(lags)
    cm, pm = m.out(K, np.float64)
    cs, ps = m.out(K, np.float64)
    cr, pr = m.out(R * K, np.float64) if with_reps else (None, None)
    st = np.zeros(R, dtype=np.int32)
    o = _options(precision, method, 0.0, 0.0, 0, dev, stream)
    rc = lib().ncf_acf_resample(n, m.inp(t), m.inp(x), m.inp(err), m.inp(sigma), int(R),
                                m.inp(z), m.inp(mult, np.int32), K, m.inp(lags), _kern(kernel),
                                float(h), pm, ps, pr, st.ctypes.data, ctypes.byref(o))
    if raise_on_error:
        _check(rc)
    return cm, cs, (cr.reshape(R, K) if cr is not None else None), st, rc


def ccf_resample(t, x, s, y, lags, kernel="gaussian", h=1.0, ex=None, ey=None, sx=None,
                 sy=None, zx=None, zy=None, multx=None, multy=None, R=None, with_reps=False,
                 precision="mixed", method="auto", raise_on_error=True, stream=None):
    """ncf_ccf_resample (series 1 = (t, x), series 2 = (s, y), each with its own
    deviates and multiplicities, (R, nx) and (R, ny))."""
    nx, ny = _numel(t), _numel(s)
    if R is None:
        for a, nn in ((zx, nx), (multx, nx), (zy, ny), (multy, ny)):
            if a is not None:
                R = _numel(a) // nn
                break
    dev = t.device if _is_torch(t) else None
    m = _Marshal(dev)
    K = _numel(lags)
    cm, pm = m.out(K, np.float64)
    cs, ps = m.out(K, np.float64)
    cr, pr = m.out(R * K, np.float64) if with_reps else (None, None)
    st = np.zeros(R, dtype=np.int32)
    o = _options(precision, method, 0.0, 0.0, 0, dev, stream)
    rc = lib().ncf_ccf_resample(nx, m.inp(t), m.inp(x), m.inp(ex), m.inp(sx), m.inp(zx),
                                m.inp(multx, np.int32), ny, m.inp(s), m.inp(y), m.inp(ey),
                                m.inp(sy), m.inp(zy), m.inp(multy, np.int32), int(R), K,
                                m.inp(lags), _kern(kernel), float(h), pm, ps, pr,
                                st.ctypes.data, ctypes.byref(o))
    if raise_on_error:
        _check(rc)
    return cm, cs, (cr.reshape(R, K) if cr is not None else None), st, rc


# ------------------------------------------------------------------ plans

class Plan:
    """A built plan (ncf_plan_acf / ncf_plan_ccf): run it on new values with
    execute(); release it with close() (also on garbage collection)."""

    def __init__(self, handle, ccf, nprob, K, device):
        self._h = handle
        self.ccf = ccf
        self.nprob = nprob
        self.K = K
        self.device = device

    def execute(self, x, y=None, with_count=True, raise_on_error=True):
        """ncf_plan_execute. Returns (c[nprob, K], b, count, status[nprob], rc).
        Device plans take torch CUDA tensors and return torch tensors (status
        included), enqueued on the plan's stream."""
        if self._h is None:
            raise ValueError("plan is closed")
        m = _Marshal(self.device)
        n = self.nprob * self.K
        c, pc, b, pb, cnt, pn = m.outs(n, with_count)
        if self.device:
            import torch
            st = torch.zeros(self.nprob, dtype=torch.int32, device=self.device)
            pst = st.data_ptr()
        else:
            st = np.zeros(self.nprob, dtype=np.int32)
            pst = st.ctypes.data
        rc = lib().ncf_plan_execute(self._h, m.inp(x), m.inp(y), pc, pb, pn, pst)
        if raise_on_error:
            _check(rc)
        rs = (lambda a: a.reshape(self.nprob, self.K) if a is not None else None)
        return rs(c), rs(b), rs(cnt), st, rc

    def info(self):
        """ncf_plan_info as a dict."""
        if self._h is None:
            raise ValueError("plan is closed")
        i = PlanInfo()
        i.struct_size = ctypes.sizeof(PlanInfo)
        _check(lib().ncf_plan_info(self._h, ctypes.byref(i)))
        return {name: getattr(i, name) for name, _ in PlanInfo._fields_ if name != "struct_size"}

    def close(self):
        if self._h is not None:
            lib().ncf_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _plan_options(precision, method, tol, sigma, grid_size, dev, stream, graph,
                  window_queue=False, autotune=False, spectral_always=False):
    o = _options(precision, method, tol, sigma, grid_size, dev, stream, window_queue,
                 spectral_always)
    if not graph:
        o.flags |= PLAN_NO_GRAPH
    if autotune:
        o.flags |= PLAN_AUTOTUNE
    return o


def plan_acf(offs, t, lags, kernel="gaussian", h=1.0, err=None, precision="mixed",
             method="auto", tol=0.0, sigma=0.0, grid_size=0, graph=True, stream=None,
             window_queue=False, autotune=False, spectral_always=False):
    """ncf_plan_acf over CSR series (times fixed, values given per execute)."""
    offs = np.ascontiguousarray(offs, dtype=np.int64)
    nser = offs.size - 1
    hs = np.ascontiguousarray(np.broadcast_to(np.asarray(h, dtype=np.float64), (nser,)))
    dev = t.device if _is_torch(t) else None
    m = _Marshal(dev)
    K = int(lags.numel() if _is_torch(lags) else np.asarray(lags).size)
    o = _plan_options(precision, method, tol, sigma, grid_size, dev, stream, graph,
                      window_queue, autotune, spectral_always)
    hp = ctypes.c_void_p()
    _check(lib().ncf_plan_acf(nser, offs.ctypes.data, m.inp(t), m.inp(err), K, m.inp(lags),
                              _kern(kernel), hs.ctypes.data, ctypes.byref(o), ctypes.byref(hp)))
    return Plan(hp.value, False, nser, K, dev)


def plan_ccf(offx, t, offy, s, lags, kernel="gaussian", h=1.0, ex=None, ey=None,
             precision="mixed", method="auto", tol=0.0, sigma=0.0, grid_size=0, graph=True,
             stream=None, window_queue=False, autotune=False, spectral_always=False):
    """ncf_plan_ccf over CSR series pairs."""
    offx = np.ascontiguousarray(offx, dtype=np.int64)
    offy = np.ascontiguousarray(offy, dtype=np.int64)
    npair = offx.size - 1
    hs = np.ascontiguousarray(np.broadcast_to(np.asarray(h, dtype=np.float64), (npair,)))
    dev = t.device if _is_torch(t) else None
    m = _Marshal(dev)
    K = int(lags.numel() if _is_torch(lags) else np.asarray(lags).size)
    o = _plan_options(precision, method, tol, sigma, grid_size, dev, stream, graph,
                      window_queue, autotune, spectral_always)
    hp = ctypes.c_void_p()
    _check(lib().ncf_plan_ccf(npair, offx.ctypes.data, m.inp(t), m.inp(ex), offy.ctypes.data,
                              m.inp(s), m.inp(ey), K, m.inp(lags), _kern(kernel),
                              hs.ctypes.data, ctypes.byref(o), ctypes.byref(hp)))
    return Plan(hp.value, True, npair, K, dev)


def plan_acf_regular(offs, t, lags, dt, kernel="gaussian", h=1.0, err=None, graph=True,
                     stream=None, autotune=False):
    """ncf_plan_acf_regular over CSR series on regular lattices."""
    offs = np.ascontiguousarray(offs, dtype=np.int64)
    nser = offs.size - 1
    hs = np.ascontiguousarray(np.broadcast_to(np.asarray(h, dtype=np.float64), (nser,)))
    dts = np.ascontiguousarray(np.broadcast_to(np.asarray(dt, dtype=np.float64), (nser,)))
    dev = t.device if _is_torch(t) else None
    m = _Marshal(dev)
    K = int(lags.numel() if _is_torch(lags) else np.asarray(lags).size)
    o = _plan_options("fp64", "auto", 0.0, 0.0, 0, dev, stream, graph, False, autotune)
    hp = ctypes.c_void_p()
    _check(lib().ncf_plan_acf_regular(nser, offs.ctypes.data, m.inp(t), m.inp(err),
                                      dts.ctypes.data, K, m.inp(lags), _kern(kernel),
                                      hs.ctypes.data, ctypes.byref(o), ctypes.byref(hp)))
    return Plan(hp.value, False, nser, K, dev)


def plan_ccf_regular(offx, t, offy, s, lags, dt, kernel="gaussian", h=1.0, ex=None, ey=None,
                     graph=True, stream=None, autotune=False):
    """ncf_plan_ccf_regular over CSR series pairs on common lattices."""
    offx = np.ascontiguousarray(offx, dtype=np.int64)
    offy = np.ascontiguousarray(offy, dtype=np.int64)
    npair = offx.size - 1
    hs = np.ascontiguousarray(np.broadcast_to(np.asarray(h, dtype=np.float64), (npair,)))
    dts = np.ascontiguousarray(np.broadcast_to(np.asarray(dt, dtype=np.float64), (npair,)))
    dev = t.device if _is_torch(t) else None
    m = _Marshal(dev)
    K = int(lags.numel() if _is_torch(lags) else np.asarray(lags).size)
    o = _plan_options("fp64", "auto", 0.0, 0.0, 0, dev, stream, graph, False, autotune)
    hp = ctypes.c_void_p()
    _check(lib().ncf_plan_ccf_regular(npair, offx.ctypes.data, m.inp(t), m.inp(ex),
                                      offy.ctypes.data, m.inp(s), m.inp(ey), dts.ctypes.data, K,
                                      m.inp(lags), _kern(kernel), hs.ctypes.data,
                                      ctypes.byref(o), ctypes.byref(hp)))
    return Plan(hp.value, True, npair, K, dev)


# ------------------------------------------------------------- diagnostics

def diag_fft(x, sign=+1, precision="mixed"):
    """ncf_diag_fft on a complex numpy array (natural order in and out)."""
    fp64 = precision in ("fp64", FP64)
    a = np.ascontiguousarray(x, dtype=np.complex128 if fp64 else np.complex64).copy()
    _check(lib().ncf_diag_fft(a.size, FP64 if fp64 else MIXED, int(sign), a.ctypes.data))
    return a


def diag_fft_radices(N):
    r = np.zeros(4, dtype=np.int32)
    n = lib().ncf_diag_fft_radices(int(N), r.ctypes.data, 4)
    _check(n if n < 0 else OK)
    return [int(v) for v in r[:n]]


def diag_type1(t, v, t_ref, L, N, M, precision="mixed"):
    t = np.ascontiguousarray(t, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.zeros(2 * (2 * M + 1))
    _check(lib().ncf_diag_type1(t.size, t.ctypes.data, v.ctypes.data, float(t_ref), float(L),
                                int(N), int(M), FP64 if precision in ("fp64", FP64) else MIXED,
                                out.ctypes.data))
    return out[0::2] + 1j * out[1::2]


def diag_grid(tmin, tmax, lags, h, acf=True, precision="mixed", lattice=True):
    """ncf_diag_grid: (L, s, N, M, P) of the planner's grid for one problem."""
    lags = np.ascontiguousarray(lags, dtype=np.float64)
    of = np.zeros(2)
    oi = np.zeros(3, dtype=np.int64)
    _check(lib().ncf_diag_grid(float(tmin), float(tmax), lags.size,
                               lags.ctypes.data, 1 if acf else 0, float(h),
                               FP64 if precision == "fp64" else MIXED,
                               1 if lattice else 0, of.ctypes.data, oi.ctypes.data))
    return float(of[0]), float(of[1]), int(oi[0]), int(oi[1]), int(oi[2])


def diag_spread_params(sigma, eps):
    out = np.zeros(2)
    _check(lib().ncf_diag_spread_params(float(sigma), float(eps), out.ctypes.data))
    return float(out[0]), float(out[1])


def profile_enable(on=True):
    lib().ncf_profile_enable(1 if on else 0)


def profile_filter(name=None):
    """Time only launches of kernel `name` (None: every kernel)."""
    lib().ncf_profile_filter(name.encode() if name else None)


def profile_read():
    recs = (ProfileRecord * 64)()
    n = lib().ncf_profile_read(ctypes.cast(recs, ctypes.c_void_p), 64)
    return {r.name.decode(): dict(launches=r.launches, total_ms=r.total_ms, work=r.work,
                                  unit=r.work_unit.decode()) for r in recs[:n]}
