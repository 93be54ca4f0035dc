"""TEST INFRASTRUCTURE ONLY -- ctypes loader for the FP64 CPU oracle.

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this module. The product library never
does. See ``ncf_oracle.c`` for what is computed and which passages of the
paper each step follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ncf_oracle.c")
_LIB = os.path.join(_HERE, "libncf_oracle.so")

GAUSSIAN = 0
RECTANGLE = 1

OK = 0
E_INVALID_ARG = -1
E_UNSORTED = -2
E_DEGENERATE = -3


def build(force: bool = False) -> str:
    """Compile the oracle with gcc: FP64, no fast-math, no FMA contraction."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-fPIC", "-shared", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        d = ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_acf.argtypes = [ctypes.c_int64, d, d, d, ctypes.c_int64, d, ctypes.c_int,
                                   ctypes.c_double, d, d, i64p, ctypes.c_int, ctypes.c_int]
        lib.oracle_ccf.argtypes = [ctypes.c_int64, d, d, d, ctypes.c_int64, d, d, d,
                                   ctypes.c_int64, d, ctypes.c_int, ctypes.c_double, d, d, i64p,
                                   ctypes.c_int, ctypes.c_int]
        lib.oracle_acf_regular.argtypes = [ctypes.c_int64, d, d, d, ctypes.c_double,
                                           ctypes.c_int64, d, ctypes.c_int, ctypes.c_double, d,
                                           d, i64p, ctypes.c_int]
        lib.oracle_ccf_regular.argtypes = [ctypes.c_int64, d, d, d, ctypes.c_int64, d, d, d,
                                           ctypes.c_double, ctypes.c_int64, d, ctypes.c_int,
                                           ctypes.c_double, d, d, i64p, ctypes.c_int]
        lib.oracle_window_sums.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, d, d, d,
                                           ctypes.c_int64, d, d, d, ctypes.c_int64, d,
                                           ctypes.c_double, d, d, d, i64p, ctypes.c_int,
                                           ctypes.c_int]
        lib.oracle_standardize.argtypes = [ctypes.c_int64, d, d, d, d]
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def kernel_id(kernel) -> int:
    if isinstance(kernel, str):
        return {"gaussian": GAUSSIAN, "g": GAUSSIAN, "rectangle": RECTANGLE, "r": RECTANGLE}[
            kernel.lower()]
    return int(kernel)


def acf(t, x, lags, kernel, h, err=None, threads=0, brute=False):
    """FP64 real-space ACF. Returns (status, c, b, count)."""
    lib = _load()
    t, x, err, lags = _f64(t), _f64(x), _f64(err), _f64(lags)
    K = lags.size
    c = np.zeros(K)
    b = np.zeros(K)
    cnt = np.zeros(K, dtype=np.int64)
    st = lib.oracle_acf(t.size, _dp(t), _dp(x), _dp(err), K, _dp(lags), kernel_id(kernel),
                        float(h), _dp(c), _dp(b),
                        cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), int(threads),
                        int(bool(brute)))
    return st, c, b, cnt


def ccf(t, x, s, y, lags, kernel, h, ex=None, ey=None, threads=0, brute=False):
    """FP64 real-space CCF (lag +tau: y lags x by tau). Returns (status, c, b, count)."""
    lib = _load()
    t, x, s, y, ex, ey, lags = (_f64(a) for a in (t, x, s, y, ex, ey, lags))
    K = lags.size
    c = np.zeros(K)
    b = np.zeros(K)
    cnt = np.zeros(K, dtype=np.int64)
    st = lib.oracle_ccf(t.size, _dp(t), _dp(x), _dp(ex), s.size, _dp(s), _dp(y), _dp(ey), K,
                        _dp(lags), kernel_id(kernel), float(h), _dp(c), _dp(b),
                        cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), int(threads),
                        int(bool(brute)))
    return st, c, b, cnt


def acf_regular(t, x, lags, dt, kernel, h, err=None, threads=0):
    """FP64 ACF in the lattice reading (times at t[0] + m dt). Returns (status, c, b, count)."""
    lib = _load()
    t, x, err, lags = _f64(t), _f64(x), _f64(err), _f64(lags)
    K = lags.size
    c = np.zeros(K)
    b = np.zeros(K)
    cnt = np.zeros(K, dtype=np.int64)
    st = lib.oracle_acf_regular(t.size, _dp(t), _dp(x), _dp(err), float(dt), K, _dp(lags),
                                kernel_id(kernel), float(h), _dp(c), _dp(b),
                                cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), int(threads))
    return st, c, b, cnt


def ccf_regular(t, x, s, y, lags, dt, kernel, h, ex=None, ey=None, threads=0):
    """FP64 CCF in the lattice reading (both series on min(t[0], s[0]) + m dt)."""
    lib = _load()
    t, x, s, y, ex, ey, lags = (_f64(a) for a in (t, x, s, y, ex, ey, lags))
    K = lags.size
    c = np.zeros(K)
    b = np.zeros(K)
    cnt = np.zeros(K, dtype=np.int64)
    st = lib.oracle_ccf_regular(t.size, _dp(t), _dp(x), _dp(ex), s.size, _dp(s), _dp(y),
                                _dp(ey), float(dt), K, _dp(lags), kernel_id(kernel), float(h),
                                _dp(c), _dp(b), cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                int(threads))
    return st, c, b, cnt


def window_sums(kernel, eps, s, v_out, w_out, t, v_win, w_win, lags, h, threads=0, brute=False):
    """Raw window sums (C, B, b, count) per lag, no floor, no normalization."""
    lib = _load()
    s, v_out, w_out, t, v_win, w_win, lags = (_f64(a) for a in
                                              (s, v_out, w_out, t, v_win, w_win, lags))
    K = lags.size
    C = np.zeros(K)
    B = np.zeros(K)
    b = np.zeros(K)
    cnt = np.zeros(K, dtype=np.int64)
    st = lib.oracle_window_sums(kernel_id(kernel), int(eps), s.size, _dp(s), _dp(v_out),
                                _dp(w_out), t.size, _dp(t), _dp(v_win), _dp(w_win), K,
                                _dp(lags), float(h), _dp(C), _dp(B), _dp(b),
                                cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                int(threads), int(bool(brute)))
    return st, C, B, b, cnt


def standardize(x, err=None):
    lib = _load()
    x, err = _f64(x), _f64(err)
    v = np.zeros(x.size)
    w = np.zeros(x.size)
    st = lib.oracle_standardize(x.size, _dp(x), _dp(err), _dp(v), _dp(w))
    return st, v, w


def _replicate(t, x, err, sigma, z, mult, r):
    """Replicate r by its definition: values perturbed by sigma * z[r], then
    sample i written out mult[r, i] times (0 drops it)."""
    xr = np.asarray(x, float) + (np.asarray(sigma, float) * z[r] if z is not None else 0.0)
    if mult is None:
        return np.asarray(t, float), xr, err
    idx = np.repeat(np.arange(len(t)), mult[r])
    return np.asarray(t, float)[idx], xr[idx], (None if err is None else np.asarray(err)[idx])


def _rep_stats(cs):
    """Per-lag mean and sample sd over the replicates whose estimate is a number."""
    C = np.array(cs)
    mean = np.array([np.mean(col[~np.isnan(col)]) if np.any(~np.isnan(col)) else np.nan
                     for col in C.T])
    sd = np.array([np.std(col[~np.isnan(col)], ddof=1) if np.sum(~np.isnan(col)) > 1 else np.nan
                   for col in C.T])
    return mean, sd


def acf_resample(t, x, lags, kernel, h, err=None, sigma=None, z=None, mult=None, threads=0):
    """Replicate ACFs (flux randomization and/or bootstrap by repetition of
    samples). Returns (statuses, c_rep[R, K], c_mean, c_sd)."""
    R = (z if z is not None else mult).shape[0]
    sts, cs = [], []
    for r in range(R):
        tr, xr, er = _replicate(t, x, err, sigma, z, mult, r)
        st, c, _, _ = acf(tr, xr, lags, kernel, h, err=er, threads=threads)
        sts.append(st)
        cs.append(c if st == OK else np.full(len(lags), np.nan))
    mean, sd = _rep_stats(cs)
    return np.array(sts), np.array(cs), mean, sd


def ccf_resample(t, x, s, y, lags, kernel, h, ex=None, ey=None, sx=None, sy=None, zx=None,
                 zy=None, multx=None, multy=None, threads=0):
    """Replicate CCFs, each series resampled with its own draws."""
    R = next(a.shape[0] for a in (zx, multx, zy, multy) if a is not None)
    sts, cs = [], []
    for r in range(R):
        tr, xr, er = _replicate(t, x, ex, sx, zx, multx, r)
        sr, yr, fr = _replicate(s, y, ey, sy, zy, multy, r)
        st, c, _, _ = ccf(tr, xr, sr, yr, lags, kernel, h, ex=er, ey=fr, threads=threads)
        sts.append(st)
        cs.append(c if st == OK else np.full(len(lags), np.nan))
    mean, sd = _rep_stats(cs)
    return np.array(sts), np.array(cs), mean, sd
