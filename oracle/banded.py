"""ctypes wrapper of the banded QR oracle ``banded.c`` (TEST INFRASTRUCTURE).

Only tests, ``__graft_entry__.smoke()`` and bench.py's cpu_baseline leg use this.
``build()`` compiles ``banded.c`` with gcc into ``liboracle_banded.so`` beside it;
``lib()`` loads it, building first only when no library is present.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "banded.c")
_SO = os.path.join(_HERE, "liboracle_banded.so")
_lib = None


def build() -> str:
    tmp = _SO + ".tmp"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", _SRC, "-o", tmp, "-lm"],
                   check=True)
    os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int64)
        L.oracle_solve.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64, ip] + [dp] * 6
        L.oracle_solve.restype = ctypes.c_int
        L.oracle_grad.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64, ip] + [dp] * 13
        L.oracle_grad.restype = ctypes.c_int
        L.oracle_max_threads.restype = ctypes.c_int
        L.oracle_cond.argtypes = ([ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64, ip] + [dp] * 5
                                  + [ctypes.c_int, dp])
        L.oracle_cond.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _t_init(batch) -> int:
    return int(getattr(batch, "t_init", 1))


def _arrays(batch):
    c = np.ascontiguousarray(batch.c, dtype=np.float64)
    b = np.ascontiguousarray(batch.b, dtype=np.float64)
    h = np.ascontiguousarray(batch.h, dtype=np.float64)
    u0 = np.ascontiguousarray(batch.u0, dtype=np.float64).reshape(batch.n_inst, _t_init(batch) * batch.n_init)
    w = np.ascontiguousarray(batch.w, dtype=np.float64)
    off = np.ascontiguousarray(batch.offsets, dtype=np.int64)
    return c, b, h, u0, w, off


def solve(batch) -> np.ndarray:
    """y [S, R+1] for every instance of a ``workloads.Batch`` (float64)."""
    c, b, h, u0, w, off = _arrays(batch)
    y = np.zeros_like(c)
    rc = lib().oracle_solve(batch.R, batch.n_init, _t_init(batch), batch.n_inst,
                            off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                            _p(c), _p(b), _p(h), _p(u0), _p(w), _p(y))
    if rc:
        raise MemoryError("banded oracle: allocation failed")
    return y


def grad(batch, gy) -> dict:
    """y, lam = M^{-1} gy and the parameter gradients for dl/dy = gy."""
    c, b, h, u0, w, off = _arrays(batch)
    g = np.ascontiguousarray(gy, dtype=np.float64).reshape(c.shape)
    out = {k: np.zeros_like(v) for k, v in (("y", c), ("lam", c), ("dc", c), ("dd", b), ("ds", h),
                                            ("du0", u0), ("dw", w))}
    rc = lib().oracle_grad(batch.R, batch.n_init, _t_init(batch), batch.n_inst,
                           off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                           _p(c), _p(b), _p(h), _p(u0), _p(w), _p(g), _p(out["y"]), _p(out["lam"]),
                           _p(out["dc"]), _p(out["dd"]), _p(out["ds"]), _p(out["du0"]), _p(out["dw"]))
    if rc:
        raise MemoryError("banded oracle: allocation failed")
    return out


def cond(batch, iters: int = 60) -> np.ndarray:
    """Estimated 2-norm condition number of each instance's normal matrix."""
    c, b, h, u0, w, off = _arrays(batch)
    kappa = np.zeros(batch.n_inst)
    rc = lib().oracle_cond(batch.R, batch.n_init, _t_init(batch), batch.n_inst,
                           off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                           _p(c), _p(b), _p(h), _p(u0), _p(w), int(iters), _p(kappa))
    if rc:
        raise MemoryError("banded oracle: allocation failed")
    return kappa


def threads() -> int:
    return int(lib().oracle_max_threads())
