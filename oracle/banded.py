"""ctypes wrapper of the banded QR oracle ``banded.c`` (TEST INFRASTRUCTURE).

Only tests, ``__graft_entry__.smoke()`` and bench.py's cpu_baseline leg use this.
``build()`` compiles ``banded.c`` with gcc twice: in double precision into
``liboracle_banded.so`` and with ``__float128`` arithmetic (``-DORACLE_QUAD``)
into ``liboracle_banded_q.so``; ``lib()`` loads one, building first only when
no library is present.

Every function takes a ``workloads.Batch``.  ``quad=True`` selects the
__float128 build: same algorithm, inputs and outputs in double, arithmetic
with a 113-bit significand, so its results are the least-squares solution,
adjoint and gradients of the double inputs rounded once to double (pinned to
the exact rational oracle in tests/test_oracle_exact.py).

Scalar weights (``batch.wrow is None``) are expanded to the per-row weight
arrays the C code takes, and their gradients are returned as the sums of the
per-row gradients (``dw`` [N, 3], summed in the oracle's arithmetic); with
per-row weights the gradients are returned per row (``dwg``, ``dwi``, ``dws``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "banded.c")
_SO = {False: os.path.join(_HERE, "liboracle_banded.so"), True: os.path.join(_HERE, "liboracle_banded_q.so")}
_lib = {}


class _Shape(ctypes.Structure):
    _fields_ = [("R", ctypes.c_int), ("V", ctypes.c_int), ("Q", ctypes.c_int), ("n_init", ctypes.c_int),
                ("t_init", ctypes.c_int)]


def build() -> str:
    for quad, so in _SO.items():
        tmp = so + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=gnu11", _SRC, "-o", tmp, "-lm"]
        if quad:
            cmd[1:1] = ["-DORACLE_QUAD"]
            cmd.append("-lquadmath")
        subprocess.run(cmd, check=True)
        os.replace(tmp, so)
    return _SO[False]


def lib(quad: bool = False):
    quad = bool(quad)
    if quad not in _lib:
        if not os.path.exists(_SO[quad]):
            build()
        L = ctypes.CDLL(_SO[quad])
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int64)
        sp = ctypes.POINTER(_Shape)
        head = [sp, ctypes.c_int64, ip] + [dp] * 7
        L.oracle_solve.argtypes = head + [dp]
        L.oracle_solve.restype = ctypes.c_int
        L.oracle_grad.argtypes = head + [dp] * 11
        L.oracle_grad.restype = ctypes.c_int
        L.oracle_cond.argtypes = head + [ctypes.c_int, dp]
        L.oracle_cond.restype = ctypes.c_int
        L.oracle_backward_error.argtypes = head + [dp, dp, dp]
        L.oracle_backward_error.restype = ctypes.c_int
        L.oracle_max_threads.restype = ctypes.c_int
        _lib[quad] = L
    return _lib[quad]


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _dims(batch):
    V = int(getattr(batch, "V", 1))
    Q = int(getattr(batch, "Q", 1))
    t_init = int(getattr(batch, "t_init", 1))
    return V, Q, t_init


def _arrays(batch):
    """Shape struct and contiguous float64 inputs, weights expanded per row."""
    V, Q, t_init = _dims(batch)
    N, S, K = batch.n_inst, batch.total_steps, V * batch.k
    ni = t_init * V * batch.n_init
    sh = _Shape(batch.R, V, Q, batch.n_init, t_init)
    c = np.ascontiguousarray(batch.c, dtype=np.float64).reshape(S, Q * K)
    d = np.ascontiguousarray(batch.b, dtype=np.float64).reshape(S, Q)
    s = np.ascontiguousarray(batch.h, dtype=np.float64).reshape(S)
    u0 = np.ascontiguousarray(batch.u0, dtype=np.float64).reshape(N, ni)
    off = np.ascontiguousarray(batch.offsets, dtype=np.int64)
    wrow = getattr(batch, "wrow", None)
    if wrow is None:
        w = np.asarray(batch.w, dtype=np.float64).reshape(N, 3)
        per_point = np.repeat(np.arange(N), np.asarray(batch.T, dtype=np.int64))
        wg = np.ascontiguousarray(np.repeat(w[per_point, 0:1], Q, axis=1))
        ws = np.ascontiguousarray(w[per_point, 2])
        wi = np.ascontiguousarray(np.repeat(w[:, 1:2], ni, axis=1))
    else:
        wg = np.ascontiguousarray(wrow["wg"], dtype=np.float64).reshape(S, Q)
        wi = np.ascontiguousarray(wrow["wi"], dtype=np.float64).reshape(N, ni)
        ws = np.ascontiguousarray(wrow["ws"], dtype=np.float64).reshape(S)
    return sh, off, (c, d, s, u0, wg, wi, ws)


def _head(batch):
    sh, off, arrs = _arrays(batch)
    return [ctypes.byref(sh), batch.n_inst, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))] + \
        [_p(a) for a in arrs], arrs


def solve(batch, quad: bool = False) -> np.ndarray:
    """y [S, V (R+1)] for every instance (float64; quad=True: computed in __float128)."""
    V, _, _ = _dims(batch)
    head, _ = _head(batch)
    y = np.zeros((batch.total_steps, V * batch.k))
    if lib(quad).oracle_solve(*head, _p(y)):
        raise MemoryError("banded oracle: allocation failed")
    return y


def grad(batch, gy, quad: bool = False) -> dict:
    """y, lam = M^{-1} gy and the parameter gradients for dl/dy = gy."""
    V, Q, t_init = _dims(batch)
    head, (c, d, s, u0, wg, wi, ws) = _head(batch)
    K = V * batch.k
    g = np.ascontiguousarray(gy, dtype=np.float64).reshape(batch.total_steps, K)
    out = {"y": np.zeros_like(g), "lam": np.zeros_like(g), "dc": np.zeros_like(c), "dd": np.zeros_like(d),
           "ds": np.zeros_like(s), "du0": np.zeros_like(u0), "dwg": np.zeros_like(wg), "dwi": np.zeros_like(wi),
           "dws": np.zeros_like(ws), "dw": np.zeros((batch.n_inst, 3))}
    rc = lib(quad).oracle_grad(*head, _p(g), *(_p(out[k]) for k in ("y", "lam", "dc", "dd", "ds", "du0", "dwg",
                                                                      "dwi", "dws", "dw")))
    if rc:
        raise MemoryError("banded oracle: allocation failed")
    out["dc"] = out["dc"].reshape(np.shape(batch.c))
    out["dd"] = out["dd"].reshape(np.shape(batch.b))
    out["du0"] = out["du0"].reshape(np.shape(batch.u0))
    if getattr(batch, "wrow", None) is not None:
        del out["dw"]      # per-row weights: the per-row gradients are the result
    return out


def cond(batch, iters: int = 60) -> np.ndarray:
    """Estimated 2-norm condition number of each instance's normal matrix."""
    head, _ = _head(batch)
    kappa = np.zeros(batch.n_inst)
    if lib(False).oracle_cond(*head, int(iters), _p(kappa)):
        raise MemoryError("banded oracle: allocation failed")
    return kappa


def backward_error(batch, y, normwise: bool = False) -> np.ndarray:
    """Per-instance normal-equation backward error of y [S, V (R+1)],
    accumulated row by row in __float128 (independent of the conditioning).
    Row-scaled (default): ||A^T W (b - A y)||_inf / || |A|^T W (|A||y| + |b|) ||_inf.
    normwise=True: ||beta - M y||_inf / (||M||_inf ||y||_inf + ||beta||_inf)."""
    V, _, _ = _dims(batch)
    head, _ = _head(batch)
    yy = np.ascontiguousarray(y, dtype=np.float64).reshape(batch.total_steps, V * batch.k)
    eta_c = np.zeros(batch.n_inst)
    eta_n = np.zeros(batch.n_inst)
    if lib(True).oracle_backward_error(*head, _p(yy), _p(eta_c), _p(eta_n)):
        raise MemoryError("banded oracle: allocation failed")
    return eta_n if normwise else eta_c


def threads() -> int:
    return int(lib(False).oracle_max_threads())
