"""CPU check of the wide-block routines (paper_2410_06074_amd/csrc/smnn_wide.h:
one 16-lane group per chunk, a row of every block per lane): tests/emu/
smnn_wide_emu.cpp runs the 16 rows as threads that meet at every broadcast,
through the same level / chunk schedule as the wide kernels, and the result
is compared with the __float128 oracle (coupled variables, App. A.1-A.2)."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from oracle import banded
from tests import gpu_helpers as H
from workloads import coupled_batch

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "emu", "smnn_wide_emu.cpp")
BUILD = os.path.join(os.path.dirname(HERE), "paper_2410_06074_amd", "_build")
DEPS = [SRC] + [os.path.join(HERE, "..", "paper_2410_06074_amd", "csrc", f) for f in ("smnn_wide.h", "smnn_core.h")]


def _build():
    os.makedirs(BUILD, exist_ok=True)
    out = os.path.join(BUILD, "libsmnn_wide_emu.so")
    if not os.path.exists(out) or os.path.getmtime(out) < max(os.path.getmtime(f) for f in DEPS):
        subprocess.run(["g++", "-std=c++17", "-O2", "-Wno-unknown-pragmas", "-shared", "-fPIC", "-pthread", SRC,
                        "-o", out], check=True)
    return out


_DP = ctypes.POINTER(ctypes.c_double)
_IP = ctypes.POINTER(ctypes.c_int64)


def run_wide(lib, bt, refine, gy, L=4):
    T = np.ascontiguousarray(bt.T, dtype=np.int64)
    S, N, K = bt.total_steps, bt.n_inst, bt.block
    f = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    c, d, s, u0, w = f(bt.c).reshape(S, -1), f(bt.b), f(bt.h), f(bt.u0), f(bt.w)
    wr = bt.wrow
    wg, wi, ws = (f(wr["wg"]), f(wr["wi"]), f(wr["ws"])) if wr is not None else (None, None, None)
    nul = ctypes.cast(None, _DP)
    pp = lambda a: a.ctypes.data_as(_DP) if a is not None else nul
    head = [K, L, bt.V, bt.Q, int(wr is not None), bt.n_init, ctypes.c_int64(N), T.ctypes.data_as(_IP)]
    arrs = [pp(x) for x in (c, d, s, u0, None if wr is not None else w, wg, wi, ws)]
    y = np.zeros((S, K))
    assert lib.emu_wide_forward(*head, *arrs, pp(y), refine) == 0
    out = {"dc": np.zeros_like(c), "dd": np.zeros_like(d), "ds": np.zeros_like(s), "du0": np.zeros_like(u0),
           "dw": np.zeros_like(w)}
    for key, a in (("dwg", wg), ("dwi", wi), ("dws", ws)):
        out[key] = np.zeros_like(a) if a is not None else None
    g = f(gy).reshape(S, K)
    assert lib.emu_wide_backward(*head, *arrs, pp(y), pp(g),
                                 *(pp(out[k]) for k in ("dc", "dd", "ds", "du0", "dw", "dwg", "dwi", "dws")),
                                 refine) == 0
    out["y"] = y
    out["dc"] = out["dc"].reshape(np.shape(bt.c))
    out["dd"] = out["dd"].reshape(np.shape(bt.b))
    return {k: v for k, v in out.items() if v is not None}


WIDE = [(2, 2, 2, False), (1, 3, 3, False), (2, 3, 3, True)]   # (R, V, Q, per-row weights)


@pytest.mark.parametrize("R,V,Q,rows", WIDE)
def test_wide_routines_match_oracle(R, V, Q, rows):
    lib = ctypes.CDLL(_build())
    # one chunk; two and three chunks (one level of separators); T = 21: a
    # second separator level (chunks of 4 at every level)
    Ts = [1, 5, 9, 21]
    bt = coupled_batch(len(Ts), Ts, R=R, V=V, Q=Q, seed=60 + 10 * V + R, weights=(1.3, 0.8, 1.1), per_row=rows,
                       h0=0.05)
    gy = np.random.default_rng(V + R).standard_normal((bt.total_steps, bt.block))
    ref = H.reference(bt, gy)
    kappa = banded.cond(bt)
    for refine in (0, 1):
        out = run_wide(lib, bt, refine, gy)
        m = H.compare_general(bt, out, ref, range(bt.n_inst))
        print("wide R=%d V=%d Q=%d rows=%s refine=%d" % (R, V, Q, rows, refine), H.summary(m),
              "kappa<=%.1e" % kappa.max(), flush=True)
        H.check("fp64r" if refine else "fp64", m, kappa, bt.R)
