"""CPU check of the kernels' partition schedule: tests/emu/smnn_emu.cpp drives
the per-lane arithmetic of paper_2410_06074_amd/csrc/smnn_core.h through the
same level / chunk / separator indexing as the HIP kernels, one chunk at a
time, compiled with g++ (optionally under AddressSanitizer).  Compared with
the banded oracle on ragged lengths that hit every chunk-boundary case."""
import ctypes
import os
import subprocess
import sys

import numpy as np
import pytest

from oracle import banded
from tests import gpu_helpers as H
from tests import metrics
from workloads import gaussian_batch

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "emu", "smnn_emu.cpp")
BUILD = os.path.join(os.path.dirname(HERE), "paper_2410_06074_amd", "_build")


def _build(asan=False):
    os.makedirs(BUILD, exist_ok=True)
    out = os.path.join(BUILD, "libsmnn_emu%s.so" % ("_asan" if asan else ""))
    if not os.path.exists(out) or os.path.getmtime(out) < max(
            os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "..", "paper_2410_06074_amd", "csrc", "smnn_core.h"))):
        flags = ["-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer"] if asan else ["-O2"]
        subprocess.run(["g++", "-std=c++17", *flags, "-Wno-unknown-pragmas", "-shared", "-fPIC", SRC, "-o", out],
                       check=True)
    return out


_DP = ctypes.POINTER(ctypes.c_double)
_IP = ctypes.POINTER(ctypes.c_int64)


def _p(a):
    return a.ctypes.data_as(_DP)


def emu_run(lib, bt, L, refine, gy, Lu=None):
    Lu = L if Lu is None else Lu
    T = np.ascontiguousarray(bt.T, dtype=np.int64)
    u0 = np.ascontiguousarray(bt.u0)
    y = np.zeros_like(bt.c)
    assert lib.emu_forward_f64(bt.k, L, Lu, bt.n_init, ctypes.c_int64(bt.n_inst), T.ctypes.data_as(_IP), _p(bt.c),
                               _p(bt.b), _p(bt.h), _p(u0), _p(bt.w), _p(y), refine) == 0
    out = {k: np.zeros_like(v) for k, v in (("dc", bt.c), ("dd", bt.b), ("ds", bt.h), ("du0", u0), ("dw", bt.w))}
    assert lib.emu_backward_f64(bt.k, L, Lu, bt.n_init, ctypes.c_int64(bt.n_inst), T.ctypes.data_as(_IP), _p(bt.c),
                                _p(bt.b), _p(bt.h), _p(u0), _p(bt.w), _p(y), _p(gy), _p(out["dc"]), _p(out["dd"]),
                                _p(out["ds"]), _p(out["du0"]), _p(out["dw"]), refine) == 0
    out["y"] = y
    return out


CASES = [(1, 4, 4), (2, 4, 4), (2, 8, 8), (3, 4, 4), (3, 8, 8), (2, 4, 8), (3, 4, 8)]
EDGE_T = [1, 2, 3, 4, 5, 7, 8, 9, 15, 16, 17, 31, 32, 33, 64, 65, 100, 1000]


@pytest.mark.parametrize("R,L,Lu", CASES)
def test_partition_schedule_matches_oracle(R, L, Lu):
    # same pass criteria as the GPU parity tests (tests/gpu_helpers.py):
    # refine 0 is the plain FP64 solve, then the fp64r form with the library's
    # default step count (two at order 3, where one leaves ~1e-8 at cond(M) ~ 1e13)
    lib = ctypes.CDLL(_build())
    bt = gaussian_batch(len(EDGE_T), EDGE_T, R=R, seed=7 * R + L + Lu, weights=(1.3, 0.8, 1.1))
    gy = np.random.default_rng(R).standard_normal(bt.c.shape)
    ref = H.reference(bt, gy)
    kappa = banded.cond(bt)
    for refine in (0, 2 if R >= 3 else 1):
        out = emu_run(lib, bt, L, refine, gy, Lu)
        m = H.compare(bt, out, ref, range(bt.n_inst))
        print("R=%d L=%d/%d refine=%d" % (R, L, Lu, refine), H.summary(m), "kappa<=%.1e" % kappa.max())
        H.check("fp64r" if refine else "fp64", m, kappa, bt.R)


def test_partition_schedule_under_address_sanitizer():
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not asan or not os.path.exists(asan):
        pytest.skip("libasan not available")
    so = _build(asan=True)
    code = ("import sys, ctypes, numpy as np; sys.path.insert(0, %r); sys.path.insert(0, %r)\n"
            "from tests.test_emu_partition import emu_run\n"
            "from workloads import gaussian_batch\n"
            "lib = ctypes.CDLL(%r)\n"
            "for R, L, Lu in %r:\n"
            "    bt = gaussian_batch(12, [1,2,3,4,5,8,9,16,17,33,64,100], R=R, seed=R)\n"
            "    emu_run(lib, bt, L, 1, np.ones_like(bt.c), Lu)\n"
            "print('asan-clean')\n") % (os.path.dirname(HERE), HERE, so, CASES)
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and "asan-clean" in r.stdout, r.stderr[-3000:]


@pytest.mark.parametrize("t_init,n_init", [(3, 2), (9, 3), (40, 1)])
def test_partition_schedule_with_several_initial_points(t_init, n_init):
    # T_init spanning several level-0 chunks, and instances shorter than T_init
    lib = ctypes.CDLL(_build())
    T = [3, 4, 5, 9, 16, 17, 33, 100]
    bt = gaussian_batch(len(T), T, R=2, seed=t_init, n_init=n_init, weights=(1.2, 0.9, 1.3), t_init=t_init)
    gy = np.random.default_rng(t_init).standard_normal(bt.c.shape)
    ref = H.reference(bt, gy)
    kappa = banded.cond(bt)
    lib.emu_set_init_points(t_init)
    try:
        for L, Lu in ((4, 4), (4, 8)):
            out = emu_run(lib, bt, L, 1, gy, Lu)
            m = H.compare(bt, out, ref, range(bt.n_inst))
            H.check("fp64r", m, kappa, bt.R)
            for i in range(bt.n_inst):
                past = out["du0"][i].reshape(t_init, n_init)[bt.T[i]:]
                assert np.all(past == 0.0)
    finally:
        lib.emu_set_init_points(1)


@pytest.mark.parametrize("R,L", [(2, 4), (1, 8), (2, 8)])
def test_reduce_with_known_factor_matches_full_reduce(R, L):
    # the fused back-substitution + reduce kernel reuses the chunk factor of
    # its back-substitution: its separator right-hand sides must equal those
    # of the full reduce bit for bit
    lib = ctypes.CDLL(_build())
    bt = gaussian_batch(len(EDGE_T), EDGE_T, R=R, seed=90 + L, weights=(1.2, 0.7, 1.4))
    v = np.random.default_rng(L).standard_normal(bt.c.shape)
    T = np.ascontiguousarray(bt.T, dtype=np.int64)
    u0 = np.ascontiguousarray(bt.u0)
    bad = lib.emu_check_reduce_rhs_f64(bt.k, L, L, bt.n_init, ctypes.c_int64(bt.n_inst), T.ctypes.data_as(_IP),
                                       _p(bt.c), _p(bt.b), _p(bt.h), _p(u0), _p(bt.w), _p(v))
    assert bad == 0


def emu_run_gen(lib, bt, L, refine, gy):
    """The CPU emulator on a batch of any instance shape (V variables, Q
    governing equations, per-row weights)."""
    T = np.ascontiguousarray(bt.T, dtype=np.int64)
    S, N, K = bt.total_steps, bt.n_inst, bt.block
    f = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    c, d, s, u0, w = f(bt.c).reshape(S, -1), f(bt.b), f(bt.h), f(bt.u0), f(bt.w)
    wr = bt.wrow
    wg, wi, ws = (f(wr["wg"]), f(wr["wi"]), f(wr["ws"])) if wr is not None else (None, None, None)
    nul = ctypes.cast(None, _DP)
    pp = lambda a: _p(a) if a is not None else nul
    y = np.zeros((S, K))
    head = [K, L, L, bt.V, bt.Q, int(wr is not None), bt.n_init, ctypes.c_int64(N), T.ctypes.data_as(_IP)]
    arrs = [pp(x) for x in (c, d, s, u0, w, wg, wi, ws)]
    assert lib.emu_forward_gen(*head, *arrs, _p(y), refine) == 0
    out = {"dc": np.zeros_like(c), "dd": np.zeros_like(d), "ds": np.zeros_like(s), "du0": np.zeros_like(u0),
           "dw": np.zeros_like(w)}
    for key, a in (("dwg", wg), ("dwi", wi), ("dws", ws)):
        out[key] = np.zeros_like(a) if a is not None else None
    g = f(gy).reshape(S, K)
    assert lib.emu_backward_gen(*head, *arrs, _p(y), _p(g), *(pp(out[k]) for k in ("dc", "dd", "ds", "du0", "dw",
                                                                                   "dwg", "dwi", "dws")),
                                refine) == 0
    out["y"] = y
    return {k: v for k, v in out.items() if v is not None}


GEN_CASES = [  # (R, V, Q, per-row weights, chunk)
    (1, 1, 1, True, 4), (2, 1, 1, True, 4), (1, 2, 2, False, 4), (1, 2, 2, True, 4), (1, 2, 1, False, 4)]


@pytest.mark.parametrize("R,V,Q,per_row,L", GEN_CASES)
def test_general_forms_match_oracle(R, V, Q, per_row, L):
    # V coupled variables with Q governing equations, and per-row weights
    # (App. A.1-A.2): the emulated partition schedule against the __float128
    # oracle, plain and refined, on ragged lengths around the chunk boundaries
    from workloads import coupled_batch
    lib = ctypes.CDLL(_build())
    # T = 1 with fewer equations than variables has fewer rows than unknowns
    Ts = [1, 2, 3, 4, 5, 8, 9, 16, 17, 33, 64, 65, 200][0 if Q >= V else 1:]
    if V == 1:
        bt = gaussian_batch(len(Ts), Ts, R=R, seed=5 + R, weights=(1.3, 0.8, 1.1), per_row=per_row)
    else:
        bt = coupled_batch(len(Ts), Ts, R=R, V=V, Q=Q, seed=11 + Q, weights=(1.3, 0.8, 1.1), per_row=per_row)
    gy = np.random.default_rng(3).standard_normal((bt.total_steps, bt.block))
    ref = H.reference(bt, gy)
    kappa = banded.cond(bt)
    for refine in (0, 1):
        out = emu_run_gen(lib, bt, L, refine, gy)
        m = H.compare_general(bt, out, ref, range(bt.n_inst))
        print("R=%d V=%d Q=%d rows=%s refine=%d" % (R, V, Q, per_row, refine), H.summary(m),
              "kappa<=%.1e" % kappa.max())
        H.check("fp64r" if refine else "fp64", m, kappa, bt.R)
