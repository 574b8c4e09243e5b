"""Property tests over the problem space: order R = 1..4, T = 1..64 (with a
few longer ragged instances), n_init = 0..R+1, T_init = 1..3, weights
log-uniform in [0.1, 10], steps in [1e-3, 1e-1].  The oracle's banded QR is
checked against the dense definition, the kernels' partition schedule
(tests/emu, on the CPU) against the oracle, and (marked gpu) the HIP path
against the oracle.  Cases whose normal matrix is singular or too badly
conditioned for FP64 comparisons (cond(M) > 1e12) are discarded; the
bounds are the least-squares forward error ~cond(M) u and a backward error
(normal-equation residual) of 1e-13 that holds at any conditioning."""
import ctypes

import numpy as np
import pytest
from hypothesis import HealthCheck, assume, given, settings
from hypothesis import strategies as st

from oracle import banded, dense
from tests import metrics
from workloads import Batch

SETTINGS = dict(max_examples=40, deadline=None, derandomize=True,
                suppress_health_check=[HealthCheck.too_slow, HealthCheck.filter_too_much])


@st.composite
def problems(draw, max_inst=1, max_T=64):
    R = draw(st.integers(1, 4))
    n_inst = draw(st.integers(1, max_inst))
    T = [draw(st.integers(1, max_T)) for _ in range(n_inst)]
    n_init = draw(st.integers(0, R + 1))
    t_init = draw(st.integers(1, 3))
    seed = draw(st.integers(0, 2 ** 31 - 1))
    h_lo = draw(st.sampled_from([1e-3, 1e-2]))
    rng = np.random.default_rng(seed)
    S, k = int(sum(T)), R + 1
    c = rng.standard_normal((S, k))
    c[:, R] = np.sign(c[:, R]) * (0.5 + np.abs(c[:, R]))
    b = rng.standard_normal(S)
    h = np.exp(rng.uniform(np.log(h_lo), np.log(1e-1), S))
    u0 = rng.standard_normal((n_inst, t_init * n_init))
    w = np.exp(rng.uniform(np.log(0.1), np.log(10.0), (n_inst, 3)))
    return Batch(R=R, n_init=n_init, T=np.asarray(T, dtype=np.int64), c=c, b=b, h=h, u0=u0, w=w,
                 name="property", t_init=t_init)


def _usable(bt):
    """cond(M) per instance, or None when an instance is rank deficient or
    cond(M) > 1e12 (beyond what FP64 comparisons resolve)."""
    for i in range(bt.n_inst):
        c, d, s, u0, w = bt.instance(i)
        A, _, wd = dense.weighted_system(c, d, s, u0, w)
        if A.shape[0] < A.shape[1]:
            return None
        sv = np.linalg.svd(np.sqrt(wd)[:, None] * A, compute_uv=False)
        if sv[-1] <= 0 or (sv[0] / sv[-1]) ** 2 > 1e12:
            return None
    return banded.cond(bt)


def backward_error(bt, y):
    """max over instances of ||A^T W (b - A y)||_inf / || |A|^T W (|A||y| + |b|) ||_inf,
    evaluated in extended precision from the dense rows of Eqs. 4-7: the
    normal equations (Eq. 9) hold to rounding for any backward-stable solve."""
    L = np.longdouble
    o = bt.offsets
    worst = 0.0
    for i in range(bt.n_inst):
        c, d, s, u0, w = bt.instance(i)
        A, b, wd = dense.weighted_system(c, d, s, u0, w)
        A, b, wd = A.astype(L), b.astype(L), wd.astype(L)
        yi = np.asarray(y[o[i]:o[i + 1]], dtype=L).ravel()
        g = A.T @ (wd * (b - A @ yi))
        scale = np.abs(A).T @ (wd * (np.abs(A) @ np.abs(yi) + np.abs(b)))
        worst = max(worst, float(np.abs(g).max() / scale.max()))
    return worst


def _lsq_tol(kappa, floor):
    # least-squares forward error: ~cond(M) u when the residual is not zero
    return max(floor, 10.0 * float(np.max(kappa)) * np.finfo(float).eps)


@settings(**SETTINGS)
@given(problems())
def test_banded_oracle_matches_dense_definition(bt):
    kappa = _usable(bt)
    assume(kappa is not None)
    c, d, s, u0, w = bt.instance(0)
    yd = dense.solve(c, d, s, u0, w)
    yb = banded.solve(bt)
    assert np.linalg.norm(yb - yd) <= _lsq_tol(kappa, 1e-12) * np.linalg.norm(yd)
    assert backward_error(bt, yb) <= 1e-13


@settings(**SETTINGS)
@given(problems(max_inst=4, max_T=80))
def test_partition_schedule_matches_oracle(bt):
    from tests.test_emu_partition import _build, emu_run
    kappa = _usable(bt)
    assume(kappa is not None)
    lib = ctypes.CDLL(_build())
    gy = np.random.default_rng(0).standard_normal(bt.c.shape)
    ref = banded.grad(bt, gy)
    lib.emu_set_init_points(bt.t_init)
    try:
        out = emu_run(lib, bt, 4, 1, gy, 4)
    finally:
        lib.emu_set_init_points(1)
    assert backward_error(bt, out["y"]) <= 1e-13
    o = bt.offsets
    for i in range(bt.n_inst):
        sl = slice(o[i], o[i + 1])
        assert max(metrics.rel_by_order(out["y"][sl], ref["y"][sl], bt.k)) <= _lsq_tol(kappa[i], 1e-10), i


@pytest.mark.gpu
@settings(**dict(SETTINGS, max_examples=25))
@given(problems(max_inst=6, max_T=200))
def test_hip_path_matches_oracle(bt):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from tests import gpu_helpers as H
    kappa = _usable(bt)
    assume(kappa is not None)
    gy = np.random.default_rng(1).standard_normal(bt.c.shape)
    ref = H.reference(bt, gy)          # the __float128 oracle
    out = H.run(bt, "fp64r", gy)
    assert (out["info"] == 0).all()
    assert backward_error(bt, out["y"]) <= 1e-13
    m = H.compare(bt, out, ref, range(bt.n_inst))
    # P1 on every instance, P2 (1e-10 per order and element by element) and
    # the gradient bound (1e-10, term-scaled) where cond(M) <= 1e14
    H.check("fp64r", m, kappa, bt.R)
