"""Pins for the banded QR oracle (oracle/banded.c): cross-checked against the
dense definition on small sizes, and against closed forms at long T."""
import numpy as np
import pytest

from oracle import banded, dense
from workloads import config, gaussian_batch, polynomial_batch
from tests import table5


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def _per_instance(bt, arr, i):
    o = bt.offsets
    return arr[o[i]:o[i + 1]]


@pytest.mark.parametrize("name,R", [("c0", 2), ("c2", 2), ("c3", 3)])
def test_banded_matches_dense_on_config_distributions(name, R):
    bt = config(name, n_inst=3, T=60 if name != "c3" else 90)
    yb = banded.solve(bt)
    for i in range(bt.n_inst):
        c, d, s, u0, w = bt.instance(i)
        yd = dense.solve(c, d, s, u0, w)
        M, _ = dense.normal_matrix(c, d, s, u0, w)
        # both are backward-stable QR solves of the same problem: kappa(A) u, kappa(A)^2 = kappa(M)
        tol = max(1e-12, 100 * np.sqrt(np.linalg.cond(M)) * np.finfo(float).eps)
        for r in range(bt.k):
            assert _rel(_per_instance(bt, yb, i)[:, r], yd[:, r]) < tol


@pytest.mark.parametrize("R", [1, 2, 3, 4])
def test_banded_matches_dense_ragged_with_edge_lengths(R):
    bt = gaussian_batch(5, [1, 2, 3, 17, 33], R=R, seed=100 + R, weights=(1.4, 0.6, 0.9))
    yb = banded.solve(bt)
    for i in range(bt.n_inst):
        c, d, s, u0, w = bt.instance(i)
        yd = dense.solve(c, d, s, u0, w)
        assert _rel(_per_instance(bt, yb, i), yd) < {1: 1e-13, 2: 1e-12, 3: 1e-10, 4: 1e-8}[R]


def test_banded_gradients_match_dense():
    bt = gaussian_batch(3, [1, 9, 40], R=2, seed=5, weights=(1.2, 0.7, 1.6))
    gy = np.random.default_rng(1).standard_normal(bt.c.shape)
    gb = banded.grad(bt, gy)
    o = bt.offsets
    for i in range(bt.n_inst):
        c, d, s, u0, w = bt.instance(i)
        gd = dense.grad(c, d, s, u0, w, gy[o[i]:o[i + 1]])
        M, _ = dense.normal_matrix(c, d, s, u0, w)
        tol = max(1e-10, 100 * np.linalg.cond(M) * np.finfo(float).eps)
        for key in ("lam", "dc", "dd", "ds"):
            assert _rel(gb[key][o[i]:o[i + 1]], gd[key]) < tol, key
        assert _rel(gb["du0"][i], gd["du0"]) < tol
        scale = np.linalg.norm(gd["dc"])
        assert np.linalg.norm(gb["dw"][i] - gd["dw"]) <= tol * max(np.linalg.norm(gd["dw"]), scale)


def test_banded_polynomial_recovery_long_sequence():
    bt, exact = polynomial_batch(2, 20000, 2, seed=7)
    y = banded.solve(bt)
    # relative error grows with the dynamic range of p^(r) over the interval
    for r, tol in zip(range(3), (1e-11, 1e-9, 1e-7)):
        assert _rel(y[:, r], exact[:, r]) < tol


@pytest.mark.parametrize("name", ["rc", "population", "language"])
def test_banded_reproduces_table5(name):
    c, d, s, u0, w, exact, printed, tk = table5.problem(name)
    from workloads import Batch
    bt = Batch(R=2, n_init=1, T=np.array([len(d)]), c=c, b=d, h=s, u0=u0[None, :], w=w[None, :])
    y = banded.solve(bt)
    got = table5.rel_mse(y, exact, tk)
    assert all(table5.matches_printed(g, p) for g, p in zip(got, printed)), (got, printed)


def test_banded_backward_error_long_sequence():
    # The weighted normal equations A^T W (b - A y) = 0 hold to rounding at any T;
    # the residual is evaluated row by row in extended precision.
    bt = config("h", n_inst=1, T=3000)
    y = banded.solve(bt)
    c, d, s, u0, w = bt.instance(0)
    T, k = c.shape
    L = np.longdouble
    yl = y.astype(L)
    g = np.zeros((T, k), dtype=L)
    absg = np.zeros((T, k), dtype=L)
    import math
    e = (c.astype(L) * yl).sum(1) - d.astype(L)
    g -= (L(w[0]) ** 2) * c.astype(L) * e[:, None]
    absg += (L(w[0]) ** 2) * np.abs(c.astype(L)) * (np.abs(c.astype(L) * yl).sum(1) + np.abs(d))[:, None]
    for r in range(len(u0)):
        g[0, r] -= L(w[1]) ** 2 * (yl[0, r] - L(u0[r]))
    for t in range(T - 1):
        st = L(s[t])
        for r in range(k):
            wr = L(w[2]) * st ** r
            af = np.zeros(2 * k, dtype=L); ab = np.zeros(2 * k, dtype=L)
            for j in range(r, k):
                af[j] = wr * st ** (j - r) / math.factorial(j - r)
                ab[k + j] = wr * (-st) ** (j - r) / math.factorial(j - r)
            af[k + r] -= wr
            ab[r] -= wr
            yy = np.concatenate([yl[t], yl[t + 1]])
            for a in (af, ab):
                rho = a @ yy
                g[t] -= a[:k] * rho; g[t + 1] -= a[k:] * rho
                absg[t] += np.abs(a[:k]) * (np.abs(a) @ np.abs(yy)); absg[t + 1] += np.abs(a[k:]) * (np.abs(a) @ np.abs(yy))
    eta = float(np.abs(g).max() / np.abs(absg).max())
    assert eta < 1e-14


def test_condition_estimate_matches_dense_svd():
    from oracle import dense as D
    bt = gaussian_batch(2, [6, 60], R=2, seed=4)
    kap = banded.cond(bt)
    for i in range(bt.n_inst):
        c, d, s, u0, w = bt.instance(i)
        M, _ = D.normal_matrix(c, d, s, u0, w)
        ref = np.linalg.cond(M)
        assert abs(kap[i] - ref) <= 0.05 * ref


@pytest.mark.parametrize("t_init,n_init", [(2, 2), (5, 1), (40, 3)])
def test_banded_matches_dense_with_several_initial_points(t_init, n_init):
    # ragged lengths below, at and above T_init; points past an instance's end
    # carry no initial row and get a zero gradient
    bt = gaussian_batch(4, [1, 3, 5, 30], R=2, seed=60 + t_init, n_init=n_init, weights=(1.2, 0.8, 1.5),
                        t_init=t_init)
    gy = np.random.default_rng(t_init).standard_normal(bt.c.shape)
    gb = banded.grad(bt, gy)
    o = bt.offsets
    for i in range(bt.n_inst):
        c, d, s, u0, w = bt.instance(i)
        if bt.T[i] * bt.k > bt.T[i] + min(t_init, bt.T[i]) * n_init + 2 * (bt.T[i] - 1) * bt.k:
            continue   # fewer rows than unknowns: not solvable
        gd = dense.grad(c, d, s, u0, w, gy[o[i]:o[i + 1]])
        M, _ = dense.normal_matrix(c, d, s, u0, w)
        tol = max(1e-10, 100 * np.linalg.cond(M) * np.finfo(float).eps)
        assert _rel(gb["y"][o[i]:o[i + 1]], gd["y"]) < tol
        for key in ("lam", "dc", "dd", "ds"):
            assert _rel(gb[key][o[i]:o[i + 1]], gd[key]) < tol, key
        assert _rel(gb["du0"][i], gd["du0"].ravel()) < tol
        assert np.all(gb["du0"][i].reshape(t_init, n_init)[bt.T[i]:] == 0.0)
