"""Pins for the exact rational oracle (oracle/exact.py), and through it for the
double and __float128 banded oracles.

The rational oracle has no rounding, so its pins are exact equalities where
the mathematics gives one (polynomial recovery, the T = 1 closed form, the
App. A.2 block formulas) and an O(eps^2) bound where it gives a limit
(central differences of the loss)."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import banded, dense, exact
from workloads import Batch, gaussian_batch


def _rel_max(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _poly_instance(T, R, V, seed):
    """Rational inputs whose constraints are consistent: per variable a
    polynomial p_v of degree R with rational coefficients; Q = V governing rows
    per point with random rational coefficients over all variables; d and the
    initial values are evaluated exactly from p."""
    rng = np.random.default_rng(seed)
    k, K = R + 1, V * (R + 1)
    Fr = lambda x: Fraction(int(x), 64)
    s = np.array([Fraction(int(rng.integers(1, 9)), 256) for _ in range(T)], dtype=object)
    tk = [Fraction(0)]
    for t in range(T - 1):
        tk.append(tk[-1] + s[t])
    coef = [[Fr(rng.integers(-64, 65)) for _ in range(k)] for _ in range(V)]

    def deriv(v, r, x):   # p_v^(r)(x)
        return sum((coef[v][j] * math.factorial(j) / math.factorial(j - r) * x ** (j - r) for j in range(r, k)),
                   Fraction(0))

    exact_y = np.array([[deriv(v, r, tk[t]) for v in range(V) for r in range(k)] for t in range(T)], dtype=object)
    Q = V
    c = np.array([[[Fr(rng.integers(-64, 65)) for _ in range(K)] for _ in range(Q)] for _ in range(T)], dtype=object)
    d = np.array([[sum((c[t, q, j] * exact_y[t, j] for j in range(K)), Fraction(0)) for q in range(Q)]
                  for t in range(T)], dtype=object)
    n_init = R
    u = np.array([[[deriv(v, r, tk[0]) for r in range(n_init)] for v in range(V)]], dtype=object)
    one = lambda shape: np.full(shape, Fraction(1), dtype=object)
    wg, wi, ws = one((T, Q)), np.full(u.shape, Fraction(3, 2), dtype=object), np.full(T, Fraction(5, 4), dtype=object)
    return (c, d, s, u, wg, wi, ws), exact_y


@pytest.mark.parametrize("T,R,V", [(1, 1, 1), (4, 1, 1), (6, 2, 1), (5, 3, 1), (4, 1, 2), (3, 2, 2)])
def test_polynomial_trajectories_recovered_exactly(T, R, V):
    # A degree <= R polynomial satisfies the Taylor rows of Eqs. 6-7 exactly,
    # so the constraints are consistent and the least-squares solution equals
    # p^(r)(t_k) with zero residual -- exactly, in rational arithmetic.
    args, want = _poly_instance(T, R, V, seed=T + 10 * R + 100 * V)
    y = exact.solve(R, *args)
    assert (y == want).all()
    for sig, co, rhs, _, _ in exact.rows(R, *args):
        assert sum((a * want.reshape(-1)[i] for i, a in co.items()), Fraction(0)) == rhs


def test_single_step_closed_form_exact():
    # T = 1: R initial values plus one governing row fix the R + 1 unknowns:
    # y_r = u_r (r < R), y_R = (d - sum_{r<R} c_r u_r) / c_R.
    for R in (1, 2, 3, 4):
        bt = gaussian_batch(1, 1, R=R, seed=40 + R)
        c, d, s, u, wg, wi, ws = bt.instance_general(0)
        y = exact.solve(R, c, d, s, u, wg, wi, ws)[0]
        C = [Fraction(x) for x in c[0, 0]]
        U = [Fraction(x) for x in u[0, 0]]
        want = U + [(Fraction(d[0, 0]) - sum(C[r] * U[r] for r in range(R))) / C[R]]
        assert list(y) == want


@pytest.mark.parametrize("T,R,weights", [(2, 1, (2.0, 0.5, 3.0)), (6, 2, (1.5, 0.3, 0.8)), (4, 3, (0.2, 4.0, 1.7))])
def test_normal_matrix_equals_appendix_blocks(T, R, weights):
    # App. A.2's block formulas (written out in oracle/dense.py) against the
    # exact row-by-row accumulation of A^T W A and A^T W b.
    bt = gaussian_batch(1, T, R=R, seed=7, weights=weights)
    M, beta = exact.normal(R, *bt.instance_general(0))
    Mb, Nb, bb = dense.normal_blocks_appendix(*bt.instance(0))
    k = R + 1
    Mf = exact.to_float(np.array(M, dtype=object))
    scale = np.abs(Mf).max()
    for t in range(T):
        assert np.abs(Mf[t * k:(t + 1) * k, t * k:(t + 1) * k] - Mb[t]).max() <= 1e-14 * scale
        if t + 1 < T:
            assert np.abs(Mf[(t + 1) * k:(t + 2) * k, t * k:(t + 1) * k] - Nb[t]).max() <= 1e-14 * scale
    assert _rel_max(exact.to_float(np.array(beta, dtype=object)), bb.reshape(-1)) <= 1e-15
    # nothing outside the block tridiagonal band
    for i in range(T * k):
        for j in range(T * k):
            if abs(i // k - j // k) > 1:
                assert M[i][j] == 0


def test_coupled_block_diagonal_system_splits_into_scalar_solves():
    # With V = 2 variables and governing rows that each touch one variable
    # only, the normal equations decouple: the solution equals the two V = 1
    # solutions (App. A.2: M_t couples variables only through C_t^T C_t).
    T, R = 5, 2
    k = R + 1
    a = gaussian_batch(1, T, R=R, seed=1, weights=(1.2, 0.7, 0.9))
    b = gaussian_batch(1, T, R=R, seed=2, weights=(1.2, 0.7, 0.9))
    ca, da, s, ua, wg, wi, ws = a.instance_general(0)
    cb, db, _, ub, _, _, _ = b.instance_general(0)
    c = np.zeros((T, 2, 2 * k))
    c[:, 0, :k] = ca[:, 0]
    c[:, 1, k:] = cb[:, 0]
    d = np.stack([da[:, 0], db[:, 0]], axis=1)
    u = np.concatenate([ua, ub], axis=1)
    y = exact.solve(R, c, d, s, u, np.full((T, 2), 1.2), np.full(u.shape, 0.7), ws)
    ya = exact.solve(R, ca, da, s, ua, wg, wi, ws)
    yb = exact.solve(R, cb, db, s, ub, wg, wi, ws)
    assert (y[:, :k] == ya).all() and (y[:, k:] == yb).all()


@pytest.mark.parametrize("T,R,V,per_row", [(4, 1, 1, False), (3, 2, 1, True), (3, 1, 2, True)])
def test_gradients_equal_exact_central_differences(T, R, V, per_row):
    # Every gradient entry against (l(theta + e) - l(theta - e)) / 2e of the
    # exact loss l = sum(g y): the difference is O(e^2) = 1e-40 relative.
    rng = np.random.default_rng(T + R + V)
    k, K, Q = R + 1, V * (R + 1), V
    c = rng.standard_normal((T, Q, K))
    for q in range(Q):
        c[:, q, q * k + R] = 1.0 + np.abs(c[:, q, q * k + R])
    d = rng.standard_normal((T, Q))
    s = 0.05 * (0.5 + rng.random(T))
    u = rng.standard_normal((1, V, R))
    if per_row:
        wg, wi, ws = 0.5 + rng.random((T, Q)), 0.5 + rng.random((1, V, R)), 0.5 + rng.random(T)
    else:
        wg, wi, ws = np.full((T, Q), 1.3), np.full((1, V, R), 0.8), np.full(T, 1.1)
    g = rng.standard_normal((T, K))
    ex = exact.grad(R, c, d, s, u, wg, wi, ws, g)
    args = [exact._F(x) for x in (c, d, s, u, wg, wi, ws)]
    eps = Fraction(1, 10 ** 20)
    names = ["dc", "dd", "ds", "du", "dwg", "dwi", "dws"]
    for a, name in enumerate(names):
        arr = args[a]
        for idx in np.ndindex(arr.shape):
            if name in ("ds", "dws") and idx[0] == T - 1:
                assert ex[name][idx] == 0     # the last step slot enters no row
                continue
            plus = [x.copy() for x in args]
            minus = [x.copy() for x in args]
            plus[a][idx] += eps
            minus[a][idx] -= eps
            fd = (exact.loss(R, *plus, g) - exact.loss(R, *minus, g)) / (2 * eps)
            scale = max(abs(ex[name][idx]), Fraction(1, 10 ** 6))
            assert abs(fd - ex[name][idx]) <= Fraction(1, 10 ** 30) * scale, (name, idx)


@pytest.mark.parametrize("T,R,V,seed", [(5, 1, 1, 0), (9, 2, 1, 1), (17, 2, 1, 2), (7, 3, 1, 3), (6, 1, 2, 4)])
def test_banded_oracles_agree_with_exact(T, R, V, seed):
    # The __float128 banded QR rounds to the same doubles as the exact
    # solution (its own error is ~1e-30); the double banded QR is within the
    # least-squares bound.
    rng = np.random.default_rng(seed)
    k, K, Q = R + 1, V * (R + 1), V
    c = rng.standard_normal((T, Q, K))
    for q in range(Q):
        c[:, q, q * k + R] = 1.0 + np.abs(c[:, q, q * k + R])
    wrow = {"wg": 0.5 + rng.random((T, Q)), "wi": 0.5 + rng.random((1, V * R)), "ws": 0.5 + rng.random(T)}
    bt = Batch(R=R, n_init=R, T=np.array([T]), c=c.reshape(T, Q * K) if V > 1 else c.reshape(T, K),
               b=rng.standard_normal((T, Q)) if Q > 1 else rng.standard_normal(T), h=0.05 * (0.5 + rng.random(T)), u0=rng.standard_normal((1, V * R)),
               w=np.ones((1, 3)), V=V, Q=Q, wrow=wrow)
    g = rng.standard_normal((T, K))
    ex = exact.grad(R, *bt.instance_general(0), g)
    q = banded.grad(bt, g, quad=True)
    dd = banded.grad(bt, g)
    kappa = float(banded.cond(bt)[0])
    for key, kq in (("y", "y"), ("lam", "lam"), ("dc", "dc"), ("dd", "dd"), ("ds", "ds"), ("du", "du0"),
                    ("dwg", "dwg"), ("dwi", "dwi"), ("dws", "dws")):
        e = exact.to_float(ex[key]).ravel()
        assert _rel_max(q[kq], e) <= 2 ** -52, key
        assert _rel_max(dd[kq], e) <= max(1e-13, 100 * kappa * 2 ** -53), key


@pytest.mark.parametrize("case", range(2))
def test_quad_oracle_reproduces_exact_fixture(case):
    # tests/golden/exact_small.json holds the rational oracle's values (written
    # by tests/golden/make_exact.py); the __float128 banded QR must round to
    # the same doubles
    from tests import fixtures
    bt, gy, want = fixtures.load_exact(case)
    q = banded.grad(bt, gy, quad=True)
    for key in ("y", "lam", "dc", "dd", "ds", "du0", "dw"):
        assert _rel_max(q[key], want[key]) <= 2 ** -52, key


@pytest.mark.parametrize("case", range(8))
def test_quad_oracle_reproduces_exact_general_fixture(case):
    # tests/golden/exact_general.json: per-row weights and two or three
    # coupled variables (App. A.1-A.2), rational oracle rounded to double
    from tests import fixtures
    bt, gy, want = fixtures.load_exact_general(case)
    q = banded.grad(bt, gy, quad=True)
    for key in want:
        assert _rel_max(q[key], want[key]) <= 2 ** -52, key


@pytest.mark.parametrize("T,R,V,Q", [(3, 1, 1, 1), (6, 2, 2, 2), (4, 1, 3, 2), (2, 3, 2, 1)])
def test_row_counts_of_eq8_with_variables_and_equations(T, R, V, Q):
    # Eq. 8 with V variables and Q equations: m = T Q + T_init V (R_init + 1)
    # + 2 (T - 1) V (R + 1) rows over n = T V (R + 1) unknowns, each kind
    # touching only its own point(s)
    rng = np.random.default_rng(T + R + V + Q)
    k, K = R + 1, V * (R + 1)
    c = rng.standard_normal((T, Q, K))
    rows = exact.rows(R, c, rng.standard_normal((T, Q)), 0.01 * (1 + rng.random(T)), rng.standard_normal((1, V, R)),
                      np.ones((T, Q)), np.ones((1, V, R)), np.ones(T))
    kinds = [r[3] for r in rows]
    assert kinds.count("gov") == T * Q
    assert kinds.count("init") == V * R
    assert kinds.count("fwd") == kinds.count("bwd") == (T - 1) * V * k
    assert len(rows) == T * Q + V * R + 2 * (T - 1) * V * k
    for sig, co, rhs, kind, key in rows:
        t = key[0]
        cols = sorted(co)
        if kind in ("gov", "init"):
            assert all(t * K <= j < (t + 1) * K for j in cols)
        else:
            v = key[1]
            assert all(j % K // k == v for j in cols)           # one variable only
            assert all(t * K <= j < (t + 2) * K for j in cols)
