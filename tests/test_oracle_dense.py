"""Pins for the dense oracle (oracle/dense.py) against what the paper and the
mathematics fix, independently of the oracle's own code paths."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import dense
from workloads import gaussian_batch, polynomial_batch
from tests import table5


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64); b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _inst(T, R, seed, n_init=None, weights=(1.0, 1.0, 1.0), t_init=1):
    bt = gaussian_batch(1, T, R=R, seed=seed, n_init=n_init, weights=weights, t_init=t_init)
    return bt.instance(0)


# ---------------------------------------------------------------- Eq. 8 counts
@pytest.mark.parametrize("T,R,n_init", [(1, 1, 1), (2, 2, 2), (7, 3, 1), (13, 4, 5), (5, 2, 0)])
def test_row_counts_match_eq8(T, R, n_init):
    c, d, s, u0, w = _inst(T, R, 0, n_init=n_init)
    A, b, wd = dense.weighted_system(c, d, s, u0, w)
    # Eq. 8 with V = Q = 1 and T_init = 1: m = TQ + T_init V (R_init+1) + 2 (T-1) V (R+1)
    assert A.shape == (T + n_init + 2 * (T - 1) * (R + 1), T * (R + 1))
    assert dense.constraint_counts(T, R, n_init) == A.shape


# ------------------------------------------- exact rational brute force (tiny T)
def _exact_rows(c, d, s, u0, w):
    """Constraint rows of Eqs. 4-7 with the weights before Eq. 9, in exact
    rational arithmetic from the binary64 inputs (written independently here)."""
    T, k = c.shape
    F = [[Fraction(x) for x in row] for row in c]
    D = [Fraction(x) for x in d]
    S = [Fraction(x) for x in s]
    U = [Fraction(x) for x in u0]
    Wg, Wi, Ws = (Fraction(x) for x in w)
    n = T * k
    rows = []  # (weight^2, coeffs dict, rhs)
    for t in range(T):
        rows.append((Wg * Wg, {t * k + r: F[t][r] for r in range(k)}, D[t]))
    for r in range(len(U)):
        rows.append((Wi * Wi, {r: Fraction(1)}, U[r]))
    for t in range(T - 1):
        for r in range(k):
            wt = (Ws * S[t] ** r) ** 2
            fw = {t * k + j: S[t] ** (j - r) / math.factorial(j - r) for j in range(r, k)}
            fw[(t + 1) * k + r] = fw.get((t + 1) * k + r, Fraction(0)) - 1
            rows.append((wt, fw, Fraction(0)))
            bw = {(t + 1) * k + j: (-S[t]) ** (j - r) / math.factorial(j - r) for j in range(r, k)}
            bw[t * k + r] = bw.get(t * k + r, Fraction(0)) - 1
            rows.append((wt, bw, Fraction(0)))
    M = [[Fraction(0)] * n for _ in range(n)]
    beta = [Fraction(0)] * n
    for wt, co, rhs in rows:
        for i, ai in co.items():
            beta[i] += wt * ai * rhs
            for j, aj in co.items():
                M[i][j] += wt * ai * aj
    # Gauss-Jordan elimination, exact
    aug = [M[i] + [beta[i]] for i in range(n)]
    for col in range(n):
        piv = next(r for r in range(col, n) if aug[r][col] != 0)
        aug[col], aug[piv] = aug[piv], aug[col]
        p = aug[col][col]
        aug[col] = [x / p for x in aug[col]]
        for r in range(n):
            if r != col and aug[r][col] != 0:
                f = aug[r][col]
                aug[r] = [x - f * y for x, y in zip(aug[r], aug[col])]
    return np.array([float(aug[i][n]) for i in range(n)]).reshape(T, k)


@pytest.mark.parametrize("T,R,seed", [(1, 1, 0), (2, 1, 1), (3, 2, 2), (2, 3, 3)])
def test_exact_rational_normal_equations(T, R, seed):
    c, d, s, u0, w = _inst(T, R, seed, weights=(1.3, 0.7, 2.1))
    exact = _exact_rows(c, d, s, u0, w)
    got = dense.solve(c, d, s, u0, w)
    assert _rel(got, exact) < 1e-12


# --------------------------------------------------- polynomial recovery (exact)
@pytest.mark.parametrize("R,tol", [(1, 1e-13), (2, 1e-11), (3, 1e-9), (4, 1e-7)])
def test_polynomial_trajectories_recovered(R, tol):
    # Any degree<=R polynomial satisfies the Taylor rows of Eqs. 6-7 exactly, so a
    # system built from it is consistent and the least-squares solution is p^(r)(t_k).
    bt, exact = polynomial_batch(1, 30, R, seed=10 + R)
    c, d, s, u0, w = bt.instance(0)
    y = dense.solve(c, d, s, u0, w)
    for r in range(R + 1):
        assert _rel(y[:, r], exact[:, r]) < tol
    A, b, wd = dense.weighted_system(c, d, s, u0, w)
    resid = np.sqrt(wd) * (A @ exact.reshape(-1) - b)
    assert np.abs(resid).max() < 1e-12 * max(1.0, np.abs(exact).max())


def test_single_step_closed_form():
    # T = 1: no smoothness rows; R initial values and one governing row make a
    # square system: y_r = u0_r (r < R), y_R = (d - sum_{r<R} c_r u0_r) / c_R.
    for R in (1, 2, 3, 4):
        c, d, s, u0, w = _inst(1, R, 40 + R)
        y = dense.solve(c, d, s, u0, w)[0]
        expect = np.concatenate([u0, [(d[0] - c[0, :R] @ u0) / c[0, R]]])
        assert _rel(y, expect) < 1e-14


# ------------------------------------------------------------------- App. A.2
@pytest.mark.parametrize("T,R,n_init,weights", [(1, 2, 2, (1, 1, 1)), (2, 1, 1, (2.0, 0.5, 3.0)),
                                                (6, 2, 2, (1.5, 0.3, 0.8)), (9, 3, 1, (0.2, 4.0, 1.7)),
                                                (5, 4, 5, (1.0, 1.0, 1.0))])
def test_appendix_blocks_equal_dense_normal_matrix(T, R, n_init, weights):
    c, d, s, u0, w = _inst(T, R, 7, n_init=n_init, weights=weights)
    M, beta = dense.normal_matrix(c, d, s, u0, w)
    Mb, Nb, bb = dense.normal_blocks_appendix(c, d, s, u0, w)
    k = R + 1
    scale = np.abs(M).max()
    for t in range(T):
        for u in range(T):
            blk = M[t * k:(t + 1) * k, u * k:(u + 1) * k]
            if u == t:
                ref = Mb[t]
            elif u == t - 1:
                ref = Nb[u]                  # block (t+1, t) is N_t  (Eq. 10)
            elif u == t + 1:
                ref = Nb[t].T
            else:
                ref = np.zeros((k, k))       # block-tridiagonal
            assert np.abs(blk - ref).max() <= 1e-14 * scale
    assert np.abs(beta.reshape(T, k) - bb).max() <= 1e-14 * max(1.0, np.abs(beta).max())


def test_normal_matrix_symmetric_positive_definite():
    for R, T in ((1, 12), (2, 20), (3, 9)):
        c, d, s, u0, w = _inst(T, R, 3)
        M, _ = dense.normal_matrix(c, d, s, u0, w)
        assert np.array_equal(M, M.T) or np.abs(M - M.T).max() < 1e-15 * np.abs(M).max()
        np.linalg.cholesky(M)  # raises if not positive definite


def test_solution_satisfies_normal_equations():
    c, d, s, u0, w = _inst(40, 2, 5, weights=(1.2, 0.9, 1.4))
    y = dense.solve(c, d, s, u0, w).reshape(-1)
    A, b, wd = dense.weighted_system(c, d, s, u0, w)
    g = A.T @ (wd * (b - A @ y))          # gradient of the weighted objective
    assert np.abs(g).max() < 1e-12 * (np.abs(A.T).sum(1) * np.sqrt(wd).max() ** 2).max() * max(1, np.abs(b).max())


# -------------------------------------------------------------------- Table 5
def test_table5_rc_row_reproduced():
    c, d, s, u0, w, exact, printed, tk = table5.problem("rc")
    y = dense.solve(c, d, s, u0, w)
    got = table5.rel_mse(y, exact, tk)
    assert all(table5.matches_printed(g, p) for g, p in zip(got, printed)), (got, printed)


# ------------------------------------------------------------------ gradients
@pytest.mark.parametrize("R,T,n_init,weights", [(1, 8, 1, (1.0, 1.0, 1.0)), (2, 9, 2, (1.3, 0.6, 2.2)),
                                                (3, 7, 2, (0.4, 3.0, 1.1))])
def test_closed_form_gradients_match_autograd(R, T, n_init, weights):
    c, d, s, u0, w = _inst(T, R, 11 + R, n_init=n_init, weights=weights)
    rng = np.random.default_rng(R)
    gy = rng.standard_normal((T, R + 1))
    ours = dense.grad(c, d, s, u0, w, gy)
    ref = dense.grad_autograd(c, d, s, u0, w, gy)
    # Both sides solve M lam = g in binary64 through different QR codes, so they
    # can differ by up to ~kappa(M) u; the bound below is that, with margin.
    M, _ = dense.normal_matrix(c, d, s, u0, w)
    tol = max(1e-9, 100 * np.linalg.cond(M) * np.finfo(float).eps)
    assert _rel(ours["y"], ref["y"]) < 1e-9
    scale = np.linalg.norm(np.concatenate([ref[k].ravel() for k in ("dc", "dd", "ds", "du0")]))
    for key in ("dc", "dd", "ds", "du0", "dw"):
        err = np.linalg.norm(ours[key] - ref[key])
        # dw is a sum of many cancelling row terms: measure it against the scale of the others
        denom = np.linalg.norm(ref[key]) if key != "dw" else max(np.linalg.norm(ref[key]), scale)
        assert err <= tol * denom, (key, err / denom, tol)


def test_closed_form_gradients_match_finite_differences():
    R, T = 2, 10
    c, d, s, u0, w = _inst(T, R, 21, weights=(1.1, 0.8, 1.3))
    rng = np.random.default_rng(2)
    gy = rng.standard_normal((T, R + 1))
    g = dense.grad(c, d, s, u0, w, gy)

    def loss(c_, d_, s_, u_, w_):
        return float(np.sum(gy * dense.solve(c_, d_, s_, u_, w_)))

    def fd(arr_name, idx, rel_step=1e-4):
        args = {"c": c.copy(), "d": d.copy(), "s": s.copy(), "u": u0.copy(), "w": w.copy()}
        base = args[arr_name][idx]
        h = rel_step * max(abs(base), 1e-3)
        args[arr_name][idx] = base + h
        lp = loss(args["c"], args["d"], args["s"], args["u"], args["w"])
        args[arr_name][idx] = base - h
        lm = loss(args["c"], args["d"], args["s"], args["u"], args["w"])
        return (lp - lm) / (2 * h)

    gmax = max(np.abs(g[key]).max() for key in ("dc", "dd", "ds", "du0"))
    checks = [("c", (3, 1), g["dc"][3, 1]), ("c", (0, 2), g["dc"][0, 2]), ("d", 5, g["dd"][5]),
              ("s", 2, g["ds"][2]), ("s", 8, g["ds"][8]), ("u", 1, g["du0"][1]),
              ("w", 0, g["dw"][0]), ("w", 1, g["dw"][1]), ("w", 2, g["dw"][2])]
    for name, idx, val in checks:
        ref = fd(name, idx)
        # central differences: O(h^2) truncation plus (solve rounding)/h
        assert abs(val - ref) <= 1e-5 * max(abs(ref), 1e-2 * gmax), (name, idx, val, ref)
    assert g["ds"][T - 1] == 0.0


def test_adjoint_solves_normal_system():
    # Eq. 14: dl/dbeta = M^{-1} dl/dy.
    c, d, s, u0, w = _inst(30, 2, 9)
    g = np.random.default_rng(0).standard_normal((30, 3))
    lam = dense.adjoint(c, d, s, u0, w, g).reshape(-1)
    M, _ = dense.normal_matrix(c, d, s, u0, w)
    eta = np.abs(M @ lam - g.reshape(-1)).max() / (np.abs(M).sum(1).max() * np.abs(lam).max() + np.abs(g).max())
    assert eta < 1e-13


# ---------------------------------------------- planted mistakes must be caught
def _solve_rows(A, b, wd):
    sw = np.sqrt(wd)
    return np.linalg.lstsq(sw[:, None] * A, sw * b, rcond=None)[0]


def test_planted_sign_error_in_backward_taylor_row_is_caught():
    R, T = 2, 25
    bt, exact = polynomial_batch(1, T, R, seed=3)
    c, d, s, u0, w = bt.instance(0)
    A, b, wd = dense.weighted_system(c, d, s, u0, w)
    m_gov = T + bt.n_init + (T - 1) * (R + 1)
    A_bad = A.copy()
    k = R + 1
    for t in range(T - 1):                        # backward rows: (-s_t) -> (+s_t)
        for r in range(k):
            row = m_gov + t * k + r
            for j in range(r + 1, k):
                if (j - r) % 2:
                    A_bad[row, (t + 1) * k + j] = -A_bad[row, (t + 1) * k + j]
    y_bad = _solve_rows(A_bad, b, wd).reshape(T, R + 1)
    assert _rel(y_bad, exact) > 1e-6          # the polynomial-recovery pin fails
    assert _rel(_solve_rows(A, b, wd).reshape(T, R + 1), exact) < 1e-11


def test_planted_missing_smoothness_weight_is_caught():
    c, d, s, u0, w = _inst(6, 2, 1, weights=(1.0, 1.0, 1.7))
    A, b, wd = dense.weighted_system(c, d, s, u0, w)
    T, k = 6, 3
    wd_bad = wd.copy()
    wd_bad[T + len(u0):] = w[2] ** 2              # drop the s_t^r factor
    M_bad = A.T @ (wd_bad[:, None] * A)
    Mb, _, _ = dense.normal_blocks_appendix(c, d, s, u0, w)
    assert np.abs(M_bad[:k, :k] - Mb[0]).max() > 1e-3   # the App. A.2 identity pin fails


# ------------------------------------------- initial values at T_init points
@pytest.mark.parametrize("T,R,n_init,t_init", [(6, 2, 2, 3), (4, 1, 1, 4), (3, 3, 4, 5), (9, 2, 3, 2)])
def test_row_counts_match_eq8_with_several_initial_points(T, R, n_init, t_init):
    c, d, s, u0, w = _inst(T, R, 1, n_init=n_init, t_init=t_init, weights=(1.0, 2.0, 0.5))
    A, b, wd = dense.weighted_system(c, d, s, u0, w)
    # Eq. 8: T_init V (R_init + 1) initial rows; points past T carry none
    assert A.shape == (T + min(t_init, T) * n_init + 2 * (T - 1) * (R + 1), T * (R + 1))
    init = np.flatnonzero(wd == 4.0)
    assert len(init) == min(t_init, T) * n_init
    for j, row in enumerate(init):   # row j fixes order j % n_init at point j // n_init
        t, r = divmod(j, n_init)
        assert np.flatnonzero(A[row]).tolist() == [t * (R + 1) + r] and b[row] == u0[t, r]


@pytest.mark.parametrize("T,R,n_init,t_init,weights", [(6, 2, 2, 3, (1.5, 0.3, 0.8)), (5, 3, 1, 5, (0.2, 4.0, 1.7)),
                                                       (3, 1, 2, 4, (1.0, 2.0, 1.0))])
def test_appendix_blocks_with_several_initial_points(T, R, n_init, t_init, weights):
    # App. A.2: U_t and u_t are non-zero for t <= T_init; the dense A^T W A
    # built from the rows of Eq. 5 must agree block by block
    c, d, s, u0, w = _inst(T, R, 8, n_init=n_init, weights=weights, t_init=t_init)
    M, beta = dense.normal_matrix(c, d, s, u0, w)
    Mb, Nb, bb = dense.normal_blocks_appendix(c, d, s, u0, w)
    k = R + 1
    scale = np.abs(M).max()
    for t in range(T):
        assert np.abs(M[t * k:(t + 1) * k, t * k:(t + 1) * k] - Mb[t]).max() <= 1e-14 * scale
        if t + 1 < T:
            assert np.abs(M[(t + 1) * k:(t + 2) * k, t * k:(t + 1) * k] - Nb[t]).max() <= 1e-14 * scale
    assert np.abs(beta.reshape(T, k) - bb).max() <= 1e-14 * max(1.0, np.abs(beta).max())


def test_every_unknown_fixed_by_initial_rows_returns_them():
    # T_init = T and R_init = R with only the initial rows weighted: M = w_i^2 I,
    # so y = u exactly
    T, R = 7, 2
    c, d, s, u0, w = _inst(T, R, 4, n_init=R + 1, t_init=T, weights=(0.0, 1.7, 0.0))
    y = dense.solve(c, d, s, u0, w)
    assert np.abs(y - u0).max() <= 1e-14 * np.abs(u0).max()


def test_gradients_with_several_initial_points_match_autograd_and_fd():
    R, T, t_init = 2, 8, 3
    c, d, s, u0, w = _inst(T, R, 31, n_init=2, t_init=t_init, weights=(1.2, 0.9, 1.4))
    assert u0.shape == (t_init, 2)
    gy = np.random.default_rng(4).standard_normal((T, R + 1))
    ours = dense.grad(c, d, s, u0, w, gy)
    ref = dense.grad_autograd(c, d, s, u0, w, gy)
    M, _ = dense.normal_matrix(c, d, s, u0, w)
    tol = max(1e-9, 100 * np.linalg.cond(M) * np.finfo(float).eps)
    for key in ("dc", "dd", "ds", "du0"):
        assert _rel(ours[key], ref[key]) < tol, key
    scale = np.linalg.norm(ref["dc"])
    assert np.linalg.norm(ours["dw"] - ref["dw"]) <= tol * max(np.linalg.norm(ref["dw"]), scale)
    # du at a later initial point, and the initial weight, by central differences
    for (t, r) in ((2, 1), (1, 0)):
        h = 1e-5
        up, um = u0.copy(), u0.copy()
        up[t, r] += h
        um[t, r] -= h
        fd = (np.sum(gy * dense.solve(c, d, s, up, w)) - np.sum(gy * dense.solve(c, d, s, um, w))) / (2 * h)
        assert abs(fd - ours["du0"][t, r]) <= 1e-6 * max(1.0, abs(fd))
    wp, wm = w.copy(), w.copy()
    wp[1] += 1e-5
    wm[1] -= 1e-5
    fd = (np.sum(gy * dense.solve(c, d, s, u0, wp)) - np.sum(gy * dense.solve(c, d, s, u0, wm))) / 2e-5
    assert abs(fd - ours["dw"][1]) <= 1e-6 * max(1.0, abs(fd))
