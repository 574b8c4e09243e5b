"""Exact rational oracle for tiny instances (TEST INFRASTRUCTURE).

Only tests and the script that writes ``tests/golden/exact_*.json`` use this.

Every binary64 input is a rational number, and so is everything the solve
computes from it: the weighted rows of Eqs. 4-7 (the smoothness weight
w_smooth s_t^r is rational), the normal equations of Eq. 9, their solution,
the adjoint of Eq. 14 and the per-row gradients.  Here all of it is carried
out in ``fractions.Fraction`` with no rounding at all, in the plainest form:

  rows        the weighted constraint rows of one instance (App. A.1), general
              V variables and Q governing equations per point, per-row
              weights (scalar weights are the case of equal entries).
  normal      M = A^T W A and beta = A^T W b accumulated row by row (the two
              products before Eq. 10).
  solve_spd   Gaussian elimination of M x = v restricted to the band of M
              (exact; M is symmetric positive definite, so no pivoting).
  solve       y of Eq. 9.
  grad        y, lam = M^{-1} g (Eq. 14) and the closed-form per-row
              gradients: a row a~.y = b~ with residual rho = a~.y - b~ and
              mu = a~.lam gives a parameter theta of that row
              -[(da~/dtheta . lam) rho + mu (da~/dtheta . y - db~/dtheta)].
  loss        sum(g * y) exactly, for central differences.

Pinned in tests/test_oracle_exact.py: polynomial trajectories give an exactly
zero residual and exactly p^(r)(t_k); the T = 1 closed form; the normal
matrix equals the App. A.2 block formulas of oracle/dense.py; every gradient
equals an exact central difference of ``loss`` to O(eps^2); the double and
__float128 banded oracles agree with it.

Instance arguments are the arrays of ``workloads.Batch.instance_general``:
c [T, Q, K], d [T, Q], s [T], u [t_init, V, n_init], wg [T, Q],
wi [t_init, V, n_init], ws [T], with K = V (R+1).
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


def _F(a):
    return np.vectorize(Fraction, otypes=[object])(np.asarray(a, dtype=np.float64))


def _frac_inputs(c, d, s, u, wg, wi, ws):
    return tuple(_F(a) if not (isinstance(a, np.ndarray) and a.dtype == object) else a
                 for a in (c, d, s, u, wg, wi, ws))


def rows(R, c, d, s, u, wg, wi, ws):
    """Weighted rows (sigma, {column: coefficient}, rhs, kind, key) of one
    instance, all Fractions.  sigma is the row's weight (W holds sigma^2)."""
    c, d, s, u, wg, wi, ws = _frac_inputs(c, d, s, u, wg, wi, ws)
    T, Q, K = c.shape
    k = R + 1
    V = K // k
    t_init, _, n_init = u.shape
    out = []
    for t in range(T):                                   # Eq. 4
        for q in range(Q):
            out.append((wg[t, q], {t * K + j: c[t, q, j] for j in range(K) if c[t, q, j] != 0}, d[t, q],
                        "gov", (t, q)))
    for t in range(min(t_init, T)):                      # Eq. 5
        for v in range(V):
            for r in range(n_init):
                out.append((wi[t, v, r], {t * K + v * k + r: Fraction(1)}, u[t, v, r], "init", (t, v, r)))
    for t in range(T - 1):                               # Eqs. 6-7, weight ws_t s_t^r
        st = s[t]
        for v in range(V):
            for r in range(k):
                sig = ws[t] * st ** r
                fw = {t * K + v * k + j: st ** (j - r) / math.factorial(j - r) for j in range(r, k)}
                fw[(t + 1) * K + v * k + r] = fw.get((t + 1) * K + v * k + r, Fraction(0)) - 1
                out.append((sig, fw, Fraction(0), "fwd", (t, v, r)))
                bw = {(t + 1) * K + v * k + j: (-st) ** (j - r) / math.factorial(j - r) for j in range(r, k)}
                bw[t * K + v * k + r] = bw.get(t * K + v * k + r, Fraction(0)) - 1
                out.append((sig, bw, Fraction(0), "bwd", (t, v, r)))
    return out


def normal(R, c, d, s, u, wg, wi, ws):
    """(M [n][n], beta [n]) as lists of Fractions."""
    T, _, K = np.shape(c)
    n = T * K
    M = [[Fraction(0)] * n for _ in range(n)]
    beta = [Fraction(0)] * n
    for sig, co, rhs, _, _ in rows(R, c, d, s, u, wg, wi, ws):
        w2 = sig * sig
        for i, ai in co.items():
            beta[i] += w2 * ai * rhs
            for j, aj in co.items():
                M[i][j] += w2 * ai * aj
    return M, beta


def solve_spd(M, v, band):
    """x with M x = v, M symmetric positive definite with M[i][j] = 0 for
    |i - j| > band; Gaussian elimination without pivoting, exact."""
    n = len(v)
    A = [row[:] for row in M]
    x = list(v)
    for j in range(n):
        p = A[j][j]
        if p <= 0:
            raise ZeroDivisionError("normal matrix is not positive definite")
        for i in range(j + 1, min(n, j + band + 1)):
            f = A[i][j] / p
            if f == 0:
                continue
            for l in range(j, min(n, j + band + 1)):
                A[i][l] -= f * A[j][l]
            x[i] -= f * x[j]
    for j in range(n - 1, -1, -1):
        acc = x[j]
        for l in range(j + 1, min(n, j + band + 1)):
            acc -= A[j][l] * x[l]
        x[j] = acc / A[j][j]
    return x


def solve(R, c, d, s, u, wg, wi, ws):
    """y [T, K] of Eq. 9, Fractions."""
    T, _, K = np.shape(c)
    M, beta = normal(R, c, d, s, u, wg, wi, ws)
    return np.array(solve_spd(M, beta, 2 * K - 1), dtype=object).reshape(T, K)


def _row_derivatives(R, s, ws, key, kind):
    """d(a~)/ds_t of a smoothness row as {column offset: value}: columns of
    the row's own variable, offsets 0..k-1 at point t, k..2k-1 at t+1."""
    t, v, r = key
    k = R + 1
    st = s[t]
    out = {}
    if kind == "fwd":     # sigma a = ws (sum_j s^j/(j-r)! y_{t,j} - s^r y_{t+1,r})
        for j in range(r, k):
            if j > 0:
                out[j] = ws[t] * j * st ** (j - 1) / math.factorial(j - r)
        if r > 0:
            out[k + r] = out.get(k + r, Fraction(0)) - ws[t] * r * st ** (r - 1)
    else:                 # sigma a = ws (sum_j (-1)^{j-r} s^j/(j-r)! y_{t+1,j} - s^r y_{t,r})
        for j in range(r, k):
            if j > 0:
                out[k + j] = ws[t] * (-1) ** (j - r) * j * st ** (j - 1) / math.factorial(j - r)
        if r > 0:
            out[r] = out.get(r, Fraction(0)) - ws[t] * r * st ** (r - 1)
    return out


def grad(R, c, d, s, u, wg, wi, ws, g):
    """Exact y, lam and gradients of l with dl/dy = g.  Returns a dict of
    object arrays (Fractions): y, lam [T, K]; dc [T, Q, K]; dd, dwg [T, Q];
    ds, dws [T] (last slot 0); du, dwi [t_init, V, n_init]."""
    c, d, s, u, wg, wi, ws = _frac_inputs(c, d, s, u, wg, wi, ws)
    T, Q, K = c.shape
    k = R + 1
    n = T * K
    M, beta = normal(R, c, d, s, u, wg, wi, ws)
    y = solve_spd(M, beta, 2 * K - 1)
    gf = [Fraction(x) for x in np.asarray(g, dtype=np.float64).reshape(-1)] if np.asarray(g).dtype != object \
        else list(np.asarray(g).reshape(-1))
    lam = solve_spd(M, gf, 2 * K - 1)
    dc = np.full(c.shape, Fraction(0), dtype=object)
    dd = np.full(d.shape, Fraction(0), dtype=object)
    dwg = np.full(d.shape, Fraction(0), dtype=object)
    ds = np.full(T, Fraction(0), dtype=object)
    dws = np.full(T, Fraction(0), dtype=object)
    du = np.full(u.shape, Fraction(0), dtype=object)
    dwi = np.full(u.shape, Fraction(0), dtype=object)
    for sig, co, rhs, kind, key in rows(R, c, d, s, u, wg, wi, ws):
        a_y = sum((ai * y[i] for i, ai in co.items()), Fraction(0))
        a_l = sum((ai * lam[i] for i, ai in co.items()), Fraction(0))
        rho = sig * (a_y - rhs)          # weighted residual
        mu = sig * a_l                   # weighted adjoint row value
        if kind == "gov":
            t, q = key
            for j in range(K):           # d(a~)/dc_j = sig e_j
                dc[t, q, j] = -(sig * lam[t * K + j] * rho + mu * sig * y[t * K + j])
            dd[t, q] = mu * sig          # d(b~)/dd = sig
            dwg[t, q] = -(a_l * rho + mu * (a_y - rhs))
        elif kind == "init":
            t, v, r = key
            du[t, v, r] = mu * sig       # d(b~)/du = sig
            dwi[t, v, r] = -(a_l * rho + mu * (a_y - rhs))
        else:
            t, v, r = key
            der = _row_derivatives(R, s, ws, key, kind)
            base = t * K + v * k
            dl = sum((val * lam[base + off if off < k else base + K + off - k] for off, val in der.items()),
                     Fraction(0))
            dy = sum((val * y[base + off if off < k else base + K + off - k] for off, val in der.items()),
                     Fraction(0))
            ds[t] += -(dl * rho + mu * dy)
            dws[t] += -(rho * mu + mu * rho) / ws[t]   # sigma is linear in ws_t
    return {"y": np.array(y, dtype=object).reshape(T, K), "lam": np.array(lam, dtype=object).reshape(T, K),
            "dc": dc, "dd": dd, "dwg": dwg, "ds": ds, "dws": dws, "du": du, "dwi": dwi}


def loss(R, c, d, s, u, wg, wi, ws, g):
    """sum(g * y) exactly (g rational)."""
    y = solve(R, c, d, s, u, wg, wi, ws).reshape(-1)
    gf = np.asarray(g).reshape(-1)
    return sum((Fraction(gi) * yi for gi, yi in zip(gf, y)), Fraction(0))


def to_float(a) -> np.ndarray:
    """Round an object array of Fractions to float64 (correctly rounded)."""
    return np.vectorize(float, otypes=[np.float64])(np.asarray(a, dtype=object))
