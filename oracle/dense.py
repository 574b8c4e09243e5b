"""Dense definition of the S-MNN weighted least-squares solve (TEST INFRASTRUCTURE).

Only tests, ``__graft_entry__.smoke()`` and bench.py's cpu_baseline leg may use
this module.  Everything is float64 NumPy (plus torch float64 on the CPU for
the autograd pin); sizes are limited by the dense m x n matrix (T up to ~1500
for R = 2).

One instance = one (batch, variable) pair, i.e. V = Q = 1 in the paper's
notation.  ``u0`` holds the initial values of Eq. 5: a vector of n_init =
R_init + 1 values fixes orders 0..R_init at the first time point (T_init = 1);
a [T_init, n_init] array fixes them at each of the first T_init points (points
past the instance's last one are ignored, and their gradients are zero).

Functions and what pins them (tests/test_oracle_dense.py):
  weighted_system   App. A.1 (A, b, W) built row by row from Eqs. 4-7 and the
                    weighting paragraph before Eq. 9.  Pinned by: Eq. 8 row
                    counts; exact recovery of degree<=R polynomial trajectories;
                    the T = 1 closed form; Table 5 (RC, population, language
                    rows reproduce the printed relative MSE); App. A.2 block
                    formulas (an independent statement of A^T W A).
  solve             Eq. 9 as the least-squares minimiser via Householder QR.
                    Pinned by an exact rational solve of the normal equations at
                    tiny T, and the pins above.
  normal_blocks_appendix
                    App. A.2 formulas for M_t, N_t, beta_t written out.  Pinned
                    against the dense A^T W A (two independent statements).
  adjoint           Eq. 14: dl/dbeta = M^{-1} dl/dy, via the QR triangular factor.
  grad_rows         Closed-form per-row gradients of a loss w.r.t. c, d, s, u, w
                    (derived from Eq. 14 and App. A.3 by the chain rule through
                    each weighted row).  Pinned against torch autograd through
                    the dense QR solve and against central finite differences.
  grad_autograd     torch float64 autograd through the dense QR solve.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg


def constraint_counts(T: int, R: int, n_init: int, t_init: int = 1):
    """Eq. 8 with V = Q = 1, R_init + 1 = n_init and T_init = t_init (capped
    at T): (m, n)."""
    m = T + min(t_init, T) * n_init + 2 * (T - 1) * (R + 1)
    n = T * (R + 1)
    return m, n


def init_values(u0):
    """u0 as a [T_init, n_init] array (a vector is one initial point)."""
    u = np.asarray(u0, dtype=np.float64)
    return u.reshape(1, -1) if u.ndim <= 1 else u


def weighted_system(c, d, s, u0, w):
    """Return (A, b, wdiag) of App. A.1 for one instance.

    c  [T, R+1]  governing coefficients c_{t,r}      (Eq. 4)
    d  [T]       governing right-hand side d_t        (Eq. 4)
    s  [T]       s_t = step between points t and t+1; s[T-1] unused (Eqs. 6-7)
    u0 [n_init] or [T_init, n_init]  initial values u_{t,r}, t < T_init,
                 r < n_init                           (Eq. 5)
    w  [3]       (w_gov, w_init, w_smooth), unsquared (weighting before Eq. 9)

    Rows are ordered [governing; initial; forward smoothness; backward
    smoothness] and unknowns as y[t*(R+1) + r] (the time-major order before
    Eq. 10).  W = diag(wdiag) holds w_gov^2, w_init^2 and (w_smooth s_t^r)^2.
    """
    c = np.asarray(c, dtype=np.float64)
    T, k = c.shape
    R = k - 1
    U = init_values(u0)
    t_init, n_init = U.shape
    m, n = constraint_counts(T, R, n_init, t_init)
    A = np.zeros((m, n))
    b = np.zeros(m)
    wd = np.zeros(m)
    row = 0
    # governing equations, Eq. 4: sum_r c_{t,r} y_{t,r} = d_t
    for t in range(T):
        A[row, t * k:(t + 1) * k] = c[t]
        b[row] = d[t]
        wd[row] = w[0] ** 2
        row += 1
    # initial values, Eq. 5: y_{t,r} = u_{t,r} for t <= T_init, r <= R_init
    for t in range(min(t_init, T)):
        for r in range(n_init):
            A[row, t * k + r] = 1.0
            b[row] = U[t, r]
            wd[row] = w[1] ** 2
            row += 1
    # forward smoothness, Eq. 6: y_{t+1,r} = sum_{r'>=r} s_t^{r'-r}/(r'-r)! y_{t,r'}
    for t in range(T - 1):
        for r in range(k):
            for rp in range(r, k):
                A[row, t * k + rp] = s[t] ** (rp - r) / math.factorial(rp - r)
            A[row, (t + 1) * k + r] = -1.0
            wd[row] = (w[2] * s[t] ** r) ** 2
            row += 1
    # backward smoothness, Eq. 7: y_{t,r} = sum_{r'>=r} (-s_t)^{r'-r}/(r'-r)! y_{t+1,r'}
    for t in range(T - 1):
        for r in range(k):
            for rp in range(r, k):
                A[row, (t + 1) * k + rp] = (-s[t]) ** (rp - r) / math.factorial(rp - r)
            A[row, t * k + r] = -1.0
            wd[row] = (w[2] * s[t] ** r) ** 2
            row += 1
    assert row == m
    return A, b, wd


def _qr(c, d, s, u0, w):
    A, b, wd = weighted_system(c, d, s, u0, w)
    sw = np.sqrt(wd)
    Q, Rf = np.linalg.qr(sw[:, None] * A, mode="reduced")
    return Q, Rf, sw * b


def solve(c, d, s, u0, w):
    """Eq. 9: y = argmin_y || W^{1/2} (A y - b) ||_2, returned as [T, R+1]."""
    T, k = np.shape(c)
    Q, Rf, sb = _qr(c, d, s, u0, w)
    y = scipy.linalg.solve_triangular(Rf, Q.T @ sb, lower=False)
    return y.reshape(T, k)


def normal_matrix(c, d, s, u0, w):
    """Dense M = A^T W A and beta = A^T W b (the two products before Eq. 10)."""
    A, b, wd = weighted_system(c, d, s, u0, w)
    return A.T @ (wd[:, None] * A), A.T @ (wd * b)


def normal_blocks_appendix(c, d, s, u0, w):
    """App. A.2 written out for V = Q = 1, R_init = n_init - 1 and any T_init.

    Returns (Mb [T,k,k], Nb [T-1,k,k], beta [T,k]) where Nb[t] is the block in
    block-row t+1, block-column t of M (Eq. 10)."""
    c = np.asarray(c, dtype=np.float64)
    T, k = c.shape
    R = k - 1
    Uv = init_values(u0)
    t_init, n_init = Uv.shape
    F = np.zeros((k, k))
    for i in range(k):
        for j in range(i, k):
            F[i, j] = 1.0 / math.factorial(j - i)
    U = np.diag([1.0 if r < n_init else 0.0 for r in range(k)])

    def uvec(t):
        return np.array([Uv[t, r] if r < n_init else 0.0 for r in range(k)])

    def Sp(t):
        return np.diag([s[t] ** r for r in range(k)])

    def Sm(t):
        return np.diag([(-s[t]) ** r for r in range(k)])

    def S2(t):
        return np.diag([s[t] ** (2 * r) for r in range(k)])

    def Sstar(t):
        if T == 1:
            return np.zeros((k, k))
        if t == 0:
            return Sp(0).T @ F.T @ F @ Sp(0) + S2(0)
        if t == T - 1:
            return Sm(T - 2).T @ F.T @ F @ Sm(T - 2) + S2(T - 2)
        return (Sp(t).T @ F.T @ F @ Sp(t) + Sm(t - 1).T @ F.T @ F @ Sm(t - 1)
                + S2(t) + S2(t - 1))

    def Sstarstar(t):
        return -Sp(t).T @ F @ Sp(t) - Sm(t).T @ F.T @ Sm(t)

    wg2, wi2, ws2 = w[0] ** 2, w[1] ** 2, w[2] ** 2
    Mb = np.zeros((T, k, k))
    Nb = np.zeros((max(T - 1, 0), k, k))
    beta = np.zeros((T, k))
    for t in range(T):
        Ct = c[t][None, :]
        Ut = U if t < t_init else np.zeros((k, k))
        ut = uvec(t) if t < t_init else np.zeros(k)
        Mb[t] = wg2 * Ct.T @ Ct + wi2 * Ut + ws2 * Sstar(t)
        beta[t] = wg2 * Ct.T[:, 0] * d[t] + wi2 * ut
    for t in range(T - 1):
        Nb[t] = ws2 * Sstarstar(t)
    return Mb, Nb, beta


def adjoint(c, d, s, u0, w, g):
    """Eq. 14: dl/dbeta = M^{-1} g with M = R^T R from the QR of W^{1/2} A."""
    T, k = np.shape(c)
    _, Rf, _ = _qr(c, d, s, u0, w)
    z = scipy.linalg.solve_triangular(Rf, np.asarray(g, dtype=np.float64).reshape(-1), trans="T", lower=False)
    lam = scipy.linalg.solve_triangular(Rf, z, lower=False)
    return lam.reshape(T, k)


def grad_rows(c, d, s, u0, w, y, lam):
    """Closed-form gradients of a loss l given y (Eq. 9) and lam = M^{-1} dl/dy.

    For a weighted row (a~ . y = b~) with residual rho = a~.y - b~ and
    mu = a~.lam, the chain rule through Eq. 14 gives, for any parameter theta
    entering that row,
        dl/dtheta = -[ (da~/dtheta . lam) rho + mu (da~/dtheta . y - db~/dtheta) ].
    Summed over the rows that contain each parameter.  Returns a dict with
    dc [T,k], dd [T], ds [T] (ds[T-1] = 0), du0 (the shape of u0), dw [3]."""
    c = np.asarray(c, dtype=np.float64)
    T, k = c.shape
    U = init_values(u0)
    t_init, n_init = U.shape
    y = np.asarray(y).reshape(T, k)
    lam = np.asarray(lam).reshape(T, k)
    wg, wi, ws = (float(v) for v in w)
    dc = np.zeros((T, k))
    dd = np.zeros(T)
    ds = np.zeros(T)
    du0 = np.zeros((t_init, n_init))
    dw = np.zeros(3)
    # governing rows: a~ = wg c_t, b~ = wg d_t
    for t in range(T):
        e = c[t] @ y[t] - d[t]
        f = c[t] @ lam[t]
        dc[t] = -wg * wg * (e * lam[t] + f * y[t])
        dd[t] = wg * wg * f
        dw[0] += -2.0 * wg * e * f
    # initial rows: a~ = wi e_{t,r}, b~ = wi u_{t,r}
    for t in range(min(t_init, T)):
        for r in range(n_init):
            du0[t, r] = wi * wi * lam[t, r]
            dw[1] += -2.0 * wi * (y[t, r] - U[t, r]) * lam[t, r]
    # smoothness rows between t and t+1 (weighted by w_s s^r)
    for t in range(T - 1):
        st = s[t]
        for r in range(k):
            for direction in (+1, -1):
                a_t = np.zeros(k)
                a_n = np.zeros(k)
                da_t = np.zeros(k)
                da_n = np.zeros(k)
                if direction > 0:
                    # ws s^r (sum_{j>=r} s^{j-r}/(j-r)! y_{t,j} - y_{t+1,r})
                    for j in range(r, k):
                        a_t[j] = ws * st ** j / math.factorial(j - r)
                        da_t[j] = ws * j * st ** (j - 1) / math.factorial(j - r) if j > 0 else 0.0
                    a_n[r] = -ws * st ** r
                    da_n[r] = -ws * r * st ** (r - 1) if r > 0 else 0.0
                else:
                    # ws s^r (sum_{j>=r} (-s)^{j-r}/(j-r)! y_{t+1,j} - y_{t,r})
                    for j in range(r, k):
                        sign = -1.0 if (j - r) % 2 else 1.0
                        a_n[j] = ws * sign * st ** j / math.factorial(j - r)
                        da_n[j] = ws * sign * j * st ** (j - 1) / math.factorial(j - r) if j > 0 else 0.0
                    a_t[r] = -ws * st ** r
                    da_t[r] = -ws * r * st ** (r - 1) if r > 0 else 0.0
                rho = a_t @ y[t] + a_n @ y[t + 1]
                mu = a_t @ lam[t] + a_n @ lam[t + 1]
                dlam = da_t @ lam[t] + da_n @ lam[t + 1]
                dy = da_t @ y[t] + da_n @ y[t + 1]
                ds[t] += -(dlam * rho + mu * dy)
                dw[2] += -2.0 * rho * mu / ws
    return {"dc": dc, "dd": dd, "ds": ds, "du0": du0.reshape(np.shape(u0)), "dw": dw}


def grad(c, d, s, u0, w, gy):
    """y, lam and the closed-form gradients for the loss with dl/dy = gy."""
    y = solve(c, d, s, u0, w)
    lam = adjoint(c, d, s, u0, w, gy)
    out = grad_rows(c, d, s, u0, w, y, lam)
    out["y"] = y
    out["lam"] = lam
    return out


def grad_autograd(c, d, s, u0, w, gy):
    """torch float64 autograd of sum(gy * y) through the dense QR solve."""
    import torch

    T, k = np.shape(c)
    t_init, n_init = init_values(u0).shape
    tc = torch.tensor(np.asarray(c, dtype=np.float64), requires_grad=True)
    td = torch.tensor(np.asarray(d, dtype=np.float64), requires_grad=True)
    ts = torch.tensor(np.asarray(s, dtype=np.float64), requires_grad=True)
    tu = torch.tensor(init_values(u0), requires_grad=True)
    tw = torch.tensor(np.asarray(w, dtype=np.float64), requires_grad=True)
    rows_a, rows_b, rows_w = [], [], []
    zero = torch.zeros((), dtype=torch.float64)
    for t in range(T):
        a = torch.zeros(T * k, dtype=torch.float64)
        a = a.index_put((torch.arange(t * k, (t + 1) * k),), tc[t])
        rows_a.append(a); rows_b.append(td[t]); rows_w.append(tw[0])
    for t in range(min(t_init, T)):
        for r in range(n_init):
            a = torch.zeros(T * k, dtype=torch.float64)
            a[t * k + r] = 1.0
            rows_a.append(a); rows_b.append(tu[t, r]); rows_w.append(tw[1])
    for direction in (+1, -1):
        for t in range(T - 1):
            for r in range(k):
                idx, val = [], []
                if direction > 0:
                    for rp in range(r, k):
                        idx.append(t * k + rp); val.append(ts[t] ** (rp - r) / math.factorial(rp - r))
                    idx.append((t + 1) * k + r); val.append(-torch.ones((), dtype=torch.float64))
                else:
                    for rp in range(r, k):
                        idx.append((t + 1) * k + rp); val.append((-ts[t]) ** (rp - r) / math.factorial(rp - r))
                    idx.append(t * k + r); val.append(-torch.ones((), dtype=torch.float64))
                a = torch.zeros(T * k, dtype=torch.float64).index_put((torch.tensor(idx),), torch.stack(val))
                rows_a.append(a); rows_b.append(zero); rows_w.append(tw[2] * ts[t] ** r)
    A = torch.stack(rows_a)
    b = torch.stack(rows_b)
    sw = torch.stack(rows_w)
    Q, Rf = torch.linalg.qr(sw[:, None] * A, mode="reduced")
    y = torch.linalg.solve_triangular(Rf, (Q.T @ (sw * b))[:, None], upper=True)[:, 0]
    loss = (torch.as_tensor(np.asarray(gy, dtype=np.float64).reshape(-1)) * y).sum()
    loss.backward()
    return {"y": y.detach().numpy().reshape(T, k), "dc": tc.grad.numpy(), "dd": td.grad.numpy(),
            "ds": ts.grad.numpy(), "du0": tu.grad.numpy().reshape(np.shape(u0)), "dw": tw.grad.numpy()}
