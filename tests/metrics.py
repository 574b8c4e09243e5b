"""Error metrics used by the parity tests.

Solutions y and adjoints lam are compared per instance and per derivative
order with the relative 2-norm error ||x - x*|| / ||x*||.

Gradients are sums of products of row residuals (rho = a.y - b) and adjoint
row values (mu = a.lam).  A residual is a small difference of large terms, so
a gradient entry inherits an absolute error of about eps * (sum of |terms|)
from a relative error eps in y or lam -- for any method, the oracle included.
Gradient errors are therefore measured against that magnitude: the same
per-row formulas evaluated with absolute values (|a|.|y| + |b| in place of
|a.y - b|, |a|.|lam| in place of |a.lam|).  The resulting ratio is comparable
with the relative error of y and lam.
"""
import math

import numpy as np


def rel_by_order(x, ref, k):
    x = np.asarray(x, dtype=np.float64).reshape(-1, k)
    ref = np.asarray(ref, dtype=np.float64).reshape(-1, k)
    out = []
    for r in range(k):
        den = np.linalg.norm(ref[:, r])
        out.append(float(np.linalg.norm(x[:, r] - ref[:, r]) / den) if den > 0 else float(np.abs(x[:, r]).max()))
    return out


def grad_scales(c, d, s, u0, w, y, lam):
    """Magnitude of the terms of each gradient entry of one instance."""
    c = np.asarray(c, dtype=np.float64)
    T, k = c.shape
    y = np.asarray(y, dtype=np.float64).reshape(T, k)
    lam = np.asarray(lam, dtype=np.float64).reshape(T, k)
    ac, ay, al = np.abs(c), np.abs(y), np.abs(lam)
    wg, wi, ws = (abs(float(v)) for v in w)
    E = (ac * ay).sum(1) + np.abs(d)          # |e| bound
    Fm = (ac * al).sum(1)                      # |f| bound
    sc = wg * wg * (E[:, None] * al + Fm[:, None] * ay)
    sd = wg * wg * Fm
    U = np.abs(np.asarray(u0, dtype=np.float64))
    U = U.reshape(1, -1) if U.ndim <= 1 else U        # [T_init, n_init]
    te, n_init = min(U.shape[0], T), U.shape[1]
    su = np.zeros(U.shape)
    su[:te] = wi * wi * al[:te, :n_init]
    sw = np.zeros(3)
    sw[0] = 2 * wg * float((E * Fm).sum())
    sw[1] = 2 * wi * float(((ay[:te, :n_init] + U[:te]) * al[:te, :n_init]).sum())
    ss = np.zeros(T)
    if T > 1:
        st = np.abs(np.asarray(s, dtype=np.float64)[:T - 1])
        inv = np.array([1.0 / math.factorial(i) for i in range(k)])
        acc_w = np.zeros(T - 1)
        for r in range(k):
            # forward row r and backward row r: same |coefficients| pattern
            for yt, yn, lt, ln in ((ay[:-1], ay[1:], al[:-1], al[1:]), (ay[1:], ay[:-1], al[1:], al[:-1])):
                rho = st ** r * yn[:, r]
                mu = st ** r * ln[:, r]
                dy = (r * st ** (r - 1) * yn[:, r]) if r > 0 else np.zeros(T - 1)
                dl = (r * st ** (r - 1) * ln[:, r]) if r > 0 else np.zeros(T - 1)
                for j in range(r, k):
                    cf = inv[j - r]
                    rho = rho + st ** j * cf * yt[:, j]
                    mu = mu + st ** j * cf * lt[:, j]
                    if j > 0:
                        dy = dy + j * st ** (j - 1) * cf * yt[:, j]
                        dl = dl + j * st ** (j - 1) * cf * lt[:, j]
                ss[:-1] += ws * ws * (dl * rho + mu * dy)
                acc_w += rho * mu
        sw[2] = 2 * ws * float(acc_w.sum())
    return {"dc": sc, "dd": sd, "ds": ss, "du0": su.reshape(np.shape(u0)), "dw": sw}


def grad_error(got, ref, scale):
    """||got - ref|| / ||scale|| (see the module docstring)."""
    got = np.asarray(got, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    scale = np.asarray(scale, dtype=np.float64).ravel()
    den = np.linalg.norm(scale)
    return float(np.linalg.norm(got - ref) / den) if den > 0 else float(np.abs(got - ref).max())


def grad_scales_general(c, d, s, u, wg, wi, ws, y, lam):
    """grad_scales for an instance of any shape (V variables, Q governing
    equations, per-row weights): c [T, Q, K], d [T, Q], s [T], u and wi
    [t_init, V, n_init], wg [T, Q], ws [T], y and lam [T, K].  Returns the
    scales of dc, dd, ds, du0, the per-row weight gradients dwg, dwi, dws and
    the three scalar-weight sums dw."""
    c = np.abs(np.asarray(c, dtype=np.float64))
    T, Q, K = c.shape
    u = np.abs(np.asarray(u, dtype=np.float64))
    t_init, V, n_init = u.shape
    k = K // V
    ay = np.abs(np.asarray(y, dtype=np.float64).reshape(T, K))
    al = np.abs(np.asarray(lam, dtype=np.float64).reshape(T, K))
    wg = np.abs(np.asarray(wg, dtype=np.float64)).reshape(T, Q)
    wi = np.abs(np.asarray(wi, dtype=np.float64)).reshape(u.shape)
    ws = np.abs(np.asarray(ws, dtype=np.float64)).reshape(T)
    E = np.einsum("tqk,tk->tq", c, ay) + np.abs(np.asarray(d, dtype=np.float64)).reshape(T, Q)
    Fm = np.einsum("tqk,tk->tq", c, al)
    out = {"dc": (wg ** 2)[:, :, None] * (E[:, :, None] * al[:, None, :] + Fm[:, :, None] * ay[:, None, :]),
           "dd": wg ** 2 * Fm, "dwg": 2 * wg * E * Fm}
    te = min(t_init, T)
    yu = ay[:te].reshape(te, V, k)[:, :, :n_init]
    lu = al[:te].reshape(te, V, k)[:, :, :n_init]
    su = np.zeros(u.shape)
    sw = np.zeros(u.shape)
    su[:te] = wi[:te] ** 2 * lu
    sw[:te] = 2 * wi[:te] * (yu + u[:te]) * lu
    out["du0"], out["dwi"] = su, sw
    ss = np.zeros(T)
    sws = np.zeros(T)
    if T > 1:
        st = np.abs(np.asarray(s, dtype=np.float64).reshape(T)[:T - 1])
        inv = np.array([1.0 / math.factorial(i) for i in range(k)])
        for v in range(V):
            yv, lv = ay[:, v * k:(v + 1) * k], al[:, v * k:(v + 1) * k]
            for r in range(k):
                for yt, yn, lt, ln in ((yv[:-1], yv[1:], lv[:-1], lv[1:]), (yv[1:], yv[:-1], lv[1:], lv[:-1])):
                    rho = st ** r * yn[:, r]
                    mu = st ** r * ln[:, r]
                    dy = (r * st ** (r - 1) * yn[:, r]) if r > 0 else np.zeros(T - 1)
                    dl = (r * st ** (r - 1) * ln[:, r]) if r > 0 else np.zeros(T - 1)
                    for j in range(r, k):
                        cf = inv[j - r]
                        rho = rho + st ** j * cf * yt[:, j]
                        mu = mu + st ** j * cf * lt[:, j]
                        if j > 0:
                            dy = dy + j * st ** (j - 1) * cf * yt[:, j]
                            dl = dl + j * st ** (j - 1) * cf * lt[:, j]
                    ss[:-1] += ws[:-1] ** 2 * (dl * rho + mu * dy)
                    sws[:-1] += 2 * ws[:-1] * rho * mu
    out["ds"], out["dws"] = ss, sws
    out["dw"] = np.array([out["dwg"].sum(), sw.sum(), sws.sum()])
    return out
