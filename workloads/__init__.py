"""Seeded synthetic inputs for the batched linear-ODE least-squares solve.

This module only draws random numbers and lays them out; it holds none of the
solve's arithmetic, so the oracle (``oracle/``) and the HIP path
(``paper_2410_06074_amd``) can both consume the same inputs without sharing
any code that computes a result.

Layout (the "natural" layout the C-ABI consumes, see ``include/smnn.h``):
per-step arrays are instance-major and time-contiguous.  Instance ``i`` owns
rows ``off[i] .. off[i] + T[i] - 1`` where ``off`` is the exclusive prefix sum
of ``T``.  ``c`` is ``[S, R+1]``, ``b`` and ``h`` are ``[S]``, ``u0`` is
``[N, t_init * n_init]`` (initial values of orders ``0..n_init-1`` at each of
the first ``t_init`` time points, point-major), ``w`` is ``[N, 3]`` (unsquared governing / initial /
smoothness weights), with ``S = sum(T)``.  ``h[off[i] + t]`` is the step size
between time points ``t`` and ``t+1``; the last slot of each instance is not
used by the solve (it is drawn anyway so every slot holds a finite value).

Value distributions follow the paper's workload shapes (standalone validation
with step 0.01, the Lorenz batch of 512, the daily multi-year SST-like grid)
as restated per configuration below; none of the paper's datasets is used.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Batch:
    R: int
    n_init: int
    T: np.ndarray          # int64 [N]
    c: np.ndarray          # [S, R+1]
    b: np.ndarray          # [S]
    h: np.ndarray          # [S]
    u0: np.ndarray         # [N, n_init]
    w: np.ndarray          # [N, 3]
    name: str = ""
    t_init: int = 1        # time points carrying initial values
    V: int = 1             # variables per instance (Sec. 3.1)
    Q: int = 1             # governing equations per time point
    wrow: dict | None = None   # per-row weights {"wg": [S, Q], "wi": [N, t_init*V*n_init], "ws": [S]}

    @property
    def n_inst(self) -> int:
        return int(self.T.shape[0])

    @property
    def block(self) -> int:
        """Unknowns per time point, V (R+1)."""
        return self.V * (self.R + 1)

    @property
    def k(self) -> int:
        return self.R + 1

    @property
    def offsets(self) -> np.ndarray:
        off = np.zeros(self.n_inst + 1, dtype=np.int64)
        np.cumsum(self.T, out=off[1:])
        return off

    @property
    def total_steps(self) -> int:
        return int(self.T.sum())

    def instance(self, i: int):
        """(c, b, h, u0, w) of instance i as float64 views/copies; u0 is
        [n_init] when t_init = 1, else [t_init, n_init].  Scalar weights and
        V = Q = 1 only (see ``instance_general``)."""
        assert self.V == 1 and self.Q == 1 and self.wrow is None
        o = self.offsets
        s, e = int(o[i]), int(o[i + 1])
        return (np.asarray(self.c[s:e], dtype=np.float64),
                np.asarray(self.b[s:e], dtype=np.float64),
                np.asarray(self.h[s:e], dtype=np.float64),
                (np.asarray(self.u0[i], dtype=np.float64) if self.t_init == 1
                 else np.asarray(self.u0[i], dtype=np.float64).reshape(self.t_init, self.n_init)),
                np.asarray(self.w[i], dtype=np.float64))

    def instance_general(self, i: int):
        """(c [T, Q, V(R+1)], d [T, Q], s [T], u [t_init, V, n_init],
        wg [T, Q], wi [t_init, V, n_init], ws [T]) of instance i, float64,
        with scalar weights expanded to their rows."""
        o = self.offsets
        s, e = int(o[i]), int(o[i + 1])
        T, K = e - s, self.block
        c = np.asarray(self.c[s:e], dtype=np.float64).reshape(T, self.Q, K)
        d = np.asarray(self.b[s:e], dtype=np.float64).reshape(T, self.Q)
        h = np.asarray(self.h[s:e], dtype=np.float64).reshape(T)
        u = np.asarray(self.u0[i], dtype=np.float64).reshape(self.t_init, self.V, self.n_init)
        if self.wrow is None:
            w = np.asarray(self.w[i], dtype=np.float64)
            wg, wi, ws = np.full((T, self.Q), w[0]), np.full(u.shape, w[1]), np.full(T, w[2])
        else:
            wg = np.asarray(self.wrow["wg"][s:e], dtype=np.float64).reshape(T, self.Q)
            wi = np.asarray(self.wrow["wi"][i], dtype=np.float64).reshape(u.shape)
            ws = np.asarray(self.wrow["ws"][s:e], dtype=np.float64).reshape(T)
        return c, d, h, u, wg, wi, ws

    def astype(self, dtype) -> "Batch":
        wrow = None if self.wrow is None else {k: v.astype(dtype) for k, v in self.wrow.items()}
        return dataclasses.replace(
            self, c=self.c.astype(dtype), b=self.b.astype(dtype),
            h=self.h.astype(dtype), u0=self.u0.astype(dtype),
            w=self.w.astype(dtype), wrow=wrow)

    def subset(self, idx) -> "Batch":
        """A new batch holding the instances in ``idx`` (in that order)."""
        o = self.offsets
        idx = list(idx)
        rows = np.concatenate([np.arange(o[i], o[i + 1]) for i in idx]) if len(idx) else np.zeros(0, np.int64)
        wrow = None if self.wrow is None else {"wg": self.wrow["wg"][rows].copy(), "ws": self.wrow["ws"][rows].copy(),
                                               "wi": self.wrow["wi"][idx].copy()}
        return Batch(R=self.R, n_init=self.n_init, T=self.T[idx].copy(),
                     c=self.c[rows].copy(), b=self.b[rows].copy(), h=self.h[rows].copy(),
                     u0=self.u0[idx].copy(), w=self.w[idx].copy(),
                     name=self.name + "[subset]", t_init=self.t_init, V=self.V, Q=self.Q, wrow=wrow)


def _gaussian_c(rng, S, R, scale=1.0):
    c = rng.standard_normal((S, R + 1)) * scale
    c[:, R] = 1.0 + np.abs(rng.standard_normal(S))
    return c


def _ar1(rng, n_series: int, T: int, rho: float) -> np.ndarray:
    """Stationary unit-variance AR(1) series, shape [n_series, T]."""
    x = np.empty((n_series, T))
    x[:, 0] = rng.standard_normal(n_series)
    e = rng.standard_normal((n_series, T))
    a = math.sqrt(1.0 - rho * rho)
    for t in range(1, T):
        x[:, t] = rho * x[:, t - 1] + a * e[:, t]
    return x


def gaussian_batch(n_inst: int, T, R: int = 2, seed: int = 0, n_init: int | None = None,
                   weights=(1.0, 1.0, 1.0), h0: float = 0.01, name: str = "", t_init: int = 1,
                   per_row: bool = False) -> Batch:
    """c_{t,r<R} ~ N(0,1), c_{t,R} = 1+|N(0,1)|, b ~ N(0,1), h = h0*(0.5+U[0,1)),
    u0 ~ N(0,1) at t_init points, constant weights (or, with ``per_row``,
    per-row weights log-uniform on [0.5, 2], drawn after everything else).
    ``T`` is an int (uniform) or an array."""
    rng = np.random.default_rng(seed)
    Ts = np.full(n_inst, int(T), dtype=np.int64) if np.isscalar(T) else np.asarray(T, dtype=np.int64)
    S = int(Ts.sum())
    n_init = R if n_init is None else n_init
    c = _gaussian_c(rng, S, R)
    b = rng.standard_normal(S)
    h = h0 * (0.5 + rng.random(S))
    u0 = rng.standard_normal((n_inst, t_init * n_init))
    w = np.tile(np.asarray(weights, dtype=np.float64), (n_inst, 1))
    wrow = row_weights(rng, Ts, n_inst, 1, 1, n_init, t_init) if per_row else None
    return Batch(R=R, n_init=n_init, T=Ts, c=c, b=b, h=h, u0=u0, w=w, name=name, t_init=t_init, wrow=wrow)


def row_weights(rng, T, n_inst: int, Q: int = 1, V: int = 1, n_init: int = 1, t_init: int = 1,
                lo: float = 0.5, hi: float = 2.0) -> dict:
    """Per-row weights (App. A.1's W = diag(w), unsquared) log-uniform on
    [lo, hi]: wg [S, Q] per governing row, wi [N, t_init * V * n_init] per
    initial row, ws [S] per step (the smoothness rows of that step)."""
    S = int(np.sum(T))
    lu = lambda shape: np.exp(rng.uniform(math.log(lo), math.log(hi), size=shape))
    return {"wg": lu((S, Q)), "wi": lu((n_inst, t_init * V * n_init)), "ws": lu(S)}


def coupled_batch(n_inst: int, T, R: int = 1, V: int = 2, Q: int | None = None, seed: int = 0,
                  n_init: int | None = None, weights=(1.0, 1.0, 1.0), h0: float = 0.01, t_init: int = 1,
                  per_row: bool = False, name: str = "") -> Batch:
    """V coupled variables per instance (Sec. 3.1) with Q governing equations
    per point (default Q = V): every coefficient c_{t,q,v,r} ~ N(0,1) except
    the leading one of equation q on variable q, c_{t,q,q,R} = 1+|N(0,1)|
    (q < V); b ~ N(0,1) [S, Q]; h = h0 (0.5+U[0,1)); u0 ~ N(0,1) for orders
    < n_init of every variable at t_init points; scalar weights, or per-row
    weights log-uniform on [0.5, 2] (``per_row``).  c is [S, Q V (R+1)]."""
    rng = np.random.default_rng(seed)
    Q = V if Q is None else Q
    Ts = np.full(n_inst, int(T), dtype=np.int64) if np.isscalar(T) else np.asarray(T, dtype=np.int64)
    S = int(Ts.sum())
    k, K = R + 1, V * (R + 1)
    n_init = R if n_init is None else n_init
    c = rng.standard_normal((S, Q, K))
    for q in range(min(Q, V)):
        c[:, q, q * k + R] = 1.0 + np.abs(rng.standard_normal(S))
    b = rng.standard_normal((S, Q))
    h = h0 * (0.5 + rng.random(S))
    u0 = rng.standard_normal((n_inst, t_init * V * n_init))
    w = np.tile(np.asarray(weights, dtype=np.float64), (n_inst, 1))
    wrow = row_weights(rng, Ts, n_inst, Q, V, n_init, t_init) if per_row else None
    return Batch(R=R, n_init=n_init, T=Ts, c=c.reshape(S, Q * K), b=b if Q > 1 else b.reshape(S), h=h, u0=u0, w=w,
                 name=name or "coupled", t_init=t_init, V=V, Q=Q, wrow=wrow)


def config(name: str, seed: int | None = None, n_inst: int | None = None, T: int | None = None) -> Batch:
    """The named workloads.  ``n_inst`` / ``T`` override the size (parity tests
    use smaller copies of the same distributions).

    c0  1 instance, R=2, T=64, Gaussian coefficients, h = 0.01*(0.5+U), w = 1.
    c1  512 x 3 = 1536 instances, R=2, T=1000, as c0 (Lorenz-sized batch).
    c2  256 x 128 = 32768 instances, R=2, T=1460, c and b smooth in t
        (stationary AR(1), rho = 0.99, unit variance), c_R = 1+|AR(1)|,
        h = 1/365, u0 ~ N(0,1), w = 1 (daily four-year grid).
    c3  2048 instances, R=3, T ~ U{50..5000} (ragged), c_{t,R} = 1+|N(0,1)|,
        other c ~ N(0, 0.5^2), b ~ N(0,1), h as c0, u0^(0..2) ~ N(0,1),
        w_gov, w_init, w_smooth each log-uniform on [0.1, 10].
    c4  4 x 8 = 32 instances, R=2, T = 1,000,000, as c0.
    h   512 x 3 = 1536 instances, R=2, T = 10,000, as c1 (throughput headline).
    hw  as h with per-row weights log-uniform on [0.5, 2] (App. A.1's W).
    v2  1536 instances of two coupled order-1 variables with two governing
        equations per point, T = 10,000 (coupled_batch).
    v3  512 instances of three coupled order-2 variables with three governing
        equations per point (the Lorenz batch of Sec. 5.1 as one coupled
        system per window), T = 1,000 (coupled_batch).
    """
    seeds = {"c0": 0, "c1": 1, "c2": 2, "c3": 3, "c4": 4, "h": 5, "hw": 6, "v2": 7, "v3": 8}
    if name not in seeds:
        raise KeyError(name)
    sd = seeds[name] if seed is None else seed
    if name == "hw":
        return gaussian_batch(n_inst or 1536, T or 10_000, R=2, seed=sd, name=name, per_row=True)
    if name == "v2":
        return coupled_batch(n_inst or 1536, T or 10_000, R=1, V=2, Q=2, seed=sd, name=name)
    if name == "v3":
        return coupled_batch(n_inst or 512, T or 1000, R=2, V=3, Q=3, seed=sd, name=name)
    if name in ("c0", "c1", "c4", "h"):
        defaults = {"c0": (1, 64), "c1": (1536, 1000), "c4": (32, 1_000_000), "h": (1536, 10_000)}
        N, TT = defaults[name]
        return gaussian_batch(n_inst or N, T or TT, R=2, seed=sd, name=name)
    rng = np.random.default_rng(sd)
    if name == "c2":
        N = n_inst or 32768
        TT = T or 1460
        R = 2
        k = R + 1
        c = np.empty((N, TT, k))
        for r in range(k):
            c[:, :, r] = _ar1(rng, N, TT, 0.99)
        c[:, :, R] = 1.0 + np.abs(c[:, :, R])
        b = _ar1(rng, N, TT, 0.99)
        h = np.full((N, TT), 1.0 / 365.0)
        u0 = rng.standard_normal((N, R))
        w = np.ones((N, 3))
        return Batch(R=R, n_init=R, T=np.full(N, TT, dtype=np.int64), c=c.reshape(N * TT, k),
                     b=b.reshape(-1), h=h.reshape(-1), u0=u0, w=w, name=name)
    # c3
    N = n_inst or 2048
    R = 3
    lo, hi = (50, 5000) if T is None else (max(1, T // 100), T)
    Ts = rng.integers(lo, hi + 1, size=N).astype(np.int64)
    S = int(Ts.sum())
    c = rng.normal(0.0, 0.5, size=(S, R + 1))
    c[:, R] = 1.0 + np.abs(rng.standard_normal(S))
    b = rng.standard_normal(S)
    h = 0.01 * (0.5 + rng.random(S))
    u0 = rng.standard_normal((N, R))
    w = np.exp(rng.uniform(math.log(0.1), math.log(10.0), size=(N, 3)))
    return Batch(R=R, n_init=R, T=Ts, c=c, b=b, h=h, u0=u0, w=w, name=name)


def polynomial_batch(n_inst: int, T: int, R: int, seed: int = 0, degree: int | None = None,
                     n_init: int | None = None, h0: float = 0.01):
    """Inputs whose least-squares system is consistent: a random polynomial p of
    degree <= R (default R) per instance, random c, d_t = sum_r c_{t,r} p^(r)(t_k)
    and u0_r = p^(r)(t_0).  Returns (batch, exact) with exact[S, R+1] holding
    p^(r) at every time point.  Only Taylor coefficients are evaluated here
    (no part of the solve)."""
    rng = np.random.default_rng(seed)
    deg = R if degree is None else degree
    n_init = R if n_init is None else n_init
    k = R + 1
    S = n_inst * T
    c = _gaussian_c(rng, S, R)
    h = h0 * (0.5 + rng.random(S))
    coef = rng.standard_normal((n_inst, deg + 1))       # p(x) = sum_j coef_j x^j
    exact = np.zeros((n_inst, T, k))
    for i in range(n_inst):
        tk = np.concatenate([[0.0], np.cumsum(h[i * T:(i + 1) * T - 1])])
        for r in range(k):
            acc = np.zeros(T)
            for j in range(r, deg + 1):
                acc += coef[i, j] * math.factorial(j) / math.factorial(j - r) * tk ** (j - r)
            exact[i, :, r] = acc
    exact = exact.reshape(S, k)
    b = np.einsum("sr,sr->s", c, exact)
    u0 = np.stack([exact[i * T, :n_init] for i in range(n_inst)]) if n_init else np.zeros((n_inst, 0))
    w = np.ones((n_inst, 3))
    batch = Batch(R=R, n_init=n_init, T=np.full(n_inst, T, dtype=np.int64), c=c, b=b, h=h,
                  u0=u0, w=w, name="poly")
    return batch, exact
