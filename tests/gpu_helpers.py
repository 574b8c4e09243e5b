"""Shared helpers of the GPU parity tests: run the HIP path through the C-ABI
(paper_2410_06074_amd.Plan) on seeded inputs and compare with the oracle.

Reference.  The banded oracle computed in __float128 (``banded.grad(...,
quad=True)``): the least-squares solution, adjoint and gradients of the
double inputs rounded once to double (pinned bit-for-bit to the rational
oracle in tests/test_oracle_exact.py).  Unlike a double-precision oracle it
carries no error of its own at any conditioning met here, so what a metric
shows is the HIP path's error.

Pass criteria, per instance (the mode's working precision u_work = 2^-53 for
the double modes, 2^-24 for float I/O):
  P1  backward error of y for the normal equations of Eq. 9, evaluated row by
      row in __float128 (``banded.backward_error``), for every instance
      whatever its conditioning:
        normwise ||beta - M y||_inf / (||M||_inf ||y||_inf + ||beta||_inf)
            <= 50 u_work in every mode (what a backward-stable SPD solve of
            the normal equations guarantees), except the plain fp64 mode at
            order >= 3, where it is printed, not asserted: there the
            partitioned elimination's separator Schur complements lose up
            to ~150 u (the sequential block Cholesky of the same matrices
            stays below 1 u), and refinement is what restores it;
        row-scaled ||A^T W (b - A y)||_inf / || |A|^T W (|A||y| + |b|) ||_inf
            <= 50 u_work in the refined modes (refinement with a row-wise
            residual makes the solve backward stable row by row; the plain
            normal-equation solve is not, and reaches ~750 u at order 3).
  P2  forward error of y:
        fp64r  <= 1e-10 per derivative order, both as a relative 2-norm
               (``y``) and as max |y - y*| / max |y*| (``y_el``), where
               cond(M) <= 1e14;
        fp32r  <= 1e-4, same metrics, where cond(M) <= 1e10 (against the
               oracle on the same float-rounded inputs);
        fp64   <= max(1e-13, 2 cond(M) 2^-52) for the instance's whole
               vector, as a relative 2-norm (``y_nw``) and as max |y - y*| /
               max |y*| (``y_iel``): the forward bound of a backward-stable
               solve, ~cond(M) u for the normwise error.  (Per order, an
               order whose values are small against the others' carries a
               larger share; those columns are printed, not asserted.)
      Instances above the thresholds are reported, not asserted.
  Gradients: term-magnitude-scaled error (tests/metrics.py) <= 1e-10 (fp64r),
      1e-5 (fp32r), max(1e-10, 2 cond(M) 2^-52) (fp64), under the same
      thresholds; raw relative errors are printed beside them.
"""
import numpy as np

from oracle import banded
from tests import metrics

MODES = ("fp64", "fp64r", "fp32r")
EPS = float(np.finfo(np.float64).eps)           # 2^-52
U_WORK = {"fp64": 2.0 ** -53, "fp64r": 2.0 ** -53, "fp32r": 2.0 ** -24}
KAPPA_P2 = {"fp64r": 1e14, "fp32r": 1e10, "fp64": np.inf}
Y_TOL = {"fp64r": 1e-10, "fp32r": 1e-4}
G_TOL = {"fp64r": 1e-10, "fp32r": 1e-5}
GRADS = ("dc", "dd", "ds", "du0", "dw")


def dtype_for(mode):
    import torch
    return torch.float32 if mode == "fp32r" else torch.float64


def io_batch(bt, mode):
    """Inputs as the HIP path sees them (float32-rounded for fp32r)."""
    return bt.astype(np.float32).astype(np.float64) if mode == "fp32r" else bt


def pack_weights(bt):
    """The per-row weight buffer of the C-ABI: governing [S][Q], initial
    [N][T_init][V][n_init], smoothness [S]."""
    wr = bt.wrow
    return np.concatenate([np.ravel(wr["wg"]), np.ravel(wr["wi"]), np.ravel(wr["ws"])])


def run(bt, mode, gy=None, chunk=0, block=0, max_blocks=0, refine_steps=-1, device="cuda:0", info=True,
        chunk_upper=0):
    """Forward (and backward when gy is given) through the C-ABI; numpy results."""
    import torch
    from paper_2410_06074_amd import Plan
    dev = torch.device(device)
    dt = dtype_for(mode)
    steps = int(bt.T[0]) if np.all(bt.T == bt.T[0]) else bt.T
    rows = bt.wrow is not None
    p = Plan(bt.R, bt.n_init, bt.n_inst, steps, mode=mode, chunk=chunk, block=block, max_blocks=max_blocks,
             refine_steps=refine_steps, chunk_upper=chunk_upper, init_points=bt.t_init, variables=bt.V,
             equations=bt.Q, row_weights=rows)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    S, K, Q, N = bt.total_steps, bt.block, bt.Q, bt.n_inst
    ni = bt.t_init * bt.V * bt.n_init
    c, b, h, u0 = t(np.reshape(bt.c, (S, Q * K))), t(np.reshape(bt.b, (S * Q,))), t(bt.h), t(np.reshape(bt.u0, (N, ni)))
    w = t(pack_weights(bt)) if rows else t(bt.w)
    y = torch.empty((p.total_steps, p.k), dtype=dt, device=dev)
    fac, ws = p.new_factor(dev), p.new_workspace(dev)
    inf = torch.full((bt.n_inst,), -7, dtype=torch.int32, device=dev) if info else None
    p.forward(c, b, h, u0, w, y, fac, ws, inf)
    out = {"plan": p}
    if gy is not None:
        g = t(np.reshape(gy, (S, K)))
        dc, db, dh = torch.empty_like(c), torch.empty_like(b), torch.empty_like(h)
        du0, dw = torch.empty_like(u0), torch.empty_like(w)
        p.backward(c, b, h, u0, w, y, fac, g, dc, db, dh, du0, dw, ws, None)
        torch.cuda.synchronize(dev)
        out["dc"] = dc.double().cpu().numpy().reshape(np.shape(bt.c))
        out["dd"] = db.double().cpu().numpy().reshape(np.shape(bt.b))
        out["ds"] = dh.double().cpu().numpy()
        out["du0"] = du0.double().cpu().numpy().reshape(np.shape(bt.u0))
        dwn = dw.double().cpu().numpy()
        if rows:
            out["dwg"] = dwn[:S * Q].reshape(np.shape(bt.wrow["wg"]))
            out["dwi"] = dwn[S * Q:S * Q + N * ni].reshape(np.shape(bt.wrow["wi"]))
            out["dws"] = dwn[S * Q + N * ni:]
        else:
            out["dw"] = dwn.reshape(N, 3)
    torch.cuda.synchronize(dev)
    out["y"] = y.double().cpu().numpy()
    if info:
        out["info"] = inf.cpu().numpy()
    return out


def reference(bt, gy):
    """The __float128 oracle's y, lam and gradients for dl/dy = gy."""
    return banded.grad(bt, gy, quad=True)


def loss_gradient(y, k):
    """dl/dy of l = sum_t y_{t,0}^2 (the loss of the full-size configurations)."""
    g = np.zeros((len(y), k))
    g[:, 0] = 2.0 * np.asarray(y)[:, 0]
    return g


def _el(x, ref, k):
    """max over derivative orders of max_t |x - ref| / max_t |ref|."""
    x = np.asarray(x, dtype=np.float64).reshape(-1, k)
    ref = np.asarray(ref, dtype=np.float64).reshape(-1, k)
    out = 0.0
    for r in range(k):
        den = np.abs(ref[:, r]).max()
        out = max(out, float(np.abs(x[:, r] - ref[:, r]).max() / den) if den > 0 else float(np.abs(x[:, r]).max()))
    return out


def _raw(x, ref):
    x = np.asarray(x, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    den = np.abs(ref).max()
    nrm = np.linalg.norm(ref)
    if den == 0:
        return float(np.abs(x).max()), float(np.abs(x).max())
    return float(np.linalg.norm(x - ref) / nrm), float(np.abs(x - ref).max() / den)


def compare(bt, out, ref, idx, ref_off=None):
    """Per-instance metrics over the instances idx (dict of arrays, one entry
    per instance of idx).  ref holds oracle arrays for the instances idx
    (packed with ref_off) or for all instances (ref_off None)."""
    o = bt.offsets
    sub = bt.subset(list(idx))
    m = {"y": [], "y_el": [], "y_nw": [], "y_iel": []}
    ys = []
    for j, i in enumerate(idx):
        sl = slice(o[i], o[i + 1])
        rs = slice(ref_off[j], ref_off[j + 1]) if ref_off is not None else sl
        ri = j if ref_off is not None else i
        ys.append(out["y"][sl])
        m["y"].append(max(metrics.rel_by_order(out["y"][sl], ref["y"][rs], bt.k)))
        m["y_el"].append(_el(out["y"][sl], ref["y"][rs], bt.k))
        nw, iel = _raw(out["y"][sl], ref["y"][rs])
        m["y_nw"].append(nw)
        m["y_iel"].append(iel)
        if "dc" in out and "dc" in ref:
            c, d, s, u0, w = bt.instance(i)
            sc = metrics.grad_scales(c, d, s, u0, w, ref["y"][rs], ref["lam"][rs])
            for key in GRADS:
                got, want = (out[key][sl], ref[key][rs]) if key in ("dc", "dd", "ds") else (out[key][i], ref[key][ri])
                if np.size(want) == 0:             # no initial rows (n_init = 0)
                    continue
                m.setdefault(key, []).append(metrics.grad_error(got, want, sc[key]))
                if key != "dw":     # a sum over all rows whose exact value may be ~0
                    raw, raw_el = _raw(got, want)
                    m.setdefault(key + "_raw", []).append(raw)
                    m.setdefault(key + "_el", []).append(raw_el)
    yall = np.concatenate(ys) if ys else np.zeros((0, bt.k))
    m["eta"] = list(banded.backward_error(sub, yall))
    m["eta_n"] = list(banded.backward_error(sub, yall, normwise=True))
    return {k: np.asarray(v, dtype=np.float64) for k, v in m.items()}


GRADS_ROW = ("dc", "dd", "ds", "du0", "dwg", "dwi", "dws")


def compare_general(bt, out, ref, idx):
    """compare() for a batch of any instance shape (V variables, Q governing
    equations, per-row weights): y per variable and order (relative 2-norm and
    element by element), every gradient in the term-scaled metric (scales
    from metrics.grad_scales_general) and as raw relative errors, and the
    backward errors of y.  ref holds oracle arrays for every instance."""
    o = bt.offsets
    K = bt.block
    m = {"y": [], "y_el": [], "y_nw": [], "y_iel": []}
    keys = GRADS_ROW if bt.wrow is not None else ("dc", "dd", "ds", "du0", "dw")
    Q, ni = bt.Q, bt.t_init * bt.V * bt.n_init
    for i in idx:
        sl = slice(o[i], o[i + 1])
        m["y"].append(max(metrics.rel_by_order(out["y"][sl], ref["y"][sl], K)))
        m["y_el"].append(_el(out["y"][sl], ref["y"][sl], K))
        nw, iel = _raw(out["y"][sl], ref["y"][sl])
        m["y_nw"].append(nw)
        m["y_iel"].append(iel)
        if "dc" not in out:
            continue
        sc = metrics.grad_scales_general(*bt.instance_general(i), ref["y"][sl], ref["lam"][sl])
        T = int(o[i + 1] - o[i])
        for key in keys:
            if key in ("dc",):
                got, want = out[key][sl].reshape(T, Q, K), ref[key][sl].reshape(T, Q, K)
            elif key in ("dd", "dwg"):
                got, want = out[key][sl].reshape(T, Q), ref[key][sl].reshape(T, Q)
            elif key in ("ds", "dws"):
                got, want = out[key][sl], ref[key][sl]
            elif key in ("du0", "dwi"):
                got = out[key].reshape(bt.n_inst, ni)[i]
                want = ref[key].reshape(bt.n_inst, ni)[i]
            else:
                got, want = out[key][i], ref[key][i]
            if np.size(want) == 0:
                continue
            m.setdefault(key, []).append(metrics.grad_error(got, want, sc[key].reshape(np.shape(want))))
            if key not in ("dw", "dwi", "dwg", "dws"):
                raw, raw_el = _raw(got, want)
                m.setdefault(key + "_raw", []).append(raw)
                m.setdefault(key + "_el", []).append(raw_el)
    sub = bt.subset(list(idx))
    rows = np.concatenate([np.arange(o[i], o[i + 1]) for i in idx])
    m["eta"] = list(banded.backward_error(sub, out["y"][rows]))
    m["eta_n"] = list(banded.backward_error(sub, out["y"][rows], normwise=True))
    return {k: np.asarray(v, dtype=np.float64) for k, v in m.items()}


def summary(m):
    """One line: worst value of every metric."""
    return " ".join("%s=%.1e" % (k, float(np.max(v))) for k, v in m.items() if np.size(v))


def y_tolerance(mode, kappa):
    if mode == "fp64":
        return max(1e-13, 2.0 * kappa * EPS)
    return Y_TOL[mode]


def g_tolerance(mode, kappa):
    if mode == "fp64":
        return max(1e-10, 2.0 * kappa * EPS)
    return G_TOL[mode]


def check(mode, m, kappa, order, grads=True):
    """Assert P1 on every instance and P2 (and the gradient bounds) on the
    instances whose cond(M) is within the mode's threshold."""
    kappa = np.broadcast_to(np.asarray(kappa, dtype=np.float64), m["eta"].shape)
    p1 = 50.0 * U_WORK[mode]
    if mode != "fp64" or order <= 2:
        bad = np.nonzero(m["eta_n"] > p1)[0]
        assert bad.size == 0, ("P1 normwise backward error", m["eta_n"][bad], kappa[bad])
    if mode != "fp64":
        bad = np.nonzero(m["eta"] > p1)[0]
        assert bad.size == 0, ("P1 row-scaled backward error", m["eta"][bad], kappa[bad])
    ykeys = ("y_nw", "y_iel") if mode == "fp64" else ("y", "y_el")
    for j in range(len(kappa)):
        if kappa[j] > KAPPA_P2[mode]:
            continue
        ty, tg = y_tolerance(mode, kappa[j]), g_tolerance(mode, kappa[j])
        for key in ykeys:
            assert m[key][j] <= ty, ("P2", key, j, m[key][j], kappa[j])
        if grads:
            for key in GRADS + ("dwg", "dwi", "dws"):
                if key in m:
                    assert m[key][j] <= tg, ("gradient", key, j, m[key][j], kappa[j])
