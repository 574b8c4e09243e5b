"""Shared helpers of the GPU parity tests: run the HIP path through the C-ABI
(paper_2410_06074_amd.Plan) on seeded inputs and compare with the oracle."""
import numpy as np

from tests import metrics

MODES = ("fp64", "fp64r", "fp32r")

# Tolerances (relative 2-norm error per instance and derivative order).
#  fp64r: the stated FP64 target.
#  fp32r: the stated FP32+refinement target; measured against the oracle run on
#         the same float32-rounded inputs.
#  fp64 : the paper's single normal-equation solve; its error is bounded by
#         about c cond(M) * 2^-53, and cond(M) ~ 1.2e9 for the Gaussian
#         configurations (estimated per instance by oracle.banded.cond), so it
#         is held to 10 * cond(M) * 2^-53 (floor 1e-12) instead of 1e-10.
Y_TOL = {"fp64r": 1e-10, "fp32r": 1e-4}
# Gradients: term-magnitude-scaled error (tests/metrics.py); the refined FP64
# adjoint leaves ~1e-15, float32 outputs ~1e-7, and the plain FP64 adjoint
# carries the same cond(M) * 2^-53 bound as its solution (du0 = w_i^2 lam_1
# has no cancellation, so it shows the adjoint's own error).
G_TOL = {"fp64r": 1e-10, "fp32r": 1e-5}


def dtype_for(mode):
    import torch
    return torch.float32 if mode == "fp32r" else torch.float64


def io_batch(bt, mode):
    """Inputs as the HIP path sees them (float32-rounded for fp32r)."""
    return bt.astype(np.float32).astype(np.float64) if mode == "fp32r" else bt


def run(bt, mode, gy=None, chunk=0, block=0, max_blocks=0, refine_steps=-1, device="cuda:0", info=True,
        chunk_upper=0):
    """Forward (and backward when gy is given) through the C-ABI; numpy results."""
    import torch
    from paper_2410_06074_amd import Plan
    dev = torch.device(device)
    dt = dtype_for(mode)
    steps = int(bt.T[0]) if np.all(bt.T == bt.T[0]) else bt.T
    p = Plan(bt.R, bt.n_init, bt.n_inst, steps, mode=mode, chunk=chunk, block=block, max_blocks=max_blocks,
             refine_steps=refine_steps, chunk_upper=chunk_upper, init_points=bt.t_init)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    c, b, h, u0, w = t(bt.c), t(bt.b), t(bt.h), t(bt.u0.reshape(bt.n_inst, bt.t_init * bt.n_init)), t(bt.w)
    y = torch.empty((p.total_steps, p.k), dtype=dt, device=dev)
    fac, ws = p.new_factor(dev), p.new_workspace(dev)
    inf = torch.full((bt.n_inst,), -7, dtype=torch.int32, device=dev) if info else None
    p.forward(c, b, h, u0, w, y, fac, ws, inf)
    out = {"plan": p}
    if gy is not None:
        g = t(gy)
        dc, db, dh = torch.empty_like(c), torch.empty_like(b), torch.empty_like(h)
        du0, dw = torch.empty_like(u0), torch.empty_like(w)
        p.backward(c, b, h, u0, w, y, fac, g, dc, db, dh, du0, dw, ws, None)
        for key, v in (("dc", dc), ("dd", db), ("ds", dh), ("du0", du0), ("dw", dw)):
            out[key] = v.double().cpu().numpy()
    torch.cuda.synchronize(dev)
    out["y"] = y.double().cpu().numpy()
    if info:
        out["info"] = inf.cpu().numpy()
    return out


def loss_gradient(y, k):
    """dl/dy of l = sum_t y_{t,0}^2 (the loss of the full-size configurations)."""
    g = np.zeros((len(y), k))
    g[:, 0] = 2.0 * np.asarray(y)[:, 0]
    return g


def compare(bt, out, ref, idx, ref_off=None):
    """Worst y error and worst gradient errors over the instances idx.
    ref holds oracle arrays for the instances idx (packed with ref_off) or for
    all instances (ref_off None)."""
    o = bt.offsets
    worst = {"y": 0.0}
    for j, i in enumerate(idx):
        sl = slice(o[i], o[i + 1])
        rs = slice(ref_off[j], ref_off[j + 1]) if ref_off is not None else sl
        ri = j if ref_off is not None else i
        worst["y"] = max(worst["y"], max(metrics.rel_by_order(out["y"][sl], ref["y"][rs], bt.k)))
        if "dc" in out and "dc" in ref:
            c, d, s, u0, w = bt.instance(i)
            sc = metrics.grad_scales(c, d, s, u0, w, ref["y"][rs], ref["lam"][rs])
            for key in ("dc", "dd", "ds"):
                worst[key] = max(worst.get(key, 0.0), metrics.grad_error(out[key][sl], ref[key][rs], sc[key]))
                den = np.linalg.norm(ref[key][rs])
                if den > 0:
                    worst[key + "_raw"] = max(worst.get(key + "_raw", 0.0),
                                              float(np.linalg.norm(out[key][sl] - ref[key][rs]) / den))
            for key in ("du0", "dw"):
                if np.size(ref[key][ri]) == 0:    # no initial rows (n_init = 0)
                    continue
                worst[key] = max(worst.get(key, 0.0), metrics.grad_error(out[key][i], ref[key][ri], sc[key]))
    return worst


def g_tolerance(mode, kappa):
    if mode == "fp64":
        return max(1e-10, 10.0 * kappa * np.finfo(np.float64).eps)
    return G_TOL[mode]


def y_tolerance(mode, kappa):
    if mode == "fp64":
        return max(1e-12, 10.0 * kappa * np.finfo(np.float64).eps)
    return Y_TOL[mode]
