"""hipGraph capture of the launch sequence, the autotuner, and the autograd
wrapper, on the GPU."""
import numpy as np
import pytest

from oracle import banded
from tests import gpu_helpers as H
from workloads import config, gaussian_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_06074_amd
    paper_2410_06074_amd.lib()


def _buffers(bt, mode, dev):
    import torch
    from paper_2410_06074_amd import Plan
    dt = H.dtype_for(mode)
    steps = int(bt.T[0]) if np.all(bt.T == bt.T[0]) else bt.T
    p = Plan(bt.R, bt.n_init, bt.n_inst, steps, mode=mode)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    ins = [t(bt.c), t(bt.b), t(bt.h), t(bt.u0), t(bt.w)]
    y = torch.empty((p.total_steps, p.k), dtype=dt, device=dev)
    fac, ws = p.new_factor(dev), p.new_workspace(dev)
    gy = t(np.random.default_rng(0).standard_normal(bt.c.shape))
    grads = [torch.empty_like(ins[0]), torch.empty_like(ins[1]), torch.empty_like(ins[2]),
             torch.empty_like(ins[3]), torch.empty_like(ins[4])]
    return p, ins, y, fac, ws, gy, grads


@pytest.mark.parametrize("mode", ["fp64r", "fp32r"])
def test_graph_replays_match_eager_bitwise(mode):
    import torch
    from paper_2410_06074_amd import CapturedSolve
    dev = torch.device("cuda:0")
    bt = gaussian_batch(37, [5, 8, 9, 300, 1001] * 7 + [2, 17], R=2, seed=4, weights=(1.2, 0.9, 1.1))
    p, ins, y, fac, ws, gy, grads = _buffers(bt, mode, dev)
    p.forward(*ins, y, fac, ws)
    p.backward(*ins, y, fac, gy, *grads, ws)
    torch.cuda.synchronize()
    eager = [y.clone()] + [g.clone() for g in grads]
    cap = CapturedSolve(p, *ins, y, fac, ws, gy=gy, grads=grads)
    for rep in range(4):
        for t in [y] + grads:
            t.zero_()                                  # eager work between replays
        torch.cuda.synchronize()
        cap.replay()
        torch.cuda.synchronize()
        for a, b in zip(eager, [y] + grads):
            assert torch.equal(a, b), rep


def test_autotuner_returns_a_working_mapping(tmp_path, monkeypatch):
    import torch
    from paper_2410_06074_amd import Plan, autotune
    monkeypatch.setenv("SMNN_TUNE_CACHE", str(tmp_path / "tune.json"))
    dev = torch.device("cuda:0")
    bt = config("c1", n_inst=64, T=500)
    p, ins, y, fac, ws, gy, grads = _buffers(bt, "fp64r", dev)
    res = autotune(bt.R, bt.n_init, bt.n_inst, 500, "fp64r", *ins, gy, iters=2)
    print("autotune", {k: v for k, v in res.items() if k != "candidates"}, "candidates", len(res["candidates"]),
          flush=True)
    assert res["chunk"] in (4, 8, 16) and res["chunk_upper"] in (4, 8, 16) and res["ms"] > 0
    assert len(res["candidates"]) >= 4
    again = autotune(bt.R, bt.n_init, bt.n_inst, 500, "fp64r", *ins, gy, iters=2)
    assert again.get("cached") and again["chunk"] == res["chunk"]
    out = H.run(bt, "fp64r", chunk=res["chunk"], block=res["block"], max_blocks=res["max_blocks"],
                chunk_upper=res["chunk_upper"])
    ref = banded.solve(bt)
    assert max(H.metrics.rel_by_order(out["y"], ref, bt.k)) < 1e-10


def test_autograd_function_matches_abi_and_gradcheck():
    import torch
    from paper_2410_06074_amd import solve
    dev = torch.device("cuda:0")
    bt = gaussian_batch(3, 40, R=2, seed=8, weights=(1.1, 0.9, 1.3))
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev).requires_grad_(True)
    c, b, h = t(bt.c.reshape(3, 40, 3)), t(bt.b.reshape(3, 40)), t(bt.h.reshape(3, 40))
    u0, w = t(bt.u0), t(bt.w)
    y = solve(c, b, h, u0, w, mode="fp64r")
    (y[..., 0] ** 2).sum().backward()
    gy = H.loss_gradient(y.detach().cpu().numpy().reshape(-1, 3), 3)
    out = H.run(bt, "fp64r", gy)
    np.testing.assert_array_equal(c.grad.cpu().numpy().reshape(-1, 3), out["dc"])
    np.testing.assert_array_equal(h.grad.cpu().numpy().reshape(-1), out["ds"])
    np.testing.assert_array_equal(w.grad.cpu().numpy(), out["dw"])

    small = gaussian_batch(1, 6, R=1, seed=2, weights=(1.2, 0.8, 1.5))
    tt = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev).requires_grad_(True)
    args = (tt(small.c.reshape(1, 6, 2)), tt(small.b.reshape(1, 6)), tt(small.h.reshape(1, 6)), tt(small.u0),
            tt(small.w))
    f = lambda *a: solve(*a, mode="fp64r")
    # finite differences of a least-squares solve: relative step 1e-6, loose tolerances
    assert torch.autograd.gradcheck(f, args, eps=1e-6, atol=1e-5, rtol=1e-4)


@pytest.mark.parametrize("mode", ["fp32r", "fp64r"])
def test_ragged_persistent_work_queue_captured(mode):
    # the ragged order-3 configuration's shape (lengths U{50..5000}, log-uniform
    # weights), 256 instances: persistent launches whose waves claim tiles from
    # the device work queue, captured in a hipGraph and replayed with eager
    # work in between; every replay bitwise equal to the one-wave-per-tile
    # eager call, which itself matches the oracle on sampled instances
    import torch
    from paper_2410_06074_amd import CapturedSolve, Plan
    dev = torch.device("cuda:0")
    bt = H.io_batch(config("c3", n_inst=256), mode)
    gy_np = np.random.default_rng(3).standard_normal(bt.c.shape)
    if mode == "fp32r":
        gy_np = gy_np.astype(np.float32).astype(np.float64)
    ref_out = H.run(bt, mode, gy_np)
    idx = [0, int(np.argmax(bt.T)), int(np.argmin(bt.T))]
    sub = bt.subset(idx)
    o, so = bt.offsets, sub.offsets
    g_sub = np.concatenate([gy_np[o[i]:o[i + 1]] for i in idx])
    ref = H.reference(sub, g_sub)
    rows = np.concatenate([np.arange(o[i], o[i + 1]) for i in idx])
    got = {"y": ref_out["y"][rows], "dc": ref_out["dc"][rows], "dd": ref_out["dd"][rows],
           "ds": ref_out["ds"][rows], "du0": ref_out["du0"][idx], "dw": ref_out["dw"][idx]}
    m = H.compare(sub, got, ref, range(len(idx)))
    kappa = banded.cond(sub)
    print("ragged persistent %s" % mode, H.summary(m), "kappa", kappa, flush=True)
    H.check(mode, m, kappa, bt.R)

    dt = H.dtype_for(mode)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    p = Plan(bt.R, bt.n_init, bt.n_inst, bt.T, mode=mode, block=128, max_blocks=96)
    ins = [t(bt.c), t(bt.b), t(bt.h), t(bt.u0), t(bt.w)]
    y = torch.empty((p.total_steps, p.k), dtype=dt, device=dev)
    fac, ws, gy = p.new_factor(dev), p.new_workspace(dev), t(gy_np)
    grads = [torch.empty_like(x) for x in ins]
    cap = CapturedSolve(p, *ins, y, fac, ws, gy=gy, grads=grads)
    want = [ref_out["y"], ref_out["dc"], ref_out["dd"], ref_out["ds"], ref_out["du0"], ref_out["dw"]]
    for rep in range(3):
        for x in [y] + grads:
            x.zero_()
        torch.cuda.synchronize()
        cap.replay()
        torch.cuda.synchronize()
        for a, b in zip(want, [y] + grads):
            assert np.array_equal(a, b.double().cpu().numpy().reshape(a.shape)), rep
