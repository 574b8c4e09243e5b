"""smnn_forward_noalloc (the forward solve on the library's static device
workspace) against smnn_forward with a caller workspace, through the C-ABI:
two calls in a row, the second with a smaller batch, so the second runs on
what the first left in the shared array."""
import numpy as np
import pytest

from tests import gpu_helpers as H
from workloads import gaussian_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_06074_amd
    paper_2410_06074_amd.lib()


def _both(bt, mode):
    import torch
    from paper_2410_06074_amd import Plan
    dev = torch.device("cuda:0")
    dt = H.dtype_for(mode)
    steps = int(bt.T[0]) if np.all(bt.T == bt.T[0]) else bt.T
    p = Plan(bt.R, bt.n_init, bt.n_inst, steps, mode=mode)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    c, b, h, u0, w = t(bt.c), t(bt.b), t(bt.h), t(bt.u0.reshape(bt.n_inst, -1)), t(bt.w)
    y_ref = torch.empty((p.total_steps, p.k), dtype=dt, device=dev)
    f_ref = p.new_factor(dev)
    i_ref = torch.full((bt.n_inst,), -7, dtype=torch.int32, device=dev)
    p.forward(c, b, h, u0, w, y_ref, f_ref, p.new_workspace(dev), i_ref)
    y = torch.full((p.total_steps, p.k), float("nan"), dtype=dt, device=dev)
    f = p.new_factor(dev)
    inf = torch.full((bt.n_inst,), -7, dtype=torch.int32, device=dev)
    p.forward_noalloc(c, b, h, u0, w, y, f, inf)
    torch.cuda.synchronize(dev)
    return p, y_ref.double().cpu().numpy(), y.double().cpu().numpy(), i_ref.cpu().numpy(), inf.cpu().numpy()


@pytest.mark.parametrize("mode", ["fp64r", "fp32r", "fp64"])
def test_noalloc_forward_matches_forward_twice(mode):
    # first a larger ragged batch (several partition levels), then a smaller one
    for n, T, seed in ((300, [1, 5, 64, 1000, 3000], 1), (7, [2, 17, 200], 2)):
        Ts = [T[i % len(T)] for i in range(n)]
        bt = H.io_batch(gaussian_batch(n, Ts, R=2, seed=seed, weights=(1.1, 0.9, 1.2)), mode)
        print("noalloc %s n=%d workspace" % (mode, n), flush=True)
        p, y_ref, y, i_ref, inf = _both(bt, mode)
        print("  workspace %d bytes" % p.workspace_bytes, flush=True)
        assert (i_ref == 0).all() and (inf == 0).all()
        # same kernels on the same inputs: identical results
        assert np.array_equal(y, y_ref)


def test_noalloc_rejects_a_workspace_beyond_the_static_array():
    from paper_2410_06074_amd import Plan
    # 4096 x 20,000 steps, fp64r: the plan's workspace is far above 128 MiB;
    # the size is checked before any argument is used
    p = Plan(2, 2, 4096, 20000, mode="fp64r")
    assert p.workspace_bytes > (128 << 20)
    st = p._L.smnn_forward_noalloc(p._h, None, None, None, None, None, None, None, 0, None, None)
    assert st == 3      # SMNN_ERR_WORKSPACE
