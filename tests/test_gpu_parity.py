"""Parity of the HIP path (through the C-ABI) with the oracle.

Small cases span several chunks, several partition levels and ragged tails;
full-size configurations are checked on sampled instances, which the oracle
solves one by one."""
import numpy as np
import pytest

from oracle import banded, dense
from tests import fixtures as golden
from tests import gpu_helpers as H
from workloads import config, gaussian_batch, polynomial_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_06074_amd
    paper_2410_06074_amd.lib()   # fails loudly if the HIP library is missing


def _print(*a):
    print(*a, flush=True)


# ------------------------------------------------------------- C0 (dense oracle)
@pytest.mark.parametrize("mode", H.MODES)
def test_c0_forward_matches_dense_definition(mode):
    bt = H.io_batch(config("c0"), mode)
    out = H.run(bt, mode)
    c, d, s, u0, w = bt.instance(0)
    ref = {"y": dense.solve(c, d, s, u0, w)}
    kappa = banded.cond(bt)
    m = H.compare(bt, out, ref, [0])
    _print("c0", mode, H.summary(m), "kappa %.2e" % kappa[0])
    H.check(mode, m, kappa, bt.R, grads=False)
    assert out["info"].tolist() == [0]


# --------------------------------------------------- exact rational fixtures
@pytest.mark.parametrize("case", range(2))
def test_exact_fixture_elementwise(case):
    # T = 5, 9, 17.  Order 2 with chunks of 4 at every level: one, two and
    # four separators, and a second partition level at T = 17.  Order 1
    # (block size 2 compiles chunks of 8 and 16) with chunks of 8: none, one
    # and two separators.  The expected values are the rational oracle's,
    # rounded once to double.  y, dc, dd, ds and du0 are compared element by
    # element (max |x - x*| / max |x*| per array); dw, whose entries are sums
    # over every row of products of row residuals and adjoint rows that can
    # cancel to far below their terms (the initial rows' residual y - u is
    # ~1e-7 of y), in the term-scaled metric of tests/metrics.py.
    bt, gy, want = golden.load_exact(case)
    L = 4 if bt.R == 2 else 8
    out = H.run(bt, "fp64r", gy, chunk=L, chunk_upper=L)
    assert (out["info"] == 0).all()
    o = bt.offsets
    worst = {}
    for i in range(bt.n_inst):
        sl = slice(o[i], o[i + 1])
        for key in ("y", "dc", "dd", "ds"):
            worst[key] = max(worst.get(key, 0.0), H._raw(out[key][sl], want[key][sl])[1])
        worst["du0"] = max(worst.get("du0", 0.0), H._raw(out["du0"][i], want["du0"][i])[1])
        c, d, s, u0, w = bt.instance(i)
        sc = H.metrics.grad_scales(c, d, s, u0, w, want["y"][sl], want["lam"][sl])
        worst["dw_scaled"] = max(worst.get("dw_scaled", 0.0), H.metrics.grad_error(out["dw"][i], want["dw"][i],
                                                                                   sc["dw"]))
        worst["dw_raw"] = max(worst.get("dw_raw", 0.0), H._raw(out["dw"][i], want["dw"][i])[1])
    _print("exact fixture R=%d T=%s" % (bt.R, bt.T.tolist()), " ".join("%s=%.1e" % kv for kv in worst.items()))
    for key, v in worst.items():
        if key != "dw_raw":
            assert v <= 1e-10, key


# --------------------------------------------- ragged edge lengths, all modes
EDGE_T = [1, 2, 3, 7, 8, 9, 15, 16, 17, 63, 64, 65, 72, 73, 200, 513, 1000]


# (order, level-0 chunk, level >= 1 chunk): every compiled-in chunk length of each order
CHUNKS = [(1, 8, 8), (1, 16, 16), (2, 4, 16), (2, 8, 8), (2, 16, 4), (3, 4, 8), (3, 8, 4), (4, 4, 4)]


@pytest.mark.parametrize("R,chunk,upper", CHUNKS)
@pytest.mark.parametrize("mode", H.MODES)
def test_ragged_lengths_forward_and_gradients(R, chunk, upper, mode):
    # R = 4 at h ~ 0.01 has cond(M) ~ 1e17 (beyond double precision): use
    # longer steps there (cond ~ 1e8)
    bt = H.io_batch(gaussian_batch(len(EDGE_T), EDGE_T, R=R, seed=10 * R + chunk + upper,
                                   weights=(1.3, 0.8, 1.1), h0=0.2 if R == 4 else 0.01), mode)
    gy = np.random.default_rng(R).standard_normal(bt.c.shape)
    if mode == "fp32r":
        gy = gy.astype(np.float32).astype(np.float64)
    ref = H.reference(bt, gy)
    out = H.run(bt, mode, gy, chunk=chunk, chunk_upper=upper)
    m = H.compare(bt, out, ref, range(bt.n_inst))
    kappa = banded.cond(bt)
    _print("ragged R=%d L=%d/%d %s" % (R, chunk, upper, mode), H.summary(m), "kappa<=%.1e" % kappa.max())
    H.check(mode, m, kappa, bt.R)
    assert (out["info"] == 0).all()


# ------------------------------------------------------- full-size, sampled
def _sampled(name, mode, idx, n_inst=None, T=None, quad=True, eta_idx=None):
    """Run a full-size configuration with dl/dy = the loss gradient on the
    sampled instances idx (zero elsewhere); compare idx with the oracle and
    evaluate the backward error of y on the instances eta_idx (default all)."""
    bt = H.io_batch(config(name, n_inst=n_inst, T=T), mode)
    sub = bt.subset(idx)
    y_ref = banded.solve(sub, quad=quad)
    g_sub = H.loss_gradient(y_ref, bt.k)
    ref = banded.grad(sub, g_sub, quad=quad)
    gy = np.zeros_like(bt.c)
    o, so = bt.offsets, sub.offsets
    for j, i in enumerate(idx):
        gy[o[i]:o[i + 1]] = g_sub[so[j]:so[j + 1]]
    out = H.run(bt, mode, gy)
    m = H.compare(bt, out, ref, idx, ref_off=so)
    kappa = banded.cond(sub)
    eta_idx = range(bt.n_inst) if eta_idx is None else eta_idx
    esub = bt.subset(list(eta_idx))
    rows = np.concatenate([np.arange(o[i], o[i + 1]) for i in eta_idx])
    eta_all = (banded.backward_error(esub, out["y"][rows]), banded.backward_error(esub, out["y"][rows], normwise=True))
    return bt, out, m, kappa, eta_all


def _report(tag, m, kappa, eta_all, mode):
    eta_c, eta_n = eta_all
    _print(tag, H.summary(m), "kappa", " ".join("%.1e" % k for k in kappa),
           "| over %d instances: eta_n max %.1e, eta max %.1e median %.1e" % (
               len(eta_c), eta_n.max(), eta_c.max(), np.median(eta_c)))
    assert eta_n.max() <= 50.0 * H.U_WORK[mode], "P1 normwise backward error"
    if mode != "fp64":
        assert eta_c.max() <= 50.0 * H.U_WORK[mode], "P1 row-scaled backward error"


@pytest.mark.parametrize("mode", H.MODES)
def test_c1_full_batch_sampled(mode):
    idx = [0, 1, 511, 1024, 1535]
    bt, out, m, kappa, eta_all = _sampled("c1", mode, idx)
    _report("c1 " + mode, m, kappa, eta_all, mode)
    H.check(mode, m, kappa, bt.R)
    assert (out["info"] == 0).all()
    assert np.isfinite(out["y"]).all()


@pytest.mark.parametrize("mode", H.MODES)
def test_headline_t10k_sampled(mode):
    idx = [0, 767, 1535]
    bt, out, m, kappa, eta_all = _sampled("h", mode, idx)
    _report("h " + mode, m, kappa, eta_all, mode)
    H.check(mode, m, kappa, bt.R)
    assert (out["info"] == 0).all()


def test_c2_fp32r_sampled_reports_conditioning():
    # AR(1) coefficients with h = 1/365: cond(M) ~ 1e12 (above the fp32r
    # threshold, so P2 is reported; P1 holds on every instance checked)
    idx = [0, 5000, 16383, 32767]
    bt, out, m, kappa, eta_all = _sampled("c2", "fp32r", idx, n_inst=32768, eta_idx=range(0, 32768, 8))
    _report("c2 fp32r", m, kappa, eta_all, "fp32r")
    H.check("fp32r", m, kappa, bt.R)
    assert (out["info"] == 0).all()


@pytest.mark.parametrize("mode", ["fp32r", "fp64r"])
def test_c3_ragged_r3_sampled(mode):
    # R = 3, log-uniform weights: cond(M) 1e13..1e16 (beyond the fp32r
    # threshold everywhere, around the fp64r one); fp64r on the same inputs is
    # the accuracy reference the fp32r form is compared with
    cfg = config("c3")
    order = np.argsort(cfg.T)
    idx = sorted({0, 1, 1000, 2047, int(order[0]), int(order[1]), int(order[-1]), int(order[-2])})
    bt, out, m, kappa, eta_all = _sampled("c3", mode, idx)
    _report("c3 %s T=%s" % (mode, bt.T[idx].tolist()), m, kappa, eta_all, mode)
    H.check(mode, m, kappa, bt.R)
    assert (out["info"] == 0).all()


def test_c4_long_sequence_sampled():
    # T = 1e6: the double-precision oracle is the reference here (its own
    # error, ~1e-9, is far below the fp32r target); P1 in __float128 on all 32
    idx = [0, 31]
    bt, out, m, kappa, eta_all = _sampled("c4", "fp32r", idx, quad=False)
    _report("c4 fp32r", m, kappa, eta_all, "fp32r")
    H.check("fp32r", m, kappa, bt.R)
    assert (out["info"] == 0).all()


# ---------------------------------------------------------- properties
@pytest.mark.parametrize("R", [1, 2, 3])
def test_polynomial_trajectory_recovered_at_long_T(R):
    bt, exact = polynomial_batch(4, 20000 if R < 3 else 4000, R, seed=R)
    out = H.run(bt, "fp64r")
    err = H.metrics.rel_by_order(out["y"], exact, bt.k)
    _print("poly R=%d" % R, ["%.1e" % e for e in err])
    assert err[0] < 1e-9 and max(err) < (1e-6 if R < 3 else 1e-4)


@pytest.mark.parametrize("mode", ["fp64r", "fp32r"])
def test_repeat_runs_bitwise_identical_and_launch_shapes_agree(mode):
    bt = H.io_batch(config("c1", n_inst=200, T=777), mode)
    gy = np.random.default_rng(0).standard_normal(bt.c.shape)
    a = H.run(bt, mode, gy)
    b = H.run(bt, mode, gy)
    for key in ("y", "dc", "dd", "ds", "du0", "dw"):
        assert np.array_equal(a[key], b[key]), key
    # persistent grid-stride launches and multi-wave workgroups (one LDS slice per wave)
    for block, max_blocks in ((64, 7), (256, 0), (128, 3)):
        c = H.run(bt, mode, gy, block=block, max_blocks=max_blocks)
        for key in ("y", "dc", "dd", "ds", "du0", "dw"):
            assert np.array_equal(a[key], c[key]), (block, max_blocks, key)


@pytest.mark.parametrize("n_init", [0, 1, 3])
def test_initial_row_counts(n_init):
    # n_init = 0 (no initial rows) is an extension.  T = 1 has one governing
    # row and n_init initial rows for three unknowns, so it is solvable only
    # for n_init >= 2
    T = [1, 5, 64, 333, 1000] if n_init >= 2 else [5, 64, 333, 1000]
    bt = gaussian_batch(len(T), T, R=2, seed=40 + n_init, n_init=n_init, weights=(1.1, 0.7, 1.3))
    gy = np.random.default_rng(n_init).standard_normal(bt.c.shape)
    ref = H.reference(bt, gy)
    kappa = banded.cond(bt)
    out = H.run(bt, "fp64r", gy)
    m = H.compare(bt, out, ref, range(bt.n_inst))
    _print("n_init=%d" % n_init, H.summary(m), "kappa<=%.1e" % kappa.max())
    assert (out["info"] == 0).all()
    H.check("fp64r", m, kappa, bt.R)


@pytest.mark.parametrize("mode", ["fp64", "fp64r", "fp32r"])
@pytest.mark.parametrize("t_init,n_init", [(2, 2), (9, 3), (40, 1)])
def test_several_initial_points(mode, t_init, n_init):
    # Eq. 5 at the first T_init points: T_init inside the first level-0 chunk,
    # spanning several chunks, and longer than the shortest instances (whose
    # points past the end carry no row and get du0 = 0)
    T = [3, 5, 8, 9, 17, 64, 333, 1000]
    bt = H.io_batch(gaussian_batch(len(T), T, R=2, seed=50 + t_init, n_init=n_init, weights=(1.2, 0.9, 1.3),
                                   t_init=t_init), mode)
    gy = np.random.default_rng(t_init).standard_normal(bt.c.shape)
    if mode == "fp32r":
        gy = gy.astype(np.float32).astype(np.float64)
    ref = H.reference(bt, gy)
    kappa = banded.cond(bt)
    out = H.run(bt, mode, gy)
    assert out["plan"].init_points == t_init
    m = H.compare(bt, out, ref, range(bt.n_inst))
    _print("init points %d x %d %s" % (t_init, n_init, mode), H.summary(m), "kappa<=%.1e" % kappa.max())
    assert (out["info"] == 0).all()
    H.check(mode, m, kappa, bt.R)
    du0 = out["du0"].reshape(bt.n_inst, t_init, n_init)
    for i, Ti in enumerate(T):
        assert np.all(du0[i, Ti:] == 0.0)


@pytest.mark.parametrize("mode", ["fp64r", "fp32r"])
def test_upper_levels_in_one_launch(mode):
    # chunks 4 / 4: T = 1028 gives 64 level-1 chunks (the most one wave
    # takes), so the in-LDS levels hold 63, 15 and 3 nodes; adding T = 1100
    # (69 chunks) moves the one-wave-per-instance launch up to level 2
    for T, top in (([5, 17, 65, 257, 1000, 1025, 1028], 1), ([5, 17, 65, 257, 1028, 1100], 2)):
        bt = H.io_batch(gaussian_batch(len(T), T, R=2, seed=len(T) + top, weights=(1.1, 0.9, 1.2)), mode)
        gy = np.random.default_rng(top).standard_normal(bt.c.shape)
        if mode == "fp32r":
            gy = gy.astype(np.float32).astype(np.float64)
        ref = H.reference(bt, gy)
        kappa = banded.cond(bt)
        out = H.run(bt, mode, gy, chunk=4, chunk_upper=4)
        assert out["plan"].top_level == top
        m = H.compare(bt, out, ref, range(bt.n_inst))
        _print("upper levels %s top=%d" % (mode, top), H.summary(m))
        assert (out["info"] == 0).all()
        H.check(mode, m, kappa, bt.R)


@pytest.mark.parametrize("mode", ["fp64r", "fp32r"])
def test_upper_levels_four_instances_per_wave(mode):
    # 4 x 4 blocks (R = 3) take 16 lanes per instance in the one-launch upper
    # levels.  Chunks 4 / 4: T = 260 gives 16 level-1 chunks (the most a
    # group takes); T = 261 (17 chunks) moves the launch up to level 2.  Seven
    # and six instances leave the last wave's groups partly empty, and T = 5
    # has no node at level 2.
    for T, top in (([5, 17, 65, 100, 200, 257, 260], 1), ([5, 17, 65, 257, 260, 261], 2)):
        bt = H.io_batch(gaussian_batch(len(T), T, R=3, seed=40 + len(T) + top, weights=(1.1, 0.9, 1.2), h0=0.05),
                        mode)
        gy = np.random.default_rng(top + 7).standard_normal(bt.c.shape)
        if mode == "fp32r":
            gy = gy.astype(np.float32).astype(np.float64)
        ref = H.reference(bt, gy)
        kappa = banded.cond(bt)
        out = H.run(bt, mode, gy, chunk=4, chunk_upper=4)
        assert out["plan"].top_level == top
        m = H.compare(bt, out, ref, range(bt.n_inst))
        _print("upper levels 4x4 %s top=%d" % (mode, top), H.summary(m))
        assert (out["info"] == 0).all()
        H.check(mode, m, kappa, bt.R)


@pytest.mark.parametrize("mode", ["fp64r", "fp32r"])
def test_weight_gradients_summed_over_several_workgroups(mode):
    # few long instances: each instance's per-chunk weight-gradient partials
    # are summed by several workgroups (slices of >= 1024 chunks) and the
    # slices added in order; ragged lengths give unequal slices
    T = [30000, 25000, 20001, 9000]
    bt = H.io_batch(gaussian_batch(len(T), T, R=2, seed=77, weights=(1.1, 0.9, 1.2)), mode)
    gy = np.random.default_rng(77).standard_normal(bt.c.shape)
    if mode == "fp32r":
        gy = gy.astype(np.float32).astype(np.float64)
    ref = H.reference(bt, gy)
    kappa = banded.cond(bt)
    out = H.run(bt, mode, gy)
    m = H.compare(bt, out, ref, range(bt.n_inst))
    _print("dw split %s" % mode, H.summary(m))
    assert (out["info"] == 0).all()
    H.check(mode, m, kappa, bt.R)


def test_failure_reported_per_instance_and_isolated():
    bt = gaussian_batch(4, [50, 300, 1000, 90], R=2, seed=3)
    clean = H.run(bt, "fp64r")
    bad = bt.subset(range(4))
    o = bad.offsets
    bad.c[o[2] + 500, 1] = np.nan          # NaN coefficient in instance 2
    bad.w[1] = (0.0, 1.0, 0.0)             # instance 1: only initial rows -> zero pivots
    out = H.run(bad, "fp64r")
    _print("info", out["info"].tolist())
    assert out["info"][0] == 0 and out["info"][3] == 0
    assert out["info"][1] > 0 and out["info"][2] > 0
    for i in (0, 3):
        assert np.array_equal(out["y"][o[i]:o[i + 1]], clean["y"][o[i]:o[i + 1]])
    assert not np.isfinite(out["y"][o[2]:o[3]]).all()


def test_workspace_too_small_is_rejected():
    import torch
    from paper_2410_06074_amd import Plan, SmnnError
    bt = gaussian_batch(2, 100, R=2, seed=0)
    p = Plan(2, 2, 2, 100, mode="fp64r")
    dev = torch.device("cuda:0")
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    y = torch.empty((200, 3), dtype=torch.float64, device=dev)
    small = torch.empty(max(p.workspace_bytes - 256, 256), dtype=torch.uint8, device=dev)
    with pytest.raises(SmnnError) as e:
        p.forward(t(bt.c), t(bt.b), t(bt.h), t(bt.u0), t(bt.w), y, p.new_factor(dev), small)
    assert e.value.status == 3


# ------------------------------------------- refinement step counts 0, 1, 2
@pytest.mark.parametrize("mode", ["fp64r", "fp32r"])
def test_refinement_steps(mode):
    # several levels (T up to 2000 with chunks 4 / 8) and, separately, a batch
    # whose instances are all a single level-0 chunk (no separator level)
    for T in ([2000, 1, 37, 512, 1999], [1, 2, 3, 4, 4]):
        bt = H.io_batch(gaussian_batch(len(T), T, R=2, seed=77 + len(T) + T[-1], weights=(0.9, 1.2, 1.4)), mode)
        gy = np.random.default_rng(5).standard_normal(bt.c.shape)
        if mode == "fp32r":
            gy = gy.astype(np.float32).astype(np.float64)
        ref = H.reference(bt, gy)
        kappa = banded.cond(bt)
        errs = []
        for steps in (0, 1, 2):
            out = H.run(bt, mode, gy, chunk=4, chunk_upper=8, refine_steps=steps)
            assert out["plan"].refine_steps == steps
            m = H.compare(bt, out, ref, range(bt.n_inst))
            errs.append(m)
            _print("refine %s T=%s steps=%d" % (mode, T, steps), H.summary(m))
            if steps == 0:
                # no refinement: the plain FP64 solve's bound (fp32r: its output rounding on top)
                if mode == "fp64r":
                    H.check("fp64", m, kappa, bt.R)
                else:
                    assert m["y"].max() <= 1e-3
            else:
                H.check(mode, m, kappa, bt.R)
        assert errs[2]["y"].max() <= max(2 * errs[1]["y"].max(), 1e-13)
