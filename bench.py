#!/usr/bin/env python3
"""Throughput of the batched S-MNN least-squares solve (forward + backward) on one MI355X.

One step = smnn_forward + smnn_backward over the whole synthetic batch, with
every input already resident in HBM (dl/dy = 2 y^(0), the gradient of
sum_t (y_t^(0))^2, is formed once from the first solution and is an input of
the backward like any other).  The default workload is the headline
configuration: 512 x 3 = 1536 instances, T = 10,000 steps, R = 2.

Prints ONE JSON line (rank 0).  Besides the contract fields it carries
  roofline      the dominant kernel's algorithmic bytes per launch divided by
                its mean launch time (hipEvent pairs recorded by the library
                around every launch during a second, traced copy of the timed
                steps), against the 8 TB/s HBM peak;
  cpu_baseline  the oracle (oracle/banded.c, OpenMP) timed on a bounded
                sample of the same workload on the host's cores;
  modes         steps/s, ms/step and sampled error against the FP64 oracle
                for every solver mode measured (the headline mode included);
  sched_frac    steps/s times the bytes per step that the paper's two-sweep
                schedule (Alg. 3 factorisation sweep, Alg. 4 substitution
                sweeps, every sweep streaming its operands from memory; one
                more pair of sweeps per refinement step, forward and adjoint)
                would move, against the 8 TB/s peak: a fixed per-step
                denominator that kernel fusion cannot inflate.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solved ODE steps/sec fwd+bwd (T=10k, R=2); % HBM roofline; err vs FP64"
HBM_PEAK_GBS = 8000.0
RHS_BETA, RHS_RESID, RHS_G, RHS_GRESID = 0, 1, 2, 3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ------------------------------------------------------------ byte model
def kernel_bytes(rec, plan, io):
    """Algorithmic HBM bytes of one traced launch: every array the launch must
    read once plus every array it must write once (metadata excluded).
    K = unknowns per point (V (R+1)), QE governing equations per point, per-row
    weights add QE + 1 values per step to the reads (and to the gradient's
    writes); separator records are a packed diagonal block and a coupling
    block (wide blocks: two full halves of the diagonal block and the coupling
    block, with two halves of the right-hand side)."""
    kind, level, rhs, out = rec[0], rec[1], rec[2], rec[3]
    K = plan.k
    QE = getattr(plan, "equations", 1)
    rows = getattr(plan, "row_weights", False)
    wide = K > 5
    Q = K * (K + 1) // 2
    REC = 3 * K * K if wide else Q + K * K
    RHSW = 2 * K if wide else K
    lv = plan.levels                       # [(nodes, chunks)] per level
    S, G0 = lv[0]
    N = plan.n_inst
    n = lambda l: lv[l][0] if l < len(lv) else 0
    n_initial = N * getattr(plan, "n_initial", plan.n_init)
    per_inst = (N * (0 if rows else 3) + n_initial * (2 if rows else 1)) * io
    wts = (QE + 1) if rows else 0          # per-row weights read per step
    base = QE * K + 1 + wts                # c, s (and weights) per step
    d_el = QE
    if kind == "reduce0":
        el = base + (d_el if rhs in (RHS_BETA, RHS_RESID) else 0) + (K if rhs in (RHS_G, RHS_GRESID) else 0) \
            + (K if rhs in (RHS_RESID, RHS_GRESID) else 0)
        w = n(1) * RHSW * 8 + (n(1) * REC * 8 if rhs == RHS_BETA else 0)
        return S * el * io + per_inst + w
    if kind == "reduceN":
        w = n(level + 1) * RHSW * 8 + (n(level + 1) * REC * 8 if rhs == RHS_BETA else 0)
        return n(level) * (REC + RHSW) * 8 + w
    if kind == "backsubN":
        return n(level) * (REC + RHSW) * 8 + n(level + 1) * K * 8 + n(level) * K * 8
    if kind == "backsub0":
        grad = out == 1
        el = base + (d_el if (rhs in (RHS_BETA, RHS_RESID) or grad) else 0) + (K if rhs in (RHS_G, RHS_GRESID) else 0) \
            + (K if rhs in (RHS_RESID, RHS_GRESID) else 0) + (K if grad else 0)
        wr = ((QE * K + QE + 1 + wts) * S * io + (0 if rows else G0 * 3 * 8) + n_initial * (2 if rows else 1) * io
              if grad else K * S * io)
        return S * el * io + per_inst + n(1) * K * 8 + wr
    if kind == "backsub_reduce0":          # rhs = the solve's form (beta or dl/dy)
        el = base + (d_el if rhs == RHS_BETA else 0) + (K if rhs == RHS_G else 0)
        return S * el * io + per_inst + n(1) * K * 8 + K * S * io + n(1) * K * 8
    if kind == "top":                      # levels >= level: its records and rhs in, its x out
        return n(level) * (REC + K) * 8 + n(level) * K * 8
    if kind == "dw_reduce":
        return G0 * 3 * 8 + N * 3 * io
    return 0


# ------------------------------------------------------------- workload
def sched_bytes_per_step(R, mode, refine):
    """Bytes per solved step of the two-sweep schedule (block size k = R+1,
    q = k(k+1)/2 packed factor entries): forward t-up sweep reads the inputs
    (k+2) and writes L (q), P (k^2), alpha (k); t-down sweep reads P, alpha and
    writes y; the adjoint reads g, P, L, writes alpha, then reads P, alpha, y,
    the inputs and writes the gradients (k+2): 2q + 4k^2 + 10k + 6 elements.
    Each refinement step adds, forward and adjoint, the residual's reads and
    one more pair of substitution sweeps: 2q + 4k^2 + 13k + 4 elements."""
    k = R + 1
    q = k * (k + 1) // 2
    elems = (2 * q + 4 * k * k + 10 * k + 6) + refine * (2 * q + 4 * k * k + 13 * k + 4)
    return elems * (4 if mode == "fp32r" else 8)


def comp_bytes_per_step(bt, mode):
    """Compulsory bytes per solved step of a forward + backward through this
    ABI (the lower bound): read the inputs c, b, h (Q K + Q + 1 values with K
    = V (R+1) unknowns per point; k + 2 for one variable), write the paper's
    per-step factor L_t, P_t (q + K^2, q = K (K+1) / 2) and y (K); then read
    dl/dy, y, the factor and the inputs once each and write the gradients (as
    many as the inputs): 3 (Q K + Q + 1) + 2 (q + K^2) + 3 K values, 54 for
    one order-2 variable, in the I/O element size (per-row weights add Q + 1
    inputs and as many gradients)."""
    K, Q = bt.block, bt.Q
    q = K * (K + 1) // 2
    inputs = Q * K + Q + 1 + ((Q + 1) if bt.wrow is not None else 0)
    return (3 * inputs + 2 * (q + K * K) + 3 * K) * (4 if mode == "fp32r" else 8)


def make_workload(name, n_inst=None, T=None):
    from workloads import config
    return config(name, n_inst=n_inst, T=T)


def pack_weights(bt):
    """The per-row weight buffer of the C-ABI (governing, initial, smoothness)."""
    import numpy as np
    wr = bt.wrow
    return np.concatenate([np.ravel(wr["wg"]), np.ravel(wr["wi"]), np.ravel(wr["ws"])])


def describe(name, bt, mode):
    sizes = {"h": "512x3", "c1": "512x3", "c2": "256x128", "c3": "2048", "c4": "4x8", "c0": "1", "hw": "512x3",
             "v2": "1536", "v3": "512"}
    T = int(bt.T[0]) if (bt.T == bt.T[0]).all() else "ragged %d..%d" % (bt.T.min(), bt.T.max())
    shape = "" if bt.V == 1 and bt.Q == 1 and bt.wrow is None else ", V=%d, Q=%d%s" % (
        bt.V, bt.Q, ", per-row weights" if bt.wrow is not None else "")
    return {"workload": "%s: %s = %d instances, T=%s, R=%d%s, forward+adjoint, mode %s"
                        % (name, sizes.get(name, "?"), bt.n_inst, T, bt.R, shape, mode),
            "instances": int(bt.n_inst), "steps_per_instance": T, "order_R": int(bt.R),
            "variables": int(bt.V), "equations": int(bt.Q), "per_row_weights": bt.wrow is not None,
            "total_steps": int(bt.total_steps), "mode": mode,
            "inputs": "seeded synthetic (workloads.config('%s'))" % name}


# --------------------------------------------------------------- GPU run
def run_mode(bt, mode, steps, warmup, sample_idx, chunk=0, chunk_upper=0, graph=True, tune=False, block=0,
             max_blocks=0):
    import numpy as np
    import torch
    from paper_2410_06074_amd import Plan
    from oracle import banded
    from tests import metrics

    dev = torch.device("cuda:0")
    dt = torch.float32 if mode == "fp32r" else torch.float64
    io = 4 if mode == "fp32r" else 8
    steps_arg = int(bt.T[0]) if (bt.T == bt.T[0]).all() else bt.T
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=dev).to(dt)
    S0 = bt.total_steps
    rows = bt.wrow is not None
    c, b, h = t(np.reshape(bt.c, (S0, -1))), t(np.reshape(bt.b, (-1,))), t(bt.h)
    u0 = t(np.reshape(bt.u0, (bt.n_inst, -1)))
    w = t(pack_weights(bt)) if rows else t(bt.w)
    tuned = None
    if tune:
        from paper_2410_06074_amd import autotune
        gy0 = torch.ones_like(c)
        tuned = autotune(bt.R, bt.n_init, bt.n_inst, steps_arg, mode, c, b, h, u0, w, gy0, iters=2)
        chunk, chunk_upper = tuned["chunk"], tuned["chunk_upper"]
        block, max_blocks = tuned["block"], tuned["max_blocks"]
        log("  autotuned:", {k: v for k, v in tuned.items() if k != "candidates"})
    plan = Plan(bt.R, bt.n_init, bt.n_inst, steps_arg, mode=mode, chunk=chunk, chunk_upper=chunk_upper,
                block=block, max_blocks=max_blocks, variables=bt.V, equations=bt.Q, row_weights=rows)
    S, K = plan.total_steps, plan.k
    y = torch.empty((S, K), dtype=dt, device=dev)
    fac, ws = plan.new_factor(dev), plan.new_workspace(dev)
    dc, db, dh = torch.empty_like(c), torch.empty_like(b), torch.empty_like(h)
    du0, dw = torch.empty_like(u0), torch.empty_like(w)
    plan.forward(c, b, h, u0, w, y, fac, ws)
    gy = torch.zeros_like(y)
    gy[:, 0::bt.k] = 2.0 * y[:, 0::bt.k]       # loss: sum of squares of every variable's value
    torch.cuda.synchronize()

    def step():
        plan.forward(c, b, h, u0, w, y, fac, ws)
        plan.backward(c, b, h, u0, w, y, fac, gy, dc, db, dh, du0, dw, ws)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms_eager = e0.elapsed_time(e1) / steps
    ms = ms_eager
    if graph:
        # the whole forward+backward launch sequence as one hipGraph replay
        from paper_2410_06074_amd import CapturedSolve
        cap = CapturedSolve(plan, c, b, h, u0, w, y, fac, ws, gy=gy, grads=(dc, db, dh, du0, dw))
        for _ in range(warmup):
            cap.replay()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            cap.replay()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps

    # traced copy of the timed steps: one event pair around every launch
    launches_per_step = 64 * max(1, len(plan.levels))
    plan.trace(launches_per_step * steps)
    e2, e3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e2.record()
    for _ in range(steps):
        step()
    e3.record()
    torch.cuda.synchronize()
    ms_traced = e2.elapsed_time(e3) / steps
    trace = plan.trace_read(launches_per_step * steps + 16)
    plan.trace(0)
    per_kind = {}
    for r in trace:
        key = "%s/l%d/rhs%d/out%d" % r[:4]
        d = per_kind.setdefault(key, {"ms": 0.0, "n": 0, "bytes": kernel_bytes(r, plan, io)})
        d["ms"] += r[4]
        d["n"] += 1
    step_bytes = sum(v["bytes"] * v["n"] for v in per_kind.values()) / steps

    # error against the FP64 oracle on sampled instances (the oracle runs on the
    # same, possibly float32-rounded, inputs)
    yn = y.double().cpu().numpy()
    sub = bt.subset(sample_idx)
    if mode == "fp32r":
        sub = sub.astype(np.float32).astype(np.float64)
    ref = banded.solve(sub)
    o, so = bt.offsets, sub.offsets
    err = 0.0
    for j, i in enumerate(sample_idx):
        err = max(err, max(metrics.rel_by_order(yn[o[i]:o[i + 1]], ref[so[j]:so[j + 1]], K)))
    kappa = [float("%.3g" % k) for k in banded.cond(sub)]
    return {"kappa": kappa, "max_blocks": max_blocks, "plan": plan, "ms": ms, "ms_eager": ms_eager, "graph": graph, "tuned": tuned, "ms_traced": ms_traced, "per_kind": per_kind, "step_bytes": step_bytes,
            "err": err, "levels": plan.levels, "chunk": [plan.chunk, plan.chunk_upper], "refine": plan.refine_steps}


KERNEL_SOURCES = ("smnn_kernels.hip", "smnn_core.h", "smnn_internal.h")


def kernel_sources_sha256():
    """Digest of the kernel sources: a measured counter value is only reported
    for the kernels it was measured on."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2410_06074_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counter_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summaries
    (profiles/*.md lines 'traffic <kernel> bytes_per_launch=<B>
    kernel_sources_sha256=<digest>'), or None if none was taken on the
    current kernel sources."""
    import glob
    import re
    digest = kernel_sources_sha256()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as f:
            for m in re.finditer(r"^traffic (\S+) bytes_per_launch=(\d+) kernel_sources_sha256=([0-9a-f]+)",
                                 f.read(), re.M):
                if m.group(1) == kernel and m.group(3) == digest:
                    return int(m.group(2))
    return None


def copy_calibration():
    """Plain device-to-device copy of a known size: the reference the HBM byte
    counters (FETCH_SIZE, WRITE_SIZE) are scaled by."""
    import torch
    n = 64 * 1024 * 1024                      # 64 Mi doubles = 512 MiB each way
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_per_direction": n * 8, "copies": 3}), flush=True)
    return 0


def copy_rate(reps=20):
    """Plain streaming rates on this GPU, timed with events: the calibration
    copy (1 read : 1 write) and elementwise kernels reading two and three
    arrays per array written (2 : 1, 3 : 1), which bracket the gradient
    kernel's mix (about 2.6 : 1).  These are the ceilings a kernel with that
    read/write mix can reach, beside the published peak."""
    import torch
    n = 64 * 1024 * 1024
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    x2 = torch.ones_like(x)
    x3 = torch.ones_like(x)
    y = torch.empty_like(x)
    kinds = (("copy", 1, lambda: y.copy_(x)),
             ("add", 2, lambda: torch.add(x, x2, out=y)),
             ("addcmul", 3, lambda: torch.addcmul(x, x2, x3, out=y)))
    out = {"bytes_per_array": n * 8}
    for name, reads, fn in kinds:
        for _ in range(3):
            fn()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(reps):
            fn()
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / reps
        out[name] = {"reads_per_write": reads, "ms": round(ms, 4),
                     "gbs_read_plus_write": round((reads + 1) * n * 8 / (ms * 1e-3) / 1e9, 1)}
    print(json.dumps(out), flush=True)
    return 0


def roofline(res):
    dom_key, dom = max(res["per_kind"].items(), key=lambda kv: kv[1]["ms"])
    avg_ms = dom["ms"] / dom["n"]
    achieved = dom["bytes"] / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": dom_key, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": counter_traffic(dom_key),
            "bytes_per_launch": int(dom["bytes"]), "avg_launch_ms": round(avg_ms, 5),
            "share_of_step": round(dom["ms"] / max(1e-9, sum(v["ms"] for v in res["per_kind"].values())), 3)}


# ------------------------------------------------------------ CPU baseline
def cpu_baseline(bt, target_s=15.0):
    """The oracle (oracle/banded.c, OpenMP over instances) on a bounded sample
    of the same workload: as many instances as take about target_s seconds,
    repeated over the whole batch when even all of it takes less."""
    import numpy as np
    from oracle import banded
    probe = bt.subset(list(range(min(8, bt.n_inst))))
    t0 = time.perf_counter()
    banded.grad(probe, np.zeros_like(probe.c))
    per_inst = max(time.perf_counter() - t0, 1e-6) / probe.n_inst
    n = int(min(bt.n_inst, max(probe.n_inst, target_s / per_inst)))
    sub = bt.subset(list(range(n)))
    gy = np.zeros_like(sub.c)
    reps, dt = 0, 0.0
    while reps == 0 or (dt < 0.5 * target_s and reps < 50):
        t0 = time.perf_counter()
        banded.grad(sub, gy)               # forward solve + adjoint + gradients
        dt += time.perf_counter() - t0
        reps += 1
    return {"value": round(reps * sub.total_steps / dt, 1), "unit": "steps/s", "cores": banded.threads(),
            "kind": "oracle",
            "sample": "%d of %d instances (T=%d each) x %d repetitions, banded-QR oracle forward + adjoint + "
                      "gradients, %.1f s" % (n, bt.n_inst, int(bt.T[0]), reps, dt)}


def lorenz_step_times():
    """One JSON line: ms per optimisation step (window upload, solve forward,
    loss, adjoint backward, Adam on a1..a7) of paper_2410_06074_amd.lorenz."""
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    from paper_2410_06074_amd.lorenz import step_time
    rows = []
    for B, T in ((512, 50), (512, 5), (512, 500), (64, 50), (4096, 50)):
        ms = step_time(B, T)
        log("lorenz B=%d T=%d: %.3f ms/step" % (B, T, ms))
        rows.append({"batch": B, "seq_len": T, "ms_per_step": round(ms, 4)})
    print(json.dumps({"metric": "Lorenz discovery optimisation step (Alg. 5), fp64r, R=2", "unit": "ms",
                      "higher_is_better": False, "data": "synthetic (RK4 Lorenz trajectory)", "rows": rows}),
          flush=True)
    return 0


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="h", choices=["h", "c1", "c2", "c3", "c4", "hw", "v2", "v3"])
    ap.add_argument("--mode", default="fp64r", choices=["fp64", "fp64r", "fp32r"])
    ap.add_argument("--side-modes", default="fp64,fp32r", help="extra modes measured (comma list, '' for none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--chunk", type=int, default=0, help="time steps per lane at level 0 (0: library default)")
    ap.add_argument("--chunk-upper", type=int, default=0, help="nodes per lane at levels >= 1 (0: default)")
    ap.add_argument("--no-graph", action="store_true", help="time eager launches instead of hipGraph replays")
    ap.add_argument("--autotune", action="store_true", help="pick the launch mapping with smnn_autotune first")
    ap.add_argument("--block", type=int, default=0, help="threads per workgroup (0: library default)")
    ap.add_argument("--max-blocks", type=int, default=0,
                    help="persistent launches of at most this many workgroups, tiles from a device work queue")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 512 MiB device copy (reference for the HBM byte counters)")
    ap.add_argument("--copy-rate", action="store_true",
                    help="only time that copy: the read + write rate a plain streaming kernel reaches")
    ap.add_argument("--lorenz", action="store_true",
                    help="only time the Lorenz discovery training step (Alg. 5) on the batch / window grid of "
                         "the paper's Lorenz performance table")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration()
    if args.copy_rate:
        return copy_rate()
    if args.lorenz:
        return lorenz_step_times()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: instances are solved independently and there is no "
              "multi-GPU path; run with --gpus 1", file=sys.stderr)
        return 2
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    import paper_2410_06074_amd
    paper_2410_06074_amd.lib()

    log("generating workload", args.config)
    bt = make_workload(args.config)
    sample = sorted({0, bt.n_inst // 2, bt.n_inst - 1})
    modes = [args.mode] + [m for m in args.side_modes.split(",") if m and m != args.mode]
    results = {}
    for m in modes:
        log("mode", m)
        results[m] = run_mode(bt, m, args.steps, args.warmup, sample, chunk=args.chunk,
                              chunk_upper=args.chunk_upper, graph=not args.no_graph, tune=args.autotune,
                              block=args.block, max_blocks=args.max_blocks)
        r = results[m]
        log("  %.3f ms/step (eager %.3f, traced %.3f), %.3e steps/s, err %.2e, chunk %s, levels %s"
            % (r["ms"], r["ms_eager"], r["ms_traced"], bt.total_steps / (r["ms"] * 1e-3), r["err"], r["chunk"],
               r["levels"]))
    head = results[args.mode]
    value = bt.total_steps / (head["ms"] * 1e-3)
    scalar_form = bt.V == 1 and bt.Q == 1 and bt.wrow is None   # the paper's schedule model covers these
    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.mode == "fp32r" else "f64",
        "data": "synthetic",
        "config": dict(describe(args.config, bt, args.mode),
                       **({"persistent_max_blocks": args.max_blocks} if args.max_blocks else {})),
        "err_vs_fp64_oracle": head["err"],
        "roofline": roofline(head),
        "step_hbm_bytes_algorithmic": int(head["step_bytes"]),
        "step_bandwidth_frac": round(head["step_bytes"] / (head["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "comp_bytes_per_step": comp_bytes_per_step(bt, args.mode),
        "comp_frac": round(value * comp_bytes_per_step(bt, args.mode) / 1e9 / HBM_PEAK_GBS, 4),
        "sampled_instances": sample,
        "sampled_cond_M": head["kappa"],
        "sched_bytes_per_step": sched_bytes_per_step(bt.R, args.mode, head["refine"]) if scalar_form else None,
        "sched_frac": round(value * sched_bytes_per_step(bt.R, args.mode, head["refine"]) / 1e9 / HBM_PEAK_GBS, 4)
                      if scalar_form else None,
        "modes": {m: {"steps_per_s": round(bt.total_steps / (r["ms"] * 1e-3), 1), "ms_per_step": round(r["ms"], 5),
                      "err_vs_fp64_oracle": r["err"], "refine_steps": r["refine"], "chunk": r["chunk"],
                      "roofline_frac": roofline(r)["frac"], "eager_ms_per_step": round(r["ms_eager"], 5),
                      "timing": "hipGraph replay" if r["graph"] else "eager launches",
                      "step_bandwidth_frac": round(r["step_bytes"] / (r["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                      "sched_frac": None if not scalar_form else round(bt.total_steps / (r["ms"] * 1e-3) * sched_bytes_per_step(bt.R, m, r["refine"])
                                          / 1e9 / HBM_PEAK_GBS, 4),
                      "traced_ms_per_step": round(r["ms_traced"], 5)}
                  for m, r in results.items()},
        "kernels": {k: {"avg_ms": round(v["ms"] / v["n"], 5), "launches": v["n"],
                        "gbs": round(v["bytes"] / (v["ms"] / v["n"] * 1e-3) / 1e9, 1)}
                    for k, v in sorted(head["per_kind"].items(), key=lambda kv: -kv[1]["ms"])},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline")
        line["cpu_baseline"] = cpu_baseline(bt, args.cpu_seconds)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
