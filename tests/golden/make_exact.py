"""Write tests/golden/exact_small.json and exact_general.json: exact solutions
and gradients of tiny ragged batches (T = 5, 9, 17; R = 1, 2; and, in
exact_general.json, per-row weights and two coupled variables), computed by
the rational oracle (oracle/exact.py) and rounded once to double.

    python tests/golden/make_exact.py

Inputs are the seeded ``workloads.gaussian_batch`` draws named in the file
and are stored beside the results (as hex floats), so a reader of the fixture
needs neither the generator nor this script.  Calls nothing but ``oracle/``
for the results."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import exact  # noqa: E402
from workloads import coupled_batch, gaussian_batch  # noqa: E402

CASES = [  # (R, T list, seed, weights)
    (1, [5, 9, 17], 901, (1.3, 0.8, 1.1)),
    (2, [5, 9, 17], 902, (1.3, 0.8, 1.1)),
]

GENERAL_CASES = [  # (R, V, Q, per-row weights, T list, seed)
    (1, 1, 1, True, [5, 9, 17], 911),
    (2, 1, 1, True, [5, 9, 17], 912),
    (1, 2, 2, False, [5, 9, 17], 913),
    (1, 2, 2, True, [5, 9, 17], 914),
    (1, 2, 1, False, [5, 9, 17], 915),
    # wide blocks (chunks of 4 at every level): 6 x 6 with three variables and
    # with two order-2 ones, 9 x 9 with per-row weights
    (1, 3, 3, False, [5, 9, 17], 916),
    (2, 2, 2, False, [5, 9, 17], 917),
    (2, 3, 3, True, [5, 9, 13], 918),
]


def _hex(a):
    return [float(x).hex() for x in np.asarray(a, dtype=np.float64).ravel()]


def main():
    out = {"source": "oracle/exact.py (rational arithmetic), rounded to double; loss gradient gy = N(0,1) draws",
           "cases": []}
    for R, Ts, seed, weights in CASES:
        bt = gaussian_batch(len(Ts), Ts, R=R, seed=seed, weights=weights)
        gy = np.random.default_rng(seed + 1).standard_normal(bt.c.shape)
        o = bt.offsets
        res = {k: [] for k in ("y", "lam", "dc", "dd", "ds", "du0", "dw")}
        for i in range(bt.n_inst):
            ex = exact.grad(R, *bt.instance_general(i), gy[o[i]:o[i + 1]])
            for key, src in (("y", "y"), ("lam", "lam"), ("dc", "dc"), ("dd", "dd"), ("ds", "ds"), ("du0", "du")):
                res[key] += _hex(exact.to_float(ex[src]))
            dw = [float(sum(ex["dwg"].ravel())), float(sum(ex["dwi"].ravel())), float(sum(ex["dws"].ravel()))]
            res["dw"] += _hex(dw)
        out["cases"].append({
            "R": R, "T": Ts, "n_init": bt.n_init, "seed": seed, "weights": list(weights),
            "inputs": {"c": _hex(bt.c), "b": _hex(bt.b), "h": _hex(bt.h), "u0": _hex(bt.u0), "w": _hex(bt.w),
                       "gy": _hex(gy)},
            "exact": res})
    with open(os.path.join(HERE, "exact_small.json"), "w") as f:
        json.dump(out, f, indent=0)
    print("wrote", os.path.join(HERE, "exact_small.json"))
    general()


def general():
    out = {"source": "oracle/exact.py (rational arithmetic), rounded to double; loss gradient gy = N(0,1) draws",
           "cases": []}
    for R, V, Q, per_row, Ts, seed in GENERAL_CASES:
        if V == 1:
            bt = gaussian_batch(len(Ts), Ts, R=R, seed=seed, weights=(1.3, 0.8, 1.1), per_row=per_row)
        else:
            bt = coupled_batch(len(Ts), Ts, R=R, V=V, Q=Q, seed=seed, weights=(1.3, 0.8, 1.1), per_row=per_row)
        gy = np.random.default_rng(seed + 1).standard_normal((bt.total_steps, bt.block))
        o = bt.offsets
        keys = ("y", "lam", "dc", "dd", "ds", "du", "dwg", "dwi", "dws")
        res = {k: [] for k in keys + ("dw",)}
        for i in range(bt.n_inst):
            ex = exact.grad(R, *bt.instance_general(i), gy[o[i]:o[i + 1]])
            for key in keys:
                res[key] += _hex(exact.to_float(ex[key]))
            # the scalar weights' gradients: exact sums of their rows'
            res["dw"] += _hex([float(sum(ex[key].ravel())) for key in ("dwg", "dwi", "dws")])
        inputs = {"c": _hex(bt.c), "b": _hex(bt.b), "h": _hex(bt.h), "u0": _hex(bt.u0), "w": _hex(bt.w),
                  "gy": _hex(gy)}
        if per_row:
            inputs.update({"wg": _hex(bt.wrow["wg"]), "wi": _hex(bt.wrow["wi"]), "ws": _hex(bt.wrow["ws"])})
        out["cases"].append({"R": R, "V": V, "Q": Q, "per_row": per_row, "T": Ts, "n_init": bt.n_init,
                             "seed": seed, "inputs": inputs, "exact": res})
    with open(os.path.join(HERE, "exact_general.json"), "w") as f:
        json.dump(out, f, indent=0)
    print("wrote", os.path.join(HERE, "exact_general.json"))


if __name__ == "__main__":
    main()
