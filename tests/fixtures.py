"""Loaders of the stored expected values under tests/golden/."""
import json
import os

import numpy as np

from workloads import Batch

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _arr(hexes):
    return np.array([float.fromhex(x) for x in hexes], dtype=np.float64)


def load_exact(case):
    """(batch, gy, want) of case `case` of exact_small.json: want holds y, lam,
    dc, dd, ds [per point], du0, dw [per instance] as the rational oracle's
    values rounded to double."""
    with open(os.path.join(GOLDEN, "exact_small.json")) as f:
        data = json.load(f)["cases"][case]
    R, Ts, n_init = data["R"], np.asarray(data["T"], dtype=np.int64), data["n_init"]
    k, N, S = R + 1, len(Ts), int(np.sum(Ts))
    inp = {key: _arr(v) for key, v in data["inputs"].items()}
    bt = Batch(R=R, n_init=n_init, T=Ts, c=inp["c"].reshape(S, k), b=inp["b"], h=inp["h"],
               u0=inp["u0"].reshape(N, n_init), w=inp["w"].reshape(N, 3), name="exact_small[%d]" % case)
    ex = {key: _arr(v) for key, v in data["exact"].items()}
    want = {"y": ex["y"].reshape(S, k), "lam": ex["lam"].reshape(S, k), "dc": ex["dc"].reshape(S, k),
            "dd": ex["dd"], "ds": ex["ds"], "du0": ex["du0"].reshape(N, n_init), "dw": ex["dw"].reshape(N, 3)}
    return bt, inp["gy"].reshape(S, k), want


def n_exact_cases():
    with open(os.path.join(GOLDEN, "exact_small.json")) as f:
        return len(json.load(f)["cases"])
