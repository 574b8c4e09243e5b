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


def load_exact_general(case):
    """(batch, gy, want) of case `case` of exact_general.json (per-row weights
    and coupled variables): want holds y, lam [S, K], dc, dd, ds, du0 and the
    per-row weight gradients dwg, dwi, dws in the batch's shapes, or dw [N, 3]
    (the three scalar-weight sums) for scalar weights."""
    with open(os.path.join(GOLDEN, "exact_general.json")) as f:
        data = json.load(f)["cases"][case]
    R, V, Q, Ts, n_init = data["R"], data["V"], data["Q"], np.asarray(data["T"], dtype=np.int64), data["n_init"]
    K, N, S = V * (R + 1), len(Ts), int(np.sum(Ts))
    inp = {key: _arr(v) for key, v in data["inputs"].items()}
    ni = V * n_init
    wrow = None
    if data["per_row"]:
        wrow = {"wg": inp["wg"].reshape(S, Q), "wi": inp["wi"].reshape(N, ni), "ws": inp["ws"]}
    bt = Batch(R=R, n_init=n_init, T=Ts, c=inp["c"].reshape(S, Q * K) if (V > 1 or Q > 1) else inp["c"].reshape(S, K),
               b=inp["b"].reshape(S, Q) if Q > 1 else inp["b"], h=inp["h"], u0=inp["u0"].reshape(N, ni),
               w=inp["w"].reshape(N, 3), name="exact_general[%d]" % case, V=V, Q=Q, wrow=wrow)
    ex = {key: _arr(v) for key, v in data["exact"].items()}
    want = {"y": ex["y"].reshape(S, K), "lam": ex["lam"].reshape(S, K), "dc": ex["dc"].reshape(np.shape(bt.c)),
            "dd": ex["dd"].reshape(np.shape(bt.b)), "ds": ex["ds"], "du0": ex["du"].reshape(N, ni)}
    dwg, dwi, dws = ex["dwg"].reshape(S, Q), ex["dwi"].reshape(N, ni), ex["dws"]
    if wrow is not None:
        want.update({"dwg": dwg, "dwi": dwi, "dws": dws})
    else:
        want["dw"] = ex["dw"].reshape(N, 3)
    return bt, inp["gy"].reshape(S, K), want


def n_exact_general_cases():
    with open(os.path.join(GOLDEN, "exact_general.json")) as f:
        return len(json.load(f)["cases"])
