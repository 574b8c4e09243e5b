"""Table 5 problems (App. B.1): coefficients, closed forms and the printed values.

Helper for the oracle pins; builds inputs only (no part of the solve)."""
import json
import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table5_smnn.json")


def load():
    with open(GOLDEN) as f:
        return json.load(f)


def problem(name, R=2):
    """(c [T,R+1], d [T], s [T], u0 [1], w [3], exact list of callables y^(r)(t), printed)."""
    g = load()
    T, h = g["steps"], g["step_size"]
    p = g["problems"][name]
    k = R + 1
    coef = np.zeros(k)
    if name == "rc":
        c0, c1, c2, u = p["c0"], p["c1"], p["c2"], p["u0"]
        coef[0], coef[1], d = 1.0 / c1, c2, c0
        tau = c1 * c2
        A = u - c0 * c1
        exact = [lambda t: c0 * c1 + A * np.exp(-t / tau),
                 lambda t: -A / tau * np.exp(-t / tau),
                 lambda t: A / tau ** 2 * np.exp(-t / tau)]
    elif name == "population":
        a, u = p["c0"], p["u0"]
        coef[0], coef[1], d = a, -1.0, 0.0
        exact = [lambda t: u * np.exp(a * t), lambda t: u * a * np.exp(a * t),
                 lambda t: u * a * a * np.exp(a * t)]
    elif name == "language":
        a, b, u = p["c0"], p["c1"], p["u0"]
        coef[0], coef[1], d = a + b, 1.0, a
        q = a / (a + b)
        exact = [lambda t: q - (q - u) * np.exp(-(a + b) * t),
                 lambda t: (q - u) * (a + b) * np.exp(-(a + b) * t),
                 lambda t: -(q - u) * (a + b) ** 2 * np.exp(-(a + b) * t)]
    else:
        raise KeyError(name)
    c = np.tile(coef, (T, 1))
    return (c, np.full(T, d), np.full(T, h), np.array([p["u0"]]), np.ones(3), exact,
            p["table5_rel_mse"], np.arange(T) * h)


def rel_mse(y, exact, tk):
    out = []
    for r, f in enumerate(exact):
        ex = f(tk)
        out.append(float(np.mean((y[:, r] - ex) ** 2) / np.var(ex)))
    return out


def matches_printed(value, printed):
    """True if value rounds to the printed two significant digits."""
    return float("%.1e" % value) == printed
