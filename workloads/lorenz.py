"""Observed data for the Lorenz discovery experiment (Sec. 5.1, App. D).

One long trajectory of the Lorenz system from x = y = z = 1 with sigma = 10,
rho = 28, beta = 8/3, sampled every 0.01 (10,000 samples by default), and
batches of random windows of it.  The paper integrates with SciPy's odeint;
this module uses the classical fourth-order Runge-Kutta method with several
sub-steps per sample.  It integrates the data only: none of the solve's
arithmetic is here, so the oracle-side tests and the GPU path share it.
"""
from __future__ import annotations

import numpy as np

SIGMA, RHO, BETA = 10.0, 28.0, 8.0 / 3.0
# a1..a7 of x' = a1 x + a2 y, y' = a3 x + a4 y + a5 x z, z' = a6 z + a7 x y
TRUE_COEFFS = (-SIGMA, SIGMA, RHO, -1.0, -1.0, -BETA, 1.0)


def lorenz_field(u: np.ndarray) -> np.ndarray:
    x, y, z = u[..., 0], u[..., 1], u[..., 2]
    return np.stack([SIGMA * (y - x), x * (RHO - z) - y, x * y - BETA * z], axis=-1)


def lorenz_trajectory(n_samples: int = 10000, dt: float = 0.01, substeps: int = 10,
                      x0=(1.0, 1.0, 1.0)) -> np.ndarray:
    """[n_samples, 3] float64: sample i is the state at time i * dt."""
    u = np.asarray(x0, dtype=np.float64).copy()
    out = np.empty((n_samples, 3))
    h = dt / substeps
    for i in range(n_samples):
        out[i] = u
        for _ in range(substeps):
            k1 = lorenz_field(u)
            k2 = lorenz_field(u + 0.5 * h * k1)
            k3 = lorenz_field(u + 0.5 * h * k2)
            k4 = lorenz_field(u + h * k3)
            u = u + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    return out


def windows(traj: np.ndarray, batch: int, T: int, rng: np.random.Generator) -> np.ndarray:
    """[batch, T, 3]: windows of T consecutive samples at uniform random starts."""
    starts = rng.integers(0, traj.shape[0] - T + 1, size=batch)
    return np.stack([traj[s:s + T] for s in starts])
