"""The Lorenz data generator (workloads.lorenz), checked on the CPU."""
import numpy as np
from scipy.integrate import solve_ivp

from workloads.lorenz import TRUE_COEFFS, lorenz_field, lorenz_trajectory, windows


def test_trajectory_matches_an_independent_integrator():
    n, dt = 300, 0.01
    traj = lorenz_trajectory(n, dt)
    ref = solve_ivp(lambda t, u: lorenz_field(u), (0.0, (n - 1) * dt), [1.0, 1.0, 1.0], method="DOP853",
                    t_eval=np.arange(n) * dt, rtol=1e-12, atol=1e-12).y.T
    assert np.abs(traj - ref).max() < 1e-7 * np.abs(ref).max()


def test_coefficients_give_the_lorenz_field():
    a1, a2, a3, a4, a5, a6, a7 = TRUE_COEFFS
    u = np.random.default_rng(0).standard_normal((50, 3)) * 10
    x, y, z = u.T
    lin = np.stack([a1 * x + a2 * y, a3 * x + a4 * y + a5 * x * z, a6 * z + a7 * x * y], axis=-1)
    assert np.allclose(lin, lorenz_field(u), rtol=1e-14, atol=1e-12)


def test_windows_are_consecutive_samples():
    traj = lorenz_trajectory(500)
    w = windows(traj, 16, 50, np.random.default_rng(1))
    assert w.shape == (16, 50, 3)
    for win in w:
        s = int(np.flatnonzero((traj == win[0]).all(axis=1))[0])
        assert np.array_equal(traj[s:s + 50], win)


def test_oracle_chain_rule_matches_finite_differences():
    # the oracle-side loss gradient the Lorenz GPU test compares against
    from tests.test_gpu_lorenz import oracle_loss_and_grad
    rng = np.random.default_rng(2)
    win = windows(lorenz_trajectory(1000), 4, 20, rng)
    a = np.asarray(TRUE_COEFFS) * (1.0 + 0.2 * rng.standard_normal(7))
    _, ga = oracle_loss_and_grad(a, win, 0.01)
    for j in range(7):
        e = np.zeros(7)
        e[j] = 1e-6 * max(1.0, abs(a[j]))
        fd = (oracle_loss_and_grad(a + e, win, 0.01)[0] - oracle_loss_and_grad(a - e, win, 0.01)[0]) / (2 * e[j])
        assert abs(fd - ga[j]) <= 1e-5 * max(1.0, np.abs(ga).max()), j
