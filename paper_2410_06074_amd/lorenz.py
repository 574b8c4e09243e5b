"""Lorenz equation discovery with the batched solve inside the training step.

This is the training step of Alg. 5 (App. C) run on the Lorenz experiment of
Sec. 5.1.  The encoder turns a batch into the coefficients c, constant terms
d, initial values u and step sizes s of every solve instance.  The solve
returns the trajectories y.  A decoder and a loss follow, and autograd carries
dl/dy back through the solver's adjoint pass (Eq. 14) to the encoder.

The encoder here is the Lorenz right-hand side with its seven coefficients
a1..a7 as the trainable parameters:
    x' = a1 x + a2 y,   y' = a3 x + a4 y + a5 x z,   z' = a6 z + a7 x y.
Every observed window of T samples gives three independent scalar instances
of order R (default 2), one per variable:
  * the variable's own linear term stays on the left, so the governing row
    over (y, y', y'', ...) is c_t = (-a_self, 1, 0, ...);
  * the cross terms, evaluated on the observed window, form d_t;
  * the initial value is the window's first sample, and s_t is the sampling
    step.
The decoder keeps the zeroth derivative, and the loss is the mean squared
error to the window.  Instances are laid out variable-major: all x windows,
then all y windows, then all z windows.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from .solver import solve


class LorenzDiscovery(torch.nn.Module):
    def __init__(self, order: int = 2, mode: str = "fp64r", dt: float = 0.01, weights=(1.0, 1.0, 1.0),
                 init=None):
        super().__init__()
        if order < 1:
            raise ValueError("the governing rows need the first derivative: order >= 1")
        self.order, self.mode, self.dt = order, mode, float(dt)
        self.weights = tuple(float(v) for v in weights)
        a0 = torch.zeros(7, dtype=torch.float64) if init is None else torch.as_tensor(init, dtype=torch.float64)
        self.a = torch.nn.Parameter(a0.clone())

    def encode(self, win: torch.Tensor):
        """(c, b, h, u0, w) of the 3B instances for windows win [B, T, 3]."""
        B, T, _ = win.shape
        k = self.order + 1
        dt_ = torch.float32 if self.mode == "fp32r" else torch.float64
        win = win.to(torch.float64)
        X, Y, Z = win[..., 0], win[..., 1], win[..., 2]
        a = self.a
        own = torch.stack([a[0], a[3], a[5]])                          # [3]
        forcing = torch.stack([a[1] * Y, a[2] * X + a[4] * X * Z, a[6] * X * Y])   # [3, B, T]
        c = torch.zeros(3, B, T, k, dtype=torch.float64, device=win.device)
        c[..., 0] = -own.view(3, 1, 1)
        c[..., 1] = 1.0
        h = torch.full((3 * B, T), self.dt, dtype=dt_, device=win.device)
        u0 = win[:, 0, :].t().reshape(3 * B, 1)
        w = torch.tensor(self.weights, dtype=dt_, device=win.device).expand(3 * B, 3).contiguous()
        return (c.reshape(3 * B, T, k).to(dt_), forcing.reshape(3 * B, T).to(dt_), h, u0.to(dt_), w)

    def forward(self, win: torch.Tensor) -> torch.Tensor:
        """Fitted trajectories [B, T, 3] (zeroth derivative of each instance)."""
        B, T, _ = win.shape
        c, b, h, u0, w = self.encode(win)
        y = solve(c, b, h, u0, w, order=self.order, n_init=1, mode=self.mode)   # [3B, T, k]
        return y[..., 0].reshape(3, B, T).permute(1, 2, 0).to(torch.float64)

    def loss(self, win: torch.Tensor) -> torch.Tensor:
        return torch.mean((self.forward(win) - win.to(torch.float64)) ** 2)


def train(model: LorenzDiscovery, traj: np.ndarray, steps: int, batch: int = 512, T: int = 50,
          lr: float = 0.5, decay_at: float = 0.7, seed: int = 0, device="cuda", log_every: int = 0):
    """Adam on a1..a7 over random windows of traj; the learning rate drops 10x
    after decay_at of the steps.  Returns the per-step losses."""
    from workloads.lorenz import windows
    rng = np.random.default_rng(seed)
    opt = torch.optim.Adam(model.parameters(), lr=lr)
    sched = torch.optim.lr_scheduler.MultiStepLR(opt, milestones=[max(1, int(decay_at * steps))], gamma=0.1)
    losses = []
    for it in range(steps):
        win = torch.as_tensor(windows(traj, batch, T, rng), device=device)
        opt.zero_grad(set_to_none=True)
        loss = model.loss(win)
        loss.backward()
        opt.step()
        sched.step()
        losses.append(float(loss.detach()))
        if log_every and (it + 1) % log_every == 0:
            print("step %d loss %.3e a %s" % (it + 1, losses[-1], np.round(model.a.detach().cpu().numpy(), 4)),
                  flush=True)
    return losses


def step_time(batch: int, T: int, iters: int = 50, warmup: int = 5, mode: str = "fp64r", device="cuda"):
    """Mean ms of one optimisation step (window upload, forward, loss,
    backward, Adam) at the given batch size and window length."""
    from workloads.lorenz import lorenz_trajectory, windows
    traj = lorenz_trajectory(max(10000, 4 * T))
    rng = np.random.default_rng(1)
    model = LorenzDiscovery(mode=mode).to(device)
    opt = torch.optim.Adam(model.parameters(), lr=1e-2)
    wins = [torch.as_tensor(windows(traj, batch, T, rng)) for _ in range(8)]

    def one(i):
        win = wins[i % len(wins)].to(device, non_blocking=False)
        opt.zero_grad(set_to_none=True)
        model.loss(win).backward()
        opt.step()

    for i in range(warmup):
        one(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(iters):
        one(i)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / iters
