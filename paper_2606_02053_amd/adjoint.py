"""Differentiable run: d J / d(mu, sigma) by the hand-written discrete adjoint.

J is the lapse at the box centre after `nsteps` RK4 steps from the initial
data of a Gaussian curvature perturbation (amplitude mu, width sigma). The
backward pass applies the adjoint step backwards through every step, starting
from lambda = dJ/du(T) (a unit vector on the centre lapse), and finally
contracts lambda_0 with the derivatives of the initial data in mu and sigma on
the device (cosmos_adjoint_gradient). Each adjoint step needs the step's start
state and its RK4 stage states (cosmos_adjoint_step_stages); where they come
from is a memory trade:

* `keep_all`: the forward pass keeps every step's start state and stage states
  (one cosmos_rk4_steps_stages call; 4 states per step), so the backward pass
  evaluates no forward stage at all. At 96^3 and 200 steps that is 142 GB of
  device memory.
* otherwise the forward pass stores the state every `checkpoint_every` steps and
  the backward pass recomputes each segment from its checkpoint; where memory
  allows (`keep_stages`) the recomputation keeps the segment's stage states,
  else the adjoint step evaluates them itself (cosmos_adjoint_step).

All three give the same gradient bitwise. Step m starts at the time t_m reached by
adding dt m times (as a multi-step library call advances it), on every path.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import _lib as C
from .solver import Solver


@dataclass
class RunConfig:
    n: int = 96
    L: float = 12.0
    nsteps: int = 200
    checkpoint_every: int = 20
    cfl: float = 0.25
    params: C.cosmos_params = field(default_factory=C.make_params)
    init_kw: dict = field(default_factory=dict)  # extra cosmos_init fields (profile, center, ...)
    # keep every step's start and stage states from the forward pass: True / False, or None to
    # decide by the free device memory (kept when they take under 60 % of it)
    keep_all: bool | None = None
    # with checkpoints: keep the stage states of a segment (3 states per step) for the reverse
    # sweep: True / False, or None to decide by the free device memory
    keep_stages: bool | None = None

    @property
    def dt(self) -> float:
        return self.cfl * self.L / self.n


def _free_bytes(dev) -> int:
    return torch.cuda.mem_get_info(dev)[0]


def _step_times(nsteps: int, dt: float) -> list[float]:
    """t_0 = 0 and t_{m+1} = t_m + dt: the start time of every step."""
    ts, t = [], 0.0
    for _ in range(nsteps):
        ts.append(t)
        t += dt
    return ts


class CosmosRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mu: torch.Tensor, sigma: torch.Tensor, cfg: RunConfig):
        s = Solver(cfg.n, cfg.L, cfg.params)
        s.init(mu=float(mu), sigma=float(sigma), **cfg.init_kw)
        dt = cfg.dt
        numel = s.u.numel()
        wanted = any(ctx.needs_input_grad[:2])
        keep_all = cfg.keep_all
        if keep_all is None:
            keep_all = wanted and 4 * cfg.nsteps * numel * 8 < 0.6 * _free_bytes(s.u.device)
        ckpts, traj = {}, None
        ts = _step_times(cfg.nsteps, dt)
        if wanted and keep_all:
            states = torch.empty((cfg.nsteps, numel), dtype=torch.float64, device=s.u.device)
            stages = torch.empty((cfg.nsteps, 3 * numel), dtype=torch.float64, device=s.u.device)
            C.cosmos_rk4_steps_stages(s.grid, s.params, 0.0, dt, cfg.nsteps, s.u, states, stages, s.ws)
            traj = (states, stages)
        else:
            for m in range(cfg.nsteps):
                if wanted and m % cfg.checkpoint_every == 0:
                    ckpts[m] = s.u.clone()
                C.cosmos_rk4_step(s.grid, s.params, ts[m], dt, s.u, s.ws)
        c = cfg.n // 2
        J = s.u[17, c, c, c].clone()
        ctx.cfg = cfg
        ctx.ckpts = ckpts
        ctx.traj = traj
        ctx.mu, ctx.sigma = float(mu), float(sigma)
        return J

    @staticmethod
    def backward(ctx, gJ: torch.Tensor):
        cfg: RunConfig = ctx.cfg
        grid, params, dt = C.make_grid(cfg.n, cfg.L), cfg.params, cfg.dt
        dev = gJ.device if gJ.is_cuda else torch.device("cuda")
        shape = (C.NFIELDS, cfg.n, cfg.n, cfg.n)
        lam = torch.zeros(shape, dtype=torch.float64, device=dev)
        c = cfg.n // 2
        lam[17, c, c, c] = gJ.to(dev, torch.float64)
        lam_next = torch.empty_like(lam)
        ws_adj = torch.empty(C.cosmos_adjoint_workspace_bytes(grid), dtype=torch.uint8, device=dev)
        ts = _step_times(cfg.nsteps, dt)
        if ctx.traj is not None:
            states, stages = ctx.traj
            for m in range(cfg.nsteps - 1, -1, -1):
                C.cosmos_adjoint_step_stages(grid, params, ts[m], dt, states[m], stages[m], lam, lam_next, ws_adj)
                lam, lam_next = lam_next, lam
            ctx.traj = None
        else:
            ws_fwd = torch.empty(C.cosmos_workspace_bytes(grid), dtype=torch.uint8, device=dev)
            seg = cfg.checkpoint_every
            keep = cfg.keep_stages
            if keep is None:
                keep = 3 * seg * lam.numel() * 8 < 0.5 * _free_bytes(dev)
            stages = torch.empty((seg, 3 * lam.numel()), dtype=torch.float64, device=dev) if keep else None
            for start in sorted(ctx.ckpts, reverse=True):
                end = min(start + seg, cfg.nsteps)
                states = [ctx.ckpts[start]]
                u = ctx.ckpts[start].clone()
                for m in range(start, end):  # recompute the segment's states (and stage states)
                    if keep:
                        C.cosmos_rk4_step_stages(grid, params, ts[m], dt, u, stages[m - start], ws_fwd)
                    elif m < end - 1:
                        C.cosmos_rk4_step(grid, params, ts[m], dt, u, ws_fwd)
                    if m < end - 1:
                        states.append(u.clone())
                for m in range(end - 1, start - 1, -1):
                    if keep:
                        C.cosmos_adjoint_step_stages(grid, params, ts[m], dt, states[m - start], stages[m - start],
                                                     lam, lam_next, ws_adj)
                    else:
                        C.cosmos_adjoint_step(grid, params, ts[m], dt, states[m - start], lam, lam_next, ws_adj)
                    lam, lam_next = lam_next, lam
        init = C.make_init(mu=ctx.mu, sigma=ctx.sigma, **cfg.init_kw)
        grad = torch.empty(2, dtype=torch.float64, device=dev)
        C.cosmos_adjoint_gradient(grid, params, init, lam, grad, ws_adj)
        grad = grad.to(gJ.device)
        return grad[0], grad[1], None


def central_lapse(mu, sigma, cfg: RunConfig):
    """J(mu, sigma) with gradients through the discrete adjoint."""
    return CosmosRun.apply(mu, sigma, cfg)
