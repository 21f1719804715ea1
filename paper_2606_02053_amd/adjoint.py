"""Differentiable run: d J / d(mu, sigma) by the hand-written discrete adjoint.

J is the lapse at the box centre after `nsteps` RK4 steps from the initial
data of a Gaussian curvature perturbation (amplitude mu, width sigma). The
forward pass stores the state every `checkpoint_every` steps; the backward
pass recomputes each segment from its checkpoint and applies the adjoint step
(cosmos_adjoint_step) backwards through it, starting from lambda = dJ/du(T)
(a unit vector on the centre lapse), and finally contracts lambda_0 with the
derivatives of the initial data in mu and sigma (cosmos_init_tangent).
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

    @property
    def dt(self) -> float:
        return self.cfl * self.L / self.n


class CosmosRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mu: torch.Tensor, sigma: torch.Tensor, cfg: RunConfig):
        s = Solver(cfg.n, cfg.L, cfg.params)
        s.init(mu=float(mu), sigma=float(sigma), **cfg.init_kw)
        dt = cfg.dt
        ckpts = {}
        for m in range(cfg.nsteps):
            if m % cfg.checkpoint_every == 0:
                ckpts[m] = s.u.clone()
            C.cosmos_rk4_step(s.grid, s.params, m * dt, dt, s.u, s.ws)
        c = cfg.n // 2
        J = s.u[17, c, c, c].clone()
        ctx.cfg = cfg
        ctx.ckpts = ckpts
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
        ws_fwd = torch.empty(C.cosmos_workspace_bytes(grid), dtype=torch.uint8, device=dev)
        for start in sorted(ctx.ckpts, reverse=True):
            end = min(start + cfg.checkpoint_every, cfg.nsteps)
            states = [ctx.ckpts[start]]
            u = ctx.ckpts[start].clone()
            for m in range(start, end - 1):  # recompute the segment's states
                C.cosmos_rk4_step(grid, params, m * dt, dt, u, ws_fwd)
                states.append(u.clone())
            for m in range(end - 1, start - 1, -1):
                C.cosmos_adjoint_step(grid, params, m * dt, dt, states[m - start], lam, lam_next, ws_adj)
                lam, lam_next = lam_next, lam
        init = C.make_init(mu=ctx.mu, sigma=ctx.sigma, **cfg.init_kw)
        du = torch.empty_like(lam)
        grads = []
        for which in (0, 1):
            C.cosmos_init_tangent(grid, params, init, which, du)
            grads.append(torch.dot(lam.reshape(-1), du.reshape(-1)).to(gJ.device))
        return grads[0], grads[1], None


def central_lapse(mu, sigma, cfg: RunConfig):
    """J(mu, sigma) with gradients through the discrete adjoint."""
    return CosmosRun.apply(mu, sigma, cfg)
