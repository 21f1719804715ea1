"""Fixed mesh refinement driver: Berger-Oliger sub-cycling over nested layers (paper: nested
refinement layers, "Statement of need" and the adiabatic-fluctuation example).

Sequencing only: every value is computed by the library (cosmos_rk4_step,
cosmos_rk4_step_stages_to, cosmos_fmr_prolong, cosmos_fmr_restrict); PyTorch holds the device arrays. The scheme is the one
stated with those entry points in include/cosmos.h:

  step of layer l (dt):   RK4 step of u_l keeping its stage states, out of place (u_n stays as u0);
                          for each half h = 0, 1: refill layer l + 1's buffer from layer l at
                          theta = h / 2 (u0 alone for h = 0, the step's continuous extension from
                          its stage states for h = 1), then step layer l + 1 by dt / 2
                          (recursively); copy layer l + 1's interior onto u_l (injection).
"""
from __future__ import annotations

import torch

from . import _lib as C


class RefinedRun:
    """Layer 0 is the periodic grid (n, L); layer k + 1 refines `boxes[k]` (origin, m) of layer k,
    given in layer k's array indices. For k >= 1 the box, its buffer (COSMOS_FMR_BUFFER / 2
    parent points) and the interpolation stencil (3 more) must lie at least COSMOS_FMR_BUFFER
    points inside layer k's faces, where layer k's values are valid throughout its step."""

    def __init__(self, n, L, boxes, params: C.cosmos_params | None = None, device: str = "cuda"):
        self.params = params if params is not None else C.make_params()
        self.device = torch.device(device)
        self.grids = [C.make_grid(n, L)]
        self.boxes = [C.make_box(o, m) for o, m in boxes]
        W = C.COSMOS_FMR_BUFFER
        for k, b in enumerate(self.boxes):
            if k >= 1:
                g = self.grids[k]
                for a in range(3):
                    lo, hi = b.origin[a] - W // 2 - 2, b.origin[a] + b.m[a] + W // 2 + 3
                    if lo < W or hi > g.n[a] - W:
                        raise ValueError(f"box {k} reaches into layer {k}'s buffer along axis {a}")
            self.grids.append(C.cosmos_fmr_child_grid(self.grids[k], b))
        f64 = dict(dtype=torch.float64, device=self.device)
        self.u = [torch.empty((C.NFIELDS, g.n[2], g.n[1], g.n[0]), **f64) for g in self.grids]
        self.ws = [torch.empty(C.cosmos_workspace_bytes(g), dtype=torch.uint8, device=self.device)
                   for g in self.grids]
        # per refined parent: a second state array (the step runs out of place, so the two alternate:
        # after a step one holds u_n for the child's interpolation in time, the other u_{n+1}), the
        # step's stage states, the prolongation workspace
        self.u0 = [torch.empty_like(self.u[k]) for k in range(len(self.boxes))]
        self.stages = [torch.empty((3,) + tuple(self.u[k].shape), **f64) for k in range(len(self.boxes))]
        self.pws = [torch.empty(C.cosmos_fmr_workspace_bytes(self.grids[k], b), dtype=torch.uint8,
                                device=self.device) for k, b in enumerate(self.boxes)]
        for w in self.ws:
            C.cosmos_status_reset(w)
        self.t = 0.0

    @property
    def h(self):
        g = self.grids[0]
        return tuple(g.L[a] / g.n[a] for a in range(3))

    def default_dt(self, cfl: float = 0.25) -> float:
        """Layer 0's step; layer k steps dt / 2^k with the same Courant number."""
        return cfl * min(self.h)

    def init(self, **kw):
        """Layer 0's initial data (cosmos_init_fields); finer layers interpolated from their parents."""
        C.cosmos_init_fields(self.grids[0], self.params, C.make_init(**kw), self.u[0])
        for k, b in enumerate(self.boxes):
            C.cosmos_fmr_prolong(self.grids[k], b, self.u[k], None, None, 0.0, False, self.u[k + 1], self.pws[k])
        self.t = 0.0

    def _step(self, k: int, t: float, dt: float):
        g, u = self.grids[k], self.u[k]
        if k == len(self.boxes):
            C.cosmos_rk4_step(g, self.params, t, dt, u, self.ws[k])
            return
        b = self.boxes[k]
        C.cosmos_rk4_step_stages_to(g, self.params, t, dt, u, self.u0[k], self.stages[k], self.ws[k])
        self.u[k], self.u0[k] = self.u0[k], u  # u_{n+1} is the layer's state now; u_n stays beside it
        u = self.u[k]
        for half in (0, 1):
            C.cosmos_fmr_prolong(g, b, self.u0[k], self.stages[k], u, 0.5 * half, True, self.u[k + 1], self.pws[k])
            self._step(k + 1, t + 0.5 * half * dt, 0.5 * dt)
        C.cosmos_fmr_restrict(g, b, self.u[k + 1], u)

    def step(self, dt: float | None = None):
        dt = self.default_dt() if dt is None else dt
        self._step(0, self.t, dt)
        self.t += dt

    def run(self, nsteps: int, dt: float | None = None):
        for _ in range(nsteps):
            self.step(dt)

    def interior(self, k: int) -> torch.Tensor:
        """Layer k's interior points (a view of its padded array; the whole grid for k = 0). A refined
        parent's state alternates between two arrays from step to step: take the view after stepping."""
        if k == 0:
            return self.u[0]
        W = C.COSMOS_FMR_BUFFER
        return self.u[k][:, W:-W, W:-W, W:-W]

    def status(self, k: int = 0) -> dict:
        """Layer k's counters (cosmos_status of its workspace)."""
        return C.cosmos_status(self.ws[k])
