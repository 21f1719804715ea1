"""Plain solver driver: owns the state and workspace tensors of one run and
calls the C ABI. dt defaults to 0.25 * min(h) (CFL 0.25 in coordinate units)."""
from __future__ import annotations

import torch

from . import _lib as C


class Solver:
    def __init__(self, n, L, params: C.cosmos_params | None = None, device: str = "cuda"):
        self.grid = C.make_grid(n, L)
        self.params = params if params is not None else C.make_params()
        self.device = torch.device(device)
        nx, ny, nz = self.grid.n
        self.shape = (C.NFIELDS, nz, ny, nx)
        self.u = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        self.ws = torch.empty(C.cosmos_workspace_bytes(self.grid), dtype=torch.uint8, device=self.device)
        self.norms = torch.empty(8, dtype=torch.float64, device=self.device)
        self.t = 0.0
        C.cosmos_status_reset(self.ws)

    @property
    def h(self):
        return tuple(self.grid.L[a] / self.grid.n[a] for a in range(3))

    def default_dt(self, cfl: float = 0.25) -> float:
        return cfl * min(self.h)

    def init(self, **kw):
        C.cosmos_init_fields(self.grid, self.params, C.make_init(**kw), self.u)
        self.t = 0.0
        return self.u

    def set_state(self, u: torch.Tensor, t: float = 0.0):
        self.u.copy_(u.to(self.device, torch.float64).reshape(self.shape))
        self.t = t

    def rhs(self, t: float | None = None, out: torch.Tensor | None = None) -> torch.Tensor:
        out = torch.empty_like(self.u) if out is None else out
        C.cosmos_rhs(self.grid, self.params, self.t if t is None else t, self.u, out, self.ws)
        return out

    def step(self, dt: float | None = None):
        dt = self.default_dt() if dt is None else dt
        C.cosmos_rk4_step(self.grid, self.params, self.t, dt, self.u, self.ws)
        self.t += dt

    def run(self, nsteps: int, dt: float | None = None):
        for _ in range(nsteps):
            self.step(dt)

    def constraints(self, want_fields: bool = False):
        H = M = None
        if want_fields:
            N = self.shape[1:]
            H = torch.empty(N, dtype=torch.float64, device=self.device)
            M = torch.empty((3,) + N, dtype=torch.float64, device=self.device)
        C.cosmos_constraints(self.grid, self.params, self.u, self.norms, H, M, self.ws)
        norms = self.norms.cpu()
        return (norms, H, M) if want_fields else norms

    def status(self):
        return C.cosmos_status(self.ws)
