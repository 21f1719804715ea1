"""Plain solver driver: owns the state and workspace tensors of one run and
calls the C ABI. dt defaults to 0.25 * min(h) (CFL 0.25 in coordinate units)."""
from __future__ import annotations

import torch

from . import _lib as C


class Solver:
    """With scalar=True the run also carries the massless scalar field: ``s`` holds
    (phi, Pi), and init / rhs / step / constraints go through the scalar entry points
    (rhs then returns (dudt, dsdt))."""

    def __init__(self, n, L, params: C.cosmos_params | None = None, device: str = "cuda", scalar: bool = False):
        self.grid = C.make_grid(n, L)
        self.params = params if params is not None else C.make_params()
        self.device = torch.device(device)
        nx, ny, nz = self.grid.n
        self.shape = (C.NFIELDS, nz, ny, nx)
        self.u = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        self.ws = torch.empty(C.cosmos_workspace_bytes(self.grid), dtype=torch.uint8, device=self.device)
        self.norms = torch.empty(8, dtype=torch.float64, device=self.device)
        self.t = 0.0
        self.scalar = scalar
        if scalar:
            self.s = torch.zeros((2, nz, ny, nx), dtype=torch.float64, device=self.device)
            self.sws = torch.empty(C.cosmos_scalar_workspace_bytes(self.grid), dtype=torch.uint8, device=self.device)
        C.cosmos_status_reset(self.ws)

    @property
    def h(self):
        return tuple(self.grid.L[a] / self.grid.n[a] for a in range(3))

    def default_dt(self, cfl: float = 0.25) -> float:
        return cfl * min(self.h)

    def init(self, sc_mu: float = 0.0, sc_sigma: float = 1.0, **kw):
        """Initial data; with the scalar field, sc_mu and sc_sigma give its iso-curvature mode."""
        if self.scalar:
            C.cosmos_init_fields_scalar(self.grid, self.params, C.make_init(**kw), sc_mu, sc_sigma, self.u, self.s)
        else:
            C.cosmos_init_fields(self.grid, self.params, C.make_init(**kw), self.u)
        self.t = 0.0
        return self.u

    def set_state(self, u: torch.Tensor, t: float = 0.0, s: torch.Tensor | None = None):
        self.u.copy_(u.to(self.device, torch.float64).reshape(self.shape))
        if s is not None:
            self.s.copy_(s.to(self.device, torch.float64).reshape(self.s.shape))
        self.t = t

    def rhs(self, t: float | None = None, out: torch.Tensor | None = None):
        out = torch.empty_like(self.u) if out is None else out
        t = self.t if t is None else t
        if self.scalar:
            ds = torch.empty_like(self.s)
            C.cosmos_rhs_scalar(self.grid, self.params, t, self.u, self.s, out, ds, self.ws, self.sws)
            return out, ds
        C.cosmos_rhs(self.grid, self.params, t, self.u, out, self.ws)
        return out

    def step(self, dt: float | None = None):
        dt = self.default_dt() if dt is None else dt
        if self.scalar:
            C.cosmos_rk4_step_scalar(self.grid, self.params, self.t, dt, self.u, self.s, self.ws, self.sws)
        else:
            C.cosmos_rk4_step(self.grid, self.params, self.t, dt, self.u, self.ws)
        self.t += dt

    def run(self, nsteps: int, dt: float | None = None):
        """nsteps steps in one library call (cosmos_rk4_steps, cosmos_rk4_steps_scalar: the same
        state bitwise as nsteps calls of step, the fluid fluxes carried from step to step)."""
        dt = self.default_dt() if dt is None else dt
        if self.scalar:
            C.cosmos_rk4_steps_scalar(self.grid, self.params, self.t, dt, nsteps, self.u, self.s, self.ws, self.sws)
        else:
            C.cosmos_rk4_steps(self.grid, self.params, self.t, dt, nsteps, self.u, self.ws)
        for _ in range(nsteps):
            self.t += dt

    def constraints(self, want_fields: bool = False):
        H = M = None
        if want_fields:
            N = self.shape[1:]
            H = torch.empty(N, dtype=torch.float64, device=self.device)
            M = torch.empty((3,) + N, dtype=torch.float64, device=self.device)
        if self.scalar:
            C.cosmos_constraints_scalar(self.grid, self.params, self.u, self.s, self.norms, H, M, self.ws, self.sws)
        else:
            C.cosmos_constraints(self.grid, self.params, self.u, self.norms, H, M, self.ws)
        norms = self.norms.cpu()
        return (norms, H, M) if want_fields else norms

    def status(self):
        return C.cosmos_status(self.ws)
