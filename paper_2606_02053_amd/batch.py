"""Batched threshold scan: many runs of different perturbation amplitude mu,
width sigma and grid size advanced together, one launch per RK4 stage for the
whole batch, with the RK4 step captured once in a hipGraph and replayed.

Each run r: cubic periodic grid n_r^3 in a box of side L, Gaussian curvature
perturbation (mu_r, sigma_r), dt_r = cfl * L / n_r, its own time t_r. The
outcome per run is the lapse at the box centre and its minimum over the grid
(a collapsing region drives the lapse down).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as C


@dataclass
class RunSpec:
    n: int
    mu: float
    sigma: float
    L: float = 12.0
    sc_mu: float = 0.0     # iso-curvature mode of the scalar field (Batch(..., scalar=True))
    sc_sigma: float = 1.0


def draw_scan(nruns: int = 64, seed: int = 2606, sizes=(48, 64, 80, 96), mu=(0.3, 0.8), sigma=(0.8, 1.6),
              L: float = 12.0):
    """Seeded draws of (n, mu, sigma) per run, in run order."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(nruns):
        n = int(rng.choice(sizes))
        out.append(RunSpec(n=n, mu=float(rng.uniform(*mu)), sigma=float(rng.uniform(*sigma)), L=L))
    return out


class Batch:
    """With scalar=True every run also carries the massless scalar field (RunSpec.sc_mu,
    sc_sigma give its iso-curvature initial data); ``scalar_state(r)`` is run r's (phi, Pi)."""

    def __init__(self, runs, params: C.cosmos_params | None = None, cfl: float = 0.25, device="cuda",
                 scalar: bool = False):
        self.runs = list(runs)
        self.params = params if params is not None else C.make_params()
        self.device = torch.device(device)
        offs, o = [], 0
        for r in self.runs:
            offs.append(o)
            o += ((C.NFIELDS * r.n ** 3 + 31) // 32) * 32
        self.offsets = offs
        self.batch = C.make_batch([r.n for r in self.runs], [r.L for r in self.runs], offs)
        self.arena = torch.zeros(o, dtype=torch.float64, device=self.device)
        self.bws = torch.empty(C.cosmos_batch_workspace_bytes(self.batch), dtype=torch.uint8, device=self.device)
        self.t = torch.zeros(len(self.runs), dtype=torch.float64, device=self.device)
        self.dt = torch.tensor([cfl * r.L / r.n for r in self.runs], dtype=torch.float64, device=self.device)
        self.graph = None
        self.graph_steps = 1
        self.scalar = scalar
        if scalar:  # laid out like the state arena: run r's (phi, Pi) at its state offset
            self.sarena = torch.zeros(o, dtype=torch.float64, device=self.device)
            self.sbws = torch.empty(C.cosmos_batch_scalar_workspace_bytes(self.batch), dtype=torch.uint8,
                                    device=self.device)

    def state(self, r: int) -> torch.Tensor:
        n = self.runs[r].n
        return self.arena[self.offsets[r]:self.offsets[r] + C.NFIELDS * n ** 3].view(C.NFIELDS, n, n, n)

    def scalar_state(self, r: int) -> torch.Tensor:
        n = self.runs[r].n
        return self.sarena[self.offsets[r]:self.offsets[r] + 2 * n ** 3].view(2, n, n, n)

    def init(self):
        for r, spec in enumerate(self.runs):
            g = C.make_grid(spec.n, spec.L)
            ini = C.make_init(mu=spec.mu, sigma=spec.sigma)
            if self.scalar:
                C.cosmos_init_fields_scalar(g, self.params, ini, spec.sc_mu, spec.sc_sigma, self.state(r),
                                            self.scalar_state(r))
            else:
                C.cosmos_init_fields(g, self.params, ini, self.state(r))
        self.t.zero_()
        C.cosmos_batch_setup(self.batch, self.params, self.bws)

    def _step(self, stream=None, nsteps: int = 1):
        if self.scalar:
            for _ in range(nsteps):
                C.cosmos_rk4_step_batched_scalar(self.batch, self.params, self.arena, self.sarena, self.t, self.dt,
                                                 self.bws, self.sbws, stream=stream)
        elif nsteps == 1:
            C.cosmos_rk4_step_batched(self.batch, self.params, self.arena, self.t, self.dt, self.bws, stream=stream)
        else:  # one call: the fluid fluxes carried from step to step
            C.cosmos_rk4_steps_batched(self.batch, self.params, self.arena, self.t, self.dt, nsteps, self.bws,
                                       stream=stream)

    def step(self):
        self._step()

    def capture(self, steps: int = 1):
        """Capture `steps` batched RK4 steps in a graph (after init); run() replays it."""
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        self.graph = torch.cuda.CUDAGraph()
        self.graph_steps = steps
        with torch.cuda.graph(self.graph, stream=s):
            self._step(stream=torch.cuda.current_stream(), nsteps=steps)
        torch.cuda.current_stream().wait_stream(s)
        return self.graph

    def run(self, nsteps: int, use_graph: bool = True):
        """nsteps steps: replays of the captured graph, then single steps for the remainder."""
        if use_graph:
            if self.graph is None:
                raise RuntimeError("call capture() first")
            reps, rest = divmod(nsteps, self.graph_steps)
            for _ in range(reps):
                self.graph.replay()
            for _ in range(rest):
                self.step()
        else:
            for _ in range(nsteps):
                self.step()

    def status(self):
        return C.cosmos_batch_status(self.batch, self.bws)

    def outcomes(self):
        """Per run: lapse at the centre point and its grid minimum (formed on the device by
        cosmos_batch_outcomes), with the run's status counters."""
        dev = torch.empty(2 * len(self.runs), dtype=torch.float64, device=self.device)
        C.cosmos_batch_outcomes(self.batch, self.arena, self.bws, dev)
        vals = dev.cpu().tolist()
        st = self.status()
        out = []
        for r, spec in enumerate(self.runs):
            out.append({"n": spec.n, "mu": spec.mu, "sigma": spec.sigma, "alpha_centre": vals[2 * r],
                        "alpha_min": vals[2 * r + 1], "collapsed": st[r]["collapsed"]})
        return out
