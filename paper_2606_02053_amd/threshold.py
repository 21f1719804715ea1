"""Threshold search for the perturbation amplitude mu: the use the batched and
adjoint forms are built for.

Collapse criterion: the lapse at the box centre after a fixed number of RK4
steps reaching a target value alpha_target (a collapsing region drives the
lapse down). The threshold mu* solves

    J(mu) = alpha_centre(T; mu, sigma) - alpha_target = 0

on a bracket [lo, hi] where J changes sign (J need not be monotone outside it;
the first sign change from lo is taken). Two stages:

* multisection on the batched form: K amplitudes spread evenly over the bracket
  run together as one batch (one launch per RK4 stage for all of them); the
  bracket shrinks by a factor K + 1 per round, where serial bisection gains one
  bit per run;
* Newton steps mu <- mu - J(mu) / J'(mu), J' by the discrete adjoint
  (adjoint.central_lapse), kept inside the bracket (a step that would leave it
  is replaced by the bracket midpoint) and narrowing it by the sign of J.

Every J evaluation runs the same stage kernel on the same grid, so the values
the two stages see agree bitwise.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import _lib as C
from .adjoint import RunConfig, central_lapse
from .batch import Batch, RunSpec


@dataclass
class ThresholdResult:
    mu: float                  # the threshold estimate
    J: float                   # alpha_centre(T) - alpha_target there
    dJ_dmu: float              # the adjoint derivative there
    bracket: tuple             # final bracket (J(lo) > 0 >= J(hi) in the decreasing case)
    batched_runs: int          # forward runs in the multisection stage
    newton_steps: int
    history: list = field(default_factory=list)  # (stage, mu, J) per evaluation


def centre_lapse_batch(mus, sigma: float, n: int, L: float, nsteps: int, params=None, isocurvature=None) -> list:
    """alpha at the box centre after nsteps for each mu, all runs in one batch (n a multiple of 16).
    With isocurvature = (zeta_mu, zeta_sigma) the scanned amplitude is that of the scalar field's
    iso-curvature mode (width sigma) on the curvature perturbation (zeta_mu, zeta_sigma)."""
    if isocurvature is None:
        b = Batch([RunSpec(n=n, mu=float(m), sigma=sigma, L=L) for m in mus], params)
    else:
        zmu, zsg = isocurvature
        b = Batch([RunSpec(n=n, mu=zmu, sigma=zsg, L=L, sc_mu=float(m), sc_sigma=sigma) for m in mus], params,
                  scalar=True)
    b.init()
    b.capture()
    b.run(nsteps)
    torch.cuda.synchronize()
    st = b.status()
    if any(x["nonfinite"] for x in st):
        raise RuntimeError("non-finite values in a batched run of the threshold scan")
    c = n // 2
    return [float(b.state(r)[17, c, c, c]) for r in range(len(mus))]


def multisection(sigma: float, lo: float, hi: float, alpha_target: float, n: int, L: float, nsteps: int,
                 K: int = 16, rounds: int = 2, params=None, history=None, isocurvature=None):
    """Shrink [lo, hi] around the first sign change of J with K batched runs per round
    (the first round also runs lo itself). Returns (lo, hi, J(lo), runs). isocurvature: see
    centre_lapse_batch."""
    J_lo = None
    runs = 0
    for _ in range(rounds):
        mus = [lo + (hi - lo) * (k + 1) / (K + 1) for k in range(K)]
        first = J_lo is None
        a = centre_lapse_batch(([lo] if first else []) + mus, sigma, n, L, nsteps, params, isocurvature)
        runs += len(a)
        if first:
            J_lo = a[0] - alpha_target
            a = a[1:]
        J = [x - alpha_target for x in a]
        if history is not None:
            history += [("batched", m, j) for m, j in zip(mus, J)]
        k = next((k for k in range(K) if (J[k] > 0) != (J_lo > 0)), None)
        if k is None:  # no sign change inside: it lies in the last interval (or nowhere)
            lo, J_lo = mus[-1], J[-1]
        else:
            hi = mus[k]
            if k > 0:
                lo, J_lo = mus[k - 1], J[k - 1]
    return lo, hi, J_lo, runs


def find_threshold(sigma: float, lo: float, hi: float, alpha_target: float, n: int = 32, L: float = 12.0,
                   nsteps: int = 50, K: int = 16, rounds: int = 2, tol: float = 1e-12, max_newton: int = 20,
                   params=None) -> ThresholdResult:
    """mu* with alpha_centre(T; mu*, sigma) = alpha_target inside [lo, hi]."""
    params = params if params is not None else C.make_params()
    history = []
    lo, hi, J_lo, runs = multisection(sigma, lo, hi, alpha_target, n, L, nsteps, K, rounds, params, history)
    cfg = RunConfig(n=n, L=L, nsteps=nsteps, checkpoint_every=max(1, min(20, nsteps)), params=params)
    mu = 0.5 * (lo + hi)
    best = (mu, float("nan"), float("nan"))
    steps = 0
    while steps < max_newton:
        steps += 1
        m = torch.tensor(mu, dtype=torch.float64, requires_grad=True)
        out = central_lapse(m, torch.tensor(sigma, dtype=torch.float64), cfg)
        out.backward()
        J, g = out.item() - alpha_target, m.grad.item()
        history.append(("newton", mu, J))
        best = (mu, J, g)
        if J == 0.0:
            break
        if (J > 0) == (J_lo > 0):
            lo, J_lo = mu, J
        else:
            hi = mu
        new = mu - J / g if g != 0.0 else 0.5 * (lo + hi)
        if not (min(lo, hi) < new < max(lo, hi)):
            new = 0.5 * (lo + hi)
        if abs(new - mu) <= tol * max(1.0, abs(mu)):
            break
        mu = new
    return ThresholdResult(mu=best[0], J=best[1], dJ_dmu=best[2], bracket=(lo, hi), batched_runs=runs,
                           newton_steps=steps, history=history)


def find_threshold_isocurvature(sigma: float, lo: float, hi: float, alpha_target: float, zeta=(0.0, 1.0),
                                n: int = 32, L: float = 12.0, nsteps: int = 50, K: int = 16, rounds: int = 6,
                                params=None) -> ThresholdResult:
    """The same search over the amplitude of the scalar field's iso-curvature mode (width sigma,
    on the curvature perturbation zeta = (mu, sigma)), by batched multisection alone (the
    adjoint does not carry the scalar field): the bracket shrinks by K + 1 per round."""
    params = params if params is not None else C.make_params()
    history = []
    lo, hi, J_lo, runs = multisection(sigma, lo, hi, alpha_target, n, L, nsteps, K, rounds, params, history,
                                      isocurvature=tuple(zeta))
    mu = 0.5 * (lo + hi)
    return ThresholdResult(mu=mu, J=float("nan"), dJ_dmu=float("nan"), bracket=(lo, hi), batched_runs=runs,
                           newton_steps=0, history=history)
