"""Threshold search for the perturbation amplitude mu: the use the batched and
adjoint forms are built for.

Collapse criterion: a run has collapsed when the lapse falls below alpha_th at some
grid point after some RK4 step up to the final time T -- the device's status counter
(params.alpha_collapse = alpha_th; each stage kernel's last stage counts the points
below it). The threshold mu* separates the amplitudes that collapse from those that do
not. Two stages:

* multisection on the batched form: K amplitudes spread evenly over the bracket
  [lo, hi] (lo not collapsing, hi collapsing) run together as one batch (one launch
  per RK4 stage for all of them), each run's collapse read from its device counters;
  the bracket shrinks by a factor K + 1 per round, where serial bisection gains one bit
  per run;
* Newton steps on the smooth surrogate J(mu) = alpha_centre(T; mu) - alpha_th, with
  J'(mu) by the discrete adjoint (adjoint.central_lapse), kept inside the bracket (a
  step that would leave it is replaced by the bracket midpoint) and narrowing it by the
  collapse test. The surrogate has its root at mu* where the lapse is lowest at the
  centre point and at the final step (a centred overdensity whose lapse keeps falling);
  the per-run outcomes (cosmos_batch_outcomes: centre lapse and grid minimum at T) show
  whether that holds.

Every evaluation runs the same stage kernel on the same grid, so the values the two
stages see agree bitwise.

find_threshold_interpolated uses the batch alone: each round's runs also give the centre lapse at
T, and the root of the cubic through the four runs around its sign change places the next
round's runs in a window 1e-4 as wide (two rounds reach rounding level).
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
    J: float                   # alpha_centre(T) - alpha_th there (nan: no Newton stage)
    dJ_dmu: float              # the adjoint derivative there
    bracket: tuple             # final bracket (lo does not collapse, hi does)
    batched_runs: int          # forward runs in the multisection stage
    newton_steps: int
    history: list = field(default_factory=list)  # (stage, mu, collapsed, alpha_centre, alpha_min) per evaluation


def scan_batch(mus, sigma: float, n: int, L: float, nsteps: int, alpha_th: float, params=None,
               isocurvature=None) -> list:
    """Run every amplitude in mus for nsteps in one batch (n a multiple of 16) and return per run
    {collapsed, alpha_centre, alpha_min}: collapsed from the device counters (the lapse fell below
    alpha_th at some point after some step), the lapse at the centre and its grid minimum at the
    end from cosmos_batch_outcomes. With isocurvature = (zeta_mu, zeta_sigma) the scanned amplitude
    is that of the scalar field's iso-curvature mode (width sigma) on the curvature perturbation
    (zeta_mu, zeta_sigma)."""
    p = C.make_params() if params is None else params
    p = C.cosmos_params(p.w, p.H0, p.eta, p.ko_eps, p.lapse_bg, p.evolve_shift, p.fluid_scheme, p.variant,
                        float(alpha_th), p.tile_x, p.tile_y, p.tile_z, p.tile_order)
    if isocurvature is None:
        b = Batch([RunSpec(n=n, mu=float(m), sigma=sigma, L=L) for m in mus], p)
    else:
        zmu, zsg = isocurvature
        b = Batch([RunSpec(n=n, mu=zmu, sigma=zsg, L=L, sc_mu=float(m), sc_sigma=sigma) for m in mus], p,
                  scalar=True)
    b.init()
    b.capture(steps=nsteps)  # the whole run as one graph: fluid fluxes carried from step to step
    b.run(nsteps)
    out = b.outcomes()
    st = b.status()
    if any(x["nonfinite"] for x in st):
        raise RuntimeError("non-finite values in a batched run of the threshold scan")
    return [{"collapsed": o["collapsed"] > 0, "alpha_centre": o["alpha_centre"], "alpha_min": o["alpha_min"]}
            for o in out]


def multisection(sigma: float, lo: float, hi: float, alpha_th: float, n: int, L: float, nsteps: int,
                 K: int = 16, rounds: int = 2, params=None, history=None, isocurvature=None):
    """Shrink [lo, hi] (lo not collapsing, hi collapsing) around the first amplitude that
    collapses, with K batched runs per round (the first round also runs both ends to check the
    bracket). Returns (lo, hi, runs). isocurvature: see scan_batch."""
    runs = 0
    first = True
    for _ in range(rounds):
        mus = [lo + (hi - lo) * (k + 1) / (K + 1) for k in range(K)]
        ends = [lo, hi] if first else []
        res = scan_batch(ends + mus, sigma, n, L, nsteps, alpha_th, params, isocurvature)
        runs += len(res)
        if first:
            if res[0]["collapsed"] or not res[1]["collapsed"]:
                raise ValueError(f"[{lo}, {hi}] does not bracket the collapse threshold")
            res = res[2:]
            first = False
        if history is not None:
            history += [("batched", m, r["collapsed"], r["alpha_centre"], r["alpha_min"]) for m, r in zip(mus, res)]
        k = next((k for k in range(K) if res[k]["collapsed"]), None)
        if k is None:  # the first collapsing amplitude lies in the last interval
            lo = mus[-1]
        else:
            hi = mus[k]
            if k > 0:
                lo = mus[k - 1]
    return lo, hi, runs


def find_threshold(sigma: float, lo: float, hi: float, alpha_th: float, n: int = 32, L: float = 12.0,
                   nsteps: int = 50, K: int = 16, rounds: int = 2, tol: float = 1e-12, max_newton: int = 20,
                   params=None) -> ThresholdResult:
    """The collapse threshold mu* in [lo, hi]: multisection on the device collapse counters, then
    Newton on alpha_centre(T; mu) - alpha_th with the adjoint derivative."""
    params = params if params is not None else C.make_params()
    history = []
    lo, hi, runs = multisection(sigma, lo, hi, alpha_th, n, L, nsteps, K, rounds, params, history)
    cfg = RunConfig(n=n, L=L, nsteps=nsteps, checkpoint_every=max(1, min(20, nsteps)), params=params)
    mu = 0.5 * (lo + hi)
    best = (mu, float("nan"), float("nan"))
    steps = 0
    while steps < max_newton:
        steps += 1
        m = torch.tensor(mu, dtype=torch.float64, requires_grad=True)
        out = central_lapse(m, torch.tensor(sigma, dtype=torch.float64), cfg)
        out.backward()
        J, g = out.item() - alpha_th, m.grad.item()
        history.append(("newton", mu, J < 0.0, out.item(), float("nan")))
        best = (mu, J, g)
        if J == 0.0:
            break
        if J > 0.0:  # the centre lapse stays above alpha_th: no collapse at this amplitude
            lo = mu
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


def _cubic_root(pts, lo: float, hi: float) -> float:
    """Root in [lo, hi] of the cubic through four (mu, J) points, J changing sign on [lo, hi]:
    bisection on the Lagrange form (no division by a derivative that may vanish)."""
    def cubic(x):
        total = 0.0
        for i, (xi, yi) in enumerate(pts):
            w = yi
            for j, (xj, _) in enumerate(pts):
                if j != i:
                    w *= (x - xj) / (xi - xj)
            total += w
        return total
    flo = cubic(lo)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid == lo or mid == hi:
            break
        fm = cubic(mid)
        if (fm > 0.0) == (flo > 0.0):
            lo, flo = mid, fm
        else:
            hi = mid
    return 0.5 * (lo + hi)


def find_threshold_interpolated(sigma: float, lo: float, hi: float, alpha_th: float, n: int = 32,
                                L: float = 12.0, nsteps: int = 50, K: int = 16, rounds: int = 2, tol: float = 1e-12,
                                params=None) -> ThresholdResult:
    """The collapse threshold by batched rounds alone: every round runs K amplitudes in one batch and
    reads each run's centre lapse at T from the device (cosmos_batch_outcomes); the root of
    alpha_centre(T; mu) - alpha_th on the cubic through the four runs around its sign change is the
    next estimate, and the next round spreads its K runs over a window 1e-4 of the previous one
    around it. The collapse counters keep [lo, hi] a bracket (lo does not collapse, hi does); a
    round whose runs do not change sign is repeated over the bracket. Where the centre lapse is
    the run's lowest, the two criteria share their root."""
    history = []
    runs, fitted = 0, 0
    a, b = lo, hi
    mu = 0.5 * (lo + hi)
    for _ in range(rounds + 4):  # a round without a sign change is repeated over the bracket
        mus = [a + (b - a) * (k + 1) / (K + 1) for k in range(K)]
        res = scan_batch(mus, sigma, n, L, nsteps, alpha_th, params)
        runs += K
        history += [("batched", m, x["collapsed"], x["alpha_centre"], x["alpha_min"]) for m, x in zip(mus, res)]
        for m, x in zip(mus, res):
            if x["collapsed"]:
                hi = min(hi, m)
            else:
                lo = max(lo, m)
        J = [x["alpha_centre"] - alpha_th for x in res]
        k = next((k for k in range(K - 1) if (J[k] > 0.0) != (J[k + 1] > 0.0)), None)
        if k is None:
            a, b = lo, hi
            continue
        i0 = min(max(k - 1, 0), K - 4)
        mu = _cubic_root(list(zip(mus[i0:i0 + 4], J[i0:i0 + 4])), mus[k], mus[k + 1])
        fitted += 1
        if fitted >= rounds or mus[k + 1] - mus[k] <= tol:
            break
        w = 1e-4 * (b - a)
        a, b = max(lo, mu - 0.5 * w), min(hi, mu + 0.5 * w)
    return ThresholdResult(mu=mu, J=float("nan"), dJ_dmu=float("nan"), bracket=(lo, hi), batched_runs=runs,
                           newton_steps=0, history=history)


def find_threshold_isocurvature(sigma: float, lo: float, hi: float, alpha_th: float, zeta=(0.0, 1.0),
                                n: int = 32, L: float = 12.0, nsteps: int = 50, K: int = 16, rounds: int = 6,
                                params=None) -> ThresholdResult:
    """The same collapse threshold over the amplitude of the scalar field's iso-curvature mode
    (width sigma, on the curvature perturbation zeta = (mu, sigma)), by batched multisection alone
    (the adjoint does not carry the scalar field): the bracket shrinks by K + 1 per round."""
    params = params if params is not None else C.make_params()
    history = []
    lo, hi, runs = multisection(sigma, lo, hi, alpha_th, n, L, nsteps, K, rounds, params, history,
                                isocurvature=tuple(zeta))
    mu = 0.5 * (lo + hi)
    return ThresholdResult(mu=mu, J=float("nan"), dJ_dmu=float("nan"), bracket=(lo, hi), batched_runs=runs,
                           newton_steps=0, history=history)
