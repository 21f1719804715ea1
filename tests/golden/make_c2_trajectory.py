"""Writes c2_128cubed_100steps.json from the CPU oracle alone.

The 128^3 configuration (periodic box L = 12 in units of the initial Hubble radius, Gaussian
curvature perturbation zeta = mu exp(-r^2 / 2 sigma^2) with mu = 0.5, sigma = 1.5 about the box
centre, radiation fluid w = 1/3 with the Hamiltonian-constraint density, H0 = 1, eta = 1, KO 0.1,
dt = 0.25 h) is evolved for 100 classic RK4 steps by the oracle (OpenMP over z-planes; each point's
arithmetic is that of the serial oracle, so the result is the serial one bitwise). Stored:

  * points: 64 linear indices p = i + 128 (j + 128 k): the centre (where the perturbation peaks),
    its six nearest neighbours along the axes, the corners, and random points (seed 2606);
  * values[q][f]: field f of the step-100 state at points[q];
  * field_absmax[f]: max over the whole grid of |field f| at step 100 (the per-field scale of the
    parity metric: error / max(field_absmax, 1e-3));
  * norms: the oracle's eight constraint norms of the step-100 state.

A GPU test runs the same 100 steps from its own initial data and compares at these points.

Run: python3 tests/golden/make_c2_trajectory.py   (about 15 minutes on 8 host threads)
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from tests.inputs import sample_points  # noqa: E402

OUT = os.path.join(HERE, "c2_128cubed_100steps.json")
N, LBOX, MU, SIGMA, STEPS = 128, 12.0, 0.5, 1.5, 100


def points():
    n = (N, N, N)
    c = N // 2 + N * (N // 2 + N * (N // 2))
    near = [c + 1, c - 1, c + N, c - N, c + N * N, c - N * N]
    base = sample_points(n, 57, seed=2606)
    return np.array(sorted(set(int(p) for p in base) | {c, *near}), dtype=np.int64)


def main():
    s = oracle.Setup(n=(N, N, N), L=(LBOX, LBOX, LBOX))
    ini = oracle.Init(mu=MU, sigma=SIGMA)
    u0 = oracle.init_fields(s, ini)
    dt = 0.25 * s.h[0]
    t0 = time.time()
    u, pf = oracle.rk4(s, u0, 0.0, dt, STEPS, parallel=True)
    wall = time.time() - t0
    pts = points()
    flat = u.reshape(oracle.NF, -1)
    norms = oracle.constraints(s, u, parallel=True)
    doc = {
        "config": {"n": N, "L": LBOX, "mu": MU, "sigma": SIGMA, "steps": STEPS, "dt": dt, "H0": 1.0,
                   "w": 1.0 / 3.0, "eta": 1.0, "ko_eps": 0.1, "profile": "gauss", "noise_amp": 0.0},
        "prim_fail": int(pf),
        "points": [int(p) for p in pts],
        "values": [[float(flat[f, p]) for f in range(oracle.NF)] for p in pts],
        "field_absmax": [float(np.abs(flat[f]).max()) for f in range(oracle.NF)],
        "norms": [float(x) for x in norms],
        "oracle_wall_s": round(wall, 1),
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=0)
        f.write("\n")
    print(f"wrote {OUT}: {len(pts)} points, oracle {wall:.0f} s, norms {norms[:5]}")


if __name__ == "__main__":
    main()
