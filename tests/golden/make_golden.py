"""Writes the stored values of this folder from the CPU oracle alone.

op_counts.json: algorithmic operation counts (adds, multiplies, divisions and square roots,
one each) that the benchmark prices its FP64 rates with, counted by the oracle's
operation-counting scalar:
  * step_per_point: one RK4 step of the centred scheme per grid point (the interior
    right-hand side, one point-flux evaluation per point and the RK4 combinations);
  * kt_interface: one Kurganov-Tadmor interface flux (reconstruction, flux and speeds of
    both states, combination), the inverse metric and fluid recovery counted once per
    state; kt_prepass_per_point = 3 interfaces per point plus the 4 x 8 operations of the
    divergence.
The counts of the limiter and recovery branches depend on the state; they are taken on
the smooth fuzz state of seed 1 (8^3).

Run: python3 tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from tests.inputs import fuzz_state  # noqa: E402


def op_counts():
    s = oracle.Setup(n=(8, 8, 8), L=(2.4, 2.4, 2.4))
    u = fuzz_state(s.n, seed=1)
    step = oracle.count_flops(s, u)["step_per_point"]
    kt = oracle.count_kt_flops(oracle.Setup(n=(8, 8, 8), L=(2.4, 2.4, 2.4), fluid_scheme=1), u)
    return {"step_per_point": float(step), "kt_interface": float(kt["flops_per_interface"]),
            "kt_prepass_per_point": float(3 * kt["flops_per_interface"] + 32)}


if __name__ == "__main__":
    with open(os.path.join(HERE, "op_counts.json"), "w") as f:
        json.dump(op_counts(), f, indent=1, sort_keys=True)
        f.write("\n")
    print(open(os.path.join(HERE, "op_counts.json")).read())
