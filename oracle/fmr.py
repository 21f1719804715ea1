"""Fixed mesh refinement on the oracle's periodic RK4 step -- TEST INFRASTRUCTURE ONLY.

Same rule as the rest of the package: only ``tests/``, ``__graft_entry__.smoke()`` and
``bench.py``'s ``cpu_baseline`` leg may import this module, and it imports nothing from the
product path.

The paper evolves on nested refinement layers (fixed mesh refinement: "Statement of need", and
the lowest, 1st and 2nd layers of the adiabatic-fluctuation example) and leaves the scheme to its
references. This module states, in its plainest form, the scheme the library implements:

* A layer refines a box of its parent by 2 in every direction, vertex-aligned: the child's
  interior point i (per axis, 0 <= i < 2 m) lies at parent index origin + i / 2.
* The child is stored with W = 12 extra points beyond each face (a buffer of 3 stencil points for
  each of the 4 RK4 stages) and advanced by the RK4 step of the whole padded array as if it were
  periodic. Whatever the wrap-around or the faces spoil reaches at most 3 points further inwards
  per stage, so after a step the outer 12 layers are stale and the interior is exact.
* Berger-Oliger sub-cycling: per parent step dt the child takes two steps of dt / 2. Before each
  child step the buffer is refilled from the parent: in space by 6-point Lagrange interpolation
  per axis (tensor product, coincident points copied; sixth order, so that the second derivatives
  of the interpolation error, which alternates from point to point, stay fourth order), in time
  by the continuous extension of the parent's RK4 step (its four stage slopes with the cubic
  weights b_i(theta); third order, a local error O(dt^4) like the step's own; the second child
  step starts at the midpoint).
* After the two child steps the parent points that the child's interior covers take the child's
  values (injection), and the child's own children are handled the same way, recursively.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import NF, Setup, rhs, rk4

W = 12  # buffer width in child points: stencil radius 3 x 4 RK4 stages


@dataclass
class Box:
    """A refined layer: `origin` (parent array index of the child's interior point 0, per axis
    x, y, z) and `m` (parent cells covered per axis: the child interior has 2 m points)."""
    origin: tuple
    m: tuple

    def shape(self):
        """(nz, ny, nx) of the padded child array."""
        return tuple(2 * self.m[a] + 2 * W for a in (2, 1, 0))


def child_setup(parent: Setup, box: Box) -> Setup:
    """Setup of the padded child array: the parent's physics, spacing halved."""
    n = tuple(2 * box.m[a] + 2 * W for a in range(3))
    L = tuple(n[a] * parent.h[a] / 2.0 for a in range(3))
    return Setup(n=n, L=L, w=parent.w, H0=parent.H0, eta=parent.eta, ko_eps=parent.ko_eps,
                 lapse_bg=parent.lapse_bg, evolve_shift=parent.evolve_shift, fluid_scheme=parent.fluid_scheme)


def interp_matrix(n_parent: int, origin: int, m: int) -> np.ndarray:
    """Rows: padded child points a = 0 .. 2 m + 2 W - 1 at parent coordinate origin + (a - W) / 2;
    columns: parent points (periodic). A coincident point copies its parent value; a midpoint
    between parent points I and I + 1 takes the quintic through I - 2 .. I + 3:
    (3, -25, 150, 150, -25, 3) / 256."""
    nf = 2 * m + 2 * W
    P = np.zeros((nf, n_parent))
    for a in range(nf):
        d = a - W
        if d % 2 == 0:
            P[a, (origin + d // 2) % n_parent] = 1.0
        else:
            i = origin + (d - 1) // 2
            for off, wgt in zip((-2, -1, 0, 1, 2, 3), (3.0, -25.0, 150.0, 150.0, -25.0, 3.0)):
                P[a, (i + off) % n_parent] += wgt / 256.0
    return P


def prolong(u_parent: np.ndarray, box: Box) -> np.ndarray:
    """The whole padded child array interpolated from a parent state (25, nz, ny, nx)."""
    nz, ny, nx = u_parent.shape[1:]
    Px = interp_matrix(nx, box.origin[0], box.m[0])
    Py = interp_matrix(ny, box.origin[1], box.m[1])
    Pz = interp_matrix(nz, box.origin[2], box.m[2])
    return np.einsum("ck,bj,ai,fkji->fcba", Pz, Py, Px, u_parent, optimize=True)


def shell_mask(box: Box) -> np.ndarray:
    """True at the padded child points within W of a face (the buffer)."""
    nz, ny, nx = box.shape()
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    inner = ((x >= W) & (x < nx - W) & (y >= W) & (y < ny - W) & (z >= W) & (z < nz - W))
    return ~inner


def rk4_dense_weights(theta: float):
    """Weights b_1..b_4 of the classic RK4 step's continuous extension: u(t0 + theta dt) =
    u0 + dt sum_i b_i(theta) k_i, with k_1..k_4 the step's stage slopes (b_i(1) = 1/6, 1/3, 1/3,
    1/6: the step itself)."""
    t2, t3 = theta * theta, theta * theta * theta
    b1 = theta - 1.5 * t2 + (2.0 / 3.0) * t3
    b23 = t2 - (2.0 / 3.0) * t3
    b4 = -0.5 * t2 + (2.0 / 3.0) * t3
    return b1, b23, b23, b4


def rk4_stages(s: Setup, u0, t: float, dt: float, parallel: bool = True):
    """The classic RK4 step written out: slopes k_1..k_4 and the new state."""
    k1, _ = rhs(s, u0, t, parallel=parallel)
    k2, _ = rhs(s, u0 + (0.5 * dt) * k1, t + 0.5 * dt, parallel=parallel)
    k3, _ = rhs(s, u0 + (0.5 * dt) * k2, t + 0.5 * dt, parallel=parallel)
    k4, _ = rhs(s, u0 + dt * k3, t + dt, parallel=parallel)
    return (k1, k2, k3, k4), u0 + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def dense(u0, ks, dt: float, theta: float):
    """The RK4 continuous extension at t0 + theta dt."""
    b = rk4_dense_weights(theta)
    return u0 + dt * (b[0] * ks[0] + b[1] * ks[1] + b[2] * ks[2] + b[3] * ks[3])


def slopes_from_stage_states(u0, U2, U3, U4, u1, dt: float):
    """The slopes of an RK4 step from its stage states U2 = u0 + dt/2 k1, U3 = u0 + dt/2 k2,
    U4 = u0 + dt k3 and its result u1 = u0 + dt/6 (k1 + 2 k2 + 2 k3 + k4)."""
    k1 = (U2 - u0) / (0.5 * dt)
    k2 = (U3 - u0) / (0.5 * dt)
    k3 = (U4 - u0) / dt
    k4 = 6.0 * (u1 - u0) / dt - k1 - 2.0 * k2 - 2.0 * k3
    return k1, k2, k3, k4


def restrict(u_child: np.ndarray, u_parent: np.ndarray, box: Box) -> np.ndarray:
    """Parent points origin .. origin + m - 1 (per axis, periodic) take the coincident child
    interior values (child interior index 2 (X - origin))."""
    out = u_parent.copy()
    nz, ny, nx = u_parent.shape[1:]
    X = [(box.origin[a] + np.arange(box.m[a])) for a in range(3)]
    C = [W + 2 * np.arange(box.m[a]) for a in range(3)]
    out[np.ix_(np.arange(NF), X[2] % nz, X[1] % ny, X[0] % nx)] = u_child[np.ix_(np.arange(NF), C[2], C[1], C[0])]
    return out


class Hierarchy:
    """Layer 0: the periodic grid `setup`; layer l + 1 refines `boxes[l]` of layer l (its origin in
    layer l's array indices; for l >= 1 the box with its buffer and the interpolation stencil must
    lie inside layer l's interior, at least W points from its faces)."""

    def __init__(self, setup: Setup, boxes):
        self.setups = [setup]
        self.boxes = list(boxes)
        for l, b in enumerate(self.boxes):
            if l >= 1:
                par = self.setups[l]
                for a in range(3):
                    lo, hi = b.origin[a] - W // 2 - 2, b.origin[a] + b.m[a] + W // 2 + 3
                    if lo < W or hi > par.n[a] - W:
                        raise ValueError(f"box {l} reaches into layer {l}'s buffer along axis {a}")
            self.setups.append(child_setup(self.setups[l], b))

    def init(self, u0: np.ndarray):
        """States of all layers from layer 0's initial data (finer layers interpolated)."""
        states = [np.ascontiguousarray(u0, dtype=np.float64)]
        for b in self.boxes:
            states.append(prolong(states[-1], b))
        return states

    def step(self, states, t: float, dt: float, level: int = 0, parallel: bool = True):
        """One step dt of layer `level` and two steps dt / 2 of each finer layer, recursively."""
        s = self.setups[level]
        u0 = states[level]
        if level == len(self.boxes):
            states[level], _ = rk4(s, u0, t, dt, 1, parallel=parallel)
            return
        ks, u1 = rk4_stages(s, u0, t, dt, parallel=parallel)
        box = self.boxes[level]
        mask = shell_mask(box)
        for half in (0, 1):
            src = u0 if half == 0 else dense(u0, ks, dt, 0.5)
            child = states[level + 1].copy()
            child[:, mask] = prolong(src, box)[:, mask]
            states[level + 1] = child
            self.step(states, t + 0.5 * half * dt, 0.5 * dt, level + 1, parallel)
        states[level] = restrict(states[level + 1], u1, box)
