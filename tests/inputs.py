"""Seeded synthetic inputs shared by the oracle side and the GPU side of the tests.

This module holds no arithmetic of the method: it only draws reproducible
states. ``fuzz_state`` builds smooth, periodic random perturbations of all 25
fields around a valid background (conformal metric positive definite, chi and
alpha in [0.5, 1.5], positive fluid energy density, subluminal momentum), so
that every term of the right-hand side is exercised -- physical initial data
zero out the traceless curvature, the connection functions, the shift and the
fluid momentum at t = 0.
"""
import numpy as np

NF = 25

# (background, amplitude) per field, in field order
_BG_AMP = ([(1.0, 0.2)]                                   # chi
           + [(1.0, 0.1), (0.0, 0.05), (0.0, 0.05), (1.0, 0.1), (0.0, 0.05), (1.0, 0.1)]  # gt
           + [(-1.0, 0.3)]                                # K
           + [(0.0, 0.1)] * 6                             # At
           + [(0.0, 0.1)] * 3                             # Gt
           + [(1.0, 0.2)]                                 # alpha
           + [(0.0, 0.1)] * 3                             # beta (both signs: both upwind branches)
           + [(1.0, 0.2)]                                 # Et
           + [(0.0, 0.05)] * 3)                           # St


def fuzz_state(n, seed, kmax=2, modes=3, scale=1.0):
    """Smooth periodic random state of shape (25, nz, ny, nx), n = (nx, ny, nz)."""
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    i = np.arange(nx)[None, None, :] / nx
    j = np.arange(ny)[None, :, None] / ny
    k = np.arange(nz)[:, None, None] / nz
    u = np.empty((NF, nz, ny, nx))
    for f in range(NF):
        bg, amp = _BG_AMP[f]
        s = np.zeros((nz, ny, nx))
        wsum = 0.0
        for _ in range(modes):
            m = rng.integers(-kmax, kmax + 1, size=3)
            if not m.any():
                m[0] = 1
            a = rng.uniform(0.5, 1.0)
            ph = rng.uniform(0, 2 * np.pi)
            s += a * np.sin(2 * np.pi * (m[0] * i + m[1] * j + m[2] * k) + ph)
            wsum += a
        u[f] = bg + scale * amp * s / wsum
    return u


def fuzz_direction(n, seed, kmax=2):
    """Smooth periodic random perturbation direction (all fields O(1))."""
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    i = np.arange(nx)[None, None, :] / nx
    j = np.arange(ny)[None, :, None] / ny
    k = np.arange(nz)[:, None, None] / nz
    v = np.empty((NF, nz, ny, nx))
    for f in range(NF):
        m = rng.integers(-kmax, kmax + 1, size=3)
        ph = rng.uniform(0, 2 * np.pi)
        v[f] = np.sin(2 * np.pi * (m[0] * i + m[1] * j + m[2] * k) + ph) + rng.uniform(-0.5, 0.5)
    return v


def sample_points(n, count, seed):
    """Distinct random linear point indices, always including the corners and the centre."""
    nx, ny, nz = n
    N3 = nx * ny * nz
    rng = np.random.default_rng(seed)
    fixed = [0, N3 - 1, nx // 2 + nx * (ny // 2 + ny * (nz // 2)), nx - 1, nx * ny - 1]
    pts = set(int(p) for p in fixed)
    while len(pts) < min(count, N3):
        pts.add(int(rng.integers(0, N3)))
    return np.array(sorted(pts), dtype=np.int64)


def fuzz_scalar(n, seed, kmax=2, modes=3, amp=(0.2, 0.1)):
    """Smooth periodic random (phi, Pi) of shape (2, nz, ny, nx): Fourier modes about 0."""
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    i = np.arange(nx)[None, None, :] / nx
    j = np.arange(ny)[None, :, None] / ny
    k = np.arange(nz)[:, None, None] / nz
    s = np.zeros((2, nz, ny, nx))
    for f in range(2):
        wsum = 0.0
        for _ in range(modes):
            m = rng.integers(-kmax, kmax + 1, size=3)
            if not m.any():
                m[0] = 1
            a = rng.uniform(0.5, 1.0)
            ph = rng.uniform(0, 2 * np.pi)
            s[f] += a * np.sin(2 * np.pi * (m[0] * i + m[1] * j + m[2] * k) + ph)
            wsum += a
        s[f] *= amp[f] / wsum
    return s
