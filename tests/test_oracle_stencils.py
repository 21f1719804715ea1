"""Pins of the oracle's difference operators, time integrator, fluid recovery
and random-number generator against closed forms (no GPU).

Operators (4th-order centred D1, D2, mixed D1_a D1_b, lopsided upwind
advection, 6th-difference Kreiss-Oliger) are checked by polynomial exactness,
by their Fourier symbols on periodic grids and by the Nyquist mode; RK4 by its
amplification polynomial; the radiation-fluid recovery by a primitive ->
conserved -> primitive round trip; SplitMix64 by its published first outputs.
"""
import numpy as np
import pytest

from tests.inputs import fuzz_state


def _coords(s, axis):
    n, L = s.n[axis], s.L[axis]
    return -0.5 * L + np.arange(n) * (L / n)


def _grid_fn(s, fn):
    x = _coords(s, 0)[None, None, :]
    y = _coords(s, 1)[None, :, None]
    z = _coords(s, 2)[:, None, None]
    return np.broadcast_to(fn(x, y, z), s.shape[1:]).copy()


@pytest.fixture
def setup(orc):
    # non-cubic, anisotropic grid: a transposed axis or spacing fails here
    return orc.Setup(n=(20, 16, 24), L=(2.0, 1.2, 3.0))


def test_first_derivative_exact_to_degree_4(orc, setup):
    ijk = (10, 8, 12)  # far from the periodic seam
    h = setup.h
    for a in range(3):
        for p in range(5):
            f = _grid_fn(setup, lambda x, y, z: [x, y, z][a] ** p + 0.3 * [y, z, x][a])
            x0 = [_coords(setup, b)[ijk[b]] for b in range(3)][a]
            exact = p * x0 ** (p - 1) if p > 0 else 0.0
            got = orc.stencil(setup, f, ijk, "d1", a)
            assert abs(got - exact) < 1e-11 * (1 + abs(exact)), (a, p, got, exact)


def test_second_derivative_exact_to_degree_5(orc, setup):
    ijk = (10, 8, 12)
    for a in range(3):
        for p in range(6):
            f = _grid_fn(setup, lambda x, y, z: [x, y, z][a] ** p)
            x0 = _coords(setup, a)[ijk[a]]
            exact = p * (p - 1) * x0 ** (p - 2) if p > 1 else 0.0
            got = orc.stencil(setup, f, ijk, "d2", a)
            assert abs(got - exact) < 1e-9 * (1 + abs(exact)), (a, p, got, exact)


def test_mixed_derivative_tensor_product(orc, setup):
    ijk = (10, 8, 12)
    x0 = [_coords(setup, b)[ijk[b]] for b in range(3)]
    for a, b in [(0, 1), (0, 2), (1, 2), (1, 0)]:
        for p in range(5):
            for q in range(5):
                f = _grid_fn(setup, lambda x, y, z: [x, y, z][a] ** p * [x, y, z][b] ** q)
                exact = (p * x0[a] ** (p - 1) if p else 0.0) * (q * x0[b] ** (q - 1) if q else 0.0)
                got = orc.stencil(setup, f, ijk, "mixed", a, b)
                assert abs(got - exact) < 1e-9 * (1 + abs(exact)), (a, b, p, q, got, exact)


def test_upwind_exact_to_degree_4_and_one_sided(orc, setup):
    ijk = (10, 8, 12)
    x0 = [_coords(setup, b)[ijk[b]] for b in range(3)]
    for a in range(3):
        for sgn in (+1.0, -1.0):
            beta = [0.0, 0.0, 0.0]
            beta[a] = 0.7 * sgn
            for p in range(5):
                f = _grid_fn(setup, lambda x, y, z: [x, y, z][a] ** p)
                exact = beta[a] * (p * x0[a] ** (p - 1) if p else 0.0)
                got = orc.stencil(setup, f, ijk, "adv", a, 0, beta)
                assert abs(got - exact) < 1e-10 * (1 + abs(exact)), (a, sgn, p)
            # the stencil only reads the upwind side: beta > 0 reads -1..+3, beta <= 0 reads -3..+1
            f = _grid_fn(setup, lambda x, y, z: np.sin([x, y, z][a]))
            base = orc.stencil(setup, f, ijk, "adv", a, 0, beta)
            g = f.copy()
            far = [-3, -2] if sgn > 0 else [2, 3]
            for off in far:
                idx = list(ijk)
                idx[a] += off
                g[idx[2], idx[1], idx[0]] += 100.0
            assert orc.stencil(setup, g, ijk, "adv", a, 0, beta) == base
            g = f.copy()
            idx = list(ijk)
            idx[a] += 3 if sgn > 0 else -3
            g[idx[2], idx[1], idx[0]] += 1.0
            assert orc.stencil(setup, g, ijk, "adv", a, 0, beta) != base
    # beta == 0 takes the U- branch and gives 0 contribution
    f = _grid_fn(setup, lambda x, y, z: x * y * z)
    assert orc.stencil(setup, f, ijk, "adv", 0, 0, [0.0, 0.0, 0.0]) == 0.0


def test_ko_annihilates_degree_5(orc, setup):
    ijk = (10, 8, 12)
    for a in range(3):
        for p in range(6):
            f = _grid_fn(setup, lambda x, y, z: [x, y, z][a] ** p)
            got = orc.stencil(setup, f, ijk, "ko", eps=0.1)
            assert abs(got) < 1e-9, (a, p, got)


@pytest.mark.parametrize("m", [1, 2, 3, 5])
def test_fourier_symbols(orc, m):
    s = orc.Setup(n=(16, 12, 20), L=(1.6, 0.9, 2.5))
    ijk = (5, 7, 3)
    for a in range(3):
        n, h = s.n[a], s.h[a]
        th = 2 * np.pi * m / n
        phase = 0.37
        idx = [np.arange(s.n[0])[None, None, :], np.arange(s.n[1])[None, :, None], np.arange(s.n[2])[:, None, None]]
        arg = th * idx[a] + phase
        f = np.broadcast_to(np.sin(arg), s.shape[1:]).copy()
        c = np.broadcast_to(np.cos(arg), s.shape[1:])[ijk[2], ijk[1], ijk[0]]
        sv = f[ijk[2], ijk[1], ijk[0]]
        d1 = (8 * np.sin(th) - np.sin(2 * th)) / (6 * h) * c
        d2 = (32 * np.cos(th) - 2 * np.cos(2 * th) - 30) / (12 * h * h) * sv
        ko = -(0.1 / h) * np.sin(th / 2) ** 6 * sv
        assert abs(orc.stencil(s, f, ijk, "d1", a) - d1) < 1e-12 * (1 + abs(d1)) * n
        assert abs(orc.stencil(s, f, ijk, "d2", a) - d2) < 1e-12 * (1 + abs(d2)) * n
        assert abs(orc.stencil(s, f, ijk, "ko", eps=0.1) - ko) < 1e-12 * (1 + abs(ko)) * n
    # mixed: symbol -s_a s_b for cos(th_a i + th_b j)
    idx = [np.arange(s.n[0])[None, None, :], np.arange(s.n[1])[None, :, None], np.arange(s.n[2])[:, None, None]]
    for a, b in [(0, 1), (0, 2), (1, 2)]:
        tha, thb = 2 * np.pi * m / s.n[a], 2 * np.pi * (m % 3 + 1) / s.n[b]
        f = np.broadcast_to(np.cos(tha * idx[a] + thb * idx[b]), s.shape[1:]).copy()
        sa = (8 * np.sin(tha) - np.sin(2 * tha)) / (6 * s.h[a])
        sb = (8 * np.sin(thb) - np.sin(2 * thb)) / (6 * s.h[b])
        exact = -sa * sb * f[ijk[2], ijk[1], ijk[0]]
        got = orc.stencil(s, f, ijk, "mixed", a, b)
        assert abs(got - exact) < 1e-11 * (1 + abs(exact)) * 20


def test_ko_nyquist(orc):
    s = orc.Setup(n=(16, 10, 12), L=(1.0, 1.0, 1.0))
    for a in range(3):
        idx = [np.arange(s.n[0])[None, None, :], np.arange(s.n[1])[None, :, None], np.arange(s.n[2])[:, None, None]]
        f = np.broadcast_to((-1.0) ** idx[a], s.shape[1:]).copy()
        for ijk in [(0, 0, 0), (5, 3, 7)]:
            got = orc.stencil(s, f, ijk, "ko", eps=0.1)
            assert got == -(0.1 / s.h[a]) * f[ijk[2], ijk[1], ijk[0]]


def test_rk4_amplification_polynomial(orc):
    # flat space with a uniform shift: every term vanishes except the
    # Gamma-driver damping, d beta/dt = -eta beta, a scalar linear ODE
    s = orc.Setup(n=(8, 8, 8), L=(4.0, 4.0, 4.0), H0=0.0, eta=1.7)
    u = np.zeros(s.shape)
    u[orc.CHI] = 1.0
    u[orc.GT + 0] = u[orc.GT + 3] = u[orc.GT + 5] = 1.0
    u[orc.ALP] = 1.0
    b = np.array([0.3, -0.2, 0.1])
    for c in range(3):
        u[orc.BET + c] = b[c]
    for dt in (0.05, 0.3, 0.9):
        v, _ = orc.rk4(s, u, 0.0, dt, 1)
        z = -s.eta * dt
        R = 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
        for c in range(3):
            assert np.allclose(v[orc.BET + c], b[c] * R, rtol=1e-15, atol=1e-16)
        # the other fields change only by the round-off of stencils applied to the
        # uniform but not exactly representable shift values
        rest = np.delete(v - u, [orc.BET, orc.BET + 1, orc.BET + 2], axis=0)
        assert np.abs(rest).max() < 1e-15


def test_fluid_recovery_round_trip(orc):
    rng = np.random.default_rng(7)
    for trial in range(200):
        w = [1.0 / 3.0, 0.2, 0.6][trial % 3]
        chi = rng.uniform(0.5, 1.5)
        A = rng.normal(size=(3, 3)) * 0.2
        gt = np.eye(3) + 0.5 * (A + A.T)
        gphys = gt / chi
        ginv = np.linalg.inv(gphys)
        rho = rng.uniform(0.1, 3.0)
        # subluminal covariant velocity: v^2 = gamma^ij v_i v_j < 1
        v = rng.normal(size=3)
        v *= rng.uniform(0.0, 0.95) / np.sqrt(v @ ginv @ v)
        W2 = 1.0 / (1.0 - v @ ginv @ v)
        X = (1 + w) * rho * W2
        E = X - w * rho
        S = X * v
        gt6 = np.array([gt[0, 0], gt[0, 1], gt[0, 2], gt[1, 1], gt[1, 2], gt[2, 2]])
        m = orc.matter_point(w, chi, gt6, E / chi ** 1.5, S / chi ** 1.5)
        assert not m["fail"]
        assert m["P"] == pytest.approx(w * rho, rel=1e-12, abs=1e-14)
        assert m["invX"] == pytest.approx(1.0 / X, rel=1e-12)
        assert m["S2"] == pytest.approx(S @ ginv @ S, rel=1e-12)
        assert np.allclose(m["Sup"], ginv @ S, rtol=1e-12, atol=1e-14)
    # fluid at rest: P = w E exactly in the closed form
    m = orc.matter_point(1.0 / 3.0, 1.0, [1, 0, 0, 1, 0, 1], 3.0, [0, 0, 0])
    assert m["P"] == pytest.approx(1.0, rel=1e-15) and not m["fail"]
    # invalid states are flagged: E <= 0, and momentum beyond the bound
    assert orc.matter_point(1.0 / 3.0, 1.0, [1, 0, 0, 1, 0, 1], -1.0, [0, 0, 0])["fail"]
    bad = orc.matter_point(1.0 / 3.0, 1.0, [1, 0, 0, 1, 0, 1], 1.0, [2.0, 0, 0])
    assert bad["fail"] and bad["P"] == pytest.approx(2.0 / 3.0 - 1.0)


def test_splitmix64_published_outputs(orc):
    # first three outputs of SplitMix64 from state 0 (reference vectors of the generator)
    assert orc.splitmix64(0, 0) == 0xE220A8397B1DCDAF
    assert orc.splitmix64(0, 1) == 0x6E789E6AA1B965F4
    assert orc.splitmix64(0, 2) == 0x06C45D188009454F


def test_sampled_evaluations_equal_full_grid(orc):
    s = orc.Setup(n=(16, 12, 14), L=(3.0, 2.5, 2.8))
    u = fuzz_state(s.n, seed=11)
    pts = np.array([0, 5, 17, 16 * 12 * 14 - 1, 1000, 2000], dtype=np.int64)
    full, _ = orc.rhs(s, u, t=0.3)
    flat = full.reshape(25, -1)
    samp = orc.rhs_at_points(s, u, pts, t=0.3)
    assert np.array_equal(samp, flat[:, pts].T)
    dt = 0.25 * min(s.h)
    step, _ = orc.rk4(s, u, 0.3, dt, 1)
    samp = orc.rk4_at_points(s, u, pts[:3], 0.3, dt)
    assert np.array_equal(samp, step.reshape(25, -1)[:, pts[:3]].T)
