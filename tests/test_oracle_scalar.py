"""Pins of the oracle's massless scalar field (phi, Pi = n.d phi) against what the
mathematics fixes independently of its code:

* flat space: the right-hand side of a Fourier mode is the exact symbol of the
  4th-order second difference (d_t Pi = D2 phi) plus the Kreiss-Oliger symbol on
  both fields, and d_t phi = Pi;
* homogeneous radiation + scalar universe: Pi a^3 is constant (a^3 = chi^(-3/2)) and
  the Friedmann (Hamiltonian) constraint with the scalar's energy is conserved, both
  up to the RK4 error, converging at 4th order in dt;
* iso-curvature initial data: the Hamiltonian constraint (scalar energy included)
  converges to zero at 4th order, the momentum constraint is exactly zero;
* constraint propagation with an inhomogeneous scalar field: H and M converge at 4th
  order under grid refinement at a fixed time;
* no scalar field = amplitude zero: the scalar entry points reproduce the plain ones
  bitwise.
"""
import numpy as np
import pytest

from inputs import fuzz_state

W = 1.0 / 3.0


def flat(n, E=0.1):
    u = np.zeros((25,) + tuple(reversed(n)))
    u[0] = u[1] = u[4] = u[6] = u[17] = 1.0
    u[21] = E
    return u


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_flat_space_fourier_mode(orc, axis):
    n, L, eps = (16, 16, 16), (4.0, 4.0, 4.0), 0.1
    s = orc.Setup(n=n, L=L, ko_eps=eps)
    h = L[axis] / n[axis]
    m = 3
    k = 2 * np.pi * m / L[axis]
    x = np.arange(n[axis]) * h - L[axis] / 2
    shape = [1, 1, 1]
    shape[2 - axis] = n[axis]
    A, B = 0.01, 0.02
    sc = np.zeros((2,) + s.shape[1:])
    sc[0] = (A * np.sin(k * x)).reshape(shape)
    sc[1] = (B * np.cos(k * x)).reshape(shape)
    du, ds, _ = orc.rhs_sc(s, flat(n), sc)
    th = k * h
    d2 = (-2 * np.cos(2 * th) + 32 * np.cos(th) - 30) / (12 * h * h)
    ko = eps / (64 * h) * (2 * np.cos(th) - 2) ** 3
    exp_phi = (B * np.cos(k * x) + ko * A * np.sin(k * x)).reshape(shape)
    exp_pi = (d2 * A * np.sin(k * x) + ko * B * np.cos(k * x)).reshape(shape)
    np.testing.assert_allclose(ds[0], np.broadcast_to(exp_phi, ds[0].shape), rtol=0, atol=1e-13)
    np.testing.assert_allclose(ds[1], np.broadcast_to(exp_pi, ds[1].shape), rtol=0, atol=1e-13)


def homogeneous(n, Pi0, H0=1.0):
    """chi = alpha = 1, K = -3 H0, fluid at rest with E_fluid = 3 H0^2 / 8 pi - Pi0^2 / 2."""
    u = flat(n, 3 * H0 * H0 / (8 * np.pi) - 0.5 * Pi0 * Pi0)
    u[7] = -3.0 * H0
    sc = np.zeros((2,) + u.shape[1:])
    sc[0] = 0.3
    sc[1] = Pi0
    return u, sc


def test_homogeneous_scalar_decay_and_friedmann(orc):
    n = (8, 8, 8)
    Pi0, T = 0.2, 0.4
    errs_inv, errs_H = [], []
    for nsteps in (4, 8, 16):
        s = orc.Setup(n=n, L=(8.0, 8.0, 8.0), lapse_bg=0)
        u, sc = homogeneous(n, Pi0)
        u, sc, pf = orc.rk4_sc(s, u, sc, 0.0, T / nsteps, nsteps)
        assert pf == 0
        chi, Pi = u[0, 0, 0, 0], sc[1, 0, 0, 0]
        assert np.ptp(u[0]) == 0.0 and np.ptp(sc[1]) == 0.0  # stays homogeneous
        errs_inv.append(abs(Pi * chi ** -1.5 - Pi0))
        errs_H.append(orc.constraints_sc(s, u, sc)[1])
    for e in (errs_inv, errs_H):
        assert e[0] > 1e-12
        assert e[0] / e[1] > 12 and e[1] / e[2] > 12, e


def test_isocurvature_initial_data_constraints(orc):
    L = 8.0
    out = []
    for n in (16, 32):
        s = orc.Setup(n=(n, n, n), L=(L, L, L))
        u, sc = orc.init_fields_sc(s, orc.Init(mu=0.0, sigma=1.6, profile=orc.PGAUSS), 0.15, 1.3)
        assert sc[1].max() == 0.0 and np.abs(sc[0]).max() > 0.1
        norms = orc.constraints_sc(s, u, sc)
        assert norms[3] == 0.0  # fluid at rest and Pi = 0: no momentum anywhere
        out.append(norms[0])
        # without the scalar's energy the same data violate the constraint at O(1)
        assert orc.constraints(s, u)[0] > 30 * norms[0]
    assert out[0] / out[1] > 12.0, out


@pytest.mark.slow
def test_constraint_propagation_with_scalar_field(orc):
    L, T = 8.0, 0.5
    out = []
    for n in (16, 32, 64):
        s = orc.Setup(n=(n, n, n), L=(L, L, L), ko_eps=0.0)
        ini = orc.Init(mu=0.1, sigma=1.6, profile=orc.PGAUSS)
        u0, sc0 = orc.init_fields_sc(s, ini, 0.15, 1.3)  # Pi develops from the field's gradients
        nsteps = n // 4
        u, sc, pf = orc.rk4_sc(s, u0, sc0, 0.0, T / nsteps, nsteps, parallel=True)
        assert pf == 0
        norms = orc.constraints_sc(s, u, sc, parallel=True)
        out.append((norms[0], norms[2]))
    out = np.array(out)
    assert np.all(out[1] / out[2] > 12.0), out
    assert np.all(out[0] / out[1] > 8.0), out


def test_zero_amplitude_equals_plain_path(orc):
    n = (12, 10, 8)
    s = orc.Setup(n=n, L=(3.0, 2.5, 2.0))
    u = fuzz_state(n, seed=2)
    sc = np.zeros((2,) + u.shape[1:])
    du, ds, _ = orc.rhs_sc(s, u, sc)
    r, _ = orc.rhs(s, u)
    # the zero scalar field adds exact zeros to the sources
    assert np.array_equal(du, r) and not ds.any()
    ini = orc.Init(mu=0.2, sigma=1.0)
    u1, sc1 = orc.init_fields_sc(s, ini, 0.0, 1.0)
    assert np.array_equal(u1, orc.init_fields(s, ini)) and not sc1.any()


def test_point_sampled_forms_match_full_grid(orc):
    """The point-sampled right-hand side and RK4 step (used at sizes where the whole grid is
    out of reach) reproduce the full-grid ones bitwise at the sampled points."""
    from inputs import fuzz_scalar, sample_points
    n = (14, 12, 16)
    s = orc.Setup(n=n, L=(3.5, 3.0, 4.0))
    u, sc = fuzz_state(n, seed=13), fuzz_scalar(n, seed=14)
    pts = sample_points(n, 5, seed=2)
    du, ds, _ = orc.rhs_sc(s, u, sc, t=0.3)
    pu, ps = orc.rhs_sc_at_points(s, u, sc, pts, t=0.3)
    assert np.array_equal(pu, du.reshape(25, -1)[:, pts].T) and np.array_equal(ps, ds.reshape(2, -1)[:, pts].T)
    dt = 0.05
    u1, s1, _ = orc.rk4_sc(s, u, sc, 0.3, dt, 1)
    qu, qs = orc.rk4_sc_at_points(s, u, sc, pts, 0.3, dt)
    assert np.allclose(qu, u1.reshape(25, -1)[:, pts].T, rtol=0, atol=1e-13)
    assert np.allclose(qs, s1.reshape(2, -1)[:, pts].T, rtol=0, atol=1e-13)


def _modes(rng, count, mmax=2):
    out = []
    for _ in range(count):
        m = rng.integers(-mmax, mmax + 1, size=3)
        if not m.any():
            m[0] = 1
        out.append((m, rng.uniform(0.5, 1.0), rng.uniform(0, 2 * np.pi)))
    return out


def _analytic(X, L, c0, amp, modes):
    """f = c0 + amp * sum_q a_q sin(2 pi m_q.x / L + ph_q) / sum_q a_q with its exact first and
    second derivatives: (f, df[3], d2f[3][3]) on the coordinate arrays X = (x, y, z)."""
    wsum = sum(a for _, a, _ in modes)
    f = np.full(X[0].shape, c0, dtype=float)
    df = np.zeros((3,) + X[0].shape)
    d2f = np.zeros((3, 3) + X[0].shape)
    for m, a, ph in modes:
        kv = 2 * np.pi * np.asarray(m, dtype=float) / L
        th = kv[0] * X[0] + kv[1] * X[1] + kv[2] * X[2] + ph
        w = amp * a / wsum
        f += w * np.sin(th)
        for i in range(3):
            df[i] += w * kv[i] * np.cos(th)
            for j in range(3):
                d2f[i, j] -= w * kv[i] * kv[j] * np.sin(th)
    return f, df, d2f


def test_wave_operator_is_covariant_laplacian_4th_order(orc):
    """With alpha = 1, beta = 0, K = Pi = 0 and no dissipation, d_t Pi is the covariant Laplacian of
    phi in the physical metric g_ij = gt_ij / chi. Reference: g^ij (d_i d_j phi - Gamma^k_ij d_k phi)
    with the Christoffel symbols of g_ij from exact derivatives of analytic chi, gt_ij, phi (the
    generic metric formula, not the conformal decomposition). The state's evolved connection
    functions are set to zero, unequal to gt^ij Gt^k_ij of this metric: the operator must not
    depend on them, so the error falls at 4th order under grid doubling. (An operator built with
    the evolved Gt^k in place of the metric's contracted connection has an O(1) error here.)"""
    rng = np.random.default_rng(44)
    L = 4.0
    spec = {"chi": (1.0, 0.15, _modes(rng, 2)), "phi": (0.0, 0.3, _modes(rng, 3))}
    gt_spec = []
    for q in range(6):
        diag = q in (0, 3, 5)
        gt_spec.append((1.0 if diag else 0.0, 0.12 if diag else 0.06, _modes(rng, 2)))
    errs = []
    for N in (16, 32, 64):
        s = orc.Setup(n=(N, N, N), L=(L, L, L), ko_eps=0.0, H0=0.0)
        x = -L / 2 + (L / N) * np.arange(N)
        Z, Y, Xx = np.meshgrid(x, x, x, indexing="ij")
        X = (Xx, Y, Z)
        chi, dchi, _ = _analytic(X, L, *spec["chi"])
        phi, dphi, d2phi = _analytic(X, L, *spec["phi"])
        gt = np.zeros((3, 3) + chi.shape)
        dgt = np.zeros((3, 3, 3) + chi.shape)
        sym = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
        u = np.zeros((25,) + chi.shape)
        u[0] = chi
        for q, (i, j) in enumerate(sym):
            f, df, _ = _analytic(X, L, *gt_spec[q])
            gt[i, j] = gt[j, i] = f
            dgt[i, j] = dgt[j, i] = df
            u[1 + q] = f
        u[17] = 1.0
        u[21] = 0.1  # fluid at rest: it does not enter d_t Pi
        # physical metric, its inverse and derivatives
        g = gt / chi
        dg = dgt / chi - gt[:, :, None] * dchi[None, None] / chi ** 2  # dg[i, j, k] = d_k g_ij
        gi = np.moveaxis(np.linalg.inv(np.moveaxis(g, (0, 1), (-2, -1))), (-2, -1), (0, 1))
        lap = np.zeros_like(chi)
        for i in range(3):
            for j in range(3):
                gam = np.zeros_like(chi)  # g^ij Gamma^k_ij d_k phi for this (i, j)
                for k in range(3):
                    for l in range(3):
                        gam += 0.5 * gi[k, l] * (dg[l, j, i] + dg[l, i, j] - dg[i, j, l]) * dphi[k]
                lap += gi[i, j] * (d2phi[i, j] - gam)
        sc = np.zeros((2,) + chi.shape)
        sc[0] = phi
        _, ds, _ = orc.rhs_sc(s, u, sc, parallel=True)
        errs.append(np.abs(ds[1] - lap).max() / np.abs(lap).max())
    assert 13.0 < errs[1] / errs[2] < 19.0 and errs[0] / errs[1] > 10.0, errs
    assert errs[2] < 1e-4, errs
