"""Physics pins of the oracle's whole discrete evolution (no GPU).

* flat space stays exactly flat (right-hand side identically zero);
* the homogeneous radiation universe follows the Friedmann closed form
  a(t) = (1 + 2 H0 t)^(1/2), with 4th-order convergence in dt;
* the initial data of the paper's initial-data paragraph satisfy the
  Hamiltonian constraint up to the 4th-order truncation error of the discrete
  Ricci scalar (ratio 16 under grid doubling), and the momentum constraint
  exactly;
* a centred perturbation stays reflection and permutation symmetric;
* constraint violations and the connection-function mismatch converge to zero
  at 4th order under evolution (a wrong coefficient anywhere breaks this).
"""
import math

import numpy as np
import pytest

from tests.inputs import fuzz_state


def test_minkowski_exactly_static(orc):
    s = orc.Setup(n=(8, 10, 12), L=(4.0, 5.0, 6.0), H0=0.0, ko_eps=0.1)
    u = orc.init_fields(s, orc.Init(mu=0.0, sigma=1.0))
    # flat space, vacuum
    assert np.all(u[orc.CHI] == 1.0) and np.all(u[orc.TRK] == 0.0) and np.all(u[orc.ET] == 0.0)
    r, _ = orc.rhs(s, u, t=0.0)
    assert np.all(r == 0.0)
    v, _ = orc.rk4(s, u, 0.0, 0.1, 100)
    assert np.array_equal(u, v)


def test_flrw_closed_form_4th_order(orc):
    s = orc.Setup(n=(8, 8, 8), L=(10.0, 10.0, 10.0), H0=1.0)
    u0 = orc.init_fields(s, orc.Init(mu=0.0, sigma=1.0))
    rho0 = 3.0 / (8.0 * math.pi)
    assert np.allclose(u0[orc.ET], rho0, rtol=1e-15)
    T = 2.0
    errs = []
    for nsteps in (10, 20, 40):
        u, pf = orc.rk4(s, u0, 0.0, T / nsteps, nsteps)
        assert pf == 0
        a2 = 1.0 + 2.0 * T
        exact = {orc.CHI: 1.0 / a2, orc.TRK: -3.0 / a2, orc.ET: rho0 / math.sqrt(a2), orc.ALP: 1.0}
        e = max(np.abs(u[f] - v).max() / abs(v) for f, v in exact.items())
        # homogeneous: every point equal, and nothing else evolves
        for f in range(25):
            assert np.ptp(u[f]) == 0.0
        # only round-off of the trace-free projection feeds the traceless curvature
        assert np.abs(u[orc.AT:orc.AT + 6]).max() < 1e-15 and np.abs(u[orc.BET:orc.BET + 3]).max() < 1e-15
        errs.append(e)
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 12.0 < r1 < 20.0 and 14.0 < r2 < 18.0, errs
    assert errs[2] < 2e-6  # dt = 0.05 over a factor-5 expansion


def test_hamiltonian_constraint_initial_data_4th_order(orc):
    # smooth periodic profile so that no kink at the box faces spoils the order
    H = []
    for n in (16, 32, 64):
        s = orc.Setup(n=(n, n, n), L=(10.0, 10.0, 10.0))
        u = orc.init_fields(s, orc.Init(mu=0.3, sigma=1.5, profile=orc.PGAUSS))
        norms = orc.constraints(s, u, parallel=True)
        H.append(norms[0])
        assert norms[3] == 0.0  # momentum constraint exactly zero at t = 0
        assert norms[5] == 0.0
    r1, r2 = H[0] / H[1], H[1] / H[2]
    assert 12.0 < r2 < 20.0 and r1 > 8.0, H


def test_sine_profile_constraint_order(orc):
    H = []
    for n in (16, 32, 64):
        s = orc.Setup(n=(n, 8, 8), L=(10.0, 10.0, 10.0))
        u = orc.init_fields(s, orc.Init(mu=0.05, profile=orc.SINE))
        H.append(orc.constraints(s, u)[1])
    assert 14.0 < H[1] / H[2] < 18.0, H


def test_gaussian_initial_data_values(orc):
    s = orc.Setup(n=(16, 16, 16), L=(10.0, 10.0, 10.0))
    mu, sigma = 0.1, 1.0
    u = orc.init_fields(s, orc.Init(mu=mu, sigma=sigma))
    c = 8
    # centre: zeta = mu, R = -e^{-2 mu}(4 * (-3 mu / sigma^2)) = 12 mu e^{-2mu} / sigma^2
    assert u[orc.CHI, c, c, c] == pytest.approx(math.exp(-2 * mu), rel=1e-15)
    R0 = 12 * mu * math.exp(-2 * mu) / sigma ** 2
    E0 = 3.0 / (8 * math.pi) + R0 / (16 * math.pi)
    assert u[orc.ET, c, c, c] == pytest.approx(E0 / math.exp(-3 * mu), rel=1e-14)
    assert np.all(u[orc.TRK] == -3.0) and np.all(u[orc.ALP] == 1.0)
    # literal density mode: uniform E = 3 H0^2 / 8 pi
    v = orc.init_fields(s, orc.Init(mu=mu, sigma=sigma, density_mode=orc.LITERAL))
    assert np.allclose(v[orc.ET] * v[orc.CHI] ** 1.5, 3 / (8 * math.pi), rtol=1e-15)


def test_white_noise_multiplicative(orc):
    s = orc.Setup(n=(16, 16, 16), L=(10.0, 10.0, 10.0))
    clean = orc.init_fields(s, orc.Init(mu=0.1, sigma=1.0, noise_amp=0.0))
    noisy = orc.init_fields(s, orc.Init(mu=0.1, sigma=1.0, noise_amp=1e-6, seed=2606))
    xi = (noisy[orc.ET] / clean[orc.ET] - 1.0) / 1e-6
    assert np.abs(xi).max() <= 1.0 + 1e-6
    assert abs(xi.mean()) < 0.05 and 0.25 < xi.var() < 0.42  # uniform on [-1, 1): var 1/3
    # point p uses counter p: xi_p = 2 (splitmix64(seed, p) >> 11) 2^-53 - 1
    for p in (0, 1, 777, 4095):
        k, j, i = np.unravel_index(p, (16, 16, 16))
        ref = 2.0 * (orc.splitmix64(2606, p) >> 11) * 2.0 ** -53 - 1.0
        assert xi[k, j, i] == pytest.approx(ref, abs=2e-9)


@pytest.mark.slow
def test_centred_gaussian_symmetric_under_evolution(orc):
    n = 16
    s = orc.Setup(n=(n, n, n), L=(8.0, 8.0, 8.0))
    u0 = orc.init_fields(s, orc.Init(mu=0.3, sigma=1.2))
    u, _ = orc.rk4(s, u0, 0.0, 0.25 * s.h[0], 3, parallel=True)
    # the fields that become non-zero only through evolution really did
    assert np.abs(u[orc.AT]).max() > 1e-6 and np.abs(u[orc.GAM]).max() > 1e-8
    assert np.abs(u[orc.ST]).max() > 1e-8
    scale = np.abs(u).reshape(25, -1).max(axis=1) + 1e-300
    idx = (-np.arange(n)) % n  # x -> -x about the centre point n/2
    # parity under x -> -x of each field (tensor components with one x index are odd)
    par_x = np.ones(25)
    for f in (orc.GT + 1, orc.GT + 2, orc.AT + 1, orc.AT + 2, orc.GAM, orc.BET, orc.ST):
        par_x[f] = -1
    refl = u[:, :, :, idx] * par_x[:, None, None, None]
    err = np.abs(refl - u).reshape(25, -1).max(axis=1) / scale
    assert err.max() < 1e-12, err
    # permutation x <-> y: components swap
    perm = list(range(25))
    for a, b in [(orc.GT + 0, orc.GT + 3), (orc.GT + 2, orc.GT + 4), (orc.AT + 0, orc.AT + 3),
                 (orc.AT + 2, orc.AT + 4), (orc.GAM, orc.GAM + 1), (orc.BET, orc.BET + 1), (orc.ST, orc.ST + 1)]:
        perm[a], perm[b] = b, a
    sw = np.transpose(u[perm], (0, 1, 3, 2))
    err = np.abs(sw - u).reshape(25, -1).max(axis=1) / scale
    assert err.max() < 1e-12, err


@pytest.mark.slow
def test_constraint_propagation_converges_4th_order(orc):
    # fixed final time, PGAUSS (smooth and periodic), grids 16^3 -> 32^3 -> 64^3
    L, T = 8.0, 0.5
    out = []
    for n in (16, 32, 64):
        s = orc.Setup(n=(n, n, n), L=(L, L, L), ko_eps=0.0)
        u0 = orc.init_fields(s, orc.Init(mu=0.2, sigma=1.6, profile=orc.PGAUSS))
        nsteps = n // 4
        dt = T / nsteps
        u, pf = orc.rk4(s, u0, 0.0, dt, nsteps, parallel=True)
        assert pf == 0
        norms = orc.constraints(s, u, parallel=True)
        g = orc.gamma_constraint(s, u)
        out.append((norms[0], norms[2], g[0]))
    out = np.array(out)
    ratios = out[1] / out[2]
    assert np.all(ratios > 12.0), (out, ratios)
    assert np.all(out[0] / out[1] > 8.0), out


def test_linear_sound_wave_travels_at_sqrt_w(orc):
    """Linear perturbation theory of the fluid: on a flat background with a tiny fluid
    density (so gravity's back-reaction is negligible) a small standing wave
    Et = E0 + A cos(k x) obeys d_t dE = -d_x S, d_t S = -w d_x dE, i.e. dE = A cos(k x)
    cos(c k t) with c = sqrt(w); the run reproduces it to the discretisation error,
    which falls at 4th order (the paper's first example compares a single-mode evolution
    with linear perturbation theory; this is that comparison for the fluid sector)."""
    w, E0, A, L, T = 1.0 / 3.0, 1e-7, 1e-11, 2.0, 0.6
    errs = []
    for n in (16, 32):
        s = orc.Setup(n=(n, 8, 8), L=(L, L * 8 / n, L * 8 / n), w=w, ko_eps=0.0, lapse_bg=0, evolve_shift=0)
        x = np.arange(n) * (L / n) - L / 2
        k = 2 * np.pi / L
        u = np.zeros(s.shape)
        u[0] = u[1] = u[4] = u[6] = u[17] = 1.0
        u[21] = (E0 + A * np.cos(k * x))[None, None, :]
        nsteps = n
        u, pf = orc.rk4(s, u, 0.0, T / nsteps, nsteps)
        assert pf == 0
        exact = A * np.cos(k * x) * np.cos(np.sqrt(w) * k * T)
        # the uniform background drifts (E0 with K = 0 is not a Friedmann state): compare the
        # zero-mean part, which is the wave
        dE = u[21, 4, 4, :] - u[21, 4, 4, :].mean()
        errs.append(np.abs(dE - exact).max() / A)
    assert errs[0] < 2e-3 and errs[0] / errs[1] > 10, errs
