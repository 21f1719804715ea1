"""Pins of the oracle's Kurganov-Tadmor fluid scheme (fluid_scheme = 1) against
what physics and the scheme's definition fix independently of its code:

* characteristic speeds: relativistic velocity addition (v +- cs) / (1 +- v cs)
  for flow along the axis, the light cone for w = 1 at any velocity, and the
  lapse / shift / conformal-factor scaling at rest;
* consistency of the numerical flux, Fh(u, u) = F(u);
* closed forms on a flat background with the fluid at rest, where the scheme
  reduces to the textbook linear case (flux of St_x = w Et, speed sqrt(w)):
  a one-point spike (all minmod slopes vanish: the local Lax-Friedrichs limit)
  and a quadratic profile (one-sided minmod slopes: interface values such that
  the divergence is exact);
* discrete conservation (the fluid part of the right-hand side sums to zero on a
  flat periodic grid for any fluid data);
* equivariance of the whole right-hand side under the reflection x -> -x;
* second-order consistency with the centred 4th-order scheme for smooth data.
"""
import numpy as np
import pytest

from inputs import fuzz_state

W = 1.0 / 3.0
ET, ST = 21, 22


def flat_rest(n, E):
    """Flat geometry (chi = alpha = 1, gt = delta, K = At = Gt = beta = 0), fluid at rest, Et = E."""
    u = np.zeros((25,) + tuple(reversed(n)))
    u[0] = 1.0
    u[1] = u[4] = u[6] = 1.0
    u[17] = 1.0
    u[ET] = E
    return u


def point(chi=1.0, alpha=1.0, beta=(0.0, 0.0, 0.0), E=1.0, S=(0.0, 0.0, 0.0)):
    u = np.zeros(25)
    u[0] = chi
    u[1] = u[4] = u[6] = 1.0
    u[17] = alpha
    u[18:21] = beta
    c32 = chi ** 1.5
    u[ET] = E / c32
    u[ST:ST + 3] = np.asarray(S) / c32
    return u


def moving(v, axis=0, rho=1.0, w=W):
    """Flat-space fluid with rest density rho moving with speed v along `axis`."""
    Wl2 = 1.0 / (1.0 - v * v)
    X = (1.0 + w) * rho * Wl2
    S = [0.0, 0.0, 0.0]
    S[axis] = X * v
    return point(E=X - w * rho, S=S)


@pytest.mark.parametrize("v", [0.0, 0.3, -0.55, 0.9])
def test_speeds_collinear_velocity_addition(orc, v):
    s = orc.Setup()
    cs = np.sqrt(W)
    lm, lp = orc.fluid_speeds(s, moving(v, 0), 0)
    assert lp == pytest.approx((v + cs) / (1 + v * cs), abs=1e-13)
    assert lm == pytest.approx((v - cs) / (1 - v * cs), abs=1e-13)


@pytest.mark.parametrize("v,axis,probe", [(0.4, 0, 0), (0.7, 1, 0), (-0.6, 2, 2), (0.8, 0, 1)])
def test_speeds_light_cone_for_stiff_fluid(orc, v, axis, probe):
    # w = 1: sound moves at the speed of light whatever the flow velocity
    s = orc.Setup(w=1.0)
    lm, lp = orc.fluid_speeds(s, moving(v, axis, w=1.0), probe)
    assert lp == pytest.approx(1.0, abs=1e-13) and lm == pytest.approx(-1.0, abs=1e-13)


def test_speeds_gauge_and_conformal_scaling_at_rest(orc):
    s = orc.Setup()
    chi, alpha, beta = 0.7, 1.3, (0.2, -0.1, 0.05)
    for a in range(3):
        lm, lp = orc.fluid_speeds(s, point(chi=chi, alpha=alpha, beta=beta, E=2.0), a)
        # gamma^aa = chi for gt = delta
        assert lp == pytest.approx(alpha * np.sqrt(W * chi) - beta[a], abs=1e-13)
        assert lm == pytest.approx(-alpha * np.sqrt(W * chi) - beta[a], abs=1e-13)


def test_numerical_flux_consistency(orc):
    s = orc.Setup()
    u = fuzz_state((8, 8, 8), seed=5)[:, 3, 2, 1]
    for a in range(3):
        np.testing.assert_allclose(orc.kt_flux(s, u, u, a), orc.flux_point(s, u)[4 * a:4 * a + 4], rtol=0,
                                   atol=1e-15)


def fluid_rhs_1d(orc, E, ko_eps=0.1):
    n = (len(E), 8, 8)
    s = orc.Setup(n=n, L=(float(len(E)), 8.0, 8.0), fluid_scheme=1, ko_eps=ko_eps)  # h = 1
    Eg = np.broadcast_to(np.asarray(E, dtype=np.float64)[None, None, :], (8, 8, len(E)))
    r, _ = orc.rhs(s, flat_rest(n, Eg))
    return r[ET, 3, 4, :], r[ST, 3, 4, :], r[ST + 1, 3, 4, :], r[ST + 2, 3, 4, :]


def test_spike_reduces_to_local_lax_friedrichs(orc):
    # E = 1 except E_k = 2: every minmod slope is 0, so the interface states are the
    # point values and Fh = average flux - sqrt(w)/2 jump; then (h = 1)
    #   dE_k/dt = -sqrt(w),  dE_{k+-1}/dt = sqrt(w)/2,  dSx_{k+-1}/dt = -+ w/2, everything else 0
    E = np.ones(16)
    k = 7
    E[k] = 2.0
    dE, dSx, dSy, dSz = fluid_rhs_1d(orc, E)
    expE = np.zeros(16)
    expE[k] = -np.sqrt(W)
    expE[k - 1] = expE[k + 1] = 0.5 * np.sqrt(W)
    expS = np.zeros(16)
    expS[k - 1], expS[k + 1] = -0.5 * W, 0.5 * W
    np.testing.assert_allclose(dE, expE, rtol=0, atol=1e-14)
    np.testing.assert_allclose(dSx, expS, rtol=0, atol=1e-14)
    assert np.abs(dSy).max() < 1e-14 and np.abs(dSz).max() < 1e-14


def test_quadratic_profile_divergence_is_exact(orc):
    # E_i = A + B (i - i0)^2 on i0 .. i0+M (increasing), then back down. Inside, the
    # minmod slopes are the backward differences, the interface jump is q_R - q_L = B
    # at every interface (the dissipation term cancels in the divergence) and the
    # interface average is A + B (j^2 + j), j = i - i0; so
    #   dE/dt = 0 and dSx/dt = -w * 2 B j = -w dE/dx exactly.
    n, i0, M, A, B = 24, 2, 14, 1.0, 0.01
    E = np.empty(n)
    for i in range(n):
        if i0 <= i <= i0 + M:
            E[i] = A + B * (i - i0) ** 2
        else:  # decreasing stretch closing the period
            frac = (i - (i0 + M)) % n / (n - M)
            E[i] = A + B * M * M * (1.0 - frac)
    dE, dSx, _, _ = fluid_rhs_1d(orc, E)
    for i in range(i0 + 2, i0 + M - 1):
        j = i - i0
        assert dE[i] == pytest.approx(0.0, abs=1e-14), i
        assert dSx[i] == pytest.approx(-W * 2.0 * B * j, abs=1e-14), i


def test_conservation_on_flat_background(orc):
    # flat geometry: every fluid source term vanishes and the KT divergence telescopes
    n = (16, 8, 12)
    u = flat_rest(n, 0.0)
    fz = fuzz_state(n, seed=11, kmax=3)
    rng = np.random.default_rng(3)
    u[ET] = fz[ET] * (1.0 + 0.3 * rng.uniform(-1, 1, size=fz[ET].shape))  # rough: many limiter branches
    for c in range(3):
        u[ST + c] = fz[ST + c] + 0.02 * rng.uniform(-1, 1, size=fz[ET].shape)
    s = orc.Setup(n=n, L=(8.0, 4.0, 6.0), fluid_scheme=1)
    r, _ = orc.rhs(s, u)
    for q in range(4):
        tot = r[ET + q].sum()
        scale = np.abs(r[ET + q]).sum()
        assert scale > 1e-3
        assert abs(tot) < 1e-13 * scale, (q, tot, scale)


def test_divergence_function_matches_flat_rhs(orc):
    # on a flat background the fluid right-hand side is minus the flux divergence alone
    n = (12, 8, 10)
    u = flat_rest(n, 0.0)
    fz = fuzz_state(n, seed=4)
    rng = np.random.default_rng(9)
    u[ET] = fz[ET] * (1.0 + 0.3 * rng.uniform(-1, 1, size=fz[ET].shape))
    for c in range(3):
        u[ST + c] = fz[ST + c] + 0.02 * rng.uniform(-1, 1, size=fz[ET].shape)
    s = orc.Setup(n=n, L=(3.0, 2.0, 2.5), fluid_scheme=1)
    r, _ = orc.rhs(s, u)
    assert np.array_equal(orc.kt_divergence(s, u), -r[ET:])


SIGN = np.ones(25)
for f in (2, 3, 9, 10, 14, 18, 22):  # odd in x: gt_xy, gt_xz, At_xy, At_xz, Gt^x, beta^x, St_x
    SIGN[f] = -1.0


def mirror_x(u):
    m = np.roll(u[..., ::-1], 1, axis=-1)  # i -> (n - i) mod n
    return SIGN[:, None, None, None] * m


@pytest.mark.parametrize("rough", [False, True])
def test_rhs_reflection_equivariance(orc, rough):
    n = (12, 8, 8)
    u = fuzz_state(n, seed=21)
    if rough:
        rng = np.random.default_rng(8)
        u[ET] *= 1.0 + 0.3 * rng.uniform(-1, 1, size=u[ET].shape)
        u[ST] += 0.02 * rng.uniform(-1, 1, size=u[ET].shape)
    s = orc.Setup(n=n, L=(6.0, 4.0, 4.0), fluid_scheme=1)
    r, _ = orc.rhs(s, u)
    rm, _ = orc.rhs(s, mirror_x(u))
    np.testing.assert_allclose(rm, mirror_x(r), rtol=0, atol=1e-11 * np.abs(r).max())


def test_second_order_consistency_with_centred_scheme(orc):
    # smooth 1D moving fluid on a flat background: the KT divergence approaches the
    # centred 4th-order one at second order (L1 over the grid)
    errs = []
    for n in (32, 64, 128):
        x = np.arange(n) / n
        E = 1.0 + 0.3 * np.sin(2 * np.pi * x) + 0.1 * np.cos(4 * np.pi * x)
        Sx = 0.2 * np.sin(2 * np.pi * x + 0.4)
        u = flat_rest((n, 8, 8), np.broadcast_to(E[None, None, :], (8, 8, n)))
        u[ST] = np.broadcast_to(Sx[None, None, :], (8, 8, n))
        rs = []
        for scheme in (0, 1):
            s = orc.Setup(n=(n, 8, 8), L=(1.0, 1.0, 1.0), fluid_scheme=scheme, ko_eps=0.0)
            r, _ = orc.rhs(s, u)
            rs.append(r[ET:ET + 2, 3, 4, :])
        errs.append(np.abs(rs[1] - rs[0]).mean())
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 1.7, (errs, rates)


def test_invalid_fluid_scheme_rejected(orc):
    s = orc.Setup(n=(8, 8, 8), fluid_scheme=2)
    with pytest.raises(ValueError):
        orc.rhs(s, fuzz_state((8, 8, 8), seed=1))


def test_stored_op_counts_current(orc):
    """The operation counts bench.py reads are the oracle's current counts."""
    import json
    import os
    from tests.golden.make_golden import op_counts
    path = os.path.join(os.path.dirname(__file__), "golden", "op_counts.json")
    with open(path) as f:
        assert json.load(f) == op_counts()
