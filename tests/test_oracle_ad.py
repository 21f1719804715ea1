"""Pins of the oracle's derivatives (no GPU).

The oracle's discrete adjoint (reverse mode on a tape) and its tangents
(forward-mode dual numbers) are two independent derivative propagations of
the same discrete map. They are pinned against each other by the dot-product
identity <lam, J v> = <J^T lam, v>, and the tangents against central finite
differences of the plain double evaluation.
"""
import numpy as np
import pytest

from tests.inputs import fuzz_direction, fuzz_state


@pytest.fixture(scope="module")
def case(orc):
    s = orc.Setup(n=(8, 8, 10), L=(2.4, 2.4, 3.0))
    u = fuzz_state(s.n, seed=21)
    v = fuzz_direction(s.n, seed=22)
    lam = fuzz_direction(s.n, seed=23)
    return s, u, v, lam


def test_jvp_matches_finite_differences(orc, case):
    s, u, v, _ = case
    dt = 0.25 * min(s.h)
    _, Jv = orc.jvp(s, u, v, "step", t=0.2, dt=dt)
    eps = 1e-6
    up, _ = orc.rk4(s, u + eps * v, 0.2, dt, 1)
    um, _ = orc.rk4(s, u - eps * v, 0.2, dt, 1)
    fd = (up - um) / (2 * eps)
    assert np.abs(Jv - fd).max() < 1e-7 * np.abs(Jv).max()
    # primal of the dual evaluation equals the double evaluation
    fu, _ = orc.jvp(s, u, v, "step", t=0.2, dt=dt)
    ref, _ = orc.rk4(s, u, 0.2, dt, 1)
    assert np.array_equal(fu, ref)


@pytest.mark.parametrize("what", ["rhs", "step"])
def test_adjoint_dot_product(orc, case, what):
    s, u, v, lam = case
    dt = 0.25 * min(s.h)
    _, Jv = orc.jvp(s, u, v, what, t=0.1, dt=dt)
    JTl = orc.vjp(s, u, lam, what, t=0.1, dt=dt)
    a = np.sum(lam * Jv)
    b = np.sum(JTl * v)
    assert a == pytest.approx(b, rel=1e-12)


def test_adjoint_columns_against_tangents(orc, case):
    # a few exact columns of J^T: J^T e_p computed by reverse mode equals row p of J
    s, u, _, _ = case
    dt = 0.25 * min(s.h)
    N = u.size
    rng = np.random.default_rng(5)
    for p in rng.integers(0, N, size=3):
        e = np.zeros(N)
        e[p] = 1.0
        row = orc.vjp(s, u, e.reshape(u.shape), "step", t=0.0, dt=dt).ravel()
        for q in rng.integers(0, N, size=4):
            eq = np.zeros(N)
            eq[q] = 1.0
            _, Jq = orc.jvp(s, u, eq.reshape(u.shape), "step", t=0.0, dt=dt)
            assert row[q] == pytest.approx(Jq.ravel()[p], rel=1e-12, abs=1e-15)


def test_init_tangent_matches_finite_differences(orc):
    s = orc.Setup(n=(12, 12, 12), L=(12.0, 12.0, 12.0))
    ini = orc.Init(mu=0.55, sigma=1.2)
    for which in (0, 1):
        du = orc.init_tangent(s, ini, which)
        h = 1e-6
        p = orc.Init(mu=ini.mu + (h if which == 0 else 0), sigma=ini.sigma + (h if which == 1 else 0))
        m = orc.Init(mu=ini.mu - (h if which == 0 else 0), sigma=ini.sigma - (h if which == 1 else 0))
        fd = (orc.init_fields(s, p) - orc.init_fields(s, m)) / (2 * h)
        assert np.abs(du - fd).max() < 1e-7 * np.abs(du).max()
