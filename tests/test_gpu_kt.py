"""GPU parity of the Kurganov-Tadmor fluid scheme (fluid_scheme = 1) against the
oracle, through the C ABI: the interface-flux pre-pass (8 x 8 x 4 bricks with
LDS-held interface fluxes) and the stage kernel taking its divergence.

Metric as in test_gpu_parity (per-field max error over max |oracle|, floor 1e-3).
Inputs: the smooth fuzz state, and a rough one (independent per-point noise on
the fluid fields) under which the minmod limiter takes every branch.
"""
import numpy as np
import pytest
import torch

from tests.inputs import fuzz_state, sample_points
from tests.test_gpu_parity import err_fields, to_dev

pytestmark = pytest.mark.gpu

KT = dict(fluid_scheme=1)


@pytest.fixture(scope="module")
def P():
    import paper_2606_02053_amd as P
    assert torch.cuda.is_available()
    return P


def rough_state(n, seed):
    u = fuzz_state(n, seed=seed)
    rng = np.random.default_rng(seed + 1000)
    u[21] *= 1.0 + 0.3 * rng.uniform(-1, 1, size=u[21].shape)
    for c in range(3):
        u[22 + c] += 0.02 * rng.uniform(-1, 1, size=u[21].shape)
    return u


def mk(P, orc, n, L, **kw):
    kw = {**KT, **kw}
    return orc.Setup(n=n, L=L, **kw), P.Solver(n, L, P.make_params(**kw))


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("rough", [False, True])
@pytest.mark.parametrize("n,L", [((20, 12, 10), (4.0, 2.5, 2.0)), ((32, 32, 32), (10.0, 10.0, 10.0))])
def test_kt_rhs(P, orc, n, L, rough, variant):
    # 20 x 12 x 10: partial pre-pass bricks along every axis and partial stage bricks
    s, sol = mk(P, orc, n, L)
    sol.params.variant = variant
    u = rough_state(n, 31) if rough else fuzz_state(n, seed=31)
    sol.set_state(to_dev(u))
    g = sol.rhs(t=0.2).cpu().numpy()
    r, _ = orc.rhs(s, u, t=0.2, parallel=True)
    e, per = err_fields(g, r)
    assert e < 1e-11, per
    # the schemes differ in the fluid equations only
    s0 = orc.Setup(n=n, L=L)
    r0, _ = orc.rhs(s0, u, t=0.2, parallel=True)
    assert np.array_equal(r0[:21], r[:21])
    assert np.abs(r0[21:] - r[21:]).max() > 1e-6


@pytest.mark.parametrize("n,L", [((20, 12, 10), (4.0, 2.5, 2.0)), ((8, 8, 8), (2.0, 2.0, 2.0))])
def test_kt_divergence_entry_point(P, orc, n, L):
    """The pre-pass alone (cosmos_kt_divergence) against the oracle's flux divergence."""
    s = orc.Setup(n=n, L=L, **KT)
    u = rough_state(n, 17)
    g = P.make_grid(n, L)
    div = torch.full((4,) + tuple(reversed(n)), float("nan"), dtype=torch.float64, device="cuda")
    P.cosmos_kt_divergence(g, P.make_params(**KT), to_dev(u), div)
    ref = orc.kt_divergence(s, u)
    got = div.cpu().numpy()
    assert np.isfinite(got).all()
    for q in range(4):
        assert np.abs(got[q] - ref[q]).max() < 1e-11 * max(np.abs(ref[q]).max(), 1e-3), q


def test_kt_rhs_options(P, orc):
    n, L = (12, 10, 14), (2.5, 2.0, 3.0)
    u = rough_state(n, 7)
    for kw in (dict(evolve_shift=0), dict(ko_eps=0.0), dict(w=0.2, eta=2.0, H0=0.5)):
        s, sol = mk(P, orc, n, L, **kw)
        sol.set_state(to_dev(u))
        g = sol.rhs(t=0.2).cpu().numpy()
        r, _ = orc.rhs(s, u, t=0.2)
        e, per = err_fields(g, r)
        assert e < 1e-11, (kw, per)


def test_kt_rk4_steps(P, orc):
    n, L = (16, 12, 14), (3.0, 2.5, 2.8)
    s, sol = mk(P, orc, n, L)
    u = rough_state(n, 5)
    sol.set_state(to_dev(u), t=0.1)
    dt = 0.25 * min(s.h)
    sol.step(dt)
    r1, _ = orc.rk4(s, u, 0.1, dt, 1, parallel=True)
    e1, per = err_fields(sol.u.cpu().numpy(), r1)
    assert e1 < 1e-11, per
    sol.run(9, dt)
    r10, _ = orc.rk4(s, r1, 0.1 + dt, dt, 9, parallel=True)
    e10, per = err_fields(sol.u.cpu().numpy(), r10)
    assert e10 < 1e-10, per


def test_kt_c1_hundred_steps(P, orc):
    """32^3 box of side 10, Gaussian zeta (mu 0.1, sigma 1), 1e-6 noise on E: 100 RK4 steps."""
    n, L = (32, 32, 32), (10.0, 10.0, 10.0)
    s, sol = mk(P, orc, n, L)
    ini = dict(mu=0.1, sigma=1.0, noise_amp=1e-6, seed=2606)
    sol.init(**ini)
    u0 = orc.init_fields(s, orc.Init(**ini))
    dt = 0.25 * s.h[0]
    sol.run(100, dt)
    r100, _ = orc.rk4(s, u0, 0.0, dt, 100, parallel=True)
    e100, per = err_fields(sol.u.cpu().numpy(), r100)
    print(f"KT C1 parity after 100 steps: {e100:.3e}")
    assert e100 < 1e-9, per
    st = sol.status()
    assert st["steps"] == 100 and st["nonfinite"] == 0 and st["prim_fail"] == 0


def test_kt_tile_invariance_bitwise(P, orc):
    from paper_2606_02053_amd import autotune
    n, L = (20, 12, 18), (4.0, 2.5, 3.5)
    s, sol = mk(P, orc, n, L)
    u = rough_state(n, 12)
    sol.set_state(to_dev(u))
    r, _ = orc.rhs(s, u, t=0.1)
    first = {}
    for kv, tile, order in autotune.CANDIDATES:
        p = autotune.with_tile(sol.params, kv, tile, order)
        assert p.fluid_scheme == 1
        out = torch.empty_like(sol.u)
        P.cosmos_rhs(sol.grid, p, 0.1, sol.u, out, sol.ws)
        if kv not in first:
            first[kv] = out
            assert err_fields(out.cpu().numpy(), r)[0] < 1e-11, kv
        assert torch.equal(out, first[kv]), (kv, tile, order)


def test_kt_conservation_flat_background(P, orc):
    """Flat geometry, rough fluid on 64^3: every fluid source term vanishes, so the
    fluid right-hand side sums to zero over the periodic grid (any size)."""
    n, L = (64, 64, 64), (8.0, 8.0, 8.0)
    u = np.zeros((25, 64, 64, 64))
    u[0] = u[1] = u[4] = u[6] = u[17] = 1.0
    rough = rough_state(n, 44)
    u[21:] = rough[21:]
    s, sol = mk(P, orc, n, L)
    sol.set_state(to_dev(u))
    g = sol.rhs(t=0.0).double()
    for q in range(4):
        tot = float(g[21 + q].sum())
        scale = float(g[21 + q].abs().sum())
        assert scale > 1.0 and abs(tot) < 1e-12 * scale, (q, tot, scale)


def test_kt_bench_configuration_sampled(P, orc):
    """256^3, L = 16, Gaussian zeta mu = 0.6, sigma = 2 in the default launch configuration:
    one right-hand side and one RK4 step at sampled points."""
    n, L = (256, 256, 256), (16.0, 16.0, 16.0)
    s, sol = mk(P, orc, n, L)
    ini = dict(mu=0.6, sigma=2.0)
    sol.init(**ini)
    pts = sample_points(n, 16, seed=3)
    idx = torch.from_numpy(pts).cuda()
    u0 = orc.init_fields(s, orc.Init(**ini))
    rhs = sol.rhs(t=0.0).reshape(25, -1)[:, idx].T.cpu().numpy()
    rr = orc.rhs_at_points(s, u0, pts, t=0.0)
    scale = np.maximum(np.abs(rr).max(axis=0), 1e-3)
    assert (np.abs(rhs - rr).max(axis=0) / scale).max() < 1e-11
    dt = 0.25 * s.h[0]
    sol.step(dt)
    g1 = sol.u.reshape(25, -1)[:, idx[:6]].T.cpu().numpy()
    r1 = orc.rk4_at_points(s, u0, pts[:6], 0.0, dt)
    scale = np.maximum(np.abs(r1).max(axis=0), 1e-3)
    assert (np.abs(g1 - r1).max(axis=0) / scale).max() < 1e-11
