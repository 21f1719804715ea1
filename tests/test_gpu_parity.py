"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Metric (per field f): ||gpu_f - oracle_f||_inf / max(||oracle_f||_inf, 1e-3),
maximised over the 25 fields; the floor covers fields that are identically
zero (shift, traceless curvature, connection functions, fluid momentum at
t = 0). Bars: 1e-11 for one right-hand side and one RK4 step, 1e-9 after 100
steps. Integer outputs (status counters, argmin) are compared exactly.
"""
import math

import numpy as np
import pytest
import torch

from tests.inputs import fuzz_state, sample_points

pytestmark = pytest.mark.gpu


def err_fields(gpu, ref):
    gpu = np.asarray(gpu).reshape(25, -1)
    ref = np.asarray(ref).reshape(25, -1)
    d = np.abs(gpu - ref).max(axis=1)
    s = np.maximum(np.abs(ref).max(axis=1), 1e-3)
    return (d / s).max(), d / s


@pytest.fixture(scope="module")
def P():
    import paper_2606_02053_amd as P
    assert torch.cuda.is_available()
    return P


def mk(P, orc, n, L, **kw):
    s = orc.Setup(n=n, L=L, **kw)
    solver = P.Solver(n, L, P.make_params(**{k: v for k, v in kw.items()}))
    return s, solver


def to_dev(u):
    return torch.from_numpy(np.ascontiguousarray(u)).cuda()


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("n,L", [((8, 8, 8), (2.4, 2.4, 2.4)), ((12, 16, 10), (3.0, 3.5, 2.5)),
                                 ((32, 32, 32), (10.0, 10.0, 10.0))])
def test_rhs_fuzz(P, orc, n, L, variant):
    s, sol = mk(P, orc, n, L)
    sol.params.variant = variant
    u = fuzz_state(n, seed=101)
    sol.set_state(to_dev(u))
    for t in (0.0, 0.37):
        g = sol.rhs(t=t).cpu().numpy()
        r, _ = orc.rhs(s, u, t=t, parallel=True)
        e, per = err_fields(g, r)
        assert e < 1e-11, per


def test_rhs_fuzz_options(P, orc):
    n, L = (12, 10, 14), (2.5, 2.0, 3.0)
    for kw in (dict(lapse_bg=0), dict(evolve_shift=0), dict(ko_eps=0.0), dict(w=0.2, eta=2.0, H0=0.5)):
        s, sol = mk(P, orc, n, L, **kw)
        u = fuzz_state(n, seed=7)
        sol.set_state(to_dev(u))
        g = sol.rhs(t=0.2).cpu().numpy()
        r, _ = orc.rhs(s, u, t=0.2)
        e, per = err_fields(g, r)
        assert e < 1e-11, (kw, per)


@pytest.mark.parametrize("profile,noise", [(0, 1e-6), (1, 0.0), (2, 0.0)])
def test_init_parity(P, orc, profile, noise):
    n, L = (16, 12, 20), (10.0, 8.0, 12.0)
    s, sol = mk(P, orc, n, L)
    ini = dict(mu=0.3, sigma=1.2, noise_amp=noise, seed=2606, profile=profile, center=(0.1, -0.2, 0.3))
    g = sol.init(**ini).cpu().numpy()
    r = orc.init_fields(s, orc.Init(**ini))
    e, per = err_fields(g, r)
    assert e < 1e-13, per
    for which in (0, 1):
        du = torch.empty_like(sol.u)
        P.cosmos_init_tangent(sol.grid, sol.params, P.make_init(**ini), which, du)
        rt = orc.init_tangent(s, orc.Init(**ini), which)
        e, per = err_fields(du.cpu().numpy(), rt)
        assert e < 1e-12, (which, per)


def test_rk4_one_step_fuzz(P, orc):
    n, L = (16, 12, 14), (3.0, 2.5, 2.8)
    s, sol = mk(P, orc, n, L)
    u = fuzz_state(n, seed=5)
    sol.set_state(to_dev(u), t=0.1)
    dt = 0.25 * min(s.h)
    sol.step(dt)
    r, _ = orc.rk4(s, u, 0.1, dt, 1, parallel=True)
    e, per = err_fields(sol.u.cpu().numpy(), r)
    assert e < 1e-11, per


def c1_setup(P, orc):
    """32^3 periodic box of side 10, Gaussian zeta (mu 0.1, sigma 1), 1e-6 white noise on E."""
    n, L = (32, 32, 32), (10.0, 10.0, 10.0)
    s, sol = mk(P, orc, n, L)
    ini = dict(mu=0.1, sigma=1.0, noise_amp=1e-6, seed=2606)
    return s, sol, ini


def test_c1_ten_steps_and_hundred(P, orc):
    s, sol, ini = c1_setup(P, orc)
    sol.init(**ini)
    u0 = orc.init_fields(s, orc.Init(**ini))
    dt = 0.25 * s.h[0]
    sol.step(dt)
    r1, _ = orc.rk4(s, u0, 0.0, dt, 1, parallel=True)
    e1, per = err_fields(sol.u.cpu().numpy(), r1)
    assert e1 < 1e-11, per
    sol.run(9, dt)
    r10, _ = orc.rk4(s, r1, dt, dt, 9, parallel=True)
    e10, per = err_fields(sol.u.cpu().numpy(), r10)
    assert e10 < 1e-10, per
    sol.run(90, dt)
    r100, _ = orc.rk4(s, r10, 10 * dt, dt, 90, parallel=True)
    e100, per = err_fields(sol.u.cpu().numpy(), r100)
    print(f"C1 parity: 1 step {e1:.3e}, 10 steps {e10:.3e}, 100 steps {e100:.3e}")
    assert e100 < 1e-9, per
    st = sol.status()
    assert st["steps"] == 100 and st["nonfinite"] == 0 and st["prim_fail"] == 0


def test_constraints_parity(P, orc):
    n, L = (16, 20, 12), (4.0, 5.0, 3.0)
    s, sol = mk(P, orc, n, L)
    u = fuzz_state(n, seed=9)
    sol.set_state(to_dev(u))
    norms, H, M = sol.constraints(want_fields=True)
    rn, rH, rM = orc.constraints(s, u, want_fields=True)
    norms = norms.numpy()
    assert np.allclose(norms[:5], rn[:5], rtol=1e-12, atol=0), (norms, rn)
    assert norms[5] == rn[5] == 0 and norms[6] == rn[6] and norms[7] == rn[7]
    Hs = np.abs(rH).max()
    assert np.abs(H.cpu().numpy() - rH).max() < 1e-12 * Hs
    Ms = np.abs(rM).max()
    assert np.abs(M.cpu().numpy() - rM).max() < 1e-12 * Ms
    # initial data: momentum constraint exactly zero, H at truncation level
    s2, sol2, ini = c1_setup(P, orc)
    sol2.init(**ini)
    g = sol2.constraints().numpy()
    r = orc.constraints(s2, orc.init_fields(s2, orc.Init(**ini)))
    assert g[3] == 0.0 and r[3] == 0.0
    assert g[0] == pytest.approx(r[0], rel=1e-11)
    assert g[7] == r[7] and g[6] == r[6]


@pytest.mark.parametrize("n", [(32, 32, 32), (20, 20, 12), (9, 13, 11), (16, 20, 12)])
def test_constraints_lds_equals_direct(P, orc, n):
    """The LDS-staged constraint kernel (variant 0) against the direct one (variant 1): the
    same point arithmetic, so H and M_i agree bitwise; the norms differ only in the order of
    their sums. Grids: one workgroup per brick in XCD slabs (32^3), more bricks than partial
    records so that workgroups stride over several bricks (20x20x12), ragged bricks (16x20x12,
    and 9x13x11, whose odd n0 sends variant 0 to the direct kernel too). The LDS variant is also
    checked against the oracle's fields."""
    L = tuple(0.25 * x for x in n)
    s = orc.Setup(n=n, L=L)
    u = to_dev(fuzz_state(n, seed=21))
    out = {}
    for variant in (0, 1):
        sol = P.Solver(n, L, P.make_params(variant=variant))
        sol.set_state(u)
        norms, H, M = sol.constraints(want_fields=True)
        out[variant] = (norms.numpy(), H.cpu().numpy(), M.cpu().numpy())
    (n0, H0, M0), (n1, H1, M1) = out[0], out[1]
    assert np.array_equal(H0, H1) and np.array_equal(M0, M1)
    np.testing.assert_allclose(n0[[0, 2, 4]], n1[[0, 2, 4]], rtol=1e-13)
    assert np.array_equal(n0[[1, 3, 5, 6, 7]], n1[[1, 3, 5, 6, 7]])
    rn, rH, rM = orc.constraints(s, u.cpu().numpy(), want_fields=True)
    assert np.abs(H0 - rH).max() < 1e-12 * np.abs(rH).max()
    assert np.abs(M0 - rM).max() < 1e-12 * np.abs(rM).max()
    np.testing.assert_allclose(n0[:5], rn[:5], rtol=1e-12)


def test_determinism_bitwise(P, orc):
    s, sol, ini = c1_setup(P, orc)
    outs = []
    for _ in range(2):
        sol.init(**ini)
        sol.run(5)
        outs.append((sol.u.clone(), sol.constraints().clone()))
    assert torch.equal(outs[0][0], outs[1][0])
    assert torch.equal(outs[0][1], outs[1][1])


def test_status_counts_match_oracle(P, orc):
    n, L = (12, 12, 12), (3.0, 3.0, 3.0)
    s, sol = mk(P, orc, n, L)
    u = fuzz_state(n, seed=3)
    # invalid fluid states: negative energy at two points, superluminal momentum at one
    u[orc.ET, 2, 3, 4] = -0.5
    u[orc.ET, 7, 1, 0] = -0.1
    u[orc.ST, 5, 5, 5] = 50.0
    sol.set_state(to_dev(u))
    P.cosmos_status_reset(sol.ws)
    dt = 0.25 * min(s.h)
    sol.step(dt)
    st = sol.status()
    _, pf = orc.rk4(s, u, 0.0, dt, 1)
    assert st["prim_fail"] == pf and pf > 0
    # a non-finite value spreads through the stencils; count points after one step
    v = fuzz_state(n, seed=4)
    v[orc.TRK, 6, 6, 6] = np.nan
    sol.set_state(to_dev(v))
    P.cosmos_status_reset(sol.ws)
    sol.step(dt)
    st = sol.status()
    r, _ = orc.rk4(s, v, 0.0, dt, 1)
    bad = int((~np.isfinite(r.reshape(25, -1))).any(axis=0).sum())
    assert st["nonfinite"] == bad and bad > 0
    norms = sol.constraints().numpy()
    rn = orc.constraints(s, r)
    assert norms[5] == rn[5]


@pytest.mark.parametrize("nn", [256, 384])
def test_bench_configuration_sampled(P, orc, nn):
    """256^3 and 384^3, L = 16, Gaussian zeta mu = 0.6, sigma = 2: initial data, one RHS and one
    RK4 step in the launch configuration the benchmark times (LDS-staged 16x4x4 bricks, XCD-blocked
    order, persistent workgroups), checked at sampled points."""
    n, L = (nn, nn, nn), (16.0, 16.0, 16.0)
    s, sol = mk(P, orc, n, L)
    assert (sol.params.variant, sol.params.tile_order) == (0, 2)
    ini = dict(mu=0.6, sigma=2.0)
    sol.init(**ini)
    pts = sample_points(n, 24, seed=1)
    idx = torch.from_numpy(pts).cuda()
    g0 = sol.u.reshape(25, -1)[:, idx].T.cpu().numpy()
    r0 = orc.init_at_points(s, orc.Init(**ini), pts)
    assert np.abs(g0 - r0).max() < 1e-13 * np.abs(r0).max()
    u0 = orc.init_fields(s, orc.Init(**ini))
    rhs = sol.rhs(t=0.0).reshape(25, -1)[:, idx].T.cpu().numpy()
    rr = orc.rhs_at_points(s, u0, pts, t=0.0)
    scale = np.maximum(np.abs(rr).max(axis=0), 1e-3)
    assert (np.abs(rhs - rr).max(axis=0) / scale).max() < 1e-11
    dt = 0.25 * s.h[0]
    sol.step(dt)
    g1 = sol.u.reshape(25, -1)[:, idx[:8]].T.cpu().numpy()
    r1 = orc.rk4_at_points(s, u0, pts[:8], 0.0, dt)
    scale = np.maximum(np.abs(r1).max(axis=0), 1e-3)
    assert (np.abs(g1 - r1).max(axis=0) / scale).max() < 1e-11
    if nn == 256:
        # the benchmark times its steps as one cosmos_rk4_steps call (fluxes carried across the
        # steps): from the initial data, two steps in one call equal two single steps bitwise
        one = sol.u.clone()  # after the single step above
        P.cosmos_rk4_step(sol.grid, sol.params, dt, dt, one, sol.ws)
        two = torch.empty_like(sol.u)
        P.cosmos_init_fields(sol.grid, sol.params, P.make_init(**ini), two)
        P.cosmos_rk4_steps(sol.grid, sol.params, 0.0, dt, 2, two, sol.ws)
        assert torch.equal(two, one)


def test_tile_invariance_bitwise(P, orc):
    """Every brick and order of one kernel variant gives bitwise the same result (partial bricks
    included); the two variants agree to round-off (the compiler contracts FMAs differently)."""
    from paper_2606_02053_amd import autotune
    n, L = (20, 12, 18), (4.0, 2.5, 3.5)
    s, sol = mk(P, orc, n, L)
    u = fuzz_state(n, seed=12)
    sol.set_state(to_dev(u))
    ref = sol.rhs(t=0.1)
    r, _ = orc.rhs(s, u, t=0.1)
    assert err_fields(ref.cpu().numpy(), r)[0] < 1e-11
    dt = 0.25 * min(s.h)
    first_rhs, first_step = {}, {}
    for kv, tile, order in autotune.CANDIDATES:
        p = autotune.with_tile(sol.params, kv, tile, order)
        out = torch.empty_like(sol.u)
        P.cosmos_rhs(sol.grid, p, 0.1, sol.u, out, sol.ws)
        v = sol.u.clone()
        P.cosmos_rk4_step(sol.grid, p, 0.1, dt, v, sol.ws)
        if kv not in first_rhs:
            first_rhs[kv], first_step[kv] = out, v
            assert err_fields(out.cpu().numpy(), r)[0] < 1e-11, kv
        assert torch.equal(out, first_rhs[kv]), (kv, tile, order)
        assert torch.equal(v, first_step[kv]), (kv, tile, order)
    assert err_fields(first_rhs[0].cpu().numpy(), first_rhs[1].cpu().numpy())[0] < 1e-13


@pytest.mark.parametrize("n,L", [((60, 32, 64), (7.5, 4.0, 8.0)), ((64, 44, 42), (8.0, 5.5, 5.25))])
def test_blocked_order_bitwise(P, orc, n, L):
    """The XCD-blocked brick order of the persistent LDS kernel visits every brick once:
    right-hand side and RK4 step equal the linear order bitwise, and sampled points match
    the oracle. 60 x 32 x 64 takes the blocked order (16 brick layers = 2 per XCD, blocks of
    32 bricks dividing each slab, a partial brick column in x); 64 x 44 x 42 (11 brick
    layers, a partial layer in z) cannot be split evenly over the XCDs and falls back to
    the linear order."""
    from paper_2606_02053_amd import autotune
    s, sol = mk(P, orc, n, L)
    u = fuzz_state(n, seed=21)
    sol.set_state(to_dev(u))
    dt = 0.25 * min(s.h)
    outs = {}
    for order in (1, 2, 0):
        p = autotune.with_tile(sol.params, 0, (16, 4, 4), order)
        out = torch.empty_like(sol.u)
        P.cosmos_rhs(sol.grid, p, 0.3, sol.u, out, sol.ws)
        v = sol.u.clone()
        P.cosmos_rk4_step(sol.grid, p, 0.3, dt, v, sol.ws)
        outs[order] = (out, v)
    for order in (2, 0):
        assert torch.equal(outs[order][0], outs[1][0]), order
        assert torch.equal(outs[order][1], outs[1][1]), order
    pts = sample_points(n, 24, seed=5)
    ref = orc.rhs_at_points(s, u, pts, t=0.3)
    got = outs[2][0].reshape(25, -1)[:, torch.from_numpy(pts).cuda()].T.cpu().numpy()
    scale = np.maximum(np.abs(ref).max(axis=0), 1e-3)
    assert (np.abs(got - ref).max(axis=0) / scale).max() < 1e-11



def test_c2_128cubed_500_steps(P, orc):
    """128^3, L = 12, Gaussian zeta mu = 0.5, sigma = 1.5, CFL 0.25, KO 0.1: initial data and
    the first RK4 step against the oracle at sampled points (the centre, where the perturbation
    peaks, included), then the configuration's 500 steps with the constraint norms every 10
    steps. At step 499 one more GPU step is checked against the oracle's step from the GPU's own
    state at sampled points (a property that holds at any step count), and the norms at step 500
    against the oracle's norms of the GPU's state."""
    n, L = (128, 128, 128), (12.0, 12.0, 12.0)
    s, sol = mk(P, orc, n, L)
    ini = dict(mu=0.5, sigma=1.5)
    sol.init(**ini)
    u0 = orc.init_fields(s, orc.Init(**ini))
    assert err_fields(sol.u.cpu().numpy(), u0)[0] < 1e-13
    c = 64 + 128 * (64 + 128 * 64)
    pts = np.unique(np.concatenate([sample_points(n, 16, seed=5), [c, c + 1, c + 3 * 128, c + 5 * 128 * 128]]))
    idx = torch.from_numpy(pts).cuda()
    dt = 0.25 * s.h[0]

    def check_step(u_before, t):
        g = sol.u.reshape(25, -1)[:, idx].T.cpu().numpy()
        r = orc.rk4_at_points(s, u_before, pts, t, dt)
        scale = np.maximum(np.abs(r).max(axis=0), 1e-3)
        return (np.abs(g - r).max(axis=0) / scale).max()

    sol.step(dt)
    e1 = check_step(u0, 0.0)
    assert e1 < 1e-11
    history = [orc.constraints(s, u0, parallel=True)[:5]]
    for _ in range(49):
        sol.run(10 if len(history) > 1 else 9, dt)
        history.append(sol.constraints().numpy()[:5])
    assert sol.status()["steps"] == 490
    sol.run(9, dt)
    u499, t499 = sol.u.cpu().numpy(), sol.t
    sol.step(dt)
    e500 = check_step(u499, t499)
    g = sol.constraints().numpy()
    rn = orc.constraints(s, sol.u.cpu().numpy(), parallel=True)
    hh = np.array(history + [g[:5]])
    print(f"C2: step 1 {e1:.3e}, step 500 {e500:.3e}; H_L2 {hh[0, 0]:.3e} max {hh[:, 0].max():.3e}, "
          f"M_L2 max {hh[:, 2].max():.3e}")
    assert e500 < 1e-11
    np.testing.assert_allclose(g[:5], rn[:5], rtol=1e-11)
    assert g[5] == 0 and g[6] == rn[6] and g[7] == rn[7]
    history.append(g[:5])
    h = np.array(history)
    st = sol.status()
    assert st["steps"] == 500 and st["nonfinite"] == 0 and st["prim_fail"] == 0
    assert np.isfinite(h).all()
    # the constraint violation stays at the discretisation level of the data
    assert h[:, 0].max() < 20 * h[0, 0] and h[:, 2].max() < 20 * h[0, 0]


def _stored_trajectory(name):
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not generated (tests/golden/make_c2_trajectory.py)")
    with open(path) as f:
        return json.load(f)


def test_c2_trajectory_100_steps_against_stored_oracle(P):
    """128^3, L = 12, Gaussian zeta mu = 0.5, sigma = 1.5, CFL 0.25, KO 0.1: 100 RK4 steps from the
    GPU's own initial data, against the oracle's 100-step state stored at 64 points (the centre
    and its axis neighbours included) by tests/golden/make_c2_trajectory.py, with the per-field
    scale of the parity metric taken over the oracle's whole grid; bar 1e-9. The step-100
    constraint norms against the oracle's."""
    g = _stored_trajectory("c2_128cubed_100steps.json")
    cfg = g["config"]
    n, L = (cfg["n"],) * 3, (cfg["L"],) * 3
    sol = P.Solver(n, L)
    assert (sol.params.variant, sol.params.tile_order) == (0, 2)  # the benchmark's launch configuration
    sol.init(mu=cfg["mu"], sigma=cfg["sigma"])
    dt = cfg["dt"]
    assert dt == 0.25 * cfg["L"] / cfg["n"]
    sol.run(cfg["steps"], dt)
    pts = np.array(g["points"], dtype=np.int64)
    got = sol.u.reshape(25, -1)[:, torch.from_numpy(pts).cuda()].T.cpu().numpy()
    ref = np.array(g["values"])
    scale = np.maximum(np.array(g["field_absmax"]), 1e-3)
    per = (np.abs(got - ref).max(axis=0) / scale)
    print(f"C2 100-step trajectory at {len(pts)} points: max error {per.max():.3e}")
    assert per.max() < 1e-9, per
    norms = sol.constraints().numpy()
    np.testing.assert_allclose(norms[:5], np.array(g["norms"][:5]), rtol=1e-9)
    assert norms[5] == g["norms"][5] and norms[6] == pytest.approx(g["norms"][6], rel=1e-12)
    st = sol.status()
    assert st["steps"] == 100 and st["nonfinite"] == 0 and st["prim_fail"] == g["prim_fail"]


@pytest.mark.parametrize("kv,tile,order,scheme", [(0, (16, 4, 4), 2, 0), (0, (16, 8, 2), 1, 0), (1, (16, 4, 4), 0, 0),
                                                  (0, (16, 4, 4), 1, 1)])
def test_rk4_steps_equals_single_steps_bitwise(P, orc, kv, tile, order, scheme):
    """cosmos_rk4_steps carries the fluid fluxes from the last stage of a step to the next step
    (the LDS-staged 16x4x4 kernel of the centred scheme; the other bricks, the direct variant
    and the Kurganov-Tadmor scheme run the pre-pass): the same state bitwise as single steps at
    t, t + dt, ..., with the step counter advanced once per step; 5 steps on a 32 x 16 x 24 grid
    whose step-5 state also matches the oracle."""
    from paper_2606_02053_amd import autotune
    n, L = (32, 16, 24), (8.0, 4.0, 6.0)
    s, sol = mk(P, orc, n, L, fluid_scheme=scheme)
    params = autotune.with_tile(sol.params, kv, tile, order)
    u = fuzz_state(n, seed=91)
    dt, t0 = 0.25 * min(s.h), 0.3
    single = to_dev(u)
    t = t0
    for _ in range(5):
        P.cosmos_rk4_step(sol.grid, params, t, dt, single, sol.ws)
        t += dt
    P.cosmos_status_reset(sol.ws)
    multi = to_dev(u)
    P.cosmos_rk4_steps(sol.grid, params, t0, dt, 5, multi, sol.ws)
    assert torch.equal(multi, single)
    assert sol.status()["steps"] == 5
    P.cosmos_rk4_steps(sol.grid, params, t0, dt, 0, multi, sol.ws)  # no step
    assert torch.equal(multi, single)
    with pytest.raises(P.CosmosError):
        P.cosmos_rk4_steps(sol.grid, params, t0, dt, -1, multi, sol.ws)
    if kv == 0 and tile == (16, 4, 4) and scheme == 0:
        ref, _ = orc.rk4(s, u, t0, dt, 5, parallel=True)
        assert err_fields(multi.cpu().numpy(), ref)[0] < 1e-10
