"""GPU parity of the massless scalar field (phi, Pi) against the oracle, through
the C ABI: initial data with an iso-curvature mode, right-hand side (both stage
kernel variants, both fluid schemes), RK4 steps, 100 steps of an iso-curvature
run, constraints. Metric as in test_gpu_parity (per-field max error over
max |oracle|, floor 1e-3), applied to the 25 geometry/fluid fields and the 2
scalar fields separately."""
import numpy as np
import pytest
import torch

from tests.inputs import fuzz_scalar, fuzz_state
from tests.test_gpu_parity import err_fields, to_dev

pytestmark = pytest.mark.gpu


def err2(gpu, ref):
    gpu = np.asarray(gpu).reshape(2, -1)
    ref = np.asarray(ref).reshape(2, -1)
    d = np.abs(gpu - ref).max(axis=1)
    s = np.maximum(np.abs(ref).max(axis=1), 1e-3)
    return (d / s).max(), d / s


@pytest.fixture(scope="module")
def P():
    import paper_2606_02053_amd as P
    assert torch.cuda.is_available()
    return P


def mk(P, orc, n, L, **kw):
    return orc.Setup(n=n, L=L, **kw), P.Solver(n, L, P.make_params(**kw), scalar=True)


@pytest.mark.parametrize("profile", [0, 2])
def test_scalar_init_parity(P, orc, profile):
    n, L = (16, 12, 20), (10.0, 8.0, 12.0)
    s, sol = mk(P, orc, n, L)
    ini = dict(mu=0.2, sigma=1.2, noise_amp=1e-6, seed=2606, profile=profile, center=(0.1, -0.2, 0.3))
    sol.init(sc_mu=0.15, sc_sigma=1.3, **ini)
    u, sc = orc.init_fields_sc(s, orc.Init(**ini), 0.15, 1.3)
    assert err_fields(sol.u.cpu().numpy(), u)[0] < 1e-13
    assert err2(sol.s.cpu().numpy(), sc)[0] < 1e-13


@pytest.mark.parametrize("variant,scheme", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("n,L", [((20, 12, 10), (4.0, 2.5, 2.0)), ((32, 32, 32), (10.0, 10.0, 10.0)),
                                 ((15, 12, 10), (3.0, 2.5, 2.0))])  # odd n0: the direct scalar kernel
def test_scalar_rhs(P, orc, n, L, variant, scheme):
    s, sol = mk(P, orc, n, L, fluid_scheme=scheme)
    sol.params.variant = variant
    u, sc = fuzz_state(n, seed=41), fuzz_scalar(n, seed=42)
    sol.set_state(to_dev(u), s=to_dev(sc))
    du, ds = sol.rhs(t=0.2)
    ru, rs, _ = orc.rhs_sc(s, u, sc, t=0.2, parallel=True)
    e, per = err_fields(du.cpu().numpy(), ru)
    assert e < 1e-11, per
    e2, per2 = err2(ds.cpu().numpy(), rs)
    assert e2 < 1e-11, per2


def test_scalar_lds_kernel_equals_direct_bitwise(P, orc):
    """The scalar stage on state arrays that are 8- but not 16-byte aligned runs the direct
    kernel (no aligned pairs for the LDS-direct loads); both kernels evaluate the same point
    routine, so the field's right-hand side and the sources it hands the geometry agree bitwise
    (the geometry's own right-hand side then comes from the direct stage kernel: equal to
    round-off)."""
    n, L = (20, 12, 18), (4.0, 2.5, 3.5)
    s, sol = mk(P, orc, n, L)
    u, sc = fuzz_state(n, seed=43), fuzz_scalar(n, seed=44)
    sol.set_state(to_dev(u), s=to_dev(sc))
    du0, ds0 = sol.rhs(t=0.2)
    N = int(np.prod(n))
    ub = torch.empty(25 * N + 1, dtype=torch.float64, device="cuda")
    sb = torch.empty(2 * N + 1, dtype=torch.float64, device="cuda")
    um, sm = ub[1:], sb[1:]  # 8-byte aligned views, 16-byte misaligned
    assert um.data_ptr() % 16 == 8 and sm.data_ptr() % 16 == 8
    um.copy_(sol.u.reshape(-1))
    sm.copy_(sol.s.reshape(-1))
    du1, ds1 = torch.empty_like(um), torch.empty_like(sm)
    P.cosmos_rhs_scalar(sol.grid, sol.params, 0.2, um, sm, du1, ds1, sol.ws, sol.sws)
    assert torch.equal(ds1, ds0.reshape(-1))
    assert err_fields(du1.reshape(25, *du0.shape[1:]).cpu().numpy(), du0.cpu().numpy())[0] < 1e-13


@pytest.mark.parametrize("n,scheme", [((20, 12, 18), 0), ((20, 12, 18), 1), ((17, 12, 18), 0)])
def test_scalar_rk4_steps_equals_single_steps(P, orc, n, scheme):
    """cosmos_rk4_steps_scalar (fluid fluxes carried from step to step): 4 steps in one call equal
    4 single steps at t, t + dt, ... bitwise, geometry and field, for both fluid schemes and for an
    odd n0 (the direct kernels); nsteps < 0 is refused."""
    L = (4.0, 2.5, 3.5)
    s, sol = mk(P, orc, n, L, fluid_scheme=scheme)
    u, sc = fuzz_state(n, seed=45), fuzz_scalar(n, seed=46)
    dt = 0.25 * min(s.h)
    sol.set_state(to_dev(u), t=0.1, s=to_dev(sc))
    for _ in range(4):
        sol.step(dt)
    one_u, one_s = sol.u.clone(), sol.s.clone()
    sol.set_state(to_dev(u), t=0.1, s=to_dev(sc))
    sol.run(4, dt)
    assert torch.equal(sol.u, one_u) and torch.equal(sol.s, one_s)
    with pytest.raises(P.CosmosError):
        P.cosmos_rk4_steps_scalar(sol.grid, sol.params, 0.1, dt, -1, sol.u, sol.s, sol.ws, sol.sws)


def test_zero_scalar_field_equals_plain_path(P, orc):
    n, L = (20, 12, 18), (4.0, 2.5, 3.5)
    u = fuzz_state(n, seed=3)
    plain = P.Solver(n, L)
    plain.set_state(to_dev(u))
    s, sol = mk(P, orc, n, L)
    sol.set_state(to_dev(u))  # s = 0
    du, ds = sol.rhs(t=0.1)
    assert torch.equal(du, plain.rhs(t=0.1)) and not ds.any()


def test_scalar_rk4_steps(P, orc):
    n, L = (16, 12, 14), (3.0, 2.5, 2.8)
    s, sol = mk(P, orc, n, L)
    u, sc = fuzz_state(n, seed=5), fuzz_scalar(n, seed=6)
    sol.set_state(to_dev(u), t=0.1, s=to_dev(sc))
    dt = 0.25 * min(s.h)
    sol.step(dt)
    ru, rs, _ = orc.rk4_sc(s, u, sc, 0.1, dt, 1, parallel=True)
    assert err_fields(sol.u.cpu().numpy(), ru)[0] < 1e-11
    assert err2(sol.s.cpu().numpy(), rs)[0] < 1e-11
    sol.run(9, dt)
    ru, rs, _ = orc.rk4_sc(s, ru, rs, 0.1 + dt, dt, 9, parallel=True)
    assert err_fields(sol.u.cpu().numpy(), ru)[0] < 1e-10
    assert err2(sol.s.cpu().numpy(), rs)[0] < 1e-10


def test_isocurvature_hundred_steps_and_constraints(P, orc):
    """32^3 box of side 10: iso-curvature Gaussian Upsilon (0.15, sigma 1.3) on a small
    adiabatic zeta (0.05, sigma 1.5), 100 RK4 steps; then the constraints."""
    n, L = (32, 32, 32), (10.0, 10.0, 10.0)
    s, sol = mk(P, orc, n, L)
    ini = dict(mu=0.05, sigma=1.5)
    sol.init(sc_mu=0.15, sc_sigma=1.3, **ini)
    u0, sc0 = orc.init_fields_sc(s, orc.Init(**ini), 0.15, 1.3)
    dt = 0.25 * s.h[0]
    sol.run(100, dt)
    ru, rs, _ = orc.rk4_sc(s, u0, sc0, 0.0, dt, 100, parallel=True)
    e, per = err_fields(sol.u.cpu().numpy(), ru)
    e2, per2 = err2(sol.s.cpu().numpy(), rs)
    print(f"iso-curvature parity after 100 steps: fields {e:.3e}, scalar {e2:.3e}")
    assert e < 1e-9 and e2 < 1e-9, (per, per2)
    st = sol.status()
    assert st["steps"] == 100 and st["nonfinite"] == 0 and st["prim_fail"] == 0
    norms, H, M = sol.constraints(want_fields=True)
    rn, rH, rM = orc.constraints_sc(s, ru, rs, want_fields=True, parallel=True)
    assert np.abs(H.cpu().numpy() - rH).max() < 1e-9 * max(np.abs(rH).max(), 1e-3)
    assert np.abs(M.cpu().numpy() - rM).max() < 1e-9 * max(np.abs(rM).max(), 1e-3)
    assert abs(norms[0].item() - rn[0]) < 1e-9 * rn[0] and norms[5].item() == rn[5] == 0


def test_scalar_constraints_parity(P, orc):
    n, L = (16, 20, 12), (4.0, 5.0, 3.0)
    s, sol = mk(P, orc, n, L)
    u, sc = fuzz_state(n, seed=9), fuzz_scalar(n, seed=10)
    sol.set_state(to_dev(u), s=to_dev(sc))
    norms, H, M = sol.constraints(want_fields=True)
    rn, rH, rM = orc.constraints_sc(s, u, sc, want_fields=True)
    assert np.abs(H.cpu().numpy() - rH).max() < 1e-11 * np.abs(rH).max()
    assert np.abs(M.cpu().numpy() - rM).max() < 1e-11 * np.abs(rM).max()
    np.testing.assert_allclose(norms.numpy()[:5], rn[:5], rtol=1e-11)
    assert norms[5].item() == rn[5] and norms[7].item() == rn[7]


def test_scalar_bench_configuration_sampled(P, orc):
    """The benchmark's scalar-field workload: 256^3, L = 16, zeta mu = 0.6, sigma = 2 and an
    iso-curvature mode Upsilon (0.1, sigma 2), default launch configuration: initial data,
    one right-hand side and one RK4 step at sampled points."""
    from tests.inputs import sample_points
    n, L = (256, 256, 256), (16.0, 16.0, 16.0)
    s, sol = mk(P, orc, n, L)
    ini = dict(mu=0.6, sigma=2.0)
    sol.init(sc_mu=0.1, sc_sigma=2.0, **ini)
    u0, sc0 = orc.init_fields_sc(s, orc.Init(**ini), 0.1, 2.0)
    assert np.abs(sol.s.cpu().numpy() - sc0).max() < 1e-13 * np.abs(sc0).max()
    # random points plus the centre and points at about one width from it, where the
    # perturbation (and so each field's scale, the metric's denominator) peaks
    c, o = n[0] // 2, 32
    near = [(c, c, c), (c + o, c, c), (c, c - o, c), (c, c, c + o), (c + o // 2, c + o // 2, c - o // 2)]
    pts = np.concatenate([[i + n[0] * (j + n[1] * k) for i, j, k in near], sample_points(n, 8, seed=4)])
    idx = torch.from_numpy(pts).cuda()
    du, ds = sol.rhs(t=0.0)
    ru, rs = orc.rhs_sc_at_points(s, u0, sc0, pts, t=0.0)
    g = du.reshape(25, -1)[:, idx].T.cpu().numpy()
    assert (np.abs(g - ru).max(axis=0) / np.maximum(np.abs(ru).max(axis=0), 1e-3)).max() < 1e-11
    g = ds.reshape(2, -1)[:, idx].T.cpu().numpy()
    assert (np.abs(g - rs).max(axis=0) / np.maximum(np.abs(rs).max(axis=0), 1e-3)).max() < 1e-11
    dt = 0.25 * s.h[0]
    sol.step(dt)
    qu, qs = orc.rk4_sc_at_points(s, u0, sc0, pts[:4], 0.0, dt)
    g = sol.u.reshape(25, -1)[:, idx[:4]].T.cpu().numpy()
    assert (np.abs(g - qu).max(axis=0) / np.maximum(np.abs(qu).max(axis=0), 1e-3)).max() < 1e-11
    g = sol.s.reshape(2, -1)[:, idx[:4]].T.cpu().numpy()
    assert (np.abs(g - qs).max(axis=0) / np.maximum(np.abs(qs).max(axis=0), 1e-3)).max() < 1e-11


def test_scalar_rhs_options(P, orc):
    n, L = (12, 10, 14), (2.5, 2.0, 3.0)
    u, sc = fuzz_state(n, seed=17), fuzz_scalar(n, seed=18)
    for kw in (dict(evolve_shift=0), dict(ko_eps=0.0), dict(lapse_bg=0), dict(w=0.2, eta=2.0, H0=0.5)):
        s, sol = mk(P, orc, n, L, **kw)
        sol.set_state(to_dev(u), s=to_dev(sc))
        du, ds = sol.rhs(t=0.2)
        ru, rs, _ = orc.rhs_sc(s, u, sc, t=0.2)
        assert err_fields(du.cpu().numpy(), ru)[0] < 1e-11, kw
        assert err2(ds.cpu().numpy(), rs)[0] < 1e-11, kw


def test_scalar_direct_variant_any_brick(P, orc):
    """The LDS-staged kernel takes the scalar sources with its 16x4x4 brick only; the direct
    variant takes any brick and agrees with it to round-off."""
    n, L = (20, 12, 18), (4.0, 2.5, 3.5)
    u, sc = fuzz_state(n, seed=19), fuzz_scalar(n, seed=20)
    ref = None
    for variant, tile in ((0, (16, 4, 4)), (1, (8, 8, 4)), (1, (16, 4, 4))):
        sol = P.Solver(n, L, P.make_params(variant=variant, tile=tile, tile_order=1), scalar=True)
        sol.set_state(to_dev(u), s=to_dev(sc))
        du, ds = sol.rhs(t=0.1)
        if ref is None:
            ref = (du, ds)
            continue
        assert err_fields(du.cpu().numpy(), ref[0].cpu().numpy())[0] < 1e-13, (variant, tile)
        assert torch.equal(ds, ref[1]), (variant, tile)  # the scalar kernel is the same
    bad = P.Solver(n, L, P.make_params(variant=0, tile=(8, 8, 4)), scalar=True)
    with pytest.raises(P.CosmosError):
        bad.rhs(t=0.0)
