"""Batched form on the GPU: every run of a batch equals the plain solver's run
(bitwise, same kernel arithmetic), hipGraph replays equal eager steps, and a
poisoned run is flagged without touching the others."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2606_02053_amd as P
    return P


def small_runs():
    from paper_2606_02053_amd.batch import RunSpec
    return [RunSpec(n=16, mu=0.4, sigma=1.0, L=6.0), RunSpec(n=32, mu=0.6, sigma=1.3, L=8.0),
            RunSpec(n=48, mu=0.3, sigma=0.9, L=12.0), RunSpec(n=16, mu=0.7, sigma=1.5, L=5.0)]


def plain_run(P, spec, nsteps, fluid_scheme=0):
    s = P.Solver(spec.n, spec.L, P.make_params(tile=(16, 4, 4), tile_order=1, variant=0, fluid_scheme=fluid_scheme))
    s.init(mu=spec.mu, sigma=spec.sigma)
    dt = 0.25 * spec.L / spec.n
    for _ in range(nsteps):
        s.step(dt)
    return s.u


def test_batched_equals_plain_bitwise(P):
    from paper_2606_02053_amd.batch import Batch
    runs = small_runs()
    b = Batch(runs)
    b.init()
    for _ in range(3):
        b.step()
    torch.cuda.synchronize()
    for r, spec in enumerate(runs):
        assert torch.equal(b.state(r), plain_run(P, spec, 3)), r
    st = b.status()
    assert all(x["steps"] == 3 and x["nonfinite"] == 0 for x in st)
    dt = b.dt.cpu().numpy()
    assert np.allclose(b.t.cpu().numpy(), 3 * dt, rtol=1e-15)


def test_graph_replay_equals_eager(P):
    from paper_2606_02053_amd.batch import Batch
    runs = small_runs()
    eager = Batch(runs)
    eager.init()
    g = Batch(runs)
    g.init()
    g.capture()
    for rep in range(3):
        eager.run(2, use_graph=False)
        g.run(2, use_graph=True)
        torch.cuda.synchronize()
        _ = g.arena.sum().item()  # eager work between replays
        for r in range(len(runs)):
            assert torch.equal(eager.state(r), g.state(r)), (rep, r)
        assert torch.equal(eager.t, g.t)


@pytest.mark.parametrize("tile,scheme", [((16, 4, 4), 0), ((8, 8, 4), 0), ((16, 4, 4), 1)])
def test_multi_step_graph_equals_single_steps(P, tile, scheme):
    """cosmos_rk4_steps_batched: a graph of 3 steps in one call (the last stage of a step writes
    the next step's fluxes with the 16x4x4 brick of the centred scheme; the 8x8x4 brick and the
    KT scheme run a pre-pass per step), replayed twice with eager work between the replays, equals
    6 eager single steps bitwise, step counters and times included; a 7th step (run(7) = two
    replays and one single step) as well."""
    from paper_2606_02053_amd.batch import Batch
    runs = small_runs()
    params = P.make_params(tile=tile, tile_order=1, variant=0, fluid_scheme=scheme)
    eager = Batch(runs, params)
    eager.init()
    g = Batch(runs, params)
    g.init()
    g.capture(steps=3)
    for rep in range(2):
        eager.run(3, use_graph=False)
        g.run(3)
        torch.cuda.synchronize()
        _ = g.arena.sum().item()  # eager work between replays
        for r in range(len(runs)):
            assert torch.equal(eager.state(r), g.state(r)), (rep, r)
        assert torch.equal(eager.t, g.t)
    eager.run(1, use_graph=False)
    g2 = Batch(runs, params)
    g2.init()
    g2.capture(steps=3)
    g2.run(7)
    for r in range(len(runs)):
        assert torch.equal(eager.state(r), g2.state(r)), r
    assert [x["steps"] for x in g2.status()] == [7] * len(runs)
    assert g2.status() == eager.status()


def test_poisoned_run_is_isolated(P):
    from paper_2606_02053_amd.batch import Batch
    runs = small_runs()
    b = Batch(runs)
    b.init()
    b.state(1)[7, 3, 3, 3] = float("nan")
    for _ in range(2):
        b.step()
    torch.cuda.synchronize()
    st = b.status()
    assert st[1]["nonfinite"] > 0
    for r in (0, 2, 3):
        assert st[r]["nonfinite"] == 0
        assert torch.equal(b.state(r), plain_run(P, runs[r], 2)), r


def test_small_work_list_equals_plain_bitwise(P):
    """Fewer work items than resident workgroups (32 bricks): the plain walk of the list
    instead of the per-XCD split; same results."""
    from paper_2606_02053_amd.batch import Batch, RunSpec
    runs = [RunSpec(n=16, mu=0.5, sigma=1.1, L=6.0), RunSpec(n=16, mu=0.8, sigma=1.4, L=7.0)]
    b = Batch(runs)
    b.init()
    for _ in range(2):
        b.step()
    torch.cuda.synchronize()
    for r, spec in enumerate(runs):
        assert torch.equal(b.state(r), plain_run(P, spec, 2)), r


def test_batched_kurganov_tadmor_equals_plain_bitwise(P):
    """fluid_scheme 1 in the batched form: the batched pre-pass (16x4x4 items) gives the same
    interface fluxes and divergence as the plain one (8x8x4 bricks), so every run matches
    the plain KT run bitwise, in eager steps and in graph replays."""
    from paper_2606_02053_amd.batch import Batch
    runs = small_runs()
    b = Batch(runs, P.make_params(fluid_scheme=1))
    b.init()
    b.step()
    b.capture()
    b.run(2)
    torch.cuda.synchronize()
    for r, spec in enumerate(runs):
        assert torch.equal(b.state(r), plain_run(P, spec, 3, fluid_scheme=1)), r
        assert not torch.equal(b.state(r), plain_run(P, spec, 3)), r  # the scheme is in effect
    assert all(x["steps"] == 3 and x["nonfinite"] == 0 for x in b.status())


@pytest.mark.parametrize("scheme", [0, 1])
def test_batched_scalar_field_equals_plain_bitwise(P, scheme):
    """The scalar field in the batched form: every run (geometry, fluid and (phi, Pi)) equals
    the plain scalar-field run bitwise, in eager steps and in graph replays."""
    from paper_2606_02053_amd.batch import Batch, RunSpec
    runs = [RunSpec(n=16, mu=0.2, sigma=1.0, L=6.0, sc_mu=0.15, sc_sigma=1.2),
            RunSpec(n=32, mu=0.1, sigma=1.3, L=8.0, sc_mu=0.1, sc_sigma=1.5),
            RunSpec(n=48, mu=0.0, sigma=1.0, L=12.0, sc_mu=0.2, sc_sigma=2.0)]
    b = Batch(runs, P.make_params(fluid_scheme=scheme), scalar=True)
    b.init()
    b.step()
    b.capture()
    b.run(2)
    torch.cuda.synchronize()
    for r, spec in enumerate(runs):
        s = P.Solver(spec.n, spec.L, P.make_params(tile=(16, 4, 4), tile_order=1, variant=0, fluid_scheme=scheme),
                     scalar=True)
        s.init(mu=spec.mu, sigma=spec.sigma, sc_mu=spec.sc_mu, sc_sigma=spec.sc_sigma)
        dt = 0.25 * spec.L / spec.n
        for _ in range(3):
            s.step(dt)
        assert torch.equal(b.state(r), s.u), r
        assert torch.equal(b.scalar_state(r), s.s), r
        assert b.scalar_state(r)[1].abs().max() > 0  # the field moves
    assert all(x["steps"] == 3 and x["nonfinite"] == 0 for x in b.status())


def _err_fields(gpu, ref):
    """Parity metric per field: ||gpu_f - ref_f||_inf / max(||ref_f||_inf, 1e-3), max over fields."""
    gpu = np.asarray(gpu).reshape(25, -1)
    ref = np.asarray(ref).reshape(25, -1)
    return (np.abs(gpu - ref).max(axis=1) / np.maximum(np.abs(ref).max(axis=1), 1e-3)).max()


def test_batched_runs_match_oracle(P, orc):
    """Every run of a small batch (16^3, 32^3, 48^3 and a second 16^3 in other boxes) after 3 RK4
    steps (one eager, two graph replays) against the oracle's full-grid run."""
    from paper_2606_02053_amd.batch import Batch
    runs = small_runs()
    b = Batch(runs)
    b.init()
    b.step()
    b.capture()
    b.run(2)
    torch.cuda.synchronize()
    for r, spec in enumerate(runs):
        s = orc.Setup(n=(spec.n,) * 3, L=(spec.L,) * 3)
        u0 = orc.init_fields(s, orc.Init(mu=spec.mu, sigma=spec.sigma))
        dt = 0.25 * spec.L / spec.n
        ref, _ = orc.rk4(s, u0, 0.0, dt, 3, parallel=True)
        e = _err_fields(b.state(r).cpu().numpy(), ref)
        assert e < 1e-10, (r, e)


def test_c4_draw_subset_trajectories_match_oracle(P, orc):
    """The first run of each grid size in the seeded 64-run scan (48^3, 64^3, 80^3, 96^3, box 12,
    its drawn mu and sigma) batched together for 5 RK4 steps in graph replays, each against the
    oracle's full-grid 5-step run."""
    from paper_2606_02053_amd.batch import Batch, draw_scan
    draw = draw_scan()
    pick = []
    for size in (48, 64, 80, 96):
        pick.append(next(r for r in draw if r.n == size))
    b = Batch(pick)
    b.init()
    b.capture()
    b.run(5)
    torch.cuda.synchronize()
    for r, spec in enumerate(pick):
        s = orc.Setup(n=(spec.n,) * 3, L=(spec.L,) * 3)
        u0 = orc.init_fields(s, orc.Init(mu=spec.mu, sigma=spec.sigma))
        ref, _ = orc.rk4(s, u0, 0.0, 0.25 * spec.L / spec.n, 5, parallel=True)
        e = _err_fields(b.state(r).cpu().numpy(), ref)
        print(f"C4 run n={spec.n} mu={spec.mu:.4f} sigma={spec.sigma:.4f}: 5 steps, error {e:.3e}")
        assert e < 1e-10, (spec, e)


def test_c4_full_draw_first_step_sampled(P, orc):
    """All 64 runs of the seeded scan (grid sizes 48^3 to 96^3 drawn with numpy's generator seeded
    2606, mu in [0.3, 0.8], sigma in [0.8, 1.6], box 12) in one batch: after one step every run
    matches the oracle's step at 12 sampled points (the centre and corners included)."""
    from paper_2606_02053_amd.batch import Batch, draw_scan
    from tests.inputs import sample_points
    runs = draw_scan()
    assert len(runs) == 64 and {r.n for r in runs} == {48, 64, 80, 96}
    b = Batch(runs)
    b.init()
    b.capture()
    b.run(1)
    torch.cuda.synchronize()
    worst = 0.0
    for r, spec in enumerate(runs):
        n = (spec.n,) * 3
        s = orc.Setup(n=n, L=(spec.L,) * 3)
        u0 = orc.init_fields(s, orc.Init(mu=spec.mu, sigma=spec.sigma))
        pts = sample_points(n, 12, seed=r)
        ref = orc.rk4_at_points(s, u0, pts, 0.0, 0.25 * spec.L / spec.n)
        got = b.state(r).reshape(25, -1)[:, torch.from_numpy(pts).cuda()].T.cpu().numpy()
        scale = np.maximum(np.abs(ref).max(axis=0), 1e-3)
        e = (np.abs(got - ref).max(axis=0) / scale).max()
        worst = max(worst, e)
        assert e < 1e-11, (r, spec, e)
    print(f"C4 draw, 64 runs, first step at sampled points: worst error {worst:.3e}")
    assert all(x["steps"] == 1 and x["nonfinite"] == 0 for x in b.status())


def test_batch_outcomes_on_device(P):
    """cosmos_batch_outcomes: each run's centre lapse and grid-minimum lapse equal the values read
    from its state."""
    from paper_2606_02053_amd.batch import Batch
    runs = small_runs()
    b = Batch(runs)
    b.init()
    b.run(2, use_graph=False)
    out = b.outcomes()
    for r, spec in enumerate(runs):
        a = b.state(r)[17]
        c = spec.n // 2
        assert out[r]["alpha_centre"] == float(a[c, c, c])
        assert out[r]["alpha_min"] == float(a.min())


def test_batched_bricks_bitwise_and_tuner(P):
    """Every brick of the batched stage kernel advances the batch to the same bits (the brick
    changes the schedule, not the arithmetic); the batch autotuner returns one of them with its
    timing table, every candidate eligible."""
    from paper_2606_02053_amd import autotune
    from paper_2606_02053_amd.batch import Batch
    runs = small_runs()
    ref = None
    for tile in autotune.BATCH_BRICKS:
        b = Batch(runs, autotune.with_tile(P.make_params(), 0, tile, 1))
        b.init()
        b.step()
        b.capture()
        b.run(1)
        torch.cuda.synchronize()
        if ref is None:
            ref = b.arena.clone()
        assert torch.equal(b.arena, ref), tile
    tile, table = autotune.tune_batch(runs, use_cache=False)
    assert tile in autotune.BATCH_BRICKS and all(r["parity"] for r in table)
    with pytest.raises(P.CosmosError):
        Batch(runs, autotune.with_tile(P.make_params(fluid_scheme=1), 0, (8, 8, 4), 1)).init()
