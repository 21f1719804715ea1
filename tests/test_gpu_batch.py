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
