"""Fixed mesh refinement on the GPU against the oracle (oracle/fmr.py): the prolongation entry point
(whole child and buffer only, parent values at the step start and from the step's continuous
extension, a box that wraps around the periodic parent), the injection, and a three-layer refined run (layer 0
periodic, two nested children, Berger-Oliger sub-cycling) layer by layer after several steps."""
import numpy as np
import pytest
import torch

from oracle import fmr
from tests.inputs import fuzz_direction, fuzz_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2606_02053_amd as P
    return P


def rel(a, b, floor=1e-6):
    """Largest per-field max-norm difference relative to the field's max-norm (floored)."""
    a = np.asarray(a).reshape(25, -1)
    b = np.asarray(b).reshape(25, -1)
    return (np.abs(a - b).max(axis=1) / np.maximum(np.abs(b).max(axis=1), floor)).max()


SMALL = ((20, 16, 24), (5.0, 4.0, 6.0), fmr.Box(origin=(15, -3, 5), m=(6, 5, 8)))  # wraps in x and y
# a box wide enough that a buffer-only refill skips the intermediate values no shell point reads
LARGE = ((40, 36, 44), (10.0, 9.0, 11.0), fmr.Box(origin=(3, 30, -4), m=(22, 18, 26)))  # wraps in y and z


@pytest.mark.parametrize("case,theta,buffer_only",
                         [("small", th, bo) for th in (0.0, 0.5, 0.3) for bo in (False, True)] +
                         [("large", 0.5, True), ("large", 0.3, False)])
def test_prolong_matches_oracle(P, case, theta, buffer_only):
    """Interpolation from a parent step's start, its continuous extension at the midpoint (the
    refill the driver does) and at another theta, whole child or buffer only, on boxes that wrap
    around the periodic parent; the oracle forms the slopes from the stage states and takes
    u0 + dt sum_i b_i k_i."""
    n, L, box = SMALL if case == "small" else LARGE
    u0 = fuzz_state(n, seed=71)
    stages = np.stack([u0 + 0.05 * fuzz_direction(n, seed=72 + q) for q in range(3)])
    u1 = u0 + 0.05 * fuzz_direction(n, seed=75)
    dt = 0.13
    if theta == 0.0:
        src = u0
    else:
        ks = fmr.slopes_from_stage_states(u0, stages[0], stages[1], stages[2], u1, dt)
        src = fmr.dense(u0, ks, dt, theta)
    ref = fmr.prolong(src, box)
    grid = P.make_grid(n, L)
    b = P._lib.make_box(box.origin, box.m)
    cg = P.cosmos_fmr_child_grid(grid, b)
    assert tuple(cg.n) == tuple(2 * box.m[a] + 2 * fmr.W for a in range(3))
    start = fuzz_state(tuple(cg.n), seed=76)
    child = torch.from_numpy(start).cuda()
    ws = torch.empty(P.cosmos_fmr_workspace_bytes(grid, b), dtype=torch.uint8, device="cuda")
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    P.cosmos_fmr_prolong(grid, b, dev(u0), dev(stages) if theta else None, dev(u1) if theta else None, theta,
                         buffer_only, child, ws)
    got = child.cpu().numpy()
    if buffer_only:
        mask = fmr.shell_mask(box)
        assert np.array_equal(got[:, ~mask], start[:, ~mask])  # the interior is left alone
        expect = start.copy()
        expect[:, mask] = ref[:, mask]
        ref = expect
    assert rel(got, ref) < 1e-13


def test_restrict_matches_oracle_bitwise(P):
    n, L = (16, 12, 20), (4.0, 3.0, 5.0)
    box = fmr.Box(origin=(13, 8, -2), m=(5, 6, 4))
    grid = P.make_grid(n, L)
    b = P._lib.make_box(box.origin, box.m)
    cg = P.cosmos_fmr_child_grid(grid, b)
    child = fuzz_state(tuple(cg.n), seed=81)
    parent = fuzz_state(n, seed=82)
    ref = fmr.restrict(child, parent, box)
    pd = torch.from_numpy(parent).cuda()
    P.cosmos_fmr_restrict(grid, b, torch.from_numpy(child).cuda(), pd)
    assert np.array_equal(pd.cpu().numpy(), ref)


def test_fmr_argument_checks(P):
    grid = P.make_grid((16, 16, 16), (4.0, 4.0, 4.0))
    with pytest.raises(P.CosmosError):
        P.cosmos_fmr_child_grid(grid, P._lib.make_box((0, 0, 0), (3, 8, 8)))  # m < 4
    b = P._lib.make_box((2, 2, 2), (6, 6, 6))
    cg = P.cosmos_fmr_child_grid(grid, b)
    u = torch.zeros((25, 16, 16, 16), dtype=torch.float64, device="cuda")
    child = torch.zeros((25, cg.n[2], cg.n[1], cg.n[0]), dtype=torch.float64, device="cuda")
    ws = torch.empty(P.cosmos_fmr_workspace_bytes(grid, b), dtype=torch.uint8, device="cuda")
    st = torch.zeros((3, 25, 16, 16, 16), dtype=torch.float64, device="cuda")
    with pytest.raises(P.CosmosError):  # theta > 0 needs the stage states and u_np1
        P.cosmos_fmr_prolong(grid, b, u, None, None, 0.5, True, child, ws)
    with pytest.raises(P.CosmosError):
        P.cosmos_fmr_prolong(grid, b, u, st, u, 1.5, True, child, ws)


def test_three_layer_run_matches_oracle(P, orc):
    """Layer 0: 24^3 periodic box of side 10; layer 1 over its central 16^3 cells; layer 2 over the
    central 8^3 cells of layer 1 (dt, dt/2, dt/4); PGAUSS data; 3 steps of layer 0."""
    n, L = 24, 10.0
    boxes = [((4, 4, 4), (16, 16, 16)), ((24, 24, 24), (8, 8, 8))]
    ini = dict(mu=0.1, sigma=2.5, profile=orc.PGAUSS)
    run = P.RefinedRun((n, n, n), (L, L, L), boxes)
    run.init(**ini)
    s = orc.Setup(n=(n,) * 3, L=(L,) * 3)
    H = fmr.Hierarchy(s, [fmr.Box(o, m) for o, m in boxes])
    st = H.init(orc.init_fields(s, orc.Init(**ini)))
    for k in range(3):
        assert rel(run.u[k].cpu().numpy(), st[k]) < 1e-13, k
    dt = run.default_dt()
    t = 0.0
    for _ in range(3):
        run.step(dt)
        H.step(st, t, dt)
        t += dt
    for k in range(3):
        e = rel(run.interior(k).cpu().numpy(), st[k][:, fmr.W:-fmr.W, fmr.W:-fmr.W, fmr.W:-fmr.W] if k else st[k])
        print(f"layer {k}: {e:.3e}")
        assert e < 1e-10, (k, e)
    assert run.status(0)["nonfinite"] == 0


def test_benchmark_shaped_hierarchy_matches_oracle(P, orc):
    """The refined benchmark's shape at half its size: layer 0 a 64^3 periodic box at h = 1/8 with
    the Gaussian zeta of the benchmark (mu = 0.6, sigma = 2.0), layer 1 over its central 32^3 cells,
    layer 2 over the central 32^3 cells of layer 1 (both 88^3 with their 12-point buffers), CFL 0.25
    on every layer; one layer-0 step (two of layer 1, four of layer 2) against the oracle. Every
    field differs by at most 1.5e-14 in absolute terms (all are O(1) or smaller; bar 1e-13). The
    per-field relative measure is larger where a field is small (the connection functions, max-norm
    5.5e-5 after one step, differ by 4e-15: 7.5e-11 on layer 0, 2.3e-10 on layer 2), so it is held
    to the 1e-9 of the trajectory bar only."""
    n, L = 64, 8.0
    boxes = [((16, 16, 16), (32, 32, 32)), ((28, 28, 28), (32, 32, 32))]
    ini = dict(mu=0.6, sigma=2.0)
    run = P.RefinedRun((n, n, n), (L, L, L), boxes)
    run.init(**ini)
    s = orc.Setup(n=(n,) * 3, L=(L,) * 3)
    H = fmr.Hierarchy(s, [fmr.Box(o, m) for o, m in boxes])
    st = H.init(orc.init_fields(s, orc.Init(**ini)))
    assert [tuple(x.shape) for x in st] == [(25, 64, 64, 64), (25, 88, 88, 88), (25, 88, 88, 88)]
    dt = run.default_dt()
    assert dt == 0.25 * s.h[0]
    run.step(dt)
    H.step(st, 0.0, dt)
    for k in range(3):
        got = run.interior(k).cpu().numpy().reshape(25, -1)
        ref = (st[k][:, fmr.W:-fmr.W, fmr.W:-fmr.W, fmr.W:-fmr.W] if k else st[k]).reshape(25, -1)
        e, a = rel(got, ref), np.abs(got - ref).max()
        print(f"layer {k}: {e:.3e} relative, {a:.3e} absolute")
        assert e < 1e-9 and a < 1e-13, (k, e, a)
    for k in range(3):
        assert run.status(k)["nonfinite"] == 0


@pytest.mark.parametrize("variant", [0, 1])
def test_out_of_place_stage_keeping_step_equals_in_place(P, variant):
    """cosmos_rk4_step_stages_to (the refined run's parent step): u is left as it was, u_next and
    the stage states equal what cosmos_rk4_step_stages leaves in u and its stages, bitwise."""
    n, L = (20, 12, 18), (4.0, 2.5, 3.5)
    grid = P.make_grid(n, L)
    params = P.make_params(variant=variant)
    u0 = torch.from_numpy(fuzz_state(n, seed=91)).cuda()
    ws = torch.empty(P.cosmos_workspace_bytes(grid), dtype=torch.uint8, device="cuda")
    dt = 0.25 * min(L[a] / n[a] for a in range(3))
    inplace, st_in = u0.clone(), torch.empty((3,) + tuple(u0.shape), dtype=torch.float64, device="cuda")
    P.cosmos_rk4_step_stages(grid, params, 0.3, dt, inplace, st_in, ws)
    u, nxt = u0.clone(), torch.full_like(u0, float("nan"))
    st = torch.full_like(st_in, float("nan"))
    P.cosmos_rk4_step_stages_to(grid, params, 0.3, dt, u, nxt, st, ws)
    assert torch.equal(u, u0) and torch.equal(nxt, inplace) and torch.equal(st, st_in)
    with pytest.raises(P.CosmosError):
        P.cosmos_rk4_step_stages_to(grid, params, 0.3, dt, u, u, st, ws)
