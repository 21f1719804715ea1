"""The C-ABI library loads, exports every entry point include/cosmos.h declares,
and rejects invalid arguments before touching the GPU (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "cosmos.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(cosmos_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


@pytest.fixture(scope="module")
def C():
    import paper_2606_02053_amd._lib as C
    return C


def test_every_declared_symbol_is_exported(C):
    names = header_functions()
    assert len(names) >= 10
    missing = [n for n in names if not hasattr(C.lib, n)]
    assert not missing, missing


def test_abi_version(C):
    assert C.cosmos_abi_version() == 1


def test_workspace_bytes(C):
    g = C.make_grid(32, 10.0)
    ws = C.cosmos_workspace_bytes(g)
    state = 25 * 32 ** 3 * 8
    assert ws >= 3 * state and ws % 256 == 0
    assert C.cosmos_workspace_bytes(C.make_grid((7, 32, 32), 10.0)) == 0
    assert C.cosmos_workspace_bytes(C.make_grid(32, -1.0)) == 0


def test_invalid_arguments_rejected_on_host(C):
    g = C.make_grid(16, 4.0)
    p = C.make_params()
    lib = C.lib
    fake = ctypes.c_void_p(0x100000)  # never dereferenced: validation fails first
    rc = lib.cosmos_rhs(ctypes.byref(g), ctypes.byref(p), 0.0, None, fake, fake, None)
    assert rc == C.COSMOS_EINVAL and "u is NULL" in C.last_error()
    rc = lib.cosmos_rhs(ctypes.byref(g), ctypes.byref(p), 0.0, fake, fake, fake, None)
    assert rc == C.COSMOS_EINVAL and "alias" in C.last_error()
    bad = C.make_grid((4, 16, 16), 4.0)
    rc = lib.cosmos_rk4_step(ctypes.byref(bad), ctypes.byref(p), 0.0, 0.1, fake, fake, None)
    assert rc == C.COSMOS_EINVAL and "grid" in C.last_error()
    rc = lib.cosmos_rk4_step(ctypes.byref(g), ctypes.byref(p), 0.0, -0.1, fake, fake, None)
    assert rc == C.COSMOS_EINVAL and "dt" in C.last_error()
    rc = lib.cosmos_rk4_step(ctypes.byref(g), ctypes.byref(p), 0.0, 0.1, ctypes.c_void_p(0x100004), fake, None)
    assert rc == C.COSMOS_EINVAL and "aligned" in C.last_error()
    q = C.make_params(fluid_scheme=2)
    rc = lib.cosmos_rk4_step(ctypes.byref(g), ctypes.byref(q), 0.0, 0.1, fake, fake, None)
    assert rc == C.COSMOS_EUNSUPPORTED
    # the Kurganov-Tadmor scheme (1) runs in the plain and batched entry points; the adjoint
    # implements the centred scheme only
    kt = C.make_params(fluid_scheme=1)
    rc = lib.cosmos_adjoint_step(ctypes.byref(g), ctypes.byref(kt), 0.0, 0.1, fake, fake, fake, fake, None)
    assert rc == C.COSMOS_EUNSUPPORTED and "adjoint" in C.last_error()
    rc = lib.cosmos_rhs_vjp(ctypes.byref(g), ctypes.byref(kt), 0.0, fake, fake, fake, fake, None)
    assert rc == C.COSMOS_EUNSUPPORTED
    base = 0x100000
    u_ = ctypes.c_void_p(base)
    rc = lib.cosmos_kt_divergence(ctypes.byref(g), ctypes.byref(kt), u_, ctypes.c_void_p(base + 8 * 25 * 16 ** 3 - 8),
                                  None)
    assert rc == C.COSMOS_EINVAL and "overlap" in C.last_error()
    rc = lib.cosmos_kt_divergence(ctypes.byref(g), ctypes.byref(kt), u_, None, None)
    assert rc == C.COSMOS_EINVAL
    ini = C.make_init(sigma=0.0)
    rc = lib.cosmos_init_fields(ctypes.byref(g), ctypes.byref(p), ctypes.byref(ini), fake, None)
    assert rc == C.COSMOS_EINVAL


def test_binding_refuses_host_tensors(C):
    import torch
    g = C.make_grid(8, 2.0)
    u = torch.zeros((25, 8, 8, 8), dtype=torch.float64)
    with pytest.raises(C.CosmosError):
        C.cosmos_rhs(g, C.make_params(), 0.0, u, u.clone(), torch.zeros(16, dtype=torch.uint8))


def test_grid_size_limits(C):
    """8 <= n_a <= 2048 and fewer than 2^29 points (32-bit byte offsets within one field)."""
    assert C.cosmos_workspace_bytes(C.make_grid((2048, 1024, 255), 1.0)) > 0
    assert C.cosmos_workspace_bytes(C.make_grid((2048, 2048, 128), 1.0)) == 0  # exactly 2^29 points
    assert C.cosmos_workspace_bytes(C.make_grid((2049, 8, 8), 1.0)) == 0
    assert C.cosmos_adjoint_workspace_bytes(C.make_grid((2048, 2048, 128), 1.0)) == 0


def test_stage_keeping_entry_points_validate_on_host(C):
    g = C.make_grid(16, 4.0)
    p = C.make_params()
    lib = C.lib
    n = 25 * 16 ** 3 * 8
    u = ctypes.c_void_p(0x10000000)  # never dereferenced: validation fails first
    ws = ctypes.c_void_p(0x40000000)
    rc = lib.cosmos_rk4_step_stages(ctypes.byref(g), ctypes.byref(p), 0.0, 0.1, u, None, ws, None)
    assert rc == C.COSMOS_EINVAL and "stages is NULL" in C.last_error()
    overlapping = ctypes.c_void_p(0x10000000 + n // 2)
    rc = lib.cosmos_rk4_step_stages(ctypes.byref(g), ctypes.byref(p), 0.0, 0.1, u, overlapping, ws, None)
    assert rc == C.COSMOS_EINVAL and "overlaps" in C.last_error()
    lam = ctypes.c_void_p(0x20000000)
    rc = lib.cosmos_adjoint_step_stages(ctypes.byref(g), ctypes.byref(p), 0.0, 0.1, u, ctypes.c_void_p(0x20000000 + 8),
                                        u, lam, ws, None)
    assert rc == C.COSMOS_EINVAL and "overlaps" in C.last_error()


def test_scalar_entry_points_validate_on_host(C):
    g = C.make_grid(16, 4.0)
    p = C.make_params()
    lib = C.lib
    assert C.cosmos_scalar_workspace_bytes(g) >= 17 * 16 ** 3 * 8
    assert C.cosmos_scalar_workspace_bytes(C.make_grid((7, 16, 16), 4.0)) == 0
    base = 0x100000
    n = 16 ** 3 * 8
    u, s, ws, sws = (ctypes.c_void_p(base), ctypes.c_void_p(base + 25 * n), ctypes.c_void_p(base + 64 * n),
                     ctypes.c_void_p(base + 128 * n))
    rc = lib.cosmos_rk4_step_scalar(ctypes.byref(g), ctypes.byref(p), 0.0, 0.1, u, s, ws, None, None)
    assert rc == C.COSMOS_EINVAL and "scalar workspace" in C.last_error()
    rc = lib.cosmos_rk4_step_scalar(ctypes.byref(g), ctypes.byref(p), 0.0, 0.1, u, ctypes.c_void_p(base + 8 * n), ws,
                                    sws, None)
    assert rc == C.COSMOS_EINVAL and "overlap" in C.last_error()
    q = C.make_params(tile=(8, 8, 4))
    rc = lib.cosmos_rk4_step_scalar(ctypes.byref(g), ctypes.byref(q), 0.0, 0.1, u, s, ws, sws, None)
    assert rc == C.COSMOS_EUNSUPPORTED and "16x4x4" in C.last_error()
    rc = lib.cosmos_rhs_scalar(ctypes.byref(g), ctypes.byref(p), 0.0, u, s, u, ctypes.c_void_p(base + 200 * n), ws,
                               sws, None)
    assert rc == C.COSMOS_EINVAL and "overlap" in C.last_error()
    ini = C.make_init()
    rc = lib.cosmos_init_fields_scalar(ctypes.byref(g), ctypes.byref(p), ctypes.byref(ini), 0.1, 0.0, u, s, None)
    assert rc == C.COSMOS_EINVAL


def test_probe_library_exports_and_rejects_bad_arguments():
    """libcosmos_probe.so (machine probes for the benchmark's achievable peaks) exports every
    function include/cosmos_probe.h declares and rejects invalid arguments on the host."""
    src = open(os.path.join(ROOT, "include", "cosmos_probe.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = sorted(set(re.findall(r"\b(cosmos_probe_[a-z0-9_]+)\s*\(", src)))
    assert len(names) == 3
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2606_02053_amd", "libcosmos_probe.so"))
    assert all(hasattr(lib, n) for n in names)
    lib.cosmos_probe_triad.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_double, ctypes.c_size_t, ctypes.c_void_p]
    lib.cosmos_probe_fma64.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p]
    lib.cosmos_probe_fma64_flops.argtypes = [ctypes.c_size_t, ctypes.c_int]
    lib.cosmos_probe_fma64_flops.restype = ctypes.c_double
    fake = 1 << 20  # never dereferenced: every call below fails its host-side checks
    assert lib.cosmos_probe_triad(None, fake, fake, 1.0, 16, None) == -1
    assert lib.cosmos_probe_triad(fake, fake + 4096, fake + 8192, 1.0, 15, None) == -1  # odd n
    assert lib.cosmos_probe_triad(fake + 8, fake + 4096, fake + 8192, 1.0, 16, None) == -1  # misaligned
    assert lib.cosmos_probe_triad(fake, fake + 64, fake + 8192, 1.0, 16, None) == -1  # a overlaps b
    assert lib.cosmos_probe_fma64(fake, 255, 10, None) == -1
    assert lib.cosmos_probe_fma64(fake, 256, 0, None) == -1
    assert lib.cosmos_probe_fma64(None, 256, 10, None) == -1
    assert lib.cosmos_probe_fma64_flops(512, 100) == 2.0 * 16 * 100 * 512


def test_fmr_geometry_on_host(C):
    """The refinement entry points' host-side geometry: the padded child grid, the workspace size
    and the argument checks that run before any launch."""
    g = C.make_grid((24, 20, 16), (6.0, 5.0, 4.0))
    b = C.make_box((3, -2, 5), (8, 6, 5))
    child = C.cosmos_fmr_child_grid(g, b)
    assert tuple(child.n) == (2 * 8 + 24, 2 * 6 + 24, 2 * 5 + 24)
    assert [child.L[a] for a in range(3)] == pytest.approx([child.n[a] * 0.25 / 2 for a in range(3)])
    ws = C.cosmos_fmr_workspace_bytes(g, b)
    # two intermediates: x interpolated (40 x 23 x 22), then y (40 x 36 x 22), 25 fields each,
    # each rounded up to 256 bytes
    up = lambda x: (x + 255) // 256 * 256  # noqa: E731
    assert ws == up(25 * 8 * (40 * 23 * 22)) + up(25 * 8 * (40 * 36 * 22))
    assert C.cosmos_fmr_workspace_bytes(g, C.make_box((0, 0, 0), (3, 6, 6))) == 0
    lib = C.lib
    fake = ctypes.c_void_p(0x100000)
    rc = lib.cosmos_fmr_prolong(ctypes.byref(g), ctypes.byref(b), fake, None, None, 0.5, 1, fake, fake, None)
    assert rc == C.COSMOS_EINVAL and "stages" in C.last_error()
    rc = lib.cosmos_fmr_prolong(ctypes.byref(g), ctypes.byref(b), fake, fake, fake, -0.5, 1, fake, fake, None)
    assert rc == C.COSMOS_EINVAL and "theta" in C.last_error()
    rc = lib.cosmos_fmr_restrict(ctypes.byref(g), ctypes.byref(b), None, fake, None)
    assert rc == C.COSMOS_EINVAL and "child_u" in C.last_error()


def test_multi_step_entry_points_validate_on_host(C):
    g = C.make_grid(16, 4.0)
    p = C.make_params()
    lib = C.lib
    n = 25 * 16 ** 3 * 8
    u = ctypes.c_void_p(0x10000000)  # never dereferenced: validation fails first, or no step runs
    ws = ctypes.c_void_p(0x40000000)
    G, Pp = ctypes.byref(g), ctypes.byref(p)
    assert lib.cosmos_rk4_steps(G, Pp, 0.0, 0.1, -1, u, ws, None) == C.COSMOS_EINVAL
    assert "nsteps -1" in C.last_error()
    assert lib.cosmos_rk4_steps(G, Pp, 0.0, 0.0, 3, u, ws, None) == C.COSMOS_EINVAL
    assert lib.cosmos_rk4_steps(G, Pp, 0.0, float("nan"), 3, u, ws, None) == C.COSMOS_EINVAL
    assert lib.cosmos_rk4_steps(G, Pp, 0.0, 0.1, 0, u, ws, None) == C.COSMOS_OK  # zero steps: nothing launched
    states = ctypes.c_void_p(0x80000000)
    stages = ctypes.c_void_p(0xC0000000)
    rc = lib.cosmos_rk4_steps_stages(G, Pp, 0.0, 0.1, -2, u, states, stages, ws, None)
    assert rc == C.COSMOS_EINVAL and "nsteps -2" in C.last_error()
    # the third of three kept states would reach into u
    below_u = ctypes.c_void_p(0x10000000 - 2 * n)
    rc = lib.cosmos_rk4_steps_stages(G, Pp, 0.0, 0.1, 3, u, below_u, stages, ws, None)
    assert rc == C.COSMOS_EINVAL and "must not overlap" in C.last_error()
    rc = lib.cosmos_rk4_steps_stages(G, Pp, 0.0, 0.1, 2, u, states, ctypes.c_void_p(0x80000000 + n), ws, None)
    assert rc == C.COSMOS_EINVAL and "must not overlap" in C.last_error()
    assert lib.cosmos_rk4_steps_stages(G, Pp, 0.0, 0.1, 0, u, states, stages, ws, None) == C.COSMOS_OK
    b = C.cosmos_batch()
    rc = lib.cosmos_rk4_steps_batched(ctypes.byref(b), Pp, u, u, u, 0, ws, None)
    assert rc == C.COSMOS_EINVAL and "nsteps 0 < 1" in C.last_error()
    base = 0x100000
    m = 16 ** 3 * 8
    us, s, wss, sws = (ctypes.c_void_p(base), ctypes.c_void_p(base + 25 * m), ctypes.c_void_p(base + 64 * m),
                       ctypes.c_void_p(base + 128 * m))
    rc = lib.cosmos_rk4_steps_scalar(G, Pp, 0.0, 0.1, -1, us, s, wss, sws, None)
    assert rc == C.COSMOS_EINVAL and "nsteps -1" in C.last_error()


def test_out_of_place_step_validates_on_host(C):
    g = C.make_grid(16, 4.0)
    p = C.make_params()
    lib = C.lib
    n = 25 * 16 ** 3 * 8
    u, nxt, stages = ctypes.c_void_p(0x10000000), ctypes.c_void_p(0x20000000), ctypes.c_void_p(0x30000000)
    ws = ctypes.c_void_p(0x40000000)
    G, Pp = ctypes.byref(g), ctypes.byref(p)
    rc = lib.cosmos_rk4_step_stages_to(G, Pp, 0.0, 0.1, u, None, stages, ws, None)
    assert rc == C.COSMOS_EINVAL and "u_next is NULL" in C.last_error()
    rc = lib.cosmos_rk4_step_stages_to(G, Pp, 0.0, 0.1, u, ctypes.c_void_p(0x10000000 + n // 2), stages, ws, None)
    assert rc == C.COSMOS_EINVAL and "must not overlap" in C.last_error()
    rc = lib.cosmos_rk4_step_stages_to(G, Pp, 0.0, 0.1, u, nxt, ctypes.c_void_p(0x20000000 + 8), ws, None)
    assert rc == C.COSMOS_EINVAL and "must not overlap" in C.last_error()
    assert lib.cosmos_rk4_step_stages_to(G, Pp, 0.0, -0.1, u, nxt, stages, ws, None) == C.COSMOS_EINVAL
