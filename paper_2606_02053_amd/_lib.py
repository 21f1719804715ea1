"""ctypes binding of libcosmos.so (include/cosmos.h): argument marshalling only.

Every compute step runs in the library's HIP kernels; PyTorch only provides
device memory (tensors) and the stream. There is no CPU fallback: if the
library is missing, importing the binding raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcosmos.so")
NFIELDS = 25

COSMOS_OK, COSMOS_EINVAL, COSMOS_EHIP, COSMOS_ENOMEM, COSMOS_ENONFINITE, COSMOS_EPRIM, COSMOS_EUNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6


class CosmosError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"cosmos error {code}: {msg}")
        self.code = code


class cosmos_grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("L", ctypes.c_double * 3)]


class cosmos_params(ctypes.Structure):
    _fields_ = [("w", ctypes.c_double), ("H0", ctypes.c_double), ("eta", ctypes.c_double),
                ("ko_eps", ctypes.c_double), ("lapse_bg", ctypes.c_int32), ("evolve_shift", ctypes.c_int32),
                ("fluid_scheme", ctypes.c_int32), ("variant", ctypes.c_int32), ("alpha_collapse", ctypes.c_double),
                ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32), ("tile_z", ctypes.c_int32),
                ("tile_order", ctypes.c_int32)]


class cosmos_init(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_double), ("sigma", ctypes.c_double), ("center", ctypes.c_double * 3),
                ("noise_amp", ctypes.c_double), ("seed", ctypes.c_uint64), ("profile", ctypes.c_int32),
                ("density_mode", ctypes.c_int32)]


class cosmos_batch(ctypes.Structure):
    _fields_ = [("nruns", ctypes.c_int32), ("n", ctypes.POINTER(ctypes.c_int32)),
                ("L", ctypes.POINTER(ctypes.c_double)), ("state_off", ctypes.POINTER(ctypes.c_int64))]


class cosmos_box(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_int32 * 3), ("m", ctypes.c_int32 * 3)]


COSMOS_FMR_BUFFER = 12


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build() (or python "
                          f"paper_2606_02053_amd/build.py); there is no CPU fallback")
    L = ctypes.CDLL(LIB_PATH)
    P, sz, i32, f64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_double
    G, Pr, In, B = (ctypes.POINTER(cosmos_grid), ctypes.POINTER(cosmos_params), ctypes.POINTER(cosmos_init),
                    ctypes.POINTER(cosmos_batch))
    sigs = {
        "cosmos_workspace_bytes": ([G], sz),
        "cosmos_status_reset": ([P, P], i32),
        "cosmos_status": ([P, P, ctypes.POINTER(ctypes.c_int64)], i32),
        "cosmos_init_fields": ([G, Pr, In, P, P], i32),
        "cosmos_init_tangent": ([G, Pr, In, i32, P, P], i32),
        "cosmos_rhs": ([G, Pr, f64, P, P, P, P], i32),
        "cosmos_kt_divergence": ([G, Pr, P, P, P], i32),
        "cosmos_rk4_step": ([G, Pr, f64, f64, P, P, P], i32),
        "cosmos_rk4_steps": ([G, Pr, f64, f64, i32, P, P, P], i32),
        "cosmos_rk4_steps_stages": ([G, Pr, f64, f64, i32, P, P, P, P, P], i32),
        "cosmos_rk4_step_stages": ([G, Pr, f64, f64, P, P, P, P], i32),
        "cosmos_rk4_step_stages_to": ([G, Pr, f64, f64, P, P, P, P, P], i32),
        "cosmos_constraints": ([G, Pr, P, P, P, P, P, P], i32),
        "cosmos_constraints_noalloc": ([G, Pr, P, P, P, P, P], i32),
        "cosmos_adjoint_step": ([G, Pr, f64, f64, P, P, P, P, P], i32),
        "cosmos_adjoint_step_stages": ([G, Pr, f64, f64, P, P, P, P, P, P], i32),
        "cosmos_adjoint_workspace_bytes": ([G], sz),
        "cosmos_rhs_vjp": ([G, Pr, f64, P, P, P, P, P], i32),
        "cosmos_adjoint_gradient": ([G, Pr, In, P, P, P, P], i32),
        "cosmos_batch_workspace_bytes": ([B], sz),
        "cosmos_batch_setup": ([B, Pr, P, P], i32),
        "cosmos_rk4_step_batched": ([B, Pr, P, P, P, P, P], i32),
        "cosmos_rk4_steps_batched": ([B, Pr, P, P, P, i32, P, P], i32),
        "cosmos_batch_status": ([B, P, P, ctypes.POINTER(ctypes.c_int64)], i32),
        "cosmos_batch_outcomes": ([B, P, P, P, P], i32),
        "cosmos_batch_scalar_workspace_bytes": ([B], sz),
        "cosmos_rk4_step_batched_scalar": ([B, Pr, P, P, P, P, P, P, P], i32),
        "cosmos_scalar_workspace_bytes": ([G], sz),
        "cosmos_init_fields_scalar": ([G, Pr, In, f64, f64, P, P, P], i32),
        "cosmos_rhs_scalar": ([G, Pr, f64, P, P, P, P, P, P, P], i32),
        "cosmos_rk4_step_scalar": ([G, Pr, f64, f64, P, P, P, P, P], i32),
        "cosmos_rk4_steps_scalar": ([G, Pr, f64, f64, i32, P, P, P, P, P], i32),
        "cosmos_constraints_scalar": ([G, Pr, P, P, P, P, P, P, P, P], i32),
        "cosmos_fmr_child_grid": ([G, ctypes.POINTER(cosmos_box), G], i32),
        "cosmos_fmr_workspace_bytes": ([G, ctypes.POINTER(cosmos_box)], sz),
        "cosmos_fmr_prolong": ([G, ctypes.POINTER(cosmos_box), P, P, P, f64, ctypes.c_int32, P, P, P], i32),
        "cosmos_fmr_restrict": ([G, ctypes.POINTER(cosmos_box), P, P, P], i32),
        "cosmos_last_error": ([], ctypes.c_char_p),
        "cosmos_abi_version": ([], i32),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(L, name, None)
        if fn is None:
            continue
        fn.argtypes = args
        fn.restype = res
    return L


lib = _load()


def last_error() -> str:
    return lib.cosmos_last_error().decode()


def _check(rc: int):
    if rc < 0:
        raise CosmosError(rc, last_error())
    return rc


def _dev(t: torch.Tensor | None, name: str, numel: int | None = None, dtype=torch.float64):
    """Pointer of a contiguous device tensor (None -> NULL)."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise CosmosError(COSMOS_EINVAL, f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise CosmosError(COSMOS_EINVAL, f"{name} must be a contiguous {dtype} tensor")
    if numel is not None and t.numel() < numel:
        raise CosmosError(COSMOS_EINVAL, f"{name} has {t.numel()} elements, needs {numel}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def make_grid(n, L) -> cosmos_grid:
    n = (n, n, n) if isinstance(n, int) else tuple(n)
    L = (L, L, L) if isinstance(L, (int, float)) else tuple(L)
    g = cosmos_grid()
    g.n[:] = [int(x) for x in n]
    g.L[:] = [float(x) for x in L]
    return g


def make_params(w=1.0 / 3.0, H0=1.0, eta=1.0, ko_eps=0.1, lapse_bg=1, evolve_shift=1, fluid_scheme=0,
                alpha_collapse=0.0, tile=(0, 0, 0), tile_order=2, variant=0) -> cosmos_params:
    """Defaults: radiation (w = 1/3), H0 = 1, Gamma-driver eta = 1, KO eps = 0.1, background-
    subtracted 1+log lapse, evolved shift; LDS-staged kernel, 16x4x4 bricks, XCD-blocked order."""
    return cosmos_params(w, H0, eta, ko_eps, lapse_bg, evolve_shift, fluid_scheme, variant, alpha_collapse,
                         int(tile[0]), int(tile[1]), int(tile[2]), int(tile_order))


def make_init(mu=0.1, sigma=1.0, center=(0.0, 0.0, 0.0), noise_amp=0.0, seed=2606, profile=0,
              density_mode=0) -> cosmos_init:
    c = cosmos_init()
    c.mu, c.sigma, c.noise_amp, c.seed, c.profile, c.density_mode = mu, sigma, noise_amp, seed, profile, density_mode
    c.center[:] = [float(x) for x in center]
    return c


def npts(g: cosmos_grid) -> int:
    return g.n[0] * g.n[1] * g.n[2]


# ---------------------------------------------------------------- the C-ABI entry points
def cosmos_workspace_bytes(grid: cosmos_grid) -> int:
    return int(lib.cosmos_workspace_bytes(ctypes.byref(grid)))


def cosmos_status_reset(ws: torch.Tensor, stream=None):
    _check(lib.cosmos_status_reset(_dev(ws, "ws", dtype=torch.uint8), _stream(stream)))


def cosmos_status(ws: torch.Tensor, stream=None):
    out = (ctypes.c_int64 * 4)()
    _check(lib.cosmos_status(_dev(ws, "ws", dtype=torch.uint8), _stream(stream), out))
    return {"nonfinite": out[0], "prim_fail": out[1], "collapsed": out[2], "steps": out[3]}


def cosmos_init_fields(grid, params, init, u: torch.Tensor, stream=None):
    _check(lib.cosmos_init_fields(ctypes.byref(grid), ctypes.byref(params), ctypes.byref(init),
                                  _dev(u, "u", NFIELDS * npts(grid)), _stream(stream)))


def cosmos_init_tangent(grid, params, init, which: int, du0: torch.Tensor, stream=None):
    _check(lib.cosmos_init_tangent(ctypes.byref(grid), ctypes.byref(params), ctypes.byref(init), int(which),
                                   _dev(du0, "du0", NFIELDS * npts(grid)), _stream(stream)))


def cosmos_adjoint_gradient(grid, params, init, lam0: torch.Tensor, grad_dev: torch.Tensor, ws, stream=None):
    _check(lib.cosmos_adjoint_gradient(ctypes.byref(grid), ctypes.byref(params), ctypes.byref(init),
                                       _dev(lam0, "lam0", NFIELDS * npts(grid)), _dev(grad_dev, "grad_dev", 2),
                                       _dev(ws, "ws", cosmos_adjoint_workspace_bytes(grid), dtype=torch.uint8),
                                       _stream(stream)))


def cosmos_rhs(grid, params, t: float, u, dudt, ws, stream=None):
    N = NFIELDS * npts(grid)
    _check(lib.cosmos_rhs(ctypes.byref(grid), ctypes.byref(params), float(t), _dev(u, "u", N),
                          _dev(dudt, "dudt", N), _dev(ws, "ws", dtype=torch.uint8), _stream(stream)))


def cosmos_kt_divergence(grid, params, u, div, stream=None):
    n = npts(grid)
    _check(lib.cosmos_kt_divergence(ctypes.byref(grid), ctypes.byref(params), _dev(u, "u", NFIELDS * n),
                                    _dev(div, "div", 4 * n), _stream(stream)))


def cosmos_rk4_step(grid, params, t: float, dt: float, u, ws, stream=None):
    _check(lib.cosmos_rk4_step(ctypes.byref(grid), ctypes.byref(params), float(t), float(dt),
                               _dev(u, "u", NFIELDS * npts(grid)), _dev(ws, "ws", cosmos_workspace_bytes(grid),
                                                                        dtype=torch.uint8), _stream(stream)))


def cosmos_rk4_steps(grid, params, t: float, dt: float, nsteps: int, u, ws, stream=None):
    _check(lib.cosmos_rk4_steps(ctypes.byref(grid), ctypes.byref(params), float(t), float(dt), int(nsteps),
                                _dev(u, "u", NFIELDS * npts(grid)), _dev(ws, "ws", cosmos_workspace_bytes(grid),
                                                                         dtype=torch.uint8), _stream(stream)))


def cosmos_rk4_steps_stages(grid, params, t: float, dt: float, nsteps: int, u, states, stages, ws, stream=None):
    N = NFIELDS * npts(grid)
    _check(lib.cosmos_rk4_steps_stages(ctypes.byref(grid), ctypes.byref(params), float(t), float(dt), int(nsteps),
                                       _dev(u, "u", N), _dev(states, "states", int(nsteps) * N),
                                       _dev(stages, "stages", 3 * int(nsteps) * N),
                                       _dev(ws, "ws", cosmos_workspace_bytes(grid), dtype=torch.uint8),
                                       _stream(stream)))


def cosmos_rk4_step_stages(grid, params, t: float, dt: float, u, stages, ws, stream=None):
    N = NFIELDS * npts(grid)
    _check(lib.cosmos_rk4_step_stages(ctypes.byref(grid), ctypes.byref(params), float(t), float(dt), _dev(u, "u", N),
                                      _dev(stages, "stages", 3 * N),
                                      _dev(ws, "ws", cosmos_workspace_bytes(grid), dtype=torch.uint8),
                                      _stream(stream)))


def cosmos_rk4_step_stages_to(grid, params, t: float, dt: float, u, u_next, stages, ws, stream=None):
    N = NFIELDS * npts(grid)
    _check(lib.cosmos_rk4_step_stages_to(ctypes.byref(grid), ctypes.byref(params), float(t), float(dt),
                                         _dev(u, "u", N), _dev(u_next, "u_next", N), _dev(stages, "stages", 3 * N),
                                         _dev(ws, "ws", cosmos_workspace_bytes(grid), dtype=torch.uint8),
                                         _stream(stream)))


def cosmos_constraints(grid, params, u, norms_dev, H_out=None, M_out=None, ws=None, stream=None):
    N3 = npts(grid)
    _check(lib.cosmos_constraints(ctypes.byref(grid), ctypes.byref(params), _dev(u, "u", NFIELDS * N3),
                                  _dev(norms_dev, "norms_dev", 8), _dev(H_out, "H_out", N3),
                                  _dev(M_out, "M_out", 3 * N3),
                                  _dev(ws, "ws", cosmos_workspace_bytes(grid), dtype=torch.uint8), _stream(stream)))


def cosmos_constraints_noalloc(grid, params, u, norms_dev, H_out=None, M_out=None, stream=None):
    N3 = npts(grid)
    _check(lib.cosmos_constraints_noalloc(ctypes.byref(grid), ctypes.byref(params), _dev(u, "u", NFIELDS * N3),
                                          _dev(norms_dev, "norms_dev", 8), _dev(H_out, "H_out", N3),
                                          _dev(M_out, "M_out", 3 * N3), _stream(stream)))


# ---- massless scalar field: s is a (2, nz, ny, nx) float64 device tensor (phi, Pi)
def cosmos_scalar_workspace_bytes(grid: cosmos_grid) -> int:
    return int(lib.cosmos_scalar_workspace_bytes(ctypes.byref(grid)))


def cosmos_init_fields_scalar(grid, params, init, sc_mu: float, sc_sigma: float, u, s, stream=None):
    n = npts(grid)
    _check(lib.cosmos_init_fields_scalar(ctypes.byref(grid), ctypes.byref(params), ctypes.byref(init), float(sc_mu),
                                         float(sc_sigma), _dev(u, "u", NFIELDS * n), _dev(s, "s", 2 * n),
                                         _stream(stream)))


def cosmos_rhs_scalar(grid, params, t: float, u, s, dudt, dsdt, ws, sws, stream=None):
    n = npts(grid)
    _check(lib.cosmos_rhs_scalar(ctypes.byref(grid), ctypes.byref(params), float(t), _dev(u, "u", NFIELDS * n),
                                 _dev(s, "s", 2 * n), _dev(dudt, "dudt", NFIELDS * n), _dev(dsdt, "dsdt", 2 * n),
                                 _dev(ws, "ws", cosmos_workspace_bytes(grid), dtype=torch.uint8),
                                 _dev(sws, "sws", cosmos_scalar_workspace_bytes(grid), dtype=torch.uint8),
                                 _stream(stream)))


def cosmos_rk4_step_scalar(grid, params, t: float, dt: float, u, s, ws, sws, stream=None):
    n = npts(grid)
    _check(lib.cosmos_rk4_step_scalar(ctypes.byref(grid), ctypes.byref(params), float(t), float(dt),
                                      _dev(u, "u", NFIELDS * n), _dev(s, "s", 2 * n),
                                      _dev(ws, "ws", cosmos_workspace_bytes(grid), dtype=torch.uint8),
                                      _dev(sws, "sws", cosmos_scalar_workspace_bytes(grid), dtype=torch.uint8),
                                      _stream(stream)))


def cosmos_rk4_steps_scalar(grid, params, t: float, dt: float, nsteps: int, u, s, ws, sws, stream=None):
    n = npts(grid)
    _check(lib.cosmos_rk4_steps_scalar(ctypes.byref(grid), ctypes.byref(params), float(t), float(dt), int(nsteps),
                                       _dev(u, "u", NFIELDS * n), _dev(s, "s", 2 * n),
                                       _dev(ws, "ws", cosmos_workspace_bytes(grid), dtype=torch.uint8),
                                       _dev(sws, "sws", cosmos_scalar_workspace_bytes(grid), dtype=torch.uint8),
                                       _stream(stream)))


def cosmos_constraints_scalar(grid, params, u, s, norms_dev, H_out=None, M_out=None, ws=None, sws=None, stream=None):
    n = npts(grid)
    _check(lib.cosmos_constraints_scalar(ctypes.byref(grid), ctypes.byref(params), _dev(u, "u", NFIELDS * n),
                                         _dev(s, "s", 2 * n), _dev(norms_dev, "norms_dev", 8),
                                         _dev(H_out, "H_out", n), _dev(M_out, "M_out", 3 * n),
                                         _dev(ws, "ws", cosmos_workspace_bytes(grid), dtype=torch.uint8),
                                         _dev(sws, "sws", cosmos_scalar_workspace_bytes(grid), dtype=torch.uint8),
                                         _stream(stream)))


def cosmos_adjoint_workspace_bytes(grid: cosmos_grid) -> int:
    return int(lib.cosmos_adjoint_workspace_bytes(ctypes.byref(grid)))


def cosmos_adjoint_step(grid, params, t: float, dt: float, u_n, lam_np1, lam_n, ws, stream=None):
    N = NFIELDS * npts(grid)
    _check(lib.cosmos_adjoint_step(ctypes.byref(grid), ctypes.byref(params), float(t), float(dt), _dev(u_n, "u_n", N),
                                   _dev(lam_np1, "lam_np1", N), _dev(lam_n, "lam_n", N),
                                   _dev(ws, "ws", cosmos_adjoint_workspace_bytes(grid), dtype=torch.uint8),
                                   _stream(stream)))


def cosmos_adjoint_step_stages(grid, params, t: float, dt: float, u_n, stages, lam_np1, lam_n, ws, stream=None):
    N = NFIELDS * npts(grid)
    _check(lib.cosmos_adjoint_step_stages(ctypes.byref(grid), ctypes.byref(params), float(t), float(dt),
                                          _dev(u_n, "u_n", N), _dev(stages, "stages", 3 * N),
                                          _dev(lam_np1, "lam_np1", N), _dev(lam_n, "lam_n", N),
                                          _dev(ws, "ws", cosmos_adjoint_workspace_bytes(grid), dtype=torch.uint8),
                                          _stream(stream)))


def cosmos_rhs_vjp(grid, params, t: float, u, kbar, ubar, ws, stream=None):
    N = NFIELDS * npts(grid)
    _check(lib.cosmos_rhs_vjp(ctypes.byref(grid), ctypes.byref(params), float(t), _dev(u, "u", N),
                              _dev(kbar, "kbar", N), _dev(ubar, "ubar", N),
                              _dev(ws, "ws", cosmos_adjoint_workspace_bytes(grid), dtype=torch.uint8),
                              _stream(stream)))


def cosmos_abi_version() -> int:
    return int(lib.cosmos_abi_version())


# ---------------------------------------------------------------- batched form
def make_batch(n_list, L_list, off_list):
    """cosmos_batch plus the ctypes arrays it points to (kept alive on the struct)."""
    k = len(n_list)
    b = cosmos_batch()
    b._n = (ctypes.c_int32 * k)(*[int(x) for x in n_list])
    b._L = (ctypes.c_double * k)(*[float(x) for x in L_list])
    b._off = (ctypes.c_int64 * k)(*[int(x) for x in off_list])
    b.nruns = k
    b.n = ctypes.cast(b._n, ctypes.POINTER(ctypes.c_int32))
    b.L = ctypes.cast(b._L, ctypes.POINTER(ctypes.c_double))
    b.state_off = ctypes.cast(b._off, ctypes.POINTER(ctypes.c_int64))
    return b


def cosmos_batch_workspace_bytes(batch) -> int:
    return int(lib.cosmos_batch_workspace_bytes(ctypes.byref(batch)))


def cosmos_batch_setup(batch, params, bws, stream=None):
    _check(lib.cosmos_batch_setup(ctypes.byref(batch), ctypes.byref(params),
                                  _dev(bws, "bws", cosmos_batch_workspace_bytes(batch), dtype=torch.uint8),
                                  _stream(stream)))


def cosmos_rk4_step_batched(batch, params, arena, t_dev, dt_dev, bws, stream=None):
    _check(lib.cosmos_rk4_step_batched(ctypes.byref(batch), ctypes.byref(params), _dev(arena, "arena"),
                                       _dev(t_dev, "t_dev", batch.nruns), _dev(dt_dev, "dt_dev", batch.nruns),
                                       _dev(bws, "bws", cosmos_batch_workspace_bytes(batch), dtype=torch.uint8),
                                       _stream(stream)))


def cosmos_rk4_steps_batched(batch, params, arena, t_dev, dt_dev, nsteps: int, bws, stream=None):
    _check(lib.cosmos_rk4_steps_batched(ctypes.byref(batch), ctypes.byref(params), _dev(arena, "arena"),
                                        _dev(t_dev, "t_dev", batch.nruns), _dev(dt_dev, "dt_dev", batch.nruns),
                                        int(nsteps),
                                        _dev(bws, "bws", cosmos_batch_workspace_bytes(batch), dtype=torch.uint8),
                                        _stream(stream)))


def cosmos_batch_scalar_workspace_bytes(batch) -> int:
    return int(lib.cosmos_batch_scalar_workspace_bytes(ctypes.byref(batch)))


def cosmos_rk4_step_batched_scalar(batch, params, arena, sarena, t_dev, dt_dev, bws, sbws, stream=None):
    _check(lib.cosmos_rk4_step_batched_scalar(ctypes.byref(batch), ctypes.byref(params), _dev(arena, "arena"),
                                              _dev(sarena, "sarena"), _dev(t_dev, "t_dev", batch.nruns),
                                              _dev(dt_dev, "dt_dev", batch.nruns),
                                              _dev(bws, "bws", cosmos_batch_workspace_bytes(batch), dtype=torch.uint8),
                                              _dev(sbws, "sbws", cosmos_batch_scalar_workspace_bytes(batch),
                                                   dtype=torch.uint8), _stream(stream)))


def cosmos_batch_outcomes(batch, arena, bws, out_dev, stream=None):
    _check(lib.cosmos_batch_outcomes(ctypes.byref(batch), _dev(arena, "arena"),
                                     _dev(bws, "bws", cosmos_batch_workspace_bytes(batch), dtype=torch.uint8),
                                     _dev(out_dev, "out_dev", 2 * batch.nruns), _stream(stream)))


def cosmos_batch_status(batch, bws, stream=None):
    out = (ctypes.c_int64 * (4 * batch.nruns))()
    _check(lib.cosmos_batch_status(ctypes.byref(batch), _dev(bws, "bws", dtype=torch.uint8), _stream(stream), out))
    return [{"nonfinite": out[4 * r], "prim_fail": out[4 * r + 1], "collapsed": out[4 * r + 2],
             "steps": out[4 * r + 3]} for r in range(batch.nruns)]


# ---------------------------------------------------------------- fixed mesh refinement
def make_box(origin, m) -> cosmos_box:
    b = cosmos_box()
    b.origin[:] = [int(x) for x in origin]
    b.m[:] = [int(x) for x in m]
    return b


def cosmos_fmr_child_grid(parent: cosmos_grid, box: cosmos_box) -> cosmos_grid:
    child = cosmos_grid()
    _check(lib.cosmos_fmr_child_grid(ctypes.byref(parent), ctypes.byref(box), ctypes.byref(child)))
    return child


def cosmos_fmr_workspace_bytes(parent: cosmos_grid, box: cosmos_box) -> int:
    return int(lib.cosmos_fmr_workspace_bytes(ctypes.byref(parent), ctypes.byref(box)))


def cosmos_fmr_prolong(parent, box, u_n, stages, u_np1, theta: float, buffer_only: bool, child_u, ws, stream=None):
    Np = NFIELDS * npts(parent)
    child = cosmos_fmr_child_grid(parent, box)
    _check(lib.cosmos_fmr_prolong(ctypes.byref(parent), ctypes.byref(box), _dev(u_n, "u_n", Np),
                                  _dev(stages, "stages", 3 * Np), _dev(u_np1, "u_np1", Np), float(theta),
                                  int(bool(buffer_only)), _dev(child_u, "child_u", NFIELDS * npts(child)),
                                  _dev(ws, "ws", cosmos_fmr_workspace_bytes(parent, box), dtype=torch.uint8),
                                  _stream(stream)))


def cosmos_fmr_restrict(parent, box, child_u, parent_u, stream=None):
    child = cosmos_fmr_child_grid(parent, box)
    _check(lib.cosmos_fmr_restrict(ctypes.byref(parent), ctypes.byref(box),
                                   _dev(child_u, "child_u", NFIELDS * npts(child)),
                                   _dev(parent_u, "parent_u", NFIELDS * npts(parent)), _stream(stream)))
