"""CPU oracle for the COSMOS evolution hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package. The product path (the HIP library and
its Python binding in ``paper_2606_02053_amd``) never imports, links or calls
anything here, and nothing here imports the product path.

The arithmetic lives in ``cosmos_oracle.hpp`` (a plain serial FP64 C++
statement of the method, templated on the scalar type so the same text also
yields forward tangents, a taped discrete adjoint and operation counts). This
module is a thin ctypes wrapper around ``liboracle.so`` built from it.

Paper passages followed (the paper's sections; its equations are unnumbered):
  * "Physical system settings": Einstein equations, perfect-fluid stress tensor,
    linear equation of state P = w rho, fluid equation of motion, and the
    initial-data paragraph (curvature perturbation zeta(x), constraint-satisfying
    fluid distribution, no elliptic solver);
  * "Statement of need" / "Examples": periodic box of size L.
Parameter conventions: ``prm = (w, H0, eta, ko_eps)``, ``iprm = (lapse_bg,
evolve_shift, fluid_scheme)``; states are float64 arrays of shape (25, nz, ny, nx).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = [os.path.join(_HERE, "oracle_capi.cpp")]
_HDR = [os.path.join(_HERE, "cosmos_oracle.hpp"), os.path.join(_HERE, "ad.hpp")]

NF = 25
FIELDS = (["chi"] + [f"gt{c}" for c in ("xx", "xy", "xz", "yy", "yz", "zz")] + ["K"]
          + [f"At{c}" for c in ("xx", "xy", "xz", "yy", "yz", "zz")] + ["Gtx", "Gty", "Gtz", "alpha"]
          + ["betax", "betay", "betaz", "Et", "Stx", "Sty", "Stz"])
CHI, GT, TRK, AT, GAM, ALP, BET, ET, ST = 0, 1, 7, 8, 14, 17, 18, 21, 22
GAUSS, SINE, PGAUSS = 0, 1, 2
HAMILTONIAN, LITERAL = 0, 1


def build(verbose: bool = False) -> str:
    """Compile liboracle.so with g++ (serial FP64, no FP contraction)."""
    cmd = ["g++", "-std=c++17", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wno-unused-variable", "-Wno-maybe-uninitialized",
           "-o", _LIB_PATH + ".tmp", *_SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i32, i64, f64, u64 = ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64
        sig = {
            "oracle_rhs": [P, P, P, P, f64, P, P, P, i32],
            "oracle_rk4_steps": [P, P, P, P, f64, f64, i32, P, P, i32],
            "oracle_rhs_at_points": [P, P, P, P, f64, P, P, i32, P],
            "oracle_rk4_at_points": [P, P, P, P, f64, f64, P, P, i32, P],
            "oracle_constraints": [P, P, P, P, P, P, P, P, i32],
            "oracle_init": [P, P, P, P, P, u64, i32, i32, P],
            "oracle_init_at_points": [P, P, P, P, P, u64, i32, i32, P, i32, P],
            "oracle_init_tangent": [P, P, P, P, P, u64, i32, i32, i32, P],
            "oracle_jvp": [P, P, P, P, i32, f64, f64, P, P, P, P],
            "oracle_vjp": [P, P, P, P, i32, f64, f64, P, P, P],
            "oracle_count_flops": [P, P, P, P, P, P],
            "oracle_geometry_point": [P, P],
            "oracle_point_rhs": [P, P, f64, P, f64, P, P],
            "oracle_matter_point": [f64, f64, P, f64, P, P],
            "oracle_flux_point": [P, P, P],
            "oracle_kt_flux": [P, P, P, i32, P],
            "oracle_rhs_sc": [P, P, P, P, f64, P, P, P, P, P, i32],
            "oracle_rk4_steps_sc": [P, P, P, P, f64, f64, i32, P, P, P, i32],
            "oracle_constraints_sc": [P, P, P, P, P, P, P, P, P, i32],
            "oracle_init_sc": [P, P, P, P, P, P, u64, i32, i32, P, P],
            "oracle_rhs_sc_at_points": [P, P, P, P, f64, P, P, P, i32, P, P],
            "oracle_rk4_sc_at_points": [P, P, P, P, f64, f64, P, P, P, i32, P, P],
            "oracle_kt_divergence": [P, P, P, P, P, P],
            "oracle_count_kt_flops": [P, P, P, P, P, P],
            "oracle_fluid_speeds": [P, P, i32, P],
            "oracle_splitmix64": [u64, u64],
            "oracle_stencil": [P, P, P, i32, i32, i32, i32, i32, i32, P, f64, P],
            "oracle_gamma_constraint": [P, P, P, P],
            "oracle_point_rhs_vjp": [P, P, f64, P, f64, P, P, P],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_uint64 if name == "oracle_splitmix64" else ctypes.c_int
        L.oracle_geomin_size.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


@dataclass
class Setup:
    """Grid and evolution parameters. n = (nx, ny, nz), L = (Lx, Ly, Lz)."""
    n: tuple = (32, 32, 32)
    L: tuple = (10.0, 10.0, 10.0)
    w: float = 1.0 / 3.0
    H0: float = 1.0
    eta: float = 1.0
    ko_eps: float = 0.1
    lapse_bg: int = 1
    evolve_shift: int = 1
    fluid_scheme: int = 0  # 0: centred flux divergence + KO; 1: Kurganov-Tadmor fluxes

    def arrays(self):
        return (np.ascontiguousarray(self.n, dtype=np.int32), np.ascontiguousarray(self.L, dtype=np.float64),
                np.array([self.w, self.H0, self.eta, self.ko_eps], dtype=np.float64),
                np.array([self.lapse_bg, self.evolve_shift, self.fluid_scheme], dtype=np.int32))

    @property
    def shape(self):
        return (NF, self.n[2], self.n[1], self.n[0])

    @property
    def h(self):
        return tuple(self.L[a] / self.n[a] for a in range(3))


@dataclass
class Init:
    mu: float = 0.1
    sigma: float = 1.0
    center: tuple = (0.0, 0.0, 0.0)
    noise_amp: float = 0.0
    seed: int = 2606
    profile: int = GAUSS
    density_mode: int = HAMILTONIAN

    def array(self):
        return np.array([self.mu, self.sigma, *self.center, self.noise_amp], dtype=np.float64)


def _check(rc, name):
    if rc != 0:
        raise ValueError(f"{name} rejected its arguments (rc={rc})")


def _state(u, s: Setup):
    u = np.ascontiguousarray(u, dtype=np.float64)
    if u.shape != s.shape:
        raise ValueError(f"state shape {u.shape} != {s.shape}")
    return u


def init_fields(s: Setup, ini: Init) -> np.ndarray:
    n, L, prm, iprm = s.arrays()
    u = np.empty(s.shape)
    _check(lib().oracle_init(_p(n), _p(L), _p(prm), _p(iprm), _p(ini.array()), ini.seed, ini.profile,
                             ini.density_mode, _p(u)), "oracle_init")
    return u


def init_at_points(s: Setup, ini: Init, pts) -> np.ndarray:
    n, L, prm, iprm = s.arrays()
    pts = np.ascontiguousarray(pts, dtype=np.int64)
    out = np.empty((len(pts), NF))
    _check(lib().oracle_init_at_points(_p(n), _p(L), _p(prm), _p(iprm), _p(ini.array()), ini.seed, ini.profile,
                                       ini.density_mode, _p(pts), len(pts), _p(out)), "oracle_init_at_points")
    return out


def init_tangent(s: Setup, ini: Init, which: int) -> np.ndarray:
    n, L, prm, iprm = s.arrays()
    du = np.empty(s.shape)
    _check(lib().oracle_init_tangent(_p(n), _p(L), _p(prm), _p(iprm), _p(ini.array()), ini.seed, ini.profile,
                                     ini.density_mode, which, _p(du)), "oracle_init_tangent")
    return du


def rhs(s: Setup, u, t: float = 0.0, parallel: bool = False):
    """Discrete right-hand side du/dt on the periodic grid. Returns (dudt, prim_fail)."""
    n, L, prm, iprm = s.arrays()
    u = _state(u, s)
    out = np.empty_like(u)
    pf = ctypes.c_int64(0)
    _check(lib().oracle_rhs(_p(n), _p(L), _p(prm), _p(iprm), t, _p(u), _p(out), ctypes.byref(pf), int(parallel)),
           "oracle_rhs")
    return out, pf.value


def rk4(s: Setup, u, t0: float, dt: float, nsteps: int = 1, parallel: bool = False):
    """nsteps classic RK4 steps from time t0. Returns (u_new, prim_fail)."""
    n, L, prm, iprm = s.arrays()
    v = _state(u, s).copy()
    pf = ctypes.c_int64(0)
    _check(lib().oracle_rk4_steps(_p(n), _p(L), _p(prm), _p(iprm), t0, dt, nsteps, _p(v), ctypes.byref(pf),
                                  int(parallel)), "oracle_rk4_steps")
    return v, pf.value


def rhs_at_points(s: Setup, u, pts, t: float = 0.0) -> np.ndarray:
    n, L, prm, iprm = s.arrays()
    u = _state(u, s)
    pts = np.ascontiguousarray(pts, dtype=np.int64)
    out = np.empty((len(pts), NF))
    _check(lib().oracle_rhs_at_points(_p(n), _p(L), _p(prm), _p(iprm), t, _p(u), _p(pts), len(pts), _p(out)),
           "oracle_rhs_at_points")
    return out


def rk4_at_points(s: Setup, u, pts, t: float, dt: float) -> np.ndarray:
    n, L, prm, iprm = s.arrays()
    u = _state(u, s)
    pts = np.ascontiguousarray(pts, dtype=np.int64)
    out = np.empty((len(pts), NF))
    _check(lib().oracle_rk4_at_points(_p(n), _p(L), _p(prm), _p(iprm), t, dt, _p(u), _p(pts), len(pts), _p(out)),
           "oracle_rk4_at_points")
    return out


def constraints(s: Setup, u, want_fields: bool = False, parallel: bool = False):
    """Returns norms[8] (and H, M arrays when want_fields)."""
    n, L, prm, iprm = s.arrays()
    u = _state(u, s)
    norms = np.empty(8)
    H = np.empty(s.shape[1:]) if want_fields else None
    M = np.empty((3,) + s.shape[1:]) if want_fields else None
    _check(lib().oracle_constraints(_p(n), _p(L), _p(prm), _p(iprm), _p(u), _p(norms), _p(H), _p(M),
                                    int(parallel)), "oracle_constraints")
    return (norms, H, M) if want_fields else norms


def jvp(s: Setup, u, v, what: str = "step", t: float = 0.0, dt: float = 0.0):
    """Forward-mode tangent of the RHS (what='rhs') or of one RK4 step ('step')."""
    n, L, prm, iprm = s.arrays()
    u = _state(u, s)
    v = _state(v, s)
    fu = np.empty_like(u)
    Jv = np.empty_like(u)
    _check(lib().oracle_jvp(_p(n), _p(L), _p(prm), _p(iprm), 0 if what == "rhs" else 1, t, dt, _p(u), _p(v), _p(fu),
                            _p(Jv)), "oracle_jvp")
    return fu, Jv


def vjp(s: Setup, u, lam, what: str = "step", t: float = 0.0, dt: float = 0.0):
    """Reverse-mode (taped) transpose-Jacobian product: the oracle's discrete adjoint."""
    n, L, prm, iprm = s.arrays()
    u = _state(u, s)
    lam = _state(lam, s)
    out = np.empty_like(u)
    _check(lib().oracle_vjp(_p(n), _p(L), _p(prm), _p(iprm), 0 if what == "rhs" else 1, t, dt, _p(u), _p(lam),
                            _p(out)), "oracle_vjp")
    return out


def count_flops(s: Setup, u) -> dict:
    n, L, prm, iprm = s.arrays()
    u = _state(u, s)
    out = np.empty(5)
    _check(lib().oracle_count_flops(_p(n), _p(L), _p(prm), _p(iprm), _p(u), _p(out)), "oracle_count_flops")
    return {"rhs_per_point_excl_flux": out[0], "flux_per_point": out[1], "rk4_combine_per_point": out[2],
            "step_per_point": out[3], "sqrt_per_rhs_point": out[4]}


GEOMIN_LAYOUT = (("chi", ()), ("gt", (6,)), ("K", ()), ("At", (6,)), ("Gam", (3,)), ("alpha", ()), ("beta", (3,)),
                 ("dchi", (3,)), ("d2chi", (6,)), ("dgt", (6, 3)), ("d2gt", (6, 6)), ("dGam", (3, 3)),
                 ("dalpha", (3,)), ("d2alpha", (6,)), ("dbeta", (3, 3)), ("d2beta", (3, 6)), ("dK", (3,)),
                 ("dAt", (6, 3)))


def pack_geomin(d: dict) -> np.ndarray:
    parts = []
    for name, shp in GEOMIN_LAYOUT:
        a = np.asarray(d.get(name, np.zeros(shp)), dtype=np.float64).reshape(shp if shp else ())
        parts.append(a.ravel())
    out = np.concatenate(parts)
    assert out.size == lib().oracle_geomin_size()
    return out


def geometry_point(d: dict) -> dict:
    out = np.empty(17)
    lib().oracle_geometry_point(_p(pack_geomin(d)), _p(out))
    return {"Ric": out[0:6], "R": out[6], "DDalpha": out[7:13], "Gd": out[13:16], "det": out[16]}


def point_rhs(s: Setup, d: dict, Et: float, St, t: float = 0.0):
    _, _, prm, iprm = s.arrays()
    out = np.empty(30)
    St = np.ascontiguousarray(St, dtype=np.float64)
    fail = lib().oracle_point_rhs(_p(prm), _p(iprm), t, _p(pack_geomin(d)), Et, _p(St), _p(out))
    return {"rhs": out[:25], "H": out[25], "M": out[26:29], "Hn": out[29], "fail": bool(fail)}


def matter_point(w, chi, gt, Et, St):
    gt = np.ascontiguousarray(gt, dtype=np.float64)
    St = np.ascontiguousarray(St, dtype=np.float64)
    out = np.empty(11)
    fail = lib().oracle_matter_point(w, chi, _p(gt), Et, _p(St), _p(out))
    return {"E": out[0], "S": out[1:4], "S2": out[4], "P": out[5], "invX": out[6], "Sup": out[7:10],
            "Strace": out[10], "fail": bool(fail)}


def flux_point(s: Setup, u25) -> np.ndarray:
    _, _, prm, _ = s.arrays()
    u25 = np.ascontiguousarray(u25, dtype=np.float64)
    out = np.empty(12)
    lib().oracle_flux_point(_p(prm), _p(u25), _p(out))
    return out


# ---- massless scalar field: sc is a float64 array of shape (2, nz, ny, nx) holding phi, Pi
def _scalar(sc, s: Setup):
    sc = np.ascontiguousarray(sc, dtype=np.float64)
    if sc.shape != (2,) + s.shape[1:]:
        raise ValueError(f"scalar state shape {sc.shape} != {(2,) + s.shape[1:]}")
    return sc


def init_fields_sc(s: Setup, ini: Init, sc_mu: float, sc_sigma: float):
    """Initial data with an iso-curvature mode Upsilon = sc_mu * profile(sc_sigma): returns (u, sc)."""
    n, L, prm, iprm = s.arrays()
    u = np.empty(s.shape)
    sc = np.empty((2,) + s.shape[1:])
    _check(lib().oracle_init_sc(_p(n), _p(L), _p(prm), _p(iprm), _p(ini.array()),
                                _p(np.array([sc_mu, sc_sigma], dtype=np.float64)), ini.seed, ini.profile,
                                ini.density_mode, _p(u), _p(sc)), "oracle_init_sc")
    return u, sc


def rhs_sc(s: Setup, u, sc, t: float = 0.0, parallel: bool = False):
    """Right-hand side with the scalar field. Returns (dudt, dscdt, prim_fail)."""
    n, L, prm, iprm = s.arrays()
    u, sc = _state(u, s), _scalar(sc, s)
    du, ds = np.empty_like(u), np.empty_like(sc)
    pf = ctypes.c_int64(0)
    _check(lib().oracle_rhs_sc(_p(n), _p(L), _p(prm), _p(iprm), t, _p(u), _p(sc), _p(du), _p(ds), ctypes.byref(pf),
                               int(parallel)), "oracle_rhs_sc")
    return du, ds, pf.value


def rk4_sc(s: Setup, u, sc, t0: float, dt: float, nsteps: int = 1, parallel: bool = False):
    """nsteps RK4 steps of (u, sc). Returns (u_new, sc_new, prim_fail)."""
    n, L, prm, iprm = s.arrays()
    v, w = _state(u, s).copy(), _scalar(sc, s).copy()
    pf = ctypes.c_int64(0)
    _check(lib().oracle_rk4_steps_sc(_p(n), _p(L), _p(prm), _p(iprm), t0, dt, nsteps, _p(v), _p(w),
                                     ctypes.byref(pf), int(parallel)), "oracle_rk4_steps_sc")
    return v, w, pf.value


def constraints_sc(s: Setup, u, sc, want_fields: bool = False, parallel: bool = False):
    """Constraint norms (as constraints()) with the scalar field's energy and momentum included."""
    n, L, prm, iprm = s.arrays()
    u, sc = _state(u, s), _scalar(sc, s)
    norms = np.empty(8)
    H = np.empty(s.shape[1:]) if want_fields else None
    M = np.empty((3,) + s.shape[1:]) if want_fields else None
    _check(lib().oracle_constraints_sc(_p(n), _p(L), _p(prm), _p(iprm), _p(u), _p(sc), _p(norms), _p(H), _p(M),
                                       int(parallel)), "oracle_constraints_sc")
    return (norms, H, M) if want_fields else norms


def rhs_sc_at_points(s: Setup, u, sc, pts, t: float = 0.0):
    """Right-hand side with the scalar field at the listed linear indices: ([npts][25], [npts][2])."""
    n, L, prm, iprm = s.arrays()
    u, sc = _state(u, s), _scalar(sc, s)
    pts = np.ascontiguousarray(pts, dtype=np.int64)
    out, sout = np.empty((len(pts), NF)), np.empty((len(pts), 2))
    _check(lib().oracle_rhs_sc_at_points(_p(n), _p(L), _p(prm), _p(iprm), t, _p(u), _p(sc), _p(pts), len(pts),
                                         _p(out), _p(sout)), "oracle_rhs_sc_at_points")
    return out, sout


def rk4_sc_at_points(s: Setup, u, sc, pts, t: float, dt: float):
    """One RK4 step of (u, sc) evaluated at the listed points only: ([npts][25], [npts][2])."""
    n, L, prm, iprm = s.arrays()
    u, sc = _state(u, s), _scalar(sc, s)
    pts = np.ascontiguousarray(pts, dtype=np.int64)
    out, sout = np.empty((len(pts), NF)), np.empty((len(pts), 2))
    _check(lib().oracle_rk4_sc_at_points(_p(n), _p(L), _p(prm), _p(iprm), t, dt, _p(u), _p(sc), _p(pts), len(pts),
                                         _p(out), _p(sout)), "oracle_rk4_sc_at_points")
    return out, sout


def kt_flux(s: Setup, uL, uR, a: int) -> np.ndarray:
    """Kurganov-Tadmor numerical flux along axis a between two interface states (25 values each)."""
    _, _, prm, _ = s.arrays()
    uL = np.ascontiguousarray(uL, dtype=np.float64)
    uR = np.ascontiguousarray(uR, dtype=np.float64)
    out = np.empty(4)
    _check(lib().oracle_kt_flux(_p(prm), _p(uL), _p(uR), a, _p(out)), "oracle_kt_flux")
    return out


def kt_divergence(s: Setup, u) -> np.ndarray:
    """Kurganov-Tadmor flux divergence of (Et, St_x, St_y, St_z), shape (4, nz, ny, nx)."""
    n, L, prm, iprm = s.arrays()
    u = _state(u, s)
    out = np.empty((4,) + s.shape[1:])
    _check(lib().oracle_kt_divergence(_p(n), _p(L), _p(prm), _p(iprm), _p(u), _p(out)), "oracle_kt_divergence")
    return out


def count_kt_flops(s: Setup, u) -> dict:
    """Operations of one Kurganov-Tadmor interface flux (the count depends on the limiter branches)."""
    n, L, prm, iprm = s.arrays()
    u = _state(u, s)
    out = np.empty(3)
    _check(lib().oracle_count_kt_flops(_p(n), _p(L), _p(prm), _p(iprm), _p(u), _p(out)), "oracle_count_kt_flops")
    return {"flops_per_interface": out[0], "sqrt_per_interface": out[1], "oracle_flops_per_interface": out[2]}


def fluid_speeds(s: Setup, u25, a: int) -> tuple:
    """(lambda_minus, lambda_plus), the fluid's characteristic speeds along axis a."""
    _, _, prm, _ = s.arrays()
    u25 = np.ascontiguousarray(u25, dtype=np.float64)
    out = np.empty(2)
    _check(lib().oracle_fluid_speeds(_p(prm), _p(u25), a, _p(out)), "oracle_fluid_speeds")
    return float(out[0]), float(out[1])


def splitmix64(seed: int, p: int) -> int:
    return int(lib().oracle_splitmix64(seed, p))


STENCIL_KINDS = {"d1": 0, "d2": 1, "mixed": 2, "adv": 3, "ko": 4}


def stencil(s: Setup, f, ijk, kind: str, a: int = 0, b: int = 1, beta=(0.0, 0.0, 0.0), eps: float = 0.1) -> float:
    """Apply one of the oracle's difference operators to a single periodic grid
    function f (shape (nz, ny, nx)) at grid point ijk = (i, j, k)."""
    n, L, _, _ = s.arrays()
    f = np.ascontiguousarray(f, dtype=np.float64)
    assert f.shape == s.shape[1:]
    out = np.empty(1)
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    _check(lib().oracle_stencil(_p(n), _p(L), _p(f), int(ijk[0]), int(ijk[1]), int(ijk[2]), STENCIL_KINDS[kind], a, b,
                                _p(beta), eps, _p(out)), "oracle_stencil")
    return float(out[0])


def gamma_constraint(s: Setup, u):
    """(rms, max) over the grid of |Gt^i - gt^jk Gt^i_jk|."""
    n, L, _, _ = s.arrays()
    u = _state(u, s)
    out = np.empty(2)
    _check(lib().oracle_gamma_constraint(_p(n), _p(L), _p(u), _p(out)), "oracle_gamma_constraint")
    return float(out[0]), float(out[1])


def point_rhs_vjp(s: Setup, d: dict, Et: float, St, rbar, t: float = 0.0):
    """Reverse mode (tape) of the pointwise right-hand side: adjoints of the packed
    inputs (GEOMIN_LAYOUT order) followed by those of Et and St."""
    _, _, prm, iprm = s.arrays()
    n = lib().oracle_geomin_size()
    out = np.empty(n + 4)
    St = np.ascontiguousarray(St, dtype=np.float64)
    rbar = np.ascontiguousarray(rbar, dtype=np.float64)
    _check(lib().oracle_point_rhs_vjp(_p(prm), _p(iprm), t, _p(pack_geomin(d)), Et, _p(St), _p(rbar), _p(out)),
           "oracle_point_rhs_vjp")
    return out
