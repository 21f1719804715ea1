"""CPU check of the HIP path's hand-written vector-Jacobian product of the
pointwise algebra: the library's __host__ __device__ pt_vjp, compiled for the
host by hipcc, against the oracle's taped reverse mode. The fluid-flux reverse
is checked against central finite differences of its own forward and the
forward against the oracle's fluxes."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def H(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("harness") / "pt_harness.so")
    subprocess.run([hipcc, "-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off", "-I",
                    os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2606_02053_amd", "csrc"), "-o",
                    out, os.path.join(ROOT, "tests", "harness", "pt_harness.hip")], check=True,
                   capture_output=True)
    L = ctypes.CDLL(out)
    P = ctypes.c_void_p
    L.harness_pt_vjp.argtypes = [P, P, ctypes.c_double, P, ctypes.c_double, P, P, P]
    L.harness_flux.argtypes = [ctypes.c_double, ctypes.c_int, P, P, P, P]
    return L


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def random_point(orc, rng):
    d = {}
    for name, shp in orc.GEOMIN_LAYOUT:
        d[name] = rng.normal(size=shp) * 0.3 if shp else rng.normal() * 0.3
    d["chi"] = 1.0 + 0.2 * rng.uniform(-1, 1)
    A = rng.normal(size=(3, 3)) * 0.08
    g = np.eye(3) + 0.5 * (A + A.T)
    d["gt"] = np.array([g[0, 0], g[0, 1], g[0, 2], g[1, 1], g[1, 2], g[2, 2]])
    d["alpha"] = 1.0 + 0.2 * rng.uniform(-1, 1)
    d["K"] = -1.0 + 0.3 * rng.uniform(-1, 1)
    Et = 1.0 + 0.2 * rng.uniform(-1, 1)
    St = rng.normal(size=3) * 0.05
    return d, Et, St


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("opts", [dict(), dict(lapse_bg=0, evolve_shift=0), dict(w=0.2, eta=2.0, H0=0.5)])
def test_pointwise_vjp_matches_oracle(orc, H, seed, opts):
    rng = np.random.default_rng(100 + seed)
    s = orc.Setup(**opts)
    n, L, prm, iprm = s.arrays()
    d, Et, St = random_point(orc, rng)
    packed = orc.pack_geomin(d)
    t = 0.3
    rbar = rng.normal(size=25)
    out = np.empty(packed.size + 4)
    rc = H.harness_pt_vjp(_p(prm), _p(iprm), t, _p(packed), Et, _p(np.ascontiguousarray(St)), _p(rbar), _p(out))
    assert rc == out.size  # every input cotangent handed over exactly once
    tape = orc.point_rhs_vjp(s, d, Et, St, rbar, t=t)
    # the constraint-only inputs (dAt) have no cotangent in either
    scale = np.abs(tape).max()
    err = np.abs(out - tape)
    assert err.max() < 1e-12 * scale, (int(err.argmax()), out[err.argmax()], tape[err.argmax()])


def test_pointwise_reverse_invalid_fluid_branch(orc, H):
    # E <= 0 takes the invalid-state branch (P = 0, 1/X = 0) in both
    rng = np.random.default_rng(7)
    s = orc.Setup()
    _, _, prm, iprm = s.arrays()
    d, _, St = random_point(orc, rng)
    packed = orc.pack_geomin(d)
    for Et, St_ in ((-0.3, St), (1.0, np.array([3.0, 0.0, 0.0]))):
        rbar = rng.normal(size=25)
        out = np.empty(packed.size + 4)
        H.harness_pt_vjp(_p(prm), _p(iprm), 0.0, _p(packed), Et, _p(np.ascontiguousarray(St_)), _p(rbar), _p(out))
        tape = orc.point_rhs_vjp(s, d, Et, St_, rbar)
        assert np.abs(out - tape).max() < 1e-12 * np.abs(tape).max()


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_flux_forward_and_reverse(orc, H, axis):
    rng = np.random.default_rng(20 + axis)
    s = orc.Setup()
    d, Et, St = random_point(orc, rng)
    u25 = np.zeros(25)
    u25[0] = d["chi"]
    u25[1:7] = d["gt"]
    u25[17] = d["alpha"]
    u25[18:21] = rng.normal(size=3) * 0.2
    u25[21] = Et
    u25[22:25] = St
    u15 = np.concatenate([[u25[0]], u25[1:7], [u25[17], u25[18 + axis], u25[21]], u25[22:25]])
    Fb = rng.normal(size=4)
    F = np.empty(4)
    ub = np.empty(13)
    H.harness_flux(1.0 / 3.0, axis, _p(u15), _p(Fb), _p(F), _p(ub))
    ref = orc.flux_point(s, u25)[4 * axis:4 * axis + 4]
    assert np.allclose(F, ref, rtol=1e-13, atol=1e-15)
    h = 1e-6
    for q in range(13):
        e = np.zeros(13)
        e[q] = h
        Fp, Fm = np.empty(4), np.empty(4)
        H.harness_flux(1.0 / 3.0, axis, _p(u15 + e), _p(Fb), _p(Fp), _p(np.empty(13)))
        H.harness_flux(1.0 / 3.0, axis, _p(u15 - e), _p(Fb), _p(Fm), _p(np.empty(13)))
        fd = Fb @ (Fp - Fm) / (2 * h)
        assert ub[q] == pytest.approx(fd, rel=1e-6, abs=1e-8), q
