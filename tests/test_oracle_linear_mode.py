"""The oracle against linear perturbation theory for a single sinusoidal mode (paper, "Examples":
the evolution of trace K for a small sinusoidal fluctuation, compared with the linear perturbation
solution). The theory (tests/linear_mode.py) is the linearised ADM system on the radiation FLRW
background in the evolved gauge, integrated to 1e-12; the oracle runs the full nonlinear BSSN +
fluid evolution of zeta = mu sin(2 pi x / L) on an (N, 8, 8) box. The mode amplitudes of K, the
lapse and the shift must converge to the theory at 4th order in the grid spacing."""
import numpy as np
import pytest

from tests import linear_mode as lm

L, H0, ETA, MU, T_END = 10.0, 1.0, 1.0, 1e-4, 6.0


def test_linear_theory_preserves_its_constraints():
    k = 2.0 * np.pi / L
    ts = np.linspace(0.25, 8.0, 32)
    r = lm.solve(k, H0, ETA, ts)
    scale = np.abs(r["dK"]).max()
    assert np.abs(r["ham"]).max() < 1e-10 * max(1.0, scale * 16.0 * np.pi)
    assert np.abs(r["mom"]).max() < 1e-10


def oracle_modes(orc, N, nsamp=12):
    s = orc.Setup(n=(N, 8, 8), L=(L, 8 * L / N, 8 * L / N), H0=H0, eta=ETA)
    u = orc.init_fields(s, orc.Init(mu=MU, profile=orc.SINE))
    dt = 0.25 * s.h[0]
    nsteps = int(round(T_END / dt))
    every = nsteps // nsamp
    ts, got = [], {"dK": [], "phi": [], "B": []}
    t = 0.0
    for m in range(nsamp):
        u, pf = orc.rk4(s, u, t, dt, every, parallel=True)
        assert pf == 0
        t += every * dt
        ts.append(t)
        a = lm.mode_amplitudes(u, N, MU, orc.TRK, orc.ALP, orc.BET)
        for q in got:
            got[q].append(a[q])
    return np.array(ts), {q: np.array(v) for q, v in got.items()}


def test_single_mode_converges_to_linear_theory(orc):
    k = 2.0 * np.pi / L
    err = {}
    for N in (32, 64):
        ts, got = oracle_modes(orc, N)
        ref = lm.solve(k, H0, ETA, ts)
        err[N] = {q: np.abs(got[q] - ref[q]).max() / np.abs(ref[q]).max() for q in got}
        print(N, {q: f"{e:.3e}" for q, e in err[N].items()})
    for q in ("dK", "phi", "B"):
        ratio = err[32][q] / err[64][q]
        assert 11.0 < ratio < 22.0, (q, err)   # 4th order: 16
        assert err[64][q] < 2e-5, (q, err)
