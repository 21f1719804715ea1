"""Linear perturbation theory of one sinusoidal curvature mode on the radiation FLRW background,
in the evolved gauge (paper, "Examples": the single-mode perturbation whose trace K is compared
with the linear perturbation solution). Test infrastructure: plain numpy/scipy, written from the
ADM equations, sharing nothing with the oracle or the HIP library.

Background (unit lapse, zero shift, P = E/3): a^2 = 1 + 2 H0 t, H = H0 / (1 + 2 H0 t),
E = 3 H^2 / (8 pi), K = -3 H.

Perturbation of a plane wave along x with wavenumber k (scalars ~ sin k x, vectors ~ cos k x,
amplitudes per unit zeta amplitude):
  gamma_ij = a^2 (delta_ij + h_ij), h = diag(hL, hT, hT);  K_ij = a^2 (-H delta_ij + k_ij),
  k = diag(kL, kT, kT);  alpha = 1 + phi;  beta^x = B;  E -> E + dE;  S_x = sg.
Linearised ADM evolution (background Christoffel symbols vanish; S - E = 3P - E = 0 to first
order; 8 pi P = H^2) with the lapse condition d_t alpha = -2 alpha (K - K_bg(t)) and the shift
condition d_t beta^i = 3/4 Gt^i - eta beta^i, Gt^x = d_x (2/3)(hL - hT) at first order:
  hL' = 2 H phi - 2 kL - 2 H hL - 2 k B          hT' = 2 H phi - 2 kT - 2 H hT
  kL' = -H kL + H^2 hL - H dK - 8 pi dE/3 + k^2 (phi + hT) / a^2 + 2 H k B
  kT' = -H kT + H^2 hT - H dK - 8 pi dE/3 + k^2 hT / (2 a^2)
  phi' = -2 dK                                   B' = k (hL - hT) / 2 - eta B
  dE' = -4 H E phi + 4/3 E dK - 4 H dE + k sg / a^2
  sg' = -3 H sg - 4/3 E k phi - k dE / 3
with dK = kL + 2 kT + H (hL + 2 hT) the perturbation of the trace K. (The linearised Ricci tensor
of the plane wave is R_xx = -hT'', R_yy = R_zz = -hT''/2; the momentum equation is the 3+1 form of
the fluid's momentum balance, whose static limit is hydrostatic equilibrium.)

Initial data of the code (conformally flat gamma = e^{2 zeta}, K = -3 H0, At = 0, fluid at rest,
E from the Hamiltonian constraint): hL = hT = 2, kL = kT = -2 H0 (K_ij proportional to gamma_ij),
phi = B = sg = 0, dE = k^2 / (4 pi).
The linearised constraints, which the system preserves:
  Hamiltonian  2 k^2 hT / a^2 - 4 H dK - 16 pi dE = 0
  momentum     -2 k (kT + H hT) - 8 pi sg = 0
"""
import numpy as np
from scipy.integrate import solve_ivp


def background(t, H0):
    t = np.asarray(t, dtype=np.float64)
    H = H0 / (1.0 + 2.0 * H0 * t)
    return H, 1.0 + 2.0 * H0 * t, 3.0 * H * H / (8.0 * np.pi)


def solve(k, H0, eta, ts):
    """Mode amplitudes at the times ts (increasing, > 0): dict of dK, phi, B, constraint residuals."""
    def rhs(t, y):
        hL, hT, kL, kT, ph, B, dE, sg = y
        H, a2, E = background(t, H0)
        dK = kL + 2.0 * kT + H * (hL + 2.0 * hT)
        return [2.0 * H * ph - 2.0 * kL - 2.0 * H * hL - 2.0 * k * B,
                2.0 * H * ph - 2.0 * kT - 2.0 * H * hT,
                -H * kL + H * H * hL - H * dK - 8.0 * np.pi * dE / 3.0 + k * k * (ph + hT) / a2 + 2.0 * H * k * B,
                -H * kT + H * H * hT - H * dK - 8.0 * np.pi * dE / 3.0 + 0.5 * k * k * hT / a2,
                -2.0 * dK,
                0.5 * k * (hL - hT) - eta * B,
                -4.0 * H * E * ph + (4.0 / 3.0) * E * dK - 4.0 * H * dE + k * sg / a2,
                -3.0 * H * sg - (4.0 / 3.0) * E * k * ph - k * dE / 3.0]
    y0 = [2.0, 2.0, -2.0 * H0, -2.0 * H0, 0.0, 0.0, k * k / (4.0 * np.pi), 0.0]
    ts = np.asarray(ts, dtype=np.float64)
    sol = solve_ivp(rhs, (0.0, float(ts[-1])), y0, t_eval=ts, rtol=1e-12, atol=1e-14, method="DOP853")
    hL, hT, kL, kT, ph, B, dE, sg = sol.y
    H, a2, _ = background(ts, H0)
    dK = kL + 2.0 * kT + H * (hL + 2.0 * hT)
    return {"dK": dK, "phi": ph, "B": B,
            "ham": 2.0 * k * k * hT / a2 - 4.0 * H * dK - 16.0 * np.pi * dE,
            "mom": -2.0 * k * (kT + H * hT) - 8.0 * np.pi * sg}


def mode_amplitudes(u, n0, mu, trk, alp, betx):
    """Amplitudes per unit mu of the sin mode of K and alpha and of the cos mode of beta^x, from a
    (25, nz, ny, nx) state on the x-line y = z = 0 of a grid whose x-coordinate is -L/2 + i h:
    half the difference of the values half a wavelength apart (terms of second order in mu,
    which repeat every half wavelength, cancel)."""
    i_m, i_p = n0 // 4, 3 * n0 // 4  # sin(k x) = -1, +1
    i_c, i_0 = n0 // 2, 0           # cos(k x) = +1, -1
    return {"dK": (u[trk, 0, 0, i_p] - u[trk, 0, 0, i_m]) / (2.0 * mu),
            "phi": (u[alp, 0, 0, i_p] - u[alp, 0, 0, i_m]) / (2.0 * mu),
            "B": (u[betx, 0, 0, i_c] - u[betx, 0, 0, i_0]) / (2.0 * mu)}
