"""Brute-force pins of the oracle's pointwise algebra (no GPU).

The oracle evaluates the conformal (BSSN chi-form) algebra: conformal
Christoffels, the conformal Ricci tensor plus its conformal-factor part, the
second covariant derivative of the lapse, the constraints and the right-hand
sides. Here the same quantities are computed a second, independent way: from
the physical metric gamma_ij = gt_ij / chi with the textbook ADM formulas
(Christoffels of gamma, Ricci from them, the ADM evolution equations for
gamma_ij and K_ij with the perfect-fluid sources of the paper's "Physical
system settings"), transformed to the conformal variables by the chain rule.
Exact derivatives come from second-order Taylor jets of random analytic
fields, so no discretisation enters.

Expected relations: R_ij, D_iD_j alpha and M_i agree; the chi, gt, At
right-hand sides agree with the ADM-derived rates; the K right-hand side
equals the ADM rate minus alpha * H (the conformal system adds the
Hamiltonian constraint to the trace equation).
"""
import math

import numpy as np
import pytest

SYM = [[0, 1, 2], [1, 3, 4], [2, 4, 5]]


class J:
    """Second-order Taylor jet in 3 variables: value, gradient, Hessian.
    The Hessian is NaN for jets obtained by differentiating a jet."""

    __slots__ = ("v", "g", "H")

    def __init__(self, v, g=None, H=None):
        self.v = float(v)
        self.g = np.zeros(3) if g is None else np.asarray(g, dtype=float)
        self.H = np.zeros((3, 3)) if H is None else np.asarray(H, dtype=float)

    @staticmethod
    def c(x):
        return x if isinstance(x, J) else J(x)

    def __add__(a, b):
        b = J.c(b)
        return J(a.v + b.v, a.g + b.g, a.H + b.H)

    __radd__ = __add__

    def __neg__(a):
        return J(-a.v, -a.g, -a.H)

    def __sub__(a, b):
        return a + (-J.c(b))

    def __rsub__(a, b):
        return J.c(b) - a

    def __mul__(a, b):
        b = J.c(b)
        return J(a.v * b.v, a.g * b.v + a.v * b.g,
                 a.H * b.v + np.outer(a.g, b.g) + np.outer(b.g, a.g) + a.v * b.H)

    __rmul__ = __mul__

    def _chain(a, f0, f1, f2):
        return J(f0, f1 * a.g, f2 * np.outer(a.g, a.g) + f1 * a.H)

    def inv(a):
        return a._chain(1 / a.v, -1 / a.v ** 2, 2 / a.v ** 3)

    def __truediv__(a, b):
        return a * J.c(b).inv()

    def __rtruediv__(a, b):
        return J.c(b) * a.inv()

    def sqrt(a):
        r = math.sqrt(a.v)
        return a._chain(r, 0.5 / r, -0.25 / (r * a.v))

    def log(a):
        return a._chain(math.log(a.v), 1 / a.v, -1 / a.v ** 2)

    def exp(a):
        e = math.exp(a.v)
        return a._chain(e, e, e)

    def d(a, k):
        return J(a.g[k], a.H[k], np.full((3, 3), np.nan))


def rand_field(rng, x0, c0, amp, modes=3):
    v, g, H = c0, np.zeros(3), np.zeros((3, 3))
    for _ in range(modes):
        k = rng.normal(size=3) * 1.3
        a = amp * rng.uniform(-1, 1)
        th = k @ x0 + rng.uniform(0, 2 * np.pi)
        v += a * math.sin(th)
        g = g + a * math.cos(th) * k
        H = H - a * math.sin(th) * np.outer(k, k)
    return J(v, g, H)


def inv3(m):
    """Inverse of a symmetric 3x3 matrix of jets (given as 3x3 nested list)."""
    c = [[None] * 3 for _ in range(3)]
    c[0][0] = m[1][1] * m[2][2] - m[1][2] * m[2][1]
    c[0][1] = m[0][2] * m[2][1] - m[0][1] * m[2][2]
    c[0][2] = m[0][1] * m[1][2] - m[0][2] * m[1][1]
    c[1][1] = m[0][0] * m[2][2] - m[0][2] * m[2][0]
    c[1][2] = m[0][2] * m[1][0] - m[0][0] * m[1][2]
    c[2][2] = m[0][0] * m[1][1] - m[0][1] * m[1][0]
    c[1][0], c[2][0], c[2][1] = c[0][1], c[0][2], c[1][2]
    det = m[0][0] * c[0][0] + m[0][1] * c[1][0] + m[0][2] * c[2][0]
    return [[c[i][j] / det for j in range(3)] for i in range(3)], det


def christoffel(g, gi):
    """Gamma^k_ij of metric g (jets) -- value and gradient valid."""
    dg = [[[g[i][j].d(k) for k in range(3)] for j in range(3)] for i in range(3)]  # dg[i][j][k] = d_k g_ij
    G = [[[None] * 3 for _ in range(3)] for _ in range(3)]
    for k in range(3):
        for i in range(3):
            for j in range(3):
                acc = J(0.0)
                for l in range(3):
                    acc = acc + 0.5 * gi[k][l] * (dg[l][j][i] + dg[l][i][j] - dg[i][j][l])
                G[k][i][j] = acc
    return G


def ricci(G):
    R = [[None] * 3 for _ in range(3)]
    for i in range(3):
        for j in range(3):
            acc = J(0.0)
            for k in range(3):
                acc = acc + G[k][i][j].d(k) - G[k][i][k].d(j)
                for l in range(3):
                    acc = acc + G[k][k][l] * G[l][i][j] - G[k][j][l] * G[l][i][k]
            R[i][j] = acc
    return R


def build_case(seed, unit_det):
    rng = np.random.default_rng(seed)
    x0 = rng.uniform(-1, 1, size=3)
    gt = [[None] * 3 for _ in range(3)]
    for i in range(3):
        for j in range(i, 3):
            gt[i][j] = rand_field(rng, x0, 1.0 if i == j else 0.0, 0.15 if i == j else 0.08)
            gt[j][i] = gt[i][j]
    if unit_det:
        _, det = inv3(gt)
        f = (det.log() * (-1.0 / 3.0)).exp()
        gt = [[gt[i][j] * f for j in range(3)] for i in range(3)]
    chi = rand_field(rng, x0, 1.0, 0.2)
    alpha = rand_field(rng, x0, 1.0, 0.2)
    beta = [rand_field(rng, x0, 0.0, 0.2) for _ in range(3)]
    K = rand_field(rng, x0, -1.0, 0.3)
    At = [[None] * 3 for _ in range(3)]
    for i in range(3):
        for j in range(i, 3):
            At[i][j] = rand_field(rng, x0, 0.0, 0.2)
            At[j][i] = At[i][j]
    gti, _ = inv3(gt)
    tr = sum((gti[i][j] * At[i][j] for i in range(3) for j in range(3)), J(0.0))
    At = [[At[i][j] - gt[i][j] * tr / 3.0 for j in range(3)] for i in range(3)]  # traceless
    # fluid from primitives: rho, covariant velocity v_i (physical)
    rho = rng.uniform(0.2, 1.0)
    return dict(rng=rng, gt=gt, gti=gti, chi=chi, alpha=alpha, beta=beta, K=K, At=At, rho=rho)


def oracle_inputs(c):
    gt, gti, chi = c["gt"], c["gti"], c["chi"]
    # conformal connection functions computed from the metric, and their gradient
    dgt = [[[gt[i][j].d(k) for k in range(3)] for j in range(3)] for i in range(3)]
    Gd = []
    for k in range(3):
        acc = J(0.0)
        for i in range(3):
            for j in range(3):
                for l in range(3):
                    acc = acc + gti[i][j] * 0.5 * gti[k][l] * (dgt[l][j][i] + dgt[l][i][j] - dgt[i][j][l])
        Gd.append(acc)
    s6 = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    d = {
        "chi": chi.v, "gt": [gt[i][j].v for i, j in s6], "K": c["K"].v, "At": [c["At"][i][j].v for i, j in s6],
        "Gam": [g.v for g in Gd], "alpha": c["alpha"].v, "beta": [b.v for b in c["beta"]],
        "dchi": chi.g, "d2chi": [chi.H[i, j] for i, j in s6],
        "dgt": [gt[i][j].g for i, j in s6], "d2gt": [[gt[i][j].H[a, b] for a, b in s6] for i, j in s6],
        "dGam": [g.g for g in Gd], "dalpha": c["alpha"].g, "d2alpha": [c["alpha"].H[i, j] for i, j in s6],
        "dbeta": [b.g for b in c["beta"]], "d2beta": [[b.H[i, j] for i, j in s6] for b in c["beta"]],
        "dK": c["K"].g, "dAt": [c["At"][i][j].g for i, j in s6],
    }
    return d


@pytest.mark.parametrize("seed,unit_det", [(1, True), (2, True), (3, False), (4, False), (5, True)])
def test_ricci_and_lapse_hessian_vs_generic(orc, seed, unit_det):
    c = build_case(seed, unit_det)
    gt, chi = c["gt"], c["chi"]
    g = [[gt[i][j] / chi for j in range(3)] for i in range(3)]
    gi, _ = inv3(g)
    G = christoffel(g, gi)
    R = ricci(G)
    al = c["alpha"]
    DDa = [[al.H[i, j] - sum(G[k][i][j].v * al.g[k] for k in range(3)) for j in range(3)] for i in range(3)]
    out = orc.geometry_point(oracle_inputs(c))
    s6 = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    Rref = np.array([R[i][j].v for i, j in s6])
    scale = np.abs(Rref).max() + 1.0
    assert np.abs(out["Ric"] - Rref).max() < 1e-12 * scale, (out["Ric"], Rref)
    Rs = sum(gi[i][j].v * R[i][j].v for i in range(3) for j in range(3))
    assert out["R"] == pytest.approx(Rs, rel=1e-12, abs=1e-12)
    assert np.allclose(out["DDalpha"], [DDa[i][j] for i, j in s6], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("seed", [11, 12, 13, 14])
def test_evolution_equations_vs_adm(orc, seed):
    w = 1.0 / 3.0
    c = build_case(seed, unit_det=True)
    rng = c["rng"]
    gt, chi, al, beta, Kt, At = c["gt"], c["chi"], c["alpha"], c["beta"], c["K"], c["At"]
    g = [[gt[i][j] / chi for j in range(3)] for i in range(3)]
    gi, _ = inv3(g)
    G = christoffel(g, gi)
    R = ricci(G)
    Kij = [[(At[i][j] + gt[i][j] * Kt / 3.0) / chi for j in range(3)] for i in range(3)]
    dbeta = [[beta[i].g[j] for j in range(3)] for i in range(3)]  # d_j beta^i
    V = lambda M: np.array([[M[i][j].v for j in range(3)] for i in range(3)])  # noqa: E731
    gv, giv, Kv, Rv = V(g), V(gi), V(Kij), V(R)
    Ktr = np.sum(giv * Kv)
    assert Ktr == pytest.approx(Kt.v, rel=1e-12)
    # perfect fluid from primitives: T = (rho + P) u u + P g, P = w rho
    rho = c["rho"]
    P = w * rho
    v = rng.normal(size=3)
    v *= 0.4 / math.sqrt(v @ giv @ v)
    W2 = 1.0 / (1.0 - v @ giv @ v)
    X = (rho + P) * W2
    E = X - P
    S = X * v
    Sij = X * np.outer(v, v) + P * gv
    Str = np.sum(giv * Sij)
    a = al.v
    DDa = np.array([[al.H[i, j] - sum(G[k][i][j].v * al.g[k] for k in range(3)) for j in range(3)]
                    for i in range(3)])
    # ADM equations (non-advective and advective parts)
    dtg = np.zeros((3, 3))
    dtK = np.zeros((3, 3))
    Kmix = giv @ Kv  # K^k_j
    for i in range(3):
        for j in range(3):
            lie_g = sum(beta[k].v * g[i][j].g[k] + gv[i][k] * dbeta[k][j] + gv[j][k] * dbeta[k][i] for k in range(3))
            dtg[i, j] = -2 * a * Kv[i, j] + lie_g
            lie_K = sum(beta[k].v * Kij[i][j].g[k] + Kv[i, k] * dbeta[k][j] + Kv[j, k] * dbeta[k][i]
                        for k in range(3))
            dtK[i, j] = (-DDa[i, j] + a * (Rv[i, j] - 2 * (Kv[i] @ Kmix[:, j]) + Ktr * Kv[i, j])
                         - 8 * math.pi * a * (Sij[i, j] - 0.5 * gv[i, j] * (Str - E)) + lie_K)
    # chain rule to the conformal variables
    dchi = -chi.v / 3.0 * np.sum(giv * dtg)
    dgt = dchi * gv + chi.v * dtg
    dKtr = np.sum(giv * dtK) - np.sum((giv @ dtg @ giv) * Kv)
    dAt = dchi * (Kv - gv * Ktr / 3.0) + chi.v * (dtK - dtg * Ktr / 3.0 - gv * dKtr / 3.0)
    # Hamiltonian constraint from the generic quantities
    Rs = np.sum(giv * Rv)
    H = Rs + Ktr ** 2 - np.sum(Kv * (giv @ Kv @ giv)) - 16 * math.pi * E
    # oracle pointwise RHS + exact advection terms
    d = oracle_inputs(c)
    chi32 = chi.v ** 1.5
    s = orc.Setup(w=w, H0=0.0)
    res = orc.point_rhs(s, d, E / chi32, S / chi32)
    assert not res["fail"]
    r = res["rhs"]
    adv = lambda f: sum(beta[k].v * f.g[k] for k in range(3))  # noqa: E731
    s6 = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    tol = 1e-11
    assert r[0] + adv(chi) == pytest.approx(dchi, rel=tol, abs=tol)
    for q, (i, j) in enumerate(s6):
        assert r[1 + q] + adv(gt[i][j]) == pytest.approx(dgt[i, j], rel=tol, abs=tol), (i, j)
        assert r[8 + q] + adv(At[i][j]) == pytest.approx(dAt[i, j], rel=tol, abs=tol), (i, j)
    assert r[7] + adv(Kt) == pytest.approx(dKtr - a * H, rel=tol, abs=tol)
    # Hamiltonian and momentum constraints: H and D_j K^j_i - d_i K - 8 pi S_i
    assert res["H"] == pytest.approx(H, rel=1e-11, abs=1e-11)
    Kup = [[sum((gi[j][k] * Kij[k][i] for k in range(3)), J(0.0)) for i in range(3)] for j in range(3)]  # K^j_i
    for i in range(3):
        DK = sum(Kup[j][i].g[j] for j in range(3))
        DK += sum(G[j][j][l].v * Kup[l][i].v - G[l][j][i].v * Kup[j][l].v for j in range(3) for l in range(3))
        Mi = DK - Kt.g[i] - 8 * math.pi * S[i]
        assert res["M"][i] == pytest.approx(Mi, rel=1e-11, abs=1e-11), i
