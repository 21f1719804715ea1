"""The oracle's fixed mesh refinement (oracle/fmr.py; paper: nested refinement layers, "Statement of
need" and the adiabatic-fluctuation example) pinned by what fixes it independently of itself:
its interpolation reproduces polynomials of the degree it claims, its time interpolant (the RK4
step's continuous extension) is exact for cubic solutions, restriction after prolongation returns
the parent, and a refined run converges
to the uniform run at the child's resolution at fourth order away from the coarse-fine interface."""
import numpy as np
import pytest

from oracle import fmr


def test_prolongation_exact_for_quintics():
    """Tensor products of polynomials of degree <= 5 per axis are reproduced at every padded
    child point (coincident points and midpoints) to rounding."""
    rng = np.random.default_rng(7)
    n = 32
    box = fmr.Box(origin=(10, 9, 11), m=(6, 5, 4))  # source blocks stay inside the grid: no wrap
    c = rng.standard_normal((3, 6))

    def poly(x, y, z):
        return (np.polyval(c[0], x) * np.polyval(c[1], y) * np.polyval(c[2], z))

    g = np.arange(n) / n
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    u = np.broadcast_to(poly(X, Y, Z), (25, n, n, n)).copy()
    u[3] *= -2.0  # fields are interpolated independently
    child = fmr.prolong(u, box)
    cx = [(box.origin[a] + (np.arange(2 * box.m[a] + 2 * fmr.W) - fmr.W) / 2.0) / n for a in range(3)]
    Zc, Yc, Xc = np.meshgrid(cx[2], cx[1], cx[0], indexing="ij")
    ref = poly(Xc, Yc, Zc)
    scale = np.abs(ref).max()
    assert np.abs(child[0] - ref).max() < 1e-13 * scale
    assert np.abs(child[3] + 2.0 * ref).max() < 2e-13 * scale
    # a degree-6 term is not reproduced at the midpoints (the claimed degree is the exact one)
    u6 = np.broadcast_to(X ** 6, (25, n, n, n)).copy()
    err6 = np.abs(fmr.prolong(u6, box)[0] - Xc ** 6).max()
    assert err6 > 1e-9


def test_rk4_continuous_extension():
    """The time interpolant: for u' = f(t) the RK4 stages are quadrature nodes, and the continuous
    extension reproduces the exact solution at every theta when f is quadratic (u cubic), but not
    when f is cubic (except at theta = 1, where the step itself is exact); for u' = lam u its
    midpoint error falls by 16 per halving of dt (local error O(dt^4)); the slopes recovered from
    the stage states are the slopes."""
    rng = np.random.default_rng(3)
    t0, dt = 0.3, 0.7
    for deg, exact in ((0, True), (1, True), (2, True), (3, False)):
        c = rng.standard_normal(deg + 1)
        F = np.polyint(c)
        ks = [np.polyval(c, t0), np.polyval(c, t0 + 0.5 * dt), np.polyval(c, t0 + 0.5 * dt), np.polyval(c, t0 + dt)]
        for theta in (0.25, 0.5, 0.8):
            err = abs(fmr.dense(0.0, ks, dt, theta) - (np.polyval(F, t0 + theta * dt) - np.polyval(F, t0)))
            assert (err < 1e-14) == exact, (deg, theta, err)
    errs = []
    for h in (0.1, 0.05, 0.025):
        lam = -1.3
        k1 = lam
        k2 = lam * (1.0 + 0.5 * h * k1)
        k3 = lam * (1.0 + 0.5 * h * k2)
        k4 = lam * (1.0 + h * k3)
        errs.append(abs(fmr.dense(1.0, (k1, k2, k3, k4), h, 0.5) - np.exp(0.5 * lam * h)))
    assert 14.0 < errs[0] / errs[1] < 18.0 and 14.0 < errs[1] / errs[2] < 18.0, errs
    b = fmr.rk4_dense_weights(1.0)
    assert np.allclose(b, (1 / 6, 1 / 3, 1 / 3, 1 / 6), rtol=0, atol=1e-15)
    u0, ks = rng.standard_normal(5), [rng.standard_normal(5) for _ in range(4)]
    U2, U3, U4 = u0 + 0.5 * dt * ks[0], u0 + 0.5 * dt * ks[1], u0 + dt * ks[2]
    u1 = u0 + dt / 6 * (ks[0] + 2 * ks[1] + 2 * ks[2] + ks[3])
    back = fmr.slopes_from_stage_states(u0, U2, U3, U4, u1, dt)
    for a, k in zip(back, ks):
        assert np.allclose(a, k, rtol=1e-12, atol=1e-12)


def test_restrict_after_prolong_returns_the_parent():
    rng = np.random.default_rng(11)
    u = rng.standard_normal((25, 12, 10, 16))
    box = fmr.Box(origin=(13, -2, 4), m=(5, 6, 4))  # wraps around the periodic parent in x and y
    child = fmr.prolong(u, box)
    back = fmr.restrict(child, np.zeros_like(u), box)
    X = [(box.origin[a] + np.arange(box.m[a])) % u.shape[3 - a] for a in range(3)]
    sel = np.ix_(np.arange(25), X[2], X[1], X[0])
    assert np.array_equal(back[sel], u[sel])
    mask = np.ones(u.shape, bool)
    mask[sel] = False
    assert not back[mask].any()  # nothing outside the box is written


@pytest.mark.slow
def test_refined_run_converges_to_uniform_fine_run(orc):
    """Smooth periodic data (PGAUSS, mu 0.1, sigma 2.5) on a 10^3 box; one child over the central
    half. After 0.625 / H0 the child's interior is compared with a uniform run at the child's
    resolution (same initial data, same total time), at N = 16 and 32 coarse points per side:
    at two coarse cells or more from the child's faces the max-norm error of every field falls by
    at least 12 (fourth order: 16), and at N = 32 the refined run is there, summed over the
    fields, more accurate than the uniform coarse run by more than 2. (Within a coarse cell of the
    faces the error falls more slowly: the buffer holds interpolated coarse values, and the second
    derivatives taken across the coarse-fine interface see their mismatch.)"""
    L = 10.0
    ini = orc.Init(mu=0.1, sigma=2.5, profile=orc.PGAUSS)
    errs, coarse_errs = {}, {}
    for N, nsteps in ((16, 2), (32, 4)):
        s = orc.Setup(n=(N,) * 3, L=(L,) * 3)
        box = fmr.Box(origin=(N // 4,) * 3, m=(N // 2,) * 3)
        H = fmr.Hierarchy(s, [box])
        u0 = orc.init_fields(s, ini)
        st = H.init(u0)
        dt = 0.25 * s.h[0]
        t = 0.0
        for _ in range(nsteps):
            H.step(st, t, dt)
            t += dt
        sf = orc.Setup(n=(2 * N,) * 3, L=(L,) * 3)
        uf, _ = orc.rk4(sf, orc.init_fields(sf, ini), 0.0, dt / 2, 2 * nsteps, parallel=True)
        uc, _ = orc.rk4(s, u0, 0.0, dt, nsteps, parallel=True)
        W, o = fmr.W, 2 * (N // 4)
        child = st[1][:, W:-W, W:-W, W:-W]
        ref = uf[:, o:o + N, o:o + N, o:o + N]
        scale = np.maximum(np.abs(ref).reshape(25, -1).max(axis=1), 1e-3)
        z, y, x = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
        far = np.minimum.reduce([x, N - 1 - x, y, N - 1 - y, z, N - 1 - z]) >= N // 4  # 2 coarse cells at N = 16
        d = np.abs(child - ref)[:, far].max(axis=1) / scale
        errs[N] = d
        # the uniform coarse run at the coincident points of the same region
        cfar = far[::2, ::2, ::2]
        cref = uf[:, ::2, ::2, ::2][:, o // 2:o // 2 + N // 2, o // 2:o // 2 + N // 2, o // 2:o // 2 + N // 2]
        ccoarse = uc[:, o // 2:o // 2 + N // 2, o // 2:o // 2 + N // 2, o // 2:o // 2 + N // 2]
        coarse_errs[N] = np.abs(ccoarse - cref)[:, cfar].max(axis=1) / scale
        print(N, "refined", " ".join(f"{v:.1e}" for v in d), "\n   uniform coarse", " ".join(f"{v:.1e}" for v in coarse_errs[N]))
    ratio = errs[16] / np.maximum(errs[32], 1e-300)
    live = errs[16] > 1e-12  # fields the data leaves untouched stay exact on both grids
    assert live.sum() >= 20
    assert np.all(ratio[live] > 12.0), ratio
    assert errs[32].sum() < 0.5 * coarse_errs[32].sum(), (errs[32], coarse_errs[32])
