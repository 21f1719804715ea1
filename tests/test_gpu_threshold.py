"""Collapse-threshold search (batched multisection on the device collapse counters +
Newton with the adjoint derivative) against the oracle: the collapse level alpha_th is
the oracle's centre lapse at the final step for a known amplitude mu*. The centre
lapse falls monotonically through the run and is the grid minimum (checked on the
oracle), so the runs that push the lapse below alpha_th at some point and step are
exactly those above mu*: the threshold is mu*. The derivative at the root is checked
against the oracle's exact forward-mode tangent."""
import pytest

pytestmark = pytest.mark.gpu


def test_threshold_search_recovers_oracle_amplitude(orc):
    from paper_2606_02053_amd.threshold import find_threshold
    n, L, nsteps, sigma, mu_star = 16, 6.0, 10, 1.2, 0.4137
    s = orc.Setup(n=(n, n, n), L=(L, L, L))
    dt = 0.25 * L / n
    c = n // 2
    ini = orc.Init(mu=mu_star, sigma=sigma)
    u, _ = orc.rk4(s, orc.init_fields(s, ini), 0.0, dt, nsteps, parallel=True)
    target = float(u[17, c, c, c])
    assert float(u[17].min()) == target  # the lapse is lowest at the centre
    res = find_threshold(sigma, 0.3, 0.5, target, n=n, L=L, nsteps=nsteps, K=8, rounds=2)
    batched = [h for h in res.history if h[0] == "batched"]
    assert len(batched) == 16 and res.batched_runs == 18
    for _, m, collapsed, a_centre, a_min in batched:  # device outcomes: minimum at the centre
        assert collapsed == (m > mu_star) and a_min == a_centre
    # the final bracket closes on the root of the GPU's J, which differs from the oracle's
    # amplitude by rounding only
    lo, hi = res.bracket
    assert min(lo, hi) - 1e-9 <= mu_star <= max(lo, hi) + 1e-9
    assert abs(res.mu - mu_star) < 1e-9, res
    assert 2 <= res.newton_steps <= 8  # mu* is off the bracket midpoints: Newton has work to do
    # dJ/dmu at the root: the oracle's exact derivative of the discrete map
    u, v = orc.init_fields(s, ini), orc.init_tangent(s, ini, 0)
    for m in range(nsteps):
        u, v = orc.jvp(s, u, v, "step", t=m * dt, dt=dt)
    assert res.dJ_dmu == pytest.approx(float(v[17, c, c, c]), rel=1e-8)


def test_interpolated_search_recovers_oracle_amplitude(orc):
    """Batched rounds alone: the cubic through the runs around the sign change of the centre lapse
    lands on the oracle's amplitude in two rounds of 8 runs; the collapse counters bracket it."""
    from paper_2606_02053_amd.threshold import find_threshold_interpolated
    n, L, nsteps, sigma, mu_star = 16, 6.0, 10, 1.2, 0.4137
    s = orc.Setup(n=(n, n, n), L=(L, L, L))
    dt = 0.25 * L / n
    c = n // 2
    u, _ = orc.rk4(s, orc.init_fields(s, orc.Init(mu=mu_star, sigma=sigma)), 0.0, dt, nsteps, parallel=True)
    target = float(u[17, c, c, c])
    res = find_threshold_interpolated(sigma, 0.3, 0.5, target, n=n, L=L, nsteps=nsteps, K=8, rounds=2)
    assert res.batched_runs == 16
    lo, hi = res.bracket
    assert lo <= mu_star <= hi and hi - lo < 0.2 / 9 * 1e-4 * 2
    assert abs(res.mu - mu_star) < 1e-9, res


def test_isocurvature_threshold_by_multisection(orc):
    """The iso-curvature amplitude whose centre lapse matches the oracle's at a known amplitude:
    the multisection bracket (K + 1 = 9 times narrower per round) closes on it."""
    from paper_2606_02053_amd.threshold import find_threshold_isocurvature
    n, L, nsteps, sigma, mu_star = 16, 6.0, 10, 1.0, 0.2763
    s = orc.Setup(n=(n, n, n), L=(L, L, L))
    dt = 0.25 * L / n
    c = n // 2
    u0, sc0 = orc.init_fields_sc(s, orc.Init(mu=0.05, sigma=1.2), mu_star, sigma)
    u, _, _ = orc.rk4_sc(s, u0, sc0, 0.0, dt, nsteps, parallel=True)
    target = float(u[17, c, c, c])
    res = find_threshold_isocurvature(sigma, 0.1, 0.4, target, zeta=(0.05, 1.2), n=n, L=L, nsteps=nsteps, K=8,
                                      rounds=4)
    lo, hi = res.bracket
    assert abs(hi - lo) < 0.3 / 9 ** 4 * 1.01
    assert min(lo, hi) - 1e-9 <= mu_star <= max(lo, hi) + 1e-9, res.bracket
    assert res.batched_runs == 2 + 4 * 8
