"""Pins of the oracle's PR with the implicit relaxation-time update (Sec. 3:
Newton iterations in the collision find the viscosity consistent with the
strain rate it produces; the oracle finds the same root by bisection).

  * the returned relaxation time reproduces itself: tau = 1/2 + 3
    nu_app(G / tau), with G the strain rate at tau = 1, on random
    non-equilibrium states and across the linear interpolation below the
    cut-off;
  * at sigma_y = 0 it is the Newtonian TRT, bitwise equal to explicit PR;
  * a node at equilibrium (zero strain rate) takes nu_0 = nu_p + m sigma_y;
  * its steady state is explicit PR's: on the Bingham channel both converge
    to the 1-D regularised solution of Eq. 36, and to each other;
  * it is stateless: the result does not depend on a stored tau.
"""
import numpy as np
import pytest

from test_oracle_flows import _channel_regularised


def _random_state(orc, lat, rng, amp):
    _, c, w, _ = orc.lattice_info(lat)
    u = rng.uniform(-0.03, 0.03, 3) * (1, 1, lat > 0)
    feq = orc.equilibrium(lat, 1.0 + rng.uniform(-0.02, 0.02), u)
    return feq + amp * w * rng.uniform(-1, 1, len(w)), c, w


@pytest.mark.parametrize("lat", [0, 1, 2])
def test_self_consistent_relaxation_time(orc, lat):
    rng = np.random.default_rng(5 + lat)
    for amp in (1e-3, 1e-5, 1e-7, 1e-9):
        for sy, m in ((1e-4, 1e4), (5e-6, 1e6), (1e-3, 1e3)):
            rh = orc.rheology(orc.PRI, 0.05, sy, m, 1e-8, 0.25, (1e-6, 0, 0))
            f, _, _ = _random_state(orc, lat, rng, amp)
            _, o = orc.collide_pri(lat, rh, f)
            tau = o["tau"]
            # explicit PR with this tau as "previous" gives it back
            _, o2 = orc.collide_pr(lat, rh, f, tau)
            assert abs(o2["tau"] - tau) <= 1e-12 * tau
            rho = f.sum()
            assert 0.5 + 3 * 0.05 <= tau <= (0.5 + 3 * (0.05 + m * sy / rho)) * (1 + 1e-12)
            assert abs(tau - (0.5 + 3 * orc.nu_app(rh, o["gamma"], f.sum()))) <= 1e-12 * tau


def test_newtonian_limit_bitwise(orc):
    rng = np.random.default_rng(9)
    for lat in (0, 1, 2):
        f, _, _ = _random_state(orc, lat, rng, 1e-3)
        rh = orc.rheology(orc.PRI, 0.07, 0.0, 1e4, 1e-8, 0.25, (1e-6, -2e-6, 0))
        rhp = orc.rheology(orc.PR, 0.07, 0.0, 1e4, 1e-8, 0.25, (1e-6, -2e-6, 0))
        a, oa = orc.collide_pri(lat, rh, f)
        b, ob = orc.collide_pr(lat, rhp, f, 123.0)
        assert np.array_equal(a, b) and oa["tau"] == 0.5 + 0.07 / (1 / 3)


def test_equilibrium_node_takes_nu0(orc):
    for lat in (0, 2):
        feq = orc.equilibrium(lat, 1.0, (0.01, 0.0, 0.0))
        rh = orc.rheology(orc.PRI, 0.1, 1e-4, 1e4, 1e-8, 0.25, (0, 0, 0))
        _, o = orc.collide_pri(lat, rh, feq)
        assert abs(o["tau"] - (0.5 + 3 * (0.1 + 1e4 * 1e-4))) <= 1e-12 * o["tau"]


def test_channel_steady_state_matches_explicit_and_reference(orc):
    H, g, nu, m = 32, 2e-5, 0.1, 1e4
    sy = g * H / 4.0
    ux = {}
    for op in (orc.PR, orc.PRI):
        rh = orc.rheology(op, nu, sy, m, 1e-8, 0.25, (g, 0, 0))
        dom = orc.Domain(0, (2, H, 1), (1, 0, 1), rh)
        dom.step(20000)
        _, u, _, _ = dom.moments()
        ux[op] = u[0].reshape(H, 2)
    import warnings
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        ref = _channel_regularised(H, g, nu, sy, m)
    # H = 32: the Lambda = 1/4 wall slip g/(24 nu) is ~1.2e-3 of the peak
    assert np.max(np.abs(ux[orc.PRI] - ref[:, None])) < 3e-3 * ref.max()
    assert np.max(np.abs(ux[orc.PRI] - ux[orc.PR])) < 1e-6 * ref.max()


def test_stateless(orc):
    """The stored relaxation time of a PRI domain plays no part: two runs
    from the same populations with different stored tau agree bitwise."""
    lat, dims = 1, (6, 5, 4)
    rh = orc.rheology(orc.PRI, 0.1, 2e-4, 1e4, 1e-8, 0.25, (1e-5, 0, 0))
    N = 120
    rng = np.random.default_rng(3)
    _, _, w, _ = orc.lattice_info(lat)
    P = w[:, None] * (1 + 1e-3 * rng.uniform(-1, 1, (len(w), N)))
    out = []
    for t0 in (0.8, 5.0):
        dom = orc.Domain(lat, dims, (1, 1, 1), rh)
        dom.set_state(P, np.full(N, t0))
        dom.step(20)
        out.append(dom.get_state()[0])
    assert np.array_equal(out[0], out[1])
