"""Pins of the oracle's implicitly-regularised Herschel-Bulkley operator
(IRHB): the implicit construction of Sec. 2.3 (s/2 + T = -sigma, Eq. 31)
solved per node for sigma = sigma_y + K g^n, which Sec. 3.2 notes can be
done numerically for other constitutive laws.  nu_p carries the
consistency K, hb_n the flow index n.

  * n = 1 is the Bingham IR of Eqs. 39-40 (closed form against bisection);
  * the solved s and sigma satisfy Eq. 31 and the law written in s, with
    the strain rate g = 3 |s| / sqrt(2) that Eqs. 32-33 identify;
  * plane channel driven by a body force, steady state against the
    analytic power-law profile u = n/(n+1) (g/K)^(1/n) (h^(1+1/n) -
    |y|^(1+1/n)) for n = 0.5 and 1.5, and against the Herschel-Bulkley
    profile (the same with h - y0 and |y| - y0, plug |y| < y0 = sigma_y/g),
    with exactly the plug nodes unyielded.
"""
import numpy as np
import pytest

H = 32


def _state(lat, rng, amp=0.05):
    import oracle
    _, _, w, _ = oracle.lattice_info(lat)
    return w * (1 + amp * (2 * rng.random(len(w)) - 1))


@pytest.mark.parametrize("lat", [0, 1, 2])
def test_flow_index_one_is_bingham_ir(orc, lat):
    rng = np.random.default_rng(10 + lat)
    worst = 0.0
    n_yielded = 0
    for k in range(300):
        f = _state(lat, rng)
        sy = (0.0, 1e-4, 3e-4, 2e-3)[k % 4]
        rb = orc.rheology(orc.IR, 0.1 + 0.05 * (k % 3), sy, g=(1e-5, -2e-5, 3e-6))
        rh = orc.rheology(orc.IRHB, 0.1 + 0.05 * (k % 3), sy, g=(1e-5, -2e-5, 3e-6), hb_n=1.0)
        a, oa = orc.collide_ir(lat, rb, f)
        b, ob = orc.collide_ir(lat, rh, f)
        worst = max(worst, float(np.abs(a - b).max()))
        assert oa["unyielded"] == ob["unyielded"]
        n_yielded += not ob["unyielded"]
    assert worst <= 1e-15
    assert 50 < n_yielded < 300  # both branches exercised


@pytest.mark.parametrize("n", [0.4, 0.7, 1.6])
def test_solution_satisfies_eq31_and_law(orc, n):
    rng = np.random.default_rng(int(10 * n))
    K, sy = 0.02, 2e-4
    checked = 0
    for _ in range(200):
        f = _state(2, rng, amp=0.08)
        rh = orc.rheology(orc.IRHB, K, sy, hb_n=n)
        _, o = orc.collide_ir(2, rh, f)
        s, sig, T = o["s"], o["sigma"], o["T"]
        # deviatoric T recovered from Eq. 31 in both regimes
        Tdev = -sig - 0.5 * s
        assert abs(np.sqrt((Tdev ** 2).sum()) - T) <= 1e-13 * max(T, 1e-30)
        if o["unyielded"]:
            assert np.all(s == 0.0) and T <= np.sqrt(2) * sy
            continue
        sn = np.sqrt((s ** 2).sum())
        g = 3 * sn / np.sqrt(2)
        law = (3 * K * g ** (n - 1) + np.sqrt(2) * sy / sn) * s
        assert np.max(np.abs(sig - law)) <= 1e-12 * np.abs(sig).max()
        checked += 1
    assert checked > 50


def _channel(orc, n, K, g, sy, steps=10000):
    rh = orc.rheology(orc.IRHB, K, sy, g=(g, 0, 0), hb_n=n)
    d = orc.Domain(orc.D2Q9, (4, H, 1), (1, 0, 1), rh)
    d.init_equilibrium()
    d.step(steps)
    _, u, _, uy = d.moments()
    d.close()
    return u[0].reshape(H, 4)[:, 0], uy.reshape(H, 4)[:, 0]


def _analytic(n, K, g, sy):
    h, y0 = H / 2.0, sy / g
    yp = np.abs(np.arange(H) + 0.5 - h)
    a = n / (n + 1) * (g / K) ** (1 / n)
    return a * ((h - y0) ** (1 + 1 / n) - np.clip(yp - y0, 0, None) ** (1 + 1 / n)), yp < y0


@pytest.mark.parametrize("n,K,g", [(0.5, 4.3e-3, 1.17e-5), (1.5, 3.0, 6.3e-6)])
def test_power_law_channel(orc, n, K, g):
    ux, uy = _channel(orc, n, K, g, 0.0)
    ref, _ = _analytic(n, K, g, 0.0)
    assert np.max(np.abs(ux - ref)) <= 3e-3 * ref.max()
    assert uy.sum() == 0


def test_herschel_bulkley_channel_plug(orc):
    n, K, g = 0.5, 4.3e-3, 1.17e-5
    sy = 4 * g  # plug half-width y0 = 4
    ux, uy = _channel(orc, n, K, g, sy)
    ref, plug = _analytic(n, K, g, sy)
    assert np.max(np.abs(ux - ref)) <= 4e-3 * ref.max()
    assert np.array_equal(uy.astype(bool), plug)
