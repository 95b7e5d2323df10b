"""Pins of the oracle's steady-state residual (the velocity change between
two records that the convergence criteria of Sec. 4.3 and 4.5 watch).

A periodic box started from a uniform rest state under a uniform force g
stays uniform, so every node carries the same output velocity.  Its momentum
grows by rho g per step and the output velocity at time t is g (t + 1/2) for
both operators (IR: (j + F/2)/rho; PR/EDM: j/rho + g/2).  Between records k
steps apart the change is k g at every node, which fixes

    residual(t) = (k / (t + 1/2))^2,   du_max = k |g|,

and the first record, compared with a zero reference, gives 1 and |g|/2.
"""
import numpy as np
import pytest


@pytest.mark.parametrize("op", [0, 1])
@pytest.mark.parametrize("lat", [0, 1, 2])
def test_uniform_acceleration_closed_form(orc, lat, op):
    dims = (4, 3, 1) if lat == 0 else (3, 2, 3)
    g = np.array([1e-5, -2e-5, 0.0 if lat == 0 else 5e-6])
    rh = orc.rheology(op, 0.1, 1e-5, 1e4, 1e-8, 0.25, g)
    dom = orc.Domain(lat, dims, (1, 1, 1), rh)
    uprev = np.zeros(3 * dom.N)
    k = 7
    gn = float(np.linalg.norm(g))
    for rec in range(6):
        t = rec * k
        r = dom.residual(uprev)
        if rec == 0:
            assert abs(r["residual"] - 1.0) < 1e-12
            assert abs(r["du_max"] - 0.5 * gn) < 1e-12 * gn
        else:
            assert abs(r["residual"] / (k / (t + 0.5)) ** 2 - 1) < 1e-9
            assert abs(r["du_max"] / (k * gn) - 1) < 1e-9
        # the kept reference is the current output velocity of every node
        assert np.allclose(uprev.reshape(3, dom.N), (g * (t + 0.5))[:, None], rtol=1e-10, atol=0)
        dom.step(k)


def test_probe_without_record_keeps_reference(orc):
    """record=False reports against the kept velocity and leaves it alone;
    a field at rest has residual 0 (zero denominator) and du_max 0."""
    rh = orc.rheology(1, 0.1, 0.0, 0.0, 1e-8, 0.25, (2e-5, 0.0, 0.0))
    dom = orc.Domain(0, (5, 4, 1), (1, 1, 1), rh)
    uprev = np.zeros(3 * dom.N)
    dom.residual(uprev)
    dom.step(3)
    kept = uprev.copy()
    a = dom.residual(uprev, record=False)
    b = dom.residual(uprev, record=False)
    assert np.array_equal(uprev, kept) and a == b
    assert abs(a["residual"] / (3 / 3.5) ** 2 - 1) < 1e-9
    rest = orc.Domain(0, (5, 4, 1), (1, 1, 1), orc.rheology(1, 0.1, 0.0, 0.0, 1e-8, 0.25, (0.0, 0.0, 0.0)))
    z = np.zeros(3 * rest.N)
    rest.step(4)
    assert rest.residual(z) == {"residual": 0.0, "du_max": 0.0}


def test_residual_decays_to_steady_channel(orc):
    """Approach to the steady plane Poiseuille flow (walls half a spacing
    outside the first and last fluid rows, so the width is H): the slowest
    transient is the Stokes mode sin(pi y / H), decaying as exp(-nu (pi/H)^2 t).
    The residual between records k steps apart is its squared amplitude ratio,
    so consecutive residuals settle to exp(-2 k nu pi^2 / H^2)."""
    H, g, nu, k = 16, 1e-5, 0.1, 100
    rh = orc.rheology(1, nu, 0.0, 0.0, 1e-8, 0.25, (g, 0.0, 0.0))
    dom = orc.Domain(0, (2, H, 1), (1, 0, 1), rh)
    uprev = np.zeros(3 * dom.N)
    res = []
    for _ in range(40):
        res.append(dom.residual(uprev)["residual"])
        dom.step(k)
    ratio = np.exp(-2 * k * nu * np.pi ** 2 / H ** 2)
    for a, b in zip(res[-6:-1], res[-5:]):
        assert abs(b / a / ratio - 1) < 1e-3
    assert all(b < a for a, b in zip(res[1:], res[2:]))
