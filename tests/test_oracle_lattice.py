"""Pins of the oracle's lattices and equilibrium against the mathematics they
must satisfy (velocity sets of Sec. 4.1; equilibrium of Sec. 2.1, Eq. 12 and
its moment identities, Eq. 13)."""
from fractions import Fraction
import itertools

import numpy as np
import pytest

LATTICES = [(0, 2, 9), (1, 3, 19), (2, 3, 27)]


@pytest.mark.parametrize("lat,d,q", LATTICES)
def test_velocity_set_shape(orc, lat, d, q):
    dd, c, w, opp = orc.lattice_info(lat)
    assert dd == d and len(w) == q
    # distinct velocities, each component in {-1,0,1}, rest velocity present
    assert len({tuple(v) for v in c}) == q
    assert np.all(np.abs(c) <= 1)
    if d == 2:
        assert np.all(c[:, 2] == 0)
    for i in range(q):
        assert np.array_equal(c[opp[i]], -c[i])
    # D3Q19 is D3Q27 without the 8 corner velocities
    if q == 19:
        assert np.all((c ** 2).sum(1) <= 2)


@pytest.mark.parametrize("lat,d,q", LATTICES)
def test_isotropy_exact(orc, lat, d, q):
    """sum w = 1, sum w c = 0, sum w c_a c_b = delta/3, odd third moment 0,
    sum w c_a c_b c_c c_d = (dd + dd + dd)/9 -- in exact rationals."""
    _, c, w, _ = orc.lattice_info(lat)
    wr = [Fraction(x).limit_denominator(1000) for x in w]
    for a, b in zip(wr, w):
        assert float(a) == b  # weights are exactly the rationals
    assert sum(wr) == 1
    axes = range(d)
    for a in axes:
        assert sum(wi * int(ci[a]) for wi, ci in zip(wr, c)) == 0
    for a, b in itertools.product(axes, axes):
        m2 = sum(wi * int(ci[a]) * int(ci[b]) for wi, ci in zip(wr, c))
        assert m2 == (Fraction(1, 3) if a == b else 0)
    for a, b, g in itertools.product(axes, axes, axes):
        assert sum(wi * int(ci[a]) * int(ci[b]) * int(ci[g]) for wi, ci in zip(wr, c)) == 0
    for a, b, g, e in itertools.product(axes, axes, axes, axes):
        m4 = sum(wi * int(ci[a]) * int(ci[b]) * int(ci[g]) * int(ci[e]) for wi, ci in zip(wr, c))
        expect = Fraction(int(a == b and g == e) + int(a == g and b == e) + int(a == e and b == g), 9)
        assert m4 == expect


@pytest.mark.parametrize("lat,d,q", LATTICES)
def test_equilibrium_moments(orc, lat, d, q):
    """Eq. 13: the equilibrium carries rho, rho u and rho cs^2 I + rho u u."""
    _, c, w, _ = orc.lattice_info(lat)
    rng = np.random.default_rng(5)
    for _ in range(20):
        rho = 1.0 + 0.1 * rng.standard_normal()
        u = 0.05 * rng.standard_normal(3)
        if d == 2:
            u[2] = 0.0
        feq = orc.equilibrium(lat, rho, u)
        assert abs(feq.sum() - rho) < 1e-15
        assert np.allclose(c.T @ feq, rho * u, atol=1e-16, rtol=0)
        Pi = np.einsum("ia,ib,i->ab", c, c, feq)
        expect = rho * np.outer(u, u) + rho / 3.0 * np.diag([1.0] * d + [0.0] * (3 - d))
        assert np.allclose(Pi, expect, atol=2e-16, rtol=0)


def test_equilibrium_rest_is_weights(orc):
    for lat, _, _ in LATTICES:
        _, _, w, _ = orc.lattice_info(lat)
        assert np.array_equal(orc.equilibrium(lat, 1.0, (0, 0, 0)), w)
