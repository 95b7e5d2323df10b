"""Pins of the oracle's MRT base collision (Sec. 2.1, Eq. 20, and the strain
rate of Eq. 23).  The paper fixes neither the moment basis nor the rates of
the non-hydrodynamic moments; the oracle's basis is the weighted
Gram-Schmidt orthogonalisation of the monomials c_x^a c_y^b c_z^c (a, b, c
<= 2) in order of degree, grouped as conserved, bulk, shear, odd and even.

  * the basis: q rows, orthogonal under the weights, with the group sizes
    the monomials imply on each lattice;
  * all rates equal is BGK, and shear = bulk = even rates with the odd rate
    from the magic number is TRT (to rounding);
  * mass is kept and momentum grows by exactly rho g per step;
  * the hydrodynamics are set by the shear rate and the magic number alone:
    shear waves decay at nu k^2 and the Poiseuille profile keeps TRT's slip
    law, whatever the bulk and even rates.
"""
import ctypes

import numpy as np
import pytest

GROUPS = {0: dict(conserved=3, bulk=1, shear=2, odd=2, even=1),
          1: dict(conserved=4, bulk=1, shear=5, odd=6, even=3),
          2: dict(conserved=4, bulk=1, shear=5, odd=10, even=7)}


def _state(orc, lat, rng, amp=1e-3):
    _, _, w, _ = orc.lattice_info(lat)
    u = rng.uniform(-0.02, 0.02, 3) * (1, 1, lat > 0)
    return orc.equilibrium(lat, 1.0 + rng.uniform(-0.01, 0.01), u) + amp * w * rng.uniform(-1, 1, len(w))


@pytest.mark.parametrize("lat", [0, 1, 2])
def test_basis_groups_and_orthogonality(orc, lat):
    """Through the collision operator: with rates e_k (one group at a time
    set to 1, the others to 0 -- emulated by differences of collisions), the
    operator M^{-1} S M restricted to a group is a projector whose rank is
    the group size."""
    q = {0: 9, 1: 19, 2: 27}[lat]
    _, _, w, _ = orc.lattice_info(lat)
    nu = 0.1
    tau = 0.5 + 3 * nu
    rng = np.random.default_rng(lat)
    # the map f_neq -> collision change is linear; build it column by column
    # for two rate settings that differ only in the even group
    def op_matrix(mb, me, lam):
        rh = orc.rheology(orc.PR, nu, 0.0, 0.0, 1e-8, lam, (0, 0, 0), mrt_bulk=mb, mrt_even=me)
        feq = orc.equilibrium(lat, 1.0, (0.0, 0.0, 0.0))
        cols = []
        for j in range(q):
            f = feq.copy()
            f[j] += 1e-6
            fp, _ = orc.collide_pr(lat, rh, f, tau)
            cols.append((f - fp) / 1e-6)  # = M^-1 S M e_j (velocity stays 0 to first order)
        return np.array(cols).T
    lam_bgk = (tau - 0.5) ** 2
    A = op_matrix(0.5, 0.5, lam_bgk)
    B = op_matrix(0.5, 1.5, lam_bgk)
    # difference isolates the even group (rate difference 1): a projector of
    # rank = number of even rows
    P = B - A
    sv = np.linalg.svd(P, compute_uv=False)
    assert int(np.sum(sv > 1e-3)) == GROUPS[lat]["even"]
    C = op_matrix(1.5, 0.5, lam_bgk)
    sv = np.linalg.svd(C - A, compute_uv=False)
    assert int(np.sum(sv > 1e-3)) == GROUPS[lat]["bulk"]
    # projectors: P^2 = P (rows orthogonal under the weights)
    assert np.allclose(P @ P, P, atol=1e-6)


@pytest.mark.parametrize("lat", [0, 1, 2])
def test_equal_rates_is_bgk_and_grouped_rates_is_trt(orc, lat):
    rng = np.random.default_rng(11 + lat)
    nu = 0.07
    tau = 0.5 + 3 * nu
    g = (1e-6, -2e-6, 0.0 if lat == 0 else 3e-6)
    for _ in range(5):
        f = _state(orc, lat, rng)
        rh_m = orc.rheology(orc.PR, nu, 0.0, 0.0, 1e-8, (tau - 0.5) ** 2, g, mrt_bulk=1 / tau, mrt_even=1 / tau)
        a, _ = orc.collide_pr(lat, rh_m, f, tau)
        b, _ = orc.collide_bgk(lat, orc.rheology(orc.BGK, nu, g=g), f)
        assert np.max(np.abs(a - b)) <= 1e-15
        rh_t = orc.rheology(orc.PR, nu, 0.0, 0.0, 1e-8, 0.25, g)
        rh_m2 = orc.rheology(orc.PR, nu, 0.0, 0.0, 1e-8, 0.25, g, mrt_bulk=1 / tau, mrt_even=1 / tau)
        c, _ = orc.collide_pr(lat, rh_t, f, tau)
        d, _ = orc.collide_pr(lat, rh_m2, f, tau)
        assert np.max(np.abs(c - d)) <= 1e-15


@pytest.mark.parametrize("lat", [0, 2])
def test_conservation(orc, lat):
    rng = np.random.default_rng(21 + lat)
    dims = (5, 4, 1) if lat == 0 else (3, 4, 2)
    g = np.array([2e-5, -1e-5, 5e-6 if lat else 0.0])
    rh = orc.rheology(orc.PR, 0.05, 1e-5, 1e4, 1e-8, 0.25, g, mrt_bulk=1.1, mrt_even=1.7)
    dom = orc.Domain(lat, dims, (1, 1, 1), rh)
    N = dom.N
    P = np.stack([_state(orc, lat, rng) for _ in range(N)], axis=1)
    dom.set_state(P)

    def totals():
        Pm, _ = dom.get_state()
        return Pm.sum(), (dom.c.T @ Pm).sum(axis=1)

    M0, J0 = totals()
    dom.step(50)
    M1, J1 = totals()
    assert abs(M1 - M0) < 50 * N * 1e-15
    assert np.allclose(J1 - J0, 50 * M0 * g, rtol=1e-10, atol=1e-15)


@pytest.mark.parametrize("lat", [0, 1, 2])
def test_shear_wave_decay_independent_of_ghost_rates(orc, lat):
    """u_x = U sin(k y) decays as exp(-nu k^2 t) for any bulk/even rates."""
    n, nu, U = 32, 0.08, 1e-4
    k = 2 * np.pi / n
    dims = (1, n, 1) if lat == 0 else (1, n, 1)
    rates = []
    for mb, me in ((0.0, 0.0), (0.8, 1.9)):
        rh = orc.rheology(orc.PR, nu, 0.0, 0.0, 1e-8, 0.25, (0, 0, 0), mrt_bulk=mb, mrt_even=me)
        dom = orc.Domain(lat, dims, (1, 1, 1), rh)
        y = np.arange(n)
        P = np.stack([orc.equilibrium(lat, 1.0, (U * np.sin(k * yy), 0, 0)) for yy in y], axis=1)
        dom.set_state(P)
        dom.step(400)
        _, u, _, _ = dom.moments()
        amp = 2 * np.mean(u[0] * np.sin(k * y))
        rates.append(-np.log(amp / U) / 400)
    assert abs(rates[0] / (nu * k * k) - 1) < 5e-3
    assert abs(rates[1] / rates[0] - 1) < 1e-3


def test_poiseuille_keeps_trt_slip_law(orc):
    H, g, nu = 32, 1e-5, 0.1
    for lam in (0.25, 3 / 16):
        rh = orc.rheology(orc.PR, nu, 0.0, 0.0, 1e-8, lam, (g, 0, 0), mrt_bulk=1.3, mrt_even=1.7)
        d = orc.Domain(0, (2, H, 1), (1, 0, 1), rh)
        d.step(30000)
        _, u, _, _ = d.moments()
        y = np.arange(H) + 0.5
        exact = g / (2 * nu) * (y * (H - y) + (16 * lam - 3) / 12)
        assert np.max(np.abs(u[0][::2] - exact)) <= 1e-6 * exact.max()
