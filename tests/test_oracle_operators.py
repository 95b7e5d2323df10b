"""Per-node pins of the oracle's collision operators (Sec. 2.1-2.4, 3.1-3.2).

Each check is a property the paper or the mathematics fixes, not a re-typing
of the oracle's formulas: conservation, the Newtonian limits the paper states
(IR reduces to the BGK second moment, Eqs. 32-33; PR with zero yield stress is
TRT, and TRT with tau_odd = tau_even is BGK), the defining equations of the
IR solve (Eqs. 31 and 38), and continuity of both models at their switches.
"""
import numpy as np
import pytest

LATS = [0, 1, 2]


def _random_node(orc, lat, rng, amp=2e-3, ueq=0.05):
    d, c, w, _ = orc.lattice_info(lat)
    rho = 1.0 + 0.02 * rng.standard_normal()
    u = ueq * rng.standard_normal(3)
    if d == 2:
        u[2] = 0
    fbar = orc.equilibrium(lat, rho, u) + w * amp * rng.standard_normal(len(w))
    return d, c, w, fbar


def _hermite2(c, w, X, d):
    """Populations whose zeroth and first moments vanish and whose second
    moment is the symmetric tensor X (second-order Hermite projection)."""
    I = np.diag([1.0] * d + [0.0] * (3 - d))
    H = np.einsum("ia,ib->iab", c, c) - I[None] / 3.0
    return w * 4.5 * np.einsum("iab,ab->i", H, X)


def _dev(M, d):
    M = M.copy()
    tr = np.trace(M[:d, :d])
    for a in range(d):
        M[a, a] -= tr / d
    return M


@pytest.mark.parametrize("lat", LATS)
@pytest.mark.parametrize("op", ["PR", "IR", "BGK"])
def test_mass_and_momentum(orc, lat, op):
    """Collision keeps mass and adds exactly F = rho g of momentum."""
    rng = np.random.default_rng(11 + lat)
    g = np.array([3e-5, -2e-5, 1e-5])
    for _ in range(25):
        d, c, w, fbar = _random_node(orc, lat, rng)
        gg = g.copy()
        if d == 2:
            gg[2] = 0
        rho, j = fbar.sum(), c.T @ fbar
        if op == "PR":
            rh = orc.rheology(orc.PR, 0.1, 1e-4, 1e4, 1e-8, 0.25, gg)
            fpost, _ = orc.collide_pr(lat, rh, fbar, 0.5 + 3 * 1.1)
        elif op == "IR":
            rh = orc.rheology(orc.IR, 0.1, 1e-4, g=gg)
            fpost, _ = orc.collide_ir(lat, rh, fbar)
        else:
            rh = orc.rheology(orc.BGK, 0.1, g=gg)
            fpost, _ = orc.collide_bgk(lat, rh, fbar)
        assert abs(fpost.sum() - rho) < 2e-15
        assert np.allclose(c.T @ fpost, j + rho * gg, atol=1e-16, rtol=0)


@pytest.mark.parametrize("lat", LATS)
@pytest.mark.parametrize("nu", [0.01, 0.1, 0.5])
def test_ir_newtonian_equals_bgk_second_moment(orc, lat, nu):
    """Sec. 2.3: with sigma = 2 rho nu D the IR construction gives the second
    moment of the BGK operator (Eqs. 32-33).  Deviatoric parts must agree."""
    rng = np.random.default_rng(3)
    for _ in range(25):
        d, c, w, fbar = _random_node(orc, lat, rng)
        rho, j = fbar.sum(), c.T @ fbar
        u = j / rho
        feq = orc.equilibrium(lat, rho, u)
        ir, _ = orc.collide_ir(lat, orc.rheology(orc.IR, nu, 0.0), fbar)
        bgk, _ = orc.collide_bgk(lat, orc.rheology(orc.BGK, nu), fbar)
        m_ir = np.einsum("ia,ib,i->ab", c, c, ir - feq)
        m_bgk = np.einsum("ia,ib,i->ab", c, c, bgk - feq)
        assert np.max(np.abs(_dev(m_ir, d) - _dev(m_bgk, d))) < 1e-15, np.max(np.abs(_dev(m_ir, d) - _dev(m_bgk, d)))
        assert abs(np.trace(m_ir[:d, :d])) < 1e-15  # trace is not carried


@pytest.mark.parametrize("lat", LATS)
def test_ir_unyielded_keeps_stress(orc, lat):
    """Unyielded branch (Eq. 40): s = 0 and sigma = -T, so the post-collision
    non-equilibrium second moment is the deviator of T itself."""
    rng = np.random.default_rng(4)
    d, c, w, _ = orc.lattice_info(lat)
    for _ in range(10):
        rho = 1.0 + 0.01 * rng.standard_normal()
        u = 0.03 * rng.standard_normal(3)
        if d == 2:
            u[2] = 0
        X = rng.standard_normal((3, 3)) * 1e-5
        X = X + X.T
        X[d:, :] = 0
        X[:, d:] = 0
        fbar = orc.equilibrium(lat, rho, u) + _hermite2(c, w, X, d)
        Tn = np.linalg.norm(_dev(X, d))
        rh = orc.rheology(orc.IR, 0.1, 1.01 * Tn / np.sqrt(2.0))
        fpost, info = orc.collide_ir(lat, rh, fbar)
        assert info["unyielded"]
        assert abs(info["T"] - Tn) < 1e-15
        feq = orc.equilibrium(lat, rho, u)
        M = np.einsum("ia,ib,i->ab", c, c, fpost - feq)
        assert np.allclose(M, _dev(X, d), atol=2e-16, rtol=1e-11)
        assert np.all(info["s"] == 0)


@pytest.mark.parametrize("lat", LATS)
def test_ir_yielded_solves_the_implicit_equation(orc, lat):
    """Yielded branch: the returned s and sigma satisfy s/2 + T = -sigma
    (Eq. 31) and the Bingham law in s, sigma = (3 nu_p + sqrt2 sigma_y/|s|) s
    (Eq. 38), with the deviator of T."""
    rng = np.random.default_rng(6)
    for _ in range(25):
        d, c, w, fbar = _random_node(orc, lat, rng)
        rho = fbar.sum()
        nu_p = 10 ** rng.uniform(-2, 0)
        rh0 = orc.rheology(orc.IR, nu_p, 0.0)
        _, i0 = orc.collide_ir(lat, rh0, fbar)
        sy = 0.3 * i0["T"] / np.sqrt(2.0)
        rh = orc.rheology(orc.IR, nu_p, sy)
        _, info = orc.collide_ir(lat, rh, fbar)
        assert not info["unyielded"]
        feq = orc.equilibrium(lat, rho, info["u"])
        T = _dev(np.einsum("ia,ib,i->ab", c, c, fbar - feq), d)
        s, sig = info["s"], info["sigma"]
        assert np.allclose(0.5 * s + T, -sig, atol=2e-16, rtol=1e-10)
        sn = np.linalg.norm(s)
        assert sn > 0
        assert np.allclose(sig, (3 * nu_p + np.sqrt(2) * sy / sn) * s, atol=2e-16, rtol=1e-9)


@pytest.mark.parametrize("lat", LATS)
def test_ir_continuous_at_yield(orc, lat):
    """Both branches of Eq. 40 meet at T = sqrt(2) sigma_y."""
    rng = np.random.default_rng(7)
    d, c, w, fbar = _random_node(orc, lat, rng)
    _, i0 = orc.collide_ir(lat, orc.rheology(orc.IR, 0.1, 0.0), fbar)
    sy_crit = i0["T"] / np.sqrt(2.0)
    lo, ilo = orc.collide_ir(lat, orc.rheology(orc.IR, 0.1, sy_crit * (1 + 1e-9)), fbar)
    hi, ihi = orc.collide_ir(lat, orc.rheology(orc.IR, 0.1, sy_crit * (1 - 1e-9)), fbar)
    assert ilo["unyielded"] and not ihi["unyielded"]
    assert np.max(np.abs(lo - hi)) < 1e-9 * i0["T"] + 2e-16


@pytest.mark.parametrize("lat", LATS)
def test_pr_newtonian_limit_is_trt_and_bgk(orc, lat):
    """Zero yield stress: nu_app = nu_p exactly, so tau_even = 1/2 + 3 nu_p;
    with Lambda = (tau - 1/2)^2 the odd time equals tau and PR is BGK."""
    rng = np.random.default_rng(8)
    for _ in range(20):
        d, c, w, fbar = _random_node(orc, lat, rng)
        nu = 10 ** rng.uniform(-2, 0)
        tau = 0.5 + 3 * nu
        g = (1e-5, 2e-6, 0.0)
        rh = orc.rheology(orc.PR, nu, 0.0, 1e6, 1e-8, (tau - 0.5) ** 2, g)
        fpr, info = orc.collide_pr(lat, rh, fbar, 0.5 + 3 * nu * rng.uniform(0.5, 2))
        assert info["nu_app"] == nu and abs(info["tau"] - tau) < 1e-15 * tau
        fb, _ = orc.collide_bgk(lat, orc.rheology(orc.BGK, nu, g=g), fbar)
        assert np.max(np.abs(fpr - fb)) < 5e-16


@pytest.mark.parametrize("lat", LATS)
def test_pr_strain_rate_from_nonequilibrium(orc, lat):
    """Sec. 2.2, Eq. 24 with Eq. 4: a node whose non-equilibrium second moment
    is -2 rho cs^2 tau D reports gamma_dot = sqrt(2 D:D)."""
    rng = np.random.default_rng(9)
    d, c, w, _ = orc.lattice_info(lat)
    for _ in range(10):
        rho = 1.0 + 0.01 * rng.standard_normal()
        u = 0.02 * rng.standard_normal(3)
        if d == 2:
            u[2] = 0
        D = rng.standard_normal((3, 3)) * 1e-4
        D = 0.5 * (D + D.T)
        D[d:, :] = 0
        D[:, d:] = 0
        tau_prev = 0.5 + 3 * 0.2
        fbar = orc.equilibrium(lat, rho, u) + _hermite2(c, w, -2 * rho / 3 * tau_prev * D, d)
        rh = orc.rheology(orc.PR, 0.1, 1e-5, 1e3, 1e-8, 0.25)
        _, info = orc.collide_pr(lat, rh, fbar, tau_prev)
        assert abs(info["gamma"] - np.sqrt(2 * np.sum(D * D))) < 1e-12 * info["gamma"]


def test_papanastasiou_viscosity(orc):
    """Eq. 36 and the zero-strain interpolation of Eq. 37: finite limit
    nu_0 = nu_p + m sigma_y / rho at zero strain, continuity at the cut-off,
    the Bingham asymptote at large m gamma, and monotone decrease."""
    nu_p, sy, m, gc = 0.1, 1.6e-4, 1e4, 1e-8
    rh = orc.rheology(orc.PR, nu_p, sy, m, gc)
    for rho in (1.0, 0.97):
        nu0 = nu_p + m * sy / rho
        assert orc.nu_app(rh, 0.0, rho) == nu0
        assert abs(orc.nu_app(rh, gc * (1 - 1e-12), rho) - orc.nu_app(rh, gc, rho)) < 1e-12 * nu0
        for gd in (1e-2, 1e-1):
            assert abs(orc.nu_app(rh, gd, rho) - (nu_p + sy / (rho * gd))) < 1e-12
        g = np.logspace(-12, 0, 400)
        v = np.array([orc.nu_app(rh, x, rho) for x in g])
        assert np.all(np.diff(v) < 0)
    # no yield stress: exactly the plastic viscosity everywhere
    rh0 = orc.rheology(orc.PR, nu_p, 0.0, m, gc)
    assert all(orc.nu_app(rh0, x) == nu_p for x in (0.0, 1e-9, 1e-8, 1e-3))
