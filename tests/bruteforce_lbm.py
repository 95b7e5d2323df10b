"""A second, literal implementation of the lattice Boltzmann update of the
paper, for brute-force comparison with the oracle on tiny grids.

It is written independently of ``oracle/lbm_oracle.c``: its own velocity
tables (typed out below, in an order neither the oracle nor the GPU library
uses), explicit Python loops over nodes, directions and tensor components,
and its own root finders where the oracle uses closed forms.  It follows the
same readings of the paper's garbled passages, each noted where used.

State: ``P[i][n]`` post-collision populations (this module's velocity
order), node index n = x + nx (y + ny z), mask 1 = solid.  Streaming pulls
f_i(x) = P_i(x - c_i) (Sec. 2, Eq. 10), with halfway bounce-back
f_i(x) = P_opp(i)(x) when x - c_i is solid or beyond a wall (Sec. 4.3).
"""
from __future__ import annotations

import math

CS2 = 1.0 / 3.0

# Velocity sets of Sec. 4.1, typed out: (cx, cy, cz, w).  D2Q9 and D3Q19 are
# subsets of D3Q27 restricted by dimension and speed.
_D2Q9 = [
    (1, 1, 0, 1 / 36), (1, 0, 0, 1 / 9), (1, -1, 0, 1 / 36),
    (0, 1, 0, 1 / 9), (0, 0, 0, 4 / 9), (0, -1, 0, 1 / 9),
    (-1, 1, 0, 1 / 36), (-1, 0, 0, 1 / 9), (-1, -1, 0, 1 / 36),
]
_D3Q19 = [
    (1, 1, 0, 1 / 36), (1, 0, 1, 1 / 36), (1, 0, 0, 1 / 18), (1, 0, -1, 1 / 36), (1, -1, 0, 1 / 36),
    (0, 1, 1, 1 / 36), (0, 1, 0, 1 / 18), (0, 1, -1, 1 / 36), (0, 0, 1, 1 / 18), (0, 0, 0, 1 / 3),
    (0, 0, -1, 1 / 18), (0, -1, 1, 1 / 36), (0, -1, 0, 1 / 18), (0, -1, -1, 1 / 36),
    (-1, 1, 0, 1 / 36), (-1, 0, 1, 1 / 36), (-1, 0, 0, 1 / 18), (-1, 0, -1, 1 / 36), (-1, -1, 0, 1 / 36),
]
_D3Q27 = [
    (1, 1, 1, 1 / 216), (1, 1, 0, 1 / 54), (1, 1, -1, 1 / 216), (1, 0, 1, 1 / 54), (1, 0, 0, 2 / 27),
    (1, 0, -1, 1 / 54), (1, -1, 1, 1 / 216), (1, -1, 0, 1 / 54), (1, -1, -1, 1 / 216),
    (0, 1, 1, 1 / 54), (0, 1, 0, 2 / 27), (0, 1, -1, 1 / 54), (0, 0, 1, 2 / 27), (0, 0, 0, 8 / 27),
    (0, 0, -1, 2 / 27), (0, -1, 1, 1 / 54), (0, -1, 0, 2 / 27), (0, -1, -1, 1 / 54),
    (-1, 1, 1, 1 / 216), (-1, 1, 0, 1 / 54), (-1, 1, -1, 1 / 216), (-1, 0, 1, 1 / 54), (-1, 0, 0, 2 / 27),
    (-1, 0, -1, 1 / 54), (-1, -1, 1, 1 / 216), (-1, -1, 0, 1 / 54), (-1, -1, -1, 1 / 216),
]
TABLES = {0: _D2Q9, 1: _D3Q19, 2: _D3Q27}
DIM = {0: 2, 1: 3, 2: 3}


def velocities(lattice):
    """[(c, w)], opp: this module's velocity order and opposite indices."""
    tab = TABLES[lattice]
    cs = [(cx, cy, cz) for cx, cy, cz, _ in tab]
    ws = [w for *_, w in tab]
    opp = [cs.index((-cx, -cy, -cz)) for cx, cy, cz in cs]
    return cs, ws, opp


def feq(cs, ws, rho, u):
    """Second-order equilibrium (Sec. 2.1, Eq. 12)."""
    uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2]
    out = []
    for c, w in zip(cs, ws):
        cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2]
        out.append(rho * w * (1.0 + cu / CS2 + cu * cu / (2 * CS2 * CS2) - uu / (2 * CS2)))
    return out


def nu_app(p, gamma, rho):
    """Papanastasiou viscosity (Eq. 36) with the zero-strain interpolation of
    Eq. 37.  Reading: the interpolation is the straight line between
    (0, nu_0) and (gamma_c, nu_app(gamma_c)) (denominator gamma_c)."""
    def pap(gm):  # 1 - exp(-m gm), evaluated without cancellation at small m gm
        return p["nu_p"] + p["sigma_y"] / (rho * gm) * (-math.expm1(-p["m"] * gm))
    if gamma >= p["gamma_c"]:
        return pap(gamma)
    nu0 = p["nu_p"] + p["m"] * p["sigma_y"] / rho
    t = gamma / p["gamma_c"]
    return (1.0 - t) * nu0 + t * pap(p["gamma_c"])


def _moments(cs, f):
    rho = sum(f)
    j = [sum(c[a] * fi for c, fi in zip(cs, f)) for a in range(3)]
    return rho, j


def _second(cs, f, g):
    """sum_i c_i c_i (f_i - g_i), a 3x3 list."""
    M = [[0.0] * 3 for _ in range(3)]
    for c, fi, gi in zip(cs, f, g):
        d = fi - gi
        for a in range(3):
            for b in range(3):
                M[a][b] += c[a] * c[b] * d
    return M


def _bisect(F, lo, hi):
    """Root of an increasing F on [lo, hi] (F(lo) <= 0 <= F(hi)), to
    adjacent doubles."""
    while True:
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            return 0.5 * (lo + hi)
        if F(mid) > 0.0:
            hi = mid
        else:
            lo = mid


def strain_rate(cs, f, fe, rho, tau, axis):
    """gamma_dot = sqrt(2 D:D) with D = -Pi_neq / (2 rho cs^2 tau) (Sec. 2.2,
    Eq. 24; reading: the density of Eq. 33 kept), full tensor; with a known
    flow axis its normal component is dropped (Sec. 4.2.2)."""
    Pn = _second(cs, f, fe)
    s = 0.0
    for a in range(3):
        for b in range(3):
            if axis and a == b == axis - 1:
                continue
            d = -Pn[a][b] / (2.0 * rho * CS2 * tau)
            s += d * d
    return math.sqrt(2.0 * s)


def collide_pr(cs, ws, opp, p, f, tau_prev, implicit=False):
    """PR: TRT with the Papanastasiou viscosity and the EDM force (Sec. 2.1,
    2.4, 3.1).  implicit: the relaxation time consistent with its own strain
    rate (Sec. 3), else the previous step's (explicit update)."""
    rho, j = _moments(cs, f)
    u = [ja / rho for ja in j]
    fe = feq(cs, ws, rho, u)
    if implicit:
        G = strain_rate(cs, f, fe, rho, 1.0, p["axis"])  # strain rate at tau = 1 scales as 1/tau
        lo = 0.5 + p["nu_p"] / CS2
        hi = 0.5 + (p["nu_p"] + p["m"] * p["sigma_y"] / rho) / CS2
        tau_prev = _bisect(lambda t: t - 0.5 - nu_app(p, G / t, rho) / CS2, lo, hi)
    gamma = strain_rate(cs, f, fe, rho, tau_prev, p["axis"])
    nu = nu_app(p, gamma, rho)
    te = 0.5 + nu / CS2
    to = 0.5 + p["lambda"] / (te - 0.5)
    fs = feq(cs, ws, rho, [u[a] + p["g"][a] for a in range(3)])
    out = []
    for i in range(len(cs)):
        k = opp[i]
        sym = 0.5 * (f[i] + f[k]) - 0.5 * (fe[i] + fe[k])
        asym = 0.5 * (f[i] - f[k]) - 0.5 * (fe[i] - fe[k])
        out.append(f[i] - sym / te - asym / to + (fs[i] - fe[i]))
    uo = [u[a] + 0.5 * p["g"][a] for a in range(3)]
    return out, te, uo, (rho * nu * gamma < p["sigma_y"])


def collide_ir(cs, ws, d, p, f, hb=False):
    """IR (Sec. 2.3, 3.2) with the force term of Sec. 2.4.  Readings: the
    equilibrium half a step back is f_eq(u) - Phi/2 with u = (j + F/2)/rho
    and Phi_i = w_i c_i.F / cs^2; only the deviator (trace / d) of T enters;
    yielded when |dev T| > sqrt(2) sigma_y; f_sigma = w_i/(2 cs^4)
    (c_i c_i - cs^2 I) : (-sigma + s/2).  The magnitude of s is found here by
    bisection of the contraction of Eq. 31 (Bingham law of Eq. 38, or the
    Herschel-Bulkley law with hb)."""
    rho, j = _moments(cs, f)
    F = [rho * ga for ga in p["g"]]
    u = [(j[a] + 0.5 * F[a]) / rho for a in range(3)]
    fe = feq(cs, ws, rho, u)
    phi = [w * (c[0] * F[0] + c[1] * F[1] + c[2] * F[2]) / CS2 for c, w in zip(cs, ws)]
    back = [fe[i] - 0.5 * phi[i] for i in range(len(cs))]
    T = _second(cs, f, back)
    if p["axis"]:
        T[p["axis"] - 1][p["axis"] - 1] = 0.0
    tr = sum(T[a][a] for a in range(d))
    Td = [[T[a][b] - (tr / d if (a == b and a < d) else 0.0) for b in range(3)] for a in range(3)]
    Tn = math.sqrt(sum(Td[a][b] * Td[a][b] for a in range(3) for b in range(3)))
    thr = math.sqrt(2.0) * p["sigma_y"]
    if Tn > thr:
        if hb:
            kk = 3.0 * p["nu_p"] * (3.0 / math.sqrt(2.0)) ** (p["hb_n"] - 1.0)
            smag = _bisect(lambda s: 0.5 * s + kk * s ** p["hb_n"] + thr - Tn, 0.0, 2.0 * (Tn - thr))
        else:
            smag = _bisect(lambda s: 0.5 * s + 3.0 * p["nu_p"] * s + thr - Tn, 0.0, 2.0 * (Tn - thr))
        # s and sigma point along -dev T; |s/2 + sigma| = |T| fixes |sigma|
        sig_mag = Tn - 0.5 * smag
        s = [[-smag * Td[a][b] / Tn for b in range(3)] for a in range(3)]
        sig = [[-sig_mag * Td[a][b] / Tn for b in range(3)] for a in range(3)]
        unyielded = False
    else:
        s = [[0.0] * 3 for _ in range(3)]
        sig = [[-Td[a][b] for b in range(3)] for a in range(3)]
        unyielded = True
    A = [[-sig[a][b] + 0.5 * s[a][b] for b in range(3)] for a in range(3)]
    out = []
    for i, (c, w) in enumerate(zip(cs, ws)):
        con = 0.0
        for a in range(3):
            for b in range(3):
                con += (c[a] * c[b] - (CS2 if (a == b and a < d) else 0.0)) * A[a][b]
        out.append(back[i] + w / (2.0 * CS2 * CS2) * con + phi[i])
    return out, u, unyielded


class Grid:
    """Tiny domain stepped by explicit loops."""

    def __init__(self, lattice, dims, periodic, params, mask=None):
        self.lat = lattice
        self.cs, self.ws, self.opp = velocities(lattice)
        self.d = DIM[lattice]
        self.q = len(self.cs)
        self.nx, self.ny, self.nz = dims
        self.N = self.nx * self.ny * self.nz
        self.per = list(periodic)
        if self.d == 2:
            self.per[2] = 1
        self.p = dict(params)
        self.mask = [0] * self.N if mask is None else [int(v) for v in mask]
        self.P = [[0.0] * self.N for _ in range(self.q)]
        self.tau = [0.5] * self.N

    def _pull(self, x, y, z):
        n = x + self.nx * (y + self.ny * z)
        f = []
        for i, c in enumerate(self.cs):
            src = [x - c[0], y - c[1], z - c[2]]
            dims = [self.nx, self.ny, self.nz]
            blocked = False
            for a in range(3):
                if src[a] < 0 or src[a] >= dims[a]:
                    if self.per[a]:
                        src[a] %= dims[a]
                    else:
                        blocked = True
            m = None if blocked else src[0] + self.nx * (src[1] + self.ny * src[2])
            if m is None or self.mask[m]:
                f.append(self.P[self.opp[i]][n])  # halfway bounce-back
            else:
                f.append(self.P[i][m])
        return f

    def _collide(self, f, tau_prev):
        op = self.p["op"]
        if op in ("PR", "PRI"):
            out, te, uo, uy = collide_pr(self.cs, self.ws, self.opp, self.p, f, tau_prev, implicit=(op == "PRI"))
            return out, te, uo, uy
        out, uo, uy = collide_ir(self.cs, self.ws, self.d, self.p, f, hb=(op == "IRHB"))
        return out, tau_prev, uo, uy

    def step(self, n=1):
        for _ in range(n):
            Pn = [[0.0] * self.N for _ in range(self.q)]
            tn = list(self.tau)
            for z in range(self.nz):
                for y in range(self.ny):
                    for x in range(self.nx):
                        k = x + self.nx * (y + self.ny * z)
                        if self.mask[k]:
                            continue
                        out, tn[k], _, _ = self._collide(self._pull(x, y, z), self.tau[k])
                        for i in range(self.q):
                            Pn[i][k] = out[i]
            self.P, self.tau = Pn, tn

    def moments(self):
        """rho, u (output velocity, [3][N]), unyielded flags at the current
        time (of the populations the next collision would see)."""
        rho = [0.0] * self.N
        u = [[0.0] * self.N for _ in range(3)]
        uy = [0] * self.N
        for z in range(self.nz):
            for y in range(self.ny):
                for x in range(self.nx):
                    k = x + self.nx * (y + self.ny * z)
                    if self.mask[k]:
                        continue
                    f = self._pull(x, y, z)
                    rho[k] = sum(f)
                    _, _, uo, flag = self._collide(f, self.tau[k])
                    for a in range(3):
                        u[a][k] = uo[a]
                    uy[k] = int(flag)
        return rho, u, uy

    def monitors(self):
        """Superficial flux (sum of u over fluid nodes / all nodes), mass,
        max |u|, unyielded and fluid counts."""
        rho, u, uy = self.moments()
        fl = [k for k in range(self.N) if not self.mask[k]]
        flux = [sum(u[a][k] for k in fl) / self.N for a in range(3)]
        umax = max([math.sqrt(sum(u[a][k] ** 2 for a in range(3))) for k in fl] or [0.0])
        return {"flux": flux, "mass": sum(rho[k] for k in fl), "umax": umax,
                "unyielded": sum(uy[k] for k in fl), "fluid": len(fl)}
