"""Plain FP64 CPU oracle of the Bingham-fluid lattice Boltzmann update
(Regulski, Leonardi & Szumbarski, arXiv:1610.01388).

TEST INFRASTRUCTURE ONLY.  Imported by the tests, by the smoke check and by
the CPU-baseline leg of the benchmark to check the GPU library; the product
package never imports it.  The arithmetic lives in ``lbm_oracle.c`` (plain C,
one node at a time); this module only builds and loads it and marshals numpy
arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
# Tests that plant mistakes in a copy of the oracle load that copy instead.
_LIB_OVERRIDE = os.environ.get("LBM_ORACLE_LIB")

D2Q9, D3Q19, D3Q27 = 0, 1, 2
PR, IR, BGK, PRI, IRHB = 0, 1, 2, 3, 4


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-fopenmp",
                               "-fno-fast-math", "-ffp-contract=off", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class Rheology(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("flow_axis", ctypes.c_int32),
                ("nu_p", ctypes.c_double), ("sigma_y", ctypes.c_double),
                ("m", ctypes.c_double), ("gamma_c", ctypes.c_double),
                ("lambda_", ctypes.c_double), ("g", ctypes.c_double * 3),
                ("mrt_bulk", ctypes.c_double), ("mrt_even", ctypes.c_double), ("hb_n", ctypes.c_double)]


def rheology(op, nu_p, sigma_y=0.0, m=0.0, gamma_c=1e-8, lam=0.25, g=(0.0, 0.0, 0.0), flow_axis=0,
             mrt_bulk=0.0, mrt_even=0.0, hb_n=1.0):
    """flow_axis: 0 off, 1/2/3 = x/y/z -- drop the axis-normal component
    from the collision (Sec. 4.2.2).  mrt_bulk, mrt_even: MRT rates of the
    bulk moment and of the even moments of order >= 4 (0: TRT).  IRHB:
    nu_p is the consistency K and hb_n the flow index."""
    r = Rheology()
    r.hb_n = hb_n
    r.op = op
    r.flow_axis = flow_axis
    r.mrt_bulk = mrt_bulk
    r.mrt_even = mrt_even
    r.nu_p = nu_p
    r.sigma_y = sigma_y
    r.m = m
    r.gamma_c = gamma_c
    r.lambda_ = lam
    for a in range(3):
        r.g[a] = g[a] if a < len(g) else 0.0
    return r


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            L = ctypes.CDLL(_LIB_OVERRIDE)
        else:
            if not os.path.exists(LIB):
                build(force=False)
            L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.orc_lattice_info.argtypes = [ctypes.c_int, ip, ip, dp, ip]
        L.orc_lattice_info.restype = ctypes.c_int
        L.orc_equilibrium.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
        L.orc_collide_pr.argtypes = [ctypes.c_int, ctypes.POINTER(Rheology), dp,
                                     ctypes.c_double, dp, dp]
        L.orc_collide_ir.argtypes = [ctypes.c_int, ctypes.POINTER(Rheology), dp, dp, dp]
        L.orc_collide_bgk.argtypes = [ctypes.c_int, ctypes.POINTER(Rheology), dp, dp, dp]
        L.orc_collide_pri.argtypes = [ctypes.c_int, ctypes.POINTER(Rheology), dp, dp, dp]
        L.orc_nu_app.argtypes = [ctypes.POINTER(Rheology), ctypes.c_double, ctypes.c_double]
        L.orc_nu_app.restype = ctypes.c_double
        L.orc_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ip,
                                 ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(Rheology)]
        L.orc_create.restype = ctypes.c_void_p
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_init_equilibrium.argtypes = [ctypes.c_void_p, ctypes.c_double, dp]
        L.orc_set_state.argtypes = [ctypes.c_void_p, dp, dp]
        L.orc_get_state.argtypes = [ctypes.c_void_p, dp, dp]
        L.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_set_threads.restype = ctypes.c_int
        L.orc_time.argtypes = [ctypes.c_void_p]
        L.orc_time.restype = ctypes.c_int64
        L.orc_moments.argtypes = [ctypes.c_void_p, dp, dp, dp, ctypes.POINTER(ctypes.c_uint8)]
        L.orc_monitors.argtypes = [ctypes.c_void_p, dp, ctypes.POINTER(ctypes.c_int64)]
        L.orc_residual.argtypes = [ctypes.c_void_p, dp, ctypes.c_int, dp]
        _lib = L
    return _lib


def set_threads(n: int = 0) -> int:
    """Threads the oracle's steps use (n > 0 sets the count); returns the
    count in effect.  Results are identical for every count."""
    return lib().orc_set_threads(int(n))


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def lattice_info(lattice):
    """(d, c[q,3], w[q], opp[q]) in the oracle's velocity order."""
    c = np.zeros((27, 3), dtype=np.int32)
    w = np.zeros(27)
    opp = np.zeros(27, dtype=np.int32)
    d = ctypes.c_int()
    q = lib().orc_lattice_info(lattice, ctypes.byref(d),
                               c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(w),
                               opp.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    if q < 0:
        raise ValueError("unknown lattice")
    return d.value, c[:q].copy(), w[:q].copy(), opp[:q].copy()


def equilibrium(lattice, rho, u):
    u = np.ascontiguousarray(np.resize(np.asarray(u, dtype=np.float64), 3))
    feq = np.zeros(27)
    q = lib().orc_equilibrium(lattice, rho, _dp(u), _dp(feq))
    return feq[:q].copy()


def collide_pr(lattice, rh, fbar, tau_prev):
    fbar = np.ascontiguousarray(fbar, dtype=np.float64)
    fpost = np.zeros(27)
    out = np.zeros(32)
    lib().orc_collide_pr(lattice, ctypes.byref(rh), _dp(fbar), tau_prev, _dp(fpost), _dp(out))
    q = fbar.size
    return fpost[:q].copy(), {"tau": out[0], "nu_app": out[1], "gamma": out[2],
                              "u": out[3:6].copy(), "unyielded": bool(out[6])}


def collide_ir(lattice, rh, fbar):
    fbar = np.ascontiguousarray(fbar, dtype=np.float64)
    fpost = np.zeros(27)
    out = np.zeros(32)
    lib().orc_collide_ir(lattice, ctypes.byref(rh), _dp(fbar), _dp(fpost), _dp(out))
    q = fbar.size
    return fpost[:q].copy(), {"u": out[0:3].copy(), "T": out[3], "unyielded": bool(out[4]),
                              "s": out[5:14].reshape(3, 3).copy(),
                              "sigma": out[14:23].reshape(3, 3).copy()}


def collide_pri(lattice, rh, fbar):
    """PR with the implicit relaxation-time update (no tau state)."""
    fbar = np.ascontiguousarray(fbar, dtype=np.float64)
    fpost = np.zeros(27)
    out = np.zeros(32)
    lib().orc_collide_pri(lattice, ctypes.byref(rh), _dp(fbar), _dp(fpost), _dp(out))
    q = fbar.size
    return fpost[:q].copy(), {"tau": out[0], "nu_app": out[1], "gamma": out[2],
                              "u": out[3:6].copy(), "unyielded": bool(out[6])}


def collide_bgk(lattice, rh, fbar):
    fbar = np.ascontiguousarray(fbar, dtype=np.float64)
    fpost = np.zeros(27)
    out = np.zeros(32)
    lib().orc_collide_bgk(lattice, ctypes.byref(rh), _dp(fbar), _dp(fpost), _dp(out))
    return fpost[:fbar.size].copy(), {"u": out[0:3].copy()}


def nu_app(rh, gamma, rho=1.0):
    return lib().orc_nu_app(ctypes.byref(rh), gamma, rho)


class Domain:
    """An oracle domain: dims (nx, ny, nz), periodic flags, uint8 mask (1 = solid)."""

    def __init__(self, lattice, dims, periodic, rh, mask=None):
        self.lattice = lattice
        self.dims = tuple(int(v) for v in dims)
        self.N = self.dims[0] * self.dims[1] * self.dims[2]
        self.d, self.c, self.w, self.opp = lattice_info(lattice)
        self.q = len(self.w)
        per = (ctypes.c_int * 3)(*[int(p) for p in periodic])
        self._mask = None
        mp = None
        if mask is not None:
            self._mask = np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
            assert self._mask.size == self.N
            mp = self._mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        self.rh = rh
        self._h = lib().orc_create(lattice, *self.dims, per, mp, ctypes.byref(rh))
        if not self._h:
            raise ValueError("oracle: invalid domain")

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def init_equilibrium(self, rho0=1.0, u0=(0.0, 0.0, 0.0)):
        u = np.ascontiguousarray(np.resize(np.asarray(u0, dtype=np.float64), 3))
        lib().orc_init_equilibrium(self._h, rho0, _dp(u))

    def set_state(self, P, tau=None):
        P = np.ascontiguousarray(P, dtype=np.float64).reshape(self.q, self.N)
        t = None if tau is None else np.ascontiguousarray(tau, dtype=np.float64).reshape(self.N)
        lib().orc_set_state(self._h, _dp(P), _dp(t))

    def get_state(self):
        P = np.zeros((self.q, self.N))
        tau = np.zeros(self.N)
        lib().orc_get_state(self._h, _dp(P), _dp(tau))
        return P, tau

    def step(self, n=1):
        lib().orc_step(self._h, int(n))

    @property
    def time(self):
        return lib().orc_time(self._h)

    def moments(self):
        rho = np.zeros(self.N)
        u = np.zeros((3, self.N))
        nu = np.zeros(self.N)
        uy = np.zeros(self.N, dtype=np.uint8)
        lib().orc_moments(self._h, _dp(rho), _dp(u), _dp(nu),
                          uy.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
        return rho, u, nu, uy

    def monitors(self):
        out = np.zeros(5)
        cnt = np.zeros(3, dtype=np.int64)
        lib().orc_monitors(self._h, _dp(out), cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
        return {"flux": out[0:3].copy(), "mass": out[3], "umax": out[4],
                "unyielded": int(cnt[0]), "nonfinite": int(cnt[1]), "fluid": int(cnt[2])}

    def residual(self, uprev, record=True):
        """Residual and max velocity change against uprev (3*N, component-
        major); with record, uprev is overwritten by the current velocity."""
        assert uprev.dtype == np.float64 and uprev.size == 3 * self.N and uprev.flags.c_contiguous
        out = np.zeros(2)
        lib().orc_residual(self._h, _dp(uprev), int(bool(record)), _dp(out))
        return {"residual": out[0], "du_max": out[1]}
