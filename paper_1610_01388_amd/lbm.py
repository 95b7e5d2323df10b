"""Python binding of liblbm.so (the C ABI of include/lbm.h).

The functions named ``lbm_*`` are one-to-one wrappers (argument marshalling
only; a non-zero status raises LbmError).  ``Domain`` is a convenience owner
that allocates the device buffers with torch on the current HIP device and
binds them with torch's current stream; every step of the update runs in the
library's kernels.  There is no CPU fallback: without the built library or
without a GPU the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LATTICES = {"D2Q9": 0, "D3Q19": 1, "D3Q27": 2}
OPERATORS = {"PR": 0, "IR": 1, "PRI": 2, "IRHB": 3}
PRECISIONS = {"FP64": 0, "FP32": 1, "FP16": 2}
SCHEMES = {"AB": 0, "AA": 1}
LAYOUTS = {"COMPACT": 0, "DENSE": 1}
PULL_FORMS = {"AUTO": 0, "SLOTS": 1, "ROWS": 2}
STATUS = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EHIP", -4: "LBM_ESTATE",
          -5: "LBM_EUNSTABLE", -6: "LBM_EFORMAT"}


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class lbm_desc(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("periodic", ctypes.c_int32 * 3),
                ("precision", ctypes.c_int32), ("scheme", ctypes.c_int32), ("layout", ctypes.c_int32)]


class lbm_rheology(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("fp64_fallback", ctypes.c_int32),
                ("nu_p", ctypes.c_double), ("sigma_y", ctypes.c_double), ("rho0", ctypes.c_double),
                ("m", ctypes.c_double), ("gamma_c", ctypes.c_double), ("lambda_trt", ctypes.c_double),
                ("g", ctypes.c_double * 3), ("fallback_band", ctypes.c_double),
                ("fp16_scale_log2", ctypes.c_int32), ("flow_axis", ctypes.c_int32),
                ("mrt_bulk", ctypes.c_double), ("mrt_even", ctypes.c_double), ("hb_n", ctypes.c_double)]


class lbm_monitor(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("flux", ctypes.c_double * 3), ("mass", ctypes.c_double),
                ("umax", ctypes.c_double), ("fluid_nodes", ctypes.c_int64),
                ("unyielded", ctypes.c_int64), ("fallback_nodes", ctypes.c_int64),
                ("nonfinite", ctypes.c_int64), ("residual", ctypes.c_double), ("du_max", ctypes.c_double)]

    def as_dict(self):
        return {"step": self.step, "flux": np.array(self.flux[:]), "mass": self.mass,
                "umax": self.umax, "fluid": self.fluid_nodes, "unyielded": self.unyielded,
                "fallback": self.fallback_nodes, "nonfinite": self.nonfinite,
                "residual": self.residual, "du_max": self.du_max}


class lbm_sizes(ctypes.Structure):
    _fields_ = [("pdf_bytes", ctypes.c_size_t), ("tau_bytes", ctypes.c_size_t),
                ("mask_bytes", ctypes.c_size_t), ("work_bytes", ctypes.c_size_t)]


EXPORTS = ["lbm_last_error", "lbm_lattice_info", "lbm_query_sizes", "lbm_create", "lbm_bind",
           "lbm_set_mask", "lbm_init_equilibrium", "lbm_write_populations", "lbm_read_populations",
           "lbm_step", "lbm_set_graph_steps", "lbm_time", "lbm_set_monitor_interval", "lbm_read_history", "lbm_monitors",
           "lbm_set_umax_limit", "lbm_monitors_async", "lbm_read_moments", "lbm_save", "lbm_load", "lbm_check_checkpoint", "lbm_set_tile",
           "lbm_get_tile", "lbm_set_tile_order", "lbm_get_tile_order", "lbm_set_pull_form", "lbm_get_pull_form",
           "lbm_autotune", "lbm_destroy",
           "lbm_batch_query_sizes", "lbm_batch_create", "lbm_batch_bind", "lbm_batch_init_equilibrium",
           "lbm_batch_write_populations", "lbm_batch_read_populations", "lbm_batch_read_moments",
           "lbm_batch_set_monitor_interval", "lbm_batch_read_history", "lbm_batch_monitors",
           "lbm_batch_set_graph_steps", "lbm_batch_step", "lbm_batch_time", "lbm_batch_get_tiles",
           "lbm_batch_get_schedule", "lbm_batch_set_schedule",
           "lbm_batch_autotune", "lbm_batch_destroy"]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load liblbm.so and declare argument types.  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() "
                          "(or python paper_1610_01388_amd/build.py)")
    # torch carries its own HIP runtime with the same soname as the system
    # one liblbm.so links against.  Loading torch first makes the dynamic
    # loader hand that runtime to liblbm.so, so one HIP runtime serves both
    # (two runtimes in one process do not share the device).
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    vp, dp, i32, i64 = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int32, ctypes.c_int64
    i32p = ctypes.POINTER(ctypes.c_int32)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    sig = {
        "lbm_last_error": ([], ctypes.c_char_p),
        "lbm_lattice_info": ([i32, i32p, i32p, dp, i32p], ctypes.c_int),
        "lbm_query_sizes": ([ctypes.POINTER(lbm_desc), ctypes.POINTER(lbm_rheology),
                             ctypes.POINTER(lbm_sizes)], ctypes.c_int),
        "lbm_create": ([ctypes.POINTER(lbm_desc), ctypes.POINTER(lbm_rheology),
                        ctypes.POINTER(vp)], ctypes.c_int),
        "lbm_bind": ([vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "lbm_set_mask": ([vp, u8p], ctypes.c_int),
        "lbm_init_equilibrium": ([vp, ctypes.c_double, dp], ctypes.c_int),
        "lbm_write_populations": ([vp, dp, dp], ctypes.c_int),
        "lbm_read_populations": ([vp, dp, dp], ctypes.c_int),
        "lbm_step": ([vp, i64], ctypes.c_int),
        "lbm_set_graph_steps": ([vp, i32], ctypes.c_int),
        "lbm_time": ([vp, ctypes.POINTER(i64)], ctypes.c_int),
        "lbm_set_monitor_interval": ([vp, i32], ctypes.c_int),
        "lbm_read_history": ([vp, ctypes.POINTER(lbm_monitor), i32, i32p], ctypes.c_int),
        "lbm_monitors": ([vp, ctypes.POINTER(lbm_monitor)], ctypes.c_int),
        "lbm_set_umax_limit": ([vp, ctypes.c_double], ctypes.c_int),
        "lbm_monitors_async": ([vp, vp], ctypes.c_int),
        "lbm_read_moments": ([vp, dp, dp, dp, u8p], ctypes.c_int),
        "lbm_save": ([vp, vp, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "lbm_load": ([vp, vp, ctypes.c_size_t], ctypes.c_int),
        "lbm_check_checkpoint": ([ctypes.POINTER(lbm_desc), ctypes.POINTER(lbm_rheology), vp, ctypes.c_size_t],
                                 ctypes.c_int),
        "lbm_set_tile": ([vp, i32, i32, i32], ctypes.c_int),
        "lbm_get_tile": ([vp, i32p, i32p, i32p], ctypes.c_int),
        "lbm_set_tile_order": ([vp, i32, i32], ctypes.c_int),
        "lbm_get_tile_order": ([vp, i32p, i32p], ctypes.c_int),
        "lbm_set_pull_form": ([vp, i32], ctypes.c_int),
        "lbm_get_pull_form": ([vp, i32p], ctypes.c_int),
        "lbm_autotune": ([vp, i32], ctypes.c_int),
        "lbm_destroy": ([vp], ctypes.c_int),
        "lbm_batch_query_sizes": ([ctypes.POINTER(lbm_desc), ctypes.POINTER(lbm_rheology), i32,
                                   ctypes.POINTER(lbm_sizes)], ctypes.c_int),
        "lbm_batch_create": ([ctypes.POINTER(lbm_desc), ctypes.POINTER(lbm_rheology), i32,
                              ctypes.POINTER(vp)], ctypes.c_int),
        "lbm_batch_bind": ([vp, vp, vp, vp, vp], ctypes.c_int),
        "lbm_batch_init_equilibrium": ([vp], ctypes.c_int),
        "lbm_batch_write_populations": ([vp, i32, dp, dp], ctypes.c_int),
        "lbm_batch_read_populations": ([vp, i32, dp, dp], ctypes.c_int),
        "lbm_batch_read_moments": ([vp, i32, dp, dp, dp, u8p], ctypes.c_int),
        "lbm_batch_set_monitor_interval": ([vp, i32], ctypes.c_int),
        "lbm_batch_read_history": ([vp, ctypes.POINTER(lbm_monitor), i32, i32p], ctypes.c_int),
        "lbm_batch_monitors": ([vp, ctypes.POINTER(lbm_monitor)], ctypes.c_int),
        "lbm_batch_set_graph_steps": ([vp, i32], ctypes.c_int),
        "lbm_batch_step": ([vp, i64], ctypes.c_int),
        "lbm_batch_time": ([vp, ctypes.POINTER(i64)], ctypes.c_int),
        "lbm_batch_get_tiles": ([vp, i32p], ctypes.c_int),
        "lbm_batch_get_schedule": ([vp, i32p, i32p], ctypes.c_int),
        "lbm_batch_set_schedule": ([vp, i32, i32], ctypes.c_int),
        "lbm_batch_autotune": ([vp, i32], ctypes.c_int),
        "lbm_batch_destroy": ([vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _check(rc):
    if rc != 0:
        raise LbmError(rc, load_library().lbm_last_error().decode())
    return rc


def _dp(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# --- one-to-one wrappers ----------------------------------------------------

def lbm_lattice_info(lattice):
    q = ctypes.c_int32()
    c = np.zeros(81, dtype=np.int32)
    w = np.zeros(27)
    opp = np.zeros(27, dtype=np.int32)
    _check(load_library().lbm_lattice_info(lattice, ctypes.byref(q),
                                           c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(w),
                                           opp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    n = q.value
    return c[:3 * n].reshape(n, 3).copy(), w[:n].copy(), opp[:n].copy()


def lbm_query_sizes(desc, rh=None):
    s = lbm_sizes()
    _check(load_library().lbm_query_sizes(ctypes.byref(desc), ctypes.byref(rh) if rh is not None else None,
                                          ctypes.byref(s)))
    return s


def lbm_create(desc, rh):
    h = ctypes.c_void_p()
    _check(load_library().lbm_create(ctypes.byref(desc), ctypes.byref(rh), ctypes.byref(h)))
    return h


def lbm_bind(h, pdf, tau, mask, work, stream):
    _check(load_library().lbm_bind(h, pdf, tau, mask, work, stream))


def lbm_set_mask(h, mask):
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    _check(load_library().lbm_set_mask(h, m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))


def lbm_init_equilibrium(h, rho0=1.0, u0=(0.0, 0.0, 0.0)):
    u = np.ascontiguousarray(np.resize(np.asarray(u0, dtype=np.float64), 3))
    _check(load_library().lbm_init_equilibrium(h, rho0, _dp(u)))


def lbm_write_populations(h, P, tau=None):
    P = np.ascontiguousarray(P, dtype=np.float64)
    t = None if tau is None else np.ascontiguousarray(tau, dtype=np.float64)
    _check(load_library().lbm_write_populations(h, _dp(P), _dp(t)))


def lbm_read_populations(h, q, N, with_tau=False):
    P = np.zeros((q, N))
    t = np.zeros(N) if with_tau else None
    _check(load_library().lbm_read_populations(h, _dp(P), _dp(t)))
    return P, t


def lbm_step(h, n):
    _check(load_library().lbm_step(h, int(n)))


def lbm_set_graph_steps(h, steps):
    _check(load_library().lbm_set_graph_steps(h, int(steps)))


def lbm_time(h):
    t = ctypes.c_int64()
    _check(load_library().lbm_time(h, ctypes.byref(t)))
    return t.value


def lbm_set_monitor_interval(h, k):
    _check(load_library().lbm_set_monitor_interval(h, int(k)))


def lbm_read_history(h, max_records=4096):
    buf = (lbm_monitor * max_records)()
    n = ctypes.c_int32()
    _check(load_library().lbm_read_history(h, buf, max_records, ctypes.byref(n)))
    return [buf[k].as_dict() for k in range(n.value)]


def lbm_monitors(h, raise_unstable=True):
    m = lbm_monitor()
    rc = load_library().lbm_monitors(h, ctypes.byref(m))
    if rc != 0 and (raise_unstable or rc != -5):
        _check(rc)
    d = m.as_dict()
    d["status"] = rc
    return d


def lbm_monitors_async(h, record_dev_ptr: int):
    """Enqueue the allocation-free monitors into device memory at
    record_dev_ptr (one lbm_monitor, 96 bytes); no synchronisation."""
    _check(load_library().lbm_monitors_async(h, ctypes.c_void_p(int(record_dev_ptr))))


def lbm_set_umax_limit(h, umax):
    _check(load_library().lbm_set_umax_limit(h, float(umax)))


def lbm_read_moments(h, N):
    rho = np.zeros(N)
    u = np.zeros((3, N))
    nu = np.zeros(N)
    uy = np.zeros(N, dtype=np.uint8)
    _check(load_library().lbm_read_moments(h, _dp(rho), _dp(u), _dp(nu),
                                           uy.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
    return rho, u, nu, uy


def lbm_save(h):
    n = ctypes.c_size_t(0)
    _check(load_library().lbm_save(h, None, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value)
    _check(load_library().lbm_save(h, buf, ctypes.byref(n)))
    return buf.raw[: n.value]


def lbm_load(h, blob: bytes):
    buf = ctypes.create_string_buffer(blob, len(blob))
    _check(load_library().lbm_load(h, buf, len(blob)))


def lbm_check_checkpoint(desc, rh, blob: bytes):
    """Validate a checkpoint blob for a domain of this descriptor and
    rheology on the host (no device); raises LbmError when it is rejected."""
    buf = ctypes.create_string_buffer(blob, len(blob))
    _check(load_library().lbm_check_checkpoint(ctypes.byref(desc), ctypes.byref(rh), buf, len(blob)))


def lbm_set_tile(h, tx, ty, tz):
    _check(load_library().lbm_set_tile(h, tx, ty, tz))


def lbm_get_tile(h):
    v = [ctypes.c_int32() for _ in range(3)]
    _check(load_library().lbm_get_tile(h, *[ctypes.byref(x) for x in v]))
    return tuple(x.value for x in v)


def lbm_set_tile_order(h, brick_rows, brick_planes):
    _check(load_library().lbm_set_tile_order(h, int(brick_rows), int(brick_planes)))


def lbm_get_tile_order(h):
    r, p = ctypes.c_int32(), ctypes.c_int32()
    _check(load_library().lbm_get_tile_order(h, ctypes.byref(r), ctypes.byref(p)))
    return r.value, p.value


def lbm_set_pull_form(h, form):
    _check(load_library().lbm_set_pull_form(h, PULL_FORMS[form] if isinstance(form, str) else int(form)))


def lbm_get_pull_form(h):
    f = ctypes.c_int32()
    _check(load_library().lbm_get_pull_form(h, ctypes.byref(f)))
    return {v: k for k, v in PULL_FORMS.items()}.get(f.value, f.value)


def lbm_autotune(h, trial_steps=10):
    _check(load_library().lbm_autotune(h, int(trial_steps)))


def lbm_destroy(h):
    _check(load_library().lbm_destroy(h))


# --- convenience owner ----------------------------------------------------------

def make_desc(lattice, dims, periodic, precision="FP64", scheme="AA", layout="COMPACT"):
    d = lbm_desc()
    d.lattice = LATTICES[lattice] if isinstance(lattice, str) else int(lattice)
    d.nx, d.ny, d.nz = (int(v) for v in dims)
    for a in range(3):
        d.periodic[a] = int(periodic[a])
    d.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    d.scheme = SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
    d.layout = LAYOUTS[layout] if isinstance(layout, str) else int(layout)
    return d


def make_rheology(op, nu_p, sigma_y=0.0, m=0.0, g=(0.0, 0.0, 0.0), rho0=1.0, gamma_c=1e-8,
                  lambda_trt=0.25, fp64_fallback=False, fallback_band=0.0, fp16_scale_log2=14, flow_axis=0,
                  mrt_bulk=0.0, mrt_even=0.0, hb_n=1.0):
    r = lbm_rheology()
    r.hb_n = float(hb_n)
    r.op = OPERATORS[op] if isinstance(op, str) else int(op)
    r.fp64_fallback = int(bool(fp64_fallback))
    r.nu_p, r.sigma_y, r.rho0 = float(nu_p), float(sigma_y), float(rho0)
    r.m, r.gamma_c, r.lambda_trt = float(m), float(gamma_c), float(lambda_trt)
    for a in range(3):
        r.g[a] = float(g[a]) if a < len(g) else 0.0
    r.fallback_band = float(fallback_band)
    r.fp16_scale_log2 = int(fp16_scale_log2)
    r.flow_axis = int(flow_axis)
    r.mrt_bulk = float(mrt_bulk)
    r.mrt_even = float(mrt_even)
    return r


class Domain:
    """Owns one lbm_domain and its torch-allocated device buffers."""

    def __init__(self, lattice, dims, periodic, op, nu_p, sigma_y=0.0, m=0.0, g=(0, 0, 0),
                 precision="FP64", scheme="AA", layout="COMPACT", mask=None, device=None, stream=None,
                 **rh_kw):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("liblbm needs a HIP GPU; none is visible")
        load_library()
        self.torch = torch
        self.desc = make_desc(lattice, dims, periodic, precision, scheme, layout)
        self.rh = make_rheology(op, nu_p, sigma_y, m, g, **rh_kw)
        self.dims = tuple(int(v) for v in dims)
        self.N = self.dims[0] * self.dims[1] * self.dims[2]
        self.c, self.w, self.opp = lbm_lattice_info(self.desc.lattice)
        self.q = len(self.w)
        sz = lbm_query_sizes(self.desc, self.rh)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        alloc = lambda n: torch.empty(max(int(n), 256), dtype=torch.uint8, device=self.device)
        self.pdf = alloc(sz.pdf_bytes)
        self.tau = alloc(sz.tau_bytes) if sz.tau_bytes else None
        self.mask_buf = alloc(sz.mask_bytes)
        self.work = alloc(sz.work_bytes)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.h = lbm_create(self.desc, self.rh)
        lbm_bind(self.h, self.pdf.data_ptr(), self.tau.data_ptr() if self.tau is not None else None,
                 self.mask_buf.data_ptr(), self.work.data_ptr(), self.stream.cuda_stream)
        if mask is not None:
            self.set_mask(mask)

    def close(self):
        if getattr(self, "h", None):
            lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_mask(self, mask):
        lbm_set_mask(self.h, np.asarray(mask, dtype=np.uint8).reshape(-1))

    def init(self, rho0=1.0, u0=(0.0, 0.0, 0.0)):
        lbm_init_equilibrium(self.h, rho0, u0)

    def step(self, n=1):
        lbm_step(self.h, n)

    def set_graph_steps(self, n):
        lbm_set_graph_steps(self.h, n)

    @property
    def time(self):
        return lbm_time(self.h)

    def moments(self):
        return lbm_read_moments(self.h, self.N)

    def monitors(self, raise_unstable=False):
        return lbm_monitors(self.h, raise_unstable)

    def set_monitor_interval(self, k):
        lbm_set_monitor_interval(self.h, k)

    def history(self):
        return lbm_read_history(self.h)

    def write_populations(self, P, tau=None):
        lbm_write_populations(self.h, P, tau)

    def read_populations(self, with_tau=False):
        return lbm_read_populations(self.h, self.q, self.N, with_tau)

    def save(self):
        return lbm_save(self.h)

    def load(self, blob):
        lbm_load(self.h, blob)

    def set_tile(self, tx, ty, tz):
        lbm_set_tile(self.h, tx, ty, tz)

    def tile(self):
        return lbm_get_tile(self.h)

    def set_tile_order(self, brick_rows=0, brick_planes=0):
        lbm_set_tile_order(self.h, brick_rows, brick_planes)

    def tile_order(self):
        return lbm_get_tile_order(self.h)

    def set_pull_form(self, form):
        lbm_set_pull_form(self.h, form)

    def pull_form(self):
        return lbm_get_pull_form(self.h)

    def autotune(self, trial_steps=10):
        lbm_autotune(self.h, trial_steps)

    def synchronize(self):
        self.stream.synchronize()


# --- batched sweep ------------------------------------------------------------

def _arrays(descs, rhs):
    n = len(descs)
    D = (lbm_desc * n)(*descs)
    R = (lbm_rheology * n)(*rhs)
    return D, R


def lbm_batch_query_sizes(descs, rhs):
    D, R = _arrays(descs, rhs)
    s = lbm_sizes()
    _check(load_library().lbm_batch_query_sizes(D, R, len(descs), ctypes.byref(s)))
    return s


def lbm_batch_create(descs, rhs):
    D, R = _arrays(descs, rhs)
    h = ctypes.c_void_p()
    _check(load_library().lbm_batch_create(D, R, len(descs), ctypes.byref(h)))
    return h


def lbm_batch_bind(h, pdf, tau, work, stream):
    _check(load_library().lbm_batch_bind(h, pdf, tau, work, stream))


def lbm_batch_init_equilibrium(h):
    _check(load_library().lbm_batch_init_equilibrium(h))


def lbm_batch_write_populations(h, sim, P, tau=None):
    P = np.ascontiguousarray(P, dtype=np.float64)
    t = None if tau is None else np.ascontiguousarray(tau, dtype=np.float64)
    _check(load_library().lbm_batch_write_populations(h, int(sim), _dp(P), _dp(t)))


def lbm_batch_read_populations(h, sim, q, N, with_tau=False):
    P = np.zeros((q, N))
    t = np.zeros(N) if with_tau else None
    _check(load_library().lbm_batch_read_populations(h, int(sim), _dp(P), _dp(t)))
    return P, t


def lbm_batch_read_moments(h, sim, N):
    rho, u, nu = np.zeros(N), np.zeros((3, N)), np.zeros(N)
    uy = np.zeros(N, dtype=np.uint8)
    _check(load_library().lbm_batch_read_moments(h, int(sim), _dp(rho), _dp(u), _dp(nu),
                                                 uy.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
    return rho, u, nu, uy


def lbm_batch_set_monitor_interval(h, k):
    _check(load_library().lbm_batch_set_monitor_interval(h, int(k)))


def lbm_batch_read_history(h, count, max_records=256):
    buf = (lbm_monitor * (max_records * count))()
    n = ctypes.c_int32()
    _check(load_library().lbm_batch_read_history(h, buf, max_records, ctypes.byref(n)))
    return [[buf[r * count + k].as_dict() for k in range(count)] for r in range(n.value)]


def lbm_batch_monitors(h, count):
    buf = (lbm_monitor * count)()
    _check(load_library().lbm_batch_monitors(h, buf))
    return [buf[k].as_dict() for k in range(count)]


def lbm_batch_set_graph_steps(h, steps):
    _check(load_library().lbm_batch_set_graph_steps(h, int(steps)))


def lbm_batch_step(h, n):
    _check(load_library().lbm_batch_step(h, int(n)))


def lbm_batch_time(h):
    t = ctypes.c_int64()
    _check(load_library().lbm_batch_time(h, ctypes.byref(t)))
    return t.value


def lbm_batch_get_tiles(h, count):
    t = np.zeros(3 * count, dtype=np.int32)
    _check(load_library().lbm_batch_get_tiles(h, t.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return t.reshape(count, 3)


def lbm_batch_get_schedule(h):
    p, x = ctypes.c_int32(), ctypes.c_int32()
    _check(load_library().lbm_batch_get_schedule(h, ctypes.byref(p), ctypes.byref(x)))
    return p.value, x.value


def lbm_batch_set_schedule(h, tile_policy, xcd_order):
    _check(load_library().lbm_batch_set_schedule(h, int(tile_policy), int(xcd_order)))


def lbm_batch_autotune(h, trial_steps=10):
    _check(load_library().lbm_batch_autotune(h, int(trial_steps)))


def lbm_batch_destroy(h):
    _check(load_library().lbm_batch_destroy(h))


class Batch:
    """Owns one lbm_batch and its torch-allocated device buffers.  cases:
    dicts with lattice, dims, periodic, op, nu_p, sigma_y, m, g (the
    inputs.batch_sweep recipe)."""

    def __init__(self, cases, precision="FP32", device=None, stream=None, **rh_kw):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("liblbm needs a HIP GPU; none is visible")
        load_library()
        self.torch = torch
        self.cases = cases
        self.descs = [make_desc(c["lattice"], c["dims"], c["periodic"], precision, "AA") for c in cases]
        self.rhs = [make_rheology(c["op"], c["nu_p"], c["sigma_y"], c.get("m", 0.0), c["g"], **rh_kw)
                    for c in cases]
        self.count = len(cases)
        self.N = [int(np.prod(c["dims"])) for c in cases]
        self.c, self.w, self.opp = lbm_lattice_info(self.descs[0].lattice)
        self.q = len(self.w)
        sz = lbm_batch_query_sizes(self.descs, self.rhs)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        alloc = lambda n: torch.empty(max(int(n), 256), dtype=torch.uint8, device=self.device)
        self.pdf = alloc(sz.pdf_bytes)
        self.tau = alloc(sz.tau_bytes) if sz.tau_bytes else None
        self.work = alloc(sz.work_bytes)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.h = lbm_batch_create(self.descs, self.rhs)
        lbm_batch_bind(self.h, self.pdf.data_ptr(), self.tau.data_ptr() if self.tau is not None else None,
                       self.work.data_ptr(), self.stream.cuda_stream)

    def close(self):
        if getattr(self, "h", None):
            lbm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        lbm_batch_step(self.h, n)

    @property
    def time(self):
        return lbm_batch_time(self.h)

    def moments(self, sim):
        return lbm_batch_read_moments(self.h, sim, self.N[sim])

    def write_populations(self, sim, P, tau=None):
        lbm_batch_write_populations(self.h, sim, P, tau)

    def read_populations(self, sim, with_tau=False):
        return lbm_batch_read_populations(self.h, sim, self.q, self.N[sim], with_tau)

    def monitors(self):
        return lbm_batch_monitors(self.h, self.count)

    def set_monitor_interval(self, k):
        lbm_batch_set_monitor_interval(self.h, k)

    def history(self):
        return lbm_batch_read_history(self.h, self.count)

    def set_graph_steps(self, n):
        lbm_batch_set_graph_steps(self.h, n)

    def tiles(self):
        return lbm_batch_get_tiles(self.h, self.count)

    def autotune(self, trial_steps=10):
        lbm_batch_autotune(self.h, trial_steps)

    def schedule(self):
        """(tile policy, work-item order) in use."""
        return lbm_batch_get_schedule(self.h)

    def set_schedule(self, tile_policy, xcd_order):
        lbm_batch_set_schedule(self.h, tile_policy, xcd_order)
