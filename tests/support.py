"""Shared helpers of the GPU parity tests: seeded initial states, the map
between the oracle's velocity order and the library's, and paired runs of
the oracle and the library on the same inputs."""
import numpy as np

import oracle
from paper_1610_01388_amd import inputs

LAT_NAMES = {0: "D2Q9", 1: "D3Q19", 2: "D3Q27"}
OP_IDS = {"PR": oracle.PR, "IR": oracle.IR, "PRI": oracle.PRI, "IRHB": oracle.IRHB}


def perm_lib_from_oracle(lat):
    """perm[k] = oracle index of the library's velocity k (same c vector)."""
    from paper_1610_01388_amd import lbm
    c_lib, w_lib, _ = lbm.lbm_lattice_info(lat)
    _, c_orc, w_orc, _ = oracle.lattice_info(lat)
    perm = np.array([int(np.flatnonzero((c_orc == v).all(1))[0]) for v in c_lib])
    assert np.array_equal(c_orc[perm], c_lib) and np.array_equal(w_orc[perm], w_lib)
    return perm


def random_state(lat, N, seed, amp=1e-2, nu_p=0.1, op="IR"):
    """Post-collision populations w_i (1 + amp r) with r uniform in [-1, 1)
    (oracle order), and a PR relaxation-time field 1/2 + 3 nu_p (1 + s),
    s uniform in [0, 1)."""
    _, _, w, _ = oracle.lattice_info(lat)
    q = len(w)
    r = inputs.uniform_array(seed, q * N, -1.0, 1.0).reshape(q, N)
    P = w[:, None] * (1.0 + amp * r)
    tau = 0.5 + 3.0 * nu_p * (1.0 + inputs.uniform_array(seed + 1, N))
    return P, tau


def random_mask(N, seed, fraction):
    return (inputs.uniform_array(seed, N) < fraction).astype(np.uint8)


def run_pair(lat, dims, periodic, op, steps, *, nu_p=0.1, sigma_y=5e-4, m=1e4, g=(2e-5, -1e-5, 5e-6),
             lam=0.25, scheme="AA", precision="FP64", mask=None, seed=1, amp=1e-2, tile=None,
             gpu_kw=None, flow_axis=0, mrt_bulk=0.0, mrt_even=0.0, pull_form=None, hb_n=1.0, hist=None):
    """Run the oracle and the library from the same seeded state; return both
    moment sets (and the populations read back).  With a list hist, the
    library's fused monitor records of every step are appended to it."""
    from paper_1610_01388_amd import lbm
    N = int(np.prod(dims))
    g = tuple(g[a] if (a < 2 or lat != 0) else 0.0 for a in range(3))
    P0, tau0 = random_state(lat, N, seed, amp, nu_p, op)
    if mask is not None:
        P0 = P0 * (1 - mask)[None, :]
    rh = oracle.rheology(OP_IDS[op], nu_p, sigma_y, m, 1e-8, lam, g, flow_axis=flow_axis, mrt_bulk=mrt_bulk,
                         mrt_even=mrt_even, hb_n=hb_n)
    od = oracle.Domain(lat, dims, periodic, rh, mask)
    od.set_state(P0, tau0)
    od.step(steps)
    ref = od.moments()
    Pref, tauref = od.get_state()

    perm = perm_lib_from_oracle(lat)
    dom = lbm.Domain(LAT_NAMES[lat], dims, periodic, op, nu_p, sigma_y, m=m, g=g, lambda_trt=lam,
                     precision=precision, scheme=scheme, flow_axis=flow_axis, mrt_bulk=mrt_bulk, mrt_even=mrt_even,
                     hb_n=hb_n,
                     **(gpu_kw or {}))
    if mask is not None:
        dom.set_mask(mask)
    if tile is not None:
        dom.set_tile(*tile)
    if pull_form is not None:
        dom.set_pull_form(pull_form)
        assert dom.pull_form() == pull_form
    dom.write_populations(P0[perm], tau0 if op == "PR" else None)
    if hist is not None:
        dom.set_monitor_interval(1)
    dom.step(steps)
    if hist is not None:
        hist.extend(dom.history())
    got = dom.moments()
    Pg, taug = dom.read_populations(with_tau=(op == "PR"))
    dom.close()
    inv = np.argsort(perm)
    return ref, got, (Pref, tauref), (Pg[inv], taug)


def l2rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
