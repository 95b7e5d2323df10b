"""Brute force on tiny grids: the oracle's full update against the second,
literal implementation in ``bruteforce_lbm.py`` (explicit loops, its own
velocity tables and root finders), for the PR, IR, PRI and IRHB operators.

The grids mix periodic axes and walls, hold wall corners (walls on two or
three axes) and one interior solid node, so halfway bounce-back at walls
and at obstacles (Sec. 2, Eq. 10; Sec. 4.3), periodic wrapping and the
superficial flux over all nodes (the mean over the whole cell, solids
counted as zero: Sec. 4.5) are all exercised.  Both sides start from the
same seeded post-collision state and run 50 steps.
"""
import numpy as np
import pytest

import bruteforce_lbm as bf
from paper_1610_01388_amd import inputs

STEPS = 50
# (lattice, dims, periodic, solid nodes, flow axis)
GRIDS = [
    (0, (2, 2, 1), (1, 1, 1), (), 0),
    (0, (3, 3, 1), (1, 0, 1), (4,), 0),      # walls across y, solid centre node
    (0, (1, 3, 1), (1, 0, 1), (), 1),        # one node wide, flow-axis correction on x
    (0, (3, 3, 1), (0, 0, 1), (), 0),        # walls on both axes: wall corners
    (1, (3, 3, 3), (1, 1, 1), (13,), 0),     # periodic box, solid centre node
    (2, (3, 3, 3), (1, 1, 1), (13,), 0),
    (2, (3, 3, 3), (0, 0, 0), (), 0),        # closed box: walls and corners on every axis
    (2, (2, 3, 4), (1, 0, 1), (9,), 3),      # walls across y, one solid, flow-axis correction on z
    (1, (2, 3, 4), (0, 1, 0), (7,), 0),
]
OPS = ["PR", "IR", "PRI", "IRHB"]


def params(op, lat, axis):
    g = (5e-5, -2e-5, 1e-5 if lat != 0 else 0.0)
    return {"op": op, "nu_p": 0.1, "sigma_y": 1.5e-5, "m": 1e3, "gamma_c": 1e-8, "lambda": 0.25, "g": g,
            "axis": axis, "hb_n": 0.6 if op == "IRHB" else 1.0}


def run_both(orc, lat, dims, per, solids, axis, op, seed):
    N = int(np.prod(dims))
    mask = np.zeros(N, dtype=np.uint8)
    for k in solids:
        mask[k] = 1
    p = params(op, lat, axis)
    oop = {"PR": orc.PR, "IR": orc.IR, "PRI": orc.PRI, "IRHB": orc.IRHB}[op]
    rh = orc.rheology(oop, p["nu_p"], p["sigma_y"], p["m"], p["gamma_c"], p["lambda"], p["g"], flow_axis=axis,
                      hb_n=p["hb_n"])
    od = orc.Domain(lat, dims, per, rh, mask)
    _, c_orc, w_orc, _ = orc.lattice_info(lat)
    cs, ws, _ = bf.velocities(lat)
    perm = [int(np.flatnonzero((c_orc == np.array(c)).all(1))[0]) for c in cs]  # brute k -> oracle index
    assert np.allclose(w_orc[perm], ws, rtol=0, atol=1e-17)
    q = len(cs)
    # seeded post-collision state w_i (1 + 0.02 r), solids empty; PR tau
    r = inputs.uniform_array(seed, q * N, -1.0, 1.0).reshape(q, N)
    P_orc = w_orc[:, None] * (1.0 + 0.02 * r) * (1 - mask)[None, :]
    tau = 0.5 + 3.0 * p["nu_p"] * (1.0 + inputs.uniform_array(seed + 1, N))
    od.set_state(P_orc, tau)
    g = bf.Grid(lat, dims, per, p, mask)
    g.P = [list(P_orc[perm[k]]) for k in range(q)]
    g.tau = list(tau)
    od.step(STEPS)
    g.step(STEPS)
    return od, g, perm, mask


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("case", range(len(GRIDS)))
def test_oracle_equals_brute_force(orc, case, op):
    lat, dims, per, solids, axis = GRIDS[case]
    od, g, perm, mask = run_both(orc, lat, dims, per, solids, axis, op, seed=100 + case)
    P, tau = od.get_state()
    Pb = np.array(g.P)
    assert np.max(np.abs(P[perm] - Pb)) <= 1e-14
    if op == "PR":
        assert np.max(np.abs(tau - np.array(g.tau)) / tau) <= 1e-13
    rho, u, _, uy = od.moments()
    rb, ub, uyb = g.moments()
    assert np.max(np.abs(rho - np.array(rb))) <= 1e-14
    assert np.max(np.abs(u - np.array(ub))) <= 1e-15
    assert np.array_equal(uy, np.array(uyb, dtype=np.uint8))
    mo = od.monitors()
    mb = g.monitors()
    assert np.max(np.abs(mo["flux"] - np.array(mb["flux"]))) <= 1e-15
    assert abs(mo["mass"] - mb["mass"]) <= 1e-13
    assert abs(mo["umax"] - mb["umax"]) <= 1e-15
    assert mo["unyielded"] == mb["unyielded"] and mo["fluid"] == mb["fluid"] == int((mask == 0).sum())


def test_brute_force_cases_exercise_both_regimes(orc):
    """The seeded states put yielded and unyielded nodes in the runs (so the
    comparison covers both branches of the IR solve and the PR plug)."""
    seen = {"IR": set(), "PR": set()}
    for case, (lat, dims, per, solids, axis) in enumerate(GRIDS):
        for op in ("IR", "PR"):
            od, _, _, mask = run_both(orc, lat, dims, per, solids, axis, op, seed=100 + case)
            _, _, _, uy = od.moments()
            fl = mask == 0
            seen[op].update(set(uy[fl].tolist()))
    assert seen["IR"] == {0, 1} and seen["PR"] == {0, 1}
