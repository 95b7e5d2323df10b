"""GPU tests of the batched sweep: every simulation of a batch advances
exactly as the same simulation run alone (bitwise) and as the oracle (FP64
bar); captured-graph replays, interleaved with eager work, match eager
stepping replay by replay; fused monitors survive replays; the tile
autotuner keeps the state."""
import numpy as np
import pytest

import oracle
from paper_1610_01388_amd import inputs
from support import l2rel, perm_lib_from_oracle, random_state

pytestmark = pytest.mark.gpu

CASES = [
    dict(lattice="D3Q19", dims=(33, 37, 4), periodic=(0, 0, 1), op="IR", nu_p=0.1, sigma_y=2e-4, m=0.0,
         g=(0.0, 0.0, 3e-5)),
    dict(lattice="D3Q19", dims=(70, 5, 3), periodic=(1, 0, 1), op="PR", nu_p=0.05, sigma_y=1e-4, m=1e4,
         g=(2e-5, 0.0, 0.0)),
    dict(lattice="D3Q19", dims=(9, 9, 9), periodic=(1, 1, 1), op="IR", nu_p=0.2, sigma_y=0.0, m=0.0,
         g=(1e-5, 1e-5, 0.0)),
    dict(lattice="D3Q19", dims=(128, 3, 2), periodic=(0, 1, 1), op="PR", nu_p=0.1, sigma_y=3e-4, m=1e3,
         g=(0.0, 2e-5, 0.0)),
    dict(lattice="D3Q19", dims=(40, 40, 4), periodic=(0, 0, 1), op="PR", nu_p=0.1, sigma_y=5e-5, m=1e5,
         g=(0.0, 0.0, 1e-5)),
]


def _states(cases, seed):
    perm = perm_lib_from_oracle(1)
    out = []
    for k, c in enumerate(cases):
        N = int(np.prod(c["dims"]))
        P, tau = random_state(1, N, seed + k, amp=1e-2, nu_p=c["nu_p"])
        out.append((P, tau, perm))
    return out


def _make_batch(cases, states, precision="FP64", graph_steps=10):
    from paper_1610_01388_amd import lbm
    b = lbm.Batch(cases, precision=precision)
    b.set_graph_steps(graph_steps)
    for k, (P, tau, perm) in enumerate(states):
        b.write_populations(k, P[perm], tau if cases[k]["op"] == "PR" else None)
    return b


def test_batch_equals_single_domains_and_oracle():
    from paper_1610_01388_amd import lbm
    states = _states(CASES, 40)
    b = _make_batch(CASES, states, graph_steps=10)
    b.step(37)  # replays of 10 steps plus eager steps
    for k, c in enumerate(CASES):
        P, tau, perm = states[k]
        d = lbm.Domain(c["lattice"], c["dims"], c["periodic"], c["op"], c["nu_p"], c["sigma_y"], m=c["m"], g=c["g"],
                       layout="DENSE")
        d.write_populations(P[perm], tau if c["op"] == "PR" else None)
        d.step(37)
        Pd, td = d.read_populations(with_tau=c["op"] == "PR")
        Pb, tb = b.read_populations(k, with_tau=c["op"] == "PR")
        assert np.array_equal(Pb, Pd), f"simulation {k} differs from its single-domain run"
        if c["op"] == "PR":
            assert np.array_equal(tb, td)
        rh = oracle.rheology(oracle.PR if c["op"] == "PR" else oracle.IR, c["nu_p"], c["sigma_y"], c["m"], 1e-8,
                             0.25, c["g"])
        od = oracle.Domain(1, c["dims"], c["periodic"], rh)
        od.set_state(P, tau)
        od.step(37)
        rho_o, u_o, _, uy_o = od.moments()
        rho_b, u_b, _, uy_b = b.moments(k)
        assert l2rel(u_b, u_o) <= 1e-10
        assert np.max(np.abs(rho_b - rho_o)) <= 1e-12
        assert np.array_equal(uy_b, uy_o)
    b.close()


def test_graph_replays_match_eager_steps():
    """Replays of the captured graph, with eager steps, host reads and
    synchronisations in between, give the eager result after every replay."""
    states = _states(CASES, 60)
    g = _make_batch(CASES, states, graph_steps=8)
    e = _make_batch(CASES, states, graph_steps=0)
    for rep in range(4):
        g.step(8)
        e.step(8)
        g.torch.cuda.synchronize()
        for k in range(len(CASES)):
            assert np.array_equal(g.read_populations(k)[0], e.read_populations(k)[0]), f"replay {rep}, sim {k}"
        g.step(3)  # eager steps between replays (odd: the next replay waits for alignment)
        e.step(3)
    g.step(13)
    e.step(13)
    for k in range(len(CASES)):
        assert np.array_equal(g.read_populations(k)[0], e.read_populations(k)[0])
    assert g.time == e.time == 4 * 11 + 13


def test_batch_monitors_through_replays():
    states = _states(CASES, 80)
    b = _make_batch(CASES, states, graph_steps=20)
    b.set_monitor_interval(10)
    e = _make_batch(CASES, states, graph_steps=0)
    e.set_monitor_interval(10)
    b.step(60)
    e.step(60)
    hb, he = b.history(), e.history()
    assert [r[0]["step"] for r in hb] == [0, 10, 20, 30, 40, 50] == [r[0]["step"] for r in he]
    for rb, re in zip(hb, he):
        for mb, me in zip(rb, re):
            assert np.array_equal(mb["flux"], me["flux"]) and mb["mass"] == me["mass"]
            assert mb["unyielded"] == me["unyielded"] and mb["fluid"] == me["fluid"]
            assert mb["residual"] == me["residual"] and mb["du_max"] == me["du_max"]
    # residuals against the single-domain kernels' fused monitors (same records)
    from paper_1610_01388_amd import lbm
    for k in (0, 3):
        c = CASES[k]
        P, tau, perm = states[k]
        d = lbm.Domain(c["lattice"], c["dims"], c["periodic"], c["op"], c["nu_p"], c["sigma_y"], m=c["m"], g=c["g"],
                       layout="COMPACT")
        d.write_populations(P[perm], tau if c["op"] == "PR" else None)
        d.set_monitor_interval(10)
        d.step(60)
        hd = d.history()
        for r, h in zip(hb, hd):
            assert abs(r[k]["residual"] - h["residual"]) <= 1e-12 * h["residual"]
            assert abs(r[k]["flux"][2] - h["flux"][2]) <= 1e-12 * abs(h["flux"][2]) + 1e-300
    now = b.monitors()
    for k, c in enumerate(CASES):
        assert now[k]["step"] == 60 and now[k]["fluid"] == int(np.prod(c["dims"])) and now[k]["nonfinite"] == 0


def test_batch_autotune_keeps_state():
    states = _states(CASES, 90)
    b = _make_batch(CASES, states, graph_steps=10)
    ref = _make_batch(CASES, states, graph_steps=10)
    for x in (b, ref):
        x.set_monitor_interval(5)
        x.step(6)
    b.autotune(4)
    assert b.time == 6
    for x in (b, ref):
        x.step(20)
    for k in range(len(CASES)):
        assert np.array_equal(b.read_populations(k)[0], ref.read_populations(k)[0])
    hb, hr = b.history(), ref.history()
    assert [r[0]["step"] for r in hb] == [0, 5, 10, 15, 20, 25] == [r[0]["step"] for r in hr]
    # monitors are sums over work items: another tile policy sums in another order
    for rb, rr in zip(hb, hr):
        for mb, mr in zip(rb, rr):
            assert abs(mb["residual"] - mr["residual"]) <= 1e-12 * mr["residual"]
    assert b.tiles().shape == (len(CASES), 3) and np.all(np.prod(b.tiles(), axis=1) == 256)
    assert b.schedule()[0] in (0, 1, 2, 3) and b.schedule()[1] in (0, 1)


def test_every_schedule_gives_the_same_state():
    """Tile policy (incl. runs of consecutive nodes) and work-item order change
    only the launch geometry."""
    from paper_1610_01388_amd import lbm
    states = _states(CASES, 95)
    ref = None
    for pol in (0, 1, 2, 3):
        for order in (0, 1):
            b = _make_batch(CASES, states, graph_steps=4)
            b.set_schedule(pol, order)
            assert b.schedule() == (pol, order)
            b.step(9)
            got = [b.read_populations(k)[0] for k in range(len(CASES))]
            if ref is None:
                ref = got
            for g, r in zip(got, ref):
                assert np.array_equal(g, r), (pol, order)
            b.close()
    with pytest.raises(lbm.LbmError):
        b = _make_batch(CASES, states)
        b.set_schedule(4, 0)


def test_duct_sweep_recipe_runs_fp32():
    """A slice of the 256-duct sweep recipe (FP32, mixed operators) runs from
    rest without instability, and each duct matches its single-domain run."""
    from paper_1610_01388_amd import lbm
    cases = inputs.batch_sweep()[:12]
    b = lbm.Batch(cases, precision="FP32")
    b.step(50)
    mons = b.monitors()
    assert all(m["nonfinite"] == 0 for m in mons)
    for k in (0, 5, 11):
        c = cases[k]
        d = lbm.Domain(c["lattice"], c["dims"], c["periodic"], c["op"], c["nu_p"], c["sigma_y"], m=c["m"], g=c["g"],
                       precision="FP32", layout="DENSE")
        d.step(50)
        assert np.array_equal(b.read_populations(k)[0], d.read_populations()[0])


OTHER_LATTICES = {
    "D2Q9": [dict(lattice="D2Q9", dims=(33, 37, 1), periodic=(0, 0, 1), op="IR", nu_p=0.1, sigma_y=2e-4, m=0.0,
                  g=(3e-5, 0.0, 0.0)),
             dict(lattice="D2Q9", dims=(70, 5, 1), periodic=(1, 0, 1), op="PR", nu_p=0.05, sigma_y=1e-4, m=1e4,
                  g=(2e-5, 0.0, 0.0)),
             dict(lattice="D2Q9", dims=(9, 300, 1), periodic=(1, 1, 1), op="IR", nu_p=0.2, sigma_y=0.0, m=0.0,
                  g=(1e-5, 1e-5, 0.0))],
    "D3Q27": [dict(lattice="D3Q27", dims=(33, 17, 4), periodic=(0, 0, 1), op="IR", nu_p=0.1, sigma_y=2e-4, m=0.0,
                   g=(0.0, 0.0, 3e-5)),
              dict(lattice="D3Q27", dims=(9, 9, 9), periodic=(1, 1, 1), op="PR", nu_p=0.05, sigma_y=1e-4, m=1e4,
                   g=(2e-5, 1e-5, 0.0)),
              dict(lattice="D3Q27", dims=(70, 5, 3), periodic=(1, 0, 0), op="PR", nu_p=0.1, sigma_y=3e-4, m=1e3,
                   g=(2e-5, 0.0, 0.0))],
}


@pytest.mark.parametrize("name,lat", [("D2Q9", 0), ("D3Q27", 2)])
def test_other_lattices_every_schedule(name, lat):
    """D2Q9 and D3Q27 batches: under every tile policy (incl. runs of
    consecutive nodes, the default) and both work-item orders each
    simulation ends bitwise equal to its single-domain run, and the default
    schedule matches the oracle (FP64 bar)."""
    from paper_1610_01388_amd import lbm
    cases = OTHER_LATTICES[name]
    perm = perm_lib_from_oracle(lat)
    states = []
    for k, c in enumerate(cases):
        P, tau = random_state(lat, int(np.prod(c["dims"])), 70 + k, amp=1e-2, nu_p=c["nu_p"])
        states.append((P, tau, perm))
    steps = 9
    ref = []
    for k, c in enumerate(cases):
        P, tau, _ = states[k]
        d = lbm.Domain(c["lattice"], c["dims"], c["periodic"], c["op"], c["nu_p"], c["sigma_y"], m=c["m"], g=c["g"],
                       layout="DENSE")
        d.write_populations(P[perm], tau if c["op"] == "PR" else None)
        d.step(steps)
        ref.append(d.read_populations()[0])
        d.close()
    for pol in (0, 1, 2, 3):
        for order in (0, 1):
            b = _make_batch(cases, states, graph_steps=4)
            b.set_schedule(pol, order)
            b.step(steps)
            for k in range(len(cases)):
                assert np.array_equal(b.read_populations(k)[0], ref[k]), (name, pol, order, k)
            b.close()
    b = _make_batch(cases, states, graph_steps=4)
    assert b.schedule() == (3, 0)
    b.step(steps)
    for k, c in enumerate(cases):
        P, tau, _ = states[k]
        rh = oracle.rheology(oracle.PR if c["op"] == "PR" else oracle.IR, c["nu_p"], c["sigma_y"], c["m"], 1e-8,
                             0.25, c["g"])
        od = oracle.Domain(lat, c["dims"], c["periodic"], rh)
        od.set_state(P, tau)
        od.step(steps)
        rho_o, u_o, _, uy_o = od.moments()
        rho_b, u_b, _, uy_b = b.moments(k)
        assert l2rel(u_b, u_o) <= 1e-10
        assert np.max(np.abs(rho_b - rho_o)) <= 1e-12
        assert np.array_equal(uy_b, uy_o)
    b.close()
