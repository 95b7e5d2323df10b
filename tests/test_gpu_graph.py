"""Single-domain stepping by captured-graph replays (lbm_set_graph_steps):
bitwise the same populations and monitor history as eager launches, after
every replay, with eager steps, host reads and synchronisations between
replays, across changes that force a new capture (tile, monitor interval,
checkpoint load), for both schemes, both compact neighbour kernels and the
dense layout."""
import numpy as np
import pytest

from support import perm_lib_from_oracle, random_mask, random_state

pytestmark = pytest.mark.gpu

CASES = [("AA", "COMPACT", "ROWS", 0.2), ("AA", "COMPACT", "SLOTS", 0.85), ("AB", "COMPACT", "ROWS", 0.2),
         ("AA", "DENSE", None, 0.2)]


@pytest.mark.parametrize("op", ["IR", "PR"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_graph_replays_equal_eager_steps(case, op):
    from paper_1610_01388_amd import lbm
    scheme, layout, form, solid = CASES[case]
    lat, dims, per = 1, (70, 13, 9), (1, 0, 1)
    N = int(np.prod(dims))
    mask = random_mask(N, 41 + case, solid)
    P0, tau0 = random_state(lat, N, 43)
    P0 = (P0 * (1 - mask)[None, :])[perm_lib_from_oracle(lat)]

    def make(graph):
        d = lbm.Domain("D3Q19", dims, per, op, 0.1, 2e-4, m=1e4, g=(2e-5, -1e-5, 5e-6), scheme=scheme,
                       layout=layout)
        d.set_mask(mask)
        if form:
            d.set_pull_form(form)
        d.write_populations(P0, tau0 if op == "PR" else None)
        d.set_monitor_interval(10)
        if graph:
            d.set_graph_steps(20)
        return d

    eager, graph = make(False), make(True)

    def same():
        Pe, te = eager.read_populations(with_tau=op == "PR")
        Pg, tg = graph.read_populations(with_tau=op == "PR")
        assert np.array_equal(Pe, Pg)
        if op == "PR":
            assert np.array_equal(te, tg)
        he, hg = eager.history(), graph.history()
        assert [h["step"] for h in he] == [h["step"] for h in hg]
        for a, b in zip(he, hg):
            assert np.array_equal(a["flux"], b["flux"]) and a["residual"] == b["residual"] and a["mass"] == b["mass"]
        assert eager.time == graph.time

    for n in (25, 40, 3, 57):  # replays start only at multiples of 20 in the even phase
        eager.step(n)
        graph.step(n)
        same()
    blob = eager.save()
    for d in (eager, graph):
        d.set_monitor_interval(5)  # a new capture
        if layout == "COMPACT" and form == "ROWS":
            d.set_tile(64, 2, 2)
    for n in (40, 20, 7):
        eager.step(n)
        graph.step(n)
        same()
    for d in (eager, graph):
        d.load(blob)  # back to an earlier state: the history restarts
    for n in (60,):
        eager.step(n)
        graph.step(n)
        same()
    eager.close()
    graph.close()


def test_graph_steps_validation():
    from paper_1610_01388_amd import lbm
    d = lbm.Domain("D2Q9", (16, 8, 1), (1, 0, 1), "IR", 0.1, 0.0)
    for bad in (-2, 3):
        with pytest.raises(lbm.LbmError) as e:
            d.set_graph_steps(bad)
        assert e.value.code == -1
    d.set_graph_steps(0)
    d.close()
