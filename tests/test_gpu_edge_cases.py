"""Degenerate inputs on the GPU: a domain with no fluid node (nothing to
update; monitors and readout report zeros, checkpoints round-trip), a single
fluid node enclosed by solids (every direction bounced back), and a
1 x 1 x 1 periodic box (every neighbour is the node itself), the last two
against the FP64 oracle, for both compact neighbour kernels and the dense
layout, AA and A/B."""
import numpy as np
import pytest

from support import l2rel, run_pair

pytestmark = pytest.mark.gpu

FORMS = [("AA", "COMPACT", "ROWS"), ("AA", "COMPACT", "SLOTS"), ("AB", "COMPACT", "SLOTS"), ("AA", "DENSE", None),
         ("AB", "DENSE", None)]


@pytest.mark.parametrize("form", range(len(FORMS)))
def test_no_fluid_node(form):
    from paper_1610_01388_amd import lbm
    scheme, layout, pull = FORMS[form]
    dims = (70, 9, 5)
    N = int(np.prod(dims))
    dom = lbm.Domain("D3Q27", dims, (1, 0, 1), "PR", 0.1, 1e-4, m=1e4, g=(1e-5, 0, 0), scheme=scheme, layout=layout)
    dom.set_mask(np.ones(N, dtype=np.uint8))
    if pull:
        dom.set_pull_form(pull)
    dom.set_monitor_interval(2)
    dom.step(7)
    m = dom.monitors()
    assert m["fluid"] == 0 and m["mass"] == 0.0 and m["umax"] == 0.0 and m["unyielded"] == 0
    assert m["status"] == 0
    assert all(h["fluid"] == 0 for h in dom.history())
    rho, u, _, uy = dom.moments()
    assert not rho.any() and not u.any() and not uy.any()
    blob = dom.save()
    dom.load(blob)
    dom.step(1)
    assert dom.time == 8
    dom.close()


@pytest.mark.parametrize("form", range(len(FORMS)))
@pytest.mark.parametrize("op", ["IR", "PR"])
def test_single_enclosed_fluid_node(op, form):
    scheme, layout, pull = FORMS[form]
    dims = (5, 5, 5)
    mask = np.ones(125, dtype=np.uint8)
    mask[62] = 0  # centre
    ref, got, pref, pgot = run_pair(2, dims, (1, 1, 1), op, 20, mask=mask, seed=3, scheme=scheme,
                                    gpu_kw={"layout": layout}, pull_form=pull)
    assert np.max(np.abs(got[0] - ref[0])) <= 1e-12
    assert np.max(np.abs(got[1] - ref[1])) <= 1e-12
    assert np.array_equal(got[3], ref[3])
    assert np.max(np.abs(pgot[0][:, 62] - pref[0][:, 62])) <= 1e-13


@pytest.mark.parametrize("form", range(len(FORMS)))
@pytest.mark.parametrize("lat", [0, 1, 2])
@pytest.mark.parametrize("op", ["IR", "PR"])
def test_one_node_periodic_box(op, lat, form):
    scheme, layout, pull = FORMS[form]
    ref, got, _, _ = run_pair(lat, (1, 1, 1), (1, 1, 1), op, 15, seed=4, scheme=scheme, gpu_kw={"layout": layout},
                              pull_form=pull)
    assert l2rel(got[1], ref[1]) <= 1e-10
    assert np.max(np.abs(got[0] - ref[0])) <= 1e-12
