"""FP64 parity with the oracle at the full sizes of the bench's other forms:
two steps (both AA phases, or two A/B steps) from a seeded random state,
every fluid node compared at the parity bar.  The main workload (256^3
pack, IR / PR, all precisions) is in test_gpu_features.py, PRI in
test_gpu_pri.py and IRHB in test_gpu_hb.py; here:

* D3Q19 on the same 256^3 pack;
* D2Q9 on the 51 x 51 tiling of the Table 2 cylinder cell (4080^2);
* the tight medium (overlapping spheres, porosity 0.15) with the default
  neighbour kernel (the slot kernel at that fluid fraction);
* the all-fluid periodic 256^3 box;
* A/B streaming and the dense layout on the 256^3 pack."""
import numpy as np
import pytest

import oracle
from paper_1610_01388_amd import inputs
from support import LAT_NAMES, l2rel, perm_lib_from_oracle, random_state

pytestmark = pytest.mark.gpu

N3 = 256


def _geometry(name):
    if name in ("d3q19_pack", "ab_pack", "dense_pack"):
        mask, _ = inputs.sphere_pack((N3, N3, N3), 8.0, 0.7, seed=1)
        case = inputs.porous_case("IR", n=N3, Bi=1.0)
        lat = 1 if name == "d3q19_pack" else 2
        return lat, case["dims"], case["periodic"], mask, case
    if name == "tight":
        mask, _ = inputs.overlapping_spheres((N3, N3, N3), 8.0, 0.15, seed=1)
        case = inputs.porous_case("IR", n=N3, Bi=1.0)
        return 2, case["dims"], case["periodic"], mask, case
    if name == "box":
        case = inputs.porous_case("IR", n=N3, Bi=1.0)
        return 2, case["dims"], case["periodic"], np.zeros(N3 ** 3, dtype=np.uint8), case
    if name == "cylinders":
        cell = inputs.cylinder_case("IR", sigma_y=1e-5)
        tiles = 51
        mask = np.tile(cell["mask"].reshape(80, 80), (tiles, tiles)).reshape(-1)
        return 0, (80 * tiles, 80 * tiles, 1), cell["periodic"], mask, cell
    raise ValueError(name)


@pytest.mark.parametrize("name", ["d3q19_pack", "cylinders", "tight", "box", "ab_pack", "dense_pack"])
def test_full_size_forms_vs_oracle(name):
    from paper_1610_01388_amd import lbm
    lat, dims, per, mask, case = _geometry(name)
    N = int(np.prod(dims))
    g = tuple(case["g"])
    P0, _ = random_state(lat, N, 71, amp=1e-3)
    P0 *= (1 - mask)[None, :]
    rh = oracle.rheology(oracle.IR, case["nu_p"], case["sigma_y"], 0.0, 1e-8, 0.25, g)
    od = oracle.Domain(lat, dims, per, rh, mask)
    od.set_state(P0, None)
    od.step(2)
    rho_o, u_o, _, uy_o = od.moments()
    od.close()
    kw = {"scheme": "AB"} if name == "ab_pack" else {"layout": "DENSE"} if name == "dense_pack" else {}
    dom = lbm.Domain(LAT_NAMES[lat], dims, per, "IR", case["nu_p"], case["sigma_y"], g=g, **kw)
    dom.set_mask(mask)
    form = dom.pull_form()
    dom.write_populations(P0[perm_lib_from_oracle(lat)])
    dom.step(2)
    rho_g, u_g, _, uy_g = dom.moments()
    dom.close()
    fluid = mask == 0
    print(f"{name}: {LAT_NAMES[lat]} {dims} fluid {int(fluid.sum())} kernel {form}: "
          f"u L2-rel {l2rel(u_g, u_o):.2e}", flush=True)
    if name == "tight":
        assert form == "SLOTS"
    assert l2rel(u_g, u_o) <= 1e-10
    assert np.max(np.abs(rho_g - rho_o)[fluid]) <= 1e-12
    assert np.array_equal(uy_g, uy_o)
