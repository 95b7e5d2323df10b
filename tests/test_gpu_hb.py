"""GPU tests of the implicitly-regularised Herschel-Bulkley operator (IRHB:
the implicit construction of Sec. 2.3, Eq. 31, solved per node for
sigma = sigma_y + K g^n, as Sec. 3.2 notes other laws can be): FP64 parity
with the oracle (which brackets the same root by bisection) on every
lattice, both schemes, both layouts and both compact neighbour kernels,
shear-thinning and shear-thickening, with solids; the FP32 bar; n = 1
equal to the Bingham IR; the steady power-law and Herschel-Bulkley
channels against their analytic profiles."""
import numpy as np
import pytest

from support import l2rel, random_mask, run_pair

pytestmark = pytest.mark.gpu

CASES = [(0, (70, 37, 1), (1, 0, 1)), (1, (70, 13, 9), (1, 0, 1)), (2, (37, 11, 13), (0, 1, 1))]
FORMS = [("AA", {"layout": "COMPACT"}, "ROWS"), ("AA", {"layout": "COMPACT"}, "SLOTS"), ("AB", {"layout": "DENSE"}, None),
         ("AB", {"layout": "COMPACT"}, "ROWS")]


@pytest.mark.parametrize("form", range(len(FORMS)))
@pytest.mark.parametrize("lat,dims,per", CASES)
@pytest.mark.parametrize("n", [0.6, 1.4])
def test_irhb_parity_fp64(n, lat, dims, per, form):
    scheme, kw, pull = FORMS[form]
    N = int(np.prod(dims))
    mask = random_mask(N, 900 + lat, 0.15)
    ref, got, _, _ = run_pair(lat, dims, per, "IRHB", 31, mask=mask, seed=23, scheme=scheme, nu_p=0.05,
                              sigma_y=5e-5, hb_n=n, gpu_kw=kw, pull_form=pull)
    fluid = mask == 0
    assert l2rel(got[1], ref[1]) <= 1e-10
    assert np.max(np.abs(got[0] - ref[0])[fluid]) <= 1e-12
    assert np.sum(got[3] != ref[3]) <= 2  # flags may differ only within rounding of the threshold
    assert 0 < ref[3][fluid].sum() < fluid.sum()  # both regimes present


def test_irhb_fp32():
    lat, dims, per = 2, (37, 11, 13), (1, 0, 1)
    mask = random_mask(int(np.prod(dims)), 91, 0.15)
    ref, got, _, _ = run_pair(lat, dims, per, "IRHB", 60, mask=mask, seed=17, precision="FP32", nu_p=0.05,
                              sigma_y=5e-5, hb_n=0.6)
    assert l2rel(got[1], ref[1]) <= 2e-5


def test_irhb_flow_index_one_is_ir():
    from paper_1610_01388_amd import lbm
    dims, per = (37, 11, 13), (1, 0, 1)
    mask = random_mask(int(np.prod(dims)), 5, 0.2)
    out = {}
    for op in ("IR", "IRHB"):
        dom = lbm.Domain("D3Q27", dims, per, op, 0.1, 3e-4, g=(2e-5, 0, 0), hb_n=1.0)
        dom.set_mask(mask)
        dom.step(200)
        out[op] = dom.moments()
        dom.close()
    assert l2rel(out["IRHB"][1], out["IR"][1]) <= 1e-12
    assert np.array_equal(out["IRHB"][3], out["IR"][3])


def _analytic(H, n, K, g, sy):
    h, y0 = H / 2.0, sy / g
    yp = np.abs(np.arange(H) + 0.5 - h)
    a = n / (n + 1) * (g / K) ** (1 / n)
    return a * ((h - y0) ** (1 + 1 / n) - np.clip(yp - y0, 0, None) ** (1 + 1 / n)), yp < y0


@pytest.mark.parametrize("n,K,g,sy", [(0.5, 4.3e-3, 1.17e-5, 0.0), (1.5, 3.0, 6.3e-6, 0.0),
                                      (0.5, 4.3e-3, 1.17e-5, 4.68e-5)])
def test_irhb_channel_against_analytic(n, K, g, sy):
    """D2Q9 4 x 32 channel from rest, 20000 steps (steady from ~10000): the
    power-law (sigma_y = 0) and Herschel-Bulkley profiles, with exactly the
    plug nodes unyielded."""
    from paper_1610_01388_amd import lbm
    H = 32
    dom = lbm.Domain("D2Q9", (4, H, 1), (1, 0, 1), "IRHB", K, sy, g=(g, 0, 0), hb_n=n)
    dom.step(20000)
    _, u, _, uy = dom.moments()
    dom.close()
    ux = u[0].reshape(H, 4)[:, 0]
    ref, plug = _analytic(H, n, K, g, sy)
    print(n, sy, float(np.max(np.abs(ux - ref)) / ref.max()), flush=True)
    assert np.max(np.abs(ux - ref)) <= 4e-3 * ref.max()
    assert np.array_equal(uy.reshape(H, 4)[:, 0].astype(bool), plug)


def test_irhb_full_size_bench_geometry():
    """The bench's IRHB form at full size (D3Q27 256^3 sphere pack, FP64, AA,
    compact, n = 0.5, K = nu_p) from a seeded random state: two steps (both
    AA phases) against two oracle steps, every fluid node at the parity bar."""
    import oracle
    from paper_1610_01388_amd import inputs, lbm
    from support import perm_lib_from_oracle, random_state
    n = 256
    mask, _ = inputs.sphere_pack((n, n, n), 8.0, 0.7, seed=1)
    case = inputs.porous_case("IR", n=n, Bi=1.0)
    P0, _ = random_state(2, n ** 3, 37, amp=1e-3)
    P0 *= (1 - mask)[None, :]
    rh = oracle.rheology(oracle.IRHB, case["nu_p"], case["sigma_y"], 0.0, 1e-8, 0.25, case["g"], hb_n=0.5)
    od = oracle.Domain(2, case["dims"], case["periodic"], rh, mask)
    od.set_state(P0, None)
    od.step(2)
    rho_o, u_o, _, uy_o = od.moments()
    od.close()
    dom = lbm.Domain("D3Q27", case["dims"], case["periodic"], "IRHB", case["nu_p"], case["sigma_y"], g=case["g"],
                     hb_n=0.5)
    dom.set_mask(mask)
    dom.write_populations(P0[perm_lib_from_oracle(2)])
    dom.step(2)
    rho_g, u_g, _, uy_g = dom.moments()
    dom.close()
    fluid = mask == 0
    print(f"IRHB 256^3: u L2-rel {l2rel(u_g, u_o):.2e}", flush=True)
    assert l2rel(u_g, u_o) <= 1e-10
    assert np.max(np.abs(rho_g - rho_o)[fluid]) <= 1e-12
    assert np.sum(uy_g != uy_o) <= 2

