"""The lattice-choice result of Sec. 4.1 on the GPU: in steady laminar duct
flow (Newtonian, 25 lu circular and square ducts at the printed U_max =
0.01167 and 0.009734), D3Q19 carries transverse currents of order 1e-7
lu/ts with both the BGK and the TRT (Lambda = 1/4) collision, while D3Q27
has none beyond rounding.  (The paper also reports the currents unchanged
at 100 lu; at fixed U_max they come out 10-100x smaller here, so that part
is not claimed.)  BGK is the PR operator with sigma_y = 0 and Lambda =
(tau - 1/2)^2; nu_p = 0.1."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

CMAX = 1.178741652
NU = 0.1


def _duct(lat, shape, lam, H=25):
    from paper_1610_01388_amd import lbm
    if shape == "square":
        U = 0.009734
        g = 16 * NU * U / (CMAX * H * H)
        mask = None
    else:
        U = 0.01167
        R = H / 2.0
        g = 4 * NU * U / (R * R)
        yy, xx = np.mgrid[0:H, 0:H]
        mask = (((xx + 0.5 - R) ** 2 + (yy + 0.5 - R) ** 2) > R * R).astype(np.uint8).reshape(-1)
    dom = lbm.Domain(lat, (H, H, 1), (0, 0, 1), "PR", NU, 0.0, g=(0.0, 0.0, g), lambda_trt=lam)
    if mask is not None:
        dom.set_mask(mask)
    prev, n = None, 0
    while n < 1_000_000:
        dom.step(20000)
        n += 20000
        u = dom.monitors()["umax"]
        if prev is not None and abs(u - prev) <= 1e-12 * u:
            break
        prev = u
    _, uu, _, _ = dom.moments()
    return float(uu[2].max()), float(np.abs(uu[:2]).max())


@pytest.mark.parametrize("lam", [(3 * NU) ** 2, 0.25], ids=["BGK", "TRT"])
@pytest.mark.parametrize("shape", ["circle", "square"])
def test_d3q19_currents_d3q27_none(shape, lam):
    u19, t19 = _duct("D3Q19", shape, lam)
    u27, t27 = _duct("D3Q27", shape, lam)
    print(f"{shape} Lambda={lam:g}: D3Q19 Umax {u19:.5f} transverse {t19:.2e}; D3Q27 Umax {u27:.5f} transverse {t27:.2e}",
          flush=True)
    assert 1e-8 <= t19 <= 1e-6
    assert t27 <= 1e-15
    assert abs(u19 - u27) <= 2e-2 * u27
