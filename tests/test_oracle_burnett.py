"""Pins of the flow-axis correction of Sec. 4.2.2: for a flow known to run
along one axis, the collision may drop that axis's normal component (PR:
the strain-rate component d_aa; IR: T_aa before the deviator).  The paper
reports what it changes, and the oracle must show the same in a D3Q27
Bingham square duct driven along z (H = 15, Bi = 0.4, nu_p = 0.0125):

  * IR: without the correction, T_zz redistributed by the deviator drives
    transverse currents near the yield surface; with it, the transverse
    velocity stays at rounding level and the axial velocity barely moves;
  * PR at large m: without the correction the Burnett-order d_zz keeps the
    strain rate from vanishing in the plug, so nu_app saturates below its
    limit nu_p + m sigma_y / rho and no node counts as unyielded; with it the
    plug reaches the limit exactly; the same holds with the implicit
    relaxation-time update of Sec. 3.
"""
import numpy as np
import pytest

H, NU, G = 15, 0.0125, 2e-6
SY = 0.4 * G * H / 4.0


def _duct(orc, op, m, axis, steps=4000):
    rh = orc.rheology(op, NU, SY, m, 1e-8, 0.25, (0.0, 0.0, G), flow_axis=axis)
    dom = orc.Domain(2, (H, H, 1), (0, 0, 1), rh)
    dom.step(steps)
    return dom.moments()


def test_ir_transverse_currents_vanish_with_correction(orc):
    _, u0, _, uy0 = _duct(orc, orc.IR, 0.0, 0)
    _, u1, _, uy1 = _duct(orc, orc.IR, 0.0, 3)
    uz = u0[2].max()
    assert np.abs(u0[:2]).max() > 1e-7 * uz          # Burnett-driven currents
    assert np.abs(u1[:2]).max() < 1e-12 * uz         # rounding only
    assert abs(u1[2].max() - uz) < 1e-4 * uz         # axial flow nearly unchanged
    assert uy1.sum() > 0 and uy0.sum() > 0


@pytest.mark.parametrize("op", ["PR", "PRI"])
@pytest.mark.parametrize("m", [1e6, 1e9])
def test_pr_plug_reaches_viscosity_limit_with_correction(orc, m, op):
    """Explicit and implicit (Sec. 3) relaxation-time updates alike."""
    nu_lim = NU + m * SY
    _, u0, nu0, uy0 = _duct(orc, getattr(orc, op), m, 0)
    _, u1, nu1, uy1 = _duct(orc, getattr(orc, op), m, 3)
    assert abs(nu1.max() - nu_lim) <= 1e-9 * nu_lim
    assert nu0.max() < (1.0 - 1e-3) * nu_lim
    assert uy1.sum() > 0
    if m >= 1e9:
        assert uy0.sum() == 0  # the saturated plug is never recognised as unyielded
