"""Plant plausible mistakes in a copy of the oracle (on the CPU) and check
that the pins catch each one (among them: streaming that ignores interior
solids, and a superficial flux divided by the fluid nodes instead of all
nodes, both caught by the brute-force comparison on tiny grids).  Several mutations are the literal forms of
passages that are garbled in the paper (the 3/2 prefactor of f_sigma, the
coefficient 4 of the IR force term, the yield test T >= sigma_y, the
deviator sigma - Tr(sigma) I, the interpolation denominator of Eq. 37); the
pins reject them, which is the evidence for the readings the oracle takes.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lbm_oracle.c")

MUTATIONS = {
    "fsigma_prefactor_literal_3_2": ("L->w[i] / (2.0 * CS2 * CS2) * contr", "1.5 * L->w[i] * contr"),
    "force_term_literal_4w_over_rho": ("phi[i] = L->w[i] * cF / CS2;", "phi[i] = 4.0 * L->w[i] * cF / rho;"),
    "yield_test_literal": ("if (Tn > sqrt2 * rh->sigma_y) {", "if (Tn >= rh->sigma_y) {"),
    "deviator_literal_full_trace": ("? tr / L->d : 0.0);", "? tr : 0.0);"),
    "ir_velocity_without_half_force": ("u[a] = (j[a] + 0.5 * F[a]) / rho;", "u[a] = j[a] / rho;"),
    "strain_rate_missing_factor_2": ("(2.0 * rho * CS2 * tau_prev)", "(rho * CS2 * tau_prev)"),
    "trt_rates_swapped": ("/ tau_even - (f_asym - e_asym) / tau_odd", "/ tau_odd - (f_asym - e_asym) / tau_even"),
    "edm_sign": ("fpost[i] = fbar[i] + omega + (feq_shift[i] - feq[i]);",
                 "fpost[i] = fbar[i] + omega + (feq[i] - feq_shift[i]);"),
    "bounce_back_without_reversal": ("fbar[i] = dom->P[dom->L.opp[i] * dom->N + n];",
                                     "fbar[i] = dom->P[i * dom->N + n];"),
    "streaming_downstream": ("int p[3] = {x - c[0], y - c[1], z - c[2]};",
                             "int p[3] = {x + c[0], y + c[1], z + c[2]};"),
    "equilibrium_u2_sign": ("- uu / (2.0 * CS2));", "+ uu / (2.0 * CS2));"),
    "d3q27_corner_weight": ("wk[3] = 1.0 / 216.0;", "wk[3] = 1.0 / 108.0;"),
    "interpolation_literal_denominator": ("return nu0 + (gamma / rh->gamma_c) * (nuc - nu0);",
                                          "return (rh->gamma_c - gamma) / gamma * nu0 + (gamma / rh->gamma_c) * nuc;"),
    "papanastasiou_sign": ("(rho * gamma) * (-expm1(-rh->m * gamma));", "(rho * gamma) * (expm1(-rh->m * gamma));"),
    "pr_output_velocity_no_half_force": ("out[3 + a] = u[a] + 0.5 * rh->g[a];", "out[3 + a] = u[a];"),
    "ir_unyielded_stress_sign": ("sig[a][b] = -Tdev[a][b];", "sig[a][b] = Tdev[a][b];"),
    "ir_relaxes_full_tensor": ("Tdev[a][b] = T[a][b] - ((a == b && a < L->d) ? tr / L->d : 0.0);",
                               "Tdev[a][b] = T[a][b];"),
    "residual_reference_not_kept": ("    if (record)\n        for (int64_t j = 0;", "    if (0)\n        for (int64_t j = 0;"),
    "residual_unsquared": ("        num += d2;", "        num += sqrt(d2);"),
    "flow_axis_off_by_one": ("if (rh->flow_axis >= 1 && rh->flow_axis <= 3) T[rh->flow_axis - 1][rh->flow_axis - 1] = 0.0;",
                             "if (rh->flow_axis >= 1 && rh->flow_axis <= 3) T[rh->flow_axis % 3][rh->flow_axis % 3] = 0.0;"),
    "pri_bisection_flipped": ("        if (F > 0.0) hi = mid;\n        else lo = mid;", "        if (F > 0.0) lo = mid;\n        else hi = mid;"),
    "pri_bracket_without_density": ("double hi = 0.5 + (rh->nu_p + rh->m * rh->sigma_y / rho) / CS2;",
                                    "double hi = 0.5 + (rh->nu_p + rh->m * rh->sigma_y) / CS2 * 0.5;"),
    "mrt_no_bulk_group": ("L->mrt_group[nrow] = first_deg2 ? MRT_BULK : MRT_SHEAR;", "L->mrt_group[nrow] = MRT_SHEAR;"),
    "mrt_inverse_without_weights": ("for (int i = 0; i < L->q; ++i) out[i] += sk * L->w[i] * L->mrt[k][i];",
                                    "for (int i = 0; i < L->q; ++i) out[i] += sk * L->mrt[k][i] / L->q;"),
    "flow_axis_pr_ignored": ("can be set to zero. */\n    if (rh->flow_axis >= 1 && rh->flow_axis <= 3) D[rh->flow_axis - 1]",
                             "can be set to zero. */\n    if (0) D[rh->flow_axis - 1]"),
    "hb_strain_factor_exponent": ("pow(3.0 / sqrt(2.0), rh->hb_n - 1.0)", "pow(3.0 / sqrt(2.0), rh->hb_n)"),
    "hb_stress_from_full_s": ("sig_mag = Tn - 0.5 * s_mag;", "sig_mag = Tn - s_mag;"),
    "hb_bracket_too_small": ("double lo = 0.0, hi = 2.0 * (Tn - sqrt(2.0) * rh->sigma_y);",
                             "double lo = 0.0, hi = (Tn - sqrt(2.0) * rh->sigma_y);"),
    "streaming_ignores_solids": ("    return dom->solid[m] ? -1 : m;", "    return m;"),
    "flux_over_fluid_nodes": ("for (int a = 0; a < 3; ++a) out[a] = flux[a] / (double)dom->N;",
                              "for (int a = 0; a < 3; ++a) out[a] = flux[a] / (double)nfl;"),
    "flow_axis_pri_ignored": ("(2.0 * rho * CS2);\n    if (rh->flow_axis >= 1 && rh->flow_axis <= 3) D[rh->flow_axis - 1]",
                              "(2.0 * rho * CS2);\n    if (0) D[rh->flow_axis - 1]"),
}

PIN_TESTS = ["tests/test_oracle_lattice.py", "tests/test_oracle_bruteforce.py", "tests/test_oracle_operators.py",
             "tests/test_oracle_flows.py", "tests/test_oracle_residual.py", "tests/test_oracle_burnett.py",
             "tests/test_oracle_mrt.py", "tests/test_oracle_pri.py", "tests/test_oracle_hb.py"]
# The pin file aimed at a mutation's area runs first (all files still run
# until one fails), so that the suite does not spend minutes on flow pins
# before reaching the one that targets the mistake.
FIRST = {"streaming_": "tests/test_oracle_bruteforce.py", "flux_": "tests/test_oracle_bruteforce.py",
         "residual_": "tests/test_oracle_residual.py", "flow_axis_": "tests/test_oracle_burnett.py",
         "pri_": "tests/test_oracle_pri.py", "mrt_": "tests/test_oracle_mrt.py", "hb_": "tests/test_oracle_hb.py"}


def _pin_order(name):
    first = [f for pre, f in FIRST.items() if name.startswith(pre)]
    return first + [f for f in PIN_TESTS if f not in first]


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_reject_planted_mistake(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not found once: {old}"
    mutated = tmp_path / "lbm_oracle.c"
    mutated.write_text(src.replace(old, new))
    (tmp_path / "lbm_oracle.h").write_text(open(os.path.join(ROOT, "oracle", "lbm_oracle.h")).read())
    so = tmp_path / "liboracle_mut.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
                           str(mutated), "-o", str(so), "-lm"])
    env = dict(os.environ, LBM_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *_pin_order(name)], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode != 0, f"pins did not catch mutation {name}:\n{r.stdout[-2000:]}"
