"""Mutation check of the oracle pins: each case plants one plausible mistake
in a copy of the oracle source (on the CPU), rebuilds it and requires the pin
suite to fail.  The mutated library is loaded only by the child pytest."""

import os
import subprocess
import sys
import tempfile

import pytest

from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    "no_coriolis_in_K_slope": ("double dm = w->eta[b] - w->eta[bm] - kx * (w->cx[bm] + w->cx[b]);",
                               "double dm = w->eta[b] - w->eta[bm];"),
    "wall_keeps_f_sign": ("w->f[b] = sg * w->f[a];\n                    w->land[b] = w->land[a];\n                }\n            }\n    /* y-sides */",
                          "w->f[b] = w->f[a];\n                    w->land[b] = w->land[a];\n                }\n            }\n    /* y-sides */"),
    "bathymetry_source_halved": ("g / (2.0 * p->dx) * (hE + hW) * (HE - HW)",
                                 "g / (4.0 * p->dx) * (hE + hW) * (HE - HW)"),
    "no_positivity_fix": ("if (eE + HE < 0.0) { eE = -HE; eW = 2.0 * w->eta[b] - eE; }",
                          "if (0) { eE = -HE; eW = 2.0 * w->eta[b] - eE; }"),
    "transverse_knp_diffusion": ("out[2] = out[0] * (out[0] >= 0.0 ? vL : vR);",
                                 "out[2] = (ap * pL * vL - am * pR * vR) * w + ap * am * w * (R[2] - L[2]);"),
    "friction_full_dt_in_stage2": ("double den = 1.0 + 0.5 * dt * sw->S[o];",
                                   "double den = 1.0 + dt * sw->S[o];"),
    "y_slope_uses_dx": ("double ky = p->dy / (2.0 * p->g);", "double ky = p->dx / (2.0 * p->g);"),
    "frs_alpha_inverted": ("double alpha = 1.0 - tanh((double)d / p->frs_d0);",
                           "double alpha = tanh((double)d / p->frs_d0);"),
    "cfl_without_quarter": ("return p->courant * 0.25 * best;", "return p->courant * best;"),
    "land_face_not_reflective": ("if (landR) { R[0] = L[0]; R[1] = -L[1]; R[2] = L[2]; }", ""),
    "stage2_wind_at_tn": ("compute_rhs(p, s, &sw->w, e1, u1, v1, t + dt,", "compute_rhs(p, s, &sw->w, e1, u1, v1, t,"),
    "minmod_central_unhalved": ("return or_minmod3(theta * dminus, 0.5 * (dminus + dplus), theta * dplus);",
                                "return or_minmod3(theta * dminus, dminus + dplus, theta * dplus);"),
    "coriolis_source_sign": ("double Cx = w->f[b] * (c * hvn - sn * hue);", "double Cx = -w->f[b] * (c * hvn - sn * hue);"),
    "desing_kappa_floor": ("double lo = fmin(h * h / (2.0 * kappa) + 0.5 * kappa, kappa);",
                           "double lo = fmin(h * h / (2.0 * kappa), kappa);"),
    "large_pond_no_strong_wind_branch": ("double cd = speed < 11.0 ? 1.2e-3 : (0.49 + 0.065 * speed) * 1e-3;",
                                         "double cd = 1.2e-3;"),
    "wind_time_weights_swapped": ("W[c] = (1.0 - s) * w10_sample(p, k, gx, gy, c) + s * w10_sample(p, kb, gx, gy, c);",
                                  "W[c] = s * w10_sample(p, k, gx, gy, c) + (1.0 - s) * w10_sample(p, kb, gx, gy, c);"),
    "dt_policy_never_updates": ("                    t_upd += p->dt_interval;\n", "                    t_upd += 1e30;\n"),
    "dt_policy_hold_not_kept": ("                    dt_hold = dt;\n", ""),
    "stress_field_through_large_pond": ("    if (p->w10_kind == 1) {  /* a stress field: interpolated as it is */",
                                        "    if (0) {"),
    "wind_samples_at_corners": ("double gx = (i + 0.5) * p->w10_nx / (double)p->nx - 0.5;",
                                "double gx = (i + 0.5) * (p->w10_nx - 1) / (double)p->nx;"),
    "energy_kinetic_unhalved": ("e += (0.5 * (hu[o] * hu[o] + hv[o] * hv[o]) / hs",
                                "e += ((hu[o] * hu[o] + hv[o] * hv[o]) / hs"),
    "energy_potential_unhalved": ("/ hs + 0.5 * p->g * eta[o] * eta[o]) * area;",
                                  "/ hs + p->g * eta[o] * eta[o]) * area;"),
    "energy_depth_not_desingularised": ("/ hs + 0.5 * p->g * eta[o] * eta[o]) * area;",
                                        "/ h + 0.5 * p->g * eta[o] * eta[o]) * area;"),
    "diagnostics_count_land": ("continue;\n            double h = eta[o] + cell_hbar(s, p->nx, i, j);\n"
                               "            double hs = or_desing(h, p->kappa);\n            m +=",
                               ";\n            double h = eta[o] + cell_hbar(s, p->nx, i, j);\n"
                               "            double hs = or_desing(h, p->kappa);\n            m +="),
    "mass_without_mean_depth": ("            m += h * area;", "            m += eta[o] * area;"),
    "mass_one_corner_depth": ("double h = eta[o] + cell_hbar(s, p->nx, i, j);\n"
                              "            double hs = or_desing(h, p->kappa);\n            m +=",
                              "double h = eta[o] + s->Hc[(size_t)j * (p->nx + 1) + i];\n"
                              "            double hs = or_desing(h, p->kappa);\n            m +="),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name):
    old, new = MUTANTS[name]
    src = open(O.SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique/found: {name}"
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "m.c")
        with open(c, "w") as fh:
            fh.write(src.replace(old, new))
        import shutil
        shutil.copy(os.path.join(os.path.dirname(O.SRC), "swe_oracle.h"), d)
        so = os.path.join(d, "libm.so")
        subprocess.check_call(["gcc", *O.CFLAGS, "-o", so, c, "-lm"])
        env = dict(os.environ, SWE_ORACLE_LIB=so, OMP_NUM_THREADS="4")
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                            "tests/test_oracle_pins.py", "-k", "not printed_case"],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
        assert r.returncode != 0, f"pins did not catch mutant {name}:\n{r.stdout[-2000:]}"
