"""The oracle's pins have teeth: each plausible mistake planted in a copy of
the oracle source (a wrong weight or generator, a dropped term, a sign, a
transposed operand or index, a reversed search direction) makes the pin
suite fail. Mutants are built and run on the CPU only."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "pagani_oracle.c")

MUTANTS = {
    "weight_w7_orbit2": ("w7[1] = 980.0 / 6561.0;", "w7[1] = 981.0 / 6561.0;"),
    "weight_w5_sign": ("w5[2] = (265.0 - 100.0 * d) / 1458.0;",
                       "w5[2] = (265.0 + 100.0 * d) / 1458.0;"),
    "generator_lambda2": ("lambda[1] = sqrt(9.0 / 70.0);",
                          "lambda[1] = sqrt(9.0 / 71.0);"),
    "dropped_orbit5": ("    for (k = 0; k < 5; k++) {\n        sum7",
                       "    for (k = 0; k < 4; k++) {\n        sum7"),
    "orbit4_wrong_index": ("x[j] = c[j] + (sj == 0 ? 1.0 : -1.0) * (lam[3] * h[j]);\n"
                           "                    f = oracle_f(",
                           "x[j] = c[j] + (sj == 0 ? 1.0 : -1.0) * (lam[3] * h[i]);\n"
                           "                    f = oracle_f("),
    "fourth_diff_ratio": ("- (P3[i] - 2.0 * fc) / 7.0);", "- (P3[i] - 2.0 * fc) / 5.0);"),
    "two_level_transposed": ("E[b] = E[b] * g + delta;", "E[b] = E[a] * g + delta;"),
    "two_level_quarter": ("double delta = fabs(V[a] + V[b] - Vp[i]) / 4.0;",
                          "double delta = fabs(V[a] + V[b] - Vp[i]) / 2.0;"),
    "classify_strict": ("(uint8_t)(E[i] > tau_rel * fabs(V[i]))",
                        "(uint8_t)(E[i] >= tau_rel * fabs(V[i]))"),
    "split_upper_corner": ("lo2[k * ld_out + j + na] = l + half;",
                           "lo2[k * ld_out + j + na] = l + ww;"),
    "search_direction": ("if (dir > 0) t = t + (mx - t) / 2.0;",
                         "if (dir < 0) t = t + (mx - t) / 2.0;"),
    "search_budget": ("if (e_abar <= P_max * allow) {",
                      "if (e_abar <= P_max * (e_it - allow)) {"),
    "search_pmax_step": ("P_max = P_max + 0.10;", "P_max = P_max + 0.05;"),
    "uniform_split_offset": ("lo[k * ld + r] = a[k] + (double)digit * width;",
                             "lo[k * ld + r] = a[k] + (double)(digit + 1) * width;"),
    "sum_uncompensated": ("    return s + c;\n}", "    return s;\n}"),
}


# mistakes in the parameter derivatives and the leaf bookkeeping, caught by
# the gradient pins
GRAD_MUTANTS = {
    "grad_gauss_u_sign": ("df[d + i] = 2.0 * (a * a) * t * f;",
                          "df[d + i] = -2.0 * (a * a) * t * f;"),
    "grad_gauss_a_factor": ("df[i] = -2.0 * a * (t * t) * f;",
                            "df[i] = -1.0 * a * (t * t) * f;"),
    "grad_product_peak_u": ("df[d + i] = f * (2.0 * t) / q;",
                            "df[d + i] = f * (2.0 * t) * q;"),
    "grad_osc_phase": ("df[d] = -2.0 * M_PI * f;", "df[d] = -M_PI * f;"),
    "grad_corner_power": ("f = pow(s, -(double)(d + 2));",
                          "f = pow(s, -(double)(d + 1));"),
    "grad_orbit4_weight": ("grad_point(family, d, par, x, w7[3], np, g, gabs);",
                           "grad_point(family, d, par, x, w7[2], np, g, gabs);"),
    "grad_no_volume": ("        g[q] = vol * g[q];", "        g[q] = g[q];"),
    "leaves_mask_inverted": ("if (skip && skip[i]) continue;",
                             "if (skip && !skip[i]) continue;"),
    "leaves_finished_dropped": ("        LEAVES(A);             /* the regions finished in this iteration */",
                                "        /* finished regions dropped */"),
}

# mistakes in the extra families of the paper's suite
SUITE_MUTANTS = {
    "c0_no_abs": ("s = s + p[i] * fabs(x[i] - p[d + i]);",
                  "s = s + p[i] * (x[i] - p[d + i]);"),
    "discontinuous_cutoff_param": ("if (!(x[i] < p[d + i])) return 0.0;",
                                   "if (!(x[i] < p[i])) return 0.0;"),
    "box_not_squared": ("            s = s + x[i] * x[i];\n        return pow(s, p[0]);",
                        "            s = s + x[i];\n        return pow(s, p[0]);"),
}

# mistakes in the four null rules and the estimate built on them
NULL4_MUTANTS = {
    "null_pair_multiplicity": ("m[3] = 2.0L * d * (d - 1);", "m[3] = 1.0L * d * (d - 1);"),
    "null_pair_mean": ("g[1][3] = 2.0L * L2[3] / d;", "g[1][3] = L2[3] / d;"),
    "null_degree_swap": ("nul[1][o] = (double)(n7 * q[2][o]);",
                         "nul[1][o] = (double)(n7 * q[1][o]);"),
    "null_rms_half": ("e3 = sqrt((nv[1] * nv[1] + nv[2] * nv[2]) / 2.0);",
                      "e3 = sqrt(nv[1] * nv[1] + nv[2] * nv[2]);"),
    "null_r_power": ("return kappa * r * r * e3;", "return kappa * r * e3;"),
    "null_ratio_inverted": ("double r = or_ratio(e3, e1), r2 = or_ratio(e5, e3), big;",
                            "double r = or_ratio(e1, e3), r2 = or_ratio(e5, e3), big;"),
    "null_kappa_d5": ("{0.0, 0.0, 2.0, 2.0, 3.8, 15.0,", "{0.0, 0.0, 2.0, 2.0, 3.8, 7.0,"),
    "null_branch_inverted": ("if (r <= OR_NULL_RC) return", "if (r > OR_NULL_RC) return"),
    "null_smallest_magnitude": ("return big > e1 ? big : e1;", "return big < e1 ? big : e1;"),
}

# mistakes in the replay mode's certification of ties (each would let a
# real disagreement of a GPU run pass as a rounding tie) and in which
# searches relax P_max, caught by the replay pins
REPLAY_MUTANTS = {
    "replay_axis_always_tie": ("if (cert) rs->axis_override++;",
                               "if (1) rs->axis_override++;"),
    "replay_class_always_tie": ("if (c_rel) rs->class_override++;",
                                "if (1) rs->class_override++;"),
    "replay_threshold_always_tie": ("else if (c_thr) rs->thr_override++;",
                                    "else if (1) rs->thr_override++;"),
    "replay_term_always_tie": ("int cert = gap <= 1e-9 * e_tot;", "int cert = 1;"),
    "replay_trigger_always_tie": (
        "int cert = gap <= 1e-9 * tau_rel * fabs(v_tot) && !trig_b;", "int cert = 1;"),
    "replay_search_unchecked": (
        "if (ok != (rec.thr_ok != 0) || trials != rec.thr_trials) {", "if (0) {"),
    "run_pmax_memory_only": ("pmax_relax == 0 || 2 * n_rel > cap,",
                             "2 * n_rel > cap,"),
    "run_reserve_under_memory": ("if (budget == 0 && !(2 * n_rel > cap))",
                                 "if (budget == 0)"),
    "run_reserve_active_regions": ("for (i = 0; i < s; i++) Af[i] = (uint8_t)!A_rel[i];",
                                   "for (i = 0; i < s; i++) Af[i] = A_rel[i];"),
    "run_reserve_never": ("if (budget == 0 && !(2 * n_rel > cap))",
                          "if (budget == 2)"),
    "run_listing_budget_sign": ("allow = tau_rel * fabs(v_tot) - e_f;    /* e_it - e_b */",
                                "allow = tau_rel * fabs(v_tot) + e_f;    /* e_it - e_b */"),
    "replay_t_unchecked": ("if (fabs(rec.t - t) > band) rs->search_hard++;",
                           "if (0) rs->search_hard++;"),
}

CASES = [(n, "test_oracle_pins.py") for n in sorted(MUTANTS)] + \
        [(n, "test_oracle_replay_pins.py") for n in sorted(REPLAY_MUTANTS)] + \
        [(n, "test_oracle_grad_pins.py") for n in sorted(GRAD_MUTANTS)] + \
        [(n, "test_oracle_suite_pins.py") for n in sorted(SUITE_MUTANTS)] + \
        [(n, "test_oracle_null4_pins.py") for n in sorted(NULL4_MUTANTS)]


@pytest.mark.parametrize("name,pins", CASES, ids=[c[0] for c in CASES])
def test_mutant_is_caught(name, pins, tmp_path):
    old, new = {**MUTANTS, **GRAD_MUTANTS, **SUITE_MUTANTS, **NULL4_MUTANTS,
                **REPLAY_MUTANTS}[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique: {name}"
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-ffp-contract=off",
                    "-shared", "-fPIC", "-o", str(lib), str(mut), "-lm"], check=True)
    env = dict(os.environ, PAGANI_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not slow", os.path.join(ROOT, "tests", pins)],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
