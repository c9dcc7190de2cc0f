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
    "orbit4_wrong_index": ("x[j] = c[j] + (sj == 0 ? 1.0 : -1.0) * (lam[3] * h[j]);",
                           "x[j] = c[j] + (sj == 0 ? 1.0 : -1.0) * (lam[3] * h[i]);"),
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
    "search_budget": ("if (e_abar <= P_max * (e_it - e_b)) {",
                      "if (e_abar <= P_max * e_b) {"),
    "uniform_split_offset": ("lo[k * ld + r] = a[k] + (double)digit * width;",
                             "lo[k * ld + r] = a[k] + (double)(digit + 1) * width;"),
    "sum_uncompensated": ("    return s + c;\n}", "    return s;\n}"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique: {name}"
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-ffp-contract=off",
                    "-shared", "-fPIC", "-o", str(lib), str(mut), "-lm"], check=True)
    env = dict(os.environ, PAGANI_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not slow", os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
