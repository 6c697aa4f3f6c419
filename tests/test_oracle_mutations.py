"""Planted mistakes in a copy of the CPU reference must fail the pins.

Each case edits one plausible mistake into a temporary copy of
``oracle/kl_oracle.c`` (a transposed operand, the product read left to
right, a wrong sign in the trace recipe, the repelling seed, the wrong
seed letter, a wrong skip in the unranking, swapped bin axes, a dropped
term, the other root of the trace quadratic), builds it with gcc, and runs
the pin tests against the planted build in a child process.  The pins pass
on the real reference and must fail on every planted copy.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "kl_oracle.c")

MUTATIONS = {
    "transposed_operand": ("r.a = x.a * y.a + x.b * y.c;", "r.a = x.a * y.a + x.c * y.b;"),
    "left_to_right_product": ("for (int j = 1; j < d; j++) m = mat_mul(m, g->g[w[j]]);",
                              "for (int j = 1; j < d; j++) m = mat_mul(g->g[w[j]], m);"),
    "recipe_sign": ("a.b = (ta * tab - 2.0 * tb + I4)", "a.b = (ta * tab - 2.0 * tb - I4)"),
    "repelling_seed": ("*out = (km > kp) ? zm : zp;", "*out = (km < kp) ? zm : zp;"),
    "first_letter_seed": ("return mobius(m, g->fix[w[d - 1]]);", "return mobius(m, g->fix[w[0]]);"),
    "unrank_skip": ("if (prev >= 0 && c == INVERSE[prev]) continue;",
                    "if (prev >= 0 && c == prev) continue;"),
    "bin_axes_swapped": ("*bin = row * w->width + col;", "*bin = col * w->width + row;"),
    "dropped_term": ("cplx disc = (ta * tb) * (ta * tb) - 4.0 * (ta * ta + tb * tb);",
                     "cplx disc = (ta * tb) * (ta * tb) - 4.0 * (ta * ta);"),
    "other_root": ("if (cimag(s) < 0 || (cimag(s) == 0 && creal(s) < 0)) s = -s;",
                   "if (cimag(s) > 0 || (cimag(s) == 0 && creal(s) > 0)) s = -s;"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    mutant = tmp_path / "kl_oracle.c"
    mutant.write_text(src.replace(old, new))
    (tmp_path / "kl_oracle.h").write_text(open(os.path.join(ROOT, "oracle", "kl_oracle.h")).read())
    lib = tmp_path / "liboracle_mutant.so"
    subprocess.run(["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-o", str(lib), str(mutant),
                    "-lm", "-lpthread"], check=True)
    env = dict(os.environ, KL_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"planted mistake {name} passed every pin:\n{r.stdout[-2000:]}"
