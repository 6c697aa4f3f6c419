"""Planted mistakes in a copy of the CPU reference must fail the pins.

Each case edits one plausible mistake into a temporary copy of
``oracle/kl_oracle.c`` (a transposed operand, the product read left to
right, a wrong sign in the trace recipe, the repelling seed, the wrong
seed letter, a wrong skip in the unranking, swapped bin axes, a dropped
term, the other root of the trace quadratic, a sign in Maskit's
generators, the repelling point of an affine map as its seed, the wrong
generator's seed fed to every word, a seed at infinity treated as finite,
a transposed good-set update, the wrong start state of the empty walk and
a scan that reads words left to right in the Cayley-table path; in the
random walks a Philox multiplier, the key schedule, swapped product
halves, the stream's half order, a skip of the letter itself instead of
its inverse, inverse maps, and the seed of the wrong letter; Cayley counts
that wrap past 2^64, and a recipe that refuses a seed at infinity),
builds it with gcc, and runs the pin tests against the planted build in a
child process.  The pins pass
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
    "repelling_seed": ("*u = (km > kp) ? zm : zp;", "*u = (km < kp) ? zm : zp;"),
    "first_letter_seed": ("int s = seed < 0 ? w[d - 1] : seed;", "int s = seed < 0 ? w[0] : seed;"),
    "unrank_skip": ("if (prev >= 0 && c == INVERSE[prev]) continue;",
                    "if (prev >= 0 && c == prev) continue;"),
    "bin_axes_swapped": ("*bin = row * w->width + col;", "*bin = col * w->width + row;"),
    "dropped_term": ("cplx disc = (ta * tb) * (ta * tb) - 4.0 * (ta * ta + tb * tb);",
                     "cplx disc = (ta * tb) * (ta * tb) - 4.0 * (ta * ta);"),
    "other_root": ("if (cimag(s) < 0 || (cimag(s) == 0 && creal(s) < 0)) s = -s;",
                   "if (cimag(s) > 0 || (cimag(s) == 0 && creal(s) > 0)) s = -s;"),
    "maskit_sign": ("mat2 a = {-I * mu, -I, -I, 0};", "mat2 a = {I * mu, -I, -I, 0};"),
    "affine_repelling_seed": ("if (cabs(m.a / m.d) < 1) {", "if (cabs(m.a / m.d) > 1) {"),
    "wrong_seed_generator": ("int s = seed < 0 ? w[d - 1] : seed;", "int s = seed < 0 ? w[d - 1] : (seed + 1) % 4;"),
    "infinite_seed_as_finite": ("return point_of(m.a * u + m.b * v, m.c * u + m.d * v);",
                                "return point_of(m.a * u + m.b, m.c * u + m.d);"),
    "cayley_good_set_transposed": ("if (t != 0 && ((good >> t) & 1u)) g |= 1u << s;",
                                   "if (t != 0 && ((good >> s) & 1u)) g |= 1u << t;"),
    "cayley_empty_walk_state": ("c->C[0][0] = 1;", "c->C[0][1] = 1;"),
    "cayley_scan_left_to_right": ("for (int j = depth - 1; j >= 0 && ok; j--) {",
                                  "for (int j = 0; j < depth && ok; j++) {"),
    "philox_multiplier": ("PHILOX_M0 = 0xD2E7470EE14C6C93ull", "PHILOX_M0 = 0xD2E7470EE14C6C95ull"),
    "philox_key_bump_late": ("if (round > 0) {", "if (round > 1) {"),
    "philox_halves_swapped": ("uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;",
                              "uint64_t y0 = lo1 ^ x1 ^ k0, y1 = hi1, y2 = lo0 ^ x3 ^ k1, y3 = hi0;"),
    "walk_value_halves": ("return (uint32_t)((n % 2) ? (w >> 32) : w);", "return (uint32_t)((n % 2) ? w : (w >> 32));"),
    "walk_skips_the_letter_itself": ("int skip = INVERSE[letters[k - 1]];", "int skip = letters[k - 1];"),
    "walk_applies_inverses": ("cplx z = mobius_h(g->g[c[k]], u, v);", "cplx z = mobius_h(g->g[INVERSE[c[k]]], u, v);"),
    "walk_seed_of_second_letter": ("cplx u = g->fu[c[0]], v = g->fv[c[0]];", "cplx u = g->fu[c[1]], v = g->fv[c[1]];"),
    "cayley_total_wraps": ("if (total > UINT64_MAX - c->C[L][s]) return -1;", "(void)0;"),
    "recipe_rejects_seed_at_infinity": ("translation */\n        if (attracting_fixed_point(m, &g->fu[k], &g->fv[k]) != 0) return -2;",
                                        "translation */\n        if (attracting_fixed_point(m, &g->fu[k], &g->fv[k]) != 0) return -2;"
                                        "\n        if (g->fv[k] == 0) return -2;"),
}
PINS = [os.path.join(ROOT, "tests", f) for f in ("test_oracle_pins.py", "test_oracle_groups.py",
                                                  "test_oracle_cayley.py", "test_oracle_walk.py")]


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
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"] + PINS,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"planted mistake {name} passed every pin:\n{r.stdout[-2000:]}"
