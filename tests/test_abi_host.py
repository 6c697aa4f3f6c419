"""Host-side checks of the C ABI (no GPU needed).

Every call here either needs no device at all (recipe, plans, counts) or is
rejected by argument validation before anything touches the device, so the
fake device addresses passed below are never dereferenced.
"""
import ctypes
import subprocess

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1709_08018_amd import kl
from paper_1709_08018_amd import workloads as wl

FAKE = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails validation first
L = kl.lib()

# A call that unexpectedly passed validation would reach the device with a
# fake address; where a device exists these host checks are not run.
pytestmark = pytest.mark.skipif(torch.cuda.is_available(),
                                reason="host-only checks with fake device addresses")


def test_library_exports_every_declared_symbol():
    declared = kl.declared_symbols()
    assert len(declared) >= 14
    out = subprocess.run(["nm", "-D", "--defined-only", kl.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    assert set(declared) <= exported, set(declared) - exported
    for name in declared:
        assert hasattr(L, name)


def test_num_words_matches_reference():
    for d in range(0, 42):
        assert kl.num_words(d) == O.num_words(d)


def _param_sets():
    ta, tb, _ = wl.draw_param_sets(32, seed=3)
    return [(wl.C1_TA, wl.C1_TB), (wl.C2_TA, wl.C2_TB)] + list(zip(ta, tb))


@pytest.mark.parametrize("ta,tb", _param_sets())
def test_generators_agree_with_reference(ta, tb):
    tab, g, fix = kl.generators(ta, tb)
    tab_r, g_r, fix_r = O.generators(complex(ta), complex(tb))
    assert abs(tab - tab_r) <= 1e-14 * max(1, abs(tab_r))
    np.testing.assert_allclose(g, g_r, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(fix, fix_r, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_plans_cover_every_depth(precision):
    for d in range(1, 41):
        p = kl.plan(d, precision)
        assert p["prefix_len"] + p["lane_len"] + p["tail_len"] == d
        assert 1 <= p["tail_len"] <= 8
        assert p["prefix_len"] <= 14 and p["lane_len"] <= 20
        if p["tail_len"] < d:
            assert p["prefix_len"] >= 1


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_default_tail_by_depth_and_context(precision):
    """A render of one depth takes 4-letter tails at depths 13-14 and 5-letter
    ones at 15-16 (enough heads for the persistent kernel), 6 letters from
    depth 17 on; a set of a batched render keeps 6 letters from depth 7 on."""
    w = (-2.0, 2.0, -2.0, 2.0, 512, 512)
    single = {d: kl.plan(d, precision)["tail_len"] for d in range(7, 23)}
    batch = {d: kl.plan_many(d, precision, w)["tail_len"] for d in range(7, 23)}
    assert [single[d] for d in range(12, 19)] == [6, 4, 4, 5, 5, 6, 6]
    assert all(single[d] == 6 for d in range(17, 23)) and all(single[d] == 6 for d in range(7, 13))
    assert all(batch[d] == 6 for d in range(7, 23))


def test_plan_overrides_and_rejects():
    p = kl.plan(18, "fp32", tail_len=6, lane_len=4)
    assert (p["tail_len"], p["lane_len"], p["prefix_len"]) == (6, 4, 8)
    for bad in [dict(tail_len=9), dict(tail_len=19), dict(lane_len=21), dict(tail_len=5, lane_len=13),
                dict(waves_per_cu=33), dict(hist_mode=7), dict(head_form=3), dict(head_form=-1)]:
        with pytest.raises(kl.KLError) as e:
            kl.plan(18, "fp32", **bad)
        assert e.value.code == kl.KL_EINVAL
    with pytest.raises(kl.KLError):
        kl.plan(0, "fp32")
    with pytest.raises(kl.KLError):
        kl.plan(41, "fp32")


def test_fp64_tail_length_limited_by_lds():
    # the FP64 homogeneous suffix table of r = 8 (280 KB) does not fit a CU's LDS
    assert kl.plan(18, "fp32", tail_len=8)["tail_len"] == 8
    assert kl.plan(18, "fp64", tail_len=7)["tail_len"] == 7
    with pytest.raises(kl.KLError) as e:
        kl.plan(18, "fp64", tail_len=8)
    assert e.value.code == kl.KL_EINVAL and "FP64" in str(e.value)
    o = kl.make_opts(precision="fp64", tail_len=8, use_stream=False)
    assert _render(window=_win(), opts=o) == kl.KL_EINVAL


_CACHE_PROBE = """
import sys
sys.path.insert(0, {root!r})
from paper_1709_08018_amd import kl
print(kl.plan(30, "fp32")["tail_len"], kl.plan(18, "fp32")["tail_len"], kl.plan(18, "fp32")["lane_len"],
      kl.plan(20, "fp64")["tail_len"])
"""


def test_autotune_cache_skips_lines_the_planner_rejects(tmp_path):
    import os
    import sys
    # depth 30 with r = 3, m = 1 leaves a 26-letter prefix table (> 14);
    # r = 8 is beyond FP64's limit; the depth-18 line for any device is valid
    # and applies; a line of the old format and one for another architecture
    # do not
    cache = tmp_path / "tune.txt"
    cache.write_text("* 0 30 0 0 0 3 1 0 0 1.0\n* 0 20 1 0 0 8 2 0 1 1.0\n* 0 18 0 0 0 5 2 16 1 0.2\n"
                     "garbage\n18 0 5 2 16 1 0.2\ngfx000 0 18 0 0 0 4 2 16 1 0.1\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", _CACHE_PROBE.format(root=root)], capture_output=True, text=True,
                         env={**os.environ, "KL_AUTOTUNE_CACHE": str(cache)}, check=True).stdout.split()
    default30 = kl.plan(30, "fp32")["tail_len"]
    default20 = kl.plan(20, "fp64")["tail_len"]
    assert out == [str(default30), "5", "2", str(default20)]


_BATCH_PROBE = """
import sys
sys.path.insert(0, {root!r})
from paper_1709_08018_amd import kl
w = (-2.0, 2.0, -2.0, 2.0, 320, 200)
a, b = kl.plan_many(16, "fp32", w), kl.plan(16, "fp32")
c = kl.plan_many(16, "fp32", (-2.0, 2.0, -2.0, 2.0, 512, 512))
print(a["tail_len"], a["lane_len"], a["waves_per_cu"], b["tail_len"], b["lane_len"], c["tail_len"], c["lane_len"])
"""


def test_batch_plans_are_keyed_by_image_size_and_separate_from_single_plans(tmp_path):
    import os
    import sys
    cache = tmp_path / "tune.txt"
    cache.write_text("* 1 16 0 320 200 5 3 24 1 3.0\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", _BATCH_PROBE.format(root=root)], capture_output=True, text=True,
                         env={**os.environ, "KL_AUTOTUNE_CACHE": str(cache)}, check=True).stdout.split()
    single = kl.plan(16, "fp32")
    default_batch = kl.plan_many(16, "fp32", (-2.0, 2.0, -2.0, 2.0, 512, 512))
    assert out == ["5", "3", "24", str(single["tail_len"]), str(single["lane_len"]),
                   str(default_batch["tail_len"]), str(default_batch["lane_len"])]


def test_binding_checks_tensors_before_the_call():
    w = (-1.0, 1.0, -1.0, 1.0, 8, 8)
    with pytest.raises(kl.KLError, match="dtype"):
        kl.render(wl.C2_TA, wl.C2_TB, 3, w, image=torch.zeros((8, 8), dtype=torch.float32))
    with pytest.raises(kl.KLError, match="elements"):
        kl.render(wl.C2_TA, wl.C2_TB, 3, w, image=torch.zeros((4, 8), dtype=torch.int32))
    with pytest.raises(kl.KLError, match="contiguous"):
        kl.render(wl.C2_TA, wl.C2_TB, 3, w, image=torch.zeros((8, 16), dtype=torch.int32)[:, ::2])
    with pytest.raises(kl.KLError, match="HIP device"):
        kl.render(wl.C2_TA, wl.C2_TB, 3, w, image=torch.zeros((8, 8), dtype=torch.int32))
    # render_many writes one dropped counter per set
    with pytest.raises(kl.KLError, match="elements"):
        kl.make_opts(dropped=torch.zeros(1, dtype=torch.int64), n_dropped=3)
    with pytest.raises(kl.KLError, match="dtype"):
        kl.make_opts(dropped=torch.zeros(3, dtype=torch.int32), n_dropped=3)
    with pytest.raises(kl.KLError, match="elements"):
        kl.render_many([2.0, 2.0], [2.0, 2.0], [3, 3], w, images=torch.zeros((1, 8, 8), dtype=torch.int32))
    with pytest.raises(kl.KLError, match="elements"):
        kl.decode(0, 10, 5, out=torch.zeros((10, 4), dtype=torch.uint8))
    with pytest.raises(kl.KLError, match="dtype"):
        kl.decode(0, 10, 5, out=torch.zeros((10, 5), dtype=torch.int8))
    with pytest.raises(kl.KLError, match="elements"):
        kl.gemm_bf16(4, 4, 4, torch.zeros(15), 4, 1, torch.zeros(16), 4, 1, torch.zeros(16), 4)
    with pytest.raises(kl.KLError, match="dtype"):
        kl.sur_adam(torch.zeros(kl.sur_num_params(), dtype=torch.float64), None, None, None, 1, 1e-3)


def _win(x0=-1.5, x1=1.5, y0=-1.5, y1=1.5, w=64, h=64):
    return kl.Window(x0, x1, y0, y1, w, h)


def _render(ta=wl.C2_TA, tb=wl.C2_TB, depth=10, window=None, image=FAKE, opts=None):
    w = ctypes.byref(window) if window is not None else None
    o = ctypes.byref(opts) if opts is not None else None
    return L.kl_render_ex(kl._c(ta), kl._c(tb), depth, w, image, o)


def test_render_argument_errors():
    good = _win()
    assert _render(depth=0, window=good) == kl.KL_EINVAL
    assert _render(depth=41, window=good) == kl.KL_EINVAL
    assert _render(window=None) == kl.KL_EINVAL
    assert _render(window=good, image=None) == kl.KL_EINVAL
    for w in [_win(x1=-1.5), _win(y1=-2.0), _win(w=0), _win(h=0), _win(w=40000), _win(h=32769),
              _win(x0=float("nan")), _win(y1=float("inf"))]:
        assert _render(window=w) == kl.KL_EINVAL
    o = kl.make_opts(precision=2, use_stream=False)
    assert _render(window=good, opts=o) == kl.KL_EINVAL
    o = kl.make_opts(min_depth=11, use_stream=False)
    assert _render(window=good, opts=o) == kl.KL_EINVAL
    n = kl.num_words(10)
    o = kl.make_opts(first=n - 5, count=6, use_stream=False)
    assert _render(window=good, opts=o) == kl.KL_ERANGE
    o = kl.make_opts(first=2 ** 64 - 1, count=2, use_stream=False)
    assert _render(window=good, opts=o) == kl.KL_ERANGE
    # tiling index space: depths 3..10
    total = sum(kl.num_words(d) for d in range(3, 11))
    o = kl.make_opts(min_depth=3, first=total, count=1, use_stream=False)
    assert _render(window=good, opts=o) == kl.KL_ERANGE
    assert "exceeds" in L.kl_last_error().decode()


def test_render_singular_and_nonfinite_traces():
    good = _win()
    assert _render(ta=0, tb=0, window=good) == kl.KL_ESINGULAR
    assert _render(ta=complex(float("nan"), 0), window=good) == kl.KL_EINVAL


def test_double_cusp_generators_keep_seeds_at_infinity():
    """ta = tb = 2: the recipe's a is the translation z + 2i (c = 0), whose
    seed, like A's, is infinity, reported as (HUGE_VAL, 0); b is parabolic at
    -i.  The same traces with a tiny offset give finite seeds again."""
    tab, g, fix = kl.generators(2 + 0j, 2 + 0j)
    assert tab == 2 + 2j
    np.testing.assert_array_equal(g[0], [[1, 2j], [0, 1]])
    assert np.isinf(fix[0].real) and fix[0].imag == 0 and np.isinf(fix[2].real)
    assert fix[1] == -1j and fix[3] == -1j
    _, _, fix2 = kl.generators(2 + 0j, 2.001 + 0j)
    assert np.isfinite(fix2).all()


def test_decode_and_eval_argument_errors():
    assert L.kl_decode(0, 1, 0, FAKE) == kl.KL_EINVAL
    assert L.kl_decode(0, 1, 41, FAKE) == kl.KL_EINVAL
    assert L.kl_decode(0, 5, 3, None) == kl.KL_EINVAL
    assert L.kl_decode(0, 0, 3, None) == kl.KL_OK          # empty request touches nothing
    assert L.kl_decode(kl.num_words(3), 1, 3, FAKE) == kl.KL_ERANGE
    assert L.kl_decode(2 ** 64 - 1, 2, 3, FAKE) == kl.KL_ERANGE
    assert L.kl_eval(kl._c(wl.C2_TA), kl._c(wl.C2_TB), 0, FAKE, 1, 0, FAKE) == kl.KL_EINVAL
    assert L.kl_eval(kl._c(wl.C2_TA), kl._c(wl.C2_TB), 5, None, 1, 0, FAKE) == kl.KL_EINVAL
    assert L.kl_eval(kl._c(wl.C2_TA), kl._c(wl.C2_TB), 5, FAKE, 1, 3, FAKE) == kl.KL_EINVAL
    assert L.kl_eval(kl._c(0), kl._c(0), 5, FAKE, 1, 0, FAKE) == kl.KL_ESINGULAR


def test_render_many_argument_errors():
    n = 3
    ta = (kl.c64 * n)(*[kl._c(wl.C2_TA)] * n)
    tb = (kl.c64 * n)(*[kl._c(wl.C2_TB)] * n)
    good = (ctypes.c_int * n)(10, 11, 12)
    w = _win()
    assert L.kl_render_many(0, ta, tb, good, ctypes.byref(w), FAKE) == kl.KL_EINVAL
    assert L.kl_render_many(n, None, tb, good, ctypes.byref(w), FAKE) == kl.KL_EINVAL
    bad = (ctypes.c_int * n)(10, 0, 12)
    assert L.kl_render_many(n, ta, tb, bad, ctypes.byref(w), FAKE) == kl.KL_EINVAL
    assert "set 1" in L.kl_last_error().decode()
    tb2 = (kl.c64 * n)(kl._c(wl.C2_TB), kl._c(wl.C2_TB), kl.c64(0, 0))
    ta2 = (kl.c64 * n)(kl._c(wl.C2_TA), kl._c(wl.C2_TA), kl.c64(0, 0))
    assert L.kl_render_many(n, ta2, tb2, good, ctypes.byref(w), FAKE) == kl.KL_ESINGULAR
    assert "set 2" in L.kl_last_error().decode()
    o = kl.make_opts(min_depth=2, use_stream=False)
    assert L.kl_render_many_ex(n, ta, tb, good, ctypes.byref(w), FAKE, ctypes.byref(o)) == kl.KL_EINVAL


def test_noalloc_rejects_before_touching_the_device():
    good = _win()
    # depth 37: an 11-letter prefix table (15 MB) exceeds the scratch array
    assert L.kl_render_noalloc(kl._c(wl.C2_TA), kl._c(wl.C2_TB), 37, ctypes.byref(good), FAKE, None) == kl.KL_ENOMEM
    assert "scratch" in L.kl_last_error().decode()
    o = kl.make_opts(min_depth=3, use_stream=False)
    assert L.kl_render_noalloc(kl._c(wl.C2_TA), kl._c(wl.C2_TB), 10, ctypes.byref(good), FAKE,
                               ctypes.byref(o)) == kl.KL_EINVAL
    assert L.kl_render_noalloc(kl._c(wl.C2_TA), kl._c(wl.C2_TB), 10, ctypes.byref(good), None, None) == kl.KL_EINVAL
    assert L.kl_render_noalloc(kl._c(0), kl._c(0), 10, ctypes.byref(good), FAKE, None) == kl.KL_ESINGULAR


def test_walk_argument_errors():
    ab = (kl.c64 * 8)(*[kl.c64(1, 0), kl.c64(1, 0), kl.c64(0, 0), kl.c64(1, 0)] * 2)
    w = kl.make_walk(0, 0, 10, 0, 5)
    assert L.kl_walk_letters(None, FAKE, None) == kl.KL_EINVAL
    assert L.kl_walk_letters(ctypes.byref(w), None, None) == kl.KL_EINVAL
    assert L.kl_walk_letters(ctypes.byref(kl.make_walk(0, 2 ** 64 - 5, 10, 0, 5)), FAKE, None) == kl.KL_ERANGE
    assert L.kl_walk_letters(ctypes.byref(kl.make_walk(0, 0, 1, 2 ** 32 - 1, 2 ** 32 - 1)), FAKE, None) == kl.KL_EINVAL
    assert L.kl_walk_letters(ctypes.byref(kl.make_walk(0, 0, 0, 0, 5)), None, None) == kl.KL_OK   # nothing to do
    good = _win()
    assert L.kl_walk_render_ex(ab, ctypes.byref(w), ctypes.byref(_win(w=0)), FAKE, None) == kl.KL_EINVAL
    assert L.kl_walk_render_ex(ab, ctypes.byref(w), ctypes.byref(good), None, None) == kl.KL_EINVAL
    assert L.kl_walk_render_ex(None, ctypes.byref(w), ctypes.byref(good), FAKE, None) == kl.KL_EINVAL
    o = kl.make_opts(precision=3, use_stream=False)
    assert L.kl_walk_render_ex(ab, ctypes.byref(w), ctypes.byref(good), FAKE, ctypes.byref(o)) == kl.KL_EINVAL
    assert L.kl_walk_eval_ex(ab, ctypes.byref(w), None, None, None) == kl.KL_EINVAL
    zero = (kl.c64 * 8)(*[kl.c64(0, 0)] * 8)
    assert L.kl_walk_eval_ex(zero, ctypes.byref(w), None, FAKE, None) == kl.KL_ESINGULAR
    # the binned render (KL_HIST_LDS): images of at most 256 tiles of 2^15
    # bins, at most 2^19 drawn points a walker; refused before anything runs
    lds = kl.make_opts(hist_mode="lds", use_stream=False)
    big = _win(w=4096, h=2056)      # 257 tiles
    assert L.kl_walk_render_ex(ab, ctypes.byref(w), ctypes.byref(big), FAKE, ctypes.byref(lds)) == kl.KL_EINVAL
    long_walk = kl.make_walk(0, 0, 1, 0, 2 ** 19 + 1)
    assert L.kl_walk_render_ex(ab, ctypes.byref(long_walk), ctypes.byref(good), FAKE, ctypes.byref(lds)) == kl.KL_EINVAL


def test_strerror_names_every_code():
    for code in (0, -1, -2, -3, -4, -5):
        assert L.kl_strerror(code)
    assert L.kl_strerror(-99) == b"unknown error"


# ---------------------------------------------------------------- explicit groups and seeds
MU_FIG = complex(-0.097, 1.838)


def _same_map(m, r):
    """2x2 matrices m, r define the same Moebius map: m = c r for some c != 0."""
    k = np.argmax(np.abs(r))
    c = m.flat[k] / r.flat[k]
    return np.allclose(m, c * r, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("mu", [MU_FIG, 2j, complex(0.3, 1.95)])
def test_maskit_group_agrees_with_reference(mu):
    ab = kl.maskit_generators(mu)
    G = O.group_maskit(mu)
    assert _same_map(ab[0], G.gens[0]) and _same_map(ab[1], G.gens[1])
    gens, seeds = kl.group_seeds(ab)
    for k in range(4):
        assert _same_map(gens[k], G.gens[k])
        np.testing.assert_allclose(np.linalg.det(gens[k]), 1.0, atol=1e-13)
    pts = G.seed_points()
    for k in range(4):
        u, v = seeds[k]
        if np.isinf(pts[k]):
            assert v == 0 and u != 0
        else:
            assert abs(u / v - pts[k]) <= 1e-12 * max(1, abs(pts[k]))


@pytest.mark.parametrize("ta,tb", _param_sets()[:8])
def test_explicit_group_of_recipe_generators_agrees_with_reference(ta, tb):
    _, g, _ = kl.generators(ta, tb)
    gens, seeds = kl.group_seeds(np.stack([g[0], g[1]]))
    R = O.group_recipe(complex(ta), complex(tb))
    pts = R.seed_points()
    for k in range(4):
        assert _same_map(gens[k], R.gens[k])
        assert abs(seeds[k, 0] / seeds[k, 1] - pts[k]) <= 1e-11 * max(1, abs(pts[k]))


def test_affine_generator_seeds_agree_with_reference():
    a = np.array([[2, 1], [0, 0.5]], complex)
    b = np.array([[2, 1], [1, 1]], complex)
    _, seeds = kl.group_seeds(np.stack([a, b]))
    pts = O.group_explicit(a, b).seed_points()
    assert seeds[0, 1] == 0 and np.isinf(pts[0])
    for k in (1, 2, 3):
        assert abs(seeds[k, 0] / seeds[k, 1] - pts[k]) < 1e-14


def test_group_argument_errors():
    w = _win()
    ab = kl._ab(kl.maskit_generators(MU_FIG))
    assert L.kl_group_seeds(None, None, None) == kl.KL_EINVAL
    assert L.kl_maskit_generators(kl._c(complex(float("nan"), 0)), (kl.c64 * 8)()) == kl.KL_EINVAL
    assert L.kl_maskit_generators(kl._c(MU_FIG), None) == kl.KL_EINVAL
    singular = kl._ab(np.array([[[1, 2], [2, 4]], [[1, 2], [0, 1]]], complex))
    assert L.kl_group_seeds(singular, None, None) == kl.KL_ESINGULAR
    identity = kl._ab(np.array([[[1, 0], [0, 1]], [[1, 2], [0, 1]]], complex))
    assert L.kl_group_seeds(identity, None, None) == kl.KL_ESINGULAR
    nonfinite = kl._ab(np.array([[[np.nan, 0], [0, 1]], [[1, 2], [0, 1]]], complex))
    assert L.kl_group_seeds(nonfinite, None, None) == kl.KL_EINVAL
    o = kl.make_opts(use_stream=False)
    assert L.kl_render_group_ex(ab, 0, ctypes.byref(w), FAKE, ctypes.byref(o)) == kl.KL_EINVAL
    assert L.kl_render_group_ex(ab, 10, ctypes.byref(w), None, ctypes.byref(o)) == kl.KL_EINVAL
    assert L.kl_render_group_ex(singular, 10, ctypes.byref(w), FAKE, ctypes.byref(o)) == kl.KL_ESINGULAR
    assert L.kl_eval_group_ex(ab, 41, FAKE, 1, None, FAKE, ctypes.byref(o)) == kl.KL_EINVAL
    assert L.kl_eval_group_ex(None, 10, FAKE, 1, None, FAKE, ctypes.byref(o)) == kl.KL_EINVAL


def test_seed_mode_errors():
    w = _win()
    for bad in (-1, 6):
        o = kl.make_opts(seed=bad, use_stream=False)
        assert _render(window=w, opts=o) == kl.KL_EINVAL
    o = kl.make_opts(seed="all", use_stream=False)
    assert L.kl_eval_ex(kl._c(wl.C2_TA), kl._c(wl.C2_TB), 10, FAKE, 1, None, FAKE,
                        ctypes.byref(o)) == kl.KL_EINVAL
    assert "four values" in L.kl_last_error().decode()


# ---------------------------------------------------------------- indexed Cayley tables
def _golden_table(name):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    rows = [line.split() for line in open(path) if line.strip() and not line.startswith("#")]
    return np.array(rows, dtype=np.uint8)


MODULAR = np.array([[0, 1, 2, 3], [1, 0, 2, 3], [2, 1, 0, 0], [3, 1, 0, 0]], np.uint8)


@pytest.mark.parametrize("name", ["t11", "klein4", "modular"])
def test_cayley_counts_agree_with_reference(name):
    table = {"t11": _golden_table("cayley_t11_indexed.txt"), "klein4": _golden_table("cayley_klein4_indexed.txt"),
             "modular": MODULAR}[name]
    t = kl.Cayley(table)
    ref = O.Cayley(table, np.array([[[1, 0], [0, 1]]] * (table.shape[1] - 1), complex))
    for d in range(1, 41):
        assert kl.cayley_num_words(t, d) == O.cayley_num_words(ref, d)


def test_cayley_argument_errors():
    w = _win()
    o = kl.make_opts(use_stream=False)
    good = kl.Cayley(MODULAR, np.array([[[0, -1], [1, 0]], [[0, -1], [1, 1]], [[1, 1], [-1, 0]]], complex))
    assert L.kl_cayley_render_ex(good.ref(), 0, ctypes.byref(w), FAKE, ctypes.byref(o)) == kl.KL_EINVAL
    assert L.kl_cayley_render_ex(good.ref(), 5, ctypes.byref(w), None, ctypes.byref(o)) == kl.KL_EINVAL
    assert L.kl_cayley_render_ex(None, 5, ctypes.byref(w), FAKE, ctypes.byref(o)) == kl.KL_EINVAL
    no_maps = kl.Cayley(MODULAR)
    assert L.kl_cayley_render_ex(no_maps.ref(), 5, ctypes.byref(w), FAKE, ctypes.byref(o)) == kl.KL_EINVAL
    bad_entry = MODULAR.copy()
    bad_entry[2, 1] = 9
    assert kl.cayley_num_words(kl.Cayley(bad_entry), 5) == 0
    assert L.kl_cayley_decode_ex(kl.Cayley(bad_entry).ref(), 0, 1, 5, FAKE, None) == kl.KL_EINVAL
    singular = kl.Cayley(MODULAR, np.array([[[1, 2], [2, 4]], [[0, -1], [1, 1]], [[1, 1], [-1, 0]]], complex))
    assert L.kl_cayley_render_ex(singular.ref(), 5, ctypes.byref(w), FAKE, ctypes.byref(o)) == kl.KL_ESINGULAR
    o4 = kl.make_opts(seed="B", use_stream=False)   # symbol 4: the table has 3
    assert L.kl_cayley_render_ex(good.ref(), 5, ctypes.byref(w), FAKE, ctypes.byref(o4)) == kl.KL_EINVAL
    # a table of up to eight symbols names each one's seed as KL_SEED_A + q; past its
    # symbols, and past the eighth, it is refused
    eight = kl.Cayley(np.hstack([np.arange(2)[:, None], np.ones((2, 8))]).astype(np.uint8),
                      np.array([[[2, 0], [0, 0.5]]] * 8, complex))
    for mode in (2 + 8, 2 + 9, -1):
        om = kl.make_opts(seed=mode, use_stream=False)
        assert L.kl_cayley_render_ex(eight.ref(), 3, ctypes.byref(w), FAKE, ctypes.byref(om)) == kl.KL_EINVAL
        assert L.kl_cayley_eval_ex(eight.ref(), 3, FAKE, 1, None, FAKE, ctypes.byref(om)) == kl.KL_EINVAL
    n = kl.cayley_num_words(good, 6)
    assert L.kl_cayley_decode_ex(good.ref(), n - 1, 2, 6, FAKE, None) == kl.KL_ERANGE
    assert L.kl_cayley_decode_ex(good.ref(), 0, 0, 6, None, None) == kl.KL_OK
    # eight symbols that never crash: 8^21 = 2^63 words of length 21 ending in state 1
    free8 = np.ones((2, 9), np.uint8)
    free8[:, 0] = 0
    assert kl.cayley_num_words(kl.Cayley(free8), 20) == 8 ** 20
    assert kl.cayley_num_words(kl.Cayley(free8), 21) == 0
    # 16 states, 7 symbols, no crash: 7^L words; 7^23 passes 2^64 while every
    # state's count (at most 7^22) stays below 2^63
    seven = np.zeros((16, 8), np.uint8)
    seven[:, 0] = np.arange(16)
    for st in range(16):
        for x in range(1, 8):
            seven[st, x] = 1 + ((x - 1) + 7 * (st & 1)) % 15
    assert kl.cayley_num_words(kl.Cayley(seven), 22) == 7 ** 22
    assert kl.cayley_num_words(kl.Cayley(seven), 23) == 0
    huge = kl.Cayley(free8, np.array([[[2, 0], [0, 0.5]]] * 8, complex))
    assert L.kl_cayley_render_ex(huge.ref(), 21, ctypes.byref(w), FAKE, ctypes.byref(o)) == kl.KL_EINVAL
