"""Block bounds (kl_opts.block_bounds) through the C ABI.

With block bounds the persistent renderer bounds, per head and per group of
27 suffixes, the bins those words can reach, and evaluates word by word only
the groups whose bound spans more than one bin.  Bar: images and dropped
counts equal, bin for bin, to the per-word renderer on the same words, and to
the histogram of the renderer's own per-word coordinates (kl_eval).
"""
import ctypes

import numpy as np
import pytest
import torch

from paper_1709_08018_amd import workloads as wl

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1709_08018_amd import kl

C2 = (wl.C2_TA, wl.C2_TB)
C1 = (wl.C1_TA, wl.C1_TB)
WIN_C2 = wl.QUASIFUCHSIAN_D18.window.as_tuple()
WIN_64 = (-1.5, 1.5, -1.5, 1.5, 64, 64)
WIN_ZOOM = (0.1, 0.6, -0.2, 0.3, 40, 40)
WIN_ANISO = (-2.0, 2.0, -2.0, 2.0, 300, 100)


def _both(render):
    """(image, dropped) of render(block_bounds=b, image=..., dropped=...) for b = False, True."""
    res = []
    for b in (False, True):
        d = torch.zeros(1, dtype=torch.int64, device="cuda")
        img = render(block_bounds=b, dropped=d)
        res.append((kl.as_u32(img).astype(np.int64), int(d.item())))
    return res


def _assert_same(render):
    (a, da), (b, db) = _both(render)
    np.testing.assert_array_equal(b, a)
    assert db == da
    return a, da


def _bins_from_pixels(px, py, win):
    W, H = win[4], win[5]
    ok = (px >= 0) & (px < W) & (py >= 0) & (py < H)   # IEEE: -0 counts as 0, NaN is outside
    img = np.zeros(W * H, np.int64)
    np.add.at(img, np.floor(py[ok]).astype(np.int64) * W + np.floor(px[ok]).astype(np.int64), 1)
    return img.reshape(H, W), int((~ok).sum())


# tail_len 4 gives depths 12 and 13 enough heads for the persistent kernel,
# which alone takes block bounds
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("depth,win,tl", [(18, WIN_C2, 0), (14, WIN_C2, 0), (13, WIN_ZOOM, 4), (12, WIN_64, 4),
                                          (13, WIN_ANISO, 4)],
                         ids=["d18", "d14", "d13_zoom", "d12_64", "d13_aniso"])
def test_bounded_equals_per_word(depth, win, tl, precision):
    img, drop = _assert_same(lambda **kw: kl.render(*C2, depth, win, tail_len=tl, precision=precision, **kw))
    assert int(img.sum()) + drop == kl.num_words(depth)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_bounded_equals_per_word_on_drawn_sets(precision):
    """Eight parameter sets of the batch's law at depths 13..17 (the planner's
    4-, 5- and 6-letter tails) on a zoomed and a whole window: block bounds
    leave every image and dropped count bit for bit as the per-word render."""
    ta, tb, depth = wl.draw_param_sets(8, seed=61, depth_range=(13, 17))
    for i in range(len(ta)):
        win = WIN_ZOOM if i % 2 else (-2.0, 2.0, -2.0, 2.0, 512, 512)
        a, b, d = complex(ta[i]), complex(tb[i]), int(depth[i])
        img, drop = _assert_same(lambda **kw: kl.render(a, b, d, win, precision=precision, **kw))
        assert int(img.sum()) + drop == kl.num_words(d), (i, d)


@pytest.mark.parametrize("seed", ["b", "A", "all"])
def test_bounded_seed_modes(seed):
    _assert_same(lambda **kw: kl.render(*C2, 14, WIN_C2, seed=seed, **kw))
    _assert_same(lambda **kw: kl.render(*C2, 14, WIN_C2, seed=seed, precision="fp64", **kw))


@pytest.mark.parametrize("tail_len", [4, 5, 7, 8])
def test_bounded_tail_lengths(tail_len):
    _assert_same(lambda **kw: kl.render(*C2, 16, WIN_64, tail_len=tail_len, **kw))


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_bounded_equals_histogram_of_own_bins(precision):
    depth, win, tl = 13, WIN_64, 4
    n = kl.num_words(depth)
    dropped = torch.zeros(1, dtype=torch.int64, device="cuda")
    img = kl.as_u32(kl.render(*C2, depth, win, block_bounds=True, dropped=dropped, tail_len=tl,
                              precision=precision)).astype(np.int64)
    p = kl.eval_values(*C2, depth, np.arange(n, dtype=np.uint64), window=win, tail_len=tl,
                       precision=precision).cpu().numpy()
    ref, drop = _bins_from_pixels(p[:, 0], p[:, 1], win)
    np.testing.assert_array_equal(img, ref)
    assert int(dropped.item()) == drop


def test_bounded_ranges_and_accumulate():
    depth, win = 15, WIN_C2
    n = kl.num_words(depth)
    cuts = sorted({0, 1, 12345, n // 3, n // 3 + 777, n - 5, n})

    def render(block_bounds, dropped):
        img = kl.new_image(win)
        for a, b in zip(cuts[:-1], cuts[1:]):
            kl.render(*C2, depth, win, image=img, first=a, count=b - a, accumulate=True, dropped=dropped,
                      block_bounds=block_bounds)
        return img
    _assert_same(render)


def test_bounded_group_with_heads_of_both_forms():
    """Maskit's group: b is a translation, so heads without a pole form occur
    and their units take the per-word walk."""
    ab = kl.maskit_generators(wl.MASKIT_MU)
    win = wl.MASKIT_D14.window.as_tuple()
    _assert_same(lambda **kw: kl.render_group(ab, 13, win, tail_len=4, **kw))
    _assert_same(lambda **kw: kl.render(*C1, 14, wl.FUCHSIAN_TILING_D10.window.as_tuple(), **kw))


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_bounded_batched_and_tiling_renders(precision):
    """The batched renderer takes block bounds for its persistent sets:
    kl_render_many and whole tiling renders equal their per-word images."""
    ta, tb, _ = wl.draw_param_sets(6, seed=11)
    depths = [14, 15, 16, 14, 13, 17]
    win = (-2.0, 2.0, -2.0, 2.0, 128, 128)
    a = kl.render_many(ta, tb, depths, win, precision=precision)
    b = kl.render_many(ta, tb, depths, win, precision=precision, block_bounds=True)
    assert torch.equal(a, b)
    # with dropped counters (the kernels that count them)
    da = torch.zeros(len(ta), dtype=torch.int64, device="cuda")
    db = torch.zeros(len(ta), dtype=torch.int64, device="cuda")
    a = kl.render_many(ta, tb, depths, win, precision=precision, dropped=da)
    b = kl.render_many(ta, tb, depths, win, precision=precision, dropped=db, block_bounds=True)
    assert torch.equal(a, b) and torch.equal(da, db)
    for i, d in enumerate(depths):
        assert int(kl.as_u32(b[i]).astype(np.int64).sum()) + int(db[i].item()) == kl.num_words(d)
    _assert_same(lambda **kw: kl.render(*C2, 15, WIN_C2, min_depth=1, precision=precision, **kw))
    _assert_same(lambda **kw: kl.render(*C2, 14, WIN_C2, min_depth=1, seed="all", precision=precision, **kw))


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_bounded_double_cusp(precision):
    """ta = tb = 2: the recipe's a is a translation seeded at infinity, so
    the suffix tables are homogeneous and heads that are powers of a have no
    pole form; block bounds leave those to the per-word walk, single and
    batched, and the images stay those of the per-word renderer."""
    win = (-1.25, 1.25, -4.0, 4.0, 320, 1024)
    _assert_same(lambda **kw: kl.render(2 + 0j, 2 + 0j, 16, win, precision=precision, **kw))
    _assert_same(lambda **kw: kl.render(2 + 0j, 2 + 0j, 13, win, precision=precision, seed="b", **kw))
    ta = np.array([2, wl.C2_TA, 2], complex)
    tb = np.array([2, wl.C2_TB, 2], complex)
    a = kl.render_many(ta, tb, [16, 15, 14], win, precision=precision)
    b = kl.render_many(ta, tb, [16, 15, 14], win, precision=precision, block_bounds=True)
    assert torch.equal(a, b)


def test_bounded_ignored_where_it_does_not_apply():
    # the LDS tile histogram, a small tiling render (per-word kernel), and non-finite FP32 coordinates
    _assert_same(lambda **kw: kl.render(*C2, 14, WIN_C2, hist_mode="lds", **kw))
    _assert_same(lambda **kw: kl.render(*C1, 10, wl.FUCHSIAN_TILING_D10.window.as_tuple(), min_depth=1, **kw))
    _assert_same(lambda **kw: kl.render(*C2, 12, (0.0, 1e-37, 0.0, 1e-37, 64, 64), **kw))


def test_block_bounds_value_is_checked():
    with pytest.raises(kl.KLError):
        o = kl.make_opts()
        o.block_bounds = 2
        img = kl.new_image(WIN_64)
        w = kl.make_window(WIN_64)
        kl._check(kl.lib().kl_render_ex(kl._c(C2[0]), kl._c(C2[1]), 10, ctypes.byref(w), img.data_ptr(),
                                        ctypes.byref(o)))


# The per-word renderer (block bounds off) on windows where nearly every head
# lies wholly outside, and one where most are inside: lanes whose words stay
# outside keep changing their run keys without adding to the image.  Images
# and dropped counts against the words' own coordinates, in both precisions.
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("win", [(0.1, 0.6, -0.2, 0.3, 40, 40), (0.9, 0.95, 0.3, 0.35, 64, 48),
                                 (-4.0, 4.0, -4.0, 4.0, 128, 128)], ids=["zoom", "tiny", "wide"])
def test_outside_heads_keep_images_and_dropped_counts(precision, win):
    depth = 13
    n = kl.num_words(depth)
    d = torch.zeros(1, dtype=torch.int64, device="cuda")
    img = kl.as_u32(kl.render(*C2, depth, win, precision=precision, dropped=d, tail_len=4)).astype(np.int64)
    p = kl.eval_values(*C2, depth, torch.arange(n, dtype=torch.int64, device="cuda"), precision=precision,
                       window=win, tail_len=4).cpu().numpy()
    ref, drop = _bins_from_pixels(p[:, 0], p[:, 1], win)
    np.testing.assert_array_equal(img, ref)
    assert int(d.item()) == drop
    assert int(img.sum()) + drop == n
