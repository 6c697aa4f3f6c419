"""Random walks (the probabilistic approach of Section 4) on the GPU against
the oracle, through the C ABI.

Bars: letters bit-exact; FP64 points within 1e-10 of max(1, |z|) (and
truly relative above 1e-6); FP32 points within 0.25 px; every image equal
to the histogram of its own points' pixel coordinates, and the FP64 image
equal to the oracle's up to points within 1e-7 px of a bin edge.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1709_08018_amd import workloads as wl

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1709_08018_amd import kl

MU = wl.MASKIT_MU
WIN_M = wl.MASKIT_D14.window.as_tuple()
WIN_C2 = (-2.0, 2.0, -2.0, 2.0, 512, 512)


def _maskit():
    ab = kl.maskit_generators(MU)
    return ab, O.group_maskit(MU)


def _recipe():
    _, g, _ = kl.generators(wl.C2_TA, wl.C2_TB)
    return np.stack([g[0], g[1]]), O.group_recipe(wl.C2_TA, wl.C2_TB)


def _dcusp():
    """ta = tb = 2: a is the translation z + 2i, its seed (and A's) infinity."""
    _, g, _ = kl.generators(2 + 0j, 2 + 0j)
    return np.stack([g[0], g[1]]), O.group_recipe(2 + 0j, 2 + 0j)


def _group(name):
    return {"recipe": _recipe, "maskit": _maskit, "dcusp": _dcusp}[name]()


def _z(t):
    a = t.cpu().numpy()
    return a[..., 0] + 1j * a[..., 1]


@pytest.mark.parametrize("seed,first,n,burn,steps", [
    (0, 0, 1000, 0, 99), (12345, 7, 333, 5, 17), (2 ** 64 - 1, 2 ** 64 - 300, 300, 0, 40), (3, 2 ** 40, 64, 0, 1),
])
def test_letters_bit_exact(seed, first, n, burn, steps):
    got = kl.walk_letters(seed, first, n, burn, steps).cpu().numpy()
    for i in list(range(min(n, 50))) + [n - 1]:
        np.testing.assert_array_equal(got[i], O.walk_letters(seed, first + i, 1 + burn + steps), err_msg=str(i))


def test_drawn_walks_letters_and_binned_renders():
    """Ten walk configurations drawn over 64-bit seeds and walker indices,
    burn-ins and step counts: sampled walkers' letters bit for bit the
    oracle's, and the binned render equal to the one-atomic-per-point render
    (image and dropped count) in both precisions."""
    ab, _ = _maskit()
    for i, (seed, first, n, burn, steps) in enumerate(wl.draw_walks(10, seed=81)):
        got = kl.walk_letters(seed, first, n, burn, steps).cpu().numpy()
        for k in sorted({0, n // 2, n - 1}):
            np.testing.assert_array_equal(got[k], O.walk_letters(seed, first + k, 1 + burn + steps),
                                          err_msg=f"{i} walker {k}")
        for precision in ("fp32", "fp64"):
            (a, da), (b, db) = _render_both(ab, seed, first, n, burn, steps, WIN_M, precision)
            np.testing.assert_array_equal(a, b, err_msg=f"{i} {precision}")
            assert da == db and int(a.sum()) + da == n * steps, (i, precision)


def _assert_fp64(z, zr, what):
    fin = np.isfinite(zr)
    assert np.all(~np.isfinite(z[~fin])), what
    assert np.isfinite(z[fin]).all(), what
    dz, a = np.abs(z[fin] - zr[fin]), np.abs(zr[fin])
    assert (dz / np.maximum(1, a)).max() < 1e-10, what
    big = a > 1e-6
    assert (dz[big] / a[big]).max() < 1e-10, what


@pytest.mark.parametrize("group", ["recipe", "maskit", "dcusp"])
@pytest.mark.parametrize("burn,steps", [(0, 40), (7, 600)])
def test_fp64_points_match_the_oracle(group, burn, steps):
    ab, g = _group(group)
    seed, first, n = 99, 1000, 300
    z = _z(kl.walk_eval(ab, seed, first, n, burn, steps, precision="fp64"))
    zr = O.walk_points(g, seed, first, n, burn, steps)
    _assert_fp64(z, zr, (group, burn, steps))


def test_fp32_pixel_error():
    ab, g = _maskit()
    seed, n, steps = 5, 4096, 64
    p = kl.walk_eval(ab, seed, 0, n, 0, steps, window=WIN_M, precision="fp32").cpu().numpy().reshape(-1, 2)
    z = O.walk_points(g, seed, 0, n, 0, steps).ravel()
    x0, x1, y0, y1, W, H = WIN_M
    with np.errstate(invalid="ignore"):
        fx, fy = (z.real - x0) * W / (x1 - x0), (z.imag - y0) * H / (y1 - y0)
        near = np.isfinite(z) & (fx > -1) & (fx < W + 1) & (fy > -1) & (fy < H + 1)
    err = np.hypot(p[near, 0] - fx[near], p[near, 1] - fy[near])
    print(f"walk FP32 pixel error over {near.sum()} points near the window: max {err.max():.3e} "
          f"p99 {np.quantile(err, 0.99):.3e} mean {err.mean():.3e}")
    assert near.sum() > 100_000
    assert err.max() <= 0.25


def _own_bins(p, win):
    W, H = win[4], win[5]
    px, py = p[..., 0].ravel(), p[..., 1].ravel()
    with np.errstate(invalid="ignore"):
        ok = (px >= 0) & (px < W) & (py >= 0) & (py < H)
    img = np.zeros(W * H, np.int64)
    np.add.at(img, np.floor(py[ok]).astype(np.int64) * W + np.floor(px[ok]).astype(np.int64), 1)
    return img.reshape(H, W), int((~ok).sum())


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("group", ["recipe", "maskit"])
def test_image_is_histogram_of_own_points(precision, group):
    ab, _ = _recipe() if group == "recipe" else _maskit()
    win = WIN_C2 if group == "recipe" else WIN_M
    seed, n, burn, steps = 8, 3001, 2, 77
    dropped = torch.zeros(1, dtype=torch.int64, device="cuda")
    img = kl.as_u32(kl.walk_render(ab, seed, 0, n, burn, steps, win, precision=precision,
                                   dropped=dropped)).astype(np.int64)
    p = kl.walk_eval(ab, seed, 0, n, burn, steps, window=win, precision=precision).cpu().numpy()
    ref, drop = _own_bins(p, win)
    np.testing.assert_array_equal(img, ref)
    assert int(dropped.item()) == drop
    assert int(img.sum()) + drop == n * steps


@pytest.mark.parametrize("group", ["recipe", "maskit", "dcusp"])
def test_fp64_image_matches_the_oracle(group):
    ab, g = _group(group)
    win = {"recipe": WIN_C2, "maskit": WIN_M, "dcusp": (-1.25, 1.25, -4.0, 4.0, 320, 1024)}[group]
    seed, n, burn, steps = 21, 2000, 3, 128
    img = kl.as_u32(kl.walk_render(ab, seed, 0, n, burn, steps, win, precision="fp64")).astype(np.int64)
    ref, _, near = O.walk_render(g, seed, 0, n, burn, steps, win, edge_tol=1e-7)
    diff = int(np.abs(img - ref.astype(np.int64)).sum())
    assert diff <= 2 * near, (diff, near)


@pytest.mark.parametrize("hist_mode", ["runs", "lds"])
def test_walker_counts_past_one_launch(hist_mode):
    """2^30 + 3,000 walkers of one drawn step each: more than one launch
    takes (2^30 walkers; the binned path stages 2^27 points a pass).  Three
    checks:
      * rendered at once, they equal the same walkers rendered in three
        uneven pieces;
      * every point is counted (image + dropped);
      * the two histogram modes agree."""
    ab, _ = _maskit()
    n = (1 << 30) + 3000
    d_all = torch.zeros(1, dtype=torch.int64, device="cuda")
    full = kl.walk_render(ab, 17, 5, n, 0, 1, WIN_M, hist_mode=hist_mode, dropped=d_all)
    assert int(kl.as_u32(full).astype(np.int64).sum()) + int(d_all.item()) == n
    acc = kl.new_image(WIN_M)
    d_acc = torch.zeros(1, dtype=torch.int64, device="cuda")
    for a, b in [(0, (1 << 29) + 7), ((1 << 29) + 7, (1 << 30) + 11), ((1 << 30) + 11, n)]:
        kl.walk_render(ab, 17, 5 + a, b - a, 0, 1, WIN_M, image=acc, accumulate=True, hist_mode=hist_mode,
                       dropped=d_acc)
    assert torch.equal(acc, full)
    assert int(d_acc.item()) == int(d_all.item())
    other = kl.walk_render(ab, 17, 5, n, 0, 1, WIN_M, hist_mode="lds" if hist_mode == "runs" else "runs")
    assert torch.equal(other, full)


def test_walker_ranges_accumulate_and_edge_cases():
    ab, _ = _maskit()
    n, steps = 1000, 50
    full = kl.walk_render(ab, 4, 0, n, 0, steps, WIN_M)
    acc = kl.new_image(WIN_M)
    for a, b in [(0, 1), (1, 257), (257, 999), (999, 1000)]:
        kl.walk_render(ab, 4, a, b - a, 0, steps, WIN_M, image=acc, accumulate=True)
    assert torch.equal(acc, full)
    # no walkers, no drawn points: an empty image
    empty = kl.walk_render(ab, 4, 0, 0, 0, steps, WIN_M)
    assert int(empty.abs().sum()) == 0
    assert int(kl.walk_render(ab, 4, 0, 10, 5, 0, WIN_M).abs().sum()) == 0
    assert kl.walk_eval(ab, 4, 0, 10, 5, 0).numel() == 0
    with pytest.raises(kl.KLError) as e:
        kl.walk_render(ab, 4, 2 ** 64 - 5, 10, 0, steps, WIN_M)
    assert e.value.code == kl.KL_ERANGE


def _render_both(ab, seed, first, n, burn, steps, win, precision, accumulate_into=None):
    """(image, dropped) of the binned path and of the one-atomic-per-point path."""
    out = []
    for mode in ("lds", "runs"):
        dropped = torch.zeros(1, dtype=torch.int64, device="cuda")
        img = kl.walk_render(ab, seed, first, n, burn, steps, win, precision=precision, dropped=dropped,
                             hist_mode=mode)
        out.append((kl.as_u32(img).astype(np.int64), int(dropped.item())))
    return out


# Binned render (points sorted by image tile of 2^15 bins in LDS, counted
# tile by tile) against the direct one: ragged walker blocks, walks whose
# drawn steps are not a multiple of the 8-step chunk, burn-in, one tile and
# many, both precisions.
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("n,burn,steps,win", [
    (1, 0, 1, WIN_M), (255, 3, 17, WIN_M), (256, 0, 16, WIN_M), (4097, 5, 64, WIN_M),
    (3000, 0, 33, (-1.05, 1.05, -0.1, 2.0, 100, 100)), (513, 2, 40, (-1.05, 1.05, -0.1, 2.0, 182, 181)),
    (20000, 0, 100, WIN_M),
], ids=["one", "ragged", "block", "tiles", "one_tile", "edge_tile", "long"])
def test_binned_render_equals_direct(precision, n, burn, steps, win):
    ab, _ = _maskit()
    (a, da), (b, db) = _render_both(ab, 7, 11, n, burn, steps, win, precision)
    np.testing.assert_array_equal(a, b)
    assert da == db
    assert int(a.sum()) + da == n * steps


def test_binned_render_matches_own_points_and_accumulates():
    ab, _ = _recipe()
    seed, n, burn, steps = 8, 5001, 2, 77
    dropped = torch.zeros(1, dtype=torch.int64, device="cuda")
    img = kl.as_u32(kl.walk_render(ab, seed, 0, n, burn, steps, WIN_C2, dropped=dropped,
                                   hist_mode="lds")).astype(np.int64)
    p = kl.walk_eval(ab, seed, 0, n, burn, steps, window=WIN_C2).cpu().numpy()
    ref, drop = _own_bins(p, WIN_C2)
    np.testing.assert_array_equal(img, ref)
    assert int(dropped.item()) == drop
    acc = kl.new_image(WIN_C2)
    for a, b in [(0, 300), (300, 4000), (4000, 5001)]:
        kl.walk_render(ab, seed, a, b - a, burn, steps, WIN_C2, image=acc, accumulate=True, hist_mode="lds")
    np.testing.assert_array_equal(kl.as_u32(acc).astype(np.int64), img)


def test_binned_render_limits():
    ab, _ = _maskit()
    # 257 tiles of 2^15 bins: the binned path is refused, the direct one renders
    big = (-1.05, 1.05, -0.1, 2.0, 4096, 2056)
    with pytest.raises(kl.KLError) as e:
        kl.walk_render(ab, 1, 0, 10, 0, 4, big, hist_mode="lds")
    assert e.value.code == kl.KL_EINVAL
    img = kl.walk_render(ab, 1, 0, 10, 0, 4, big, hist_mode="auto")
    assert int(kl.as_u32(img).astype(np.int64).sum()) <= 40
    # no points: an empty image either way
    assert int(kl.walk_render(ab, 1, 0, 0, 0, 4, WIN_M, hist_mode="lds").abs().sum()) == 0
    assert int(kl.walk_render(ab, 1, 0, 10, 3, 0, WIN_M, hist_mode="lds").abs().sum()) == 0
