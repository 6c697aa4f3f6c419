"""GPU path vs the CPU reference, through the C ABI.

Bars: decoding bit-exact; FP64 word values within 1e-10 * max(1, |z|);
FP32 word values within 0.25 pixel; images equal to the histogram of the
renderer's own per-word bins (exact), and to the reference image up to
words the reference places within the value tolerance of a bin edge.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1709_08018_amd import workloads as wl

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1709_08018_amd import kl

C2 = (wl.C2_TA, wl.C2_TB)
C1 = (wl.C1_TA, wl.C1_TB)
WIN_C2 = wl.QUASIFUCHSIAN_D18.window.as_tuple()
WIN_C3 = wl.QUASIFUCHSIAN_D22.window.as_tuple()
WIN_C1 = wl.FUCHSIAN_TILING_D10.window.as_tuple()
# edge band (px) of FP32 image comparisons with the oracle: above every
# measured per-word error (pole form 1.7e-4 px at depth 18, ratio form 7.2e-4)
FP32_EDGE_PX = 1e-3


def _z(t):
    a = t.cpu().numpy()
    return a[:, 0] + 1j * a[:, 1]


def _ref_pixels(z, win):
    x0, x1, y0, y1, W, H = win
    return (z.real - x0) * W / (x1 - x0), (z.imag - y0) * H / (y1 - y0)


def _bins_from_pixels(px, py, win):
    W, H = win[4], win[5]
    # the renderer's rule: 0 <= px < W and 0 <= py < H as IEEE comparisons
    # (-0 counts as 0; NaN compares false)
    ok = (px >= 0) & (px < W) & (py >= 0) & (py < H)
    img = np.zeros(W * H, np.int64)
    np.add.at(img, np.floor(py[ok]).astype(np.int64) * W + np.floor(px[ok]).astype(np.int64), 1)
    return img.reshape(H, W), int((~ok).sum())


# ---------------------------------------------------------------- decode
@pytest.mark.parametrize("depth", list(range(1, 11)))
def test_decode_all_words(depth):
    got = kl.decode(0, kl.num_words(depth), depth).cpu().numpy()
    np.testing.assert_array_equal(got, O.enumerate_words(depth))


@pytest.mark.parametrize("depth", [18, 22, 31, 40])
def test_decode_sampled_ranges(depth):
    n = kl.num_words(depth)
    rng = np.random.default_rng(depth)
    starts = [0, n - 300] + [int(x) for x in rng.integers(0, n - 2000, size=4, dtype=np.uint64)]
    counts = [1, 255, 256, 257, 1000, 300]
    for first, count in zip(starts, counts):
        count = min(count, n - first)
        got = kl.decode(first, count, depth).cpu().numpy()
        for j in list(range(min(count, 8))) + [count - 1]:
            np.testing.assert_array_equal(got[j], O.unrank(first + j, depth))


@pytest.mark.parametrize("depth", list(range(16, 33)))
def test_decode_packed_path_every_word_of_ranges(depth):
    """Depths 16..32 into an aligned destination take the packed stream
    staging: 8 (even depths) or 16 (odd) consecutive words a thread, whose
    low part (the last 3..8 digits: the short digit group, widened by six
    when it has fewer than three) wraps at most once among them, picking the
    letters above it for the high digits or for those plus one.  Ranges
    that start just before a wrap of the low part, of the shortest group and
    of the group above, that cross tiles of 2048 and 4096 words, and that end
    at the last word, every word against the oracle's enumeration; the same
    range into an unaligned destination (byte staging) gives the same
    bytes."""
    n = kl.num_words(depth)
    p = (depth - 1) % 6
    low = 3 ** p if p else 729              # radix of the shortest digit group
    radix = 3 ** (p if p >= 3 else p + 6)   # radix of the packed kernel's low part
    starts = [0, low - 5, low * 729 - 11, 3 * low * 729 - 2, n // 3 + 7, n - 4101,
              radix - 13, radix * 729 - 7, 5 * radix - 1]
    counts = [4101, 37, 2049, 300, 2048, 4101, 4097, 300, 33]
    def oracle_words(first, count):
        # the oracle's unranking word by word (its depth-first enumeration
        # walks every word before `first`)
        return np.stack([O.unrank(first + j, depth) for j in range(count)])

    for first, count in zip(starts, counts):
        first = max(0, min(first, n - 1))
        count = min(count, n - first)
        got = kl.decode(first, count, depth).cpu().numpy()
        np.testing.assert_array_equal(got, oracle_words(first, count))
    first, count = n // 5, 3001
    buf = torch.full((count * depth + 16,), 255, dtype=torch.uint8, device="cuda")
    view = buf[3:3 + count * depth]
    kl._check(kl.lib().kl_decode_ex(first, count, depth, view.data_ptr(), kl._stream(None)))
    host = buf.cpu().numpy()
    np.testing.assert_array_equal(host[3:3 + count * depth].reshape(count, depth), oracle_words(first, count))
    assert (host[:3] == 255).all() and (host[3 + count * depth:] == 255).all()


@pytest.mark.parametrize("depth,count", [(18, 12_000_000), (17, 12_000_000), (32, 9_000_000), (40, 3_000_000)])
def test_decode_many_tiles_per_workgroup(depth, count):
    """Ranges long enough that every workgroup takes many tiles: rows at both
    ends of every 2048-word and 256-word tile boundary in a stretch (4096-word
    tiles at odd depths fall on them too), and random rows, against the
    oracle's unranking."""
    n = kl.num_words(depth)
    first = n // 7
    out = kl.decode(first, count, depth)
    rng = np.random.default_rng(depth)
    rows = set(rng.integers(0, count, size=3000).tolist()) | {0, 1, count - 2, count - 1}
    for b in range(2048 * 1700, 2048 * 1800, 256):
        if b + 1 < count:
            rows |= {b - 1, b, b + 1}
    rows = np.array(sorted(r for r in rows if 0 <= r < count))
    got = out[torch.as_tensor(rows, device="cuda")].cpu().numpy()
    want = np.stack([O.unrank(first + int(r), depth) for r in rows])
    np.testing.assert_array_equal(got, want)


def test_decode_drawn_ranges():
    """24 ranges drawn at depths 1..40, up to 5,000 words from anywhere in
    the index space, decoded into 16-byte aligned and misaligned
    destinations (the packed path at depths 16-32 when aligned, the byte
    path otherwise): bit for bit the oracle's words, and nothing written
    outside the range's bytes."""
    for i, (depth, first, count) in enumerate(wl.draw_decode_ranges(24, seed=71)):
        off = 16 if i % 2 == 0 else 16 + 1 + i % 7
        nbytes = count * depth
        buf = torch.full((nbytes + 48,), 255, dtype=torch.uint8, device="cuda")
        view = buf[off:off + nbytes]
        kl._check(kl.lib().kl_decode_ex(first, count, depth, view.data_ptr(), kl._stream(None)))
        host = buf.cpu().numpy()
        # the oracle's enumeration walks the word tree (depths up to 20);
        # deeper words are unranked one by one
        want = (O.enumerate_words(depth, first, count) if depth <= 20 else
                np.stack([O.unrank(first + k, depth) for k in range(count)]))
        np.testing.assert_array_equal(host[off:off + nbytes].reshape(count, depth), want,
                                      err_msg=f"{depth} {first} {count}")
        assert (host[:off] == 255).all() and (host[off + nbytes:] == 255).all()


def test_decode_misaligned_destination():
    depth = 7
    n = kl.num_words(depth)
    buf = torch.full((n * depth + 8,), 255, dtype=torch.uint8, device="cuda")
    for off in (1, 2, 3, 5):
        buf.fill_(255)
        view = buf[off:off + n * depth]
        kl.lib()  # binding loaded
        kl._check(kl.lib().kl_decode_ex(0, n, depth, view.data_ptr(), kl._stream(None)))
        host = buf.cpu().numpy()
        np.testing.assert_array_equal(host[off:off + n * depth].reshape(n, depth), O.enumerate_words(depth))
        assert (host[:off] == 255).all() and (host[off + n * depth:] == 255).all()


# ---------------------------------------------------------------- values
REL_FLOOR = 1e-6


def _fp64_case(ta, tb, depth, idx):
    """Largest error of the FP64 path's values against the oracle's: the bar
    is 1e-10 relative to max(1, |z|); values with |z| above REL_FLOOR must
    also be within 1e-10 of |z| itself (truly relative)."""
    z = _z(kl.eval_values(ta, tb, depth, idx, precision="fp64"))
    zr = O.eval_values(ta, tb, depth, idx)
    dz = np.abs(z - zr)
    big = np.abs(zr) > REL_FLOOR
    rel = (dz[big] / np.abs(zr[big])).max() if big.any() else 0.0
    assert rel < 1e-10, f"relative error {rel:.3e} ({int((~big).sum())} values below {REL_FLOOR})"
    return (dz / np.maximum(1, np.abs(zr))).max()


def test_fp64_values_all_words_small():
    assert _fp64_case(*C1, 8, np.arange(kl.num_words(8), dtype=np.uint64)) < 1e-10
    assert _fp64_case(*C2, 11, np.arange(kl.num_words(11), dtype=np.uint64)) < 1e-10


@pytest.mark.parametrize("depth", [5, 18, 22, 30, 40])
def test_fp64_values_sampled(depth):
    idx = wl.sample_indices(kl.num_words(depth), 20000 if depth <= 22 else 2000, seed=depth)
    idx = np.concatenate([idx, np.array([0, kl.num_words(depth) - 1], np.uint64)])
    assert _fp64_case(*C2, depth, idx) < 1e-10


def test_fp64_values_batch_law():
    ta, tb, _ = wl.draw_param_sets(12, seed=21)
    for a, b in zip(ta, tb):
        idx = wl.sample_indices(kl.num_words(14), 3000, seed=1)
        assert _fp64_case(complex(a), complex(b), 14, idx) < 1e-10


def test_values_on_drawn_parameter_sets_and_depths():
    """32 parameter sets of the batch's law (Re ta, Re tb in [1.8, 3.0], Im
    in [-0.3, 0.3]) at depths drawn from 5..30, 2,000 sampled words each:
    FP64 values within the 1e-10 bar of the oracle's, and FP32 pixel
    coordinates on a 1024^2 window over [-2, 2]^2 within 0.25 px of the
    oracle's for every word near the window."""
    ta, tb, depth = wl.draw_param_sets(32, seed=41, depth_range=(5, 30))
    win = (-2.0, 2.0, -2.0, 2.0, 1024, 1024)
    worst = 0.0
    for i in range(len(ta)):
        a, b, d = complex(ta[i]), complex(tb[i]), int(depth[i])
        idx = wl.sample_indices(kl.num_words(d), 2000, seed=100 + i)
        assert _fp64_case(a, b, d, idx) < 1e-10, (i, d)
        p = kl.eval_values(a, b, d, idx, precision="fp32", window=win).cpu().numpy()
        fx, fy = _ref_pixels(O.eval_values(a, b, d, idx), win)
        near = (fx > -1) & (fx < win[4] + 1) & (fy > -1) & (fy < win[5] + 1)
        if near.any():
            err = np.hypot(p[near, 0] - fx[near], p[near, 1] - fy[near]).max()
            worst = max(worst, err)
            assert err <= 0.25, (i, d, err)
    print(f"largest FP32 pixel error over the drawn sets: {worst:.3e} px")


@pytest.mark.parametrize("depth,win", [(18, WIN_C2), (22, WIN_C3)])
def test_fp32_pixel_error(depth, win):
    idx = wl.sample_indices(kl.num_words(depth), 100000, seed=0)
    p = kl.eval_values(*C2, depth, idx, precision="fp32", window=win).cpu().numpy()
    fx, fy = _ref_pixels(O.eval_values(*C2, depth, idx), win)
    err = np.hypot(p[:, 0] - fx, p[:, 1] - fy)
    inside = (fx > -1) & (fx < win[4] + 1) & (fy > -1) & (fy < win[5] + 1)
    print(f"depth {depth}: FP32 pixel error max {err[inside].max():.3e} p99 {np.quantile(err[inside], .99):.3e}"
          f" mean {err[inside].mean():.3e} over {inside.sum()} words near the window")
    assert err[inside].max() <= 0.25


def test_eval_out_of_range_index_gives_nan():
    n = kl.num_words(6)
    z = _z(kl.eval_values(*C2, 6, np.array([0, n - 1, n, 2 ** 63], np.uint64).view(np.int64)))
    assert np.isfinite(z[:2]).all() and np.isnan(z[2:]).all()


# ---------------------------------------------------------------- images
# tail_len 4 gives these depths enough heads for the persistent kernel; the
# planner's 6 leaves them to the per-word kernel
@pytest.mark.parametrize("tail_len", [0, 4])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("depth,win", [(12, WIN_C2), (13, (-2.0, 2.0, -2.0, 2.0, 300, 100))])
def test_image_is_histogram_of_own_bins(precision, depth, win, tail_len):
    n = kl.num_words(depth)
    dropped = torch.zeros(1, dtype=torch.int64, device="cuda")
    img = kl.as_u32(kl.render(*C2, depth, win, precision=precision, dropped=dropped,
                              tail_len=tail_len)).astype(np.int64)
    p = kl.eval_values(*C2, depth, np.arange(n, dtype=np.uint64), precision=precision, window=win,
                       tail_len=tail_len).cpu().numpy()
    ref, drop = _bins_from_pixels(p[:, 0], p[:, 1], win)
    np.testing.assert_array_equal(img, ref)
    assert int(dropped.item()) == drop
    assert int(img.sum()) + drop == n


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_drawn_sets_images_are_histograms_of_own_bins(precision):
    """Six parameter sets of the batch's law at depths 9..15 (the planner's
    splits, which at depths 13-15 take shorter tails and the persistent
    kernel): each image and dropped count equal the histogram of kl_eval's
    pixel coordinates of every word, bit for bit."""
    ta, tb, depth = wl.draw_param_sets(6, seed=53, depth_range=(9, 15))
    win = (-2.0, 2.0, -1.5, 1.5, 640, 480)
    for i in range(len(ta)):
        a, b, d = complex(ta[i]), complex(tb[i]), int(depth[i])
        n = kl.num_words(d)
        dropped = torch.zeros(1, dtype=torch.int64, device="cuda")
        img = kl.as_u32(kl.render(a, b, d, win, precision=precision, dropped=dropped)).astype(np.int64)
        p = kl.eval_values(a, b, d, np.arange(n, dtype=np.uint64), precision=precision, window=win).cpu().numpy()
        ref, drop = _bins_from_pixels(p[:, 0], p[:, 1], win)
        np.testing.assert_array_equal(img, ref, err_msg=f"set {i}, depth {d}")
        assert int(dropped.item()) == drop, (i, d)


@pytest.mark.parametrize("case", ["c1_tiling", "c2_d11", "c2_d12_aniso"])
def test_fp64_image_matches_reference(case):
    if case == "c1_tiling":
        (ta, tb), depth, win, mind = C1, 10, WIN_C1, 1
    elif case == "c2_d11":
        (ta, tb), depth, win, mind = C2, 11, WIN_C2, 11
    else:
        (ta, tb), depth, win, mind = C2, 12, (-2.0, 2.0, -1.5, 1.5, 512, 200), 12
    img = kl.as_u32(kl.render(ta, tb, depth, win, precision="fp64", min_depth=mind)).astype(np.int64)
    ref, _, near = O.render(ta, tb, depth, win, min_depth=mind, edge_tol=1e-7, nthreads=8)
    diff = int(np.abs(img - ref.astype(np.int64)).sum())
    assert diff <= 2 * near, (diff, near)


def test_fp32_image_close_to_reference():
    win = WIN_C2
    img = kl.as_u32(kl.render(*C2, 12, win, precision="fp32")).astype(np.int64)
    ref, _, near = O.render(*C2, 12, win, edge_tol=FP32_EDGE_PX, nthreads=8)
    diff = int(np.abs(img - ref.astype(np.int64)).sum())
    print(f"FP32 image L1 difference {diff} of {ref.sum()} counts; {near} words within {FP32_EDGE_PX} px of an edge")
    assert diff <= 2 * near


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_range_additivity_and_ragged_ranges(precision):
    depth, win = 14, WIN_C2
    n = kl.num_words(depth)
    full = kl.render(*C2, depth, win, precision=precision)
    cuts = sorted({0, 1, 12345, 999_999, 1_500_001, n - 7, n})
    acc = kl.new_image(win)
    for a, b in zip(cuts[:-1], cuts[1:]):
        kl.render(*C2, depth, win, image=acc, precision=precision, first=a, count=b - a, accumulate=True)
    assert torch.equal(acc, full)
    # small ragged ranges against the reference (FP64 only: exact-ish)
    if precision == "fp64":
        for first, count in [(0, 1), (5, 300), (n // 3, 20000), (n - 1, 1), (n // 2, 0)]:
            img = kl.as_u32(kl.render(*C2, depth, win, precision="fp64", first=first, count=count)).astype(np.int64)
            ref, _, near = O.render(*C2, depth, win, first=first, count=count, edge_tol=1e-7)
            assert int(np.abs(img - ref).sum()) <= 2 * near
            assert img.sum() <= count


@pytest.mark.parametrize("depth", [33, 40])
def test_deep_index_ranges(depth):
    """Renders of index ranges at depths 33 and 40.  Head indices there need
    64 bits, and at depth 40 (4 * 3^39, about 1.6e19 words) word indices pass
    2^63.  The ranges are:
      * one that crosses 2^63 (at depth 33, the middle);
      * one that ends at the last word;
      * 1,000 words at the start.
    Each range is rendered into a 512^2 window fitted to the oracle's values
    of 4,000 of its words.  At depth 40 the first range spans about 1e-9, a
    deep zoom.  The long ranges hold over 8,192 whole heads: the persistent
    kernel renders those and the per-word kernel renders the ragged ends.
    In both precisions:
      * each image and dropped count equal the histogram of kl_eval's pixel
        coordinates of the same words, bit for bit;
      * on the 4,000 words, FP64 values are within 1e-10 of the oracle's, and
        FP32 pixel coordinates within 0.25 px for words near the window."""
    n = kl.num_words(depth)
    mid = 1 << 63 if depth == 40 else n // 2
    for first, count in [(mid - 3_000_017, 6_100_003), (n - 6_200_011, 6_200_011), (0, 1000)]:
        print(f"depth {depth}: words [{first}, {first + count})", flush=True)
        rng = np.random.default_rng(first % 1000)
        sample = np.unique(np.uint64(first) + rng.integers(0, count, 4000).astype(np.uint64))
        z = O.eval_values(*C2, depth, sample)
        mx, my = 0.1 * np.ptp(z.real) + 1e-12, 0.1 * np.ptp(z.imag) + 1e-12
        win = (z.real.min() - mx, z.real.max() + mx, z.imag.min() - my, z.imag.max() + my, 512, 512)
        W, H = win[4], win[5]
        idx = np.uint64(first) + np.arange(count, dtype=np.uint64)
        for precision in ("fp32", "fp64"):
            dropped = torch.zeros(1, dtype=torch.int64, device="cuda")
            img = kl.as_u32(kl.render(*C2, depth, win, precision=precision, first=first, count=count,
                                      dropped=dropped)).astype(np.int64)
            p = kl.eval_values(*C2, depth, idx, precision=precision, window=win).cpu().numpy()
            px, py = p[:, 0], p[:, 1]
            ok = (px >= 0) & (px < W) & (py >= 0) & (py < H)
            key = np.floor(py[ok]).astype(np.int64) * W + np.floor(px[ok]).astype(np.int64)
            ref = np.bincount(key, minlength=W * H).reshape(H, W)
            np.testing.assert_array_equal(img, ref, err_msg=f"{precision} [{first}, +{count})")
            assert int(dropped.item()) == int((~ok).sum()), (precision, first)
            assert int(img.sum()) + int(dropped.item()) == count
            del p, px, py, ok, key
        assert _fp64_case(*C2, depth, sample) < 1e-10, first
        q = kl.eval_values(*C2, depth, sample, precision="fp32", window=win).cpu().numpy()
        fx, fy = _ref_pixels(z, win)
        near = (fx > -1) & (fx < W + 1) & (fy > -1) & (fy < H + 1)
        err = np.maximum(np.abs(q[:, 0] - fx), np.abs(q[:, 1] - fy))[near]
        print(f"  {int(near.sum())} sampled words near the window; largest FP32 error {err.max():.2e} px")
        assert near.sum() > 0.9 * len(sample) and err.max() < 0.25, (first, err.max())


@pytest.mark.parametrize("W,H", [(32768, 32768), (1, 1), (32768, 1), (1, 32768)])
def test_extreme_windows(W, H):
    """Windows at the library's limits: 32768 x 32768 bins (2^30, a 4 GiB
    image, the largest accepted), a single bin, a single row and a single
    column, over [-1.5, 1.5]^2 at depth 12.  In both precisions, and with
    register runs and the LDS tile histogram, the image and dropped count
    equal the histogram of kl_eval's pixel coordinates of every word, bit for
    bit (compared sparsely on the GPU)."""
    depth = 12
    win = (-1.5, 1.5, -1.5, 1.5, W, H)
    n = kl.num_words(depth)
    idx = torch.arange(n, dtype=torch.int64, device="cuda")
    img = kl.new_image(win)
    for precision in ("fp32", "fp64"):
        p = kl.eval_values(*C2, depth, idx, precision=precision, window=win)
        px, py = p[:, 0], p[:, 1]
        ok = (px >= 0) & (px < W) & (py >= 0) & (py < H)
        key = torch.floor(py[ok]).to(torch.int64) * W + torch.floor(px[ok]).to(torch.int64)
        want_bins, want_counts = torch.unique(key, return_counts=True)
        for hist_mode in ("runs", "lds"):
            print(f"{W}x{H} {precision} {hist_mode}", flush=True)
            dropped = torch.zeros(1, dtype=torch.int64, device="cuda")
            kl.render(*C2, depth, win, image=img, precision=precision, hist_mode=hist_mode, dropped=dropped)
            flat = img.view(-1)
            bins = torch.nonzero(flat).view(-1)
            assert torch.equal(bins, want_bins), (precision, hist_mode)
            assert torch.equal(flat[bins].to(torch.int64), want_counts), (precision, hist_mode)
            assert int(dropped.item()) == int((~ok).sum().item()) == n - int(want_counts.sum().item())
    del img


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_deep_tiling_ranges_cross_depths(precision):
    """Tiling renders (every depth from 1 to 30, about 1.4e14 words) of index
    ranges that cross from depth 29 into depth 30, and that end at the
    tiling's last word.  Each image equals the histogram of kl_eval's pixel
    coordinates of the same words, taken depth by depth.  The FP64 image is
    also within the edge bar of the oracle's render of the range."""
    depth, mind, win = 30, 1, WIN_C2
    W, H = win[4], win[5]
    starts = [0]
    for d in range(mind, depth + 1):
        starts.append(starts[-1] + kl.num_words(d))
    b29 = starts[depth - mind]           # first word of depth 30 in the tiling's index space
    total = starts[-1]
    for first, count in [(b29 - 1_200_007, 2_500_011), (total - 900_001, 900_001)]:
        dropped = torch.zeros(1, dtype=torch.int64, device="cuda")
        img = kl.as_u32(kl.render(*C2, depth, win, min_depth=mind, precision=precision, first=first, count=count,
                                  dropped=dropped)).astype(np.int64)
        ref = np.zeros((H, W), np.int64)
        drop = 0
        for d in range(mind, depth + 1):
            lo, hi = max(first, starts[d - mind]), min(first + count, starts[d - mind + 1])
            if lo >= hi:
                continue
            local = np.uint64(lo - starts[d - mind]) + np.arange(hi - lo, dtype=np.uint64)
            p = kl.eval_values(*C2, d, local, precision=precision, window=win).cpu().numpy()
            ok = (p[:, 0] >= 0) & (p[:, 0] < W) & (p[:, 1] >= 0) & (p[:, 1] < H)
            key = np.floor(p[ok, 1]).astype(np.int64) * W + np.floor(p[ok, 0]).astype(np.int64)
            ref += np.bincount(key, minlength=W * H).reshape(H, W)
            drop += int((~ok).sum())
        np.testing.assert_array_equal(img, ref, err_msg=f"{precision} [{first}, +{count})")
        assert int(dropped.item()) == drop
        if precision == "fp64":
            oimg, _, near = O.render(*C2, depth, win, min_depth=mind, first=first, count=count, edge_tol=1e-7,
                                     nthreads=8)
            assert int(np.abs(img - oimg.astype(np.int64)).sum()) <= 2 * near


def test_tiling_ranges_cross_depths():
    depth, mind, win = 9, 2, WIN_C1
    total = sum(kl.num_words(d) for d in range(mind, depth + 1))
    full = kl.render(*C1, depth, win, min_depth=mind, precision="fp64")
    acc = kl.new_image(win)
    for a, b in [(0, 10), (10, 5000), (5000, total - 3), (total - 3, total)]:
        kl.render(*C1, depth, win, image=acc, min_depth=mind, precision="fp64", first=a, count=b - a,
                  accumulate=True)
    assert torch.equal(acc, full)


@pytest.mark.parametrize("depth", [14, 18])
def test_lds_tile_histogram_equals_direct_runs(depth):
    a = kl.render(*C2, depth, WIN_C2, hist_mode="runs")
    b = kl.render(*C2, depth, WIN_C2, hist_mode="lds")
    assert torch.equal(a, b)
    c = kl.render(*C1, 10, WIN_C1, min_depth=1, hist_mode="lds")
    d = kl.render(*C1, 10, WIN_C1, min_depth=1, hist_mode="runs")
    assert torch.equal(c, d)


# ---------------------------------------------------------------- head forms
@pytest.mark.parametrize("head_form", [1, 2])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_ratio_form_heads_render_their_own_bins(head_form, precision):
    """Heads applied as the ratio (A y + B) / (C y + D) -- every head, or
    every odd one so that waves mix both forms -- draw exactly the bins
    kl_eval gives their words under the same head form, with either
    histogram strategy and in the batched renderer."""
    depth, win = 13, (-1.7, 1.3, -1.4, 1.6, 640, 480)
    tl = 4   # enough heads for the persistent kernel
    n = kl.num_words(depth)
    dropped = torch.zeros(1, dtype=torch.int64, device="cuda")
    img = kl.render(*C2, depth, win, precision=precision, dropped=dropped, head_form=head_form, tail_len=tl)
    p = kl.eval_values(*C2, depth, np.arange(n, dtype=np.uint64), precision=precision, window=win,
                       head_form=head_form, tail_len=tl).cpu().numpy()
    ref, drop = _bins_from_pixels(p[:, 0], p[:, 1], win)
    np.testing.assert_array_equal(kl.as_u32(img).astype(np.int64), ref)
    assert int(dropped.item()) == drop
    lds = kl.render(*C2, depth, win, precision=precision, head_form=head_form, hist_mode="lds", tail_len=tl)
    assert torch.equal(lds, img)
    many = kl.render_many([C2[0]] * 2, [C2[1]] * 2, [depth, depth], win, precision=precision,
                          head_form=head_form, tail_len=tl)
    assert torch.equal(many[0], img) and torch.equal(many[1], img)


@pytest.mark.parametrize("head_form", [0, 1, 2])
def test_head_forms_meet_the_fp32_bar(head_form):
    """Pole form and ratio form both stay within 0.25 pixel of the FP64
    reference per word, and their images within the near-edge bound."""
    depth, win = 18, WIN_C2
    idx = wl.sample_indices(kl.num_words(depth), 100000, seed=3)
    p = kl.eval_values(*C2, depth, idx, precision="fp32", window=win, head_form=head_form).cpu().numpy()
    fx, fy = _ref_pixels(O.eval_values(*C2, depth, idx), win)
    err = np.hypot(p[:, 0] - fx, p[:, 1] - fy)
    inside = (fx > -1) & (fx < win[4] + 1) & (fy > -1) & (fy < win[5] + 1)
    print(f"head_form {head_form}: FP32 pixel error max {err[inside].max():.3e} mean {err[inside].mean():.3e}")
    assert err[inside].max() <= 0.25
    img = kl.as_u32(kl.render(*C2, 12, win, precision="fp32", head_form=head_form)).astype(np.int64)
    ref, _, near = O.render(*C2, 12, win, edge_tol=FP32_EDGE_PX, nthreads=8)
    assert int(np.abs(img - ref.astype(np.int64)).sum()) <= 2 * near


def test_run_to_run_bit_equality():
    a = kl.render(*C2, 16, WIN_C2)
    b = kl.render(*C2, 16, WIN_C2)
    assert torch.equal(a, b)


def test_table_buffer_reuse_across_calls_and_streams():
    """Renders on the null stream reuse one table buffer per device, which
    grows when a call needs more; renders on other streams take temporaries.
    Calls enqueued back to back, without synchronising, in an order that
    grows the buffer and shrinks the tables again and mixes in a side stream,
    give the images that each call gives alone."""
    cases = [(C2, 12, WIN_C2, "fp32"), (C2, 18, WIN_C2, "fp32"), (C1, 10, WIN_C1, "fp64"),
             (C2, 19, WIN_C2, "fp64"), (C2, 14, WIN_C2, "fp32")]
    alone = []
    for g, d, w, p in cases:
        alone.append(kl.render(*g, d, w, precision=p))
        torch.cuda.synchronize()
    side = torch.cuda.Stream()
    out = []
    for i, (g, d, w, p) in enumerate(cases):
        if i == 2:
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                out.append(kl.render(*g, d, w, precision=p))
            torch.cuda.current_stream().wait_stream(side)
        else:
            out.append(kl.render(*g, d, w, precision=p))
    torch.cuda.synchronize()
    for (g, d, w, p), a, b in zip(cases, alone, out):
        assert torch.equal(a, b), (d, p)


@pytest.mark.parametrize("depth", [1, 2, 3, 4, 5])
def test_shallow_depths(depth):
    win = (-2.0, 2.0, -2.0, 2.0, 64, 64)
    for ta, tb in (C1, C2):
        img = kl.as_u32(kl.render(ta, tb, depth, win, precision="fp64")).astype(np.int64)
        ref, drop, near = O.render(ta, tb, depth, win, edge_tol=1e-9)
        assert int(np.abs(img - ref).sum()) <= 2 * near


def test_window_edge_cases():
    # a window far from the limit set drops every word; a 1x1 window keeps the ones inside
    n = kl.num_words(10)
    dropped = torch.zeros(1, dtype=torch.int64, device="cuda")
    img = kl.render(*C2, 10, (100.0, 101.0, 100.0, 101.0, 8, 8), dropped=dropped)
    assert int(img.sum()) == 0 and int(dropped.item()) == n
    one = kl.as_u32(kl.render(*C2, 10, (-1.5, 1.5, -1.5, 1.5, 1, 1), precision="fp64")).astype(np.int64)
    ref, _, near = O.render(*C2, 10, (-1.5, 1.5, -1.5, 1.5, 1, 1), edge_tol=1e-7)
    assert abs(int(one.sum()) - int(ref.sum())) <= near
    # accumulate with an empty range leaves the image as it was
    img = kl.render(*C2, 10, WIN_C2)
    before = img.clone()
    kl.render(*C2, 10, WIN_C2, image=img, first=5, count=0, accumulate=True)
    assert torch.equal(img, before)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_non_finite_and_far_coordinates_are_dropped(precision):
    """A window so narrow that its scale to pixels leaves FP32's range: the
    FP32 coordinates are infinite or NaN, the FP64 ones finite and far
    outside.  Both renders drop exactly the words the histogram of their own
    coordinates drops."""
    depth, win = 12, (0.0, 1e-37, 0.0, 1e-37, 64, 64)
    n = kl.num_words(depth)
    dropped = torch.zeros(1, dtype=torch.int64, device="cuda")
    img = kl.as_u32(kl.render(*C2, depth, win, precision=precision, dropped=dropped)).astype(np.int64)
    p = kl.eval_values(*C2, depth, np.arange(n, dtype=np.uint64), precision=precision, window=win).cpu().numpy()
    if precision == "fp32":
        assert (~np.isfinite(p)).any()
    ref, drop = _bins_from_pixels(p[:, 0], p[:, 1], win)
    np.testing.assert_array_equal(img, ref)
    assert int(dropped.item()) == drop


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_homogeneous_suffix_form(precision):
    depth, win = 12, WIN_C2
    tl = 4   # enough heads for the persistent kernel
    n = kl.num_words(depth)
    idx = np.arange(n, dtype=np.uint64)
    p = kl.eval_values(*C2, depth, idx, precision=precision, window=win, suffix_form=1, tail_len=tl).cpu().numpy()
    img = kl.as_u32(kl.render(*C2, depth, win, precision=precision, suffix_form=1, tail_len=tl)).astype(np.int64)
    ref, _ = _bins_from_pixels(p[:, 0], p[:, 1], win)
    np.testing.assert_array_equal(img, ref)
    if precision == "fp64":
        z = _z(kl.eval_values(*C2, depth, idx[::7], precision="fp64", suffix_form=1))
        zr = O.eval_values(*C2, depth, idx[::7])
        assert (np.abs(z - zr) / np.maximum(1, np.abs(zr))).max() < 1e-10


# ---------------------------------------------------------------- batched
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_render_many_equals_single_renders(precision):
    """A batched render draws each set's image bit for bit as a single render
    of that set under the same split (the split the batch plans for the set,
    kl_plan_many; a single render of depths 13-16 plans a shorter tail by
    default, which rounds differently)."""
    ta, tb, depth = wl.draw_param_sets(10, seed=7, depth_range=(5, 13))
    win = wl.BATCH_WINDOW.as_tuple()
    dropped = torch.zeros(len(ta), dtype=torch.int64, device="cuda")
    imgs = kl.render_many(ta, tb, depth, win, precision=precision, dropped=dropped)
    for i in range(len(ta)):
        d1 = torch.zeros(1, dtype=torch.int64, device="cuda")
        p = kl.plan_many(int(depth[i]), precision, win)
        single = kl.render(ta[i], tb[i], int(depth[i]), win, precision=precision, dropped=d1,
                           tail_len=p["tail_len"], lane_len=p["lane_len"])
        assert torch.equal(imgs[i], single), i
        assert int(dropped[i].item()) == int(d1.item())
        assert int(kl.as_u32(imgs[i]).sum()) + int(d1.item()) == kl.num_words(int(depth[i]))


def test_render_many_with_twenty_thousand_sets():
    """20,000 parameter sets of the batch's law at depths 3 to 13 in one
    batched render (64 x 64 images over [-2, 2]^2).  The shallow sets take
    the per-word batch kernel and the deeper ones the persistent batched
    kernel, so both search thousands of sets.  Every set's image sum plus
    its dropped count equals its words, and 40 sets spread over the batch
    equal their single renders under the batch's split, bit for bit."""
    ta, tb, depth = wl.draw_param_sets(20_000, seed=97, depth_range=(3, 13))
    win = (-2.0, 2.0, -2.0, 2.0, 64, 64)
    dropped = torch.zeros(len(ta), dtype=torch.int64, device="cuda")
    imgs = kl.render_many(ta, tb, depth, win, dropped=dropped)
    words = torch.as_tensor([kl.num_words(int(d)) for d in depth], dtype=torch.int64, device="cuda")
    sums = imgs.view(len(ta), -1).to(torch.int64).sum(1)
    assert torch.equal(sums + dropped, words)
    for i in np.linspace(0, len(ta) - 1, 40).astype(int):
        d1 = torch.zeros(1, dtype=torch.int64, device="cuda")
        p = kl.plan_many(int(depth[i]), "fp32", win)
        single = kl.render(ta[i], tb[i], int(depth[i]), win, dropped=d1, tail_len=p["tail_len"],
                           lane_len=p["lane_len"])
        assert torch.equal(imgs[i], single), i
        assert int(dropped[i].item()) == int(d1.item()), i


# ---------------------------------------------------------------- full size
def test_full_quasifuchsian_d18_invariants_and_samples():
    depth, win = 18, WIN_C2
    n = kl.num_words(depth)
    dropped = torch.zeros(1, dtype=torch.int64, device="cuda")
    img = kl.render(*C2, depth, win, dropped=dropped)
    img2 = kl.render(*C2, depth, win)
    assert torch.equal(img, img2)
    h = kl.as_u32(img).astype(np.int64)
    assert int(h.sum()) + int(dropped.item()) == n
    # every sampled word the renderer bins is counted where its own arithmetic puts it,
    # and lies within 0.25 px of the reference value
    idx = wl.sample_indices(n, 50000, seed=2)
    p = kl.eval_values(*C2, depth, idx, window=win).cpu().numpy()
    fx, fy = _ref_pixels(O.eval_values(*C2, depth, idx), win)
    ok = (p[:, 0] >= 0) & (p[:, 0] < win[4]) & (p[:, 1] >= 0) & (p[:, 1] < win[5])
    assert np.hypot(p[ok, 0] - fx[ok], p[ok, 1] - fy[ok]).max() <= 0.25
    # bin-for-bin equality with the histogram of every word's own coordinates:
    # test_gpu_fullsize.py


def test_full_batch256_invariants_and_samples():
    """The batched workload at its full size, in the launch the benchmark
    times: 256 parameter sets of depths 12..18, 512 x 512 each, one
    kl_render_many.  Every image holds its set's words exactly (bins plus
    dropped words); a depth-18 set and a depth-12 set equal their single
    renders bit for bit; and on four sets, sampled words lie within 0.25 px
    of the oracle's FP64 value.  (Those four images against the histogram of
    all their words' own coordinates: test_gpu_fullsize.py.)"""
    ta, tb, depth = wl.batch256(seed=0)
    win = wl.BATCH_WINDOW.as_tuple()
    dropped = torch.zeros(len(ta), dtype=torch.int64, device="cuda")
    imgs = kl.render_many(ta, tb, depth, win, dropped=dropped)
    sums = kl.as_u32(imgs).astype(np.int64).reshape(len(ta), -1).sum(axis=1)
    drops = dropped.cpu().numpy()
    for i in range(len(ta)):
        assert int(sums[i]) + int(drops[i]) == kl.num_words(int(depth[i])), i
    picks = [int(np.argmax(depth)), int(np.argmin(depth)), 17, 200]
    for i in picks[:2]:
        single = kl.render(ta[i], tb[i], int(depth[i]), win)
        assert torch.equal(imgs[i], single), i
    for i in picks:
        d = int(depth[i])
        idx = wl.sample_indices(kl.num_words(d), 4000, seed=i)
        pnt = kl.eval_values(ta[i], tb[i], d, idx, window=win).cpu().numpy()
        fx, fy = _ref_pixels(O.eval_values(complex(ta[i]), complex(tb[i]), d, idx), win)
        ok = (pnt[:, 0] >= 0) & (pnt[:, 0] < win[4]) & (pnt[:, 1] >= 0) & (pnt[:, 1] < win[5])
        assert np.hypot(pnt[ok, 0] - fx[ok], pnt[ok, 1] - fy[ok]).max() <= 0.25, i


def test_autotune_keeps_eval_and_render_consistent():
    depth, win = 11, WIN_C2
    plan, ms = kl.autotune(*C2, depth, win)
    assert plan["tail_len"] + plan["lane_len"] + plan["prefix_len"] == depth and ms > 0
    assert kl.plan(depth, "fp32") ["tail_len"] == plan["tail_len"]
    n = kl.num_words(depth)
    img = kl.as_u32(kl.render(*C2, depth, win)).astype(np.int64)
    p = kl.eval_values(*C2, depth, np.arange(n, dtype=np.uint64), window=win).cpu().numpy()
    ref, _ = _bins_from_pixels(p[:, 0], p[:, 1], win)
    np.testing.assert_array_equal(img, ref)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("seed", ["own", "all"])
def test_tiling_render_equals_sum_of_single_depths(precision, seed):
    """A tiling render of its whole index space runs as one batched render
    (every depth and seed a set of it); it equals the single-depth renders
    of each depth and seed added up, counts and dropped words alike."""
    depth, mind, win = 12, 1, WIN_C2
    dropped = torch.zeros(1, dtype=torch.int64, device="cuda")
    img = kl.render(wl.C2_TA, wl.C2_TB, depth, win, precision=precision, min_depth=mind, seed=seed, dropped=dropped)
    acc = kl.new_image(win)
    dacc = torch.zeros(1, dtype=torch.int64, device="cuda")
    first = True
    for s in (["a", "b", "A", "B"] if seed == "all" else [seed]):
        for d in range(mind, depth + 1):
            kl.render(wl.C2_TA, wl.C2_TB, d, win, image=acc, precision=precision, seed=s, accumulate=not first,
                      dropped=dacc)
            first = False
    assert torch.equal(img, acc)
    assert int(dropped.item()) == int(dacc.item())
    copies = 4 if seed == "all" else 1
    assert int(kl.as_u32(img).astype(np.int64).sum()) + int(dropped.item()) == copies * sum(
        kl.num_words(d) for d in range(mind, depth + 1))


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_tiling_takes_its_deepest_depth_tail(precision):
    """A tiling whose deepest depth plans a shorter tail when rendered alone
    (depth 14: 4 letters) takes that tail at every depth long enough for it:
    it equals the single-depth renders added up under that tail, and its
    index ranges add up to it."""
    depth, mind, win = 14, 1, (-2.0, 2.0, -2.0, 2.0, 512, 512)
    r = kl.plan(depth, precision)["tail_len"]
    assert r == 4
    full = kl.render(*C2, depth, win, precision=precision, min_depth=mind)
    acc = kl.new_image(win)
    for d in range(mind, depth + 1):
        kl.render(*C2, d, win, image=acc, precision=precision, accumulate=d > mind, tail_len=r if d > r else 0)
    assert torch.equal(full, acc)
    total = sum(kl.num_words(d) for d in range(mind, depth + 1))
    acc2 = kl.new_image(win)
    cuts = [0, 1000, total // 3, total - 5, total]
    for a, b in zip(cuts[:-1], cuts[1:]):
        kl.render(*C2, depth, win, image=acc2, precision=precision, min_depth=mind, first=a, count=b - a,
                  accumulate=a > 0)
    assert torch.equal(full, acc2)
