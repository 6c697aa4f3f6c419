"""GPU path vs the CPU reference for the seed modes and for groups given by
their generators (Maskit's embedding of the paper's figures), through the
C ABI.

Maskit's group has a translation among its generators: seeds at infinity,
heads whose map fixes infinity (the ratio fallback of the pole form) and
suffix points at infinity (the homogeneous suffix table) all occur, so these
cases run the renderer's rarely used paths on a real workload.
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
WIN_MASKIT = wl.MASKIT_D14.window.as_tuple()
MU = wl.MASKIT_MU
SEEDS = ["a", "b", "A", "B"]


def _z(t):
    a = t.cpu().numpy()
    return a[:, 0] + 1j * a[:, 1]


def _ref_pixels(z, win):
    x0, x1, y0, y1, W, H = win
    return (z.real - x0) * W / (x1 - x0), (z.imag - y0) * H / (y1 - y0)


def _bins_from_pixels(px, py, win):
    W, H = win[4], win[5]
    ok = (px >= 0) & (px < W) & (py >= 0) & (py < H)   # IEEE: -0 counts as 0, NaN is outside
    img = np.zeros(W * H, np.int64)
    np.add.at(img, np.floor(py[ok]).astype(np.int64) * W + np.floor(px[ok]).astype(np.int64), 1)
    return img.reshape(H, W), int((~ok).sum())


def _rel_err(z, zr, floor=1e-6):
    """Error against max(1, |z|); values with |z| above `floor` must also be
    within 1e-10 of |z| itself (truly relative)."""
    fin = np.isfinite(zr)
    assert np.isfinite(z[fin]).all()
    dz, a = np.abs(z[fin] - zr[fin]), np.abs(zr[fin])
    big = a > floor
    if big.any():
        rel = (dz[big] / a[big]).max()
        assert rel < 1e-10, f"relative {rel:.3e}; {int((~big).sum())} values below {floor}"
    return (dz / np.maximum(1, a)).max()


# ---------------------------------------------------------------- seed modes
@pytest.mark.parametrize("seed", SEEDS)
def test_seeded_fp64_values(seed):
    G = O.group_recipe(*C2)
    p = SEEDS.index(seed)
    idx = np.arange(kl.num_words(10), dtype=np.uint64)
    assert _rel_err(_z(kl.eval_values(*C2, 10, idx, precision="fp64", seed=seed)),
                    O.eval_group(G, 10, idx, seed=p)) < 1e-10
    idx = wl.sample_indices(kl.num_words(18), 20000, seed=p)
    assert _rel_err(_z(kl.eval_values(*C2, 18, idx, precision="fp64", seed=seed)),
                    O.eval_group(G, 18, idx, seed=p)) < 1e-10


@pytest.mark.parametrize("seed", SEEDS)
def test_seeded_fp32_pixel_error(seed):
    G = O.group_recipe(*C2)
    idx = wl.sample_indices(kl.num_words(18), 100000, seed=7)
    p = kl.eval_values(*C2, 18, idx, precision="fp32", window=WIN_C2, seed=seed).cpu().numpy()
    fx, fy = _ref_pixels(O.eval_group(G, 18, idx, seed=SEEDS.index(seed)), WIN_C2)
    err = np.hypot(p[:, 0] - fx, p[:, 1] - fy)
    near = (fx > -1) & (fx < WIN_C2[4] + 1) & (fy > -1) & (fy < WIN_C2[5] + 1)
    assert err[near].max() <= 0.25


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_seeded_image_is_histogram_of_own_bins(precision):
    depth, win = 12, WIN_C2
    tl = 4   # enough heads for the persistent kernel
    n = kl.num_words(depth)
    dropped = torch.zeros(1, dtype=torch.int64, device="cuda")
    img = kl.as_u32(kl.render(*C2, depth, win, precision=precision, seed="b", dropped=dropped,
                              tail_len=tl)).astype(np.int64)
    p = kl.eval_values(*C2, depth, np.arange(n, dtype=np.uint64), precision=precision, window=win,
                       seed="b", tail_len=tl).cpu().numpy()
    ref, drop = _bins_from_pixels(p[:, 0], p[:, 1], win)
    np.testing.assert_array_equal(img, ref)
    assert int(dropped.item()) == drop


@pytest.mark.parametrize("case", ["c1_tiling", "c2_d11"])
def test_all_seeds_fp64_image_matches_reference(case):
    """The paper's index-search loop: every word drawn once from each
    generator's fixed point."""
    if case == "c1_tiling":
        (ta, tb), depth, win, mind = C1, 8, wl.FUCHSIAN_TILING_D10.window.as_tuple(), 1
    else:
        (ta, tb), depth, win, mind = C2, 11, WIN_C2, 11
    dropped = torch.zeros(1, dtype=torch.int64, device="cuda")
    img = kl.as_u32(kl.render(ta, tb, depth, win, precision="fp64", min_depth=mind, seed="all",
                              dropped=dropped)).astype(np.int64)
    G = O.group_recipe(complex(ta), complex(tb))
    ref, drop, near = O.render_group(G, depth, win, seed=4, min_depth=mind, edge_tol=1e-7, nthreads=8)
    assert int(np.abs(img - ref.astype(np.int64)).sum()) <= 2 * near
    words = sum(kl.num_words(d) for d in range(mind, depth + 1))
    assert int(img.sum()) + int(dropped.item()) == 4 * words


@pytest.mark.parametrize("seed", ["B", "all"])
def test_render_many_with_seeds_equals_single_renders(seed):
    ta, tb, _ = wl.draw_param_sets(5, seed=31)
    depths = np.array([12, 13, 12, 14, 9])
    win = (-2.0, 2.0, -2.0, 2.0, 256, 256)
    many = kl.render_many(ta, tb, depths, win, seed=seed)
    for i in range(5):
        p = kl.plan_many(int(depths[i]), "fp32", win)   # the batch's split for the set
        one = kl.render(complex(ta[i]), complex(tb[i]), int(depths[i]), win, seed=seed,
                        tail_len=p["tail_len"], lane_len=p["lane_len"])
        assert torch.equal(many[i], one), i


# ---------------------------------------------------------------- explicit groups
@pytest.mark.parametrize("traces", ["c2", "double_cusp"])
def test_explicit_recipe_generators_give_the_recipe_values(traces):
    """The recipe's matrices given as an explicit group give the recipe's
    values (the double cusp: with seeds at infinity, infinite on the same
    words) and, at the double cusp, the same image."""
    ta, tb = C2 if traces == "c2" else (2 + 0j, 2 + 0j)
    _, g, _ = kl.generators(ta, tb)
    ab = np.stack([g[0], g[1]])
    idx = wl.sample_indices(kl.num_words(16), 20000, seed=2)
    for seed in ("own", "a", "B"):
        za = _z(kl.eval_group(ab, 16, idx, precision="fp64", seed=seed))
        zb = _z(kl.eval_values(ta, tb, 16, idx, precision="fp64", seed=seed))
        fin = np.isfinite(zb)
        np.testing.assert_array_equal(np.isfinite(za), fin)
        assert (np.abs(za[fin] - zb[fin]) / np.maximum(1, np.abs(zb[fin]))).max() < 1e-10
    if traces == "double_cusp":
        assert torch.equal(kl.render_group(ab, 14, WIN_DC), kl.render(ta, tb, 14, WIN_DC))


@pytest.mark.parametrize("seed", ["own", "b", "A"])
def test_maskit_fp64_values(seed):
    ab = kl.maskit_generators(MU)
    G = O.group_maskit(MU)
    s = -1 if seed == "own" else SEEDS.index(seed)
    idx = np.arange(kl.num_words(9), dtype=np.uint64)
    z = _z(kl.eval_group(ab, 9, idx, precision="fp64", seed=seed))
    zr = O.eval_group(G, 9, idx, seed=s)
    assert _rel_err(z, zr) < 1e-10
    idx = wl.sample_indices(kl.num_words(14), 20000, seed=4)
    assert _rel_err(_z(kl.eval_group(ab, 14, idx, precision="fp64", seed=seed)), O.eval_group(G, 14, idx, seed=s)) < 1e-10


def test_maskit_values_on_drawn_mu():
    """12 Maskit parameters drawn inside the slice (Re mu in [-1, 1], Im mu in
    [2.0, 2.6]) at depths 8..16, 2,000 sampled words each, the words' own
    seeds: FP64 values within the 1e-10 bar of the oracle's, FP32 pixel
    coordinates within 0.25 px of the oracle's near the window."""
    mus, depths = wl.draw_maskit_mu(12, seed=5)
    worst = 0.0
    for i, (mu, d) in enumerate(zip(mus, depths)):
        ab = kl.maskit_generators(complex(mu))
        G = O.group_maskit(complex(mu))
        d = int(d)
        idx = wl.sample_indices(kl.num_words(d), 2000, seed=200 + i)
        zr = O.eval_group(G, d, idx, seed=-1)
        assert _rel_err(_z(kl.eval_group(ab, d, idx, precision="fp64")), zr) < 1e-10, (i, mu, d)
        p = kl.eval_group(ab, d, idx, precision="fp32", window=WIN_MASKIT).cpu().numpy()
        fx, fy = _ref_pixels(zr, WIN_MASKIT)
        near = np.isfinite(fx) & np.isfinite(fy) & (fx > -1) & (fx < WIN_MASKIT[4] + 1) & (fy > -1) & \
            (fy < WIN_MASKIT[5] + 1)
        if near.any():
            err = np.hypot(p[near, 0] - fx[near], p[near, 1] - fy[near]).max()
            worst = max(worst, err)
            assert err <= 0.25, (i, mu, d, err)
    print(f"largest FP32 pixel error over the drawn parameters: {worst:.3e} px")


@pytest.mark.parametrize("seed", ["own", "b"])
def test_maskit_fp32_pixel_error(seed):
    ab = kl.maskit_generators(MU)
    G = O.group_maskit(MU)
    idx = wl.sample_indices(kl.num_words(14), 100000, seed=9)
    p = kl.eval_group(ab, 14, idx, precision="fp32", window=WIN_MASKIT, seed=seed).cpu().numpy()
    fx, fy = _ref_pixels(O.eval_group(G, 14, idx, seed=-1 if seed == "own" else SEEDS.index(seed)), WIN_MASKIT)
    near = np.isfinite(fx) & np.isfinite(fy) & (fx > -1) & (fx < WIN_MASKIT[4] + 1) & (fy > -1) & (fy < WIN_MASKIT[5] + 1)
    err = np.hypot(p[near, 0] - fx[near], p[near, 1] - fy[near])
    assert near.sum() > 1000 and err.max() <= 0.25, err.max()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_maskit_tiling_image_is_histogram_of_own_bins(precision):
    ab = kl.maskit_generators(MU)
    depth, win = 10, WIN_MASKIT
    dropped = torch.zeros(1, dtype=torch.int64, device="cuda")
    img = kl.as_u32(kl.render_group(ab, depth, win, precision=precision, min_depth=1, seed="b",
                                    dropped=dropped)).astype(np.int64)
    ref = np.zeros_like(img)
    drop = 0
    for d in range(1, depth + 1):
        p = kl.eval_group(ab, d, np.arange(kl.num_words(d), dtype=np.uint64), precision=precision, window=win,
                          seed="b").cpu().numpy()
        r, dr = _bins_from_pixels(p[:, 0], p[:, 1], win)
        ref += r
        drop += dr
    np.testing.assert_array_equal(img, ref)
    assert int(dropped.item()) == drop


def test_maskit_all_seeds_fp64_image_matches_reference():
    """The configuration of the paper's index-search figure at a smaller
    depth: Maskit's group, tiling mode, every generator's fixed point."""
    ab = kl.maskit_generators(MU)
    depth, win = 9, WIN_MASKIT
    dropped = torch.zeros(1, dtype=torch.int64, device="cuda")
    img = kl.as_u32(kl.render_group(ab, depth, win, precision="fp64", min_depth=1, seed="all",
                                    dropped=dropped)).astype(np.int64)
    ref, drop, near = O.render_group(O.group_maskit(MU), depth, win, seed=4, min_depth=1, edge_tol=1e-7,
                                     nthreads=8)
    assert int(np.abs(img - ref.astype(np.int64)).sum()) <= 2 * near
    assert int(img.sum()) + int(dropped.item()) == 4 * sum(kl.num_words(d) for d in range(1, depth + 1))
    assert int(dropped.item()) == drop or abs(int(dropped.item()) - drop) <= near


DC = (2 + 0j, 2 + 0j)
WIN_DC = (-1.25, 1.25, -4.0, 4.0, 320, 1024)   # the gasket's strip |Re z| <= 1, four translates


def test_double_cusp_values_and_images():
    """ta = tb = 2, the double cusp (the Apollonian gasket).  The recipe's a
    is the translation z -> z + 2i, so a and A take their seeds at infinity.
    Heads that are powers of a fix infinity, and the suffix tables hold
    points at infinity: the recipe path runs the homogeneous and ratio forms.
    The checks:
      * FP64 values within 1e-10 of the oracle's, and infinite on the same
        words (a^d and A^d);
      * FP32 pixel coordinates within 0.25 px;
      * limit-set and tiling images in both precisions equal the histograms
        of their own bins;
      * the FP64 images are within the edge bar of the oracle's."""
    W, H = WIN_DC[4], WIN_DC[5]
    _, _, fix = kl.generators(*DC)
    assert np.isinf(fix[0]) and np.isinf(fix[2]) and abs(fix[1] + 1j) < 1e-14 and abs(fix[3] + 1j) < 1e-14
    worst = 0.0
    for d in (1, 5, 9, 14, 22):
        n = kl.num_words(d)
        idx = np.arange(n, dtype=np.uint64) if n <= 50000 else wl.sample_indices(n, 20000, seed=d)
        z = _z(kl.eval_values(*DC, d, idx, precision="fp64"))
        zr = O.eval_values(*DC, d, idx)
        np.testing.assert_array_equal(np.isfinite(z), np.isfinite(zr), err_msg=f"depth {d}")
        assert _rel_err(z, zr) < 1e-10, d
        p = kl.eval_values(*DC, d, idx, precision="fp32", window=WIN_DC).cpu().numpy()
        fin = np.isfinite(zr)
        fx, fy = _ref_pixels(zr[fin], WIN_DC)
        near = (fx > -1) & (fx < W + 1) & (fy > -1) & (fy < H + 1)
        err = np.maximum(np.abs(p[fin, 0] - fx), np.abs(p[fin, 1] - fy))[near]
        worst = max(worst, float(err.max()))
    print(f"double cusp: largest FP32 error {worst:.2e} px")
    assert worst < 0.25
    for depth, mind in ((12, 12), (10, 1)):
        for precision in ("fp32", "fp64"):
            dropped = torch.zeros(1, dtype=torch.int64, device="cuda")
            img = kl.as_u32(kl.render(*DC, depth, WIN_DC, precision=precision, min_depth=mind,
                                      dropped=dropped)).astype(np.int64)
            ref, drop = np.zeros((H, W), np.int64), 0
            for d in range(mind, depth + 1):
                q = kl.eval_values(*DC, d, np.arange(kl.num_words(d), dtype=np.uint64), precision=precision,
                                   window=WIN_DC).cpu().numpy()
                r, dd = _bins_from_pixels(q[:, 0], q[:, 1], WIN_DC)
                ref += r
                drop += dd
            np.testing.assert_array_equal(img, ref, err_msg=f"{precision} depth {depth} from {mind}")
            assert int(dropped.item()) == drop
        oref, _, near = O.render(*DC, depth, WIN_DC, min_depth=mind, edge_tol=1e-7, nthreads=8)
        diff = int(np.abs(img - oref.astype(np.int64)).sum())
        assert diff <= 2 * near, (depth, mind, diff, near)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_double_cusp_in_a_batch_equals_single_renders(precision):
    """A batch that mixes the double cusp (seeds at infinity, homogeneous
    suffix tables) with ordinary sets at depths 9 to 17 draws each image bit
    for bit as a single render of that set under the batch's split.  The
    depth-17 sets go to the persistent batched kernel."""
    ta = np.array([2, wl.C2_TA, 2, wl.C1_TA, 2], complex)
    tb = np.array([2, wl.C2_TB, 2, wl.C1_TB, 2], complex)
    depth = np.array([17, 12, 9, 17, 14], np.int32)
    win = WIN_DC
    dropped = torch.zeros(len(ta), dtype=torch.int64, device="cuda")
    imgs = kl.render_many(ta, tb, depth, win, precision=precision, dropped=dropped)
    for i in range(len(ta)):
        d1 = torch.zeros(1, dtype=torch.int64, device="cuda")
        p = kl.plan_many(int(depth[i]), precision, win)
        single = kl.render(complex(ta[i]), complex(tb[i]), int(depth[i]), win, precision=precision, dropped=d1,
                           tail_len=p["tail_len"], lane_len=p["lane_len"])
        assert torch.equal(imgs[i], single), i
        assert int(dropped[i].item()) == int(d1.item())
        assert int(kl.as_u32(imgs[i]).sum()) + int(d1.item()) == kl.num_words(int(depth[i]))
