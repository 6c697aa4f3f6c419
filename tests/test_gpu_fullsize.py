"""Parity at the full sizes, in the launch configurations the benchmark times.

* The depth-18 FP32 image of the timed render (516,560,652 words, 2048^2 over
  [-1.5, 1.5]^2) equals, bin for bin, the histogram of kl_eval's pixel
  coordinates of every one of its words under the same split and arithmetic.
* The same image against the oracle's full FP64 render: the two differ only
  by words the oracle places within 1e-3 px of a bin edge (the FP32 path's
  measured per-word error stays below 5e-4 px), so the L1 difference is at
  most twice their number.
* The FP64 depth-18 image against the oracle, with the edge band at 1e-7 px.
* The per-word pixel error on 10^6 indices drawn with PCG64 seed 0, at depth
  18 (2048^2) and depth 22 (4096^2): at most 0.25 px.
* Four sets of the 256-set batch (one of depth 18, one of depth 12 and two
  more), each in full, against the histogram of its own words' coordinates.

A word's value is the orbit point of the seed under the word's maps applied
right to left (Section 1), drawn into the image (Section 6, index search).
"""
import os

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1709_08018_amd import workloads as wl

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1709_08018_amd import kl

D18 = wl.QUASIFUCHSIAN_D18
D22 = wl.QUASIFUCHSIAN_D22
# the oracle's full depth-18 render, on the host's CPU share
NTHREADS = max(1, min(len(os.sched_getaffinity(0)), 16))
# edge band of the FP32 image comparison (px), above every measured
# per-word error of the pole form (max 1.7e-4 px at depth 18, 4.8e-4 at 22)
FP32_EDGE_PX = 1e-3


def own_bins_histogram(ta, tb, depth, win, precision="fp32", chunk=1 << 25, **opts):
    """Histogram of the renderer's own pixel coordinates (kl_eval with the
    window) of every word of `depth`, binned on the GPU by the renderer's
    rule: inside when 0 <= px < W and 0 <= py < H as IEEE comparisons (-0
    counts as 0; NaN and infinities are outside), bin floor(py) * W +
    floor(px)."""
    n = kl.num_words(depth)
    W, H = win[4], win[5]
    hist = torch.zeros(W * H, dtype=torch.int64, device="cuda")
    dropped = 0
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        idx = torch.arange(a, b, dtype=torch.int64, device="cuda")
        p = kl.eval_values(ta, tb, depth, idx, precision=precision, window=win, **opts)
        px, py = p[:, 0], p[:, 1]
        ok = (px >= 0) & (px < W) & (py >= 0) & (py < H)
        key = torch.floor(py[ok]).to(torch.int64) * W + torch.floor(px[ok]).to(torch.int64)
        hist += torch.bincount(key, minlength=W * H)
        dropped += int((~ok).sum().item())
        del idx, p, px, py, ok, key
    return hist.view(H, W), dropped


def _image(t):
    return torch.as_tensor(kl.as_u32(t).astype(np.int64))


def test_d18_fp32_image_is_histogram_of_all_its_words():
    win = D18.window.as_tuple()
    n = kl.num_words(18)
    dropped = torch.zeros(1, dtype=torch.int64, device="cuda")
    img = kl.render(D18.ta, D18.tb, 18, win, dropped=dropped)
    ref, drop = own_bins_histogram(D18.ta, D18.tb, 18, win)
    got = _image(img)
    diff = int((got - ref.cpu()).abs().sum())
    print(f"d18 FP32: {int(got.sum())} counts, {drop} dropped; L1 vs own-bin histogram {diff}")
    assert diff == 0
    assert int(dropped.item()) == drop
    assert int(got.sum()) + drop == n


@pytest.mark.parametrize("precision,edge", [("fp32", FP32_EDGE_PX), ("fp64", 1e-7)])
def test_d18_image_against_full_oracle_render(precision, edge):
    win = D18.window.as_tuple()
    img = kl.as_u32(kl.render(D18.ta, D18.tb, 18, win, precision=precision)).astype(np.int64)
    ref, drop, near = O.render(D18.ta, D18.tb, 18, win, edge_tol=edge, nthreads=NTHREADS)
    diff = int(np.abs(img - ref.astype(np.int64)).sum())
    print(f"d18 {precision}: L1 vs oracle {diff} of {int(ref.sum())} counts; {near} words within {edge} px "
          f"of a bin edge")
    assert diff <= 2 * near


@pytest.mark.parametrize("W", [D18, D22], ids=["d18", "d22"])
def test_seeded_million_index_pixel_error(W):
    win = W.window.as_tuple()
    n = kl.num_words(W.depth)
    idx = wl.sample_indices(n, 1_000_000, seed=0)
    p = kl.eval_values(W.ta, W.tb, W.depth, idx, precision="fp32", window=win).cpu().numpy()
    z = O.eval_values(W.ta, W.tb, W.depth, idx)
    x0, x1, y0, y1, Wd, Hd = win
    fx, fy = (z.real - x0) * Wd / (x1 - x0), (z.imag - y0) * Hd / (y1 - y0)
    near = (fx > -1) & (fx < Wd + 1) & (fy > -1) & (fy < Hd + 1)
    err = np.hypot(p[near, 0] - fx[near], p[near, 1] - fy[near])
    print(f"{W.name}: FP32 pixel error over {int(near.sum())} of 10^6 sampled words near the window: "
          f"max {err.max():.3e} p99 {np.quantile(err, 0.99):.3e} mean {err.mean():.3e}")
    assert near.sum() > 300_000
    assert err.max() <= 0.25
    # the FP32 image comparison above relies on this band
    assert err.max() < FP32_EDGE_PX


def test_batch256_depth18_set_is_histogram_of_all_its_words():
    ta, tb, depth = wl.batch256(seed=0)
    win = wl.BATCH_WINDOW.as_tuple()
    dropped = torch.zeros(len(ta), dtype=torch.int64, device="cuda")
    imgs = kl.render_many(ta, tb, depth, win, dropped=dropped)
    for i in (int(np.argmax(depth)), int(np.argmin(depth)), 17, 200):
        d = int(depth[i])
        p = kl.plan_many(d, "fp32", win)   # the words' values under the batch's split for the set
        ref, drop = own_bins_histogram(complex(ta[i]), complex(tb[i]), d, win, tail_len=p["tail_len"],
                                       lane_len=p["lane_len"])
        got = _image(imgs[i])
        assert int((got - ref.cpu()).abs().sum()) == 0, (i, d)
        assert int(dropped[i].item()) == drop, (i, d)
