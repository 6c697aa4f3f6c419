"""The batch autotuner (kl_autotune_many): the plans it keeps make the
batched render no slower than the planner's, every later batched render of
that image size takes them, and under them every image is the histogram of
its own words' coordinates (kl_eval with the same split) and its words
stay within 0.25 px of the oracle's FP64 values."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1709_08018_amd import workloads as wl

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1709_08018_amd import kl

# an image size no other test renders at, so that the tuned plans (kept for
# the rest of the process) reach no other test
WIN = (-2.0, 2.0, -2.0, 2.0, 320, 200)


def _own_bins(p, win):
    W, H = win[4], win[5]
    px, py = p[:, 0], p[:, 1]
    ok = (px >= 0) & (px < W) & (py >= 0) & (py < H)
    img = np.zeros(W * H, np.int64)
    np.add.at(img, np.floor(py[ok]).astype(np.int64) * W + np.floor(px[ok]).astype(np.int64), 1)
    return img.reshape(H, W), int((~ok).sum())


def test_batch_tuned_plans_against_own_bins_and_oracle():
    ta, tb, depth = wl.draw_param_sets(24, seed=31, depth_range=(11, 14))
    plans, best, default = kl.autotune_many(ta, tb, depth, WIN)
    print(f"batch of 24: planner {default:.3f} ms, tuned {best:.3f} ms")
    assert best <= default
    for i, d in enumerate(depth):
        p = kl.plan_many(int(d), "fp32", WIN)
        assert (p["tail_len"], p["lane_len"]) == (plans[i]["tail_len"], plans[i]["lane_len"])
        assert p["tail_len"] + p["lane_len"] + p["prefix_len"] == d
    dropped = torch.zeros(len(ta), dtype=torch.int64, device="cuda")
    imgs = kl.render_many(ta, tb, depth, WIN, dropped=dropped)
    for i in range(len(ta)):
        d = int(depth[i])
        n = kl.num_words(d)
        split = dict(tail_len=plans[i]["tail_len"], lane_len=plans[i]["lane_len"])
        pts = kl.eval_values(ta[i], tb[i], d, np.arange(n, dtype=np.uint64), window=WIN, **split).cpu().numpy()
        ref, drop = _own_bins(pts, WIN)
        np.testing.assert_array_equal(kl.as_u32(imgs[i]).astype(np.int64), ref, err_msg=str(i))
        assert int(dropped[i].item()) == drop
        # sampled words within 0.25 px of the oracle under the tuned split
        idx = wl.sample_indices(n, 2000, seed=i)
        z = O.eval_values(complex(ta[i]), complex(tb[i]), d, idx)
        x0, x1, y0, y1, W, H = WIN
        fx, fy = (z.real - x0) * W / (x1 - x0), (z.imag - y0) * H / (y1 - y0)
        sel = pts[idx.astype(np.int64)]
        near = (fx > -1) & (fx < W + 1) & (fy > -1) & (fy < H + 1)
        assert np.hypot(sel[near, 0] - fx[near], sel[near, 1] - fy[near]).max() <= 0.25, i
    # the same plans given to single renders draw the same images
    for i in (0, 7, 23):
        single = kl.render(ta[i], tb[i], int(depth[i]), WIN, tail_len=plans[i]["tail_len"],
                           lane_len=plans[i]["lane_len"])
        assert torch.equal(single, imgs[i]), i
