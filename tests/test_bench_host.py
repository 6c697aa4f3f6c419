"""Host logic of bench.py: the HBM traffic figure is read from the committed
counter summary only when that summary was taken on the current kernel
source and split; the oracle baselines of the tiling and batch legs compare
what they are given with the oracle's own images."""
import hashlib

import bench

SPLIT = {"prefix_len": 9, "lane_len": 3, "tail_len": 6}


def _summary(tmp_path, src_hash, split="prefix 9, lane 3, tail 6 letters; 32 waves per CU"):
    p = tmp_path / "pmc.txt"
    p.write_text("# HBM traffic (KiB per dispatch)\n"
                 "# command: rocprofv3 --pmc FETCH_SIZE -- python3 bench.py\n"
                 f"kernels.hip sha256[:16]: {src_hash}\n"
                 f"split: {split}\n"
                 "render_kernel FETCH_SIZE KiB per dispatch (mean of 4): 1204.7\n"
                 "hbm_bytes_per_launch: 40753009\n")
    return str(p)


def _current_hash():
    return hashlib.sha256(open(bench.KERNEL_SRC, "rb").read()).hexdigest()[:16]


def test_traffic_read_when_source_and_split_match(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PMC_SUMMARY", _summary(tmp_path, _current_hash()))
    assert bench._traffic_from_profile(SPLIT) == 40753009.0


def test_traffic_null_for_another_source(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PMC_SUMMARY", _summary(tmp_path, "0" * 16))
    assert bench._traffic_from_profile(SPLIT) is None


def test_traffic_null_for_another_split(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PMC_SUMMARY", _summary(tmp_path, _current_hash(), "prefix 8, lane 4, tail 6 letters"))
    assert bench._traffic_from_profile(SPLIT) is None


def test_traffic_null_without_summary(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PMC_SUMMARY", str(tmp_path / "absent.txt"))
    assert bench._traffic_from_profile(SPLIT) is None


def test_multi_gpu_request_exits_with_a_message():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "single GPU" in (r.stdout + r.stderr)


def test_valu_figure_read_with_the_same_checks(tmp_path, monkeypatch):
    p = tmp_path / "valu.txt"
    p.write_text(f"kernels.hip sha256[:16]: {_current_hash()}\n"
                 "split: prefix 9, lane 3, tail 6 letters; 32 waves per CU\n"
                 "VALU instructions per wave-word (64 words): 20.49\n")
    monkeypatch.setattr(bench, "VALU_SUMMARY", str(p))
    assert bench._valu_per_wave_word(SPLIT) == 20.49
    p.write_text("kernels.hip sha256[:16]: 0000000000000000\nsplit: prefix 9, lane 3, tail 6 letters\n"
                 "VALU instructions per wave-word (64 words): 20.49\n")
    assert bench._valu_per_wave_word(SPLIT) is None


def test_issue_fraction_read_from_the_counter_summary(tmp_path, monkeypatch):
    p = tmp_path / "valu.txt"
    p.write_text(f"kernels.hip sha256[:16]: {_current_hash()}\n"
                 "split: prefix 9, lane 3, tail 6 letters; 32 waves per CU\n"
                 "VALU issue fraction (SQ_INSTS_VALU x 4 cycles / (GRBM_GUI_ACTIVE / 8 XCDs x 1024 SIMDs), "
                 "per dispatch): 0.977 (median of 684; min 0.926, max 1.005)\n")
    monkeypatch.setattr(bench, "VALU_SUMMARY", str(p))
    assert bench._profile_value(bench.VALU_SUMMARY, "VALU issue fraction", SPLIT) == 0.977


def test_tiling_baseline_compares_the_image_with_the_oracle():
    """The tiling leg's oracle baseline: L1 0 for the oracle's own FP64
    image, and every count for an empty image."""
    import numpy as np

    from oracle import oracle as O
    from paper_1709_08018_amd import workloads as wl

    W = wl.FUCHSIAN_TILING_D10
    own, _, _ = O.render(W.ta, W.tb, W.depth, W.window.as_tuple(), min_depth=1)
    words = sum(O.num_words(d) for d in range(1, W.depth + 1))
    r = bench.cpu_baseline_tiling(W, words, own.astype(np.int64))
    assert r["fp64_l1_vs_oracle"] == 0 and r["kind"] == "oracle"
    r = bench.cpu_baseline_tiling(W, words, np.zeros_like(own, dtype=np.int64))
    assert r["fp64_l1_vs_oracle"] == int(own.sum())


def test_batch_baseline_samples_every_nth_set():
    """The batch leg's oracle baseline renders sets 0, 16, ..., compares each
    with the batched image of the same set, and reports the bar."""
    import numpy as np

    from oracle import oracle as O
    from paper_1709_08018_amd import workloads as wl

    ta, tb, depth = wl.batch256(seed=0)
    win = wl.BATCH_WINDOW
    # shallow stand-ins keep the oracle's work small; the sampling is what is checked
    depth = np.full_like(depth, 6)
    imgs = np.zeros((len(ta), win.height, win.width), np.uint32)
    for i in range(0, len(ta), 64):
        imgs[i] = O.render(complex(ta[i]), complex(tb[i]), 6, win.as_tuple())[0]
    r = bench.cpu_baseline_batch(ta, tb, depth, win, imgs, every=64)
    assert r["sample"].startswith("sets 0, 64, ... every 64th of the batch (4 sets")
    assert r["l1_vs_oracle"] == 0 and r["within_bar"]
    imgs[64] = 0
    r = bench.cpu_baseline_batch(ta, tb, depth, win, imgs, every=64)
    assert r["l1_vs_oracle"] == int(O.render(complex(ta[64]), complex(tb[64]), 6, win.as_tuple())[0].sum())
