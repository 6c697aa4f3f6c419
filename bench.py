#!/usr/bin/env python3
"""Benchmark of the indexed Kleinian-attractor renderer on one MI355X.

Workload (one step): the limit set of the quasi-Fuchsian group with traces
ta = 1.91 + 0.05i, tb = 2 at depth 18 -- all 4*3^17 = 516,560,652 reduced
words, decoded from their indices, evaluated right to left from their seeds
(FP64 prefixes, FP32 suffix maps) and binned into a 2048 x 2048 uint32 image
over [-1.5, 1.5]^2.  A step is one kl_render_ex call: image clear, prefix
and suffix tables, persistent renderer, per-word ragged end.

Prints one JSON line: whole-job words/s (Gwords/s), the renderer kernel's
FP32 roofline position (its average duration measured with HIP events on
its own stream), and the CPU reference timed on this host's cores.

    python bench.py [--gpus 1] [--steps 200] [--warmup 400] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gwords/s and VALU roofline fraction at depth 18; surrogate vs plain scan time @IoU≥0.95"
# algorithmic FP32 work per word of the renderer, the head's map in pole
# form P + Q / (y + S) applied to the suffix point y: u = y + S (2 flops),
# |u|^2 (3), reciprocal (1), per pixel coordinate one product and two FMAs (10)
FLOPS_PER_WORD = 16
FP32_PEAK_TFLOPS = 157.3  # MI355X FP32 vector peak (counts packed FMA)
# the GPU clock ramps up over the first ~100 ms of work: before the counted
# warm-up steps, steps run untimed until this much wall time has passed
CLOCK_RAMP_MS = 300.0
FP64_PEAK_TFLOPS = 78.6   # MI355X FP64 vector peak
EVENT_EVERY = 10
PMC_SUMMARY = os.path.join(ROOT, "profiles", "render_kernel_quasifuchsian_d18_pmc.txt")
VALU_SUMMARY = os.path.join(ROOT, "profiles", "render_kernel_quasifuchsian_d18_valu.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_1709_08018_amd", "csrc", "kernels.hip")


def _hip():
    lib = ctypes.CDLL("libamdhip64.so.7")  # the runtime torch already loaded
    lib.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
    lib.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
    lib.hipEventDestroy.argtypes = [ctypes.c_void_p]
    return lib


def _profile_value(path, key, plan):
    """A figure from a committed counter summary, if the summary was taken on
    the current kernel source and split; else None."""
    if not os.path.exists(path):
        return None
    src_hash = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]
    vals = {}
    for line in open(path):
        if ": " in line:
            k, v = line.split(": ", 1)
            vals[k.split(" (")[0].strip() if k.startswith("VALU issue fraction") else k.strip()] = v.strip()
    if vals.get("kernels.hip sha256[:16]") != src_hash:
        return None
    split = f"prefix {plan['prefix_len']}, lane {plan['lane_len']}, tail {plan['tail_len']}"
    if split not in vals.get("split", ""):
        return None
    try:
        return float(vals[key].split()[0])
    except (KeyError, ValueError):
        return None


def _traffic_from_profile(plan):
    """HBM bytes per launch (FETCH_SIZE and WRITE_SIZE, copy-calibrated)."""
    return _profile_value(PMC_SUMMARY, "hbm_bytes_per_launch", plan)


def _valu_per_wave_word(plan):
    """VALU instructions per 64 words (SQ_INSTS_VALU over the words)."""
    return _profile_value(VALU_SUMMARY, "VALU instructions per wave-word (64 words)", plan)


# The host this runs on grants one process a CPU share of 16 cores per GPU,
# whatever the machine reports; the oracle's threaded render uses at most
# that share.
CPU_SHARE = 16


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl_obj, seconds_hint: float):
    """The oracle timed on this host: the full workload on every core of the
    process's CPU share (one thread per core, contiguous index ranges), and
    one thread on a contiguous sixteenth of the index space."""
    from oracle import oracle as ref

    affinity = len(os.sched_getaffinity(0))
    threads = min(affinity, CPU_SHARE)
    n = ref.num_words(wl_obj.depth)
    win = wl_obj.window.as_tuple()
    t0 = time.perf_counter()
    img, dropped, _ = ref.render(wl_obj.ta, wl_obj.tb, wl_obj.depth, win, nthreads=threads)
    dt = time.perf_counter() - t0
    n1 = n // 16
    t0 = time.perf_counter()
    ref.render(wl_obj.ta, wl_obj.tb, wl_obj.depth, win, first=n // 3, count=n1, nthreads=1)
    dt1 = time.perf_counter() - t0
    return {"value": n / dt / 1e9, "unit": "Gwords/s", "cores": threads, "kind": "oracle",
            "sample": f"the full workload ({n} words, depth {wl_obj.depth}), FP64 depth-first walk, "
                      f"{threads} threads over contiguous index ranges, {dt:.2f} s",
            "single_thread": {"value": n1 / dt1 / 1e9, "unit": "Gwords/s", "words": n1, "seconds": round(dt1, 3),
                              "sample": f"words [{n // 3}, {n // 3 + n1}) of depth {wl_obj.depth}, one thread"},
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(), "affinity_cpus": affinity,
            "cpu_share": CPU_SHARE}, img, dropped


# The oracle, timed beside the GPU legs: each returns a leg's "cpu_baseline"
# object, with the leg's GPU image (or sampled values) compared against it.
def _oracle():
    from oracle import oracle as ref
    return ref


def cpu_baseline_d22(W, idx, p):
    """The FP32 path's pixel error on the sampled words against the oracle's
    FP64 values, and the oracle's rate on that sample."""
    import numpy as np
    ref = _oracle()
    t0 = time.perf_counter()
    z = ref.eval_values(W.ta, W.tb, W.depth, idx)
    dt = time.perf_counter() - t0
    x0, x1, y0, y1, Wd, Hd = W.window.as_tuple()
    fx, fy = (z.real - x0) * Wd / (x1 - x0), (z.imag - y0) * Hd / (y1 - y0)
    near = (fx > -1) & (fx < Wd + 1) & (fy > -1) & (fy < Hd + 1)
    err = np.hypot(p[near, 0] - fx[near], p[near, 1] - fy[near])
    return {"kind": "oracle", "value": round(len(idx) / dt / 1e9, 5), "unit": "Gwords/s", "cores": 1,
            "sample": f"{len(idx)} sampled words, values by random access",
            "fp32_pixel_error": {"max": float(err.max()), "p99": float(np.quantile(err, 0.99)),
                                 "mean": float(err.mean()), "words": int(near.sum())}}


def cpu_baseline_maskit(W, words, img):
    """The oracle's render of the same tiling (all four seeds), timed, and the
    GPU's FP64 image against it."""
    import numpy as np
    ref = _oracle()
    threads = min(len(os.sched_getaffinity(0)), CPU_SHARE)
    t0 = time.perf_counter()
    ref_img, _, near = ref.render_group(ref.group_maskit(W.ta), W.depth, W.window.as_tuple(), seed=4,
                                        min_depth=W.min_depth, edge_tol=1e-7, nthreads=threads)
    dt = time.perf_counter() - t0
    return {"kind": "oracle", "value": round(4 * words / dt / 1e9, 4), "unit": "Gpoints/s", "cores": threads,
            "sample": "the full workload", "seconds": round(dt, 3),
            "fp64_l1_vs_oracle": int(np.abs(img - ref_img.astype(np.int64)).sum()),
            "oracle_near_edge_words": int(near)}


def cpu_baseline_cayley_t11(ta, tb, depth, win, words, img):
    """The oracle's render of the reduced words (the words of Table 2), timed,
    and the table path's image against it."""
    import numpy as np
    ref = _oracle()
    threads = min(len(os.sched_getaffinity(0)), CPU_SHARE)
    t0 = time.perf_counter()
    rimg, _, near = ref.render(ta, tb, depth, win, edge_tol=1e-7, nthreads=threads)
    dt = time.perf_counter() - t0
    return {"kind": "oracle", "value": round(words / dt / 1e9, 4), "unit": "Gwords/s", "cores": threads,
            "sample": "the full workload", "seconds": round(dt, 3),
            "l1_vs_oracle": int(np.abs(img - rimg.astype(np.int64)).sum()), "oracle_near_edge_words": int(near)}


def cpu_baseline_cayley_modular(table, maps, win, words, img):
    """The oracle's table render of the same tiling (every symbol's fixed
    point), timed, and the GPU image against it."""
    import numpy as np
    ref = _oracle()
    t0 = time.perf_counter()
    rimg, _, near = ref.cayley_render(ref.Cayley(table, maps), 40, win, seed=3, min_depth=1, edge_tol=1e-7)
    dt = time.perf_counter() - t0
    return {"kind": "oracle", "value": round(3 * words / dt / 1e9, 4), "unit": "Gpoints/s", "cores": 1,
            "sample": "the full workload", "seconds": round(dt, 3),
            "l1_vs_oracle": int(np.abs(img - rimg.astype(np.int64)).sum()), "oracle_near_edge_words": int(near)}


def cpu_baseline_batch(ta, tb, depth, win, imgs, every=16):
    """The oracle's renders of every `every`-th set of the batch, timed on
    the process's CPU share, and the batched FP32 images of those sets
    against them (L1 within twice the words the oracle places within
    1e-3 px of a bin edge)."""
    import numpy as np
    ref = _oracle()
    threads = min(len(os.sched_getaffinity(0)), CPU_SHARE)
    sets = list(range(0, len(ta), every))
    win = win.as_tuple()
    words, l1, near, dt = 0, 0, 0, 0.0
    for i in sets:
        t0 = time.perf_counter()
        rimg, _, nr = ref.render(complex(ta[i]), complex(tb[i]), int(depth[i]), win, edge_tol=1e-3, nthreads=threads)
        dt += time.perf_counter() - t0
        words += ref.num_words(int(depth[i]))
        l1 += int(np.abs(imgs[i].astype(np.int64) - rimg.astype(np.int64)).sum())
        near += int(nr)
    return {"kind": "oracle", "value": round(words / dt / 1e9, 4), "unit": "Gwords/s", "cores": threads,
            "sample": f"sets {sets[0]}, {sets[1]}, ... every {every}th of the batch ({len(sets)} sets, {words} words), "
                      f"FP64 depth-first walk, {dt:.2f} s",
            "l1_vs_oracle": l1, "oracle_near_edge_words": near, "within_bar": l1 <= 2 * near}


def cpu_baseline_tiling(W, words, img):
    """The oracle's render of the whole tiling, timed, and the GPU's FP64
    image against it."""
    import numpy as np
    ref = _oracle()
    threads = min(len(os.sched_getaffinity(0)), CPU_SHARE)
    t0 = time.perf_counter()
    rimg, _, near = ref.render(W.ta, W.tb, W.depth, W.window.as_tuple(), min_depth=1, edge_tol=1e-7, nthreads=threads)
    dt = time.perf_counter() - t0
    return {"kind": "oracle", "value": round(words / dt / 1e9, 4), "unit": "Gwords/s", "cores": threads,
            "sample": "the full workload", "seconds": round(dt, 3),
            "fp64_l1_vs_oracle": int(np.abs(img - rimg.astype(np.int64)).sum()), "oracle_near_edge_words": int(near)}


def cpu_baseline_decode(first, depth, rows, got):
    """The oracle's unranking of the sampled rows, timed, against the kernel's."""
    import numpy as np
    ref = _oracle()
    t0 = time.perf_counter()
    want = np.array([ref.unrank(first + r, depth) for r in rows])
    dt = time.perf_counter() - t0
    return {"kind": "oracle", "value": round(len(rows) / dt / 1e9, 9), "unit": "Gwords/s", "cores": 1,
            "sample": f"{len(rows)} words by random access", "rows_equal": bool(np.array_equal(want, got))}


def _time(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def leg_d22(args):
    """Depth 22 streamed by index range: FP32 suffix path vs full FP64, and the
    FP32 path's pixel error against the CPU reference on 10^6 sampled words."""
    import numpy as np
    import torch

    from paper_1709_08018_amd import kl
    from paper_1709_08018_amd import workloads as wl

    W = wl.QUASIFUCHSIAN_D22
    n = kl.num_words(W.depth)
    chunks = 8
    cuts = [n * i // chunks for i in range(chunks + 1)]
    image = kl.new_image(W.window)
    dropped = torch.zeros(1, dtype=torch.int64, device="cuda")
    res = {}
    for prec in ("fp32", "fp64"):
        def run():
            for a, b in zip(cuts[:-1], cuts[1:]):
                kl.render(W.ta, W.tb, W.depth, W.window, image=image, precision=prec, first=a, count=b - a,
                          accumulate=a > 0, dropped=dropped)
        ms = _time(run, max(1, args.steps // 4), 1)
        h = kl.as_u32(image).astype(np.int64)
        assert int(h.sum()) + int(dropped.item()) == n
        res[prec] = {"ms": round(ms, 3), "gwords_per_s": round(n / ms / 1e6, 2), "max_bin": int(h.max()),
                     "valu_frac": _valu_frac(n, ms, prec)}
    idx = wl.sample_indices(n, 1_000_000, seed=0)
    p = kl.eval_values(W.ta, W.tb, W.depth, idx, precision="fp32", window=W.window).cpu().numpy()
    return {"workload": W.name, "words": n, "chunks": chunks, **res,
            "cpu_baseline": cpu_baseline_d22(W, idx, p)}


def _valu_frac(words, ms, precision):
    """FLOPS_PER_WORD x words in ms, as a fraction of the vector peak of the
    precision the suffix points are mapped in."""
    peak = FP64_PEAK_TFLOPS if precision == "fp64" else FP32_PEAK_TFLOPS
    return {"of_peak_tflops": peak, "frac": round(FLOPS_PER_WORD * words / (ms * 1e-3) / 1e12 / peak, 4)}


def _kernel_ms(render, reps):
    """Mean persistent-kernel time in ms of render(kernel_events=...) over
    reps calls, from a HIP event pair recorded around its launches."""
    import ctypes

    hip = _hip()
    ev = []
    for _ in range(2):
        e = ctypes.c_void_p()
        if hip.hipEventCreate(ctypes.byref(e)) != 0:
            raise RuntimeError("hipEventCreate failed")
        ev.append(e.value)
    total = 0.0
    for _ in range(reps):
        render(kernel_events=(ev[0], ev[1]))
        hip.hipEventSynchronize(ctypes.c_void_p(ev[1]))
        ms = ctypes.c_float()
        hip.hipEventElapsedTime(ctypes.byref(ms), ev[0], ev[1])
        total += ms.value
    for e in ev:
        hip.hipEventDestroy(e)
    return total / reps


def leg_bounded(args):
    """Block bounds (kl_opts.block_bounds) on the depth-18 workload, FP32 and
    FP64: each head bounds where each group of 27 suffixes lands, and only
    groups whose bound spans more than one bin are evaluated word by word.
    Step time and persistent-kernel time against the per-word renderer on
    the same words, the two images and dropped counts compared bin for bin;
    and depth 22 streamed in 8 index ranges, both ways."""
    import numpy as np
    import torch

    from paper_1709_08018_amd import kl
    from paper_1709_08018_amd import workloads as wl

    out = {"workload": "block_bounds"}
    for W, chunks, prec in ((wl.QUASIFUCHSIAN_D18, 1, "fp32"), (wl.QUASIFUCHSIAN_D18, 1, "fp64"),
                            (wl.QUASIFUCHSIAN_D22, 8, "fp32")):
        n = kl.num_words(W.depth)
        cuts = [n * i // chunks for i in range(chunks + 1)]
        res = {"words": n, "chunks": chunks}
        imgs = {}
        for bounded in (False, True):
            image = kl.new_image(W.window)
            dropped = torch.zeros(1, dtype=torch.int64, device="cuda")

            def run(dropped=None, **kw):
                for a, b in zip(cuts[:-1], cuts[1:]):
                    rng = {} if chunks == 1 else {"first": a, "count": b - a}
                    kl.render(W.ta, W.tb, W.depth, W.window, image=image, accumulate=a > 0, dropped=dropped,
                              block_bounds=bounded, precision=prec, **rng, **kw)
            steps = max(2, args.steps // (4 * chunks))
            ms = _time(run, steps, max(2, steps // 4))
            key = "bounded" if bounded else "per_word"
            res[key] = {"ms": round(ms, 4), "gwords_per_s": round(n / ms / 1e6, 1)}
            if chunks == 1:
                res[key]["kernel_ms"] = round(_kernel_ms(lambda **kw: run(**kw), steps), 4)
                if not bounded:
                    res[key]["kernel_valu_frac"] = _valu_frac(n, res[key]["kernel_ms"], prec)
            run(dropped=dropped)
            imgs[bounded] = (kl.as_u32(image).astype(np.int64), int(dropped.item()))
        res["images_equal"] = bool(np.array_equal(imgs[False][0], imgs[True][0]))
        res["dropped_equal"] = imgs[False][1] == imgs[True][1]
        res["speedup"] = round(res["per_word"]["ms"] / res["bounded"]["ms"], 2)
        assert res["images_equal"] and res["dropped_equal"], "block bounds changed the image"
        out[W.name if prec == "fp32" else W.name + "_fp64"] = res
    # the batched renderer: the 256 parameter sets of depths 12..18 in one launch
    ta, tb, depth = wl.batch256(seed=0)
    win = wl.BATCH_WINDOW
    words = sum(kl.num_words(int(d)) for d in depth)
    res = {"words": words}
    imgs = {}
    for bounded in (False, True):
        images = kl.new_image(win, len(ta))
        ms = _time(lambda: kl.render_many(ta, tb, depth, win, images=images, block_bounds=bounded),
                   max(2, args.steps // 8), 2)
        res["bounded" if bounded else "per_word"] = {"ms": round(ms, 3), "gwords_per_s": round(words / ms / 1e6, 1)}
        imgs[bounded] = images
    res["images_equal"] = bool(torch.equal(imgs[False], imgs[True]))
    res["speedup"] = round(res["per_word"]["ms"] / res["bounded"]["ms"], 2)
    assert res["images_equal"], "block bounds changed a batched image"
    out["batch256"] = res
    return out


def leg_decode(args):
    """kl_decode at depth 18: 2^27 consecutive words from a third of the way
    into the index space, written as a (count x 18) byte array.  The kernel
    is bound by its HBM writes: 18 bytes per word."""
    import torch

    from paper_1709_08018_amd import kl

    d, count = 18, 1 << 27
    first = kl.num_words(d) // 3
    out = torch.empty((count, d), dtype=torch.uint8, device="cuda")
    for _ in range(3):
        kl.decode(first, count, d, out=out)
    reps = max(5, args.steps // 10)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        kl.decode(first, count, d, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbs = count * d / ms / 1e6
    # the same bytes written with no compute: torch's fill kernel on 8-byte
    # elements, and zero_(); the better of the two is the plain-write rate
    wide = out.view(-1)[: (count * d) // 8 * 8].view(torch.int64)
    plain = {}
    for name, op in (("fill_int64", lambda: wide.fill_(7)), ("zero", lambda: out.zero_())):
        op()
        e0.record()
        for _ in range(reps):
            op()
        e1.record()
        torch.cuda.synchronize()
        plain[name] = round(count * d / (e0.elapsed_time(e1) / reps) / 1e6, 1)
    # the same bytes in the store orders of libkl_calib.so: one chunk a
    # workgroup in launch order, or a persistent grid writing tiles in turn
    # as the decode kernel does (36,864 B: its tile at depth 18)
    clib = ctypes.CDLL(os.path.join(ROOT, "paper_1709_08018_amd", "libkl_calib.so"))
    clib.kl_calib_store.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)]
    gbs_pat = (ctypes.c_double * clib.kl_calib_store_patterns())()
    if clib.kl_calib_store(ctypes.c_void_p(out.data_ptr()), ctypes.c_uint64(count * d), gbs_pat) != 0:
        raise RuntimeError("kl_calib_store failed")
    names = ("chunk_4k", "chunk_16k", "chunk_64k", "persistent_tiles_4k", "persistent_tiles_36k",
             "persistent_tiles_144k")
    patterns = {n: round(g, 1) for n, g in zip(names, gbs_pat)}
    for _ in range(2):
        kl.decode(first, count, d, out=out)
    rows = [0, 1, count // 2, count - 1]
    got = out[rows].cpu().numpy()
    return {"workload": "decode_d18", "words": count, "first": first, "ms": round(ms, 4),
            "gwords_per_s": round(count / ms / 1e6, 2),
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": 8000.0, "unit": "GB/s",
                         "frac": round(gbs / 8000.0, 3), "bytes_per_word": d,
                         "plain_write_gbs": plain, "store_pattern_gbs": patterns,
                         "frac_of_own_store_pattern": round(gbs / patterns["persistent_tiles_36k"], 3)},
            "cpu_baseline": cpu_baseline_decode(first, d, rows, got)}


def leg_batch(args):
    """256 parameter sets of depths 12..18: one batched persistent launch vs
    256 single renders enqueued back to back on one stream; with the
    planner's plans, with the plans kl_autotune_many keeps for the batch as a
    whole (the same plans given to the single renders, images compared), and
    the single renders with kl_autotune's plans for single renders."""
    import numpy as np
    import torch

    from paper_1709_08018_amd import kl
    from paper_1709_08018_amd import workloads as wl

    ta, tb, depth = wl.batch256(seed=0)
    win = wl.BATCH_WINDOW
    words = sum(kl.num_words(int(d)) for d in depth)
    imgs = kl.new_image(win, len(ta))

    def batched():
        kl.render_many(ta, tb, depth, win, images=imgs)

    def separate(plans=None):
        for i in range(len(ta)):
            o = {} if plans is None else {"tail_len": plans[i]["tail_len"], "lane_len": plans[i]["lane_len"],
                                          "waves_per_cu": plans[i]["waves_per_cu"]}
            kl.render(ta[i], tb[i], int(depth[i]), win, image=imgs[i], **o)

    reps = max(2, args.steps // 4)
    # the planner's plans: one batched launch, then 256 plain kl_render calls
    # (a single render plans shorter tails at depths 13-16 than a set of a
    # batch does, so the images are compared under the batch's plans)
    ms_b_default = _time(batched, reps, 1)
    ref = imgs.clone()
    ms_s_default = _time(separate, reps, 1)
    separate([kl.plan_many(int(d), "fp32", win) for d in depth])
    same_default = bool(torch.equal(ref, imgs))
    # plans tuned for the batch as a whole (timing whole batched launches)
    t0 = time.perf_counter()
    plans, tuned_ms, default_ms = kl.autotune_many(ta, tb, depth, win)
    tune_s = time.perf_counter() - t0
    ms_b_tuned = _time(batched, reps, 1)
    ref = imgs.clone()
    ms_s_same = _time(lambda: separate(plans), reps, 1)
    same_tuned = bool(torch.equal(ref, imgs))
    by_depth = {}
    for i, d in enumerate(depth):
        by_depth[int(d)] = {k: plans[i][k] for k in ("tail_len", "lane_len", "prefix_len", "waves_per_cu")}
    # the single renders with plans tuned for single renders, one per depth
    t0 = time.perf_counter()
    scratch = kl.new_image(win)
    for d in sorted({int(x) for x in depth}):
        i = int(np.nonzero(depth == d)[0][0])
        kl.autotune(ta[i], tb[i], d, win, scratch=scratch)
    tune1_s = time.perf_counter() - t0
    ms_s_single = _time(separate, reps, 1)
    ms_b = min(ms_b_default, ms_b_tuned)
    batched()
    torch.cuda.synchronize()
    cpu = cpu_baseline_batch(ta, tb, depth, win, kl.as_u32(imgs)) if not args.no_cpu_baseline else None
    return {"workload": "batch256", "sets": len(ta), "words": words,
            "batched_ms": round(ms_b, 3), "separate_ms": round(ms_s_default, 3),
            "speedup": round(ms_s_default / ms_b, 3), "batched_gwords_per_s": round(words / ms_b / 1e6, 2),
            "default_plans": {"batched_ms": round(ms_b_default, 3), "separate_ms": round(ms_s_default, 3),
                              "images_identical": same_default},
            "batch_tuned_plans": {"batched_ms": round(ms_b_tuned, 3), "tuner_batched_ms": round(tuned_ms, 3),
                                  "tuner_default_ms": round(default_ms, 3), "separate_same_plans_ms": round(ms_s_same, 3),
                                  "images_identical": same_tuned, "tune_seconds": round(tune_s, 2),
                                  "plans": by_depth},
            "single_tuned_plans": {"separate_ms": round(ms_s_single, 3), "tune_seconds": round(tune1_s, 2)},
            "note": "speedup: the faster batched launch against 256 plain renders with the planner's plans",
            "cpu_baseline": cpu}


def leg_tiling(args):
    """Real traces ta = tb = 3, tiling mode over depths 1..10 (FP64 and FP32)."""
    from paper_1709_08018_amd import kl
    from paper_1709_08018_amd import workloads as wl

    W = wl.FUCHSIAN_TILING_D10
    words = sum(kl.num_words(d) for d in range(1, W.depth + 1))
    image = kl.new_image(W.window)
    out = {"workload": W.name, "words": words}
    for prec in ("fp32", "fp64"):
        ms = _time(lambda: kl.render(W.ta, W.tb, W.depth, W.window, image=image, min_depth=1, precision=prec),
                   args.steps, args.warmup)
        out[prec] = {"ms": round(ms, 4), "gwords_per_s": round(words / ms / 1e6, 3)}
    if not args.no_cpu_baseline:
        kl.render(W.ta, W.tb, W.depth, W.window, image=image, min_depth=1, precision="fp64")
        out["cpu_baseline"] = cpu_baseline_tiling(W, words, kl.as_u32(image).astype("int64"))
    return out


def leg_maskit(args):
    """The configuration of the paper's index-search figure: Maskit's group
    at mu = -0.097 + 1.838i, tiling mode over depths 1..14, every word drawn
    from each generator's fixed point in turn (9,565,936 words, 4 points
    each), 1024^2 over one period of the translation b.  FP32 and FP64 step
    times, and the FP64 image against the CPU reference's."""
    import numpy as np

    from paper_1709_08018_amd import kl
    from paper_1709_08018_amd import workloads as wl

    W = wl.MASKIT_D14
    ab = kl.maskit_generators(W.ta)
    words = sum(kl.num_words(d) for d in range(W.min_depth, W.depth + 1))
    image = kl.new_image(W.window)
    out = {"workload": W.name, "mu": [W.ta.real, W.ta.imag], "words": words, "points": 4 * words}
    for prec in ("fp32", "fp64"):
        ms = _time(lambda: kl.render_group(ab, W.depth, W.window, image=image, min_depth=W.min_depth, seed="all",
                                           precision=prec), max(2, args.steps // 4), 3)
        # the same tiling with 6-letter tails throughout (the planner gives a
        # tiling its deepest depth's single-render tail, 4 letters here)
        ms6 = _time(lambda: kl.render_group(ab, W.depth, W.window, image=image, min_depth=W.min_depth, seed="all",
                                            precision=prec, tail_len=6), max(2, args.steps // 4), 3)
        out[prec] = {"ms": round(ms, 4), "gpoints_per_s": round(4 * words / ms / 1e6, 3),
                     "tail_len": kl.plan(W.depth, prec)["tail_len"], "ms_tail_6": round(ms6, 4)}
    kl.render_group(ab, W.depth, W.window, image=image, min_depth=W.min_depth, seed="all", precision="fp64")
    img = kl.as_u32(image).astype(np.int64)
    out["points_in_window"] = int(img.sum())
    out["cpu_baseline"] = cpu_baseline_maskit(W, words, img)
    return out


def leg_splits(args):
    """Single renders of one depth against the tail length: depths 13..18,
    FP32, images of 512^2 to 4096^2 over [-1.5, 1.5]^2, averaged over four
    parameter sets (the quasi-Fuchsian pair and sets 3, 50 and 120 of the
    256-set batch); microseconds per render with the planner's split and
    with 6-, 5- and 4-letter tails."""
    from paper_1709_08018_amd import kl
    from paper_1709_08018_amd import workloads as wl

    ta, tb, _ = wl.batch256(seed=0)
    sets = [(wl.C2_TA, wl.C2_TB)] + [(complex(ta[i]), complex(tb[i])) for i in (3, 50, 120)]
    reps = max(3, args.steps // 20)
    rows = []
    for W in (512, 1024, 2048, 4096):
        win = (-1.5, 1.5, -1.5, 1.5, W, W)
        image = kl.new_image(win)
        for d in range(13, 19):
            row = {"image": f"{W}x{W}", "depth": d, "planner_tail_len": kl.plan(d, "fp32", win)["tail_len"]}
            for r in (0, 6, 5, 4):
                ms = _time(lambda: [kl.render(a, b, d, win, image=image, tail_len=r) for a, b in sets], reps, 2)
                row["planner_us" if r == 0 else f"tail_{r}_us"] = round(ms * 1e3 / len(sets), 1)
            rows.append(row)
    return {"workload": "splits", "rows": rows}


def leg_cayley(args):
    """Words of indexed Cayley tables (Section 5) on the general table path:
    (1) the once-punctured torus table (Table 2) with the depth-16
    quasi-Fuchsian maps, 57,395,628 words, against the specialised renderer
    on the same words; (2) the modular group PSL(2, Z) = <a, b | a^2 = b^3 = 1>
    in tiling mode over depths 1..40 from every symbol's fixed point.  Both
    images are checked against the CPU reference."""
    import numpy as np

    from paper_1709_08018_amd import kl
    from paper_1709_08018_amd import workloads as wl

    out = {"workload": "cayley"}
    t11 = np.array([[0, 1, 2, 3, 4], [1, 1, 2, 0, 4], [2, 1, 2, 3, 0], [3, 0, 2, 3, 4], [4, 1, 0, 3, 4]], np.uint8)
    maps = kl.generators(wl.C2_TA, wl.C2_TB)[1]   # a, b, A, B from the library's recipe
    win = wl.QUASIFUCHSIAN_D18.window.as_tuple()
    t = kl.Cayley(t11, maps)
    d = 16
    n = kl.cayley_num_words(t, d)
    image = kl.new_image(win)
    ms = _time(lambda: kl.cayley_render(t, d, win, image=image), max(2, args.steps // 10), 2)
    ms_spec = _time(lambda: kl.render(wl.C2_TA, wl.C2_TB, d, win, image=kl.new_image(win), precision="fp64"),
                    max(2, args.steps // 10), 2)
    kl.cayley_render(t, d, win, image=image)
    img = kl.as_u32(image).astype(np.int64)
    out["t11_d16"] = {"words": n, "ms": round(ms, 4), "gwords_per_s": round(n / ms / 1e6, 3),
                      "specialised_fp64_ms": round(ms_spec, 4),
                      "cpu_baseline": cpu_baseline_cayley_t11(wl.C2_TA, wl.C2_TB, d, win, n, img)}
    mod = np.array([[0, 1, 2, 3], [1, 0, 2, 3], [2, 1, 0, 0], [3, 1, 0, 0]], np.uint8)
    mod_maps = np.array([[[0, -1], [1, 0]], [[0, -1], [1, 1]], [[1, 1], [-1, 0]]], complex)
    tm = kl.Cayley(mod, mod_maps)
    wm = (-2.0, 2.0, 0.0, 1.25, 2048, 640)
    words = sum(kl.cayley_num_words(tm, dd) for dd in range(1, 41))
    image = kl.new_image(wm)
    ms = _time(lambda: kl.cayley_render(tm, 40, wm, image=image, min_depth=1, seed="all"), max(2, args.steps // 10), 2)
    img = kl.as_u32(image).astype(np.int64)
    out["modular_tiling_d40"] = {"words": words, "points": 3 * words, "ms": round(ms, 4),
                                 "gpoints_per_s": round(3 * words / ms / 1e6, 3),
                                 "cpu_baseline": cpu_baseline_cayley_modular(mod, mod_maps, wm, words, img)}
    return out


def leg_surrogate(args):
    """Learned occupancy surrogate at depth 14, 128^2 over [-2,2]^2: 20,000
    training sets (PCG64 seed 1; the last 2,000 calibrate the gate) and 2,000
    held-out sets (seed 2).  Times the held-out scan -- surrogate forward,
    gate, fallback renders of the rejected sets -- against the plain
    renderer, at the IoU target 0.95 and at lower targets."""
    from paper_1709_08018_amd import surrogate as S

    res, _ = S.run(train_n=18000, calib_n=2000, test_n=2000, steps=12000, batch=128, lr=2e-3, log_every=1000)
    res["metric"] = "surrogate vs plain scan time @IoU>=0.95"
    return res


def cpu_baseline_walk(W, img):
    """The oracle's walk render of the Fig. 3 points, timed on one thread,
    and the GPU's FP64 image against it."""
    import numpy as np
    ref = _oracle()
    g = ref.group_maskit(W.mu)
    t0 = time.perf_counter()
    rimg, _, near = ref.walk_render(g, W.seed, 0, W.n_walkers, W.burn_in, W.n_steps, W.window.as_tuple(),
                                    edge_tol=1e-7)
    dt = time.perf_counter() - t0
    return {"kind": "oracle", "value": round(W.points / dt / 1e9, 5), "unit": "Gpoints/s", "cores": 1,
            "sample": f"the full workload ({W.points} points)", "seconds": round(dt, 3),
            "fp64_l1_vs_oracle": int(np.abs(img - rimg.astype(np.int64)).sum()), "oracle_near_edge_words": int(near)}


def leg_surrogate_kernels(args):
    """The surrogate's kernels alone, with untrained parameters: the fused
    forward pass on 512 sets and a training step on 128 (the timings of the
    surrogate leg's kernel_rates, without its data and training)."""
    from paper_1709_08018_amd import surrogate as S
    from paper_1709_08018_amd import workloads as wl

    ta, tb = wl.surrogate_sets(512, seed=2)
    params = S.init_params(0)
    return {"workload": "surrogate_kernels", "kernel_rates": S.kernel_rates(params, ta, tb, reps=max(5, args.steps // 10))}


def leg_walk(args):
    """The probabilistic approach (Section 4, Fig. 3): random walks in
    Maskit's group at mu = -0.097 + 1.838i, 2^20 drawn points, FP32 and FP64,
    against the indexed renderer on the same group, window and image: the
    depth-13 limit set (2,125,764 words) beside a walk of as many points, and
    2^30 points beside the depth-19 limit set.  Coverage: the occupied
    pixels (count > 0) of each image, and the IoU of the two occupancies."""
    import numpy as np
    import torch

    from paper_1709_08018_amd import kl
    from paper_1709_08018_amd import workloads as wl

    def occ(t):
        return kl.as_u32(t) > 0

    def iou(a, b):
        u = int((a | b).sum())
        return 1.0 if u == 0 else int((a & b).sum()) / u

    W = wl.WALK_FIG3
    ab = kl.maskit_generators(W.mu)
    win = W.window.as_tuple()
    image = kl.new_image(win)
    out = {"workload": W.name, "mu": [W.mu.real, W.mu.imag], "points": W.points, "walkers": W.n_walkers,
           "steps": W.n_steps, "burn_in": W.burn_in, "seed": W.seed,
           "reading": "first letter uniform, each step uniform over the three letters that keep the word "
                      "reduced, from the first letter's attracting fixed point; no commutator boost"}
    steps = max(5, args.steps // 4)
    for prec in ("fp32", "fp64"):
        ms = _time(lambda: kl.walk_render(ab, W.seed, 0, W.n_walkers, W.burn_in, W.n_steps, win, image=image,
                                          precision=prec), steps, 3)
        out[prec] = {"ms": round(ms, 4), "gpoints_per_s": round(W.points / ms / 1e6, 3)}
    dropped = torch.zeros(1, dtype=torch.int64, device="cuda")
    kl.walk_render(ab, W.seed, 0, W.n_walkers, W.burn_in, W.n_steps, win, image=image, precision="fp64",
                   dropped=dropped)
    img = kl.as_u32(image).astype(np.int64)
    out["points_in_window"] = int(img.sum())
    out["dropped"] = int(dropped.item())
    out["cpu_baseline"] = cpu_baseline_walk(W, img)
    # equal point counts: the indexed limit set against a walk of as many points
    cmp = []
    for Wc, depth in ((wl.WALK_D13_POINTS, 13), (wl.WALK_LARGE, 19)):
        idx_img = kl.new_image(win)
        walk_img = kl.new_image(win)
        ms_i = _time(lambda: kl.render_group(ab, depth, win, image=idx_img), steps, 3)
        ms_w = _time(lambda: kl.walk_render(ab, Wc.seed, 0, Wc.n_walkers, Wc.burn_in, Wc.n_steps, win,
                                            image=walk_img), steps, 3)
        oi, ow = occ(idx_img), occ(walk_img)
        cmp.append({"indexed_depth": depth, "indexed_words": kl.num_words(depth), "walk": Wc.name,
                    "walk_points": Wc.points, "indexed_ms": round(ms_i, 4), "walk_ms": round(ms_w, 4),
                    "indexed_gwords_per_s": round(kl.num_words(depth) / ms_i / 1e6, 2),
                    "walk_gpoints_per_s": round(Wc.points / ms_w / 1e6, 2),
                    "occupied_pixels": {"indexed": int(oi.sum()), "walk": int(ow.sum())},
                    "occupancy_iou": round(iou(oi, ow), 4)})
    out["indexed_vs_walk"] = cmp
    # the two histogram paths on every walk workload (the renders above take
    # the planner's choice): one global atomic per point, and the binned path
    # (points sorted by image tile in LDS, counted tile by tile); images equal
    paths = []
    for Wc in (W, wl.WALK_D13_POINTS, wl.WALK_LARGE):
        row = {"walk": Wc.name, "points": Wc.points}
        imgs = {}
        for mode in ("runs", "lds"):
            img = kl.new_image(win)
            row[mode + "_ms"] = round(_time(lambda: kl.walk_render(ab, Wc.seed, 0, Wc.n_walkers, Wc.burn_in,
                                                                   Wc.n_steps, win, image=img, hist_mode=mode),
                                            steps, 3), 4)
            imgs[mode] = img
        row["images_equal"] = bool(torch.equal(imgs["runs"], imgs["lds"]))
        paths.append(row)
    out["histogram_paths"] = paths
    return out


def surrogate_summary():
    """The metric's second half, measured in the headline run: the learned
    surrogate trained on 18,000 renders of depth 14 (the surrogate leg's
    configuration), its gate calibrated on 2,000 more at the IoU target 0.95,
    and the scan of 2,000 held-out sets -- surrogate, gate and fallback
    renders -- timed against the plain renderer's scan (median of 5 each)."""
    from paper_1709_08018_amd import surrogate as S

    res, _ = S.run(train_n=18000, calib_n=2000, test_n=2000, steps=12000, batch=128, lr=2e-3, log_every=0)
    sc = res["scan"]
    return {"metric": "surrogate vs plain scan time @IoU>=0.95", "iou_target": S.IOU_TARGET,
            "held_out_sets": res["held_out_sets"], "accepted": sc["accepted"],
            "gated_scan_s": sc["surrogate_seconds"], "plain_scan_s": sc["plain_seconds"],
            "speedup": sc["speedup"], "held_out_mean_iou": round(res["held_out"]["mean_iou_surrogate"], 4),
            "held_out_max_iou": round(res["held_out_iou_quantiles"]["max"], 4),
            "scan_min_iou_vs_plain": round(sc["min_iou_vs_plain"], 4), "train_sets": res["train_sets"],
            "train_seconds": res["train_seconds"], "data_seconds": res["data_seconds"]}


def leg_surrogate_curve(args):
    """Held-out IoU of the surrogate against the number of training renders
    (18k, 100k, 500k sets at depth 14), each trained for 12,000 steps of 128
    sets, and 500k for 48,000 steps: whether more data closes the gap to the
    gate's IoU target of 0.95."""
    import numpy as np
    import torch

    from paper_1709_08018_amd import kl
    from paper_1709_08018_amd import surrogate as S
    from paper_1709_08018_amd import workloads as wl

    ta_te, tb_te = wl.surrogate_sets(2000, seed=2)
    occ_te = S.render_occupancy(ta_te, tb_te)
    ta_all, tb_all = wl.surrogate_sets(500_000, seed=1)
    t0 = time.perf_counter()
    occ_all = S.render_occupancy(ta_all, tb_all)
    torch.cuda.synchronize()
    data_s = time.perf_counter() - t0
    rows = []
    for n, steps in ((18_000, 12_000), (100_000, 12_000), (500_000, 12_000), (500_000, 48_000)):
        t0 = time.perf_counter()
        params, hist = S.train(ta_all[:n], tb_all[:n], occ_all[:n], steps, 128, 2e-3, 0, log_every=steps)
        torch.cuda.synchronize()
        tr_s = time.perf_counter() - t0
        logits = S.predict(params, ta_te, tb_te)
        iou = kl.iou(occ_te, logits=logits).cpu().numpy()
        rows.append({"train_sets": n, "steps": steps, "epochs": round(steps * 128 / n, 2), "train_seconds": round(tr_s, 1),
                     "final_loss": round(hist[-1][1], 5) if hist else None,
                     "held_out_mean_iou": round(float(iou.mean()), 4),
                     "held_out_p90_iou": round(float(np.quantile(iou, 0.9)), 4),
                     "held_out_max_iou": round(float(iou.max()), 4),
                     "held_out_at_0.95": int((iou >= 0.95).sum())})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    return {"workload": "surrogate_curve", "held_out_sets": 2000, "data_seconds_500k": round(data_s, 1), "curve": rows}


def leg_calib(args):
    """Instruction-throughput calibration of the VALU roofline (libkl_calib.so):
    SIMD cycles per wave64 instruction of each class the renderer's word loop
    issues, at the device's reported clock."""
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1709_08018_amd", "libkl_calib.so"))
    ms = (ctypes.c_double * 9)()
    cyc = (ctypes.c_double * 9)()
    ghz = ctypes.c_double()
    if lib.kl_calib_valu(ms, cyc, ctypes.byref(ghz)) != 0:
        raise RuntimeError("kl_calib_valu failed")
    names = ["v_fma_f32", "v_mul_f32", "v_add_f32", "v_add_u32", "v_rcp_f32", "v_mad_u32_u24",
             "v_cvt_flr_i32_f32+v_add_f32", "v_cmp_gt_u32+v_cndmask_b32", "v_fma_f64"]
    return {"workload": "calib", "clock_ghz": ghz.value,
            "cycles_per_wave64_group": {n: round(c, 3) for n, c in zip(names, cyc)},
            "ms": {n: round(m, 4) for n, m in zip(names, ms)}}


def leg_hist(args):
    """Depth-18 step time per histogram strategy and split."""
    import numpy as np
    import torch

    from paper_1709_08018_amd import kl
    from paper_1709_08018_amd import workloads as wl

    W = wl.QUASIFUCHSIAN_D18
    image = kl.new_image(W.window)
    rows = []
    for r in (5, 6, 7):
        for m in (2, 3, 4):
            for wpc in (16, 32):
                for hist in ("runs", "lds"):
                    opts = dict(tail_len=r, lane_len=m, waves_per_cu=wpc, hist_mode=hist)
                    ms = _time(lambda: kl.render(W.ta, W.tb, W.depth, W.window, image=image, **opts), 5, 1)
                    rows.append({**opts, "step_ms": round(ms, 4)})
    rows.sort(key=lambda x: x["step_ms"])
    return {"workload": W.name, "candidates": rows}


def fp64_leg(W, image, n_words, hip, steps=20):
    """The same step on the FP64 path (every step of the arithmetic in FP64):
    its step time, and its render kernel's rate against the FP64 vector peak."""
    import numpy as np
    import torch

    from paper_1709_08018_amd import kl

    plan = kl.plan(W.depth, "fp64")
    ev = []
    for _ in range(2 * steps):
        e = ctypes.c_void_p()
        if hip.hipEventCreate(ctypes.byref(e)) != 0:
            raise RuntimeError("hipEventCreate failed")
        ev.append(e.value)
    for _ in range(5):
        kl.render(W.ta, W.tb, W.depth, W.window, image=image, precision="fp64")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        kl.render(W.ta, W.tb, W.depth, W.window, image=image, precision="fp64",
                  kernel_events=(ev[2 * i], ev[2 * i + 1]))
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    kms = []
    for i in range(steps):
        f = ctypes.c_float()
        hip.hipEventElapsedTime(ctypes.byref(f), ev[2 * i], ev[2 * i + 1])
        kms.append(f.value)
    for e in ev:
        hip.hipEventDestroy(e)
    kernel_ms = float(np.mean(kms))
    R = 3 ** plan["tail_len"]
    kw = (n_words // R) * R
    return {"ms_per_step": round(ms, 4), "value": round(n_words / (ms * 1e-3) / 1e9, 3), "unit": "Gwords/s",
            "kernel_ms": round(kernel_ms, 4),
            "frac_of_fp64_peak": round(FLOPS_PER_WORD * kw / (kernel_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4),
            "split": {k: plan[k] for k in ("prefix_len", "lane_len", "tail_len")}, "steps": steps}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=400,
                    help="untimed steps after the clock ramp (CLOCK_RAMP_MS of untimed steps first)")
    ap.add_argument("--workload", default="quasifuchsian_d18",
                    choices=["quasifuchsian_d18", "quasifuchsian_d22", "decode", "bounded", "batch256", "fuchsian_tiling_d10",
                             "maskit_tiling_d14", "cayley", "surrogate", "surrogate_kernels", "surrogate_curve", "hist",
                             "calib", "walk", "splits"])
    ap.add_argument("--no-surrogate", action="store_true",
                    help="leave the surrogate's training and gated scan out of the headline line")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after the steps, copy 256 MiB device to device twice (a kernel of known HBM "
                         "traffic that scales counter-based byte counts)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the renderer shards by "
              f"index range with one image reduction, which this library does not implement.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1709_08018_amd import kl
    from paper_1709_08018_amd import workloads as wl

    torch.cuda.set_device(0)
    legs = {"quasifuchsian_d22": leg_d22, "decode": leg_decode, "bounded": leg_bounded, "batch256": leg_batch, "fuchsian_tiling_d10": leg_tiling,
            "maskit_tiling_d14": leg_maskit, "splits": leg_splits, "cayley": leg_cayley, "surrogate": leg_surrogate, "hist": leg_hist,
            "calib": leg_calib, "walk": leg_walk, "surrogate_kernels": leg_surrogate_kernels,
            "surrogate_curve": leg_surrogate_curve}
    if args.workload in legs:
        print(json.dumps(legs[args.workload](args)), flush=True)
        return
    W = wl.QUASIFUCHSIAN_D18
    n_words = kl.num_words(W.depth)
    plan = kl.plan(W.depth, "fp32")
    image = kl.new_image(W.window)
    dropped = torch.zeros(1, dtype=torch.int64, device="cuda")
    hip = _hip()
    # the renderer's kernel time is sampled on every EVENT_EVERY-th timed step
    # (an event pair costs a few microseconds of queue time per step)
    sampled = list(range(0, args.steps, EVENT_EVERY))
    events = []
    for _ in range(max(2, 2 * len(sampled))):
        e = ctypes.c_void_p()
        if hip.hipEventCreate(ctypes.byref(e)) != 0:
            raise RuntimeError("hipEventCreate failed")
        events.append(e.value)

    def step(i=None):
        j = None if i is None or i % EVENT_EVERY else i // EVENT_EVERY
        ev = None if j is None else (events[2 * j], events[2 * j + 1])
        kl.render(W.ta, W.tb, W.depth, W.window, image=image, kernel_events=ev)

    ramp_steps, t_ramp = 0, time.perf_counter()
    while (time.perf_counter() - t_ramp) * 1e3 < CLOCK_RAMP_MS:
        for _ in range(20):
            step()
        ramp_steps += 20
        torch.cuda.synchronize()
    ramp_ms = (time.perf_counter() - t_ramp) * 1e3
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    kernel_ms = []
    for j in range(len(sampled)):
        ms = ctypes.c_float()
        hip.hipEventElapsedTime(ctypes.byref(ms), events[2 * j], events[2 * j + 1])
        kernel_ms.append(ms.value)
    # the kernel alone, after the timed steps: 3 warm-up and 20 timed renders,
    # each waited for, with events around the persistent kernel's launch
    reps = []
    for r in range(23):
        kl.render(W.ta, W.tb, W.depth, W.window, image=image, kernel_events=(events[0], events[1]))
        hip.hipEventSynchronize(ctypes.c_void_p(events[1]))
        ms = ctypes.c_float()
        hip.hipEventElapsedTime(ctypes.byref(ms), events[0], events[1])
        if r >= 3:
            reps.append(ms.value)
    for e in events:
        hip.hipEventDestroy(e)
    kernel_avg = float(np.mean(kernel_ms))

    if args.calib_copy:
        src = torch.empty(64 * 2 ** 20, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()

    # the timed steps do not count dropped words (kl_render does not); one
    # more render with the counter checks that every word was counted once
    h_timed = kl.as_u32(image).astype(np.int64)
    kl.render(W.ta, W.tb, W.depth, W.window, image=image, dropped=dropped)
    h = kl.as_u32(image).astype(np.int64)
    assert np.array_equal(h, h_timed), "image differs with the dropped counter on"
    total = int(h.sum()) + int(dropped.item())
    assert total == n_words, f"image + dropped = {total} != {n_words}"

    # words handled by the persistent kernel: every whole head (all of them
    # for a full render, whose word count is a multiple of 3^tail_len)
    R = 3 ** plan["tail_len"]
    kernel_words = (n_words // R) * R
    achieved = FLOPS_PER_WORD * kernel_words / (kernel_avg * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP32_PEAK_TFLOPS, 4), "traffic": _traffic_from_profile(plan),
                "kernel": "render_kernel<float, %s, false>" % ("true" if plan["hist_mode"] == 2 else "false"),
                "kernel_ms": round(kernel_avg, 4),
                "kernel_ms_alone": {"reps": len(reps), "warmup": 3, "median": round(float(np.median(reps)), 4),
                                    "min": round(float(np.min(reps)), 4), "mean": round(float(np.mean(reps)), 4),
                                    "note": "renders waited for one at a time after the timed steps"},
                "flops_per_word": FLOPS_PER_WORD, "words_per_launch": kernel_words}
    # VALU issue (committed counter summary of the current source and split):
    # instructions per 64 words, and the fraction of the VALU issue slots the
    # kernel fills -- its VALU instructions at 4 cycles each on the 1024 SIMDs,
    # over the GPU-active cycles the same dispatches count (GRBM_GUI_ACTIVE)
    roofline["valu_instr_per_wave_word"] = _valu_per_wave_word(plan)
    roofline["valu_issue_frac"] = _profile_value(VALU_SUMMARY, "VALU issue fraction", plan)

    out = {
        "metric": METRIC,
        "value": round(n_words / (ms_per_step * 1e-3) / 1e9, 3),
        "unit": "Gwords/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": W.name, "depth": W.depth, "words": n_words,
                   "ta": [W.ta.real, W.ta.imag], "tb": [W.tb.real, W.tb.imag],
                   "image": f"{W.window.width}x{W.window.height} u32 over [-1.5,1.5]^2",
                   "arithmetic": "FP64 generators, seeds and prefix products; FP32 suffix maps",
                   "split": {k: plan[k] for k in ("prefix_len", "lane_len", "tail_len", "waves_per_cu")},
                   "dropped": int(dropped.item())},
        "roofline": roofline,
        "clock_ramp": {"ms": round(ramp_ms, 1), "steps": ramp_steps,
                       "note": "untimed steps run before the counted warm-up until the GPU clock has ramped"},
        "fp64": fp64_leg(W, image, n_words, hip),
    }
    if not args.no_surrogate:
        out["surrogate"] = surrogate_summary()
    if not args.no_cpu_baseline:
        cb, ref_img, ref_drop = cpu_baseline(W, 15.0)
        out["cpu_baseline"] = cb
        diff = int(np.abs(h - ref_img.astype(np.int64)).sum())
        out["config"]["l1_vs_reference_image"] = diff
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
