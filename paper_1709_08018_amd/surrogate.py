"""Occupancy surrogate: training data from the renderer, training on the
GPU with the library's own kernels, an uncertainty gate, and the plain
renderer as fallback and as the reference for IoU.

Every compute step (renders, occupancy, forward, backward, Adam, gate
statistic, IoU) runs in libkl; this module orders the calls, slices device
buffers and makes the host-side accept / reject decision.

    python -m paper_1709_08018_amd.surrogate [--train-n 18000] [--steps 3000] ...
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from . import kl
from . import workloads as wl

DEPTH = wl.SURROGATE_DEPTH
WINDOW = wl.SURROGATE_WINDOW
IOU_TARGET = 0.95

# (name, shape) of the flat parameter vector, as include/kl_surrogate.h lays it out
SHAPES = [(4, 256), (256,), (256, 256), (256,), (16, 64, 4, 4), (64,), (64, 32, 4, 4), (32,),
          (32, 16, 4, 4), (16,), (16, 1, 4, 4), (1,)]


def init_params(seed: int) -> torch.Tensor:
    """He-normal weights (std sqrt(2 / fan-in)), zero biases but the last."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape in SHAPES:
        if len(shape) == 1:
            parts.append(np.zeros(shape))
        elif len(shape) == 2:
            parts.append(rng.normal(0, math.sqrt(2.0 / shape[0]), shape))
        else:
            parts.append(rng.normal(0, math.sqrt(2.0 / (shape[0] * 4)), shape))
    # last bias at the logit of a 3% occupancy prior (limit sets cover 2-8% of the window)
    parts[-1][:] = math.log(0.03 / 0.97)
    flat = np.concatenate([p.ravel() for p in parts]).astype(np.float32)
    assert flat.size == kl.sur_num_params()
    return torch.as_tensor(flat).cuda()


def render_occupancy(ta, tb, depth: int = DEPTH, chunk: int = 1024) -> torch.Tensor:
    """Occupancy (count > 0) of the plain renders, (n, 128, 128) uint8 on the GPU."""
    n = len(ta)
    out = torch.empty((n, WINDOW.height, WINDOW.width), dtype=torch.uint8, device="cuda")
    imgs = kl.new_image(WINDOW, min(chunk, n))
    for i in range(0, n, chunk):
        c = min(chunk, n - i)
        kl.render_many(ta[i:i + c], tb[i:i + c], np.full(c, depth), WINDOW, images=imgs[:c])
        kl.occupancy(imgs[:c], out=out[i:i + c])
    return out


def predict(params: torch.Tensor, ta, tb, batch: int = 512) -> torch.Tensor:
    n = len(ta)
    out = torch.empty((n, 128, 128), dtype=torch.float32, device="cuda")
    ws = kl.sur_workspace(min(batch, n))
    ta_d, tb_d = kl.as_c64(ta), kl.as_c64(tb)
    for i in range(0, n, batch):
        c = min(batch, n - i)
        kl.sur_forward(params, ta_d[i:i + c], tb_d[i:i + c], workspace=ws, out=out[i:i + c])
    return out


def train(ta, tb, occ: torch.Tensor, steps: int, batch: int = 128, lr: float = 2e-3, seed: int = 0,
          params: torch.Tensor | None = None, log_every: int = 0):
    """Adam with a cosine learning-rate decay over contiguous batches whose order
    is reshuffled every epoch.  Returns (params, [(step, loss)])."""
    n = len(ta)
    batch = min(batch, n)
    if params is None:
        params = init_params(seed)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    grad = torch.zeros_like(params)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    ws = kl.sur_workspace(batch)
    ta_d, tb_d = kl.as_c64(ta), kl.as_c64(tb)
    rng = np.random.default_rng(seed)
    starts = np.arange(0, n - batch + 1, batch)
    order = rng.permutation(starts)
    hist = []
    for step in range(1, steps + 1):
        k = (step - 1) % len(order)
        if k == 0 and step > 1:
            order = rng.permutation(starts)
        s0 = int(order[k])
        lr_t = lr * 0.5 * (1 + math.cos(math.pi * (step - 1) / steps))
        kl.sur_train_step(params, m, v, grad, step, lr_t, ta_d[s0:s0 + batch], tb_d[s0:s0 + batch],
                          occ[s0:s0 + batch], ws, loss)
        if log_every and (step % log_every == 0 or step == steps):
            hist.append((step, float(loss.item())))
            print(f"[surrogate] step {step}/{steps} loss {hist[-1][1]:.5f}", file=sys.stderr, flush=True)
    return params, hist


def gate_threshold(uncertainty: np.ndarray, iou: np.ndarray, target: float = IOU_TARGET) -> float:
    """Largest uncertainty u such that every calibration set with uncertainty
    <= u reaches IoU >= target (-inf when even the most certain one fails)."""
    unc = np.asarray(uncertainty, np.float64)
    fail = unc[np.asarray(iou) < target]
    limit = fail.min() if len(fail) else np.inf
    # strictly below the most certain failing set: a passing set that ties
    # with it cannot be told apart at scan time
    ok = unc[unc < limit]
    return float(ok.max()) if len(ok) else -np.inf


def scan(params: torch.Tensor, ta, tb, tau: float, depth: int = DEPTH, batch: int = 512):
    """Occupancy images of all sets: the surrogate's where the gate accepts it,
    the plain renderer's elsewhere.  Returns (occ, accepted, seconds)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    logits = predict(params, ta, tb, batch)
    unc = kl.sur_uncertainty(logits).cpu().numpy()
    accepted = unc <= tau
    occ = torch.empty((len(ta), 128, 128), dtype=torch.uint8, device="cuda")
    kl.sur_predict_occupancy(logits, out=occ)
    rej = np.nonzero(~accepted)[0]
    if len(rej):
        rendered = render_occupancy(ta[rej], tb[rej], depth)
        occ[torch.as_tensor(rej, device="cuda")] = rendered
    torch.cuda.synchronize()
    return occ, accepted, time.perf_counter() - t0


def plain_scan(ta, tb, depth: int = DEPTH):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    occ = render_occupancy(ta, tb, depth)
    torch.cuda.synchronize()
    return occ, time.perf_counter() - t0


def evaluate(params, ta, tb, occ_true, tau):
    """IoU of the surrogate alone, and of the gated scan, against the plain renders."""
    logits = predict(params, ta, tb)
    iou_sur = kl.iou(occ_true, logits=logits).cpu().numpy()
    unc = kl.sur_uncertainty(logits).cpu().numpy()
    acc = unc <= tau
    return {"mean_iou_surrogate": float(iou_sur.mean()), "median_iou_surrogate": float(np.median(iou_sur)),
            "accepted": int(acc.sum()), "acceptance_rate": float(acc.mean()),
            "accepted_min_iou": float(iou_sur[acc].min()) if acc.any() else None,
            "accepted_mean_iou": float(iou_sur[acc].mean()) if acc.any() else None,
            "accepted_below_target": int((iou_sur[acc] < IOU_TARGET).sum())}, iou_sur, unc


def sensitivity(ta, tb, occ, eps_list=(1e-3, 3e-3, 1e-2, 3e-2), n=500, seed=5, depth=DEPTH):
    """How far the occupancy moves with the traces: IoU between each set's
    plain render (occ) and the plain render at traces moved a distance eps in
    a random direction of (Re ta, Im ta, Re tb, Im tb).  A predictor that
    reaches the IoU target must resolve the traces to about the eps at which
    this IoU falls below it."""
    rng = np.random.default_rng(seed)
    n = min(n, len(ta))
    out = []
    for eps in eps_list:
        d = rng.normal(size=(n, 4))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        ta2 = np.asarray(ta[:n]) + eps * (d[:, 0] + 1j * d[:, 1])
        tb2 = np.asarray(tb[:n]) + eps * (d[:, 2] + 1j * d[:, 3])
        iou = kl.iou(occ[:n], pred_occ=render_occupancy(ta2, tb2, depth)).cpu().numpy()
        out.append({"eps": eps, "sets": n, "mean_iou": round(float(iou.mean()), 4),
                    "median_iou": round(float(np.median(iou)), 4),
                    "frac_at_target": round(float((iou >= IOU_TARGET).mean()), 4)})
    return out


def _median_of(fn, reps):
    """Run fn() reps times; its last return value is seconds.  Returns the last
    result and the median time."""
    times, out = [], None
    for _ in range(reps):
        out = fn()
        times.append(out[-1])
    return out, float(np.median(times))


FWD_FLOP_PER_SET = 2 * 18_154_496   # two flops per multiply-add of one forward pass (the shapes above)


def kernel_rates(params, ta, tb, batch=512, reps=20):
    """Event-timed forward pass on `batch` sets and training step on 128."""
    ws = kl.sur_workspace(batch)
    ta_d, tb_d = kl.as_c64(ta[:batch]), kl.as_c64(tb[:batch])
    out = torch.empty((batch, 128, 128), dtype=torch.float32, device="cuda")
    for _ in range(3):
        kl.sur_forward(params, ta_d, tb_d, workspace=ws, out=out)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        kl.sur_forward(params, ta_d, tb_d, workspace=ws, out=out)
    e1.record()
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1) / reps
    b = 128
    p = params.clone()
    m, v, g = torch.zeros_like(p), torch.zeros_like(p), torch.zeros_like(p)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    occ = torch.zeros((b, 128, 128), dtype=torch.uint8, device="cuda")
    ws = kl.sur_workspace(b)
    for st in range(1, 4):
        kl.sur_train_step(p, m, v, g, st, 1e-5, ta_d[:b], tb_d[:b], occ, ws, loss)
    e0.record()
    for st in range(4, 4 + reps):
        kl.sur_train_step(p, m, v, g, st, 1e-5, ta_d[:b], tb_d[:b], occ, ws, loss)
    e1.record()
    torch.cuda.synchronize()
    step_ms = e0.elapsed_time(e1) / reps
    return {"forward_sets": batch, "forward_ms": round(fwd_ms, 4),
            "forward_tflops": round(batch * FWD_FLOP_PER_SET / fwd_ms / 1e9, 1),
            "train_step_sets": b, "train_step_ms": round(step_ms, 4),
            "train_step_tflops": round(3 * b * FWD_FLOP_PER_SET / step_ms / 1e9, 1)}


def run(train_n=18000, calib_n=2000, test_n=2000, steps=3000, batch=128, lr=2e-3, depth=DEPTH, seed=0,
        log_every=250):
    t = time.perf_counter()
    ta_all, tb_all = wl.surrogate_sets(train_n + calib_n, seed=1)
    ta_te, tb_te = wl.surrogate_sets(test_n, seed=2)
    occ_all = render_occupancy(ta_all, tb_all, depth)
    torch.cuda.synchronize()
    data_s = time.perf_counter() - t
    print(f"[surrogate] rendered {train_n + calib_n} training sets in {data_s:.1f} s", file=sys.stderr, flush=True)
    t = time.perf_counter()
    params, hist = train(ta_all[:train_n], tb_all[:train_n], occ_all[:train_n], steps, batch, lr, seed,
                         log_every=log_every)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t
    # calibrate the gate on the held-back part of the training draw
    occ_cal = occ_all[train_n:]
    logits_cal = predict(params, ta_all[train_n:], tb_all[train_n:])
    iou_cal = kl.iou(occ_cal, logits=logits_cal).cpu().numpy()
    unc_cal = kl.sur_uncertainty(logits_cal).cpu().numpy()
    tau = gate_threshold(unc_cal, iou_cal)
    # held-out: plain scan (the IoU reference) and gated surrogate scan
    plain_scan(ta_te[:64], tb_te[:64], depth)  # warm-up
    (occ_true, _), plain_s = _median_of(lambda: plain_scan(ta_te, tb_te, depth), 5)
    scan(params, ta_te[:64], tb_te[:64], tau, depth)  # warm-up
    (occ_scan, accepted, _), scan_s = _median_of(lambda: scan(params, ta_te, tb_te, tau, depth), 5)
    scan_iou = kl.iou(occ_true, pred_occ=occ_scan).cpu().numpy()
    ev, iou_sur, _ = evaluate(params, ta_te, tb_te, occ_true, tau)
    # what the gate buys at other quality bars: calibrated on the calibration sets,
    # applied to the held-out sets, timed as a full scan
    tradeoff = []
    for target in (0.5, 0.6, 0.7, 0.8, 0.9, IOU_TARGET):
        tau_t = gate_threshold(unc_cal, iou_cal, target)
        (occ_t, acc_t, _), sec_t = _median_of(lambda: scan(params, ta_te, tb_te, tau_t, depth), 5)
        iou_t = kl.iou(occ_true, pred_occ=occ_t).cpu().numpy()
        tradeoff.append({"iou_target": target, "accepted": int(acc_t.sum()), "seconds": round(sec_t, 4),
                         "speedup": round(plain_s / sec_t, 3), "min_iou": float(iou_t.min()),
                         "sets_below_target": int((iou_t < target).sum())})
    # baselines without the trained network: untrained weights, and the mean training image
    sens = sensitivity(ta_te, tb_te, occ_true, depth=depth)
    rates = kernel_rates(params, ta_te, tb_te)
    untrained = evaluate(init_params(seed + 1), ta_te, tb_te, occ_true, tau)[0]
    mean_img = (occ_all[:train_n].float().mean(0) >= 0.5).to(torch.uint8)
    iou_mean = kl.iou(occ_true, pred_occ=mean_img.expand(test_n, 128, 128).contiguous()).cpu().numpy()
    return {
        "workload": "surrogate", "depth": depth, "train_sets": train_n, "calibration_sets": calib_n,
        "held_out_sets": test_n, "steps": steps, "batch": batch, "lr": lr,
        "data_seconds": round(data_s, 2), "train_seconds": round(train_s, 2),
        "final_loss": hist[-1][1] if hist else None, "gate_uncertainty_threshold": tau,
        "calibration_accepted": int((unc_cal <= tau).sum()),
        "held_out": ev,
        "scan": {"plain_seconds": round(plain_s, 4), "surrogate_seconds": round(scan_s, 4),
                 "speedup": round(plain_s / scan_s, 3), "accepted": int(accepted.sum()),
                 "min_iou_vs_plain": float(scan_iou.min()), "mean_iou_vs_plain": float(scan_iou.mean()),
                 "sets_below_target": int((scan_iou < IOU_TARGET).sum())},
        "baselines": {"untrained_mean_iou": untrained["mean_iou_surrogate"],
                      "mean_image_mean_iou": float(iou_mean.mean())},
        "held_out_iou_quantiles": {q: float(np.quantile(iou_sur, float(q))) for q in ("0.1", "0.5", "0.9", "0.99")}
        | {"max": float(iou_sur.max())},
        "tradeoff": tradeoff,
        "parameter_sensitivity": sens,
        "kernel_rates": rates,
        "timing": "plain and gated scans: median of 5 runs each",
    }, params


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-n", type=int, default=18000)
    ap.add_argument("--calib-n", type=int, default=2000)
    ap.add_argument("--test-n", type=int, default=2000)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=128)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--depth", type=int, default=DEPTH)
    ap.add_argument("--save", default=None, help="write the trained parameters (float32 .npy) here")
    a = ap.parse_args()
    res, params = run(a.train_n, a.calib_n, a.test_n, a.steps, a.batch, a.lr, a.depth)
    if a.save:
        np.save(a.save, params.cpu().numpy())
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
