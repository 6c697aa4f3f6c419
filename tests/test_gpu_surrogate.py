"""Surrogate kernels vs the FP64 reference network (oracle/nn_ref.py).

Operands of every matrix product are rounded to bfloat16 on both sides (the
reference emulates the GPU's rounding points); the GPU accumulates in FP32,
the reference in FP64.
"""
import numpy as np
import pytest
import torch

from oracle import nn_ref as N
from paper_1709_08018_amd import workloads as wl

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1709_08018_amd import kl


def _dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


@pytest.mark.parametrize("M,N_,K,ta,tb,split", [
    (1, 1, 1, False, False, False), (7, 13, 5, False, False, False), (64, 64, 32, False, False, False),
    (100, 70, 129, False, False, False), (33, 256, 4, False, False, False), (130, 65, 300, True, False, False),
    (70, 90, 77, False, True, False), (16, 16, 20000, True, False, True), (256, 256, 64, True, True, True),
])
def test_gemm_matches_bf16_reference(M, N_, K, ta, tb, split):
    rng = np.random.default_rng(M * 7 + N_ + K)
    A = rng.normal(size=(M, K)).astype(np.float32)
    B = rng.normal(size=(K, N_)).astype(np.float32)
    Ad = _dev(A.T.copy() if ta else A)
    Bd = _dev(B.T.copy() if tb else B)
    C = torch.zeros((M, N_), dtype=torch.float32, device="cuda")
    lam, lak = (1, M) if ta else (K, 1)
    lbk, lbn = (1, K) if tb else (N_, 1)
    kl.gemm_bf16(M, N_, K, Ad, lam, lak, Bd, lbk, lbn, C, N_)
    ref = N.bf16(A) @ N.bf16(B)
    scale = np.abs(N.bf16(A)) @ np.abs(N.bf16(B))
    err = np.abs(C.cpu().numpy() - ref)
    assert (err <= 2e-6 * scale + 1e-6).all(), err.max()


def test_gemm_bias_relu_and_accumulate():
    rng = np.random.default_rng(9)
    M, N_, K = 45, 37, 50
    A = rng.normal(size=(M, K)).astype(np.float32)
    B = rng.normal(size=(K, N_)).astype(np.float32)
    bias = rng.normal(size=N_).astype(np.float32)
    C = torch.zeros((M, N_), dtype=torch.float32, device="cuda")
    kl.gemm_bf16(M, N_, K, _dev(A), K, 1, _dev(B), N_, 1, C, N_, bias=_dev(bias), relu=True)
    ref = np.maximum(N.bf16(A) @ N.bf16(B) + bias, 0)
    np.testing.assert_allclose(C.cpu().numpy(), ref, atol=1e-4, rtol=1e-5)
    kl.gemm_bf16(M, N_, K, _dev(A), K, 1, _dev(B), N_, 1, C, N_, accumulate=True)
    np.testing.assert_allclose(C.cpu().numpy(), ref + N.bf16(A) @ N.bf16(B), atol=2e-4, rtol=1e-5)


def _params(seed=0):
    rng = np.random.default_rng(seed + 100)
    return N.init_params(seed) + rng.normal(scale=0.02, size=N.N_PARAMS)


def _sets(n, seed):
    ta, tb = wl.surrogate_sets(n, seed)
    return ta, tb


U32 = 2.0 ** -24


def _gamma(n):
    """Bound of an FP32 sum of n terms in any order, relative to the sum of
    their magnitudes: (n - 1) u / (1 - (n - 1) u)."""
    return (n - 1) * U32 / (1 - (n - 1) * U32)


def _close(name, got, ref, S, n):
    """Element by element: |got - ref| <= gamma(n) S + the rounding of an
    FP32 store."""
    got, ref, S = (np.asarray(a, np.float64) for a in (got, ref, S))
    bound = _gamma(n) * S + U32 * np.abs(ref)
    err = np.abs(got - ref)
    bad = err > bound
    if bad.any():
        i = np.unravel_index(np.argmax(err - bound), err.shape)
        raise AssertionError(f"{name}: {int(bad.sum())} of {err.size} elements beyond their bound; worst at {i}: "
                             f"got {got[i]!r} ref {ref[i]!r} bound {bound[i]!r}")
    return float((err / np.maximum(bound, 1e-300)).max())


def _nchw(x_nhwc, B, H, C):
    return x_nhwc.reshape(B, H, H, C).transpose(0, 3, 1, 2)


def _nhwc(x_nchw):
    return x_nchw.transpose(0, 2, 3, 1)


def test_training_layers_match_reference_element_by_element():
    """Every layer of the training forward and backward on the GPU, checked
    on its own FP32 inputs (read from the workspace, kl_sur_workspace_tensor):
    the reference rounds those same inputs to bfloat16 as the GPU does and
    sums the exact bfloat16 products in FP64, so the GPU's result may differ
    only by its FP32 sums, element by element within gamma(n) times the sum
    of the terms' magnitudes (n terms, in any order); permutations and ReLU
    masks match exactly.  Layer shapes: nn_ref's header."""
    B = 4
    flat = _params(1).astype(np.float32).astype(np.float64)
    P = N.unflatten(flat)
    ta, tb = _sets(B, 12)
    rng = np.random.default_rng(3)
    targets = (rng.random((B, 128, 128)) < 0.05).astype(np.uint8)
    ws = kl.sur_workspace(B)
    loss, grad = kl.sur_loss_grad(_dev(flat), ta, tb, _dev(targets, torch.uint8), workspace=ws)
    torch.cuda.synchronize()
    T = {n: kl.sur_workspace_tensor(ws, B, n).cpu().numpy().astype(np.float64) for n in kl.SUR_TENSORS}
    G = N.unflatten(grad.cpu().numpy().astype(np.float64))
    bf, A = N.bf16, np.abs
    worst = {}

    # features: the FP64 formula rounded once to FP32
    np.testing.assert_array_equal(T["u"].reshape(B, 4), N.features(ta, tb).astype(np.float32))
    u = T["u"].reshape(B, 4)
    # linear layers (bias and ReLU; ReLU cannot increase an error)
    for name, x, W, b, n_in in (("h1", u, P["W1"], P["b1"], 4), ("h2", T["h1"].reshape(B, 256), P["W2"], P["b2"], 256)):
        ref = np.maximum(bf(x) @ bf(W) + b, 0)
        worst[name] = _close(name, T[name].reshape(B, 256), ref, A(bf(x)) @ A(bf(W)) + A(b), n_in + 1)
    # X0 is H2 rearranged
    h2 = T["h2"].reshape(B, 16, 4, 4)
    np.testing.assert_array_equal(_nchw(T["x0"], B, 4, 16), h2)
    # transposed convolutions, NHWC buffers
    ins = [("x0", 4, 16), ("y1", 16, 64), ("y2", 32, 32), ("y3", 64, 16)]
    outs = ["y1", "y2", "y3", "logits"]
    for n, ((K, c, st, pd), (xin, Hi, Ci), yout) in enumerate(zip(N.CONVS, ins, outs)):
        x = _nchw(T[xin], B, Hi, Ci)
        z = N.convT(bf(x), bf(P[K]), P[c], st, pd)
        S = N.convT(A(bf(x)), A(bf(P[K])), A(P[c]), st, pd)
        taps = (-(-4 // st)) ** 2
        if n < 3:
            worst[yout] = _close(yout, T[yout], _nhwc(np.maximum(z, 0)).ravel(), _nhwc(S).ravel(), Ci * taps + 1)
        else:
            worst[yout] = _close(yout, T[yout].reshape(B, 128, 128), z[:, 0], S[:, 0], Ci * taps + 1)
    # loss gradient: (sigmoid(z) - t) / n from the GPU's logits (expf and a few FP32 roundings)
    zl = T["logits"].reshape(B, 128, 128)
    sg = 1 / (1 + np.exp(-zl))
    npx = zl.size
    dref = (sg - targets) / npx
    dl = T["dlogits"].reshape(B, 128, 128)
    assert (np.abs(dl - dref) <= 8 * U32 * (1 + np.abs(sg - targets)) / npx).all()
    # transposed convolutions backward: the input gradient (then the ReLU mask of
    # the forward activation), the weight gradient and the bias gradient
    douts = [("dlogits", 128, 1), ("dy3", 64, 16), ("dy2", 32, 32), ("dy1", 16, 64)]
    dins = ["dy3", "dy2", "dy1", "dx0"]
    for n in range(3, -1, -1):
        K, c, st, pd = N.CONVS[n]
        dname, Ho, Co = douts[3 - n]
        xin, Hi, Ci = ins[n]
        d = _nchw(T[dname], B, Ho, Co)
        x = _nchw(T[xin], B, Hi, Ci)
        dx, dK, db = N.convT_backward(x, P[K], d, st, pd, rnd=bf)
        Sx, SK, _ = N.convT_backward(A(bf(x)), A(bf(P[K])), A(bf(d)), st, pd)
        if n > 0:
            mask = T[xin] > 0
            worst[dins[3 - n]] = _close(dins[3 - n], T[dins[3 - n]], _nhwc(dx).ravel() * mask,
                                        _nhwc(Sx).ravel() * mask, Co * 16)
        else:
            worst["dx0"] = _close("dx0", T["dx0"], _nhwc(dx).ravel(), _nhwc(Sx).ravel(), Co * 16)
        worst["g" + K] = _close("grad " + K, G[K], dK, SK, B * Hi * Hi)
        worst["g" + c] = _close("grad " + c, G[c], d.sum(axis=(0, 2, 3)), A(d).sum(axis=(0, 2, 3)), B * Ho * Ho)
    # DH2 is DX0 rearranged and masked by H2 > 0
    dh2 = _nchw(T["dx0"], B, 4, 16).reshape(B, 256) * (T["h2"].reshape(B, 256) > 0)
    np.testing.assert_array_equal(T["dh2"].reshape(B, 256), dh2)
    h1 = T["h1"].reshape(B, 256)
    worst["gW2"] = _close("grad W2", G["W2"], bf(h1).T @ bf(dh2), A(bf(h1)).T @ A(bf(dh2)), B)
    worst["gb2"] = _close("grad b2", G["b2"], dh2.sum(0), A(dh2).sum(0), B)
    dh1 = T["dh1"].reshape(B, 256)
    ref = (bf(dh2) @ bf(P["W2"]).T) * (h1 > 0)
    worst["dh1"] = _close("dh1", dh1, ref, (A(bf(dh2)) @ A(bf(P["W2"])).T) * (h1 > 0), 256)
    worst["gW1"] = _close("grad W1", G["W1"], bf(u).T @ bf(dh1), A(bf(u)).T @ A(bf(dh1)), B)
    worst["gb1"] = _close("grad b1", G["b1"], dh1.sum(0), A(dh1).sum(0), B)
    print("largest error / bound per layer:", {k: round(v, 4) for k, v in worst.items()})
    # the loss: the mean BCE of the GPU's logits
    assert abs(loss.item() - N.bce_loss(zl, targets)[0]) <= 1e-5 * N.bce_loss(zl, targets)[0]


def test_fused_forward_matches_the_training_forward():
    """Inference (one fused kernel per set, activations in LDS as bfloat16)
    rounds the same operands to bfloat16 as the training forward; the two
    differ by the order of their FP32 sums, and where that moves an
    activation across a bfloat16 rounding boundary, by one bfloat16 step of
    it.  So nearly every logit (all but 0.2%; measured 0.08%) agrees within
    gamma(n) of the last layer's magnitudes, computed from the training
    path's own last input, and every logit within one bfloat16 step of the
    last layer's magnitudes."""
    B = 36
    flat = _params(0).astype(np.float32).astype(np.float64)
    P = N.unflatten(flat)
    ta, tb = _sets(B, 11)
    rng = np.random.default_rng(8)
    targets = (rng.random((B, 128, 128)) < 0.05).astype(np.uint8)
    ws = kl.sur_workspace(B)
    kl.sur_loss_grad(_dev(flat), ta, tb, _dev(targets, torch.uint8), workspace=ws)
    z_train = kl.sur_workspace_tensor(ws, B, "logits").cpu().numpy().astype(np.float64).reshape(B, 128, 128)
    y3 = _nchw(kl.sur_workspace_tensor(ws, B, "y3").cpu().numpy().astype(np.float64), B, 64, 16)
    z = kl.sur_forward(_dev(flat), ta, tb).cpu().numpy().astype(np.float64)
    K, c, st, pd = N.CONVS[3]
    S = N.convT(np.abs(N.bf16(y3)), np.abs(N.bf16(P[K])), np.abs(P[c]), st, pd)[:, 0]
    err = np.abs(z - z_train)
    tight = 2 * _gamma(65) * S + 2 * U32 * np.abs(z_train)
    frac = float((err > tight).mean())
    print(f"fused vs training logits: {frac:.2e} of {err.size} beyond 2 gamma(65) S; max err / S {(err / S).max():.2e}")
    assert frac < 2e-3
    assert (err <= 2.0 ** -8 * S + tight).all()


def test_fused_forward_logits_match_reference_statistically():
    """The fused forward against the FP64 reference from the features on:
    rounding differences compound over six layers, so this is checked on the
    whole image: the logits' RMS error stays within 1e-3 of their RMS."""
    flat = _params(0)
    ta, tb = _sets(36, 11)
    z = kl.sur_forward(_dev(flat), ta, tb).cpu().numpy()
    ref, _ = N.forward(flat.astype(np.float32).astype(np.float64), ta, tb, rnd=N.bf16)
    rms = np.sqrt((ref ** 2).mean())
    assert np.sqrt(((z - ref) ** 2).mean()) <= 1e-3 * rms


def test_fused_forward_is_batch_independent():
    """Inference runs one set per workgroup: a set's logits do not depend on
    the batch around it, from a batch of one to the largest batch."""
    flat = _dev(_params(5))
    ta, tb = _sets(512, 13)
    full = kl.sur_forward(flat, ta, tb)
    assert torch.isfinite(full).all()
    for i in (0, 1, 255, 256, 511):
        one = kl.sur_forward(flat, ta[i:i + 1], tb[i:i + 1])
        assert torch.equal(one[0], full[i]), i
    part = kl.sur_forward(flat, ta[100:137], tb[100:137])
    assert torch.equal(part, full[100:137])


def test_fused_forward_agrees_with_the_training_forward():
    """Inference (fused decoder) and training (column form) round the same
    operands to bfloat16; only the order of FP32 sums differs."""
    flat = _params(6)
    ta, tb = _sets(24, 14)
    rng = np.random.default_rng(8)
    targets = (rng.random((24, 128, 128)) < 0.05).astype(np.uint8)
    loss, _ = kl.sur_loss_grad(_dev(flat), ta, tb, _dev(targets, torch.uint8))
    z = kl.sur_forward(_dev(flat), ta, tb).cpu().numpy().astype(np.float64)
    assert abs(N.bce_loss(z, targets)[0] - loss.item()) <= 1e-4 * abs(loss.item())


def test_adam_matches_reference():
    rng = np.random.default_rng(4)
    p = rng.normal(size=N.N_PARAMS)
    g = rng.normal(size=N.N_PARAMS)
    m = rng.normal(size=N.N_PARAMS) * 0.1
    v = np.abs(rng.normal(size=N.N_PARAMS)) * 0.01
    pd, md, vd = _dev(p), _dev(m), _dev(v)
    kl.sur_adam(pd, _dev(g), md, vd, 7, 1e-3)
    rp, rm, rv = N.adam(p.astype(np.float32).astype(np.float64), g.astype(np.float32).astype(np.float64),
                        m.astype(np.float32).astype(np.float64), v.astype(np.float32).astype(np.float64), 7, 1e-3)
    # FP32 vs FP64: errors are relative to the magnitudes of the terms combined;
    # 0.999 and 1 - 0.999 carry a relative representation error of 1.3e-5 in FP32
    m32, v32, g32 = (x.astype(np.float32).astype(np.float64) for x in (m, v, g))
    assert (np.abs(md.cpu().numpy() - rm) <= 1e-6 * (0.9 * np.abs(m32) + 0.1 * np.abs(g32)) + 1e-12).all()
    assert (np.abs(vd.cpu().numpy() - rv) <= 3e-5 * (0.999 * v32 + 0.001 * g32 ** 2) + 1e-15).all()
    assert (np.abs(pd.cpu().numpy() - rp) <= 2e-7 * np.abs(rp) + 5e-7).all()


def test_occupancy_uncertainty_iou():
    rng = np.random.default_rng(6)
    counts = rng.integers(0, 3, size=(5, 128, 128)).astype(np.int32)
    occ = kl.occupancy(_dev(counts, torch.int32)).cpu().numpy()
    np.testing.assert_array_equal(occ, counts > 0)
    z = rng.normal(scale=4, size=(5, 128, 128)).astype(np.float32)
    u = kl.sur_uncertainty(_dev(z)).cpu().numpy()
    p = 1 / (1 + np.exp(-z.astype(np.float64)))
    ent = -(p * np.log(p) + (1 - p) * np.log(1 - p))
    np.testing.assert_allclose(u, ent.reshape(5, -1).mean(1), rtol=1e-4)
    t = (rng.random((5, 128, 128)) < 0.1).astype(np.uint8)
    t[4] = 0
    z[4] = -1.0
    io = kl.iou(_dev(t, torch.uint8), logits=_dev(z)).cpu().numpy()
    np.testing.assert_allclose(io, N.iou(z > 0, t > 0), rtol=1e-6)
    io2 = kl.iou(_dev(t, torch.uint8), pred_occ=_dev((z > 0).astype(np.uint8), torch.uint8)).cpu().numpy()
    np.testing.assert_allclose(io2, io)


def _targets(ta, tb, depth):
    return kl.occupancy(kl.render_many(ta, tb, np.full(len(ta), depth), wl.SURROGATE_WINDOW))


def test_training_follows_reference_trajectory():
    """Twelve Adam steps on the GPU and in the FP64 reference (BF16 operands
    emulated) from the same start: the losses stay together step by step."""
    ta, tb = _sets(8, 14)
    occ = _targets(ta, tb, 10)
    occ_h = occ.cpu().numpy()
    flat = N.init_params(5)
    flat[-1] = np.log(occ_h.mean() / (1 - occ_h.mean()))
    params = _dev(flat)
    m, v, grad = torch.zeros_like(params), torch.zeros_like(params), torch.zeros_like(params)
    loss = torch.zeros(1, device="cuda")
    ws = kl.sur_workspace(8)
    ta_d, tb_d = kl.as_c64(ta), kl.as_c64(tb)
    rp, rm, rv = flat.copy(), np.zeros_like(flat), np.zeros_like(flat)
    for step in range(1, 13):
        kl.sur_train_step(params, m, v, grad, step, 1e-3, ta_d, tb_d, occ, ws, loss)
        ref_loss, g = N.loss_and_grad(rp, ta, tb, occ_h, rnd=N.bf16)
        rp, rm, rv = N.adam(rp, g, rm, rv, step, 1e-3)
        assert abs(loss.item() - ref_loss) <= 0.02 * ref_loss, (step, loss.item(), ref_loss)


def test_training_reduces_loss():
    ta, tb = _sets(64, 13)
    occ = _targets(ta, tb, 10)
    p0 = float(occ.float().mean())
    flat = N.init_params(2)
    flat[-1] = np.log(p0 / (1 - p0))   # last bias at the prior's logit
    params = _dev(flat)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    grad = torch.zeros_like(params)
    loss = torch.zeros(1, device="cuda")
    ws = kl.sur_workspace(16)
    ta_d, tb_d = kl.as_c64(ta), kl.as_c64(tb)
    losses = []
    for step in range(1, 201):
        i = (step * 16) % 64
        kl.sur_train_step(params, m, v, grad, step, 1e-3, ta_d[i:i + 16], tb_d[i:i + 16], occ[i:i + 16], ws, loss)
        losses.append(loss.item())
    const = -(p0 * np.log(p0) + (1 - p0) * np.log(1 - p0))
    assert np.mean(losses[-16:]) < 0.8 * const, (const, losses[:8], losses[-8:])


def test_gated_scan_keeps_accepted_predictions_and_renders_the_rest():
    """scan(): the sets the gate accepts keep the surrogate's predicted
    occupancy (logits > 0), the others are the plain renderer's occupancy bit
    for bit; after a short training, every calibration set at or below the
    calibrated threshold reaches the IoU target."""
    from paper_1709_08018_amd import surrogate as S
    ta, tb = _sets(96, 21)
    occ = _targets(ta, tb, 10)
    params, _ = S.train(ta[:64], tb[:64], occ[:64], steps=150, batch=16, lr=2e-3, seed=0)
    logits = S.predict(params, ta[64:], tb[64:])
    iou = kl.iou(occ[64:], logits=logits).cpu().numpy()
    unc = kl.sur_uncertainty(logits).cpu().numpy()
    target = float(np.median(iou))
    tau = S.gate_threshold(unc, iou, target)
    assert (iou[unc <= tau] >= target).all()
    tau_s = float(np.median(unc))
    scan_occ, accepted, _ = S.scan(params, ta[64:], tb[64:], tau_s, depth=10)
    np.testing.assert_array_equal(accepted, unc <= tau_s)
    assert accepted.any() and (~accepted).any()
    pred = (logits > 0).to(torch.uint8)
    for i in range(len(accepted)):
        want = pred[i] if accepted[i] else occ[64 + i]
        assert torch.equal(scan_occ[i], want), i
