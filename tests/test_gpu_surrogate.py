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


def test_forward_matches_reference():
    # 36 sets: every layer's buffers exceed 2^21 elements, beyond one thread per element of a capped grid
    flat = _params(0)
    ta, tb = _sets(36, 11)
    z = kl.sur_forward(_dev(flat), ta, tb).cpu().numpy()
    ref, _ = N.forward(flat, ta, tb, rnd=N.bf16)
    rms = np.sqrt((ref ** 2).mean())
    assert np.abs(z - ref).max() <= 2e-2 * rms + 1e-4, (np.abs(z - ref).max(), rms)


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


def test_loss_and_gradients_match_reference():
    flat = _params(1)
    ta, tb = _sets(12, 12)
    rng = np.random.default_rng(3)
    targets = (rng.random((12, 128, 128)) < 0.05).astype(np.uint8)
    loss, grad = kl.sur_loss_grad(_dev(flat), ta, tb, _dev(targets, torch.uint8))
    ref_loss, ref_grad = N.loss_and_grad(flat, ta, tb, targets, rnd=N.bf16)
    assert abs(loss.item() - ref_loss) <= 1e-3 * abs(ref_loss)
    g = grad.cpu().numpy().astype(np.float64)
    off = 0
    for name, shape in N.LAYOUT:
        n = int(np.prod(shape))
        a, b = g[off:off + n], ref_grad[off:off + n]
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        assert rel <= 3e-2, (name, rel)
        off += n


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
