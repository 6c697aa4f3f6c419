"""Pins of the FP64 reference network against independent facts.

Transposed convolution with stride 1 is a full 2-D convolution, and with
stride s it is a full convolution of the input with zeros inserted between
samples (scipy computes both); gradients equal central finite differences;
Adam's first step has the closed form lr * g / (|g| + eps); the loss equals
the textbook cross entropy of the sigmoid.
"""
import numpy as np
import pytest
from scipy import signal

from oracle import nn_ref as N


def _convT_scipy(x, K, s, p):
    B, Ci, H, W = x.shape
    _, Co, kh, kw = K.shape
    up = np.zeros((B, Ci, (H - 1) * s + 1, (W - 1) * s + 1))
    up[:, :, ::s, ::s] = x
    Ho, Wo = (H - 1) * s - 2 * p + kh, (W - 1) * s - 2 * p + kw
    out = np.zeros((B, Co, Ho, Wo))
    for b in range(B):
        for o in range(Co):
            acc = sum(signal.convolve2d(up[b, c], K[c, o], mode="full") for c in range(Ci))
            out[b, o] = acc[p:p + Ho, p:p + Wo]
    return out


@pytest.mark.parametrize("s,p", [(1, 0), (2, 1), (4, 0), (2, 0), (3, 1)])
def test_convT_equals_scipy_convolution(s, p):
    rng = np.random.default_rng(s * 10 + p)
    x = rng.normal(size=(2, 3, 5, 4))
    K = rng.normal(size=(3, 2, 4, 4))
    bias = np.zeros(2)
    np.testing.assert_allclose(N.convT(x, K, bias, s, p), _convT_scipy(x, K, s, p), atol=1e-12)


def test_shapes_and_param_count():
    assert N.N_PARAMS == 4 * 256 + 256 + 256 * 256 + 256 + 16 * 64 * 16 + 64 + 64 * 32 * 16 + 32 + 32 * 16 * 16 + 16 + 16 * 16 + 1
    flat = N.init_params(0)
    z, _ = N.forward(flat, np.array([2.1 + 0.1j, 2.5 - 0.2j]), np.array([2.0, 2.9 + 0.3j]))
    assert z.shape == (2, 128, 128)


def test_bce_matches_textbook_formula():
    rng = np.random.default_rng(1)
    z = rng.normal(scale=3, size=(3, 8, 8))
    t = rng.integers(0, 2, size=z.shape)
    sig = 1 / (1 + np.exp(-z))
    ref = -(t * np.log(sig) + (1 - t) * np.log(1 - sig)).mean()
    loss, grad = N.bce_loss(z, t)
    assert abs(loss - ref) < 1e-12
    eps = 1e-6
    k = (1, 3, 4)
    zp, zm = z.copy(), z.copy()
    zp[k] += eps
    zm[k] -= eps
    fd = (N.bce_loss(zp, t)[0] - N.bce_loss(zm, t)[0]) / (2 * eps)
    assert abs(fd - grad[k]) < 1e-9


def test_gradients_equal_finite_differences():
    rng = np.random.default_rng(2)
    flat = N.init_params(3) + rng.normal(scale=0.05, size=N.N_PARAMS)   # non-zero biases too
    ta = np.array([2.2 + 0.1j, 2.7 - 0.25j, 1.9 + 0.02j])
    tb = np.array([2.4 - 0.1j, 2.0 + 0.2j, 2.95 + 0.0j])
    targets = rng.integers(0, 2, size=(3, 128, 128))
    _, grad = N.loss_and_grad(flat, ta, tb, targets)
    offsets = np.cumsum([0] + [int(np.prod(s)) for _, s in N.LAYOUT])
    eps = 1e-6
    for t, (name, _) in enumerate(N.LAYOUT):
        idx = rng.integers(offsets[t], offsets[t + 1], size=4)
        for i in idx:
            fp, fm = flat.copy(), flat.copy()
            fp[i] += eps
            fm[i] -= eps
            fd = (N.loss_and_grad(fp, ta, tb, targets)[0] - N.loss_and_grad(fm, ta, tb, targets)[0]) / (2 * eps)
            assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (name, i, fd, grad[i])


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(4)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    new, m, v = N.adam(p, g, np.zeros(50), np.zeros(50), 1, 1e-3)
    np.testing.assert_allclose(new, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)


def test_bf16_rounding():
    assert N.bf16(1.0) == 1.0
    assert N.bf16(1.0 + 2 ** -8) == 1.0                # tie -> even
    assert N.bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6  # tie -> even (up)
    assert N.bf16(1.0 + 2 ** -7) == 1.0 + 2 ** -7
    x = np.random.default_rng(5).normal(size=1000)
    assert (np.abs(N.bf16(x) - x) <= np.abs(x) * 2 ** -8).all()
    assert (np.abs(N.bf16(x) - x) > 0).any()


def test_iou():
    a = np.zeros((3, 4, 4), bool)
    b = np.zeros((3, 4, 4), bool)
    a[0, 0, :2] = True
    b[0, 0, 1:3] = True
    a[1, 2, 2] = b[1, 2, 2] = True
    np.testing.assert_allclose(N.iou(a, b), [1 / 3, 1.0, 1.0])
