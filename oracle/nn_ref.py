"""FP64 numpy reference of the occupancy surrogate network.

TEST INFRASTRUCTURE ONLY: the test suite and the smoke check are its only
users; it shares no code with the GPU library.  Plain definitions, written
out: no fusion, no blocking.

Network (parameters (ta, tb) -> 128 x 128 occupancy logits):
  u  = [(Re ta - 2.4)/0.6, Im ta/0.3, (Re tb - 2.4)/0.6, Im tb/0.3]
  h1 = relu(u W1 + b1)                    4 -> 256
  h2 = relu(h1 W2 + b2)                   256 -> 256, read as 16 x 4 x 4 (c, y, x)
  c1 = relu(convT(h2, K1, s=4, p=0))      16 -> 64 channels, 4 -> 16 pixels
  c2 = relu(convT(c1, K2, s=2, p=1))      64 -> 32, 16 -> 32
  c3 = relu(convT(c2, K3, s=2, p=1))      32 -> 16, 32 -> 64
  z  =      convT(c3, K4, s=2, p=1)       16 -> 1, 64 -> 128   (logits)
with convT(x, K, s, p)[b, o, s*i - p + ky, s*j - p + kx] += x[b, c, i, j] K[c, o, ky, kx]
plus a per-channel bias; loss = mean over pixels and samples of the binary
cross entropy of sigmoid(z) against the 0/1 occupancy; Adam updates.

`rnd` marks where the GPU rounds operands to bfloat16 (round to nearest
even); pass `rnd=bf16` to emulate it, `rnd=None` for plain FP64.
"""
from __future__ import annotations

import numpy as np

# (name, shape) in the order of the flat parameter vector
LAYOUT = [
    ("W1", (4, 256)), ("b1", (256,)),
    ("W2", (256, 256)), ("b2", (256,)),
    ("K1", (16, 64, 4, 4)), ("c1", (64,)),
    ("K2", (64, 32, 4, 4)), ("c2", (32,)),
    ("K3", (32, 16, 4, 4)), ("c3", (16,)),
    ("K4", (16, 1, 4, 4)), ("c4", (1,)),
]
CONVS = [("K1", "c1", 4, 0), ("K2", "c2", 2, 1), ("K3", "c3", 2, 1), ("K4", "c4", 2, 1)]
N_PARAMS = sum(int(np.prod(s)) for _, s in LAYOUT)
IMG = 128


def unflatten(flat):
    out, o = {}, 0
    for name, shape in LAYOUT:
        n = int(np.prod(shape))
        out[name] = np.asarray(flat[o:o + n], np.float64).reshape(shape)
        o += n
    return out


def flatten(d):
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in LAYOUT])


def init_params(seed: int) -> np.ndarray:
    """He-style initialisation (normal, std sqrt(2 / fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shape in LAYOUT:
        if len(shape) == 1:
            d[name] = np.zeros(shape)
        elif len(shape) == 2:
            d[name] = rng.normal(0, np.sqrt(2.0 / shape[0]), shape)
        else:  # convT: fan-in per output pixel = Cin * (k / s)^2; use Cin * 4
            d[name] = rng.normal(0, np.sqrt(2.0 / (shape[0] * 4)), shape)
    return flatten(d)


def bf16(x):
    """Round to bfloat16 (nearest even) via float32, returned as float64."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _id(x):
    return np.asarray(x, np.float64)


def features(ta, tb):
    ta = np.asarray(ta, np.complex128)
    tb = np.asarray(tb, np.complex128)
    return np.stack([(ta.real - 2.4) / 0.6, ta.imag / 0.3, (tb.real - 2.4) / 0.6, tb.imag / 0.3], axis=1)


def _taps(n_in, n_out, s, p, k):
    """Input positions i whose output s*i - p + k lies in [0, n_out): a slice
    of inputs and the matching strided slice of outputs."""
    lo = max(0, -((k - p) // s) if k - p < 0 else 0)
    while s * lo - p + k < 0:
        lo += 1
    hi = n_in - 1
    while hi >= lo and s * hi - p + k >= n_out:
        hi -= 1
    if hi < lo:
        return None
    o0 = s * lo - p + k
    return slice(lo, hi + 1), slice(o0, o0 + s * (hi - lo) + 1, s)


def convT(x, K, bias, s, p, rnd=None):
    """Transposed convolution by its scatter definition (kernel size from K):
    for every tap (ky, kx), input pixel (i, j) adds x[:, :, i, j] K[:, :, ky, kx]
    to output pixel (s i - p + ky, s j - p + kx)."""
    r = rnd or _id
    x, K = r(x), r(K)
    B, Ci, H, W = x.shape
    _, Co, kh, kw = K.shape
    Ho, Wo = (H - 1) * s - 2 * p + kh, (W - 1) * s - 2 * p + kw
    out = np.zeros((B, Co, Ho, Wo))
    for ky in range(kh):
        ty = _taps(H, Ho, s, p, ky)
        for kx in range(kw):
            tx = _taps(W, Wo, s, p, kx)
            if ty is None or tx is None:
                continue
            contrib = np.einsum("bchw,co->bohw", x[:, :, ty[0], tx[0]], K[:, :, ky, kx])
            out[:, :, ty[1], tx[1]] += contrib
    return out + bias[None, :, None, None]


def convT_backward(x, K, dout, s, p, rnd=None):
    """Adjoints of convT: (dx, dK, dbias), each by its own gather definition:
    input pixel (i, j) and tap (ky, kx) read dout at (s i - p + ky, s j - p + kx)."""
    r = rnd or _id
    xr, Kr, dr = r(x), r(K), r(dout)
    B, Ci, H, W = x.shape
    _, Co, kh, kw = K.shape
    Ho, Wo = dout.shape[2], dout.shape[3]
    dx = np.zeros_like(xr)
    dK = np.zeros_like(Kr)
    for ky in range(kh):
        ty = _taps(H, Ho, s, p, ky)
        for kx in range(kw):
            tx = _taps(W, Wo, s, p, kx)
            if ty is None or tx is None:
                continue
            g = dr[:, :, ty[1], tx[1]]
            dx[:, :, ty[0], tx[0]] += np.einsum("bohw,co->bchw", g, Kr[:, :, ky, kx])
            dK[:, :, ky, kx] = np.einsum("bchw,bohw->co", xr[:, :, ty[0], tx[0]], g)
    db = dout.sum(axis=(0, 2, 3))
    return dx, dK, db


def forward(flat, ta, tb, rnd=None):
    """Logits (B, 128, 128) and the activations the backward pass needs."""
    r = rnd or _id
    P = unflatten(flat)
    u = features(ta, tb)
    h1 = np.maximum(r(u) @ r(P["W1"]) + P["b1"], 0)
    h2 = np.maximum(r(h1) @ r(P["W2"]) + P["b2"], 0)
    x = h2.reshape(-1, 16, 4, 4)
    acts = [x]
    for n, (K, c, s, p) in enumerate(CONVS):
        z = convT(acts[-1], P[K], P[c], s, p, rnd)
        acts.append(np.maximum(z, 0) if n < 3 else z)
    cache = {"u": u, "h1": h1, "h2": h2, "acts": acts, "P": P}
    return acts[-1][:, 0], cache


def bce_loss(logits, targets):
    """Mean binary cross entropy of sigmoid(z) against t, and d loss / d z."""
    z = np.asarray(logits, np.float64)
    t = np.asarray(targets, np.float64)
    loss = np.maximum(z, 0) - z * t + np.log1p(np.exp(-np.abs(z)))
    grad = (1.0 / (1.0 + np.exp(-z)) - t) / z.size
    return loss.mean(), grad


def backward(cache, dlogits, rnd=None):
    r = rnd or _id
    P = cache["P"]
    acts = cache["acts"]
    g = {}
    d = np.asarray(dlogits, np.float64)[:, None]
    for n in range(3, -1, -1):
        K, c, s, p = CONVS[n]
        if n < 3:
            d = d * (acts[n + 1] > 0)
        dx, g[K], g[c] = convT_backward(acts[n], P[K], d, s, p, rnd)
        d = dx
    dh2 = d.reshape(-1, 256) * (cache["h2"] > 0)
    g["W2"] = r(cache["h1"]).T @ r(dh2)
    g["b2"] = dh2.sum(0)
    dh1 = (r(dh2) @ r(P["W2"]).T) * (cache["h1"] > 0)
    g["W1"] = r(cache["u"]).T @ r(dh1)
    g["b1"] = dh1.sum(0)
    return flatten(g)


def loss_and_grad(flat, ta, tb, targets, rnd=None):
    logits, cache = forward(flat, ta, tb, rnd)
    loss, dz = bce_loss(logits, targets)
    return loss, backward(cache, dz, rnd)


def adam(flat, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (step counts from 1); returns new (params, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mhat = m / (1 - beta1 ** step)
    vhat = v / (1 - beta2 ** step)
    return flat - lr * mhat / (np.sqrt(vhat) + eps), m, v


def iou(pred, target):
    """|P and T| / |P or T| per sample (1 when both are empty)."""
    p = np.asarray(pred, bool).reshape(len(pred), -1)
    t = np.asarray(target, bool).reshape(len(target), -1)
    inter = (p & t).sum(1)
    union = (p | t).sum(1)
    return np.where(union == 0, 1.0, inter / np.maximum(union, 1))
