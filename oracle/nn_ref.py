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


# ---------------------------------------------------------------- element-wise error scales
# An error model of the GPU's arithmetic against this reference (rnd = bf16
# throughout), carried layer by layer next to the FP64 values: for every
# element a scale sigma of the GPU's rounding error, and a worst-case part
# `hard` for the rare events the model does not cover.
#  * The GPU rounds the same operands to bfloat16, from FP32 values within
#    about sigma of the reference's.  Rounding erases an error much smaller
#    than a bfloat16 step unless it crosses a rounding boundary, which it
#    does with probability about sigma / step, by one step: a variance of
#    about sigma * step (plus sigma^2, for values so small that the step is
#    below sigma).
#  * Products of bfloat16 numbers are exact in FP32; the n roundings of an
#    FP32 sum, each at most u32 = 2^-24 of a partial sum at most S = the sum
#    of the terms' magnitudes, add a variance of at most n (u32 S)^2
#    (probabilistic rounding-error analysis in the manner of Higham and
#    Mary, SIAM J. Sci. Comput. 2019: independent errors add in quadrature;
#    the worst-case bound, linear in n and compounded through the layers'
#    absolute values, exceeds the logits themselves).  A bias add or an
#    FP32 store adds one rounding.
#  * Independent variances add through the linear maps with the squares of
#    their coefficients; ReLU does not increase an error.
#  * A backward ReLU mask whose forward input lies within KSIGMA sigma of 0
#    may differ on the GPU: the masked value then counts in full in `hard`,
#    which propagates with the coefficients' magnitudes.
# A GPU value passes when it lies within KSIGMA sigma + hard of the
# reference.
U32 = 2.0 ** -24
KSIGMA = 8.0


def _step(x):
    """Spacing of bfloat16 numbers at |x| (8 significant bits); 0 at 0."""
    a = np.abs(np.asarray(x, np.float64))
    e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    return np.where(a > 0, 2.0 ** (e - 7), 0.0)


def _round_var(x, sig):
    """Variance of bf16 of the GPU's value against bf16 of the reference's."""
    return sig * _step(x) + sig * sig


def _hard_after_round(x, hard):
    """Worst case of a bf16 rounding of a value with a worst-case error."""
    return np.where(hard > 0, hard + _step(x) + _step(np.abs(x) + hard), 0.0)


def _mask(d, sd, hd, z, sz, hz):
    """d * (z > 0) on the GPU, where z may differ by sz (scale) and hz (worst
    case): (value, sigma, hard)."""
    m = z > 0
    unsure = np.abs(z) <= KSIGMA * sz + hz
    return d * m, np.where(m, sd, 0.0), np.where(unsure, np.abs(d) + sd + hd, np.where(m, hd, 0.0))


def _taps_per_output(s, k):
    """Taps of a k x k transposed convolution with stride s that reach one output pixel."""
    return (-(-k // s)) ** 2


def _linear(xr, vx, hx, W, b, n):
    """y = xr @ W + b with input variances vx and worst cases hx (after the
    bf16 rounding), W already rounded: (y, sigma_y, hard_y)."""
    y = xr @ W + b
    S = np.abs(xr) @ np.abs(W)
    var = vx @ (W * W) + n * (U32 * S) ** 2 + (U32 * y) ** 2
    return y, np.sqrt(var), hx @ np.abs(W)


def forward_scales(flat, ta, tb):
    """The reference logits (bf16 at the GPU's rounding points), the error
    scale sigma and worst-case part hard of the GPU's FP32 logits, element by
    element, and the activations with theirs for `loss_and_grad_scales`."""
    P = unflatten(flat)
    u = features(ta, tb)
    su = 4 * U32 * (np.abs(u) + 4.0)   # the features are formed in FP32 on the GPU
    hu = np.zeros_like(u)
    z1, s1, h1h = _linear(bf16(u), _round_var(u, su), hu, bf16(P["W1"]), P["b1"], 4)
    h1 = np.maximum(z1, 0)
    z2, s2, h2h = _linear(bf16(h1), _round_var(h1, s1), _hard_after_round(h1, h1h), bf16(P["W2"]), P["b2"], 256)
    h2 = np.maximum(z2, 0)
    x = h2.reshape(-1, 16, 4, 4)
    acts, pre = [x], [(z2.reshape(-1, 16, 4, 4), s2.reshape(-1, 16, 4, 4), h2h.reshape(-1, 16, 4, 4))]
    sx, hx = s2.reshape(-1, 16, 4, 4), h2h.reshape(-1, 16, 4, 4)
    for n, (K, c, s, p) in enumerate(CONVS):
        Kr = bf16(P[K])
        xr = bf16(acts[-1])
        z = convT(xr, Kr, P[c], s, p)
        zero = np.zeros_like(P[c])
        nt = Kr.shape[0] * _taps_per_output(s, Kr.shape[2])
        S = convT(np.abs(xr), np.abs(Kr), zero, s, p)
        var = convT(_round_var(acts[-1], sx), Kr * Kr, zero, s, p) + nt * (U32 * S) ** 2 + (U32 * z) ** 2
        hz = convT(_hard_after_round(acts[-1], hx), np.abs(Kr), zero, s, p)
        sx, hx = np.sqrt(var), hz
        pre.append((z, sx, hx))
        acts.append(np.maximum(z, 0) if n < 3 else z)
    cache = {"u": u, "su": su, "z1": z1, "s1": s1, "h1h": h1h, "h1": h1, "z2": z2, "s2": s2, "h2h": h2h, "h2": h2,
             "acts": acts, "pre": pre, "P": P}
    return acts[-1][:, 0], pre[-1][1][:, 0], pre[-1][2][:, 0], cache


def loss_and_grad_scales(flat, ta, tb, targets):
    """The reference loss and gradient (bf16 at the GPU's rounding points)
    and, element by element, the error scale sigma and worst-case part hard
    of the GPU's FP32 gradient, following `backward` step by step."""
    logits, slog, hlog, cache = forward_scales(flat, ta, tb)
    loss, dz = bce_loss(logits, targets)
    P, acts, pre = cache["P"], cache["acts"], cache["pre"]
    # sigmoid is 1/4-Lipschitz; the GPU's sigmoid and difference add a few roundings
    sd = np.sqrt((slog / 4) ** 2 + (8 * U32) ** 2) / dz.size
    d, sdd, hd = dz[:, None], sd[:, None], (hlog / 4 / dz.size)[:, None]
    g, sg, hg = {}, {}, {}
    B = dz.shape[0]
    for n in range(3, -1, -1):
        K, c, s, p = CONVS[n]
        if n < 3:
            z, sz, hz = pre[n + 1]
            d, sdd, hd = _mask(d, sdd, hd, z, sz, hz)
        x = acts[n]
        sx, hx = pre[n][1], pre[n][2]
        xr, dr, Kr = bf16(x), bf16(d), bf16(P[K])
        vx, vd = _round_var(x, sx), _round_var(d, sdd)
        hxr, hdr = _hard_after_round(x, hx), _hard_after_round(d, hd)
        ones = np.ones_like(x)
        dxv, gK, gb = convT_backward(x, P[K], d, s, p, rnd=bf16)
        # dx: each input pixel gathers Co outputs over the taps that reach it
        n_dx = Kr.shape[1] * Kr.shape[2] * Kr.shape[3]
        S_dx, _, _ = convT_backward(ones, np.abs(Kr), np.abs(dr), s, p)
        v_dx, _, _ = convT_backward(ones, Kr * Kr, vd, s, p)
        h_dx, _, _ = convT_backward(ones, np.abs(Kr), hdr, s, p)
        s_dx = np.sqrt(v_dx + n_dx * (U32 * S_dx) ** 2 + (U32 * dxv) ** 2)
        # dK: for each tap, a sum over the batch and the input pixels
        n_dk = B * x.shape[2] * x.shape[3]
        _, S_k, _ = convT_backward(np.abs(xr), np.abs(Kr), np.abs(dr), s, p)
        _, v1, _ = convT_backward(xr * xr, Kr, vd, s, p)
        _, v2, _ = convT_backward(vx, Kr, dr * dr, s, p)
        _, h1k, _ = convT_backward(np.abs(xr) + hxr, Kr, hdr, s, p)
        _, h2k, _ = convT_backward(hxr, Kr, np.abs(dr), s, p)
        g[K], sg[K], hg[K] = gK, np.sqrt(v1 + v2 + n_dk * (U32 * S_k) ** 2), h1k + h2k
        n_db = B * d.shape[2] * d.shape[3]
        g[c] = gb
        sg[c] = np.sqrt((sdd ** 2).sum(axis=(0, 2, 3)) + n_db * (U32 * np.abs(d).sum(axis=(0, 2, 3))) ** 2)
        hg[c] = hd.sum(axis=(0, 2, 3))
        d, sdd, hd = dxv, s_dx, h_dx
    d2, s2, h2 = d.reshape(-1, 256), sdd.reshape(-1, 256), hd.reshape(-1, 256)
    dh2, sdh2, hdh2 = _mask(d2, s2, h2, cache["z2"], cache["s2"], cache["h2h"])
    h1 = cache["h1"]
    h1r, dr = bf16(h1), bf16(dh2)
    vh1, vd = _round_var(h1, cache["s1"]), _round_var(dh2, sdh2)
    hh1, hdr = _hard_after_round(h1, cache["h1h"]), _hard_after_round(dh2, hdh2)
    g["W2"] = h1r.T @ dr
    sg["W2"] = np.sqrt((h1r * h1r).T @ vd + vh1.T @ (dr * dr) + B * (U32 * (np.abs(h1r).T @ np.abs(dr))) ** 2)
    hg["W2"] = (np.abs(h1r) + hh1).T @ hdr + hh1.T @ np.abs(dr)
    g["b2"] = dh2.sum(0)
    sg["b2"] = np.sqrt((sdh2 ** 2).sum(0) + B * (U32 * np.abs(dh2).sum(0)) ** 2)
    hg["b2"] = hdh2.sum(0)
    W2 = bf16(P["W2"])
    v, sv, hv = _linear(dr, vd, hdr, W2.T, 0.0, 256)
    dh1, sdh1, hdh1 = _mask(v, sv, hv, cache["z1"], cache["s1"], cache["h1h"])
    u = cache["u"]
    ur, qr = bf16(u), bf16(dh1)
    vu, vq = _round_var(u, cache["su"]), _round_var(dh1, sdh1)
    hq = _hard_after_round(dh1, hdh1)
    g["W1"] = ur.T @ qr
    sg["W1"] = np.sqrt((ur * ur).T @ vq + vu.T @ (qr * qr) + B * (U32 * (np.abs(ur).T @ np.abs(qr))) ** 2)
    hg["W1"] = np.abs(ur).T @ hq
    g["b1"] = dh1.sum(0)
    sg["b1"] = np.sqrt((sdh1 ** 2).sum(0) + B * (U32 * np.abs(dh1).sum(0)) ** 2)
    hg["b1"] = hdh1.sum(0)
    return loss, flatten(g), flatten(sg), flatten(hg)
