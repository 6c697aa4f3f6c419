"""Python binding of libkl (``include/kl.h``).

Argument marshalling only: every step of a render runs in the HIP library.
PyTorch supplies device buffers and the current stream; the library never
sees a torch type.  Importing this module loads ``libkl.so``; a missing or
unloadable library raises ``KLError`` (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import torch  # loads the HIP runtime that libkl shares

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libkl.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "kl.h")
HEADERS = [HEADER, os.path.join(os.path.dirname(PKG), "include", "kl_surrogate.h")]

KL_OK, KL_EINVAL, KL_ERANGE, KL_ESINGULAR, KL_EDEVICE, KL_ENOMEM = 0, -1, -2, -3, -4, -5
PREC = {"fp32": 0, "fp64": 1}
HIST = {"auto": 0, "runs": 1, "lds": 2}
SEED = {"own": 0, "all": 1, "a": 2, "b": 3, "A": 4, "B": 5}


class KLError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libkl error {code}: {msg}")
        self.code = code


class c64(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class Window(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_double), ("x1", ctypes.c_double), ("y0", ctypes.c_double),
                ("y1", ctypes.c_double), ("width", ctypes.c_uint32), ("height", ctypes.c_uint32)]


class Opts(ctypes.Structure):
    _fields_ = [("min_depth", ctypes.c_int), ("precision", ctypes.c_int), ("use_range", ctypes.c_int),
                ("first_idx", ctypes.c_uint64), ("count", ctypes.c_uint64), ("accumulate", ctypes.c_int),
                ("stream", ctypes.c_void_p), ("dropped_out", ctypes.c_void_p), ("tail_len", ctypes.c_int),
                ("lane_len", ctypes.c_int), ("hist_mode", ctypes.c_int), ("waves_per_cu", ctypes.c_int),
                ("suffix_form", ctypes.c_int), ("seed_mode", ctypes.c_int), ("head_form", ctypes.c_int),
                ("kernel_events", ctypes.c_void_p * 2), ("block_bounds", ctypes.c_int)]


class CayleyT(ctypes.Structure):
    _fields_ = [("n_states", ctypes.c_int), ("n_symbols", ctypes.c_int),
                ("table", ctypes.POINTER(ctypes.c_uint8)), ("maps", ctypes.POINTER(c64))]


class Walk(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("first_walker", ctypes.c_uint64), ("n_walkers", ctypes.c_uint64),
                ("burn_in", ctypes.c_uint32), ("n_steps", ctypes.c_uint32)]


class Plan(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int), ("tail_len", ctypes.c_int), ("lane_len", ctypes.c_int),
                ("prefix_len", ctypes.c_int), ("hist_mode", ctypes.c_int), ("waves_per_cu", ctypes.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build
            build.build()
        try:
            L = ctypes.CDLL(LIB_PATH)
        except OSError as e:
            raise KLError(KL_EDEVICE, f"cannot load {LIB_PATH}: {e}") from e
        vp, u64, i = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
        W = ctypes.POINTER(Window)
        O = ctypes.POINTER(Opts)
        C = ctypes.POINTER(c64)
        L.kl_num_words.argtypes = [i]
        L.kl_num_words.restype = u64
        L.kl_decode.argtypes = [u64, u64, i, vp]
        L.kl_decode_ex.argtypes = [u64, u64, i, vp, vp]
        L.kl_render.argtypes = [c64, c64, i, W, vp]
        L.kl_render_ex.argtypes = [c64, c64, i, W, vp, O]
        L.kl_render_noalloc.argtypes = [c64, c64, i, W, vp, O]
        L.kl_render_many.argtypes = [i, C, C, ctypes.POINTER(i), W, vp]
        L.kl_render_many_ex.argtypes = [i, C, C, ctypes.POINTER(i), W, vp, O]
        L.kl_eval.argtypes = [c64, c64, i, vp, u64, i, vp]
        L.kl_eval_ex.argtypes = [c64, c64, i, vp, u64, W, vp, O]
        L.kl_generators.argtypes = [c64, c64, C, C, C]
        CT = ctypes.POINTER(CayleyT)
        L.kl_cayley_num_words.argtypes = [CT, i]
        L.kl_cayley_num_words.restype = u64
        L.kl_cayley_decode_ex.argtypes = [CT, u64, u64, i, vp, vp]
        L.kl_cayley_eval_ex.argtypes = [CT, i, vp, u64, W, vp, O]
        L.kl_cayley_render_ex.argtypes = [CT, i, W, vp, O]
        for f in ("kl_cayley_decode_ex", "kl_cayley_eval_ex", "kl_cayley_render_ex"):
            getattr(L, f).restype = i
        L.kl_group_seeds.argtypes = [C, C, C]
        L.kl_maskit_generators.argtypes = [c64, C]
        L.kl_render_group_ex.argtypes = [C, i, W, vp, O]
        L.kl_eval_group_ex.argtypes = [C, i, vp, u64, W, vp, O]
        L.kl_plan.argtypes = [i, i, W, O, ctypes.POINTER(Plan)]
        WK = ctypes.POINTER(Walk)
        L.kl_walk_letters.argtypes = [WK, vp, vp]
        L.kl_walk_eval_ex.argtypes = [C, WK, W, vp, O]
        L.kl_walk_render_ex.argtypes = [C, WK, W, vp, O]
        for f in ("kl_walk_letters", "kl_walk_eval_ex", "kl_walk_render_ex"):
            getattr(L, f).restype = i
        L.kl_autotune.argtypes = [c64, c64, i, W, i, vp, ctypes.POINTER(Plan), ctypes.POINTER(ctypes.c_double)]
        L.kl_autotune_many.argtypes = [i, C, C, ctypes.POINTER(i), W, i, vp, ctypes.POINTER(Plan),
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.kl_plan_many.argtypes = [i, i, W, ctypes.POINTER(Plan)]
        L.kl_autotune_many.restype = i
        L.kl_plan_many.restype = i
        L.kl_strerror.argtypes = [i]
        L.kl_strerror.restype = ctypes.c_char_p
        L.kl_last_error.argtypes = []
        L.kl_last_error.restype = ctypes.c_char_p
        for f in ("kl_decode", "kl_decode_ex", "kl_render", "kl_render_ex", "kl_render_noalloc", "kl_render_many",
                  "kl_render_many_ex", "kl_eval", "kl_eval_ex", "kl_generators", "kl_plan", "kl_autotune",
                  "kl_group_seeds", "kl_maskit_generators", "kl_render_group_ex", "kl_eval_group_ex"):
            getattr(L, f).restype = i
        sz, i64, f32 = ctypes.c_size_t, ctypes.c_int64, ctypes.c_float
        L.kl_sur_num_params.argtypes = []
        L.kl_sur_num_params.restype = sz
        L.kl_sur_workspace_bytes.argtypes = [i]
        L.kl_sur_workspace_bytes.restype = sz
        L.kl_sur_workspace_tensor.argtypes = [i, i, ctypes.POINTER(sz), ctypes.POINTER(sz)]
        L.kl_sur_workspace_tensor.restype = i
        L.kl_sur_forward.argtypes = [vp, vp, vp, i, vp, vp, sz, vp]
        L.kl_sur_loss_grad.argtypes = [vp, vp, vp, vp, i, vp, vp, vp, sz, vp]
        L.kl_sur_adam.argtypes = [vp, vp, vp, vp, i, f32, vp]
        L.kl_sur_train_step.argtypes = [vp, vp, vp, vp, i, f32, vp, vp, vp, i, vp, vp, sz, vp]
        L.kl_occupancy.argtypes = [vp, u64, vp, vp]
        L.kl_sur_predict_occupancy.argtypes = [vp, u64, vp, vp]
        L.kl_sur_uncertainty.argtypes = [vp, i, vp, vp]
        L.kl_iou.argtypes = [vp, vp, vp, i, vp, vp]
        L.kl_gemm_bf16.argtypes = [i, i, i, vp, i64, i64, vp, i64, i64, vp, i64, vp, i, i, vp]
        for f in ("kl_sur_forward", "kl_sur_loss_grad", "kl_sur_adam", "kl_sur_train_step", "kl_occupancy",
                  "kl_sur_uncertainty", "kl_iou", "kl_gemm_bf16", "kl_sur_predict_occupancy"):
            getattr(L, f).restype = i
        _lib = L
    return _lib


def declared_symbols():
    """Names of the functions include/kl.h and include/kl_surrogate.h declare."""
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(kl_\w+)\s*\(", text))
    return sorted(names)


def _check(rc):
    if rc != KL_OK:
        msg = lib().kl_last_error().decode(errors="replace")
        raise KLError(rc, f"{lib().kl_strerror(rc).decode()}: {msg}")


_U32 = tuple(t for t in (torch.int32, getattr(torch, "uint32", None)) if t is not None)
_U64 = tuple(t for t in (torch.int64, getattr(torch, "uint64", None)) if t is not None)


def _dev_ptr(t, name, dtypes, min_numel, allow_none=False):
    """Device address of tensor t after checking what the library will
    assume of it: a torch tensor of one of `dtypes`, contiguous, with at
    least `min_numel` elements, on the current HIP device.  The library
    takes plain addresses and cannot check any of this itself."""
    if t is None:
        if allow_none:
            return None
        raise KLError(KL_EINVAL, f"{name} is None")
    if not isinstance(t, torch.Tensor):
        raise KLError(KL_EINVAL, f"{name} must be a torch.Tensor, not {type(t).__name__}")
    if t.dtype not in dtypes:
        raise KLError(KL_EINVAL, f"{name} has dtype {t.dtype}; expected {' or '.join(map(str, dtypes))}")
    if not t.is_contiguous():
        raise KLError(KL_EINVAL, f"{name} is not contiguous")
    if t.numel() < min_numel:
        raise KLError(KL_EINVAL, f"{name} holds {t.numel()} elements; the call writes or reads {min_numel}")
    if t.device.type != "cuda":
        raise KLError(KL_EINVAL, f"{name} is on {t.device}, not on a HIP device")
    if t.device.index != torch.cuda.current_device():
        raise KLError(KL_EINVAL, f"{name} is on {t.device}, not on the current device "
                                 f"cuda:{torch.cuda.current_device()}")
    return t.data_ptr()


def _c(z) -> c64:
    z = complex(z)
    return c64(z.real, z.imag)


def make_window(window) -> Window:
    if isinstance(window, Window):
        return window
    if hasattr(window, "as_tuple"):
        window = window.as_tuple()
    x0, x1, y0, y1, w, h = window
    return Window(float(x0), float(x1), float(y0), float(y1), int(w), int(h))


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(stream)


def make_opts(*, min_depth=0, precision="fp32", first=None, count=None, accumulate=False, stream=None,
              dropped=None, tail_len=0, lane_len=0, hist_mode="auto", waves_per_cu=0, suffix_form=0,
              head_form=0, seed="own", kernel_events=None, block_bounds=False, use_stream=True,
              n_dropped=1) -> Opts:
    o = Opts()
    o.dropped_out = _dev_ptr(dropped, "dropped", _U64, n_dropped, allow_none=True)
    o.min_depth = int(min_depth)
    o.precision = PREC[precision] if isinstance(precision, str) else int(precision)
    if first is not None or count is not None:
        o.use_range = 1
        o.first_idx = int(first or 0)
        o.count = int(count)
    o.accumulate = int(bool(accumulate))
    o.stream = _stream(stream).value if use_stream else None
    o.tail_len = int(tail_len)
    o.lane_len = int(lane_len)
    o.hist_mode = HIST[hist_mode] if isinstance(hist_mode, str) else int(hist_mode)
    o.waves_per_cu = int(waves_per_cu)
    o.suffix_form = int(suffix_form)
    o.head_form = int(head_form)
    o.seed_mode = SEED[seed] if isinstance(seed, str) else int(seed)
    o.block_bounds = int(bool(block_bounds))
    if kernel_events is not None:
        o.kernel_events[0] = kernel_events[0]
        o.kernel_events[1] = kernel_events[1]
    return o


def num_words(depth: int) -> int:
    return int(lib().kl_num_words(depth))


def generators(ta, tb):
    """Host-side trace recipe: (tab, gens[4, 2, 2] complex, fix[4] complex);
    a seed at infinity (a and A at ta = tb = 2, the double cusp) is inf+0j."""
    tab = c64()
    gens = (c64 * 16)()
    fix = (c64 * 4)()
    _check(lib().kl_generators(_c(ta), _c(tb), ctypes.byref(tab), gens, fix))
    g = np.array([complex(x.re, x.im) for x in gens]).reshape(4, 2, 2)
    f = np.array([complex(x.re, x.im) for x in fix])
    return complex(tab.re, tab.im), g, f


def plan(depth: int, precision="fp32", window=None, **opts) -> dict:
    p = Plan()
    o = make_opts(precision=precision, use_stream=False, **opts)
    w = None if window is None else ctypes.byref(make_window(window))
    _check(lib().kl_plan(depth, o.precision, w, ctypes.byref(o), ctypes.byref(p)))
    return {k: getattr(p, k) for k, _ in Plan._fields_}


def _device():
    if not torch.cuda.is_available():
        raise KLError(KL_EDEVICE, "no HIP device is visible")
    return torch.device("cuda", torch.cuda.current_device())


def decode(first: int, count: int, depth: int, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Letters of words first..first+count-1 of `depth`, shape (count, depth), uint8 on the GPU."""
    if out is None:
        out = torch.empty((count, depth), dtype=torch.uint8, device=_device())
    ptr = _dev_ptr(out, "out", (torch.uint8,), int(count) * max(int(depth), 0)) if count else None
    _check(lib().kl_decode_ex(int(first), int(count), int(depth), ptr, _stream(stream)))
    return out


def new_image(window, n: int | None = None) -> torch.Tensor:
    w = make_window(window)
    shape = (w.height, w.width) if n is None else (n, w.height, w.width)
    return torch.zeros(shape, dtype=torch.int32, device=_device())


def render(ta, tb, depth: int, window, image: torch.Tensor | None = None, **opts) -> torch.Tensor:
    """Density image (int32 storage holding uint32 counts), shape (height, width)."""
    w = make_window(window)
    if image is None:
        image = new_image(w)
    ptr = _dev_ptr(image, "image", _U32, w.width * w.height)
    o = make_opts(**opts)
    _check(lib().kl_render_ex(_c(ta), _c(tb), int(depth), ctypes.byref(w), ptr, ctypes.byref(o)))
    return image


def render_noalloc(ta, tb, depth: int, window, image: torch.Tensor, **opts) -> torch.Tensor:
    """kl_render_noalloc: kl_render_ex of one depth with the tables in the
    library's scratch array; the caller supplies the image."""
    w = make_window(window)
    ptr = _dev_ptr(image, "image", _U32, w.width * w.height)
    o = make_opts(**opts)
    _check(lib().kl_render_noalloc(_c(ta), _c(tb), int(depth), ctypes.byref(w), ptr, ctypes.byref(o)))
    return image


def render_many(ta, tb, depths, window, images: torch.Tensor | None = None, **opts) -> torch.Tensor:
    ta = np.asarray(ta, np.complex128).ravel()
    tb = np.asarray(tb, np.complex128).ravel()
    depths = np.asarray(depths, np.int32).ravel()
    n = len(ta)
    w = make_window(window)
    if images is None:
        images = new_image(w, n)
    cta = (c64 * n)(*[c64(z.real, z.imag) for z in ta])
    ctb = (c64 * n)(*[c64(z.real, z.imag) for z in tb])
    cd = (ctypes.c_int * n)(*[int(d) for d in depths])
    ptr = _dev_ptr(images, "images", _U32, n * w.width * w.height)
    o = make_opts(n_dropped=n, **opts)
    _check(lib().kl_render_many_ex(n, cta, ctb, cd, ctypes.byref(w), ptr, ctypes.byref(o)))
    return images


def eval_values(ta, tb, depth: int, idx, precision="fp32", window=None, **opts) -> torch.Tensor:
    """Values (or, with a window, renderer pixel coordinates) of the words idx: float64 (n, 2)."""
    if not isinstance(idx, torch.Tensor):
        idx = torch.as_tensor(np.ascontiguousarray(idx, np.uint64).view(np.int64))
    idx = idx.to(device=_device(), dtype=torch.int64).contiguous()
    n = idx.numel()
    out = torch.empty((n, 2), dtype=torch.float64, device=_device())
    o = make_opts(precision=precision, **opts)
    w = None if window is None else ctypes.byref(make_window(window))
    _check(lib().kl_eval_ex(_c(ta), _c(tb), int(depth), idx.data_ptr() if n else None, n, w,
                            out.data_ptr() if n else None, ctypes.byref(o)))
    return out


def autotune(ta, tb, depth: int, window, precision="fp32", scratch: torch.Tensor | None = None):
    w = make_window(window)
    if scratch is None:
        scratch = new_image(w)
    p = Plan()
    ms = ctypes.c_double(0.0)
    _check(lib().kl_autotune(_c(ta), _c(tb), int(depth), ctypes.byref(w), PREC[precision],
                             _dev_ptr(scratch, "scratch", _U32, w.width * w.height),
                             ctypes.byref(p), ctypes.byref(ms)))
    return {k: getattr(p, k) for k, _ in Plan._fields_}, ms.value


def autotune_many(ta, tb, depths, window, precision="fp32", scratch: torch.Tensor | None = None):
    """kl_autotune_many: (each set's plan, tuned batch ms, planner's batch ms)."""
    ta = np.asarray(ta, np.complex128).ravel()
    tb = np.asarray(tb, np.complex128).ravel()
    depths = np.asarray(depths, np.int32).ravel()
    n = len(ta)
    w = make_window(window)
    if scratch is None:
        scratch = new_image(w, n)
    cta = (c64 * n)(*[c64(z.real, z.imag) for z in ta])
    ctb = (c64 * n)(*[c64(z.real, z.imag) for z in tb])
    cd = (ctypes.c_int * n)(*[int(d) for d in depths])
    plans = (Plan * n)()
    best, default = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(lib().kl_autotune_many(n, cta, ctb, cd, ctypes.byref(w), PREC[precision],
                                  _dev_ptr(scratch, "scratch", _U32, n * w.width * w.height), plans,
                                  ctypes.byref(best), ctypes.byref(default)))
    return [{k: getattr(p, k) for k, _ in Plan._fields_} for p in plans], best.value, default.value


def plan_many(depth: int, precision="fp32", window=None) -> dict:
    """kl_plan_many: the plan a set of this depth takes in a batched render."""
    p = Plan()
    _check(lib().kl_plan_many(int(depth), PREC[precision], ctypes.byref(make_window(window)), ctypes.byref(p)))
    return {k: getattr(p, k) for k, _ in Plan._fields_}


def as_u32(image: torch.Tensor) -> np.ndarray:
    """Copy an image tensor to the host as uint32 counts."""
    return image.detach().cpu().numpy().view(np.uint32)


# ---------------------------------------------------------------- surrogate
F32, F64, U8 = (torch.float32,), (torch.float64,), (torch.uint8,)
IMG = 128 * 128


def sur_num_params() -> int:
    return int(lib().kl_sur_num_params())


def sur_workspace(batch: int) -> torch.Tensor:
    n = int(lib().kl_sur_workspace_bytes(batch))
    return torch.empty(n, dtype=torch.uint8, device=_device())


SUR_TENSORS = ["u", "h1", "h2", "x0", "y1", "y2", "y3", "logits", "dlogits", "dy3", "dy2", "dy1", "dx0", "dh2",
               "dh1"]


def sur_workspace_tensor(workspace: torch.Tensor, batch: int, name: str) -> torch.Tensor:
    """A view of one FP32 buffer of the training path in `workspace`
    (kl_sur_workspace_tensor), flat."""
    off, n = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().kl_sur_workspace_tensor(int(batch), SUR_TENSORS.index(name), ctypes.byref(off), ctypes.byref(n)))
    if off.value + 4 * n.value > workspace.numel():
        raise KLError(KL_EINVAL, "workspace too small for this batch")
    return workspace[off.value:off.value + 4 * n.value].view(torch.float32)


def as_c64(z) -> torch.Tensor:
    """Complex values as a device (n, 2) float64 tensor (kl_c64 layout)."""
    z = np.asarray(z, np.complex128).ravel()
    return torch.as_tensor(np.stack([z.real, z.imag], 1)).to(_device())


def _traces(ta, tb):
    ta_d = ta if isinstance(ta, torch.Tensor) else as_c64(ta)
    tb_d = tb if isinstance(tb, torch.Tensor) else as_c64(tb)
    B = ta_d.shape[0] if ta_d.dim() else 0
    return ta_d, tb_d, B


def _ws(workspace, B):
    ws = workspace if workspace is not None else sur_workspace(B)
    return _dev_ptr(ws, "workspace", U8, 0), ws.numel()


def sur_forward(params, ta, tb, workspace=None, out=None, stream=None):
    ta_d, tb_d, B = _traces(ta, tb)
    wp, wn = _ws(workspace, B)
    if out is None:
        out = torch.empty((B, 128, 128), dtype=torch.float32, device=_device())
    n = sur_num_params()
    _check(lib().kl_sur_forward(_dev_ptr(params, "params", F32, n), _dev_ptr(ta_d, "ta", F64, 2 * B),
                                _dev_ptr(tb_d, "tb", F64, 2 * B), B, _dev_ptr(out, "out", F32, B * IMG), wp, wn,
                                _stream(stream)))
    return out


def sur_loss_grad(params, ta, tb, targets, workspace=None, grad=None, stream=None):
    ta_d, tb_d, B = _traces(ta, tb)
    wp, wn = _ws(workspace, B)
    if grad is None:
        grad = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float32, device=_device())
    n = sur_num_params()
    _check(lib().kl_sur_loss_grad(_dev_ptr(params, "params", F32, n), _dev_ptr(ta_d, "ta", F64, 2 * B),
                                  _dev_ptr(tb_d, "tb", F64, 2 * B), _dev_ptr(targets, "targets", U8, B * IMG), B,
                                  _dev_ptr(grad, "grad", F32, n), _dev_ptr(loss, "loss", F32, 1), wp, wn,
                                  _stream(stream)))
    return loss, grad


def sur_adam(params, grad, m, v, step, lr, stream=None):
    n = sur_num_params()
    _check(lib().kl_sur_adam(_dev_ptr(params, "params", F32, n), _dev_ptr(grad, "grad", F32, n),
                             _dev_ptr(m, "m", F32, n), _dev_ptr(v, "v", F32, n), int(step), float(lr),
                             _stream(stream)))


def sur_train_step(params, m, v, grad, step, lr, ta_d, tb_d, targets, workspace, loss, stream=None):
    B = ta_d.shape[0]
    n = sur_num_params()
    _check(lib().kl_sur_train_step(_dev_ptr(params, "params", F32, n), _dev_ptr(m, "m", F32, n),
                                   _dev_ptr(v, "v", F32, n), _dev_ptr(grad, "grad", F32, n), int(step), float(lr),
                                   _dev_ptr(ta_d, "ta", F64, 2 * B), _dev_ptr(tb_d, "tb", F64, 2 * B),
                                   _dev_ptr(targets, "targets", U8, B * IMG), B, _dev_ptr(loss, "loss", F32, 1),
                                   _dev_ptr(workspace, "workspace", U8, 0), workspace.numel(), _stream(stream)))


def occupancy(counts: torch.Tensor, out=None, stream=None) -> torch.Tensor:
    if out is None:
        out = torch.empty(counts.shape, dtype=torch.uint8, device=counts.device)
    n = counts.numel()
    _check(lib().kl_occupancy(_dev_ptr(counts, "counts", _U32, n), n, _dev_ptr(out, "out", U8, n),
                              _stream(stream)))
    return out


def sur_predict_occupancy(logits: torch.Tensor, out=None, stream=None) -> torch.Tensor:
    if out is None:
        out = torch.empty(logits.shape, dtype=torch.uint8, device=logits.device)
    n = logits.numel()
    _check(lib().kl_sur_predict_occupancy(_dev_ptr(logits, "logits", F32, n), n, _dev_ptr(out, "out", U8, n),
                                          _stream(stream)))
    return out


def sur_uncertainty(logits: torch.Tensor, stream=None) -> torch.Tensor:
    B = logits.shape[0]
    out = torch.empty(B, dtype=torch.float32, device=logits.device)
    _check(lib().kl_sur_uncertainty(_dev_ptr(logits, "logits", F32, B * IMG), B, _dev_ptr(out, "out", F32, B),
                                    _stream(stream)))
    return out


def iou(target_occ: torch.Tensor, logits: torch.Tensor | None = None, pred_occ: torch.Tensor | None = None,
        stream=None) -> torch.Tensor:
    B = target_occ.shape[0]
    out = torch.empty(B, dtype=torch.float32, device=target_occ.device)
    _check(lib().kl_iou(_dev_ptr(logits, "logits", F32, B * IMG, allow_none=True),
                        _dev_ptr(pred_occ, "pred_occ", U8, B * IMG, allow_none=True),
                        _dev_ptr(target_occ, "target_occ", U8, B * IMG), B, _dev_ptr(out, "out", F32, B),
                        _stream(stream)))
    return out


def _span(rows, cols, s_row, s_col):
    """Elements a strided rows x cols operand reaches (0 when empty)."""
    if rows <= 0 or cols <= 0:
        return 0
    return (rows - 1) * int(s_row) + (cols - 1) * int(s_col) + 1


def gemm_bf16(M, N, K, A, lda_m, lda_k, B, ldb_k, ldb_n, C, ldc, bias=None, relu=False, accumulate=False,
              stream=None):
    _check(lib().kl_gemm_bf16(M, N, K, _dev_ptr(A, "A", F32, _span(M, K, lda_m, lda_k)), lda_m, lda_k,
                              _dev_ptr(B, "B", F32, _span(K, N, ldb_k, ldb_n)), ldb_k, ldb_n,
                              _dev_ptr(C, "C", F32, _span(M, N, ldc, 1)), ldc,
                              _dev_ptr(bias, "bias", F32, N, allow_none=True), int(relu), int(accumulate),
                              _stream(stream)))
    return C


# ---------------------------------------------------------------- explicit groups
def _ab(ab):
    """Two generators (a, b) as 2x2 complex arrays -> the 8-entry c64 array the library takes."""
    ab = np.asarray(ab, np.complex128).reshape(8)
    return (c64 * 8)(*[c64(z.real, z.imag) for z in ab])


def maskit_generators(mu) -> np.ndarray:
    """Maskit's a, b for parameter mu: (2, 2, 2) complex."""
    out = (c64 * 8)()
    _check(lib().kl_maskit_generators(_c(mu), out))
    return np.array([complex(z.re, z.im) for z in out]).reshape(2, 2, 2)


def group_seeds(ab):
    """(gens[4, 2, 2], seeds[4, 2]) of a group given by a, b: the normalised maps and
    each generator's attracting fixed point as a homogeneous pair (u, v)."""
    g = (c64 * 16)()
    sd = (c64 * 8)()
    _check(lib().kl_group_seeds(_ab(ab), g, sd))
    return (np.array([complex(z.re, z.im) for z in g]).reshape(4, 2, 2),
            np.array([complex(z.re, z.im) for z in sd]).reshape(4, 2))


def render_group(ab, depth: int, window, image: torch.Tensor | None = None, **opts) -> torch.Tensor:
    """kl_render_ex for a group given by its generators a, b."""
    w = make_window(window)
    if image is None:
        image = new_image(w)
    ptr = _dev_ptr(image, "image", _U32, w.width * w.height)
    o = make_opts(**opts)
    _check(lib().kl_render_group_ex(_ab(ab), int(depth), ctypes.byref(w), ptr, ctypes.byref(o)))
    return image


def eval_group(ab, depth: int, idx, precision="fp32", window=None, **opts) -> torch.Tensor:
    """kl_eval_ex for a group given by its generators a, b."""
    if not isinstance(idx, torch.Tensor):
        idx = torch.as_tensor(np.ascontiguousarray(idx, np.uint64).view(np.int64))
    idx = idx.to(device=_device(), dtype=torch.int64).contiguous()
    n = idx.numel()
    out = torch.empty((n, 2), dtype=torch.float64, device=_device())
    o = make_opts(precision=precision, **opts)
    w = None if window is None else ctypes.byref(make_window(window))
    _check(lib().kl_eval_group_ex(_ab(ab), int(depth), idx.data_ptr() if n else None, n, w,
                                  out.data_ptr() if n else None, ctypes.byref(o)))
    return out


# ---------------------------------------------------------------- indexed Cayley tables
class Cayley:
    """An indexed Cayley table (uint8 [n_states, n_symbols + 1], column 0
    unused) and, for values and renders, one 2x2 complex map per symbol."""

    def __init__(self, table, maps=None):
        self._table = np.ascontiguousarray(table, np.uint8)
        n_states, cols = self._table.shape
        self._maps = None
        mp = None
        if maps is not None:
            mv = np.asarray(maps, np.complex128).reshape(-1)
            self._maps = (c64 * len(mv))(*[c64(z.real, z.imag) for z in mv])
            mp = ctypes.cast(self._maps, ctypes.POINTER(c64))
        self.struct = CayleyT(n_states, cols - 1, self._table.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), mp)

    def ref(self):
        return ctypes.byref(self.struct)


def cayley_num_words(t: Cayley, depth: int) -> int:
    return int(lib().kl_cayley_num_words(t.ref(), depth))


def cayley_decode(t: Cayley, first: int, count: int, depth: int, stream=None) -> torch.Tensor:
    out = torch.empty((count, depth), dtype=torch.uint8, device=_device())
    _check(lib().kl_cayley_decode_ex(t.ref(), first, count, depth, out.data_ptr() if count else None,
                                     _stream(stream)))
    return out


def cayley_eval(t: Cayley, depth: int, idx, window=None, **opts) -> torch.Tensor:
    if not isinstance(idx, torch.Tensor):
        idx = torch.as_tensor(np.ascontiguousarray(idx, np.uint64).view(np.int64))
    idx = idx.to(device=_device(), dtype=torch.int64).contiguous()
    n = idx.numel()
    out = torch.empty((n, 2), dtype=torch.float64, device=_device())
    o = make_opts(**opts)
    w = None if window is None else ctypes.byref(make_window(window))
    _check(lib().kl_cayley_eval_ex(t.ref(), int(depth), idx.data_ptr() if n else None, n, w,
                                   out.data_ptr() if n else None, ctypes.byref(o)))
    return out


def cayley_render(t: Cayley, depth: int, window, image: torch.Tensor | None = None, **opts) -> torch.Tensor:
    w = make_window(window)
    if image is None:
        image = new_image(w)
    ptr = _dev_ptr(image, "image", _U32, w.width * w.height)
    o = make_opts(**opts)
    _check(lib().kl_cayley_render_ex(t.ref(), int(depth), ctypes.byref(w), ptr, ctypes.byref(o)))
    return image


# ---------------------------------------------------------------- random walks (Section 4)
def make_walk(seed: int, first_walker: int, n_walkers: int, burn_in: int, n_steps: int) -> Walk:
    return Walk(int(seed), int(first_walker), int(n_walkers), int(burn_in), int(n_steps))


def walk_letters(seed: int, first_walker: int, n_walkers: int, burn_in: int, n_steps: int,
                 stream=None) -> torch.Tensor:
    """Letters c_0 .. c_{burn_in + n_steps} of each walker: (n_walkers, 1 + burn_in + n_steps) uint8."""
    wk = make_walk(seed, first_walker, n_walkers, burn_in, n_steps)
    out = torch.empty((n_walkers, 1 + burn_in + n_steps), dtype=torch.uint8, device=_device())
    ptr = _dev_ptr(out, "letters_out", (torch.uint8,), out.numel()) if n_walkers else None
    _check(lib().kl_walk_letters(ctypes.byref(wk), ptr, _stream(stream)))
    return out


def walk_eval(ab, seed: int, first_walker: int, n_walkers: int, burn_in: int, n_steps: int, window=None,
              **opts) -> torch.Tensor:
    """Drawn points (or pixel coordinates with a window): (n_walkers, n_steps, 2) float64."""
    wk = make_walk(seed, first_walker, n_walkers, burn_in, n_steps)
    out = torch.empty((n_walkers, n_steps, 2), dtype=torch.float64, device=_device())
    ptr = _dev_ptr(out, "z_out", (torch.float64,), out.numel()) if out.numel() else None
    o = make_opts(**opts)
    w = None if window is None else ctypes.byref(make_window(window))
    _check(lib().kl_walk_eval_ex(_ab(ab), ctypes.byref(wk), w, ptr, ctypes.byref(o)))
    return out


def walk_render(ab, seed: int, first_walker: int, n_walkers: int, burn_in: int, n_steps: int, window,
                image: torch.Tensor | None = None, **opts) -> torch.Tensor:
    """The walkers' drawn points binned: (height, width) int32 storage of uint32 counts."""
    wk = make_walk(seed, first_walker, n_walkers, burn_in, n_steps)
    w = make_window(window)
    if image is None:
        image = new_image(w)
    ptr = _dev_ptr(image, "image", _U32, w.width * w.height)
    o = make_opts(**opts)
    _check(lib().kl_walk_render_ex(_ab(ab), ctypes.byref(wk), ctypes.byref(w), ptr, ctypes.byref(o)))
    return image
