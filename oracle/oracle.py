"""ctypes wrapper of the CPU reference library ``liboracle.so``.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg are the only users of this module.  It imports
nothing from the GPU package and the GPU package imports nothing from it.

Every function here is argument marshalling around ``kl_oracle.c``; the
arithmetic lives there (FP64, plain definitions; see its header comment for
the passages of the paper each part follows).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
# A test that plants mistakes in a copy of the reference points this at the
# planted build; nothing else sets it.
_OVERRIDE = os.environ.get("KL_ORACLE_LIB")
SOURCES = [os.path.join(HERE, "kl_oracle.c")]


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(LIB_PATH):
        cmd = ["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-Wall",
               "-Wno-unused-function", "-o", LIB_PATH + ".tmp"] + SOURCES + ["-lm", "-lpthread"]
        subprocess.run(cmd, check=True)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _OVERRIDE:
            L = ctypes.CDLL(_OVERRIDE)
        else:
            if not os.path.exists(LIB_PATH):
                build(force=False)
            L = ctypes.CDLL(LIB_PATH)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        dp = ctypes.POINTER(ctypes.c_double)
        d = ctypes.c_double
        L.oracle_num_words.argtypes = [ctypes.c_int]
        L.oracle_num_words.restype = ctypes.c_uint64
        L.oracle_num_tree_nodes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.oracle_num_tree_nodes.restype = ctypes.c_uint64
        L.oracle_unrank.argtypes = [ctypes.c_uint64, ctypes.c_int, u8p]
        L.oracle_enumerate.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, u8p]
        L.oracle_generators.argtypes = [d, d, d, d, dp, dp, dp]
        L.oracle_word_value.argtypes = [u8p, ctypes.c_int, dp, dp, ctypes.c_int, dp]
        L.oracle_eval.argtypes = [d, d, d, d, ctypes.c_int, u64p, ctypes.c_uint64,
                                  ctypes.c_int, dp]
        L.oracle_render.argtypes = [d, d, d, d, ctypes.c_int, ctypes.c_int,
                                    d, d, d, d, ctypes.c_uint32, ctypes.c_uint32,
                                    ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, d,
                                    u32p, u64p, u64p]
        L.oracle_group_recipe.argtypes = [d, d, d, d, dp, dp]
        L.oracle_group_explicit.argtypes = [dp, dp, dp]
        L.oracle_group_maskit.argtypes = [d, d, dp, dp]
        L.oracle_eval_group.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, u64p, ctypes.c_uint64,
                                        ctypes.c_int, dp]
        L.oracle_render_group.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          d, d, d, d, ctypes.c_uint32, ctypes.c_uint32,
                                          ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, d,
                                          u32p, u64p, u64p]
        L.oracle_cayley_num_words.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.oracle_cayley_num_words.restype = ctypes.c_uint64
        L.oracle_cayley_unrank.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_int, u8p]
        L.oracle_cayley_scan.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, u8p, ctypes.c_uint64, u64p]
        L.oracle_cayley_eval.argtypes = [u8p, ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, ctypes.c_int, u64p,
                                         ctypes.c_uint64, ctypes.c_int, dp]
        L.oracle_cayley_render.argtypes = [u8p, ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int, d, d, d, d, ctypes.c_uint32, ctypes.c_uint32, d,
                                           u32p, u64p, u64p]
        for f in (L.oracle_cayley_unrank, L.oracle_cayley_scan, L.oracle_cayley_eval, L.oracle_cayley_render):
            f.restype = ctypes.c_int
        u64 = ctypes.c_uint64
        L.oracle_philox4x64_10.argtypes = [u64p, u64p, u64p]
        L.oracle_walk_letters.argtypes = [u64, u64, ctypes.c_uint32, u8p]
        L.oracle_walk_points.argtypes = [dp, dp, u64, u64, u64, ctypes.c_uint32, ctypes.c_uint32, dp]
        L.oracle_walk_render.argtypes = [dp, dp, u64, u64, u64, ctypes.c_uint32, ctypes.c_uint32,
                                         d, d, d, d, ctypes.c_uint32, ctypes.c_uint32, d, u32p, u64p, u64p]
        for f in (L.oracle_philox4x64_10, L.oracle_walk_letters, L.oracle_walk_points, L.oracle_walk_render):
            f.restype = ctypes.c_int
        for f in (L.oracle_unrank, L.oracle_enumerate, L.oracle_generators,
                  L.oracle_word_value, L.oracle_eval, L.oracle_render, L.oracle_group_recipe,
                  L.oracle_group_explicit, L.oracle_group_maskit, L.oracle_eval_group,
                  L.oracle_render_group):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


class OracleError(RuntimeError):
    pass


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what} failed with code {rc}")


def num_words(depth: int) -> int:
    return int(lib().oracle_num_words(depth))


def num_tree_nodes(m: int, depth: int, tiling: bool) -> int:
    return int(lib().oracle_num_tree_nodes(m, depth, int(tiling)))


def unrank(index: int, depth: int) -> np.ndarray:
    w = np.zeros(depth, np.uint8)
    _check(lib().oracle_unrank(index, depth, _ptr(w, ctypes.c_uint8)), "unrank")
    return w


def enumerate_words(depth: int, first: int = 0, count: int | None = None) -> np.ndarray:
    n = num_words(depth)
    if count is None:
        count = n - first
    out = np.zeros((count, depth), np.uint8)
    _check(lib().oracle_enumerate(depth, first, count, _ptr(out, ctypes.c_uint8)),
           "enumerate")
    return out


def generators(ta: complex, tb: complex):
    """Returns (tab, gens[4,2,2] complex, fix[4] complex)."""
    tab = np.zeros(2)
    gens = np.zeros(32)
    fix = np.zeros(8)
    _check(lib().oracle_generators(ta.real, ta.imag, tb.real, tb.imag,
                                   _ptr(tab, ctypes.c_double), _ptr(gens, ctypes.c_double),
                                   _ptr(fix, ctypes.c_double)), "generators")
    return (complex(tab[0], tab[1]), gens.view(np.complex128).reshape(4, 2, 2),
            fix.view(np.complex128).copy())


def word_value(word, gens, fix, literal: bool = False) -> complex:
    w = np.ascontiguousarray(word, np.uint8)
    g = np.ascontiguousarray(np.asarray(gens, np.complex128).reshape(-1)).view(np.float64)
    f = np.ascontiguousarray(np.asarray(fix, np.complex128)).view(np.float64)
    z = np.zeros(2)
    _check(lib().oracle_word_value(_ptr(w, ctypes.c_uint8), len(w), _ptr(g, ctypes.c_double),
                                   _ptr(f, ctypes.c_double), int(literal),
                                   _ptr(z, ctypes.c_double)), "word_value")
    return complex(z[0], z[1])


def eval_values(ta: complex, tb: complex, depth: int, idx, literal: bool = False) -> np.ndarray:
    idx = np.ascontiguousarray(idx, np.uint64)
    z = np.zeros(2 * len(idx))
    _check(lib().oracle_eval(ta.real, ta.imag, tb.real, tb.imag, depth,
                             _ptr(idx, ctypes.c_uint64), len(idx), int(literal),
                             _ptr(z, ctypes.c_double)), "eval")
    return z.view(np.complex128)


def render(ta: complex, tb: complex, depth: int, window, *, min_depth: int | None = None,
           first: int = 0, count: int | None = None, nthreads: int = 1,
           edge_tol: float = 0.0, image: np.ndarray | None = None):
    """Render into a uint32 image.  window = (x0, x1, y0, y1, width, height).

    Returns (image[height, width], dropped, near_edge)."""
    x0, x1, y0, y1, W, H = window
    if min_depth is None:
        min_depth = depth
    total = sum(num_words(d) for d in range(min_depth, depth + 1))
    if count is None:
        count = total - first
    if image is None:
        image = np.zeros((H, W), np.uint32)
    dropped = ctypes.c_uint64(0)
    near = ctypes.c_uint64(0)
    _check(lib().oracle_render(ta.real, ta.imag, tb.real, tb.imag, depth, min_depth,
                               x0, x1, y0, y1, W, H, first, count, nthreads, edge_tol,
                               _ptr(image, ctypes.c_uint32), ctypes.byref(dropped),
                               ctypes.byref(near)), "render")
    return image, int(dropped.value), int(near.value)


class Group:
    """A group as the *_group functions take it: gens[4, 2, 2] complex
    (a, b, A, B) and seeds[4, 2] complex (homogeneous fixed points u : v)."""

    def __init__(self, gens: np.ndarray, seeds: np.ndarray):
        self.gens = np.ascontiguousarray(gens, np.complex128).reshape(4, 2, 2)
        self.seeds = np.ascontiguousarray(seeds, np.complex128).reshape(4, 2)

    def _arrays(self):
        return (np.ascontiguousarray(self.gens.reshape(-1)).view(np.float64),
                np.ascontiguousarray(self.seeds.reshape(-1)).view(np.float64))

    def seed_points(self) -> np.ndarray:
        """Each generator's seed as a point (inf where v = 0)."""
        u, v = self.seeds[:, 0], self.seeds[:, 1]
        with np.errstate(divide="ignore", invalid="ignore"):
            return np.where(v == 0, np.inf, u / np.where(v == 0, 1, v))


def _group_from(fn, *args) -> Group:
    gens = np.zeros(32)
    seeds = np.zeros(16)
    _check(fn(*args, _ptr(gens, ctypes.c_double), _ptr(seeds, ctypes.c_double)), "group")
    return Group(gens.view(np.complex128), seeds.view(np.complex128))


def group_recipe(ta: complex, tb: complex) -> Group:
    return _group_from(lib().oracle_group_recipe, ta.real, ta.imag, tb.real, tb.imag)


def group_explicit(a, b) -> Group:
    ab = np.ascontiguousarray(np.concatenate([np.asarray(a, np.complex128).reshape(-1),
                                              np.asarray(b, np.complex128).reshape(-1)])).view(np.float64)
    return _group_from(lib().oracle_group_explicit, _ptr(ab, ctypes.c_double))


def group_maskit(mu: complex) -> Group:
    return _group_from(lib().oracle_group_maskit, mu.real, mu.imag)


def eval_group(group: Group, depth: int, idx, seed: int = -1, literal: bool = False) -> np.ndarray:
    g, s = group._arrays()
    idx = np.ascontiguousarray(idx, np.uint64)
    z = np.zeros(2 * len(idx))
    _check(lib().oracle_eval_group(_ptr(g, ctypes.c_double), _ptr(s, ctypes.c_double), seed, depth,
                                   _ptr(idx, ctypes.c_uint64), len(idx), int(literal),
                                   _ptr(z, ctypes.c_double)), "eval_group")
    return z.view(np.complex128)


def render_group(group: Group, depth: int, window, *, seed: int = -1, min_depth: int | None = None,
                 first: int = 0, count: int | None = None, nthreads: int = 1, edge_tol: float = 0.0,
                 image: np.ndarray | None = None):
    """As render(), for an explicit group and seed mode (-1 own, 0..3 one
    generator's fixed point, 4 each in turn).  Returns (image, dropped, near_edge)."""
    g, s = group._arrays()
    x0, x1, y0, y1, W, H = window
    if min_depth is None:
        min_depth = depth
    total = sum(num_words(d) for d in range(min_depth, depth + 1))
    if count is None:
        count = total - first
    if image is None:
        image = np.zeros((H, W), np.uint32)
    dropped = ctypes.c_uint64(0)
    near = ctypes.c_uint64(0)
    _check(lib().oracle_render_group(_ptr(g, ctypes.c_double), _ptr(s, ctypes.c_double), seed, depth,
                                     min_depth, x0, x1, y0, y1, W, H, first, count, nthreads, edge_tol,
                                     _ptr(image, ctypes.c_uint32), ctypes.byref(dropped),
                                     ctypes.byref(near)), "render_group")
    return image, int(dropped.value), int(near.value)


class Cayley:
    """An indexed Cayley table: table[n_states, n_symbols + 1] of next states
    (column 0 unused), and one 2x2 complex map per symbol."""

    def __init__(self, table, maps):
        self.table = np.ascontiguousarray(table, np.uint8)
        self.n_states, cols = self.table.shape
        self.n_symbols = cols - 1
        self.maps = np.ascontiguousarray(np.asarray(maps, np.complex128).reshape(self.n_symbols, 2, 2))

    def _args(self):
        return _ptr(self.table, ctypes.c_uint8), self.n_states, self.n_symbols

    def _maps(self):
        return np.ascontiguousarray(self.maps.reshape(-1)).view(np.float64)


def cayley_num_words(c: Cayley, depth: int) -> int:
    return int(lib().oracle_cayley_num_words(*c._args(), depth))


def cayley_unrank(c: Cayley, index: int, depth: int) -> np.ndarray:
    w = np.zeros(depth, np.uint8)
    _check(lib().oracle_cayley_unrank(*c._args(), index, depth, _ptr(w, ctypes.c_uint8)), "cayley_unrank")
    return w


def cayley_scan(c: Cayley, depth: int) -> np.ndarray:
    """The paper's scan of all m^d digit strings: the survivors, in order."""
    n = ctypes.c_uint64(0)
    _check(lib().oracle_cayley_scan(*c._args(), depth, None, 0, ctypes.byref(n)), "cayley_scan")
    out = np.zeros((n.value, depth), np.uint8)
    _check(lib().oracle_cayley_scan(*c._args(), depth, _ptr(out, ctypes.c_uint8), n.value, ctypes.byref(n)),
           "cayley_scan")
    return out


def cayley_eval(c: Cayley, depth: int, idx, seed: int = -1, literal: bool = False) -> np.ndarray:
    m = c._maps()
    idx = np.ascontiguousarray(idx, np.uint64)
    z = np.zeros(2 * len(idx))
    _check(lib().oracle_cayley_eval(*c._args(), _ptr(m, ctypes.c_double), seed, depth,
                                    _ptr(idx, ctypes.c_uint64), len(idx), int(literal),
                                    _ptr(z, ctypes.c_double)), "cayley_eval")
    return z.view(np.complex128)


def cayley_render(c: Cayley, depth: int, window, *, seed: int = -1, min_depth: int | None = None,
                  edge_tol: float = 0.0):
    """Returns (image[H, W], dropped, near_edge)."""
    m = c._maps()
    x0, x1, y0, y1, W, H = window
    image = np.zeros((H, W), np.uint32)
    dropped = ctypes.c_uint64(0)
    near = ctypes.c_uint64(0)
    _check(lib().oracle_cayley_render(*c._args(), _ptr(m, ctypes.c_double), seed, depth,
                                      depth if min_depth is None else min_depth, x0, x1, y0, y1, W, H, edge_tol,
                                      _ptr(image, ctypes.c_uint32), ctypes.byref(dropped),
                                      ctypes.byref(near)), "cayley_render")
    return image, int(dropped.value), int(near.value)


# ---------------------------------------------------------------- random walks (Section 4)
def philox4x64_10(counter, key) -> np.ndarray:
    """Philox4x64-10 of a counter (4 uint64) under a key (2 uint64): 4 uint64."""
    c = np.ascontiguousarray(counter, np.uint64)
    k = np.ascontiguousarray(key, np.uint64)
    out = np.zeros(4, np.uint64)
    _check(lib().oracle_philox4x64_10(_ptr(c, ctypes.c_uint64), _ptr(k, ctypes.c_uint64),
                                      _ptr(out, ctypes.c_uint64)), "philox")
    return out


def walk_letters(seed: int, walker: int, n: int) -> np.ndarray:
    """Letters c_0 .. c_{n-1} of one walker (c_0 first, i.e. rightmost)."""
    out = np.zeros(max(n, 1), np.uint8)
    _check(lib().oracle_walk_letters(seed, walker, n, _ptr(out, ctypes.c_uint8)), "walk_letters")
    return out[:n]


def walk_points(group: Group, seed: int, first_walker: int, n_walkers: int, burn_in: int,
                n_steps: int) -> np.ndarray:
    """Drawn points of the walkers, (n_walkers, n_steps) complex (inf at infinity)."""
    g, s = group._arrays()
    z = np.zeros(2 * max(n_walkers * n_steps, 1))
    _check(lib().oracle_walk_points(_ptr(g, ctypes.c_double), _ptr(s, ctypes.c_double), seed, first_walker,
                                    n_walkers, burn_in, n_steps, _ptr(z, ctypes.c_double)), "walk_points")
    return z.view(np.complex128)[:n_walkers * n_steps].reshape(n_walkers, n_steps)


def walk_render(group: Group, seed: int, first_walker: int, n_walkers: int, burn_in: int, n_steps: int,
                window, *, edge_tol: float = 0.0, image: np.ndarray | None = None):
    """The walkers' points binned; returns (image, dropped, near_edge)."""
    g, s = group._arrays()
    x0, x1, y0, y1, W, H = window
    if image is None:
        image = np.zeros((H, W), np.uint32)
    dropped = ctypes.c_uint64(0)
    near = ctypes.c_uint64(0)
    _check(lib().oracle_walk_render(_ptr(g, ctypes.c_double), _ptr(s, ctypes.c_double), seed, first_walker,
                                    n_walkers, burn_in, n_steps, x0, x1, y0, y1, W, H, edge_tol,
                                    _ptr(image, ctypes.c_uint32), ctypes.byref(dropped), ctypes.byref(near)),
           "walk_render")
    return image, int(dropped.value), int(near.value)
