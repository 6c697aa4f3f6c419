"""Workload definitions and seeded parameter draws.

This module holds only the parameters of the workloads (traces, depths,
windows) and the seeded random draws of parameter sets.  It contains none
of the method's arithmetic, so both the GPU path and the CPU reference can
be fed from it.

Workloads (traces are those of the trace recipe; windows are
(x0, x1, y0, y1, width, height)):
  fuchsian_tiling_d10   ta = tb = 3 (real, Fuchsian), tiling mode over
                        depths 1..10, 512 x 512 over [-2, 2]^2
  quasifuchsian_d18     ta = 1.91 + 0.05i, tb = 2, limit set at depth 18,
                        2048 x 2048 over [-1.5, 1.5]^2
  quasifuchsian_d22     same traces, depth 22, 4096 x 4096 over
                        [-1.5, 1.5]^2, streamed by index range
  batch256              256 parameter sets: Re ta, Re tb ~ U[1.8, 3.0],
                        Im ta, Im tb ~ U[-0.3, 0.3], depth ~ U{12..18},
                        512 x 512 over [-2, 2]^2 each
  surrogate             parameter sets drawn as batch256 at depth 14,
                        128 x 128 occupancy over [-2, 2]^2
  maskit_tiling_d14     Maskit's group at mu = -0.097 + 1.838i (the
                        parameter of the paper's figures), tiling mode over
                        depths 1..14, every generator's fixed point fed to
                        every word (the paper's index-search loop);
                        1024 x 1024 over one period of the translation b,
                        [-1.05, 1.05] x [-0.1, 2.0]
  walk_maskit_fig3      random walks (the probabilistic approach) in
                        Maskit's group at the same mu: 2^14 walkers of 64
                        drawn points (2^20 points, Fig. 3), the same window
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

C2_TA = complex(1.91, 0.05)
C2_TB = complex(2.0, 0.0)
C1_TA = complex(3.0, 0.0)
C1_TB = complex(3.0, 0.0)


@dataclass(frozen=True)
class Window:
    x0: float
    x1: float
    y0: float
    y1: float
    width: int
    height: int

    def as_tuple(self):
        return (self.x0, self.x1, self.y0, self.y1, self.width, self.height)

    @property
    def pixel(self) -> float:
        return (self.x1 - self.x0) / self.width


@dataclass(frozen=True)
class Workload:
    name: str
    ta: complex
    tb: complex
    depth: int
    min_depth: int
    window: Window


FUCHSIAN_TILING_D10 = Workload("fuchsian_tiling_d10", C1_TA, C1_TB, 10, 1,
                               Window(-2.0, 2.0, -2.0, 2.0, 512, 512))
QUASIFUCHSIAN_D18 = Workload("quasifuchsian_d18", C2_TA, C2_TB, 18, 18,
                             Window(-1.5, 1.5, -1.5, 1.5, 2048, 2048))
QUASIFUCHSIAN_D22 = Workload("quasifuchsian_d22", C2_TA, C2_TB, 22, 22,
                             Window(-1.5, 1.5, -1.5, 1.5, 4096, 4096))
BATCH_WINDOW = Window(-2.0, 2.0, -2.0, 2.0, 512, 512)
SURROGATE_WINDOW = Window(-2.0, 2.0, -2.0, 2.0, 128, 128)
SURROGATE_DEPTH = 14
MASKIT_MU = complex(-0.097, 1.838)
# ta holds Maskit's parameter mu for this workload; tb is unused
MASKIT_D14 = Workload("maskit_tiling_d14", MASKIT_MU, complex(0.0, 0.0), 14, 1,
                      Window(-1.05, 1.05, -0.1, 2.0, 1024, 1024))


@dataclass(frozen=True)
class WalkWorkload:
    """Random walks (the probabilistic approach): walkers x drawn points each."""
    name: str
    mu: complex          # Maskit's parameter
    seed: int
    n_walkers: int
    burn_in: int
    n_steps: int
    window: Window

    @property
    def points(self) -> int:
        return self.n_walkers * self.n_steps


# The configuration of the paper's probabilistic rendering (Fig. 3): Maskit's
# group at mu = -0.097 + 1.838i, 1,048,576 points (2^14 walkers of 64 drawn
# points each), the window of maskit_tiling_d14
WALK_FIG3 = WalkWorkload("walk_maskit_fig3", MASKIT_MU, 0, 1 << 14, 0, 64, MASKIT_D14.window)
# as many points as the depth-13 limit set has words (4 * 3^12 = 3^11 walkers x 12)
WALK_D13_POINTS = WalkWorkload("walk_maskit_d13_points", MASKIT_MU, 1, 3 ** 11, 0, 12, MASKIT_D14.window)
# 2^30 points
WALK_LARGE = WalkWorkload("walk_maskit_2p30", MASKIT_MU, 2, 1 << 24, 0, 64, MASKIT_D14.window)


def draw_maskit_mu(n: int, seed: int, depth_range=(8, 16)):
    """n Maskit parameters mu with depths, from numpy's PCG64 with the given
    seed: Re mu ~ U[-1, 1], Im mu ~ U[2.0, 2.6] (inside the Maskit slice);
    depth ~ uniform integer in depth_range (inclusive)."""
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-1.0, 1.0, size=n) + 1j * rng.uniform(2.0, 2.6, size=n)
    lo, hi = depth_range
    depth = rng.integers(lo, hi + 1, size=n)
    return mu.astype(np.complex128), depth.astype(np.int32)


def draw_decode_ranges(n: int, seed: int, max_count: int = 5000):
    """n index ranges (depth, first, count) from numpy's PCG64 with the given
    seed: depth ~ uniform integer in 1..40, count ~ uniform in 1..max_count
    (at most the depth's words), first ~ uniform over the indices that leave
    room for count words."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        d = int(rng.integers(1, 41))
        total = 4 * 3 ** (d - 1)
        count = int(rng.integers(1, min(max_count, total) + 1))
        first = int(rng.integers(0, total - count + 1, dtype=np.uint64))
        out.append((d, first, count))
    return out


def draw_walks(n: int, seed: int):
    """n walk configurations (walk seed, first walker, walkers, burn-in, drawn
    steps) from numpy's PCG64 with the given seed: the walk seed and first
    walker uniform over 64 bits (the walker range kept below 2^64), 1..3000
    walkers, burn-in 0..20, 1..120 drawn steps."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        walk_seed = int(rng.integers(0, 2 ** 64, dtype=np.uint64))
        walkers = int(rng.integers(1, 3001))
        first = int(rng.integers(0, 2 ** 64 - walkers, dtype=np.uint64))
        out.append((walk_seed, first, walkers, int(rng.integers(0, 21)), int(rng.integers(1, 121))))
    return out


def draw_param_sets(n: int, seed: int, depth_range=(12, 18)):
    """n parameter sets (ta, tb, depth) from numpy's PCG64 with the given seed.

    Re ta, Re tb ~ U[1.8, 3.0]; Im ta, Im tb ~ U[-0.3, 0.3];
    depth ~ uniform integer in depth_range (inclusive)."""
    rng = np.random.default_rng(seed)
    re = rng.uniform(1.8, 3.0, size=(n, 2))
    im = rng.uniform(-0.3, 0.3, size=(n, 2))
    lo, hi = depth_range
    depth = rng.integers(lo, hi + 1, size=n)
    ta = re[:, 0] + 1j * im[:, 0]
    tb = re[:, 1] + 1j * im[:, 1]
    return ta.astype(np.complex128), tb.astype(np.complex128), depth.astype(np.int32)


def batch256(seed: int = 0):
    return draw_param_sets(256, seed, (12, 18))


def surrogate_sets(n: int, seed: int):
    ta, tb, _ = draw_param_sets(n, seed, (SURROGATE_DEPTH, SURROGATE_DEPTH))
    return ta, tb


def sample_indices(n_words: int, n: int, seed: int = 0) -> np.ndarray:
    """n word indices drawn uniformly from [0, n_words) with PCG64(seed)."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.integers(0, n_words, size=n, dtype=np.uint64))
