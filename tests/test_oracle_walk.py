"""Pins of the oracle's random-walk renderer (the probabilistic approach of
Section 4, row f4) against what fixes it independently of its own code:

* Philox4x64-10 against numpy's implementation of the same published
  generator (numpy.random.Philox, whose first output block is that of its
  counter plus one), across carries between counter words.
* The letter law: every walk is a reduced word; each decision reaches all
  three allowed letters; first letters and steps are uniform within
  statistical bounds.
* Every drawn point is the value of the reduced word c_n ... c_1 c_0 with
  its own seed (Section 1), as the oracle's product evaluator computes it
  from the word's index -- a different computation from the walk's
  literal point-by-point maps -- for recipe groups and for Maskit's group
  (whose b fixes infinity).
* Real traces: every point of long walks lies on the unit circle.
"""
import numpy as np
import pytest

from oracle import oracle as O

INV = np.array([2, 3, 0, 1])
C1 = (complex(3, 0), complex(3, 0))
C2 = (complex(1.91, 0.05), complex(2.0, 0.0))
MU = complex(-0.097, 1.838)


def _numpy_block(key, counter):
    """Philox4x64-10 of `counter` under `key` from numpy (which encrypts its counter plus one)."""
    k = int(key[0]) | (int(key[1]) << 64)
    c = sum(int(x) << (64 * i) for i, x in enumerate(counter))
    c = (c - 1) % (1 << 256)
    return np.random.Philox(key=k, counter=c).random_raw(4).astype(np.uint64)


@pytest.mark.parametrize("key,counter", [
    ((0, 0), (0, 0, 0, 0)), ((0, 0), (1, 0, 0, 0)), ((1, 0), (0, 0, 0, 0)),
    ((0xDEADBEEF, 0x1234), (7, 3, 0, 0)), ((2 ** 64 - 1, 2 ** 64 - 1), (2 ** 64 - 1, 5, 9, 2 ** 63)),
    ((42, 0), (0, 2 ** 64 - 1, 0, 0)), ((42, 0), (12345, 678, 2 ** 40, 1)),
])
def test_philox_matches_numpy(key, counter):
    got = O.philox4x64_10(np.array(counter, np.uint64), np.array(key, np.uint64))
    np.testing.assert_array_equal(got, _numpy_block(key, counter))


def test_philox_consecutive_blocks_match_numpy_stream():
    key = (987654321, 0)
    ref = np.random.Philox(key=key[0], counter=0).random_raw(4 * 50).astype(np.uint64)
    got = np.concatenate([O.philox4x64_10(np.array([j, 0, 0, 0], np.uint64), np.array(key, np.uint64))
                          for j in range(1, 51)])
    np.testing.assert_array_equal(got, ref)


def _letters(seed, walker, n):
    return O.walk_letters(seed, walker, n).astype(int)


def test_walks_are_reduced_words():
    for w in [0, 1, 17, 2 ** 40, 2 ** 64 - 1]:
        c = _letters(3, w, 5000)
        assert set(np.unique(c)) <= {0, 1, 2, 3}
        assert not np.any(c[1:] == INV[c[:-1]]), w


def test_first_letter_is_the_top_bits_of_the_first_value():
    # value 0 of walker w: low half of the first output of the block at counter (0, w, 0, 0)
    for seed, w in [(0, 0), (5, 9), (2 ** 63, 2 ** 50)]:
        r = _numpy_block((seed, 0), (0, w, 0, 0))
        assert _letters(seed, w, 1)[0] == (int(r[0]) & 0xFFFFFFFF) >> 30


def test_letter_law_is_uniform():
    # first letters over many walkers, and steps given the previous letter
    firsts = np.array([_letters(11, w, 1)[0] for w in range(20000)])
    counts = np.bincount(firsts, minlength=4)
    assert np.all(np.abs(counts - 5000) < 5 * np.sqrt(5000 * 0.75)), counts
    steps = np.zeros((4, 4), int)
    for w in range(40):
        c = _letters(11, w, 10000)
        np.add.at(steps, (c[:-1], c[1:]), 1)
    for p in range(4):
        row = steps[p]
        assert row[INV[p]] == 0
        allowed = np.delete(row, INV[p])
        n = allowed.sum()
        assert np.all(np.abs(allowed - n / 3) < 5 * np.sqrt(n * 2 / 9)), (p, row)


def _rank(word):
    """Index of a reduced word (leftmost letter first) in lexicographic order."""
    d = len(word)
    idx = int(word[0])
    for j in range(1, d):
        t = int(word[j]) - (1 if word[j] > INV[word[j - 1]] else 0)
        idx = idx * 3 + t
    return idx


def test_rank_inverts_unrank():
    rng = np.random.default_rng(4)
    for d in (1, 2, 5, 13, 30):
        for i in rng.integers(0, O.num_words(d), size=20, dtype=np.uint64):
            assert _rank(O.unrank(int(i), d)) == int(i)


@pytest.mark.parametrize("burn_in", [0, 3])
def test_points_are_word_values_recipe(burn_in):
    seed, steps = 7, 38 - burn_in
    g = O.group_recipe(*C2)
    for w in [0, 1, 999, 2 ** 33 + 5]:
        c = _letters(seed, w, 1 + burn_in + steps)
        z = O.walk_points(g, seed, w, 1, burn_in, steps)[0]
        for s in range(steps):
            n = burn_in + 1 + s
            word = c[:n + 1][::-1]                 # c_n ... c_1 c_0, leftmost first
            zr = O.eval_values(*C2, n + 1, np.array([_rank(word)], np.uint64))[0]
            assert abs(z[s] - zr) <= 1e-12 * max(1.0, abs(zr)), (w, s)


def test_points_are_word_values_maskit_with_seeds_at_infinity():
    seed, steps = 9, 39
    g = O.group_maskit(MU)
    seen_inf = 0
    for w in range(64):
        c = _letters(seed, w, 1 + steps)
        z = O.walk_points(g, seed, w, 1, 0, steps)[0]
        for s in range(steps):
            word = c[:s + 2][::-1]
            zr = O.eval_group(g, s + 2, np.array([_rank(word)], np.uint64))[0]
            if not np.isfinite(zr):
                assert not np.isfinite(z[s])
                seen_inf += 1
                continue
            assert abs(z[s] - zr) <= 1e-11 * max(1.0, abs(zr)), (w, s)
    assert seen_inf > 0   # walks from b's fixed point at infinity that stay there


def test_real_traces_keep_every_point_on_the_unit_circle():
    g = O.group_recipe(*C1)
    z = O.walk_points(g, 1, 100, 8, 0, 20000)
    assert np.abs(np.abs(z) - 1).max() < 1e-9


def test_burn_in_drops_the_first_points():
    g = O.group_recipe(*C2)
    a = O.walk_points(g, 2, 5, 3, 0, 50)
    b = O.walk_points(g, 2, 5, 3, 10, 40)
    np.testing.assert_array_equal(a[:, 10:], b)


def test_render_counts_every_point():
    g = O.group_maskit(MU)
    win = (-1.05, 1.05, -0.1, 2.0, 256, 256)
    img, drop, _ = O.walk_render(g, 0, 0, 300, 5, 200, win)
    assert int(img.sum()) + drop == 300 * 200
    z = O.walk_points(g, 0, 0, 300, 5, 200).ravel()
    x0, x1, y0, y1, W, H = win
    with np.errstate(invalid="ignore"):
        fx, fy = (z.real - x0) * W / (x1 - x0), (z.imag - y0) * H / (y1 - y0)
        ok = np.isfinite(z) & (fx >= 0) & (fx < W) & (fy >= 0) & (fy < H)
    ref = np.zeros(W * H, np.int64)
    np.add.at(ref, np.floor(fy[ok]).astype(int) * W + np.floor(fx[ok]).astype(int), 1)
    np.testing.assert_array_equal(img.ravel().astype(np.int64), ref)


def test_letters_from_numpy_raw_values():
    """The stream layout: decision k of walker w reads block k // 8 (counter
    (k // 8, w, 0, 0), key (seed, 0)), half k % 2 of output (k % 8) // 2."""
    seed, w, n = 77, 123456789, 40
    vals = []
    for j in range((n + 7) // 8):
        r = _numpy_block((seed, 0), (j, w, 0, 0))
        for x in r:
            vals += [int(x) & 0xFFFFFFFF, int(x) >> 32]
    c = [vals[0] >> 30]
    for k in range(1, n):
        t = (vals[k] * 3) >> 32
        allowed = [x for x in range(4) if x != INV[c[-1]]]
        c.append(allowed[t])
    np.testing.assert_array_equal(_letters(seed, w, n), c)
