"""Pins of the oracle's indexed Cayley tables (Section 5).

The general table path is fixed by: the paper's own tables and scan
(Section 6: every m^d digit string, kept when its right-to-left table walk
never crashes), closed-form counts, the free group's table reproducing the
specialised reduced-word order and renders, and the integer structure of the
modular group's orbit of i.
"""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1709_08018_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_table(name):
    rows = [line.split() for line in open(os.path.join(GOLDEN, name)) if line.strip() and not line.startswith("#")]
    return np.array(rows, dtype=np.uint8)


T11 = _read_table("cayley_t11_indexed.txt")
KLEIN4 = _read_table("cayley_klein4_indexed.txt")
# PSL(2, Z) = <a, b | a^2 = b^3 = 1>, normal forms alternating a with b or B
# (b^-1 = b^2): symbols 1 = a, 2 = b, 3 = B; the state is the symbol read last.
MODULAR = np.array([[0, 1, 2, 3],
                    [1, 0, 2, 3],
                    [2, 1, 0, 0],
                    [3, 1, 0, 0]], np.uint8)
MOD_MAPS = np.array([[[0, -1], [1, 0]], [[0, -1], [1, 1]], [[1, 1], [-1, 0]]], complex)
# a language that is not closed under reversal: "1" may not stand immediately
# left of "2" (reading right to left, symbol 1 crashes in state 2)
ONEWAY = np.array([[0, 1, 2],
                   [0, 1, 2],
                   [0, 0, 2]], np.uint8)


def _id_maps(m):
    return np.array([[[1, 0], [0, 1]]] * m, complex)


def _cayley(table, maps=None):
    m = table.shape[1] - 1
    return O.Cayley(table, _id_maps(m) if maps is None else maps)


def test_free_group_table_reproduces_reduced_words():
    R = O.group_recipe(wl.C2_TA, wl.C2_TB)
    c = O.Cayley(T11, R.gens)
    for d in range(1, 8):
        assert O.cayley_num_words(c, d) == 4 * 3 ** (d - 1)
        words = np.array([O.cayley_unrank(c, i, d) for i in range(O.num_words(d))])
        np.testing.assert_array_equal(words - 1, O.enumerate_words(d))
    for d in (20, 40):
        for i in wl.sample_indices(O.num_words(d), 50, seed=d):
            np.testing.assert_array_equal(O.cayley_unrank(c, int(i), d) - 1, O.unrank(int(i), d))


@pytest.mark.parametrize("name,table,dmax", [("t11", T11, 6), ("klein4", KLEIN4, 7), ("modular", MODULAR, 9),
                                             ("oneway", ONEWAY, 10)])
def test_unrank_equals_the_paper_scan(name, table, dmax):
    c = _cayley(table)
    for d in range(1, dmax + 1):
        scan = O.cayley_scan(c, d)
        assert len(scan) == O.cayley_num_words(c, d)
        got = np.array([O.cayley_unrank(c, i, d) for i in range(len(scan))]).reshape(len(scan), d)
        np.testing.assert_array_equal(got, scan)


def test_closed_form_counts():
    k4, mod = _cayley(KLEIN4), _cayley(MODULAR)
    for d in range(1, 30):
        # Klein four: of the three symbols read in a non-identity state exactly one gives the identity
        assert O.cayley_num_words(k4, d) == 3 * 2 ** (d - 1)
        # PSL(2,Z): alternating words; a rightmost a leaves ceil((d-1)/2) free choices of b or B,
        # a rightmost b or B leaves floor((d-1)/2)
        assert O.cayley_num_words(mod, d) == 2 ** ((d) // 2) + 2 * 2 ** ((d - 1) // 2)


def test_counts_past_64_bits_are_refused():
    """16 states, 7 symbols and no crash: symbol x in state s leads to state
    1 + (x - 1 + 7 (s mod 2)) mod 15, so every string is regular and there
    are exactly 7^L words of length L, and a state's count is at most the
    previous length's total.  7^22 fits 64 bits.  7^23 does not, though each
    state's count (at most 7^22) stays below 2^63; it is refused (0) rather
    than wrapped."""
    S, m = 16, 7
    t = np.zeros((S, m + 1), np.uint8)
    t[:, 0] = np.arange(S)
    for st in range(S):
        for x in range(1, m + 1):
            t[st, x] = 1 + ((x - 1) + 7 * (st & 1)) % 15
    c = O.Cayley(t, np.array([[[2, 0], [0, 0.5]]] * m, complex))
    for d in (1, 2, 10, 22):
        assert O.cayley_num_words(c, d) == 7 ** d
    assert 7 ** 23 >= 2 ** 64 and 7 ** 22 < 2 ** 63
    assert O.cayley_num_words(c, 23) == 0


def test_free_group_table_values_and_render_equal_the_recipe_path():
    R = O.group_recipe(wl.C2_TA, wl.C2_TB)
    c = O.Cayley(T11, R.gens)
    d = 9
    idx = wl.sample_indices(O.num_words(d), 2000, seed=1)
    # the table path scales each map to determinant 1 by 1/sqrt(det), det = 1 up to rounding
    for seed in (-1, 0, 1, 2, 3):
        zc = O.cayley_eval(c, d, idx, seed=seed)
        zr = O.eval_group(R, d, idx, seed=seed)
        assert (np.abs(zc - zr) / np.maximum(1, np.abs(zr))).max() < 1e-12
    win = (-1.5, 1.5, -1.5, 1.5, 128, 128)
    img_c, drop_c, _ = O.cayley_render(c, 9, win, min_depth=3)
    img_r, drop_r, near = O.render_group(R, 9, win, min_depth=3, edge_tol=1e-9)
    assert int(np.abs(img_c.astype(np.int64) - img_r).sum()) <= 2 * near and abs(drop_c - drop_r) <= near


def test_modular_orbit_of_i_has_integer_structure():
    """g(i) = (ac + bd + i)/(c^2 + d^2) for g = [[a, b], [c, d]] in SL(2, Z):
    1/Im z and Re z / Im z are integers for every word value from seed i."""
    c = O.Cayley(MODULAR, MOD_MAPS)
    d = 16
    idx = np.arange(O.cayley_num_words(c, d), dtype=np.uint64)
    z = O.cayley_eval(c, d, idx, seed=0)       # symbol 1 = a fixes i
    q = 1 / z.imag
    assert np.abs(q - np.round(q)).max() < 1e-6 * q.max()
    p = z.real * q
    assert np.abs(p - np.round(p)).max() < 1e-6 * np.abs(p).max()
    zl = O.cayley_eval(c, d, idx, seed=0, literal=True)
    assert np.abs(zl - z).max() < 1e-9


def test_cayley_render_invariants():
    c = O.Cayley(MODULAR, MOD_MAPS)
    win = (-2.0, 2.0, 0.0, 1.2, 200, 60)
    total = sum(O.cayley_num_words(c, d) for d in range(1, 13))
    img, drop, _ = O.cayley_render(c, 12, win, seed=3, min_depth=1)   # each symbol's fixed point in turn
    assert int(img.sum()) + drop == 3 * total
