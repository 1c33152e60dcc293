"""Pins of the oracle's gap-free Morton ranks (Section 4.2, steps D and E)."""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "morton_gaps_3x3.json")


def table_from_codes(codes):
    """(box counter, offset) entries where the offset of rank r is code(r) - r;
    an entry starts wherever the offset changes (and at rank 0)."""
    codes = np.asarray(codes, dtype=np.int64)
    off = codes - np.arange(codes.size)
    starts = [0] + [r for r in range(1, codes.size) if off[r] != off[r - 1]]
    return [(r, int(off[r])) for r in starts]


def test_paper_example_3x3(orc):
    g = json.load(open(GOLDEN))
    gaps = set()
    for a, b in g["gaps_between"]:
        gaps.update(range(a + 1, b))
    printed_codes = [c for c in range(g["max_code"] + 1) if c not in gaps]
    assert printed_codes == [0, 1, 2, 3, 4, 6, 8, 9, 12]
    # 2D Morton codes of the 3x3 boxes (brute force) agree with the printed ones
    assert list(brute.all_box_codes(g["dims"], D=2)) == printed_codes
    # step D table
    bc, off = orc.gap_table(g["dims"], D=2)
    assert list(zip(bc.tolist(), off.tolist())) == table_from_codes(printed_codes)
    assert list(zip(bc.tolist(), off.tolist())) == [(0, 0), (5, 1), (6, 2), (8, 4)]
    # step E: code of rank r = r + offset
    _, codes = orc.ranks(g["dims"], np.zeros((0, 2), np.int64), D=2, rank_list=np.arange(9))
    assert codes.tolist() == printed_codes


def _check_dims(orc, dims, D):
    axes = [np.arange(d) for d in dims]
    q = np.stack([m.ravel() for m in np.meshgrid(*axes, indexing="ij")], axis=1)
    r_table, _ = orc.ranks(dims, q, D=D)
    r_sort = brute.ranks_by_sorting(dims, q, D=D)
    np.testing.assert_array_equal(r_table, r_sort)
    nb = int(np.prod(dims))
    assert sorted(r_table.tolist()) == list(range(nb))      # a bijection onto 0..#boxes-1
    codes_sorted = brute.all_box_codes(dims, D=D)
    _, codes = orc.ranks(dims, np.zeros((0, D), np.int64), D=D, rank_list=np.arange(nb))
    np.testing.assert_array_equal(codes, codes_sorted)
    bc, off = orc.gap_table(dims, D=D)
    assert list(zip(bc.tolist(), off.tolist())) == table_from_codes(codes_sorted)


@pytest.mark.parametrize("D", [2, 3])
def test_ranks_all_small_dims(orc, D):
    rng = range(1, 13) if D == 3 else range(1, 41)
    for dims in itertools.product(rng, repeat=D):
        if D == 3 and sum(dims) % 3:     # a third of the 3D combinations keeps this fast
            continue
        _check_dims(orc, list(dims), D)


def test_ranks_random_dims_to_40(orc):
    g = np.random.default_rng(11)
    for _ in range(40):
        dims = g.integers(1, 41, size=3).tolist()
        _check_dims(orc, dims, 3)


def test_power_of_two_has_no_gaps(orc):
    for L in range(0, 6):
        bc, off = orc.gap_table([2 ** L] * 3, D=3)
        assert bc.tolist() == [0] and off.tolist() == [0]


def test_morton_bit_order(orc):
    # x occupies the lowest bit, then y, then z
    assert orc.morton([1, 0, 0], 1) == 1
    assert orc.morton([0, 1, 0], 1) == 2
    assert orc.morton([0, 0, 1], 1) == 4
    assert orc.morton([2, 0, 0], 2) == 8
    assert orc.morton([3, 3, 3], 2) == 63
