"""Pins of the Hilbert-order variant (Section 4.2 compares the Morton order
with the Hilbert curve): the curve itself from its defining properties, the
ranks of the boxes from their definition, and a step in that order against
the Morton step."""
import itertools

import numpy as np
import pytest


def cube(b):
    s = 1 << b
    return np.array(list(itertools.product(range(s), repeat=3)), np.int64)[:, ::-1].copy()   # x fastest


@pytest.mark.parametrize("b", [1, 2, 3, 4])
def test_curve_is_a_hilbert_curve(orc, b):
    # a bijection onto [0, 8^b) that starts at the origin and moves by one
    # box along one axis at every step (a continuous curve through the
    # lattice), and that visits every aligned 2^k block in one piece
    q = cube(b)
    h = orc.hilbert(q, b).astype(np.int64)
    assert np.array_equal(np.sort(h), np.arange(8 ** b))
    path = q[np.argsort(h)]
    assert np.array_equal(path[0], [0, 0, 0])
    steps = np.abs(np.diff(path, axis=0))
    assert np.all(steps.sum(axis=1) == 1)
    for k in range(1, b):
        blk = path >> k
        change = np.any(blk[1:] != blk[:-1], axis=1)
        assert change.sum() == 8 ** (b - k) - 1     # each block entered once


@pytest.mark.parametrize("b", [2, 3, 4, 5])
def test_curve_refines_the_coarser_curve(orc, b):
    # the top 3(b-1) bits of the index of a point are the index of its parent
    # block on the curve of one level less: the curve nests
    g = np.random.default_rng(b)
    q = g.integers(0, 1 << b, size=(500, 3))
    fine = orc.hilbert(q, b)
    coarse = orc.hilbert(q >> 1, b - 1)
    np.testing.assert_array_equal(fine >> np.uint64(3), coarse)


def test_curve_differs_from_morton(orc):
    q = cube(2)
    h = orc.hilbert(q, 2)
    m = np.array([orc.morton(x, 2) for x in q], np.uint64)
    assert not np.array_equal(h, m)


@pytest.mark.parametrize("dims", [(1, 1, 1), (2, 2, 2), (3, 2, 1), (5, 7, 3), (8, 8, 8), (9, 4, 13), (17, 3, 6)])
def test_hilbert_box_ranks_from_the_definition(orc, dims):
    # one agent in every box; the canonical order of the grid must be the
    # super-boxes (2x2x2 blocks) by Hilbert index over the smallest
    # power-of-two cube holding them, each one's boxes in Morton order (x
    # lowest), and the ranks gap-free
    dims = np.array(dims)
    q = np.array(list(itertools.product(*[range(d) for d in dims[::-1]])), np.int64)[:, ::-1].copy()
    pos = (q + 0.5) * 10.0
    g = orc.grid(pos, 0.1, order=1)
    np.testing.assert_array_equal(g["dims"], dims)
    key = g["key"].astype(np.int64)
    assert np.array_equal(np.sort(key), np.arange(len(q)))
    sd = (dims + 1) // 2
    L = int(np.ceil(np.log2(max(sd.max(), 1)))) if sd.max() > 1 else 0
    hs = orc.hilbert(q >> 1, L).astype(np.int64)
    octant = (q[:, 0] & 1) | ((q[:, 1] & 1) << 1) | ((q[:, 2] & 1) << 2)
    want = np.lexsort((octant, hs))
    np.testing.assert_array_equal(np.argsort(key), want)
    np.testing.assert_array_equal(g["perm"], want)
    np.testing.assert_array_equal(np.diff(g["cell_start"].astype(np.int64)), np.ones(len(q), np.int64))


def test_morton_and_hilbert_steps_agree(orc):
    # the order changes only the summation order of the pair terms: the same
    # neighbour sets and non-zero counts, positions within a few ulps, and
    # the static skip exact in both orders
    from paper_2301_06984_amd import workloads
    w = workloads.c1(n=3000, seed=31)
    res = {}
    for order in (0, 1):
        for skip in (False, True):
            p = orc.Params(order=order, detect_static=skip)
            st = orc.State.initial(w.pos, w.diam)
            for _ in range(6):
                orc.step(st, p)
            res[order, skip] = st
    for order in (0, 1):
        np.testing.assert_array_equal(res[order, True].pos, res[order, False].pos)
    a, b = res[0, False], res[1, False]
    np.testing.assert_array_equal(a.nnz, b.nnz)
    np.testing.assert_array_equal(a.moved, b.moved)
    scale = np.maximum(np.abs(a.pos).max(axis=1), float(w.diam.max()))
    assert np.all(np.abs(a.pos - b.pos).max(axis=1) <= 1e-12 * scale)
    assert not np.array_equal(a.pos, b.pos)   # the order did change the sums somewhere
