"""Pins of the oracle's uniform grid (Section 3.1): keys, order, box starts,
and the 3x3x3 search against brute-force neighbour sets."""
import numpy as np
import pytest

from oracle import brute
from paper_2301_06984_amd import workloads


def _cases():
    yield "c1-small-f64", workloads.c1(n=1500, seed=21).pos, workloads.c1(n=1500, seed=21).diam
    w = workloads.c2(n=2000, seed=22)
    yield "c2-small-f32", w.pos, w.diam
    p, d = workloads.uniform_cube(800, 60.0, seed=23, dtype=np.float32)   # dense: many contacts
    yield "dense-f32", p, d
    p, d = workloads.uniform_cube(600, 400.0, seed=24)                    # sparse
    yield "sparse-f64", p - 200.0, d                                      # negative coordinates


CASES = list(_cases())


@pytest.mark.parametrize("name,pos,diam", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("cell_factor", [1.0, 1.7])
def test_keys_order_starts(orc, name, pos, diam, cell_factor):
    R = float(diam.astype(np.float64).max())
    inv_h = 1.0 / (R * cell_factor)
    g = orc.grid(pos, inv_h)
    key_bf, cmin, dims = brute.keys(pos, inv_h)
    np.testing.assert_array_equal(g["cmin"], cmin)
    np.testing.assert_array_equal(g["dims"], dims)
    np.testing.assert_array_equal(g["key"].astype(np.int64), key_bf)
    n = pos.shape[0]
    perm = np.lexsort((np.arange(n), key_bf))
    np.testing.assert_array_equal(g["perm"], perm.astype(np.uint32))
    counts = np.bincount(key_bf, minlength=int(np.prod(dims)))
    cs = np.concatenate([[0], np.cumsum(counts)]).astype(np.uint32)
    np.testing.assert_array_equal(g["cell_start"], cs)


@pytest.mark.parametrize("name,pos,diam", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("cell_factor", [1.0, 1.3])
def test_neighbor_sets_brute_force(orc, name, pos, diam, cell_factor):
    R = float(diam.astype(np.float64).max())
    start, nbr = orc.neighbors(pos, R, 1.0 / (R * cell_factor))
    sets = brute.neighbor_sets(pos, R)
    total = 0
    for i, s in enumerate(sets):
        np.testing.assert_array_equal(nbr[start[i]:start[i + 1]], s)
        total += s.size
    assert total > 0


def test_radius_larger_than_cell_is_rejected_by_construction(orc):
    # the oracle always uses a box edge >= R (cell_factor < 1 is clamped to 1)
    p = orc.Params(cell_factor=0.5)
    pos, diam = workloads.uniform_cube(200, 50.0, seed=3)
    assert orc.inv_cell(diam, p) == 1.0 / float(diam.max())


def test_single_agent_and_coincident(orc):
    pos = np.array([[1.0, 2.0, 3.0]])
    g = orc.grid(pos, 0.1)
    assert g["nboxes"] == 1 and g["key"].tolist() == [0] and g["cell_start"].tolist() == [0, 1]
    # two agents at the same centre: neighbours (distance 0 < R) but no contact term
    pos = np.array([[5.0, 5.0, 5.0], [5.0, 5.0, 5.0]])
    diam = np.array([10.0, 10.0])
    s = orc.State.initial(pos, diam)
    orc.step(s, orc.Params())
    assert s.nnz.tolist() == [0, 0]
    np.testing.assert_array_equal(s.force, 0.0)
    np.testing.assert_array_equal(s.pos, pos)
