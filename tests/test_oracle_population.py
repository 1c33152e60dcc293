"""Pins of the dynamic population (Section 3.2): removal by hole filling
from the tail, addition by appending, and condition (iii) of the static test
(Section 5) for added agents."""
import json
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "removal_swap.json")


def labelled(orc, n):
    """A state whose rows carry their original index in every field."""
    idx = np.arange(n, dtype=np.float64)
    st = orc.State.initial(np.stack([idx, 2 * idx, 3 * idx], axis=1), idx + 1.0)
    st.moved = (np.arange(n) % 2).astype(np.uint8)
    st.nnz = np.arange(n, dtype=np.int32)
    st.force = np.stack([idx, -idx, idx * idx], axis=1)
    return st


def old_index(st):
    return st.pos[:, 0].astype(np.int64)


def test_removal_golden(orc):
    for case in json.load(open(GOLDEN))["cases"]:
        st = orc.remove_agents(labelled(orc, case["n"]), case["remove"])
        np.testing.assert_array_equal(old_index(st), case["order"], err_msg=str(case))


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_removal_properties(orc, seed):
    g = np.random.default_rng(seed)
    n = int(g.integers(1, 400))
    m = int(g.integers(0, n + 1))
    rm = g.choice(n, m, replace=False)
    st0 = labelled(orc, n)
    st = orc.remove_agents(st0, rm)
    src = old_index(st)
    new_size = n - m
    assert src.size == new_size
    # exactly the agents that stay, each once, with all of its fields
    np.testing.assert_array_equal(np.sort(src), np.setdiff1d(np.arange(n), rm))
    for f in ("pos", "diam", "moved", "nnz", "force"):
        np.testing.assert_array_equal(getattr(st, f), getattr(st0, f)[src])
    # an agent left of the new size that stays keeps its index; the others
    # (at most m of them) come from right of it, in ascending order
    keep_left = np.setdiff1d(np.arange(new_size), rm)
    np.testing.assert_array_equal(src[keep_left], keep_left)
    moved_in = src[src >= new_size]
    assert moved_in.size <= m
    assert np.all(np.diff(moved_in) > 0)
    assert np.all(np.diff(np.nonzero(src >= new_size)[0]) > 0)


def test_removal_rejects_bad_ids(orc):
    st = labelled(orc, 5)
    for bad in ([5], [-1], [1, 1]):
        with pytest.raises(ValueError):
            orc.remove_agents(st, bad)


def test_addition_appends_moved_agents(orc):
    st = orc.add_agents(labelled(orc, 4), [[10.0, 0.0, 0.0], [20.0, 0.0, 0.0]], [9.0, 11.0])
    assert st.pos.shape == (6, 3)
    np.testing.assert_array_equal(st.moved[4:], [1, 1])
    np.testing.assert_array_equal(st.nnz[4:], [0, 0])
    np.testing.assert_array_equal(st.force[4:], 0.0)
    np.testing.assert_array_equal(st.diam[4:], [9.0, 11.0])


def test_added_neighbour_unsets_static(orc):
    # two touching spheres relax apart, then rest at distance 10.5 > 10 (no
    # contact): static from the step after they stop.  A new sphere placed
    # in contact with one of them makes it non-static (condition (iii)) and
    # pushes it; the other one, out of reach (more than R away), stays static.
    pos = np.array([[0.0, 0.0, 0.0], [10.5, 0.0, 0.0]])
    diam = np.array([10.0, 10.0])
    p = orc.Params(detect_static=True, interaction_radius=12.0)
    st = orc.State.initial(pos, diam)
    for _ in range(3):
        stat, _ = orc.step(st, p, want_static=True)
    np.testing.assert_array_equal(stat, [1, 1])
    st = orc.add_agents(st, [[-9.0, 0.0, 0.0]], [10.0])
    x0 = st.pos.copy()
    stat, _ = orc.step(st, p, want_static=True)
    np.testing.assert_array_equal(stat, [0, 1, 0])
    assert st.pos[0, 0] > x0[0, 0] and st.pos[2, 0] < x0[2, 0]     # pushed apart
    np.testing.assert_array_equal(st.pos[1], x0[1])
