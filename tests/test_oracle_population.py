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


# ---- diameter changes (growth, shrinking): condition (ii) of Section 5
def _rest_then(orc, pos, diam, p, nsteps=3):
    st = orc.State.initial(np.array(pos, np.float64), np.array(diam, np.float64))
    for _ in range(nsteps):
        stat, _ = orc.step(st, p, want_static=True)
    return st, stat


def _skip_on_off(orc, st, p):
    """One step with the static skip and one without, from copies of st."""
    on, off = st.copy(), st.copy()
    stat, _ = orc.step(on, p, want_static=True)
    orc.step(off, orc.Params(**{**p.__dict__, "detect_static": False}))
    return on, off, stat


def _unmarked(orc, st, ids, diam):
    """A planted mistake: the diameters change but nobody counts as moved."""
    bad = st.copy()
    bad.diam[np.asarray(ids)] = diam
    return bad


@pytest.mark.parametrize("case", ["growth", "shrink"])
def test_diameter_change_unsets_static(orc, case):
    # growth: spheres 0 and 1 rest 10.5 apart with no contact; growing 1 to
    # 11.2 makes an overlap of 0.1, where the pair term is attractive
    # (k*0.1 - gamma*sqrt(rho*0.1) < 0).  shrink: they rest in contact at
    # overlap 0.72, where the repulsion (about 0.098) stays below the threshold
    # 0.2; shrinking 1 to 8.88 leaves an overlap of 0.16, near the deepest
    # attraction (about -0.29), which exceeds the threshold.  Sphere 2 is
    # out of reach (farther than R from both) and stays static.
    if case == "growth":
        pos, f_adh, new = [[0.0, 0, 0], [10.5, 0, 0], [40.0, 0, 0]], 0.0, 11.2
    else:
        pos, f_adh, new = [[0.0, 0, 0], [9.28, 0, 0], [40.0, 0, 0]], 0.2, 8.88
    p = orc.Params(detect_static=True, interaction_radius=12.0, f_adh=f_adh)
    st, stat = _rest_then(orc, pos, [10.0, 10.0, 10.0], p)
    np.testing.assert_array_equal(stat, [1, 1, 1])
    x0 = st.pos.copy()
    ch = orc.set_diameters(st, [1], [new], radius=12.0)
    np.testing.assert_array_equal(ch.moved, [0, 1, 0])
    assert ch.diam[1] == new and st.diam[1] == 10.0          # the input state is left as it was
    on, off, stat = _skip_on_off(orc, ch, p)
    np.testing.assert_array_equal(stat, [0, 0, 1])
    np.testing.assert_array_equal(on.pos, off.pos)
    np.testing.assert_array_equal(on.nnz, off.nnz)
    assert on.pos[0, 0] > x0[0, 0] and on.pos[1, 0] < x0[1, 0]   # drawn together
    np.testing.assert_array_equal(on.pos[2], x0[2])
    # without the mark the skip keeps both at rest: the mark is what makes the skip exact
    bad_on, bad_off, _ = _skip_on_off(orc, _unmarked(orc, st, [1], [new]), p)
    np.testing.assert_array_equal(bad_on.pos, x0)
    assert not np.array_equal(bad_on.pos, bad_off.pos)


def test_diameter_unchanged_value_is_no_move(orc):
    st = labelled(orc, 6)
    ch = orc.set_diameters(st, [0, 2, 5], [1.0, 7.5, 6.0])   # agents 0 and 5 keep theirs
    np.testing.assert_array_equal(ch.moved, np.where(np.arange(6) == 2, 1, st.moved))
    np.testing.assert_array_equal(ch.diam, [1.0, 2.0, 7.5, 4.0, 5.0, 6.0])
    for f in ("pos", "nnz", "force"):
        np.testing.assert_array_equal(getattr(ch, f), getattr(st, f))


def test_diameter_change_rejects_bad_input(orc):
    st = labelled(orc, 5)
    for ids, d in (([5], [1.0]), ([-1], [1.0]), ([1, 1], [1.0, 2.0]), ([0], [0.0]), ([0], [np.nan]),
                   ([0], [-2.0]), ([0, 1], [1.0])):
        with pytest.raises(ValueError):
            orc.set_diameters(st, ids, d)
    with pytest.raises(ValueError):
        orc.set_diameters(st, [0], [12.5], radius=12.0)
    orc.set_diameters(st, [0], [12.0], radius=12.0)   # at R is allowed
