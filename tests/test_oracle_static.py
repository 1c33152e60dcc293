"""Pins of the static-agent skip (Section 5): skipping never changes the
trajectory, and constructed cases for each of the conditions."""
import numpy as np
import pytest

from paper_2301_06984_amd import workloads


def run_both(orc, pos, diam, steps, **kw):
    on = orc.State.initial(pos, diam)
    off = orc.State.initial(pos, diam)
    p_on = orc.Params(detect_static=True, **kw)
    p_off = orc.Params(detect_static=False, **kw)
    stat, nnz_off = [], []
    for _ in range(steps):
        s, _ = orc.step(on, p_on, want_static=True)
        orc.step(off, p_off)
        np.testing.assert_array_equal(on.pos, off.pos)
        np.testing.assert_array_equal(on.moved, off.moved)
        stat.append(s)
        nnz_off.append(off.nnz.copy())
    return on, off, np.array(stat), np.array(nnz_off)


def test_skip_equals_no_skip_c2_construction(orc):
    w = workloads.c2(n=6000, seed=41)
    on, off, stat, _ = run_both(orc, w.pos, w.diam, 12)
    frac = stat[1:].mean(axis=1)
    assert stat[0].sum() == 0                 # nothing is static at the first step
    assert frac.min() > 0.3                   # the force-free shell is skipped


def test_skip_equals_no_skip_with_threshold_and_departures(orc):
    g = np.random.default_rng(42)
    n = 1500
    pos = g.uniform(0, 95, size=(n, 3))
    diam = g.uniform(2.0, 12.0, size=n)
    on, off, stat, nnz_off = run_both(orc, pos, diam, 15, f_adh=0.6, mu=1.5, delta_max=9.0)
    # departures: static agents that kept one contact while the no-skip run saw it leave
    departures = 0
    nnz_on = None
    s_on = orc.State.initial(pos, diam)
    p_on = orc.Params(detect_static=True, f_adh=0.6, mu=1.5, delta_max=9.0)
    for t in range(15):
        st, _ = orc.step(s_on, p_on, want_static=True)
        nnz_on = s_on.nnz
        departures += int(np.sum(st.astype(bool) & (nnz_on == 1) & (nnz_off[t] == 0)))
    assert stat[1:].sum() > 100
    assert departures > 0


def test_lattice_all_static_from_step_one(orc):
    pos, diam = workloads.lattice(7, 12.5, diam=12.0)
    st = orc.State.initial(pos, diam)
    p = orc.Params(detect_static=True)
    s0, _ = orc.step(st, p, want_static=True)
    assert s0.sum() == 0
    for _ in range(3):
        s, _ = orc.step(st, p, want_static=True)
        assert s.all()
    np.testing.assert_array_equal(st.pos, pos)


def test_two_cancelling_contacts_never_static(orc):
    # centre agent with two symmetric contacts: F = 0 exactly but two non-zero terms
    pos = np.array([[0.0, 0.0, 0.0], [9.5, 0.0, 0.0], [-9.5, 0.0, 0.0]])
    diam = np.array([10.0, 10.0, 10.0])
    probe = orc.State.initial(pos, diam)
    orc.step(probe, orc.Params(mu=0.0))
    np.testing.assert_array_equal(probe.force[0], 0.0)
    fout = abs(float(probe.force[1, 0]))
    p = orc.Params(detect_static=True, f_adh=2 * fout)      # outer agents stay below the threshold
    st = orc.State.initial(pos, diam)
    for t in range(4):
        s, _ = orc.step(st, p, want_static=True)
        assert st.nnz.tolist() == [2, 1, 1]
        assert s[0] == 0                                    # condition (iv) blocks the centre
        if t > 0:
            assert s[1] == 1 and s[2] == 1
    np.testing.assert_array_equal(st.pos, pos)


def test_neighbour_move_unsets_static(orc):
    # a static agent whose neighbour (within R, not in contact) moves is recomputed
    pos = np.array([[0.0, 0.0, 0.0], [11.0, 0.0, 0.0], [16.0, 0.0, 0.0]])
    diam = np.array([8.0, 12.0, 12.0])       # 0-1 within R = 12 but S = 10; 1-2 in contact
    st = orc.State.initial(pos, diam)
    p = orc.Params(detect_static=True)
    orc.step(st, p)
    s, _ = orc.step(st, p, want_static=True)
    assert st.moved[1] == 1                  # agent 1 keeps moving
    assert s[0] == 0                         # so agent 0 is not static
    far = orc.State.initial(np.array([[0.0, 0, 0], [30.0, 0, 0], [35.0, 0, 0]]), diam)
    orc.step(far, p)
    s, _ = orc.step(far, p, want_static=True)
    assert s[0] == 1


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_skip_off_reports_no_static(orc, dtype):
    pos, diam = workloads.lattice(4, 13.0, dtype=dtype)
    st = orc.State.initial(pos, diam)
    for _ in range(3):
        s, _ = orc.step(st, orc.Params(detect_static=False), want_static=True)
        assert s.sum() == 0
