"""Pins of the oracle's pair force, displacement rule and step invariants
(Section 5 and Algorithm 1, with the force-law reading in abm_oracle.cpp)."""
import math

import numpy as np
import pytest

from oracle import brute
from paper_2301_06984_amd import workloads


def f_closed(delta, r1, r2, k=2.0, gamma=1.0):
    rho = r1 * r2 / (r1 + r2)
    return k * delta - gamma * math.sqrt(rho * delta)


@pytest.mark.parametrize("s,d1,d2", [(9.0, 10.0, 10.0), (7.5, 8.0, 11.0), (11.99, 12.0, 12.0), (4.0, 8.0, 8.0)])
def test_two_sphere_closed_form(orc, s, d1, d2):
    pos = np.array([[0.0, 0.0, 0.0], [s, 0.0, 0.0]])
    diam = np.array([d1, d2])
    st = orc.State.initial(pos, diam)
    orc.step(st, orc.Params(mu=0.0))
    f = f_closed(0.5 * (d1 + d2) - s, 0.5 * d1, 0.5 * d2)
    np.testing.assert_allclose(st.force[0], [-f, 0.0, 0.0], rtol=1e-14, atol=1e-14)
    np.testing.assert_array_equal(st.force[1], -st.force[0])
    assert st.nnz.tolist() == [1, 1]


def test_no_contact_no_force(orc):
    pos = np.array([[0.0, 0.0, 0.0], [10.5, 0.0, 0.0]])    # within R = 12, outside contact (S = 10)
    st = orc.State.initial(pos, np.array([8.0, 12.0]))
    orc.step(st, orc.Params())
    assert st.nnz.tolist() == [0, 0]
    np.testing.assert_array_equal(st.force, 0.0)


def test_two_sphere_relaxation_to_equilibrium(orc):
    # equilibrium overlap delta* = gamma^2 rho / k^2; for r = 5: rho = 2.5, delta* = 0.625
    # the overlap map delta -> delta - 2 mu f(delta) has slope 1 - mu k = 0.8 at delta*
    pos = np.array([[0.0, 0.0, 0.0], [9.0, 0.0, 0.0]])
    st = orc.State.initial(pos, np.array([10.0, 10.0]))
    p = orc.Params()
    errs = []
    for _ in range(120):
        orc.step(st, p)
        delta = 10.0 - (st.pos[1, 0] - st.pos[0, 0])
        errs.append(delta - 0.625)
    assert abs(errs[-1]) < 1e-10
    assert all(e > 0 for e in errs[:60])              # monotone approach from above
    ratios = [errs[i + 1] / errs[i] for i in range(10, 40)]
    np.testing.assert_allclose(ratios, 0.8, atol=5e-3)
    assert errs[0] < 1.0 - 0.625


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_forces_match_all_pairs(orc, dtype):
    pos, diam = workloads.uniform_cube(900, 70.0, seed=31, dtype=dtype)
    st = orc.State.initial(pos, diam)
    orc.step(st, orc.Params(mu=0.0))
    R = float(diam.astype(np.float64).max())
    F, nnz, absum = brute.forces(pos, diam, 2.0, 1.0, R)
    np.testing.assert_array_equal(st.nnz, nnz)
    err = np.abs(st.force - F).max(axis=1)
    assert np.all(err <= 1e-13 * np.maximum(absum, 1.0))
    assert (nnz > 1).sum() > 100


def test_newton_third_law(orc):
    w = workloads.c1(n=3000, seed=32)
    st = orc.State.initial(w.pos, w.diam)
    orc.step(st, orc.Params())
    total = st.force.sum(axis=0)
    bound = st.force.shape[0] * np.finfo(np.float64).eps * np.abs(st.force).max() * 4
    assert np.all(np.abs(total) <= bound)
    assert np.abs(st.force).max() > 1.0


def test_translation_invariance_bitwise_and_relabel(orc):
    g = np.random.default_rng(33)
    pos = np.round(g.uniform(0, 120, size=(1200, 3)) * 2 ** 20) / 2 ** 20   # exact under integer shifts
    diam = np.round(g.uniform(8, 12, size=1200) * 2 ** 10) / 2 ** 10
    R = diam.max()
    base = orc.State.initial(pos, diam)
    orc.step(base, orc.Params(mu=0.0))
    # shift by a whole number of boxes: same keys, same order -> identical bits
    sh = orc.State.initial(pos + 37 * R, diam)
    assert np.all((pos + 37 * R) - 37 * R == pos)
    orc.step(sh, orc.Params(mu=0.0))
    np.testing.assert_array_equal(sh.force, base.force)
    # arbitrary shift: different boxes, same neighbour sets -> same forces up to order
    sh2 = orc.State.initial(pos + 1000.3125, diam)
    orc.step(sh2, orc.Params(mu=0.0))
    np.testing.assert_allclose(sh2.force, base.force, rtol=0, atol=1e-12)
    # relabelling the agents permutes the forces
    perm = g.permutation(pos.shape[0])
    rl = orc.State.initial(pos[perm], diam[perm])
    orc.step(rl, orc.Params(mu=0.0))
    np.testing.assert_allclose(rl.force, base.force[perm], rtol=0, atol=1e-12)
    np.testing.assert_array_equal(rl.nnz, base.nnz[perm])


def test_threshold_boundary(orc):
    pos = np.array([[0.0, 0.0, 0.0], [9.0, 0.0, 0.0]])
    diam = np.array([10.0, 10.0])
    probe = orc.State.initial(pos, diam)
    orc.step(probe, orc.Params(mu=0.0))
    Fn = math.sqrt(float(probe.force[0, 0]) ** 2)
    at = orc.State.initial(pos, diam)
    orc.step(at, orc.Params(f_adh=Fn))                       # |F| == f_adh: no move
    np.testing.assert_array_equal(at.pos, pos)
    assert at.moved.tolist() == [0, 0]
    below = orc.State.initial(pos, diam)
    orc.step(below, orc.Params(f_adh=math.nextafter(Fn, 0.0)))
    assert below.moved.tolist() == [1, 1]
    np.testing.assert_allclose(below.pos[0, 0], -0.1 * Fn, rtol=1e-15)


def test_clamp(orc):
    pos = np.array([[0.0, 0.0, 0.0], [3.0, 4.0, 0.0]])       # deep overlap, large force
    st = orc.State.initial(pos, np.array([12.0, 12.0]))
    _, disp = orc.step(st, orc.Params(mu=10.0, delta_max=0.75), want_disp=True)
    n = np.sqrt((disp * disp).sum(axis=1))
    np.testing.assert_allclose(n, 0.75, rtol=2 * np.finfo(float).eps)
    np.testing.assert_allclose(disp[0] / n[0], [-0.6, -0.8, 0.0], atol=1e-15)


def test_jacobi_update_order_free(orc):
    # positions are committed after all forces: the result does not depend on agent order
    w = workloads.c1(n=800, seed=34)
    a = orc.run(w.pos, w.diam, 3, orc.Params())
    perm = np.random.default_rng(0).permutation(800)
    b = orc.run(w.pos[perm], w.diam[perm], 3, orc.Params())
    np.testing.assert_allclose(b.pos, a.pos[perm], rtol=0, atol=1e-11)


def test_fp32_rounds_once(orc):
    pos = np.array([[0.0, 0.0, 0.0], [9.0, 0.0, 0.0]], np.float32)
    diam = np.array([10.0, 10.0], np.float32)
    s64 = orc.State.initial(pos.astype(np.float64), diam.astype(np.float64))
    _, disp = orc.step(s64, orc.Params(), want_disp=True)
    s32 = orc.State.initial(pos, diam)
    orc.step(s32, orc.Params())
    np.testing.assert_array_equal(s32.force, s64.force)
    np.testing.assert_array_equal(s32.pos, (pos.astype(np.float64) + disp).astype(np.float32))
