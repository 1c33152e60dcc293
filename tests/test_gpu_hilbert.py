"""The Hilbert order of the super-boxes, the variant order next to Morton
order (Section 4.2): grids and steps against the oracle in the same order,
the static skip and batches bit for bit against the same order's other
runs, and the order's argument checks."""
import numpy as np
import pytest

import oracle
from gpu_helpers import assert_grid_equal, gpu_state, make_sim, note, to_dev
from paper_2301_06984_amd import abm, workloads

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,detect_static", [("f64", False), ("f32", True), ("f32", False)])
def test_hilbert_steps_match_oracle(precision, detect_static):
    # every step from the GPU's state against one oracle step in the same
    # order.  The grid (keys, canonical order, box starts) and the integer
    # outcome are exact.  The pair terms are summed in another order than the
    # oracle's canonical one: the walk takes an agent's 8 super-boxes in
    # their Morton order.  So positions agree to the tolerance: 1e-12
    # relative in FP64, and one float spacing in FP32, whose rounding of the
    # new position can differ
    w = workloads.c2(n=20000, seed=41) if precision == "f32" else workloads.c1(n=6000, seed=42)
    note(f"hilbert {precision} static={detect_static} n={w.n}")
    sim = make_sim(w.pos, w.diam, order="hilbert", detect_static=detect_static)
    p = oracle.Params(order=1, detect_static=detect_static)
    g = dict(pos=w.pos.copy(), moved=np.ones(w.n, np.uint8), nnz=np.zeros(w.n, np.int32))
    for t in range(8):
        st = oracle.State(g["pos"].copy(), w.diam.copy(), g["moved"].astype(np.uint8).copy(),
                          g["nnz"].astype(np.int32).copy(), np.zeros((w.n, 3)), t)
        before = st.pos.copy()
        stat, _ = oracle.step(st, p, want_static=detect_static)
        sim.step(1)
        g = gpu_state(sim)
        if precision == "f64":
            tol = 1e-12 * np.maximum(np.abs(st.pos).max(axis=1), float(w.diam.max()))[:, None]
        else:
            tol = np.spacing(np.abs(st.pos)).astype(np.float64)
        d = np.abs(g["pos"].astype(np.float64) - st.pos.astype(np.float64))
        assert np.all(d <= tol), (t, d.max())
        np.testing.assert_array_equal(g["moved"], st.moved, err_msg=f"step {t}")
        np.testing.assert_array_equal(g["nnz"], st.nnz, err_msg=f"step {t}")
        if detect_static:
            np.testing.assert_array_equal(sim.query("static").cpu().numpy(), stat, err_msg=f"step {t}")
        if t in (0, 1, 7):   # a full build, then update builds
            assert_grid_equal(sim, before, w.diam, p)


def test_hilbert_static_skip_is_exact():
    # the walk's order is the same with and without the skip, so the skip
    # changes nothing, bit for bit
    w = workloads.c2(n=30000, seed=45)
    note(f"hilbert skip on/off n={w.n}")
    on = make_sim(w.pos, w.diam, order="hilbert", detect_static=True)
    off = make_sim(w.pos, w.diam, order="hilbert", detect_static=False)
    on.step(12)
    off.step(12)
    np.testing.assert_array_equal(gpu_state(on)["pos"], gpu_state(off)["pos"])
    np.testing.assert_array_equal(gpu_state(on)["nnz"], gpu_state(off)["nnz"])
    assert on.query("static").cpu().numpy().mean() > 0.3


def test_hilbert_batched_equals_plain_runs():
    w = workloads.c4(nsims=12, nmin=50, nmax=3000, seed=43, steps=6)
    off = w.offsets
    note(f"hilbert batched {len(off) - 1} sims n={w.n}")
    b = abm.BatchedSim(to_dev(w.pos), to_dev(w.diam), off, common=dict(order="hilbert", detect_static=True))
    b.step(w.steps)
    got = b.query("positions").cpu().numpy()
    for s in range(len(off) - 1):
        a, e = off[s], off[s + 1]
        sim = make_sim(w.pos[a:e], w.diam[a:e], order="hilbert", detect_static=True)
        sim.step(w.steps)
        np.testing.assert_array_equal(got[a:e], sim.query("positions").cpu().numpy(), err_msg=f"sim {s}")


def test_hilbert_order_arguments():
    w = workloads.c4(nsims=2, nmin=200, nmax=400, seed=44)
    note("hilbert argument checks")
    with pytest.raises(abm.ABMError) as e:
        abm.BatchedSim(to_dev(w.pos), to_dev(w.diam), w.offsets, params=[dict(order=0), dict(order=1)])
    assert e.value.code == abm.ABM_E_INVAL
    with pytest.raises(abm.ABMError) as e:
        make_sim(w.pos, w.diam, order=2)
    assert e.value.code == abm.ABM_E_INVAL
    sim = make_sim(w.pos, w.diam, order="hilbert")
    with pytest.raises(abm.ABMError) as e:
        sim.set_params(order=0)
    assert e.value.code == abm.ABM_E_UNSUPPORTED
    sim.step(2)
    sim.sync()


def test_hilbert_adjoint_matches_oracle():
    # the reverse step in the Hilbert order against the oracle's reverse mode
    # in that order: the pair terms are summed in another order than the
    # oracle's (see the steps above), so positions agree to 1e-12 and the
    # gradients to the adjoint's 1e-9
    import torch
    g = np.random.default_rng(46)
    n = 3000
    side = (n / workloads.C1_DENSITY) ** (1 / 3)
    pos = g.uniform(0, side, size=(n, 3))
    diam = g.uniform(8, 12, size=n)
    target = pos + g.normal(0, 0.5, size=(n, 3))
    note(f"hilbert adjoint n={n}")
    sim = make_sim(pos, diam, order="hilbert")
    sim.forward_record(12, 5)
    xT = sim.query("positions").double()
    gx0, gp = sim.backward(2.0 * (xT - torch.from_numpy(target).cuda()) / (3 * n))
    ref = oracle.adjoint(pos, diam, 12, oracle.Params(order=1), target)
    assert np.abs(xT.cpu().numpy() - ref["posT"]).max() <= 1e-12 * np.abs(ref["posT"]).max()
    np.testing.assert_allclose(gp.cpu().numpy(), [ref["dL_dk"], ref["dL_dgamma"]], rtol=1e-9)
    assert np.abs(gx0.cpu().numpy() - ref["dL_dx0"]).max() <= 1e-9 * np.abs(ref["dL_dx0"]).max()
