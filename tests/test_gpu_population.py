"""GPU parity of the dynamic population (Section 3.2) against the oracle:
removal and addition move exactly the oracle's agents under the oracle's
ids, and the steps after them (full grid builds over the new population,
the static test with added agents) match the oracle step by step."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import assert_grid_equal, gpu_state, make_sim, note, to_dev
from paper_2301_06984_amd import abm, workloads

pytestmark = pytest.mark.gpu


def ref_state(g, diam):
    n = g["pos"].shape[0]
    return oracle.State(g["pos"].copy(), diam.copy(), g["moved"].astype(np.uint8).copy(),
                        g["nnz"].astype(np.int32).copy(), np.zeros((n, 3), np.float64), 1)


def assert_same(g, st):
    np.testing.assert_array_equal(g["pos"], st.pos)
    np.testing.assert_array_equal(g["moved"], st.moved)
    np.testing.assert_array_equal(g["nnz"], st.nnz)


def step_and_compare(sim, diam, p, want_static):
    """One step of the GPU against one oracle step from the GPU's state."""
    g = gpu_state(sim)
    ref = ref_state(g, diam)
    stat, _ = oracle.step(ref, p, want_static=want_static)
    sim.step(1)
    got = gpu_state(sim)
    scale = np.maximum(np.abs(ref.pos).max(axis=1), float(diam.max()))
    if ref.pos.dtype == np.float32:
        tol = np.spacing(np.abs(ref.pos).max(axis=1)).astype(np.float64)
    else:
        tol = 1e-12 * scale
    assert np.all(np.abs(got["pos"].astype(np.float64) - ref.pos).max(axis=1) <= tol)
    np.testing.assert_array_equal(got["moved"], ref.moved)
    np.testing.assert_array_equal(got["nnz"], ref.nnz)
    if want_static:
        np.testing.assert_array_equal(sim.query("static").cpu().numpy(), stat)
    return g["pos"]


@pytest.mark.parametrize("precision,detect_static", [("f64", False), ("f64", True), ("f32", True)])
def test_remove_add_match_oracle(precision, detect_static):
    w = workloads.c2(n=6000, seed=93) if precision == "f32" else workloads.c1(n=4000, seed=91)
    pos, diam = w.pos, w.diam.copy()
    R = float(diam.max())
    note(f"population {precision} static={detect_static} n={pos.shape[0]}")
    sim = make_sim(pos, diam, capacity=pos.shape[0] + 1500, detect_static=detect_static, interaction_radius=R)
    p = oracle.Params(detect_static=detect_static, interaction_radius=R)
    g = np.random.default_rng(7)
    for _ in range(3):
        step_and_compare(sim, diam, p, detect_static)
    n = pos.shape[0]
    # removal: the oracle's agents under the oracle's ids, bit for bit
    rm = g.choice(n, 600, replace=False)
    before = ref_state(gpu_state(sim), diam)
    note("remove 600")
    sim.remove_agents(torch.from_numpy(rm).cuda())
    exp = oracle.remove_agents(before, rm)
    assert sim.population() == (n - 600, n + 1500)
    assert_same(gpu_state(sim), exp)
    diam = exp.diam
    before_step = step_and_compare(sim, diam, p, detect_static)
    assert_grid_equal(sim, before_step, diam, p)     # the step's grid: a full build over the new population
    step_and_compare(sim, diam, p, detect_static)
    # addition: appended as moved, within the box range, diameters up to R
    m = 900
    lo, hi = before_step.min(axis=0), before_step.max(axis=0)
    new_pos = g.uniform(lo, hi, size=(m, 3)).astype(pos.dtype)
    new_diam = g.uniform(0.6 * R, R, size=m).astype(pos.dtype)
    new_diam[0] = R
    before = ref_state(gpu_state(sim), diam)
    note("add 900")
    sim.add_agents(to_dev(new_pos), to_dev(new_diam))
    exp = oracle.add_agents(before, new_pos, new_diam)
    assert_same(gpu_state(sim), exp)
    diam = exp.diam
    for _ in range(3):
        step_and_compare(sim, diam, p, detect_static)
    # remove again, including added agents and the last ids
    n2 = sim.population()[0]
    rm2 = np.concatenate([np.arange(n2 - 50, n2), g.choice(n2 - 50, 250, replace=False)])
    before = ref_state(gpu_state(sim), diam)
    sim.remove_agents(torch.from_numpy(rm2).cuda())
    exp = oracle.remove_agents(before, rm2)
    assert_same(gpu_state(sim), exp)
    step_and_compare(sim, exp.diam, p, detect_static)


def test_population_errors_leave_state():
    w = workloads.c1(n=1000, seed=95)
    R = float(w.diam.max())
    sim = make_sim(w.pos, w.diam, capacity=1100, interaction_radius=R)
    sim.step(2)
    sim.sync()
    base = gpu_state(sim)
    note("population errors")
    cases = [
        ("capacity", lambda: sim.add_agents(to_dev(np.zeros((101, 3))), to_dev(np.full(101, 10.0)))),
        ("diameter", lambda: sim.add_agents(to_dev(np.zeros((2, 3))), to_dev(np.array([10.0, 2 * R])))),
        ("repeated id", lambda: sim.remove_agents(torch.tensor([3, 5, 3], device="cuda"))),
        ("id range", lambda: sim.remove_agents(torch.tensor([1000], device="cuda"))),
        ("negative id", lambda: sim.remove_agents(torch.tensor([-1], device="cuda"))),
        ("all agents", lambda: sim.remove_agents(torch.arange(1000, device="cuda"))),
    ]
    for name, fn in cases:
        with pytest.raises(abm.ABMError) as e:
            fn()
        assert e.value.code == abm.ABM_E_INVAL, name
        assert sim.population() == (1000, 1100), name
        after = gpu_state(sim)
        for k in base:
            np.testing.assert_array_equal(after[k], base[k], err_msg=name)
    # still steps as before the failed calls
    ref = make_sim(w.pos, w.diam, capacity=1100, interaction_radius=R)
    ref.step(3)
    sim.step(1)
    np.testing.assert_array_equal(gpu_state(sim)["pos"], gpu_state(ref)["pos"])


def test_population_invalidates_graph_and_batched_is_unsupported():
    w = workloads.c1(n=2000, seed=97)
    R = float(w.diam.max())
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        sim = make_sim(w.pos, w.diam, capacity=2100, interaction_radius=R, stream=s)
        sim.step(2)
        sim.graph_capture(2)
        sim.graph_launch()
        sim.sync()
        sim.remove_agents(torch.tensor([0, 7], device="cuda"))
        with pytest.raises(abm.ABMError) as e:
            sim.graph_launch()
        assert e.value.code == abm.ABM_E_STATE
        sim.step(1)
        sim.sync()
    wb = workloads.c4(nsims=3, nmin=200, nmax=400)
    b = abm.BatchedSim(to_dev(wb.pos), to_dev(wb.diam), wb.offsets)
    with pytest.raises(abm.ABMError) as e:
        b.remove_agents(torch.tensor([0], device="cuda"))
    assert e.value.code == abm.ABM_E_UNSUPPORTED


def pick_diameters(g, diam, ids, R):
    """Half grow (up to R), half shrink, a few keep their value."""
    d = diam[ids].astype(np.float64)
    new = np.where(np.arange(ids.size) % 2 == 0, np.minimum(R, d + g.uniform(0.2, 2.0, ids.size)),
                   d - g.uniform(0.3, 2.0, ids.size))
    new[::17] = d[::17]
    return new.astype(diam.dtype)


@pytest.mark.parametrize("precision,detect_static", [("f64", False), ("f32", True), ("f32", False)])
def test_set_diameters_match_oracle(precision, detect_static):
    w = workloads.c2(n=6000, seed=99) if precision == "f32" else workloads.c1(n=4000, seed=98)
    pos, diam = w.pos, w.diam.copy()
    R = float(diam.max())
    note(f"diameters {precision} static={detect_static} n={pos.shape[0]}")
    sim = make_sim(pos, diam, detect_static=detect_static, interaction_radius=R)
    p = oracle.Params(detect_static=detect_static, interaction_radius=R)
    g = np.random.default_rng(11)
    for _ in range(3):
        step_and_compare(sim, diam, p, detect_static)
    n = pos.shape[0]
    ids = g.choice(n, 500, replace=False)
    if detect_static:   # half of them among the agents the last step skipped
        stat = np.nonzero(sim.query("static").cpu().numpy())[0]
        assert stat.size > 250
        ids = np.unique(np.concatenate([g.choice(stat, 250, replace=False), ids]))[:500]
        g.shuffle(ids)
    new = pick_diameters(g, diam, ids, R)
    before = ref_state(gpu_state(sim), diam)
    note("set 500 diameters")
    sim.set_diameters(torch.from_numpy(ids).cuda(), to_dev(new))
    exp = oracle.set_diameters(before, ids, new, radius=R)
    assert_same(gpu_state(sim), exp)
    np.testing.assert_array_equal(sim.query("diameters").cpu().numpy(), exp.diam)
    diam = exp.diam
    # the next grid is an update build over unchanged positions: the oracle's grid
    before_step = step_and_compare(sim, diam, p, detect_static)
    assert_grid_equal(sim, before_step, diam, p)
    for _ in range(3):
        step_and_compare(sim, diam, p, detect_static)


def test_static_switched_on_between_steps():
    """The static test switched on between steps: the first step that runs it
    already skips every agent the oracle calls static (the moved octants of
    the super-boxes come from the agents, not from steps that did not run
    the test), and it stays so over the update builds that follow."""
    w = workloads.c2(n=6000, seed=101)
    pos, diam = w.pos, w.diam.copy()
    R = float(diam.max())
    note(f"static switched on n={pos.shape[0]}")
    sim = make_sim(pos, diam, detect_static=False, interaction_radius=R)
    p = oracle.Params(detect_static=False, interaction_radius=R)
    for _ in range(3):
        step_and_compare(sim, diam, p, False)
    sim.set_params(detect_static=True)
    p = oracle.Params(detect_static=True, interaction_radius=R)
    for _ in range(4):
        step_and_compare(sim, diam, p, True)
    assert sim.query("static").cpu().numpy().sum() > pos.shape[0] // 4


def test_set_diameters_errors_leave_state():
    w = workloads.c1(n=1000, seed=96)
    R = float(w.diam.max())
    sim = make_sim(w.pos, w.diam, interaction_radius=R)
    sim.step(2)
    sim.sync()
    base = gpu_state(sim)
    base_d = sim.query("diameters").cpu().numpy()
    note("diameter errors")
    ids = lambda v: torch.tensor(v, device="cuda")
    cases = [
        ("above R", ids([3, 4]), [9.0, R * 1.01], abm.ABM_E_INVAL),
        ("repeated id", ids([3, 5, 3]), [9.0, 9.0, 9.0], abm.ABM_E_INVAL),
        ("id range", ids([1000]), [9.0], abm.ABM_E_INVAL),
        ("negative id", ids([-1]), [9.0], abm.ABM_E_INVAL),
        ("zero", ids([2]), [0.0], abm.ABM_E_NONFINITE),
        ("nan", ids([2, 6]), [9.0, float("nan")], abm.ABM_E_NONFINITE),
    ]
    for name, i, d, code in cases:
        with pytest.raises(abm.ABMError) as e:
            sim.set_diameters(i, to_dev(np.array(d, dtype=w.diam.dtype)))
        assert e.value.code == code, name
        after = gpu_state(sim)
        for k in base:
            np.testing.assert_array_equal(after[k], base[k], err_msg=name)
        np.testing.assert_array_equal(sim.query("diameters").cpu().numpy(), base_d, err_msg=name)
    # still steps as before the failed calls
    ref = make_sim(w.pos, w.diam, interaction_radius=R)
    ref.step(3)
    sim.step(1)
    np.testing.assert_array_equal(gpu_state(sim)["pos"], gpu_state(ref)["pos"])


def test_set_diameters_batched_and_graph():
    # every simulation of a batch takes the change exactly as it does alone,
    # and a graph captured before the change replays the steps after it
    wb = workloads.c4(nsims=5, nmin=300, nmax=1500, seed=12, steps=6)
    off = wb.offsets
    g = np.random.default_rng(13)
    note(f"batched diameters {len(off) - 1} sims")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b = abm.BatchedSim(to_dev(wb.pos), to_dev(wb.diam), off, common=dict(detect_static=True), stream=s)
        b.step(2)
        b.graph_capture(2)
        ids, new = [], []
        for k in range(len(off) - 1):
            a, e = off[k], off[k + 1]
            loc = g.choice(e - a, 40, replace=False)
            ids.append(a + loc)
            new.append(pick_diameters(g, wb.diam[a:e], loc, float(wb.diam[a:e].max())))
        ids, new = np.concatenate(ids), np.concatenate(new)
        b.set_diameters(torch.from_numpy(ids).cuda(), to_dev(new))
        b.graph_launch()
        b.step(1)
        b.sync()
    got = b.query("positions").cpu().numpy()
    got_d = b.query("diameters").cpu().numpy()
    for k in range(len(off) - 1):
        a, e = off[k], off[k + 1]
        sel = (ids >= a) & (ids < e)
        sim = make_sim(wb.pos[a:e], wb.diam[a:e], detect_static=True)
        sim.step(2)
        sim.set_diameters(torch.from_numpy(ids[sel] - a).cuda(), to_dev(new[sel]))
        sim.step(3)
        np.testing.assert_array_equal(got[a:e], sim.query("positions").cpu().numpy(), err_msg=f"sim {k}")
        np.testing.assert_array_equal(got_d[a:e], sim.query("diameters").cpu().numpy(), err_msg=f"sim {k}")
