"""Parity at the workloads' full sizes, in the launch configuration the
benchmark times: the whole grid against the oracle where it finishes in
seconds, sampled agents against the all-pairs definition otherwise, and
properties that hold at any size."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import assert_grid_equal, gpu_state, make_sim, note, to_dev
from paper_2301_06984_amd import abm, workloads

pytestmark = pytest.mark.gpu

BENCH = dict(sort_every=1, block_size=256, detect_static=False, super_slack=1.2)   # the benchmark's launch configuration


def check_samples(pos, diam, got_pos, nsamples, seed, params=oracle.Params(), got_nnz=None):
    """New positions of sampled agents against the oracle's all-pairs
    sampler, bit for bit: both add each agent's pair terms in canonical
    (Morton box rank, id) order, which is also the GPU's order in the
    Hilbert box order (its walk takes the 2x2x2 blocks in Morton order)."""
    ids = np.random.default_rng(seed).choice(pos.shape[0], nsamples, replace=False)
    note(f"sampler: {nsamples} agents of {pos.shape[0]}")
    F, nnz, newp = oracle.sample_step(pos, diam, ids, params)
    np.testing.assert_array_equal(got_pos[ids], newp)
    if got_nnz is not None:
        np.testing.assert_array_equal(got_nnz[ids], nnz)
    return ids, nnz


@pytest.mark.parametrize("detect_static", [False, True])
def test_headline_1e7_first_step(detect_static):
    w = workloads.headline()
    note(f"headline n={w.n} side={w.meta['side']:.1f} static test {detect_static}")
    sim = make_sim(w.pos, w.diam, **{**BENCH, "detect_static": detect_static})
    sim.step(1)
    sim.sync()
    note("headline grid parity")
    assert_grid_equal(sim, w.pos, w.diam, oracle.Params())
    got = sim.query("positions").cpu().numpy()
    _, nnz = check_samples(w.pos, w.diam, got, 96, 1)
    gn = sim.query("nnz").cpu().numpy()
    assert gn.mean() > 0.3
    note("headline 20 more steps")
    sim.step(20)
    sim.sync()
    x = sim.query("positions").cpu().numpy()
    assert np.isfinite(x).all()
    # a later step: its grid is an update of the last one (agents re-laid out
    # every step, extent unchanged); grid and sampled agents against the oracle
    note("headline step 22 (update build) grid + samples")
    sim.step(1)
    sim.sync()
    assert_grid_equal(sim, x, w.diam, oracle.Params())
    check_samples(x, w.diam, sim.query("positions").cpu().numpy(), 96, 2)


def test_c1_density_1e7_shared_terms_sampled():
    """C1's density with 1e7 agents (about 47 candidates and 4 contacts per
    agent), in the walk the library takes there (2-wide, the wave sharing
    its pair terms, 14 queue rows): the first step and a later update-build
    step, sampled agents against the oracle's all-pairs sampler bit for bit,
    non-zero counts exactly."""
    n = 10_000_000
    side = (n / workloads.C1_DENSITY) ** (1.0 / 3.0)
    pos, diam = workloads.uniform_cube(n, side, (1, n), dtype=np.float32)
    note(f"c1 density n={n} side={side:.1f}")
    sim = make_sim(pos, diam, **{**BENCH, "walk_chunk": 2, "share_terms": 2})
    sim.step(1)
    sim.sync()
    _, nnz = check_samples(pos, diam, sim.query("positions").cpu().numpy(), 64, 11,
                           got_nnz=sim.query("nnz").cpu().numpy())
    assert nnz.mean() > 2.0   # several contacts per agent: the terms are shared out
    note("c1 density steps 2-4")
    sim.step(3)
    sim.sync()
    x = sim.query("positions").cpu().numpy()
    note("c1 density step 5 (update build) sampled")
    sim.step(1)
    sim.sync()
    check_samples(x, diam, sim.query("positions").cpu().numpy(), 64, 12, got_nnz=sim.query("nnz").cpu().numpy())


def test_c2_full_parity_and_skip():
    w = workloads.c2()
    note(f"c2 n={w.n}")
    on = make_sim(w.pos, w.diam, **{**BENCH, "detect_static": True})
    off = make_sim(w.pos, w.diam, **{**BENCH, "detect_static": False})
    on.step(1)
    st = oracle.State.initial(w.pos, w.diam)
    oracle.step(st, oracle.Params(detect_static=True))
    g = gpu_state(on)
    np.testing.assert_array_equal(g["nnz"], st.nnz)
    np.testing.assert_array_equal(g["moved"], st.moved)
    assert np.all(np.abs(g["pos"].astype(np.float64) - st.pos) <= np.spacing(np.abs(st.pos)).astype(np.float64))
    exact = np.mean(np.all(g["pos"] == st.pos, axis=1))
    note(f"c2 first step bit-exact fraction {exact:.6f}")
    off.step(1)
    on.step(49)
    off.step(49)
    a, b = gpu_state(on), gpu_state(off)
    np.testing.assert_array_equal(a["pos"], b["pos"])
    # one more step from the GPU's state, against the oracle from that same state
    mid = oracle.State(a["pos"].copy(), w.diam.copy(), a["moved"].copy(), a["nnz"].copy(),
                       np.zeros((w.n, 3)), 50)
    oracle.step(mid, oracle.Params(detect_static=True))
    on.step(1)
    c = gpu_state(on)
    np.testing.assert_array_equal(c["moved"], mid.moved)
    assert np.all(np.abs(c["pos"].astype(np.float64) - mid.pos) <= np.spacing(np.abs(mid.pos)).astype(np.float64))
    frac = on.stats()["n_static"] / w.n
    note(f"c2 skip fraction at step 51: {frac:.3f}")
    assert frac > 0.4
    on.step(49)
    off.step(50)
    np.testing.assert_array_equal(gpu_state(on)["pos"], gpu_state(off)["pos"])


def test_c3_clustered_all_steps_sampled():
    # the clustered workload over its 20 steps, re-laid out every 10th step:
    # sampled agents of steps 1, 10, 11 and 20 (full and update builds, both
    # sides of a re-layout, the clamp active almost everywhere) against the
    # sampler fed the GPU's state before the step
    w = workloads.c3()
    note(f"c3 n={w.n}")
    sim = make_sim(w.pos, w.diam, sort_every=w.sort_every, block_size=256)
    t = 0
    x = w.pos
    for at in (1, 10, 11, 20):
        if at - 1 > t:
            note(f"c3 steps {t + 1}..{at - 1}")
            sim.step(at - 1 - t)
            sim.sync()
            t = at - 1
            x = sim.query("positions").cpu().numpy()
        note(f"c3 step {at}")
        sim.step(1)
        sim.sync()
        t = at
        got = sim.query("positions").cpu().numpy()
        gn = sim.query("nnz").cpu().numpy()
        _, nnz = check_samples(x, w.diam, got, 24, 30 + at, got_nnz=gn)
        assert nnz.mean() > 5
        x = got


def test_c4_batched_graph_sampled_sims():
    w = workloads.c4()
    note(f"c4 nsims={len(w.offsets) - 1} n={w.n}")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b = abm.BatchedSim(to_dev(w.pos), to_dev(w.diam), w.offsets, stream=s)
        b.graph_capture(w.steps)
        b.graph_launch()
        b.sync()
        got = b.query("positions").cpu().numpy()
    for sidx in np.random.default_rng(4).choice(len(w.offsets) - 1, 6, replace=False):
        a, e = w.offsets[sidx], w.offsets[sidx + 1]
        note(f"c4 sim {sidx} n={e - a}")
        sim = make_sim(w.pos[a:e], w.diam[a:e])
        sim.step(w.steps)
        np.testing.assert_array_equal(got[a:e], sim.query("positions").cpu().numpy())
    # three simulations of the batch against the oracle's 50 steps: the
    # smallest, and two of fewer than 20,000 agents drawn by seed
    sizes = np.diff(w.offsets)
    small = np.flatnonzero(sizes < 20_000)
    pick = [int(np.argmin(sizes))] + [int(x) for x in np.random.default_rng(44).choice(small, 2, replace=False)]
    for sidx in pick:
        a, e = w.offsets[sidx], w.offsets[sidx + 1]
        note(f"c4 sim {sidx} n={e - a} against the oracle")
        ref = oracle.run(w.pos[a:e], w.diam[a:e], w.steps, oracle.Params())
        np.testing.assert_array_equal(got[a:e], ref.pos)


def test_c5_adjoint_full():
    w = workloads.c5()
    note(f"c5 adjoint n={w.n}")
    sim = make_sim(w.pos, w.diam)
    sim.forward_record(w.steps, w.meta["ckpt_every"])
    xT = sim.query("positions").double()
    t = torch.from_numpy(w.target).cuda()
    gx0, gp = sim.backward(2.0 * (xT - t) / (3 * w.n))
    note("c5 oracle adjoint")
    ref = oracle.adjoint(w.pos, w.diam, w.steps, oracle.Params(), w.target)
    np.testing.assert_array_equal(xT.cpu().numpy(), ref["posT"].astype(np.float64))
    np.testing.assert_allclose(gp.cpu().numpy(), [ref["dL_dk"], ref["dL_dgamma"]], rtol=1e-8)
    assert np.abs(gx0.cpu().numpy() - ref["dL_dx0"]).max() <= 1e-8 * np.abs(ref["dL_dx0"]).max()


def test_headline_1e7_hilbert_order():
    # the headline workload in the Hilbert order: the grid of a full build and
    # of an update build against the oracle's, sampled agents against the
    # all-pairs definition, and the same integer outcome as the Morton order
    # (the order changes only the summation order of the pair terms)
    w = workloads.headline()
    note(f"headline hilbert n={w.n}")
    p = oracle.Params(order=1)
    sim = make_sim(w.pos, w.diam, order="hilbert", **BENCH)
    ref = make_sim(w.pos, w.diam, **BENCH)
    sim.step(1)
    ref.step(1)
    sim.sync()
    note("headline hilbert grid parity")
    assert_grid_equal(sim, w.pos, w.diam, p)
    got = sim.query("positions").cpu().numpy()
    check_samples(w.pos, w.diam, got, 96, 3)
    np.testing.assert_array_equal(sim.query("nnz").cpu().numpy(), ref.query("nnz").cpu().numpy())
    np.testing.assert_array_equal(sim.query("moved").cpu().numpy(), ref.query("moved").cpu().numpy())
    d = np.abs(got.astype(np.float64) - ref.query("positions").cpu().numpy().astype(np.float64))
    assert np.all(d <= np.spacing(np.abs(got)).astype(np.float64))
    del ref
    note("headline hilbert 10 more steps, then an update build")
    sim.step(10)
    sim.sync()
    x = sim.query("positions").cpu().numpy()
    sim.step(1)
    sim.sync()
    assert_grid_equal(sim, x, w.diam, p)
    check_samples(x, w.diam, sim.query("positions").cpu().numpy(), 96, 4)


def test_headline_1e7_fp64_state():
    # the headline workload with FP64 state: a full build, then an update
    # build from the GPU's state, grid and sampled agents against the oracle
    w = workloads.headline(dtype=np.float64)
    note(f"headline fp64 n={w.n}")
    sim = make_sim(w.pos, w.diam, **BENCH)
    sim.step(1)
    sim.sync()
    got = sim.query("positions").cpu().numpy()
    check_samples(w.pos, w.diam, got, 96, 5, got_nnz=sim.query("nnz").cpu().numpy())
    note("headline fp64 5 more steps, then an update build")
    sim.step(5)
    sim.sync()
    x = sim.query("positions").cpu().numpy()
    sim.step(1)
    sim.sync()
    assert_grid_equal(sim, x, w.diam, oracle.Params())
    check_samples(x, w.diam, sim.query("positions").cpu().numpy(), 96, 6, got_nnz=sim.query("nnz").cpu().numpy())


def test_uniform_1e8_sampled():
    # 1e8 spheres uniform at the c2 density (the scale sweep's workload):
    # the first step and a later update build, sampled against the oracle
    n = 100_000_000
    side = (n / workloads.C2_DENSITY) ** (1.0 / 3.0)
    note(f"uniform 1e8: generating (side {side:.1f})")
    p, d = workloads.uniform_cube(n, side, (6, n), dtype=np.float32)
    sim = make_sim(p, d, detect_static=False, sort_every=1, block_size=512, box_slack=1.05)
    note("uniform 1e8 step 1")
    sim.step(1)
    sim.sync()
    check_samples(p, d, sim.query("positions").cpu().numpy(), 48, 7, got_nnz=sim.query("nnz").cpu().numpy())
    note("uniform 1e8 steps 2-3, then step 4 (update build)")
    sim.step(2)
    sim.sync()
    x = sim.query("positions").cpu().numpy()
    sim.step(1)
    sim.sync()
    check_samples(x, d, sim.query("positions").cpu().numpy(), 48, 8, got_nnz=sim.query("nnz").cpu().numpy())


def test_uniform_1e9_sampled():
    # 1e9 spheres uniform at the c2 density: 2e9 loose slots, near the 32-bit
    # limit of the slot space; the first step (full build) and the next
    # (update build), sampled against the oracle
    n = 1_000_000_000
    side = (n / workloads.C2_DENSITY) ** (1.0 / 3.0)
    note(f"uniform 1e9: generating (side {side:.1f})")
    p, d = workloads.uniform_cube(n, side, (6, n), dtype=np.float32)
    sim = make_sim(p, d, detect_static=False, sort_every=1, block_size=256, box_slack=1.05, super_slack=1.2)
    note("uniform 1e9 step 1")
    sim.step(1)
    sim.sync()
    x = sim.query("positions").cpu().numpy()
    check_samples(p, d, x, 32, 9, got_nnz=sim.query("nnz").cpu().numpy())
    del p
    note("uniform 1e9 step 2 (update build)")
    sim.step(1)
    sim.sync()
    check_samples(x, d, sim.query("positions").cpu().numpy(), 32, 10, got_nnz=sim.query("nnz").cpu().numpy())


def test_uniform_1_72e9_sampled():
    # 1.72e9 spheres uniform at the c2 density (the agent count of the
    # paper's largest run): 3.44e9 loose slots and 3.9e9 boxes, past 2^31,
    # built from chunks of 1e8 agents (as the scale sweep builds it) with a
    # super-box table sized for the grid; the first step (full build) and the
    # next (update build), sampled against the oracle with the same R
    n, chunk = 1_720_000_000, 100_000_000
    side = (n / workloads.C2_DENSITY) ** (1.0 / 3.0)
    params = oracle.Params(interaction_radius=12.0)
    ps, ds, sim = [], [], None
    for k in range((n + chunk - 1) // chunk):
        m = min(chunk, n - k * chunk)
        p, d = workloads.uniform_cube(m, side, (6, n, k), dtype=np.float32)
        ps.append(p)
        ds.append(d)
        if sim is None:
            sim = make_sim(p, d, capacity=n, interaction_radius=12.0, super_slack=1.2, box_slack=1.05,
                           detect_static=False, sort_every=1, block_size=256)
        else:
            sim.add_agents(to_dev(p), to_dev(d))
        note(f"uniform 1.72e9: {k * chunk + m} agents in the context")
    p, d = np.concatenate(ps), np.concatenate(ds)
    del ps, ds
    note("uniform 1.72e9 step 1")
    sim.step(1)
    sim.sync()
    x = sim.query("positions").cpu().numpy()
    check_samples(p, d, x, 32, 11, params=params, got_nnz=sim.query("nnz").cpu().numpy())
    del p
    note("uniform 1.72e9 step 2 (update build)")
    sim.step(1)
    sim.sync()
    check_samples(x, d, sim.query("positions").cpu().numpy(), 32, 12, params=params,
                  got_nnz=sim.query("nnz").cpu().numpy())
    assert sim.stats()["error"] == 0
