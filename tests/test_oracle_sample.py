"""Pin of the oracle's all-pairs sampler (oracle.sample_step).

The sampler checks the full-size GPU runs, where the oracle's grid step would
take too long.  It finds each sampled agent's neighbours by scanning all
agents (Section 3.1's neighbourhood, no grid) and adds the pair terms in
canonical (box rank, id) order.  Here it must equal the grid-based first step
(oracle.step, pinned by the other oracle tests) bit for bit: force, non-zero
count and new position, for every agent, in cases with three or more
contacts per agent (where the order of the sum shows), with the threshold and
the clamp both active, with a box edge above R, in FP32 and FP64 storage and
in both box orders."""
import numpy as np
import pytest

import oracle
from paper_2301_06984_amd import workloads


def first_step(pos, diam, params):
    st = oracle.State.initial(pos, diam)
    oracle.step(st, params)
    return st


def assert_sample_equals_step(pos, diam, params, ids=None):
    n = pos.shape[0]
    ids = np.arange(n) if ids is None else np.asarray(ids)
    st = first_step(pos, diam, oracle.Params(**{**params.__dict__, "detect_static": False}))
    F, nnz, newp = oracle.sample_step(pos, diam, ids, params)
    ref_F = np.ascontiguousarray(st.force[ids])
    np.testing.assert_array_equal(nnz, st.nnz[ids])
    np.testing.assert_array_equal(F.view(np.uint64), ref_F.view(np.uint64))
    np.testing.assert_array_equal(newp, st.pos[ids])
    return nnz


def dense_cube(n, phi, seed, dtype):
    g = np.random.default_rng(seed)
    d = g.uniform(8.0, 12.0, n)
    side = (np.sum(np.pi / 6.0 * d ** 3) / phi) ** (1.0 / 3.0)
    p = g.uniform(0.0, side, (n, 3))
    return p.astype(dtype), d.astype(dtype)


def test_sample_equals_step_c1_small_fp64():
    w = workloads.c1(n=2000, seed=11)
    nnz = assert_sample_equals_step(w.pos, w.diam, oracle.Params())
    assert nnz.max() >= 3


def test_sample_equals_step_c2_small_fp32():
    w = workloads.c2(n=20_000, seed=12)
    assert w.pos.dtype == np.float32
    ids = np.random.default_rng(0).choice(w.n, 3000, replace=False)
    nnz = assert_sample_equals_step(w.pos, w.diam, oracle.Params(), ids)
    assert nnz.max() >= 2


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_sample_equals_step_dense_cube(dtype):
    pos, diam = dense_cube(3000, 0.6, 13, dtype)
    nnz = assert_sample_equals_step(pos, diam, oracle.Params())
    # the sum order matters only from three terms on: most agents have them
    assert np.mean(nnz >= 3) > 0.5


def test_sample_equals_step_threshold_and_clamp():
    pos, diam = dense_cube(3000, 0.5, 14, np.float64)
    p = oracle.Params(f_adh=2.0, delta_max=0.3)
    st = first_step(pos, diam, p)
    fn = np.sqrt(np.sum(st.force ** 2, axis=1))
    mu = p.mu * fn
    assert np.any((fn > 0) & (fn <= p.f_adh)), "some agents must stay below the threshold"
    assert np.any(mu > p.delta_max), "some displacements must be clamped"
    assert_sample_equals_step(pos, diam, p)


def test_sample_equals_step_box_edge_above_r_and_hilbert():
    pos, diam = dense_cube(2500, 0.45, 15, np.float32)
    assert_sample_equals_step(pos, diam, oracle.Params(cell_factor=1.37))
    assert_sample_equals_step(pos, diam, oracle.Params(order=1))


def test_sample_independent_of_threads():
    pos, diam = dense_cube(2000, 0.6, 16, np.float64)
    ids = np.arange(0, 2000, 7)
    a = oracle.sample_step(pos, diam, ids, oracle.Params(nthreads=1))
    b = oracle.sample_step(pos, diam, ids, oracle.Params(nthreads=5))
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def test_sample_order_is_not_id_order():
    # the canonical order differs from plain id order for some agent with
    # three or more contacts, and the two sums then differ in the last bit
    # for some of them: the equality above would catch a sampler that summed
    # in id order
    pos, diam = dense_cube(3000, 0.6, 13, np.float64)
    st = first_step(pos, diam, oracle.Params())
    ids = np.arange(3000)
    start, nb = oracle.neighbors(pos, oracle.radius(diam, oracle.Params()),
                                 oracle.inv_cell(diam, oracle.Params()))
    R = float(diam.max())
    differs = 0
    for i in ids[:600]:
        js = np.sort(nb[start[i]:start[i + 1]]).astype(np.int64)
        F = np.zeros(3)
        for j in js:
            e = pos[i] - pos[j]
            s2 = (e[0] * e[0] + e[1] * e[1]) + e[2] * e[2]
            S = 0.5 * diam[i] + 0.5 * diam[j]
            if not (0.0 < s2 < S * S) or not (s2 < R * R):
                continue
            dist = np.sqrt(s2)
            delta = S - dist
            rho = (0.5 * diam[i] * 0.5 * diam[j]) / S
            f = 2.0 * delta - 1.0 * np.sqrt(rho * delta)
            F = F + (f / dist) * e
        differs += int(np.any(F != st.force[i]))
    assert differs > 0
