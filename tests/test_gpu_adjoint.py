"""Reverse-mode step on the GPU against the oracle's reverse mode and FP64
finite differences; the autograd wrapper."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import make_sim, note, to_dev
from paper_2301_06984_amd import abm, workloads

pytestmark = pytest.mark.gpu


def case(n, seed, dtype=np.float64):
    g = np.random.default_rng(seed)
    side = (n / workloads.C1_DENSITY) ** (1 / 3)
    pos = g.uniform(0, side, size=(n, 3)).astype(dtype)
    diam = g.uniform(8, 12, size=n).astype(dtype)
    target = pos.astype(np.float64) + g.normal(0, 0.5, size=(n, 3))
    return pos, diam, target


def gpu_grad(pos, diam, target, steps, ckpt, tapes="auto", info=None, **kw):
    sim = make_sim(pos, diam, **kw)
    sim.forward_record(steps, ckpt, tapes=tapes)
    xT = sim.query("positions").double()
    t = torch.from_numpy(target).cuda()
    n = pos.shape[0]
    loss = float(((xT - t) ** 2).mean())
    gx0, gp = sim.backward(2.0 * (xT - t) / (3 * n))
    if info is not None:
        info.update(sim.record_info())
    return loss, gx0.cpu().numpy(), gp.cpu().numpy(), xT.cpu().numpy()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_adjoint_matches_oracle(dtype):
    pos, diam, target = case(3000, 1, dtype)
    note(f"adjoint vs oracle {dtype.__name__}")
    loss, gx0, gp, xT = gpu_grad(pos, diam, target, 12, 5)
    ref = oracle.adjoint(pos, diam, 12, oracle.Params(), target)
    assert abs(loss - ref["loss"]) <= 1e-12 * abs(ref["loss"])
    np.testing.assert_allclose(gp, [ref["dL_dk"], ref["dL_dgamma"]], rtol=1e-9)
    scale = np.abs(ref["dL_dx0"]).max()
    assert np.abs(gx0 - ref["dL_dx0"]).max() <= 1e-9 * scale


def test_adjoint_fd_fp64():
    pos, diam, target = case(400, 2)
    note("adjoint FD")
    steps = 8
    loss, gx0, gp, _ = gpu_grad(pos, diam, target, steps, 3)

    def L(p=None, **kw):
        sim = make_sim(pos if p is None else p, diam, **kw)
        sim.step(steps)
        x = sim.query("positions").cpu().numpy()
        return float(np.mean((x - target) ** 2))

    # Central differences converge to the derivative as h^2 until rounding
    # takes over: with h cut by 4 each time, the error against the adjoint must
    # shrink by at least 8 (16 in the limit) or already lie below the rounding
    # floor (a few ulp of the loss over h), and the smallest error must be
    # tight.  A wrong adjoint stalls at its own error instead.
    L0 = L()

    def floor(h):
        return 1e-15 * abs(L0) / h

    for name, idx in (("k", 0), ("gamma", 1)):
        base = 2.0 if name == "k" else 1.0
        hs = [4e-6 * base, 1e-6 * base, 2.5e-7 * base, 6.25e-8 * base]
        errs = [abs((L(**{name: base + h}) - L(**{name: base - h})) / (2 * h) - gp[idx]) for h in hs]
        for e0, e1, h1 in zip(errs, errs[1:], hs[1:]):
            assert e1 <= e0 / 8.0 or e1 <= floor(h1), (name, errs)
        assert errs[-1] <= 1e-7 * abs(gp[idx]) + floor(hs[-1]), (name, errs)
    # initial positions: the truncation error is far below the rounding floor
    # already at h = 4e-6, so the differences must agree with the adjoint to
    # that floor plus 1e-6 relative at two step sizes
    g = np.random.default_rng(3)
    for c in g.choice(pos.size, 16, replace=False):
        an = gx0.ravel()[c]
        for h in (4e-6, 1e-6):
            pp = pos.copy().ravel(); pp[c] += h
            pm = pos.copy().ravel(); pm[c] -= h
            fd = (L(pp.reshape(-1, 3)) - L(pm.reshape(-1, 3))) / (2 * h)
            assert abs(fd - an) <= 1e-6 * abs(an) + floor(h), (c, h, fd, an)


def test_stepfn_autograd():
    pos, diam, target = case(1500, 4)
    note("StepFn autograd")
    x0 = to_dev(pos).requires_grad_(True)
    k = torch.tensor(2.0, dtype=torch.float64, requires_grad=True)
    gam = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    xT = abm.StepFn.apply(x0, to_dev(diam), k, gam, 10, 5, None)
    loss = ((xT - torch.from_numpy(target).cuda()) ** 2).mean()
    loss.backward()
    ref = oracle.adjoint(pos, diam, 10, oracle.Params(), target)
    np.testing.assert_allclose([k.grad.item(), gam.grad.item()], [ref["dL_dk"], ref["dL_dgamma"]], rtol=1e-9)
    assert np.abs(x0.grad.cpu().numpy() - ref["dL_dx0"]).max() <= 1e-9 * np.abs(ref["dL_dx0"]).max()


def test_state_restored_after_backward():
    pos, diam, target = case(800, 5)
    note("adjoint state restore")
    sim = make_sim(pos, diam)
    sim.forward_record(6, 4)
    x_after = sim.query("positions").cpu().numpy()
    sim.backward(torch.zeros((800, 3), dtype=torch.float64, device="cuda"))
    np.testing.assert_array_equal(sim.query("positions").cpu().numpy(), x_after)
    sim.step(2)
    ref = make_sim(pos, diam)
    ref.step(8)
    np.testing.assert_array_equal(sim.query("positions").cpu().numpy(), ref.query("positions").cpu().numpy())


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_contact_tapes_bitwise(dtype):
    """The reverse steps on contact tapes (every step's, or each recomputed
    segment's) give the walked grid's result bit for bit, with or without
    re-layouts during the record (lambda is kept by id)."""
    pos, diam, target = case(3000, 6, dtype)
    res = {}
    for sort_every in (0, 1, 3):
        for tapes, mode in (("none", 0), ("segment", 1), ("all", 2)):
            note(f"adjoint tapes={tapes} sort_every={sort_every} {dtype.__name__}")
            info = {}
            res[tapes, sort_every] = gpu_grad(pos, diam, target, 12, 5, tapes=tapes, info=info, sort_every=sort_every)
            assert info["tapes"] == mode, info
            assert info["taped_reverse_steps"] == (0 if mode == 0 else 12), info
            assert 0 < info["worst_contacts"] <= 32 or mode == 0, info
    for key, r in res.items():
        for a, b in zip(res["none", 0], r):
            np.testing.assert_array_equal(np.asarray(a), np.asarray(b), err_msg=str(key))


def test_contact_tape_overflow_falls_back():
    """A cluster where agents touch more than 32 others: the record cannot tape
    every step, the backward tapes each recomputed segment and walks the grid
    of the steps whose tape is incomplete; the result is still bit for bit that
    of the walked grids."""
    pos, diam, target = case(2000, 7)
    g = np.random.default_rng(8)
    centre = pos.mean(axis=0)
    v = g.normal(size=(48, 3))
    v *= (g.uniform(0.0, 1.0, size=(48, 1)) ** (1 / 3) * 2.5) / np.linalg.norm(v, axis=1, keepdims=True)
    pos[:48] = centre + v   # 48 spheres of diameter >= 8 within 5 of each other
    note("adjoint tape overflow")
    info = {}
    ref = gpu_grad(pos, diam, target, 10, 4, tapes="none")
    got = gpu_grad(pos, diam, target, 10, 4, tapes="all", info=info)
    assert info["tapes"] == 1 and info["worst_contacts"] > 32, info
    assert 0 < info["taped_reverse_steps"] < 10, info
    for a, b in zip(ref, got):
        np.testing.assert_array_equal(np.asarray(a), np.asarray(b))


@pytest.mark.parametrize("n,steps,ckpt", [(1, 3, 2), (2, 3, 10), (65, 5, 2), (65, 4, 4)])
def test_contact_tapes_edge_cases(n, steps, ckpt):
    """Tiny inputs, a checkpoint interval longer than the run and a last
    segment shorter than the others: every tape mode gives the walked result
    bit for bit, and the oracle's reverse mode to 1e-9."""
    g = np.random.default_rng(90 + n)
    side = max(6.0, (n / workloads.C1_DENSITY) ** (1 / 3) / 2)   # denser than C1: contacts from the start
    pos = g.uniform(0, side, size=(n, 3))
    diam = g.uniform(8, 12, size=n)
    target = pos + g.normal(0, 0.5, size=(n, 3))
    res = {}
    for tapes in ("none", "segment", "all"):
        note(f"adjoint edge n={n} steps={steps} ckpt={ckpt} tapes={tapes}")
        info = {}
        res[tapes] = gpu_grad(pos, diam, target, steps, ckpt, tapes=tapes, info=info)
        if tapes == "none":
            assert info["taped_reverse_steps"] == 0, info
        elif info["worst_contacts"] <= 32:
            assert info["taped_reverse_steps"] == steps, info
        else:   # a step with more than 32 contacts per agent walks its grid
            assert 0 <= info["taped_reverse_steps"] < steps and info["tapes"] == 1, info
    for tapes in ("segment", "all"):
        for a, b in zip(res["none"], res[tapes]):
            np.testing.assert_array_equal(np.asarray(a), np.asarray(b))
    ref = oracle.adjoint(pos, diam, steps, oracle.Params(), target)
    loss, gx0, gp, _ = res["all"]
    assert abs(loss - ref["loss"]) <= 1e-12 * abs(ref["loss"])
    np.testing.assert_allclose(gp, [ref["dL_dk"], ref["dL_dgamma"]], rtol=1e-9, atol=1e-300)
    scale = max(np.abs(ref["dL_dx0"]).max(), 1e-300)
    assert np.abs(gx0 - ref["dL_dx0"]).max() <= 1e-9 * scale
