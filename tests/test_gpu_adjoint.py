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


def gpu_grad(pos, diam, target, steps, ckpt, **kw):
    sim = make_sim(pos, diam, **kw)
    sim.forward_record(steps, ckpt)
    xT = sim.query("positions").double()
    t = torch.from_numpy(target).cuda()
    n = pos.shape[0]
    loss = float(((xT - t) ** 2).mean())
    gx0, gp = sim.backward(2.0 * (xT - t) / (3 * n))
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

    # Central differences at h and h/4; their difference estimates the FD
    # truncation error (large near grazing contacts, where f'(delta) ~ delta^-1/2).
    for name, idx in (("k", 0), ("gamma", 1)):
        base = 2.0 if name == "k" else 1.0

        def fd_at(h):
            return (L(**{name: base + h}) - L(**{name: base - h})) / (2 * h)

        f1, f4 = fd_at(1e-6 * base), fd_at(0.25e-6 * base)
        tol = 1e-7 * abs(f4) + 2.0 * abs(f1 - f4) + 1e-10
        assert abs(f4 - gp[idx]) <= tol, (name, f1, f4, gp[idx])
    g = np.random.default_rng(3)
    for c in g.choice(pos.size, 16, replace=False):
        def fd_x(h):
            pp = pos.copy().ravel(); pp[c] += h
            pm = pos.copy().ravel(); pm[c] -= h
            return (L(pp.reshape(-1, 3)) - L(pm.reshape(-1, 3))) / (2 * h)

        f1, f4 = fd_x(1e-6), fd_x(0.25e-6)
        an = gx0.ravel()[c]
        assert abs(f4 - an) <= 1e-6 * abs(an) + 2.0 * abs(f1 - f4) + 1e-9, (c, f1, f4, an)


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
