"""Pins of the oracle's reverse-mode step: central finite differences in
FP64, a forward-mode scalar recurrence for two spheres, and a dot-product
test of the transposed Jacobian."""
import math

import numpy as np

from paper_2301_06984_amd import workloads


def small_case(n=160, seed=51):
    g = np.random.default_rng(seed)
    side = (n / workloads.C1_DENSITY) ** (1 / 3)
    pos = g.uniform(0, side, size=(n, 3))
    diam = g.uniform(8, 12, size=n)
    target = pos + g.normal(0, 0.5, size=(n, 3))
    return pos, diam, target


def test_parameter_gradients_vs_fd(orc):
    pos, diam, target = small_case()
    steps = 6
    res = orc.adjoint(pos, diam, steps, orc.Params(), target)
    for name, key in (("k", "dL_dk"), ("gamma", "dL_dgamma")):
        base = getattr(orc.Params(), name)
        h = 1e-6 * base
        lp = orc.loss_only(pos, diam, steps, orc.Params(**{name: base + h}), target)
        lm = orc.loss_only(pos, diam, steps, orc.Params(**{name: base - h}), target)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - res[key]) <= 1e-6 * abs(fd) + 1e-12, (name, fd, res[key])
    assert abs(res["dL_dk"]) > 0 and abs(res["dL_dgamma"]) > 0


def test_position_gradients_vs_fd(orc):
    pos, diam, target = small_case(seed=52)
    steps = 5
    p = orc.Params()
    res = orc.adjoint(pos, diam, steps, p, target)
    g = np.random.default_rng(0)
    coords = g.choice(pos.size, size=32, replace=False)
    for c in coords:
        h = 1e-6
        pp = pos.copy().ravel(); pp[c] += h
        pm = pos.copy().ravel(); pm[c] -= h
        fd = (orc.loss_only(pp.reshape(-1, 3), diam, steps, p, target)
              - orc.loss_only(pm.reshape(-1, 3), diam, steps, p, target)) / (2 * h)
        an = res["dL_dx0"].ravel()[c]
        assert abs(fd - an) <= 1e-5 * abs(an) + 1e-9, (c, fd, an)
    v = g.normal(size=pos.shape)
    h = 1e-6
    fd = (orc.loss_only(pos + h * v, diam, steps, p, target)
          - orc.loss_only(pos - h * v, diam, steps, p, target)) / (2 * h)
    an = float(np.sum(res["dL_dx0"] * v))
    assert abs(fd - an) <= 1e-6 * abs(an) + 1e-9


def test_dot_product_single_step(orc):
    # L = <w, x_1> is reached with target = x_1 - w * 3n / 2; then dL/dx0 = J^T w.
    pos, diam, _ = small_case(n=120, seed=53)
    n = pos.shape[0]
    p = orc.Params()
    x1 = orc.run(pos, diam, 1, p).pos
    g = np.random.default_rng(1)
    w = g.normal(size=pos.shape)
    v = g.normal(size=pos.shape)
    res = orc.adjoint(pos, diam, 1, p, x1 - w * 1.5 * n)
    JTw = res["dL_dx0"]
    h = 1e-6
    Jv = (orc.run(pos + h * v, diam, 1, p).pos - orc.run(pos - h * v, diam, 1, p).pos) / (2 * h)
    lhs = float(np.sum(Jv * w))
    rhs = float(np.sum(v * JTw))
    assert abs(lhs - rhs) <= 1e-6 * abs(rhs)


def test_two_sphere_forward_mode(orc):
    # Two equal spheres on the x axis: the overlap follows
    # delta <- delta - 2 mu f(delta); propagate d(delta)/dk and d(delta)/dgamma
    # forward and compare with the reverse-mode gradients of
    # L = mean((x_T - x_0)^2) = (s_T - s_0)^2 / 12.
    r, s0, mu, k, gam, T = 5.0, 9.2, 0.1, 2.0, 1.0, 25
    rho = r * r / (2 * r)
    delta, dk, dg = 2 * r - s0, 0.0, 0.0
    for _ in range(T):
        sq = math.sqrt(rho * delta)
        f = k * delta - gam * sq
        fd = k - gam * rho / (2 * sq)
        dk, dg = dk * (1 - 2 * mu * fd) - 2 * mu * delta, dg * (1 - 2 * mu * fd) + 2 * mu * sq
        delta = delta - 2 * mu * f
    sT = 2 * r - delta
    dL_dk = (sT - s0) / 6 * (-dk)
    dL_dg = (sT - s0) / 6 * (-dg)
    pos = np.array([[0.0, 0.0, 0.0], [s0, 0.0, 0.0]])
    res = orc.adjoint(pos, np.array([2 * r, 2 * r]), T, orc.Params(), pos.copy())
    assert abs(res["posT"][1, 0] - res["posT"][0, 0] - sT) < 1e-12
    np.testing.assert_allclose(res["dL_dk"], dL_dk, rtol=1e-10)
    np.testing.assert_allclose(res["dL_dgamma"], dL_dg, rtol=1e-10)


def test_clamped_and_threshold_paths(orc):
    # strong overlaps with a small clamp, and a threshold that masks weak agents
    pos, diam, target = small_case(n=100, seed=54)
    p = orc.Params(mu=0.5, delta_max=0.4, f_adh=0.3)
    steps = 4
    res = orc.adjoint(pos, diam, steps, p, target)
    for name, key in (("k", "dL_dk"), ("gamma", "dL_dgamma")):
        base = getattr(p, name)
        h = 1e-7 * base
        kw = {f: getattr(p, f) for f in ("mu", "delta_max", "f_adh")}
        lp = orc.loss_only(pos, diam, steps, orc.Params(**{name: base + h}, **kw), target)
        lm = orc.loss_only(pos, diam, steps, orc.Params(**{name: base - h}, **kw), target)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - res[key]) <= 1e-5 * abs(fd) + 1e-11, (name, fd, res[key])
