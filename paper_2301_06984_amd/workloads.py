"""Seeded synthetic workloads for the agent step.

This module only draws inputs (positions, diameters, targets).  It holds none
of the method's arithmetic, so both the CPU oracle tests and the GPU path can
consume exactly the same arrays.  Every draw goes through
``numpy.random.Generator(PCG64(seed))``; values are produced in float64 and
cast once to float32 for the single-precision workloads.

The paper's benchmark models (Table 1 of the evaluation, and the cell-sorting
model of the Biocellion comparison) are not available; these generators stand
in for them with the structural features the paper names: random versus
lattice initialisation, regions that do not move (static regions, Section 5)
and agent counts from 1e3 to 5e7.

Workloads
---------
``c1``        10,000 spheres, FP64, uniform in a 0-215 cube, d ~ U[8, 12].
``c2``        1e6 spheres, FP32, density chosen for ~12 candidates in the 27-box
              stencil (cell edge 12): a uniform inner cube holding half of the
              agents, and a jittered, overlap-free lattice in the outer shell
              (the other half) whose agents are force-free, hence static.
``headline``  the c2 construction at 1e7 spheres.
``c3``        5e7 spheres, FP32, 1000 Gaussian blobs (sigma 40) in a 20,000 cube,
              lognormal diameters (mean 10, sd 1.5).
``c4``        512 independent simulations, agent counts log-uniform in
              [1e3, 2e5], uniform cubes at volume fraction U[0.3, 0.6].
``c5``        1e5 spheres, FP32, uniform cube at c1's density, plus a seeded
              target for a mean-squared-error loss on final positions.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

# Density of the c2 construction: 12 candidates in the 27 boxes of edge 12.
C2_DENSITY = 12.0 / (27.0 * 12.0 ** 3)
# Density of c1: 1e4 agents in a 215^3 cube.
C1_DENSITY = 1.0e4 / 215.0 ** 3


def rng_for(seed) -> np.random.Generator:
    """PCG64 generator; ``seed`` may be an int or a tuple of ints."""
    if isinstance(seed, (tuple, list)):
        return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(seed))))
    return np.random.Generator(np.random.PCG64(seed))


@dataclasses.dataclass
class Workload:
    name: str
    pos: np.ndarray            # (n, 3) row-major, float32 or float64
    diam: np.ndarray           # (n,), same dtype as pos
    steps: int
    detect_static: bool = False
    sort_every: int = 1
    target: Optional[np.ndarray] = None   # c5 only, float64 (n, 3)
    offsets: Optional[np.ndarray] = None  # c4 only, int64 (nsims + 1,)
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    @property
    def precision(self) -> str:
        return "f64" if self.pos.dtype == np.float64 else "f32"


def _cast(pos, diam, dtype):
    return np.ascontiguousarray(pos, dtype=dtype), np.ascontiguousarray(diam, dtype=dtype)


def uniform_cube(n: int, side: float, seed, dmin=8.0, dmax=12.0, dtype=np.float64):
    """n positions U[0, side)^3 and diameters U[dmin, dmax]."""
    g = rng_for(seed)
    pos = g.uniform(0.0, side, size=(n, 3))
    diam = g.uniform(dmin, dmax, size=n)
    return _cast(pos, diam, dtype)


def c1(n: int = 10_000, seed: int = 1, side: Optional[float] = None, steps: int = 10) -> Workload:
    if side is None:
        side = (n / C1_DENSITY) ** (1.0 / 3.0)
    pos, diam = uniform_cube(n, side, seed, dtype=np.float64)
    return Workload("c1", pos, diam, steps=steps, detect_static=False,
                    meta=dict(side=side, seed=seed))


def _shell_lattice(g: np.random.Generator, side: float, inner_lo: float, inner_hi: float,
                   count: int, spacing: float, jitter: float):
    """Exactly ``count`` sites of a cubic lattice in [0, side)^3 outside the
    inner cube [inner_lo, inner_hi)^3, chosen at random, with uniform jitter."""
    # Shrink the spacing in 1% steps while too few sites fit; sites stay more
    # than 12 (the largest diameter) apart, so the shell has no contacts.
    s = spacing
    while True:
        m = int(math.floor(side / s))
        ax = (np.arange(m) + 0.5) * s
        inside_axis = (ax >= inner_lo) & (ax < inner_hi)
        n_inner = int(inside_axis.sum()) ** 3
        if m ** 3 - n_inner >= count:
            break
        s *= 0.99
        if s <= 12.05:
            raise ValueError("shell lattice too small for the requested agent count")
        jitter = min(jitter, 0.5 * (s - 12.05))
    # enumerate shell sites without materialising interior ones twice
    ix, iy, iz = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    ix, iy, iz = ix.ravel(), iy.ravel(), iz.ravel()
    shell = ~(inside_axis[ix] & inside_axis[iy] & inside_axis[iz])
    sites = np.flatnonzero(shell)
    chosen = g.choice(sites, size=count, replace=False)
    chosen.sort()
    pts = np.stack([ax[ix[chosen]], ax[iy[chosen]], ax[iz[chosen]]], axis=1)
    pts += g.uniform(-jitter, jitter, size=pts.shape)
    return pts, s


def c2_construction(n: int, seed: int, density: float = C2_DENSITY, jitter: float = 1.8):
    """Uniform inner cube (half of the agents) + jittered lattice shell."""
    g = rng_for(seed)
    side = (n / density) ** (1.0 / 3.0)
    inner = side * 2.0 ** (-1.0 / 3.0)
    lo = 0.5 * (side - inner)
    hi = lo + inner
    n_in = n // 2
    n_out = n - n_in
    p_in = g.uniform(lo, hi, size=(n_in, 3))
    p_out, spacing = _shell_lattice(g, side, lo, hi, n_out, density ** (-1.0 / 3.0), jitter)
    pos = np.concatenate([p_in, p_out], axis=0)
    diam = g.uniform(8.0, 12.0, size=n)
    order = g.permutation(n)          # ids carry no spatial information
    pos = pos[order]
    diam = diam[order]
    meta = dict(side=side, inner_lo=lo, inner_hi=hi, lattice_spacing=spacing, seed=seed)
    return pos, diam, meta


def c2(n: int = 1_000_000, seed: int = 2, steps: int = 100, detect_static: bool = True) -> Workload:
    pos, diam, meta = c2_construction(n, seed)
    pos, diam = _cast(pos, diam, np.float32)
    return Workload("c2", pos, diam, steps=steps, detect_static=detect_static, meta=meta)


def headline(n: int = 10_000_000, seed: int = 2, steps: int = 100,
             detect_static: bool = False, dtype=np.float32) -> Workload:
    """The c2 construction scaled to 1e7 agents (cube side ~3387.7)."""
    pos, diam, meta = c2_construction(n, seed)
    pos, diam = _cast(pos, diam, dtype)
    return Workload("headline", pos, diam, steps=steps, detect_static=detect_static, meta=meta)


def lognormal_params(mean: float, sd: float):
    s2 = math.log(1.0 + (sd / mean) ** 2)
    return math.log(mean) - 0.5 * s2, math.sqrt(s2)


def c3(n_blobs: int = 1000, per_blob: int = 50_000, box: float = 20_000.0, sigma: float = 40.0,
       seed: int = 3, steps: int = 20, margin: float = 160.0) -> Workload:
    g = rng_for(seed)
    centres = g.uniform(margin, box - margin, size=(n_blobs, 3))
    n = n_blobs * per_blob
    pos = np.repeat(centres, per_blob, axis=0) + g.normal(0.0, sigma, size=(n, 3))
    mu_ln, s_ln = lognormal_params(10.0, 1.5)
    diam = g.lognormal(mu_ln, s_ln, size=n)
    pos, diam = _cast(pos, diam, np.float32)
    return Workload("c3", pos, diam, steps=steps, detect_static=False, sort_every=10,
                    meta=dict(box=box, sigma=sigma, n_blobs=n_blobs, seed=seed))


def c4(nsims: int = 512, nmin: float = 1e3, nmax: float = 2e5, seed: int = 4, steps: int = 50,
       phi_lo: float = 0.3, phi_hi: float = 0.6) -> Workload:
    """Concatenated independent simulations; sim s draws from seed (seed, s)."""
    pos_l, diam_l, sizes, sides, phis = [], [], [], [], []
    for s in range(nsims):
        g = rng_for((seed, s))
        ns = int(round(math.exp(g.uniform(math.log(nmin), math.log(nmax)))))
        phi = g.uniform(phi_lo, phi_hi)
        d = g.uniform(8.0, 12.0, size=ns)
        side = (float(np.sum(math.pi / 6.0 * d ** 3)) / phi) ** (1.0 / 3.0)
        p = g.uniform(0.0, side, size=(ns, 3))
        pos_l.append(p)
        diam_l.append(d)
        sizes.append(ns)
        sides.append(side)
        phis.append(phi)
    offsets = np.zeros(nsims + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    pos, diam = _cast(np.concatenate(pos_l), np.concatenate(diam_l), np.float32)
    return Workload("c4", pos, diam, steps=steps, offsets=offsets,
                    meta=dict(sides=sides, phis=phis, seed=seed))


def c5(n: int = 100_000, seed: int = 5, steps: int = 50, dtype=np.float32,
       target_sd: float = 0.5) -> Workload:
    g = rng_for(seed)
    side = (n / C1_DENSITY) ** (1.0 / 3.0)
    pos = g.uniform(0.0, side, size=(n, 3))
    diam = g.uniform(8.0, 12.0, size=n)
    target = pos + g.normal(0.0, target_sd, size=(n, 3))
    pos, diam = _cast(pos, diam, dtype)
    return Workload("c5", pos, diam, steps=steps, target=target,
                    meta=dict(side=side, seed=seed, ckpt_every=10))


def lattice(m: int, spacing: float, diam: float = 10.0, dtype=np.float64, origin: float = 0.0):
    """m^3 agents on a cubic lattice (used for constructed static-skip cases)."""
    ax = origin + np.arange(m) * spacing
    x, y, z = np.meshgrid(ax, ax, ax, indexing="ij")
    pos = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    d = np.full(pos.shape[0], diam)
    return _cast(pos, d, dtype)
