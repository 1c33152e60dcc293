"""Brute-force numpy cross-checks for the oracle -- TEST INFRASTRUCTURE ONLY.

Independent of ``abm_oracle.cpp``: all-pairs neighbour sets and forces, box
keys from the closed form floor(x / h) - min, and Morton ranks by sorting the
codes of every box in the space.  Meant for small inputs (N up to a few
thousand, boxes up to ~1e6).
"""
from __future__ import annotations

import numpy as np


def cells(pos, inv_h: float):
    """Integer box coordinates floor(x * inv_h), evaluated in float64."""
    return np.floor(pos.astype(np.float64) * inv_h).astype(np.int64)


def morton_codes(q, D: int = 3):
    """Bit interleave with the first coordinate in the lowest bit."""
    q = np.asarray(q, dtype=np.int64).reshape(-1, D)
    out = np.zeros(q.shape[0], dtype=np.uint64)
    for b in range(21):
        for a in range(D):
            out |= ((q[:, a] >> b) & 1).astype(np.uint64) << np.uint64(D * b + a)
    return out


def all_box_codes(dims, D: int = 3):
    axes = [np.arange(int(d)) for d in dims[:D]]
    mesh = np.meshgrid(*axes, indexing="ij")
    q = np.stack([m.ravel() for m in mesh], axis=1)
    return np.sort(morton_codes(q, D))


def ranks_by_sorting(dims, q, D: int = 3):
    codes = all_box_codes(dims, D)
    return np.searchsorted(codes, morton_codes(q, D)).astype(np.int64)


def keys(pos, inv_h: float):
    c = cells(pos, inv_h)
    cmin = c.min(axis=0)
    dims = c.max(axis=0) - cmin + 1
    q = c - cmin
    return ranks_by_sorting(dims, q), cmin, dims


def sq_dist(pos):
    """Pairwise ((ex^2 + ey^2) + ez^2) in float64 (numpy does not fuse)."""
    p = pos.astype(np.float64)
    ex = p[:, None, 0] - p[None, :, 0]
    ey = p[:, None, 1] - p[None, :, 1]
    ez = p[:, None, 2] - p[None, :, 2]
    return (ex * ex + ey * ey) + ez * ez, (ex, ey, ez)


def neighbor_sets(pos, R: float):
    s2, _ = sq_dist(pos)
    np.fill_diagonal(s2, np.inf)
    m = s2 < R * R
    return [np.flatnonzero(m[i]).astype(np.uint32) for i in range(pos.shape[0])]


def forces(pos, diam, k: float, gamma: float, R: float):
    """All-pairs force F_i and count of non-zero terms (any summation order)."""
    s2, (ex, ey, ez) = sq_dist(pos)
    n = pos.shape[0]
    r = 0.5 * diam.astype(np.float64)
    S = r[:, None] + r[None, :]
    contact = (s2 > 0) & (s2 < S * S) & (s2 < R * R)
    np.fill_diagonal(contact, False)
    dist = np.sqrt(np.where(contact, s2, 1.0))
    delta = np.where(contact, S - dist, 0.0)
    rho = (r[:, None] * r[None, :]) / S
    f = np.where(contact, k * delta - gamma * np.sqrt(rho * delta), 0.0)
    scale = f / dist
    F = np.stack([(scale * ex).sum(1), (scale * ey).sum(1), (scale * ez).sum(1)], axis=1)
    nnz = ((f != 0) & contact).sum(1).astype(np.int32)
    absum = np.abs(scale * np.sqrt(ex * ex + ey * ey + ez * ez)).sum(1)
    assert F.shape == (n, 3)
    return F, nnz, absum
