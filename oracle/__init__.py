"""CPU oracle of the agent step -- TEST INFRASTRUCTURE ONLY.

Thin ctypes wrapper over ``liboracle.so`` (built from ``abm_oracle.cpp``) plus
``oracle.brute`` (an O(N^2) numpy cross-check).  Only the tests, the smoke
check and the benchmark's CPU-baseline leg may import this package; the
product library never does.  See ``abm_oracle.cpp`` for the model and the
passages of the paper each part follows.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np

from . import build as _build

_lib = None


class _Params(C.Structure):
    _fields_ = [("k", C.c_double), ("gamma", C.c_double), ("mu", C.c_double), ("f_adh", C.c_double),
                ("delta_max", C.c_double), ("interaction_radius", C.c_double),
                ("cell_factor", C.c_double), ("detect_static", C.c_int32), ("nthreads", C.c_int32),
                ("order", C.c_int32)]


@dataclasses.dataclass
class Params:
    k: float = 2.0
    gamma: float = 1.0
    mu: float = 0.1
    f_adh: float = 0.0
    delta_max: float = 3.0
    interaction_radius: float = 0.0
    cell_factor: float = 1.0
    detect_static: bool = False
    nthreads: int = 0
    order: int = 0           # 0: Morton order of the boxes; 1: Hilbert order of the 2x2x2 super-boxes

    def c(self) -> _Params:
        return _Params(self.k, self.gamma, self.mu, self.f_adh, self.delta_max, self.interaction_radius,
                       self.cell_factor, int(bool(self.detect_static)), int(self.nthreads), int(self.order))


def lib():
    global _lib
    if _lib is None:
        path = _build.ensure_built()
        L = C.CDLL(path)
        P = C.c_void_p
        i64 = C.c_int64
        L.orc_gap_table.restype = i64
        L.orc_gap_table.argtypes = [C.c_int32, P, P, P, i64]
        L.orc_ranks.restype = i64
        L.orc_ranks.argtypes = [C.c_int32, P, i64, P, P, i64, P, P]
        L.orc_morton.restype = C.c_uint64
        L.orc_morton.argtypes = [C.c_int32, P, C.c_int32]
        L.orc_hilbert.restype = i64
        L.orc_hilbert.argtypes = [i64, P, C.c_int32, P]
        for suf in ("f64", "f32"):
            g = getattr(L, f"orc_grid_{suf}")
            g.restype = i64
            g.argtypes = [i64, P, C.c_double, P, P, P, P, P, i64, C.c_int32]
            nb = getattr(L, f"orc_neighbors_{suf}")
            nb.restype = i64
            nb.argtypes = [i64, P, C.c_double, C.c_double, P, P, i64]
            st = getattr(L, f"orc_step_{suf}")
            st.restype = C.c_int
            st.argtypes = [i64, P, P, P, P, P, i64, C.POINTER(_Params), P, P]
            sm = getattr(L, f"orc_sample_{suf}")
            sm.restype = C.c_int
            sm.argtypes = [i64, P, P, C.POINTER(_Params), i64, P, P, P, P]
            ad = getattr(L, f"orc_adjoint_{suf}")
            ad.restype = C.c_int
            ad.argtypes = [i64, P, P, C.c_int32, C.POINTER(_Params), P, P, P, P, P]
        L.orc_max_threads.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _suffix(pos):
    if pos.dtype == np.float64:
        return "f64"
    if pos.dtype == np.float32:
        return "f32"
    raise TypeError("positions must be float32 or float64")


def max_threads() -> int:
    return int(lib().orc_max_threads())


# ---------------------------------------------------------------- Section 4.2
def gap_table(dims, D: int = 3):
    """(box_counter, offset) entries of the step-D walk for a D-dim box."""
    d = np.ascontiguousarray(dims, dtype=np.int64)
    cap = 1024
    while True:
        bc = np.zeros(cap, np.int64)
        off = np.zeros(cap, np.int64)
        ne = lib().orc_gap_table(D, _ptr(d), _ptr(bc), _ptr(off), cap)
        if ne < 0:
            raise ValueError(f"orc_gap_table failed ({ne})")
        if ne <= cap:
            return bc[:ne].copy(), off[:ne].copy()
        cap = int(ne)


def ranks(dims, q, D: int = 3, rank_list=None):
    """Gap-free Morton rank of boxes q (n x D), and Morton codes of ranks."""
    d = np.ascontiguousarray(dims, dtype=np.int64)
    qq = np.ascontiguousarray(q, dtype=np.int64).reshape(-1, D)
    out = np.zeros(qq.shape[0], np.int64)
    rl = np.ascontiguousarray(rank_list if rank_list is not None else np.zeros(0), dtype=np.int64)
    codes = np.zeros(rl.shape[0], np.uint64)
    rc = lib().orc_ranks(D, _ptr(d), qq.shape[0], _ptr(qq), _ptr(out), rl.shape[0], _ptr(rl), _ptr(codes))
    if rc != 0:
        raise ValueError("orc_ranks failed")
    return out, codes


def morton(q, levels: int, D: int = 3) -> int:
    qq = np.ascontiguousarray(q, dtype=np.int64)
    return int(lib().orc_morton(D, _ptr(qq), levels))


# ---------------------------------------------------------------- Section 3.1
def radius(diam, params: Params) -> float:
    if params.interaction_radius > 0:
        return float(params.interaction_radius)
    return float(np.max(diam.astype(np.float64)))


def inv_cell(diam, params: Params) -> float:
    R = radius(diam, params)
    return 1.0 / (R * max(params.cell_factor, 1.0))


def hilbert(q, b: int):
    """Hilbert index (Skilling's transform) of points q (n x 3) below 2^b."""
    qq = np.ascontiguousarray(q, dtype=np.int64).reshape(-1, 3)
    out = np.zeros(qq.shape[0], np.uint64)
    if lib().orc_hilbert(qq.shape[0], _ptr(qq), int(b), _ptr(out)) != 0:
        raise ValueError("orc_hilbert failed")
    return out


def grid(pos, inv_h: float, order: int = 0):
    """Box keys, canonical order and box starts of the uniform grid (order 0:
    Morton order of the boxes; 1: Hilbert order of the 2x2x2 super-boxes,
    Morton order inside each)."""
    pos = np.ascontiguousarray(pos)
    n = pos.shape[0]
    cmin = np.zeros(3, np.int64)
    dims = np.zeros(3, np.int64)
    key = np.zeros(n, np.uint32)
    perm = np.zeros(n, np.uint32)
    fn = getattr(lib(), f"orc_grid_{_suffix(pos)}")
    nb = fn(n, _ptr(pos), float(inv_h), _ptr(cmin), _ptr(dims), _ptr(key), _ptr(perm), None, 0, int(order))
    if nb < 0:
        raise ValueError(f"orc_grid failed ({nb})")
    cs = np.zeros(nb + 1, np.uint32)
    nb2 = fn(n, _ptr(pos), float(inv_h), _ptr(cmin), _ptr(dims), None, None, _ptr(cs), nb + 1, int(order))
    assert nb2 == nb
    return dict(cmin=cmin, dims=dims, key=key, perm=perm, cell_start=cs, nboxes=int(nb))


def neighbors(pos, R: float, inv_h: float):
    """CSR (start[n+1], ids) of N(i) = {j != i : |x_i - x_j|^2 < R^2}."""
    pos = np.ascontiguousarray(pos)
    n = pos.shape[0]
    start = np.zeros(n + 1, np.int64)
    fn = getattr(lib(), f"orc_neighbors_{_suffix(pos)}")
    cap = max(16 * n, 1024)
    while True:
        nbr = np.zeros(cap, np.uint32)
        tot = fn(n, _ptr(pos), float(R), float(inv_h), _ptr(start), _ptr(nbr), cap)
        if tot < 0:
            raise ValueError(f"orc_neighbors failed ({tot})")
        if tot <= cap:
            return start, nbr[:tot].copy()
        cap = int(tot)


# ---------------------------------------------------------------- the step
@dataclasses.dataclass
class State:
    pos: np.ndarray          # (n, 3) float32/float64
    diam: np.ndarray         # (n,)
    moved: np.ndarray        # (n,) uint8
    nnz: np.ndarray          # (n,) int32
    force: np.ndarray        # (n, 3) float64
    t: int = 0

    @staticmethod
    def initial(pos, diam) -> "State":
        n = pos.shape[0]
        return State(np.array(pos, copy=True), np.array(diam, copy=True), np.ones(n, np.uint8),
                     np.zeros(n, np.int32), np.zeros((n, 3), np.float64), 0)

    def copy(self) -> "State":
        return State(self.pos.copy(), self.diam.copy(), self.moved.copy(), self.nnz.copy(),
                     self.force.copy(), self.t)


# ---------------------------------------------------------------- Section 3.2
def remove_agents(state: State, ids) -> State:
    """Remove the agents ``ids`` (distinct indices below n) the way Section
    3.2 keeps the agent vector dense: it shrinks to new_size = n - m, and an
    agent to be removed left of new_size leaves a hole, filled by an agent
    right of new_size that stays.  Reading of the pairing (the paper's figure
    is not in its text): the k-th hole in ascending index takes the k-th such
    agent in ascending index.  Every other agent keeps its index, which is its
    id.  Returns the new state."""
    n = state.pos.shape[0]
    ids = np.asarray(ids, dtype=np.int64).reshape(-1)
    m = ids.size
    if m and (ids.min() < 0 or ids.max() >= n or np.unique(ids).size != m):
        raise ValueError("ids must be distinct and below n")
    new_size = n - m
    removed = np.zeros(n, bool)
    removed[ids] = True
    holes = np.nonzero(removed[:new_size])[0]                 # left of new_size, ascending
    fillers = new_size + np.nonzero(~removed[new_size:])[0]   # right of new_size and kept, ascending
    assert holes.size == fillers.size
    src = np.arange(new_size)
    src[holes] = fillers                                      # new index j holds old agent src[j]
    return State(state.pos[src].copy(), state.diam[src].copy(), state.moved[src].copy(), state.nnz[src].copy(),
                 state.force[src].copy(), state.t)


def add_agents(state: State, pos, diam) -> State:
    """Append new agents (Section 3.2: additions grow the vectors), ids n, n+1,
    ...  A new agent has no history: it counts as moved, so no agent within
    R of it is static in the next step (condition (iii) of Section 5), and it
    has no non-zero pair term and no force yet."""
    pos = np.asarray(pos, dtype=state.pos.dtype).reshape(-1, 3)
    diam = np.asarray(diam, dtype=state.diam.dtype).reshape(-1)
    m = pos.shape[0]
    return State(np.concatenate([state.pos, pos]), np.concatenate([state.diam, diam]),
                 np.concatenate([state.moved, np.ones(m, np.uint8)]), np.concatenate([state.nnz, np.zeros(m, np.int32)]),
                 np.concatenate([state.force, np.zeros((m, 3), np.float64)]), state.t)


def set_diameters(state: State, ids, diam, radius: float = None) -> State:
    """Give the agents ``ids`` (distinct indices below n) the diameters
    ``diam`` between steps: growth, shrinking, or the mother's half of a
    division.  Condition (ii) of Section 5 forbids a static agent whose own
    or a neighbour's attributes changed in a way that could raise a pair
    force.  Under f = k*delta - gamma*sqrt(rho*delta) a smaller diameter can
    raise it too (a smaller overlap deepens the attraction), so every agent
    whose diameter changed counts as moved in the last step, which unsets
    it and each agent within R of it.  With ``radius`` given, a diameter
    above it is refused (it would let contacts escape the neighbour
    search).  Returns the new state."""
    ids = np.asarray(ids, dtype=np.int64).reshape(-1)
    n = state.pos.shape[0]
    m = ids.size
    new = np.asarray(diam, dtype=state.diam.dtype).reshape(-1)
    if new.size != m:
        raise ValueError("one diameter per id")
    if m and (ids.min() < 0 or ids.max() >= n or np.unique(ids).size != m):
        raise ValueError("ids must be distinct and below n")
    if m and not (np.all(np.isfinite(new)) and np.all(new > 0)):
        raise ValueError("diameters must be finite and positive")
    if m and radius is not None and np.any(new.astype(np.float64) > radius):
        raise ValueError("diameter above the interaction radius")
    d = state.diam.copy()
    moved = state.moved.copy()
    changed = d[ids] != new
    d[ids] = new
    moved[ids[changed]] = 1
    return State(state.pos.copy(), d, moved, state.nnz.copy(), state.force.copy(), state.t)


def step(state: State, params: Params, want_static: bool = False, want_disp: bool = False):
    """Advance ``state`` by one step in place; returns (static, disp) if asked."""
    n = state.pos.shape[0]
    st = np.zeros(n, np.uint8) if want_static else None
    disp = np.zeros((n, 3), np.float64) if want_disp else None
    fn = getattr(lib(), f"orc_step_{_suffix(state.pos)}")
    pc = params.c()
    rc = fn(n, _ptr(state.pos), _ptr(state.diam), _ptr(state.moved), _ptr(state.nnz), _ptr(state.force),
            int(state.t), C.byref(pc), _ptr(st), _ptr(disp))
    if rc != 0:
        raise ValueError(f"orc_step failed ({rc})")
    state.t += 1
    return st, disp


def sample_step(pos, diam, ids, params: Params):
    """First-step force, non-zero count and new position of the agents
    ``ids``, from the all-pairs definition (no grid)."""
    pos = np.ascontiguousarray(pos)
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    ns = ids.shape[0]
    F = np.zeros((ns, 3), np.float64)
    nnz = np.zeros(ns, np.int32)
    newp = np.zeros((ns, 3), pos.dtype)
    fn = getattr(lib(), f"orc_sample_{_suffix(pos)}")
    pc = params.c()
    rc = fn(pos.shape[0], _ptr(pos), _ptr(np.ascontiguousarray(diam)), C.byref(pc), ns, _ptr(ids), _ptr(F),
            _ptr(nnz), _ptr(newp))
    if rc != 0:
        raise ValueError(f"orc_sample failed ({rc})")
    return F, nnz, newp


def run(pos, diam, steps: int, params: Params) -> State:
    s = State.initial(pos, diam)
    for _ in range(steps):
        step(s, params)
    return s


def adjoint(pos0, diam, nsteps: int, params: Params, target):
    """Loss = mean((x_T - target)^2) and its gradients (reverse mode)."""
    pos0 = np.ascontiguousarray(pos0)
    n = pos0.shape[0]
    posT = np.zeros_like(pos0)
    loss = np.zeros(1, np.float64)
    gx = np.zeros((n, 3), np.float64)
    gp = np.zeros(2, np.float64)
    tgt = np.ascontiguousarray(target, dtype=np.float64)
    fn = getattr(lib(), f"orc_adjoint_{_suffix(pos0)}")
    pc = params.c()
    rc = fn(n, _ptr(pos0), _ptr(np.ascontiguousarray(diam)), int(nsteps), C.byref(pc), _ptr(tgt), _ptr(posT),
            _ptr(loss), _ptr(gx), _ptr(gp))
    if rc != 0:
        raise ValueError(f"orc_adjoint failed ({rc})")
    return dict(posT=posT, loss=float(loss[0]), dL_dx0=gx, dL_dk=float(gp[0]), dL_dgamma=float(gp[1]))


def loss_only(pos0, diam, nsteps: int, params: Params, target) -> float:
    s = run(pos0, diam, nsteps, params)
    r = s.pos.astype(np.float64) - target
    return float(np.mean(r * r))
