"""Helpers shared by the GPU parity tests (not collected by pytest)."""
from __future__ import annotations

import sys

import numpy as np
import torch

import oracle
from paper_2301_06984_amd import abm


def note(msg: str):
    """Name the case on stdout before each GPU step, flushed."""
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def to_dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def make_sim(pos: np.ndarray, diam: np.ndarray, **kw) -> abm.Sim:
    return abm.Sim(to_dev(pos), to_dev(diam), **kw)


def oracle_params(**kw) -> oracle.Params:
    names = {f for f in oracle.Params.__dataclass_fields__}
    return oracle.Params(**{k: v for k, v in kw.items() if k in names})


def gpu_state(sim: abm.Sim):
    return dict(pos=sim.query("positions").cpu().numpy(), moved=sim.query("moved").cpu().numpy(),
                nnz=sim.query("nnz").cpu().numpy())


def assert_grid_equal(sim: abm.Sim, pos_before: np.ndarray, diam: np.ndarray, params: oracle.Params):
    """Keys, canonical order and box starts of the last GPU grid == oracle."""
    g = oracle.grid(pos_before, oracle.inv_cell(diam, params), order=params.order)
    ext = sim.query("extent").numpy()[0]
    np.testing.assert_array_equal(ext[:3], g["cmin"])
    np.testing.assert_array_equal(ext[3:6], g["dims"])
    assert ext[6] == g["nboxes"]
    key = sim.query("key").cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(key, g["key"])
    perm = sim.query("perm").cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(perm, g["perm"])
    cs = sim.query("cell_start").cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(cs, g["cell_start"])


def assert_neighbors_equal(sim: abm.Sim, pos_before: np.ndarray, diam: np.ndarray, params: oracle.Params):
    """N(i) of the last GPU grid == the oracle's, as sets of agent ids."""
    got = sim.query("neighbors").cpu().numpy().view(np.uint32)
    cnt = sim.query("neighbor_count").cpu().numpy().view(np.uint32)
    start, ids = oracle.neighbors(pos_before, oracle.radius(diam, params), oracle.inv_cell(diam, params))
    n = pos_before.shape[0]
    np.testing.assert_array_equal(cnt, np.diff(start).astype(np.uint32))
    exp = np.full_like(got, 0xFFFFFFFF)
    for i in range(n):
        row = np.sort(ids[start[i]:start[i + 1]])
        exp[i, :row.size] = row
    np.testing.assert_array_equal(got, exp)
