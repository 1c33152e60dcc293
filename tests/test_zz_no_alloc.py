"""abm_extent_of_noalloc (the grid extent with the library's own fixed
scratch, for callers that cannot allocate) against abm_extent_of (the same
kernels with a caller-owned scratch), through the C ABI: two calls in a row,
the second with a smaller input, then a refused input and a call after it."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2301_06984_amd import abm, workloads

pytestmark = pytest.mark.gpu


def _fields(e):
    return (e.radius, e.inv_cell, tuple(e.cmin), tuple(e.dims), e.nboxes)


def _noalloc(pos, diam, params):
    out = abm.abm_extent()
    rc = abm.lib().abm_extent_of_noalloc(pos.shape[0], pos.data_ptr(), diam.data_ptr(), C.byref(params),
                                         torch.cuda.current_stream().cuda_stream, C.byref(out))
    return rc, out


def test_noalloc_extent_matches_extent_of():
    dev = torch.device("cuda:0")
    # call 1: 10,000 spheres in FP64, default radius (the largest diameter)
    w1 = workloads.c1(n=10_000, seed=11)
    p1 = abm.default_params(precision="f64")
    pos1, d1 = torch.from_numpy(w1.pos).to(dev), torch.from_numpy(w1.diam).to(dev)
    print("[gpu] noalloc extent: call 1, 10000 agents f64", flush=True)
    rc, got1 = _noalloc(pos1, d1, p1)
    assert rc == abm.ABM_OK, abm.lib().abm_last_error().decode()
    ref1 = abm.extent_of(pos1, d1, p1)
    assert _fields(got1) == _fields(ref1)
    assert got1.radius == float(w1.diam.max())
    # call 2: a smaller input (3,000 spheres in FP32 at another place, a given
    # radius and a box edge factor): nothing of call 1 may survive in the scratch
    w2 = workloads.c2(n=3_000, seed=12)
    p2 = abm.default_params(precision="f32", interaction_radius=11.5, cell_factor=1.3)
    pos2 = torch.from_numpy(w2.pos * np.float32(0.25) - np.float32(40.0)).to(dev)
    d2 = torch.from_numpy(w2.diam).to(dev)
    print("[gpu] noalloc extent: call 2, 3000 agents f32", flush=True)
    rc, got2 = _noalloc(pos2, d2, p2)
    assert rc == abm.ABM_OK, abm.lib().abm_last_error().decode()
    ref2 = abm.extent_of(pos2, d2, p2)
    assert _fields(got2) == _fields(ref2)
    assert got2.radius == 11.5 and got2.cmin[0] < 0
    assert _fields(got2) != _fields(got1)
    # a non-finite diameter is refused; the next call is not affected by it
    bad = d2.clone()
    bad[17] = float("nan")
    print("[gpu] noalloc extent: non-finite diameter", flush=True)
    rc, _ = _noalloc(pos2, bad, p2)
    assert rc == abm.ABM_E_NONFINITE
    print("[gpu] noalloc extent: call after the refused one, 1000 agents", flush=True)
    rc, got3 = _noalloc(pos2[:1000], d2[:1000], p2)
    assert rc == abm.ABM_OK, abm.lib().abm_last_error().decode()
    assert _fields(got3) == _fields(abm.extent_of(pos2[:1000], d2[:1000], p2))
    # sizes: n must be in [1, ABM_NOALLOC_MAX_AGENTS]; refused before any work
    out = abm.abm_extent()
    for n in (0, -1, 2 ** 32 - 1):
        rc = abm.lib().abm_extent_of_noalloc(n, pos2.data_ptr(), d2.data_ptr(), C.byref(p2),
                                             torch.cuda.current_stream().cuda_stream, C.byref(out))
        assert rc == abm.ABM_E_INVAL
        assert "ABM_NOALLOC_MAX_AGENTS" in abm.lib().abm_last_error().decode()
