"""Python binding of libabm (the C ABI declared in include/abm.h).

Argument marshalling only: every step of the path runs in the HIP kernels of
libabm.so.  PyTorch provides device memory and the stream.  The library must
be built (``python -m paper_2301_06984_amd.build``); importing this module on
a machine without it raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libabm.so")

ABM_OK, ABM_E_INVAL, ABM_E_NONFINITE, ABM_E_GRID, ABM_E_WORKSPACE, ABM_E_HIP, ABM_E_STATE, ABM_E_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6, -7
ABM_F32, ABM_F64 = 0, 1
ABM_ORDER_MORTON, ABM_ORDER_HILBERT = 0, 1
ABI_VERSION = 6   # the layout of the structs below
FIELD = dict(positions=0, forces=1, moved=2, static=3, nnz=4, key=5, perm=6, cell_start=7, extent=8,
             storage_ids=9, neighbor_count=10, neighbors=11, diameters=12)
EXTENT_SCRATCH_BYTES = 1024

# every symbol include/abm.h declares
EXPORTS = ["abm_abi_version", "abm_default_params", "abm_last_error", "abm_extent_of", "abm_workspace_bytes",
           "abm_init", "abm_init_batched", "abm_set_params", "abm_step", "abm_sync", "abm_query",
           "abm_get_stats", "abm_state_bytes", "abm_export_state", "abm_import_state", "abm_graph_capture",
           "abm_graph_launch", "abm_record_bytes", "abm_forward_record", "abm_backward", "abm_set_timing",
           "abm_get_timing", "abm_destroy", "abm_workspace_bytes_capacity", "abm_init_capacity", "abm_add_agents",
           "abm_remove_agents", "abm_set_diameters", "abm_population", "abm_extent_of_noalloc", "abm_record_sizes",
           "abm_record_info"]
TIMED_PHASES = ["setup", "keys", "scan", "scatter", "fixup", "force"]


class abm_params(C.Structure):
    _fields_ = [("k", C.c_double), ("gamma", C.c_double), ("mu", C.c_double), ("f_adh", C.c_double),
                ("delta_max", C.c_double), ("interaction_radius", C.c_double), ("cell_factor", C.c_double),
                ("precision", C.c_int32), ("detect_static", C.c_int32), ("sort_every", C.c_int32),
                ("block_size", C.c_int32), ("keep_forces", C.c_int32), ("walk_chunk", C.c_int32),
                ("order", C.c_int32), ("share_terms", C.c_int32), ("super_fraction", C.c_double)]


class abm_extent(C.Structure):
    _fields_ = [("radius", C.c_double), ("inv_cell", C.c_double), ("cmin", C.c_int64 * 3),
                ("dims", C.c_int64 * 3), ("nboxes", C.c_int64)]


class abm_stats(C.Structure):
    _fields_ = [("step", C.c_int64), ("n_static", C.c_int64), ("n_moved", C.c_int64), ("error", C.c_uint32),
                ("build", C.c_uint32), ("sum_force", C.c_double * 3), ("max_displacement", C.c_double),
                ("skip_fraction", C.c_double)]


class abm_timing(C.Structure):
    _fields_ = [("steps", C.c_int64), ("ms", C.c_double * 8)]


class ABMError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where} failed ({code}): {msg}")
        self.code = code


_lib = None


def lib():
    """Load libabm.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2301_06984_amd.build`")
        L = C.CDLL(LIB_PATH)
        P, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
        sig = {
            "abm_abi_version": (C.c_int, []),
            "abm_default_params": (None, [C.POINTER(abm_params)]),
            "abm_last_error": (C.c_char_p, []),
            "abm_extent_of": (C.c_int, [i64, P, P, C.POINTER(abm_params), P, P, C.POINTER(abm_extent)]),
            "abm_extent_of_noalloc": (C.c_int, [i64, P, P, C.POINTER(abm_params), P, C.POINTER(abm_extent)]),
            "abm_workspace_bytes": (C.c_int, [i32, P, P, C.POINTER(abm_params), C.POINTER(i64)]),
            "abm_init": (C.c_int, [C.POINTER(P), i64, P, P, C.POINTER(abm_params), i64, P, i64, P]),
            "abm_init_batched": (C.c_int, [C.POINTER(P), i32, P, P, P, P, P, P, i64, P]),
            "abm_set_params": (C.c_int, [P, C.POINTER(abm_params)]),
            "abm_step": (C.c_int, [P, i32]),
            "abm_sync": (C.c_int, [P]),
            "abm_query": (C.c_int, [P, i32, P, i64, i32]),
            "abm_get_stats": (C.c_int, [P, C.POINTER(abm_stats)]),
            "abm_state_bytes": (C.c_int, [P, C.POINTER(i64)]),
            "abm_export_state": (C.c_int, [P, P, i64]),
            "abm_import_state": (C.c_int, [P, P, i64]),
            "abm_graph_capture": (C.c_int, [P, i32]),
            "abm_graph_launch": (C.c_int, [P]),
            "abm_record_bytes": (C.c_int, [P, i32, i32, C.POINTER(i64)]),
            "abm_record_sizes": (C.c_int, [P, i32, i32, P]),
            "abm_record_info": (C.c_int, [P, P]),
            "abm_forward_record": (C.c_int, [P, i32, i32, P, i64]),
            "abm_backward": (C.c_int, [P, P, P, P]),
            "abm_set_timing": (C.c_int, [P, i32]),
            "abm_get_timing": (C.c_int, [P, C.POINTER(abm_timing)]),
            "abm_destroy": (None, [P]),
            "abm_workspace_bytes_capacity": (C.c_int, [i64, i64, C.POINTER(abm_params), C.POINTER(i64)]),
            "abm_init_capacity": (C.c_int, [C.POINTER(P), i64, i64, P, P, C.POINTER(abm_params), i64, P, i64, P]),
            "abm_add_agents": (C.c_int, [P, i64, P, P]),
            "abm_remove_agents": (C.c_int, [P, i64, P]),
            "abm_set_diameters": (C.c_int, [P, i64, P, P]),
            "abm_population": (C.c_int, [P, C.POINTER(i64), C.POINTER(i64)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        if L.abm_abi_version() != ABI_VERSION:
            raise RuntimeError(f"{LIB_PATH} has ABI {L.abm_abi_version()}, this binding {ABI_VERSION}: rebuild it")
        _lib = L
    return _lib


def _check(code: int, where: str):
    if code != ABM_OK:
        raise ABMError(code, where, lib().abm_last_error().decode())


def default_params(**kw) -> abm_params:
    p = abm_params()
    lib().abm_default_params(C.byref(p))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = ABM_F64 if v in ("f64", "float64", "double") else ABM_F32
        if k == "order" and isinstance(v, str):
            v = {"morton": ABM_ORDER_MORTON, "hilbert": ABM_ORDER_HILBERT}[v]
        if isinstance(v, bool):
            v = int(v)
        setattr(p, k, v)
    return p


def _stream_handle(stream: Optional[torch.cuda.Stream]) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dtype_of(p: abm_params):
    return torch.float64 if p.precision == ABM_F64 else torch.float32


def _ptr(t: torch.Tensor) -> int:
    return int(t.data_ptr())


def extent_of(pos: torch.Tensor, diam: torch.Tensor, params: abm_params, stream=None) -> abm_extent:
    """Grid extent of positions on the device (abm_extent_of)."""
    scratch = torch.empty(EXTENT_SCRATCH_BYTES, dtype=torch.uint8, device=pos.device)
    out = abm_extent()
    _check(lib().abm_extent_of(pos.shape[0], _ptr(pos), _ptr(diam), C.byref(params), _ptr(scratch),
                               _stream_handle(stream), C.byref(out)), "abm_extent_of")
    return out


def extent_of_noalloc(pos: torch.Tensor, diam: torch.Tensor, params: abm_params, stream=None) -> abm_extent:
    """Grid extent without a scratch tensor (abm_extent_of_noalloc: the
    library's own fixed device scratch)."""
    out = abm_extent()
    _check(lib().abm_extent_of_noalloc(pos.shape[0], _ptr(pos), _ptr(diam), C.byref(params),
                                       _stream_handle(stream), C.byref(out)), "abm_extent_of_noalloc")
    return out


def box_capacity_for(nboxes: int, slack: float) -> int:
    return int(min(nboxes * slack + 4096, 2 ** 32 - 2))


def grown_supers(ext: "abm_extent", grow: int = 3) -> int:
    """Super-boxes (aligned 2x2x2 blocks of boxes) of the grid ``ext`` grown
    by ``grow`` boxes along each axis: room for extents that change by a box
    or two as agents move (one more box on an even axis adds a block)."""
    supers = 1
    for a in range(3):
        supers *= (int(ext.dims[a]) + grow + 1) // 2
    return supers


def super_fraction_for(ext: "abm_extent", box_capacity: int, slack: float) -> float:
    """abm_params.super_fraction for a super-box table of about ``slack``
    times the super-boxes of the grid ``ext`` grown by three boxes per axis."""
    return min(1.0, max(slack * grown_supers(ext) - 64.0, 1.0) / box_capacity)


class Sim:
    """One simulation: ``Sim(pos, diam, **params)`` with device tensors
    (n x 3 and n, float32 or float64 per ``precision``)."""

    def __init__(self, pos: torch.Tensor, diam: torch.Tensor, *, box_slack: float = 1.5,
                 box_capacity: Optional[int] = None, capacity: Optional[int] = None,
                 super_slack: Optional[float] = None, stream: Optional[torch.cuda.Stream] = None, **params):
        """super_slack: size the super-box table for ``super_slack`` times the
        super-boxes of the initial grid grown by three boxes per axis
        (abm_params.super_fraction) instead of for any grid of the box
        capacity."""
        if "precision" not in params:
            params["precision"] = "f64" if pos.dtype == torch.float64 else "f32"
        self.params = default_params(**params)
        dt = _dtype_of(self.params)
        if pos.dtype != dt or diam.dtype != dt or not pos.is_cuda or not diam.is_cuda:
            raise TypeError(f"pos and diam must be CUDA tensors of {dt}")
        self.pos_in = pos.contiguous()
        self.diam_in = diam.contiguous()
        self.n = int(pos.shape[0])
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        ext = extent_of(self.pos_in, self.diam_in, self.params, self.stream)
        self.extent0 = ext
        self.box_capacity = int(box_capacity) if box_capacity else box_capacity_for(ext.nboxes, box_slack)
        if super_slack is not None:
            self.params.super_fraction = super_fraction_for(ext, self.box_capacity, float(super_slack))
        nbytes = C.c_int64()
        self.ctx = C.c_void_p()
        if capacity is None:
            offs = (C.c_int64 * 2)(0, self.n)
            caps = (C.c_int64 * 1)(self.box_capacity)
            _check(lib().abm_workspace_bytes(1, offs, caps, C.byref(self.params), C.byref(nbytes)),
                   "abm_workspace_bytes")
            self.ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=pos.device)
            _check(lib().abm_init(C.byref(self.ctx), self.n, _ptr(self.pos_in), _ptr(self.diam_in),
                                  C.byref(self.params), self.box_capacity, _ptr(self.ws), self.ws.numel(),
                                  int(self.stream.cuda_stream)), "abm_init")
        else:
            _check(lib().abm_workspace_bytes_capacity(int(capacity), self.box_capacity, C.byref(self.params),
                                                      C.byref(nbytes)), "abm_workspace_bytes_capacity")
            self.ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=pos.device)
            _check(lib().abm_init_capacity(C.byref(self.ctx), self.n, int(capacity), _ptr(self.pos_in),
                                           _ptr(self.diam_in), C.byref(self.params), self.box_capacity,
                                           _ptr(self.ws), self.ws.numel(), int(self.stream.cuda_stream)),
                   "abm_init_capacity")

    # ---------------------------------------------------------------- population
    def add_agents(self, pos: torch.Tensor, diam: torch.Tensor):
        """Append agents (ids n, n+1, ...); needs a context made with ``capacity``."""
        dt = _dtype_of(self.params)
        pos = pos.to(dtype=dt).contiguous()
        diam = diam.to(dtype=dt).contiguous()
        if not pos.is_cuda or not diam.is_cuda or pos.shape[0] != diam.shape[0]:
            raise TypeError("pos (m x 3) and diam (m) must be CUDA tensors")
        _check(lib().abm_add_agents(self.ctx, int(pos.shape[0]), _ptr(pos), _ptr(diam)), "abm_add_agents")
        self.n = self.population()[0]

    def remove_agents(self, ids: torch.Tensor):
        """Remove agents by id; ids stay dense (see abm_remove_agents)."""
        ids = ids.to(dtype=torch.int64).contiguous()
        if not ids.is_cuda:
            raise TypeError("ids must be a CUDA tensor")
        _check(lib().abm_remove_agents(self.ctx, int(ids.numel()), _ptr(ids)), "abm_remove_agents")
        self.n = self.population()[0]

    def set_diameters(self, ids: torch.Tensor, diam: torch.Tensor):
        """New diameters for agents by id; a changed agent counts as moved (see abm_set_diameters)."""
        ids = ids.to(dtype=torch.int64).contiguous()
        diam = diam.to(dtype=_dtype_of(self.params)).contiguous()
        if not ids.is_cuda or not diam.is_cuda or ids.numel() != diam.numel():
            raise TypeError("ids and diam must be CUDA tensors of one value per id")
        _check(lib().abm_set_diameters(self.ctx, int(ids.numel()), _ptr(ids), _ptr(diam)), "abm_set_diameters")

    def population(self):
        n, cap = C.c_int64(), C.c_int64()
        _check(lib().abm_population(self.ctx, C.byref(n), C.byref(cap)), "abm_population")
        return int(n.value), int(cap.value)

    # ---------------------------------------------------------------- stepping
    def step(self, nsteps: int = 1):
        _check(lib().abm_step(self.ctx, int(nsteps)), "abm_step")

    def sync(self):
        _check(lib().abm_sync(self.ctx), "abm_sync")

    def set_params(self, **kw):
        p = abm_params.from_buffer_copy(self.params)
        for k, v in kw.items():
            setattr(p, k, int(v) if isinstance(v, bool) else v)
        _check(lib().abm_set_params(self.ctx, C.byref(p)), "abm_set_params")
        self.params = p

    def set_timing(self, enable=True):
        """True (or 1): events around every kernel of each step; 2: around
        the force kernel only; False (0): off."""
        mode = 2 if (not isinstance(enable, bool) and enable == 2) else int(bool(enable))
        _check(lib().abm_set_timing(self.ctx, mode), "abm_set_timing")

    def timing(self) -> dict:
        """Accumulated per-kernel times (ms) of the timed steps."""
        t = abm_timing()
        _check(lib().abm_get_timing(self.ctx, C.byref(t)), "abm_get_timing")
        out = {name: t.ms[k] for k, name in enumerate(TIMED_PHASES)}
        out["steps"] = t.steps
        return out

    def graph_capture(self, nsteps: int):
        _check(lib().abm_graph_capture(self.ctx, int(nsteps)), "abm_graph_capture")

    def graph_launch(self):
        _check(lib().abm_graph_launch(self.ctx), "abm_graph_launch")

    # ---------------------------------------------------------------- queries
    def query(self, field: str) -> torch.Tensor:
        dev = self.ws.device
        n = self.n
        if field == "positions":
            out = torch.empty((n, 3), dtype=_dtype_of(self.params), device=dev)
        elif field == "diameters":
            out = torch.empty(n, dtype=_dtype_of(self.params), device=dev)
        elif field == "forces":
            out = torch.empty((n, 3), dtype=torch.float64, device=dev)
        elif field in ("moved", "static"):
            out = torch.empty(n, dtype=torch.uint8, device=dev)
        elif field == "nnz":
            out = torch.empty(n, dtype=torch.int32, device=dev)
        elif field in ("key", "perm", "storage_ids", "neighbor_count"):
            out = torch.empty(n, dtype=torch.int32, device=dev)
        elif field == "neighbors":
            width = max(1, int(self.query("neighbor_count").max().item()))
            out = torch.empty((n, width), dtype=torch.int32, device=dev)
        elif field == "cell_start":
            nb = int(self.query("extent")[:, 6].sum())
            out = torch.empty(nb + 1, dtype=torch.int32, device=dev)
        elif field == "extent":
            out = torch.empty((self.nsims, 7), dtype=torch.int64)
            _check(lib().abm_query(self.ctx, FIELD[field], out.data_ptr(), out.numel() * 8, 0), "abm_query")
            return out
        else:
            raise ValueError(field)
        _check(lib().abm_query(self.ctx, FIELD[field], _ptr(out), out.numel() * out.element_size(), 1), "abm_query")
        if field in ("key", "perm", "storage_ids", "cell_start"):
            out = out.view(torch.int32)
        return out

    @property
    def nsims(self) -> int:
        return 1

    def positions(self) -> torch.Tensor:
        return self.query("positions")

    def stats(self) -> dict:
        s = abm_stats()
        _check(lib().abm_get_stats(self.ctx, C.byref(s)), "abm_get_stats")
        return dict(step=s.step, n_static=s.n_static, n_moved=s.n_moved, error=s.error,
                    sum_force=tuple(s.sum_force), max_displacement=s.max_displacement,
                    skip_fraction=s.skip_fraction, update_build=bool(s.build & 1), rebuilt_sims=s.build >> 1)

    # ---------------------------------------------------------------- checkpoint
    def export_state(self) -> bytes:
        nb = C.c_int64()
        _check(lib().abm_state_bytes(self.ctx, C.byref(nb)), "abm_state_bytes")
        buf = (C.c_char * nb.value)()
        _check(lib().abm_export_state(self.ctx, buf, nb.value), "abm_export_state")
        return bytes(buf)

    def import_state(self, blob: bytes):
        buf = (C.c_char * len(blob)).from_buffer_copy(blob)
        _check(lib().abm_import_state(self.ctx, buf, len(blob)), "abm_import_state")

    # ---------------------------------------------------------------- adjoint
    def record_sizes(self, nsteps: int, ckpt_every: int) -> dict:
        """Bytes of a record without contact tapes, with one segment's, with every step's."""
        sz = (C.c_int64 * 3)()
        _check(lib().abm_record_sizes(self.ctx, int(nsteps), int(ckpt_every), sz), "abm_record_sizes")
        return dict(none=int(sz[0]), segment=int(sz[1]), all=int(sz[2]))

    def forward_record(self, nsteps: int, ckpt_every: int, tapes: str = "auto"):
        """Record nsteps steps for backward().  tapes: "all" (every step's
        contacts kept: the backward recomputes nothing), "segment" (taped while
        each segment is recomputed), "none" (the reverse steps walk a grid), or
        "auto": the largest that takes at most half the free device memory."""
        sizes = self.record_sizes(nsteps, ckpt_every)
        if tapes == "auto":
            free = torch.cuda.mem_get_info(self.ws.device)[0]
            tapes = next((k for k in ("all", "segment") if sizes[k] <= free // 2), "none")
        if tapes not in sizes:
            raise ValueError(f"tapes must be auto, all, segment or none, not {tapes!r}")
        self.rec = torch.empty(sizes[tapes], dtype=torch.uint8, device=self.ws.device)
        _check(lib().abm_forward_record(self.ctx, int(nsteps), int(ckpt_every), _ptr(self.rec), self.rec.numel()),
               "abm_forward_record")

    def record_info(self) -> dict:
        """The record's tapes (-1 no record, 0 none, 1 per segment, 2 every
        step), the reverse steps of the last backward that read a tape, and the
        largest contact count a tape saw."""
        info = (C.c_int32 * 3)()
        _check(lib().abm_record_info(self.ctx, info), "abm_record_info")
        return dict(tapes=int(info[0]), taped_reverse_steps=int(info[1]), worst_contacts=int(info[2]))

    def backward(self, dL_dxT: torch.Tensor):
        g = dL_dxT.to(torch.float64).contiguous()
        gx0 = torch.empty_like(g)
        gp = torch.zeros(2, dtype=torch.float64, device=g.device)
        _check(lib().abm_backward(self.ctx, _ptr(g), _ptr(gx0), _ptr(gp)), "abm_backward")
        return gx0, gp

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            lib().abm_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchedSim(Sim):
    """Many independent simulations in one context: ``BatchedSim(pos, diam,
    offsets, params=[dict, ...])``; simulation s owns agents
    offsets[s]:offsets[s+1]."""

    def __init__(self, pos: torch.Tensor, diam: torch.Tensor, offsets: Sequence[int],
                 params: Optional[Sequence[dict]] = None, *, box_slack: float = 1.5,
                 super_slack: Optional[float] = 1.2, stream: Optional[torch.cuda.Stream] = None,
                 common: Optional[dict] = None):
        """Each simulation owns a fixed range of the super-box table, which the
        grid build scans every step: with super_slack (default 1.2) a range
        holds at least super_slack times the super-boxes of the simulation's
        initial grid grown by three boxes per axis (abm_params.super_fraction,
        the largest fraction any simulation needs); None sizes every range for
        any grid of its box capacity."""
        offsets = [int(o) for o in offsets]
        ns = len(offsets) - 1
        common = dict(common or {})
        if "precision" not in common:
            common["precision"] = "f64" if pos.dtype == torch.float64 else "f32"
        plist = [default_params(**{**common, **(params[s] if params else {})}) for s in range(ns)]
        self.params = plist[0]
        self.pos_in = pos.contiguous()
        self.diam_in = diam.contiguous()
        self.n = int(pos.shape[0])
        self._nsims = ns
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        caps, frac = [], 0.0
        for s in range(ns):
            a, b = offsets[s], offsets[s + 1]
            ext = extent_of(self.pos_in[a:b], self.diam_in[a:b], plist[s], self.stream)
            caps.append(box_capacity_for(ext.nboxes, box_slack))
            if super_slack is not None:   # each range holds ceil(f * capacity) + 64 entries
                frac = max(frac, super_fraction_for(ext, caps[-1], float(super_slack)))
        if super_slack is not None:
            for p in plist:
                p.super_fraction = frac
        self.box_capacity = sum(caps)
        offs = (C.c_int64 * (ns + 1))(*offsets)
        capa = (C.c_int64 * ns)(*caps)
        parr = (abm_params * ns)(*plist)
        nbytes = C.c_int64()
        _check(lib().abm_workspace_bytes(ns, offs, capa, C.byref(plist[0]), C.byref(nbytes)), "abm_workspace_bytes")
        self.ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=pos.device)
        self.ctx = C.c_void_p()
        _check(lib().abm_init_batched(C.byref(self.ctx), ns, offs, _ptr(self.pos_in), _ptr(self.diam_in), parr, capa,
                                      _ptr(self.ws), self.ws.numel(), int(self.stream.cuda_stream)),
               "abm_init_batched")

    @property
    def nsims(self) -> int:
        return self._nsims


class StepFn(torch.autograd.Function):
    """x_T = StepFn.apply(x0, diam, k, gamma, nsteps, ckpt_every, params_dict).

    Runs nsteps steps on the GPU from x0, recording a checkpoint every
    ckpt_every steps and, where they fit in device memory, every step's
    contact tape; backward gives dL/dx0, dL/dk and dL/dgamma through the
    hand-written reverse-mode kernels."""

    @staticmethod
    def forward(ctx, x0, diam, k, gamma, nsteps: int, ckpt_every: int, params: Optional[dict] = None):
        kw = dict(params or {})
        kw.update(k=float(k), gamma=float(gamma), detect_static=False)
        sim = Sim(x0.detach(), diam.detach(), **kw)
        sim.forward_record(nsteps, ckpt_every)
        xT = sim.positions()
        ctx.sim = sim
        ctx.dtypes = (x0.dtype, torch.as_tensor(k).dtype, torch.as_tensor(gamma).dtype)
        return xT

    @staticmethod
    def backward(ctx, grad_xT):
        gx0, gp = ctx.sim.backward(grad_xT)
        sim = ctx.sim
        ctx.sim = None
        sim.close()
        dx, dk, dg = ctx.dtypes
        return gx0.to(dx), None, gp[0].to(dk), gp[1].to(dg), None, None, None
