"""Autotuner for the batched form.

Picks, for one batch of simulations, the four knobs that change the cost of
a step but not its neighbour sets:

* ``cell_factor``  box edge as a multiple of the interaction radius R (>= 1;
  a larger box means fewer boxes and more candidates per box);
* ``block_size``   threads per block of the force kernel (its LDS walk
  scratch bounds how many blocks fit on a compute unit);
* ``sort_every``   how often the agents are re-laid out in Morton order;
* ``walk_chunk``   candidate slots the neighbour walk tests together (2 or 4).

It times a few steps of the actual batch for each candidate value and does one
pass of coordinate descent (re-layout cadence, block size, walk width, then box
edge), keeping the other knobs at the best values found so far.  Re-layout
cadence, block size and walk width leave the results bitwise unchanged.  The box edge
changes the canonical order and so the order of the force sums, within
rounding.  A graph-captured replay must cover an even number of whole
re-layout periods, so other cadences are skipped when ``graph_steps`` is
given.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import torch

from . import abm

Config = Dict[str, float]

DEFAULT_CELL_FACTORS = (1.0, 1.25, 1.5)
DEFAULT_BLOCK_SIZES = (128, 256, 512)
DEFAULT_SORT_EVERY = (1, 2, 5, 10)
DEFAULT_WALK_CHUNKS = (2, 4)


@dataclasses.dataclass
class TuneResult:
    params: Config                               # the chosen cell_factor, block_size, sort_every, walk_chunk
    ms_per_step: float                           # its measured time per step
    trials: List[Tuple[Config, float]]           # every configuration timed, in order


def time_batched(pos: torch.Tensor, diam: torch.Tensor, offsets: Sequence[int], cfg: Config, *, steps: int = 4,
                 warmup: int = 2, stream: Optional[torch.cuda.Stream] = None, common: Optional[dict] = None) -> float:
    """Milliseconds per step of a fresh batched context with the knobs in cfg
    (HIP events on the context's stream, after warm-up steps)."""
    s = stream if stream is not None else torch.cuda.current_stream()
    sim = abm.BatchedSim(pos, diam, offsets, stream=s, common={**(common or {}), **cfg})
    try:
        sim.step(warmup)
        sim.sync()
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record(s)
        sim.step(steps)
        stop.record(s)
        sim.sync()
        stop.synchronize()
        return start.elapsed_time(stop) / steps
    finally:
        sim.close()


def coordinate_descent(timer: Callable[[Config], float], *, cell_factors: Sequence[float] = DEFAULT_CELL_FACTORS,
                       block_sizes: Sequence[int] = DEFAULT_BLOCK_SIZES,
                       sort_every: Sequence[int] = DEFAULT_SORT_EVERY,
                       walk_chunks: Sequence[int] = DEFAULT_WALK_CHUNKS,
                       graph_steps: Optional[int] = None) -> TuneResult:
    """One pass of coordinate descent over the four knobs with cost timer(cfg)."""
    if graph_steps is not None:
        # a replay must start from the same internal buffers: whole re-layout
        # periods, an even number of them
        sort_every = [k for k in sort_every if k > 0 and graph_steps % k == 0 and (graph_steps // k) % 2 == 0]
    if not (cell_factors and block_sizes and sort_every and walk_chunks):
        raise ValueError("every knob needs at least one candidate value")
    best: Config = dict(cell_factor=float(cell_factors[0]),
                        block_size=int(256 if 256 in block_sizes else block_sizes[0]),
                        sort_every=int(1 if 1 in sort_every else sort_every[0]),
                        walk_chunk=int(walk_chunks[0]))
    seen: Dict[Tuple, float] = {}
    trials: List[Tuple[Config, float]] = []

    def cost(cfg: Config) -> float:
        key = (cfg["cell_factor"], cfg["block_size"], cfg["sort_every"], cfg["walk_chunk"])
        if key not in seen:
            seen[key] = float(timer(dict(cfg)))
            trials.append((dict(cfg), seen[key]))
        return seen[key]

    best_ms = cost(best)
    for knob, values in (("sort_every", sort_every), ("block_size", block_sizes), ("walk_chunk", walk_chunks),
                         ("cell_factor", cell_factors)):
        for v in values:
            cand = dict(best)
            cand[knob] = type(best[knob])(v)
            ms = cost(cand)
            if ms < best_ms:
                best, best_ms = cand, ms
    return TuneResult(params=best, ms_per_step=best_ms, trials=trials)


def autotune_batched(pos: torch.Tensor, diam: torch.Tensor, offsets: Sequence[int], *,
                     graph_steps: Optional[int] = None, steps: int = 4, warmup: int = 2,
                     cell_factors: Sequence[float] = DEFAULT_CELL_FACTORS,
                     block_sizes: Sequence[int] = DEFAULT_BLOCK_SIZES,
                     sort_every: Sequence[int] = DEFAULT_SORT_EVERY,
                     walk_chunks: Sequence[int] = DEFAULT_WALK_CHUNKS,
                     stream: Optional[torch.cuda.Stream] = None, common: Optional[dict] = None) -> TuneResult:
    """Tune cell_factor, block_size, sort_every and walk_chunk for this batch
    on the GPU.  The inputs are copied by every trial context and left
    unchanged."""
    return coordinate_descent(
        lambda cfg: time_batched(pos, diam, offsets, cfg, steps=steps, warmup=warmup, stream=stream, common=common),
        cell_factors=cell_factors, block_sizes=block_sizes, sort_every=sort_every, walk_chunks=walk_chunks,
        graph_steps=graph_steps)
