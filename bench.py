#!/usr/bin/env python3
"""Benchmark of the agent step on one MI355X.

Headline: agent-steps/s of the plain step (grid build + static flags + force
+ move, the force of static agents skipped) on 1e7 spheres in FP32 state, the
c2 construction scaled to 1e7 agents (uniform inner cube + force-free jittered
lattice shell, cube side 3387.7, d ~ U[8, 12]).  Beside it, on the same GPU:
the same steps without the static skip and in the Hilbert order, the batched
form (512 simulations, 50 steps in one graph launch) and the adjoint form (1e5
spheres, 50 steps forward + backward), each as agent-steps/s; the dominant kernel's roofline from HIP
events around it over the timed region; and the CPU oracle timed on a bounded
sample of the same workload.

Prints one JSON line (rank 0).  Inputs are resident in HBM before timing.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "agent-steps/s (grid+force+move) at 1e7 agents; batched & adjoint vs plain step"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
# Algorithmic bytes per agent of the step: read x, y, z, d; write x, y, z;
# one 4-byte box key and one 4-byte list index written and read.
STEP_BYTES = {"f32": 4 * 4 + 3 * 4 + 16, "f64": 4 * 8 + 3 * 8 + 16}
# ... of the force/move kernel alone: read x, y, z, d and the 4-byte slot
# index of the agent; write x, y, z.
FORCE_BYTES = {"f32": 4 * 4 + 4 + 3 * 4, "f64": 4 * 8 + 4 + 3 * 8}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_force_headline_traffic.json")


def measured_traffic(n, prec, block_size, order="morton", skip=True):
    """HBM bytes per force launch from the committed FETCH_SIZE/WRITE_SIZE
    counter runs (scaled by a plain copy's reading), or None when the kernel
    sources changed since the counters were taken or the configuration
    differs from the profiled one (1e7 agents, FP32 state, the recorded threads per block,
    Morton order, static skip on)."""
    import hashlib
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
        h = hashlib.sha256()
        for name in rec["sources"]:
            with open(os.path.join(ROOT, "paper_2301_06984_amd", "csrc", name), "rb") as f:
                h.update(f.read())
    except (OSError, KeyError, ValueError):
        return None
    if (h.hexdigest() != rec["source_sha256"] or n != 10_000_000 or prec != "f32"
            or block_size != rec.get("block_size") or order != "morton" or not skip):
        return None
    return float(rec["traffic_bytes"])


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def timed_steps(sim, steps, timing=0):
    """Wall time of `steps` steps; timing 2: HIP events around the force
    kernel of each step, 1: around every kernel (for the phase breakdown)."""
    import torch
    if timing:
        sim.set_timing(timing)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sim.sync()
    tm = sim.timing() if timing else None
    if timing:
        sim.set_timing(False)
    return t1 - t0, tm


def cpu_baseline(w, budget_s: float, skip: bool):
    """The oracle (as it is) on the same workload, whole steps until the budget is used."""
    import numpy as np
    import oracle
    st = oracle.State.initial(w.pos, w.diam)
    p = oracle.Params(detect_static=skip)
    steps = 0
    t0 = time.perf_counter()
    while True:
        oracle.step(st, p)
        steps += 1
        el = time.perf_counter() - t0
        log(f"cpu oracle step {steps}: {el:.1f} s")
        if el >= budget_s or steps >= 3:
            break
    cores = oracle.max_threads()
    del np
    return dict(value=w.n * steps / el, unit="agent-steps/s", cores=int(cores), kind="oracle",
                sample=f"{steps} full step(s) of the {w.n}-agent headline workload (FP64 C++ oracle, OpenMP, "
                       f"{el:.1f} s)")


DEFAULT_SWEEP = "1e3,1e4,1e5,1e6,1e7,1e8,3e8,1e9"


def scale_sweep(sizes, block_size):
    """Plain step (skip off, re-layout every step) on n spheres uniform in a
    cube at c2's density (about 12 candidates per agent), d ~ U[8, 12],
    FP32 state, seed (6, n): agent-steps/s per n (steps timed without
    events), HIP-event phase times (from up to 20 steps after them), and the
    workspace size."""
    import numpy as np
    import torch
    from paper_2301_06984_amd import abm, workloads
    for n in sizes:
        side = (n / workloads.C2_DENSITY) ** (1.0 / 3.0)
        log(f"sweep n={n}: generating (side {side:.1f})")
        p, d = workloads.uniform_cube(n, side, (6, n), dtype=np.float32)
        pos = torch.from_numpy(p).cuda()
        diam = torch.from_numpy(d).cuda()
        del p, d
        # the grid grows by a box or two per axis as the agents relax: a
        # tight box capacity keeps the largest runs inside the GPU's memory
        sim = abm.Sim(pos, diam, detect_static=False, sort_every=1, block_size=block_size,
                      box_slack=1.5 if n < 100_000_000 else 1.05)
        steps = int(min(200, max(5, 2e8 // n)))
        sim.step(3)
        sim.sync()
        el, _ = timed_steps(sim, steps)   # no events in the timed steps
        _, tm = timed_steps(sim, min(steps, 20), timing=1)   # phase breakdown: the steps after them
        value = n * steps / el
        rec = dict(sweep="uniform cube at c2 density, d~U[8,12], FP32 state, seed (6, n)", n=int(n), steps=steps,
                   value=value, unit="agent-steps/s", ms_per_step=1e3 * el / steps,
                   step_frac=round(value * STEP_BYTES["f32"] / (HBM_PEAK_GBS * 1e9), 4),
                   workspace_gb=round(sim.ws.numel() / 1e9, 2),
                   phase_ms={k: round(tm[k] / tm["steps"], 4) for k in abm.TIMED_PHASES})
        print(json.dumps(rec), flush=True)
        sim.close()
        del sim, pos, diam
        torch.cuda.empty_cache()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=10_000_000)
    ap.add_argument("--block-size", type=int, default=512)
    ap.add_argument("--skip", action=argparse.BooleanOptionalAction, default=True,
                    help="the static skip (Section 5) in the headline run (--no-skip: every force computed)")
    ap.add_argument("--order", choices=["morton", "hilbert"], default="morton",
                    help="order of the boxes for the headline run (the legs keep their own)")
    ap.add_argument("--sort-every", type=int, default=1)
    ap.add_argument("--no-extras", action="store_true", help="leave out the Hilbert, static-skip, dynamic, batched and adjoint legs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--json-out", default=None)
    ap.add_argument("--sweep", nargs="?", const=DEFAULT_SWEEP, default=None,
                    help="instead of the headline: agent-steps/s of the plain step on a uniform cube at c2's "
                         "density for each N of a comma-separated list (one JSON line per N)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of 1 GiB five times (scales rocprof byte counters)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        a.fill_(1)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "device copy", "bytes_read": 1 << 30, "bytes_written": 1 << 30,
                          "launches": 5}), flush=True)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the spatial decomposition over GPUs is designed, not built).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2301_06984_amd import abm, build as hip_build, tune, workloads

    if not os.path.exists(abm.LIB_PATH):
        hip_build.build()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.sweep:
        scale_sweep([int(float(x)) for x in args.sweep.split(",")], args.block_size)
        return

    # ---------------------------------------------------------------- headline
    log(f"generating headline workload n={args.n}")
    w = workloads.headline(n=args.n)
    pos = torch.from_numpy(w.pos).to(dev)
    diam = torch.from_numpy(w.diam).to(dev)
    sim = abm.Sim(pos, diam, detect_static=args.skip, sort_every=args.sort_every, block_size=args.block_size,
                  order=args.order)
    sim.step(args.warmup)
    sim.sync()
    log("timed region")
    el, tm = timed_steps(sim, args.steps, timing=2)
    value = w.n * args.steps / el
    ms_step = 1e3 * el / args.steps
    force_ms = tm["force"] / tm["steps"]
    # the phase breakdown: the next K steps, with events around every kernel
    el_ph, tm_ph = timed_steps(sim, args.steps, timing=1)
    phases = {k: tm_ph[k] / tm_ph["steps"] for k in abm.TIMED_PHASES}
    dominant = max(abm.TIMED_PHASES, key=lambda k: phases[k])
    prec = w.precision
    force_bytes = FORCE_BYTES[prec] * w.n
    ach = force_bytes / (force_ms * 1e-3) / 1e9
    traffic = measured_traffic(w.n, prec, args.block_size, args.order, args.skip)
    roof = dict(bound="hbm", kernel="k_force (static flags + force + move)", achieved=round(ach, 1),
                peak=HBM_PEAK_GBS, unit="GB/s", frac=round(ach / HBM_PEAK_GBS, 4),
                traffic=None if traffic is None else round(traffic), traffic_unit="bytes per launch",
                algorithmic_bytes=force_bytes,
                bytes_per_agent=FORCE_BYTES[prec], avg_launch_ms=round(force_ms, 4),
                dominant_phase=dominant, phase_ms={k: round(v, 4) for k, v in phases.items()},
                phase_ms_note="the K steps after the timed ones, with events around every kernel "
                              f"({1e3 * el_ph / args.steps:.4f} ms per step there)",
                step_bytes_per_agent=STEP_BYTES[prec],
                step_frac=round(value * STEP_BYTES[prec] / (HBM_PEAK_GBS * 1e9), 4))
    log(f"headline {value:.3e} agent-steps/s, {ms_step:.3f} ms/step, phases {phases}")
    sim_stats = sim.stats()
    del sim

    extras = {}
    if not args.no_extras:
        # Hilbert order of the super-boxes (the other curve Section 4.2
        # compares): the same steps, only the order of the boxes changed
        sh = abm.Sim(pos, diam, detect_static=args.skip, sort_every=args.sort_every, block_size=args.block_size,
                     order="hilbert")
        sh.step(args.warmup)
        sh.sync()
        elh, _ = timed_steps(sh, args.steps, timing=2)
        _, tmh = timed_steps(sh, args.steps, timing=1)
        extras["hilbert"] = dict(value=w.n * args.steps / elh, unit="agent-steps/s",
                                 ms_per_step=round(1e3 * elh / args.steps, 4),
                                 speedup_vs_morton=round(el / elh, 3),
                                 phase_ms={k: round(tmh[k] / tmh["steps"], 4) for k in abm.TIMED_PHASES},
                                 note="2x2x2 super-boxes along a Hilbert curve, Morton order inside each; "
                                      "phase_ms from the K steps after the timed ones, as under roofline")
        log(f"hilbert {extras['hilbert']}")
        del sh
        # the other setting of the static skip (same workload; the shell is
        # force-free and static from its first step)
        s2 = abm.Sim(pos, diam, detect_static=not args.skip, sort_every=args.sort_every, block_size=args.block_size)
        s2.step(args.warmup)
        el2, _ = timed_steps(s2, args.steps, timing=2)   # timed as the headline
        el_on, el_off = (el, el2) if args.skip else (el2, el)
        son = (sim_stats if args.skip else s2.stats())
        extras["static_skip"] = dict(skip_on=w.n * args.steps / el_on, skip_off=w.n * args.steps / el_off,
                                     unit="agent-steps/s", speedup_on_vs_off=round(el_off / el_on, 3),
                                     static_fraction_last_step=round(son["n_static"] / w.n, 4))
        log(f"static skip {extras['static_skip']}")
        del s2
        # dynamic population (Section 3.2): 1% of the agents removed and as
        # many added between two steps; the next grid is a full build
        sd = abm.Sim(pos, diam, detect_static=False, sort_every=args.sort_every, block_size=args.block_size,
                     capacity=w.n + w.n // 50)
        sd.step(args.warmup)
        sd.sync()
        gd = np.random.default_rng(8)
        m = w.n // 100
        rm = torch.from_numpy(gd.choice(w.n, m, replace=False)).to(dev)
        R = float(w.diam.max())
        side = float(w.meta["side"])
        newp = torch.from_numpy(gd.uniform(0.0, side, size=(m, 3)).astype(w.pos.dtype)).to(dev)
        newd = torch.from_numpy(gd.uniform(8.0, R, size=m).astype(w.diam.dtype)).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sd.remove_agents(rm)
        t1 = time.perf_counter()
        sd.add_agents(newp, newd)
        t2 = time.perf_counter()
        el_full, _ = timed_steps(sd, 1)
        el_upd, _ = timed_steps(sd, 1)
        extras["dynamic"] = dict(removed=m, added=m, remove_ms=round(1e3 * (t1 - t0), 3),
                                 add_ms=round(1e3 * (t2 - t1), 3),
                                 removed_per_s=m / (t1 - t0), added_per_s=m / (t2 - t1),
                                 next_step_ms=round(1e3 * el_full, 3), following_step_ms=round(1e3 * el_upd, 3),
                                 note="calls include their stream synchronisations; the next step's grid is a "
                                      "full build, the following one an update")
        log(f"dynamic {extras['dynamic']}")
        del sd, rm, newp, newd
        del pos, diam
        torch.cuda.empty_cache()
        # batched: 512 simulations, 50 steps in one graph launch, with the
        # knobs the autotuner picks for this batch (tuning is not timed)
        wb = workloads.c4()
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            pb, db = torch.from_numpy(wb.pos).to(dev), torch.from_numpy(wb.diam).to(dev)
            tuned = tune.autotune_batched(pb, db, wb.offsets, graph_steps=wb.steps, stream=s)
            log(f"autotuned {tuned.params}: {tuned.ms_per_step:.3f} ms/step over {len(tuned.trials)} trials")
            b = abm.BatchedSim(pb, db, wb.offsets, stream=s, common=dict(tuned.params))
            b.graph_capture(wb.steps)
            b.graph_launch()          # warm-up replay
            b.sync()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            b.graph_launch()
            b.sync()
            elb = time.perf_counter() - t0
            del b
            # the same simulations without batching: one plain context each,
            # default knobs, each replaying a graph of its own 10 steps
            kp = 10
            plain_sims = []
            for k in range(len(wb.offsets) - 1):
                a, e = int(wb.offsets[k]), int(wb.offsets[k + 1])
                sp = abm.Sim(pb[a:e].contiguous(), db[a:e].contiguous(), stream=s)
                sp.step(2)
                sp.graph_capture(kp)
                sp.graph_launch()     # warm-up replay
                plain_sims.append(sp)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for sp in plain_sims:
                sp.graph_launch()
            torch.cuda.synchronize()
            elc = (time.perf_counter() - t0) / kp
            del plain_sims, sp
        extras["batched"] = dict(value=wb.n * wb.steps / elb, unit="agent-steps/s", nsims=len(wb.offsets) - 1,
                                 agents=int(wb.n), steps=wb.steps, launch="one hipGraph replay of 50 steps",
                                 ms_per_step=round(1e3 * elb / wb.steps, 4),
                                 plain_contexts_ms_per_step=round(1e3 * elc, 4),
                                 speedup_vs_plain_contexts=round(elc / (elb / wb.steps), 3),
                                 plain_contexts="the same simulations, one plain context each, each replaying a "
                                                "graph of 10 steps, one after another on one stream",
                                 ratio_vs_plain=round((wb.n * wb.steps / elb) / value, 3),
                                 autotuned=tuned.params, tune_trials=len(tuned.trials),
                                 untuned_ms_per_step=round(tuned.trials[0][1], 4),
                                 tuned_ms_per_step=round(tuned.ms_per_step, 4))
        log(f"batched {extras['batched']}")
        del pb, db
        torch.cuda.empty_cache()
        # adjoint: 1e5 spheres, 50 steps, checkpoint every 10, forward + backward
        wa = workloads.c5()
        pa = torch.from_numpy(wa.pos).to(dev)
        da = torch.from_numpy(wa.diam).to(dev)
        plain = abm.Sim(pa, da, sort_every=0)
        plain.step(5)
        elp, _ = timed_steps(plain, wa.steps)
        adj = abm.Sim(pa, da, sort_every=0)
        adj.forward_record(wa.steps, 10)      # warm-up
        xT = adj.positions().double()
        tgt = torch.from_numpy(wa.target).to(dev)
        adj.backward(2.0 * (xT - tgt) / (3 * wa.n))
        adj2 = abm.Sim(pa, da, sort_every=0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        adj2.forward_record(wa.steps, 10)
        xT = adj2.positions().double()
        gx, gp = adj2.backward(2.0 * (xT - tgt) / (3 * wa.n))
        torch.cuda.synchronize()
        ela = time.perf_counter() - t0
        extras["adjoint"] = dict(value=wa.n * wa.steps / ela, unit="agent-steps/s (forward+backward)",
                                 agents=wa.n, steps=wa.steps, ckpt_every=10,
                                 plain_forward=wa.n * wa.steps / elp,
                                 ratio_vs_plain_forward=round(elp / ela, 3),
                                 dL_dk=float(gp[0]), dL_dgamma=float(gp[1]))
        log(f"adjoint {extras['adjoint']}")

    cpu = None
    if not args.no_cpu:
        log("cpu baseline")
        cpu = cpu_baseline(w, args.cpu_budget, args.skip)

    out = {"metric": METRIC, "value": value, "unit": "agent-steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "headline: 1e7 spheres, c2 construction (uniform inner cube + jittered "
                                  "force-free lattice shell), side 3387.7, d~U[8,12], seed 2",
                      "n": w.n, "state": prec, "arithmetic": "f64", "detect_static": bool(args.skip),
                      "sort_every": args.sort_every, "block_size": args.block_size, "order": args.order},
           "roofline": roof, "cpu_baseline": cpu, **extras}
    line = json.dumps(out)
    print(line, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
