#!/usr/bin/env python3
"""Benchmark of the agent step on one MI355X.

Headline: agent-steps/s of the plain step (grid build + static flags + force
+ move) on 1e7 spheres in FP32 state, the c2 construction scaled to 1e7
agents (uniform inner cube + force-free jittered lattice shell, cube side
3387.7, d ~ U[8, 12]), with the static test off, so that every force is
evaluated: the run the roofline is taken on.  The dominant kernel's time
comes from HIP events around it over the timed steps; its HBM bytes and VALU
instructions per launch from the committed rocprofv3 record
(profiles/k_force_headline_counters.json, used only while the kernel
sources match it).

Legs on the same GPU: the static test on (speedup and skip fraction), the
Hilbert order, population changes, FP64 state, c1's density at 1e7 agents,
c2, the clustered 5e7-agent workload, the batched form (512 simulations, 50
steps in one graph launch, against plain contexts and against one simulation
of as many agents) and the adjoint form (1e5 spheres, 50 steps forward +
backward); and the CPU oracle timed on bounded samples of the headline
workload, at all host cores and at one thread.

Prints one JSON line.  Inputs are resident in HBM before timing.
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
# VALU issue peak: 256 CUs x 4 SIMDs, one wave64 instruction per SIMD every 4
# cycles (16 lanes), at 2.4 GHz: 6.14e11 wave instructions/s, 3.93e13 lane
# operations/s (FP64 FMA runs at that rate on this chip).
CUS, SIMDS, CLOCK_HZ = 256, 4, 2.4e9
VALU_WAVE_INSTR_PEAK = CUS * SIMDS * CLOCK_HZ / 4.0
VALU_LANE_OPS_PEAK = 64.0 * VALU_WAVE_INSTR_PEAK
# Algorithmic bytes per agent-step of the whole step (the method's own
# minimum): read x, y, z, d; write x, y, z; one 4-byte box key and one 4-byte
# list index written and read.
STEP_BYTES = {"f32": 4 * 4 + 3 * 4 + 16, "f64": 4 * 8 + 3 * 8 + 16}

PROFILES = os.path.join(ROOT, "profiles")
COUNTERS_FILE = os.path.join(PROFILES, "k_force_headline_counters.json")
FORCE_SOURCES = ["force_kernels.hip", "force_loop.h", "abm_device.h", "abm_internal.h", "hilbert_order.h"]
# the force kernel instantiation of the roofline run: FP32 state, one
# simulation, static test off, re-layout on, 2-wide walk
ROOF_KERNEL = "abm::k_force<float, false, false, true, 2, false, false>"


def force_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for name in FORCE_SOURCES:
        with open(os.path.join(ROOT, "paper_2301_06984_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counter_record(block_size):
    """The committed rocprofv3 record of the roofline run's force kernel
    (VALU instructions, HBM bytes per launch), or None when the kernel sources
    changed since it was taken or the block size differs."""
    try:
        with open(COUNTERS_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != force_sources_sha() or rec.get("block_size") != block_size:
        return None
    return rec


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


def host_description():
    """CPU model, sockets x cores, threads and memory of this host (lscpu, /proc/meminfo)."""
    import subprocess
    d = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            k, v = k.strip(), v.strip()
            if k in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)"):
                d[k] = v
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    d["MemTotal"] = line.split(":")[1].strip()
    except OSError:
        pass
    d["usable_cpus"] = len(os.sched_getaffinity(0))
    return d


def cpu_oracle_rate(w, steps, nthreads, skip):
    """The oracle as it is, one untimed step, then `steps` timed steps."""
    import oracle
    st = oracle.State.initial(w.pos, w.diam)
    p = oracle.Params(detect_static=skip, nthreads=nthreads)
    oracle.step(st, p)
    t0 = time.perf_counter()
    for _ in range(steps):
        oracle.step(st, p)
    el = time.perf_counter() - t0
    return w.n * steps / el, el


def cpu_baseline(skip: bool):
    """The CPU oracle on bounded samples of the headline workload: all the
    host's cores on the full 1e7 agents, and one thread on the same
    construction at 1e6 agents."""
    import oracle
    from paper_2301_06984_amd import workloads
    cores = int(oracle.max_threads())
    w = workloads.headline()
    log(f"cpu oracle, {cores} threads, 1e7 agents")
    v_all, el_all = cpu_oracle_rate(w, 2, 0, skip)
    del w
    w1 = workloads.headline(n=1_000_000)
    log("cpu oracle, 1 thread, 1e6 agents")
    v_one, el_one = cpu_oracle_rate(w1, 1, 1, skip)
    return dict(value=v_all, unit="agent-steps/s", cores=cores, kind="oracle",
                sample=f"2 steps after an untimed one of the 1e7-agent headline workload, {cores} OpenMP threads, "
                       f"{el_all:.1f} s (FP64 C++ oracle, static test {'on' if skip else 'off'})",
                value_1thread=v_one,
                sample_1thread=f"1 step after an untimed one of the same construction at 1e6 agents, 1 thread, "
                               f"{el_one:.1f} s",
                host=host_description())


DEFAULT_SWEEP = "1e3,1e4,1e5,1e6,1e7,1e8,3e8,1e9,1.72e9"
# above this many agents the sweep builds its context from chunks of agents
# (the inputs of one piece would not fit beside the workspace)
SWEEP_CHUNKED_ABOVE = 1_000_000_000
SWEEP_CHUNK = 100_000_000


def scale_sweep(sizes, block_size):
    """Plain step (skip off, re-layout every step) on n spheres uniform in a
    cube at c2's density (about 12 candidates per agent), d ~ U[8, 12],
    FP32 state, seed (6, n): agent-steps/s per n (steps timed without
    events), HIP-event phase times (from up to 20 steps after them), and the
    workspace size.  Above SWEEP_CHUNKED_ABOVE agents the positions come in
    chunks of SWEEP_CHUNK (chunk k from seed (6, n, k)): a context of the
    first chunk with room for n agents, the others added with
    abm_add_agents, R fixed at 12 (the largest diameter the draw allows)."""
    import numpy as np
    import torch
    from paper_2301_06984_amd import abm, workloads
    for n in sizes:
        side = (n / workloads.C2_DENSITY) ** (1.0 / 3.0)
        # the grid grows by a box or two per axis as the agents relax: a
        # tight box capacity (and from 1e8 agents a super-box table sized
        # for the grid) keeps the largest runs inside the GPU's memory
        kw = dict(detect_static=False, sort_every=1, block_size=block_size,
                  box_slack=1.5 if n < 100_000_000 else 1.05)
        if n >= 100_000_000:
            kw["super_slack"] = 1.2
        if n <= SWEEP_CHUNKED_ABOVE:
            log(f"sweep n={n}: generating (side {side:.1f})")
            p, d = workloads.uniform_cube(n, side, (6, n), dtype=np.float32)
            pos = torch.from_numpy(p).cuda()
            diam = torch.from_numpy(d).cuda()
            del p, d
            sim = abm.Sim(pos, diam, **kw)
            del pos, diam
            made = "one piece, seed (6, n)"
        else:
            nchunks = (n + SWEEP_CHUNK - 1) // SWEEP_CHUNK
            free, total = torch.cuda.mem_get_info()
            log(f"sweep n={n}: {nchunks} chunks (side {side:.1f}); device memory free {free / 1e9:.1f} of "
                f"{total / 1e9:.1f} GB")
            sim = None
            for k in range(nchunks):
                m = min(SWEEP_CHUNK, n - k * SWEEP_CHUNK)
                p, d = workloads.uniform_cube(m, side, (6, n, k), dtype=np.float32)
                pos = torch.from_numpy(p).cuda()
                diam = torch.from_numpy(d).cuda()
                del p, d
                if sim is None:
                    sim = abm.Sim(pos, diam, capacity=n, interaction_radius=12.0, **kw)
                else:
                    sim.add_agents(pos, diam)
                del pos, diam
                log(f"sweep n={n}: {min(n, (k + 1) * SWEEP_CHUNK)} agents in the context")
            made = f"{nchunks} chunks of {SWEEP_CHUNK} (seed (6, n, k)), added with abm_add_agents; R = 12"
        steps = int(min(200, max(5, 2e8 // n)))
        sim.step(3)
        sim.sync()
        el, _ = timed_steps(sim, steps)   # no events in the timed steps
        _, tm = timed_steps(sim, min(steps, 20), timing=1)   # phase breakdown: the steps after them
        value = n * steps / el
        rec = dict(sweep="uniform cube at c2 density, d~U[8,12], FP32 state", made=made, n=int(n), steps=steps,
                   value=value, unit="agent-steps/s", ms_per_step=1e3 * el / steps,
                   step_frac=round(value * STEP_BYTES["f32"] / (HBM_PEAK_GBS * 1e9), 4),
                   workspace_gb=round(sim.ws.numel() / 1e9, 2),
                   phase_ms={k: round(tm[k] / tm["steps"], 4) for k in abm.TIMED_PHASES})
        print(json.dumps(rec), flush=True)
        sim.close()
        del sim
        torch.cuda.empty_cache()


def run_plain(pos, diam, steps, warmup, timing=2, **kw):
    """Plain context on device tensors: warm-up, then `steps` timed steps
    (events around the force kernel with timing 2); returns the context, the
    wall time and the force kernel's mean time per step (ms)."""
    from paper_2301_06984_amd import abm
    sim = abm.Sim(pos, diam, **kw)
    sim.step(warmup)
    sim.sync()
    el, tm = timed_steps(sim, steps, timing=timing)
    force_ms = tm["force"] / tm["steps"] if tm else None
    return sim, el, force_ms


def leg(extras, name, fn, only=None):
    """Run one extra leg (unless `only` names others); its failure is
    recorded, not fatal to the line."""
    if only is not None and name not in only:
        return
    try:
        extras[name] = fn()
        log(f"{name} {extras[name]}")
    except Exception as e:  # noqa: BLE001 -- reported in the JSON line
        extras[name] = {"error": f"{type(e).__name__}: {e}"}
        log(f"{name} failed: {e}")
    import torch
    torch.cuda.empty_cache()


def summarize_profiles(kt_dir, valu_dir, fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, block_size):
    """Write profiles/k_force_headline_counters.json from the rocprofv3 CSVs
    of the roofline run (bench.py --profile-run): per-launch VALU and other
    instruction counts and HBM bytes of the force kernel over the
    steady-state steps (update builds; the first, full-build launch apart),
    the byte counters scaled by what a plain 1 GiB copy reads and writes."""
    import csv
    import glob

    def rows(d, pattern):
        out = []
        for f in glob.glob(os.path.join(d, "**", pattern), recursive=True):
            with open(f) as fh:
                out += list(csv.DictReader(fh))
        return out

    def per_dispatch(d, kernel):
        by = {}
        for r in rows(d, "*counter_collection.csv"):
            if kernel in r["Kernel_Name"]:
                by.setdefault(int(r["Dispatch_Id"]), {})[r["Counter_Name"]] = float(r["Counter_Value"])
        ids = sorted(by)
        return [by[i] for i in ids]

    def steady(dl):
        return dl[1:] if len(dl) > 1 else dl

    def mean(dl, c):
        v = [x[c] for x in dl if c in x]
        return sum(v) / len(v) if v else None

    vd = per_dispatch(valu_dir, ROOF_KERNEL)
    fd = per_dispatch(fetch_dir, ROOF_KERNEL)
    wd = per_dispatch(write_dir, ROOF_KERNEL)
    cf = per_dispatch(copy_fetch_dir, "copyBuffer")
    cw = per_dispatch(copy_write_dir, "copyBuffer")
    gib = float(1 << 30)
    fscale = gib / (1024.0 * mean(cf, "FETCH_SIZE"))
    wscale = gib / (1024.0 * mean(cw, "WRITE_SIZE"))
    times = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in rows(kt_dir, "*kernel_trace.csv")
             if ROOF_KERNEL in r["Kernel_Name"]]
    sv = steady(vd)
    rec = {
        "kernel": ROOF_KERNEL,
        "workload": "headline 1e7 spheres, FP32 state, static test off, re-layout every step",
        "block_size": block_size,
        "dispatches": f"steady state: launches 2..{len(vd)} (update builds); launch 1 (full build) reported apart",
        "per_launch": {c: mean(sv, c) for c in ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS",
                                               "SQ_INSTS_VMEM_RD", "SQ_WAVE_CYCLES", "SQ_WAIT_INST_ANY",
                                               "SQ_BUSY_CYCLES")},
        "full_build_launch": {c: vd[0].get(c) for c in ("SQ_INSTS_VALU", "SQ_WAVES")} if vd else None,
        "fetch_kib": mean(steady(fd), "FETCH_SIZE"),
        "write_kib": mean(steady(wd), "WRITE_SIZE"),
        "full_build_fetch_kib": fd[0]["FETCH_SIZE"] if fd else None,
        "full_build_write_kib": wd[0]["WRITE_SIZE"] if wd else None,
        "fetch_scale": fscale,
        "write_scale": wscale,
        "kernel_trace_ns": {"steady_mean": sum(times[1:]) / max(len(times) - 1, 1) if times else None,
                            "first": times[0] if times else None, "launches": len(times)},
        "sources": FORCE_SOURCES,
        "source_sha256": force_sources_sha(),
    }
    rec["traffic_bytes"] = 1024.0 * (rec["fetch_kib"] * fscale + rec["write_kib"] * wscale)
    with open(COUNTERS_FILE, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec, indent=1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=10_000_000)
    ap.add_argument("--block-size", type=int, default=256)
    ap.add_argument("--order", choices=["morton", "hilbert"], default="morton",
                    help="order of the boxes for the headline run (the legs keep their own)")
    ap.add_argument("--sort-every", type=int, default=1)
    ap.add_argument("--no-extras", action="store_true",
                    help="leave out every leg but the headline (static test, FP64 state, densities, clustered, "
                         "Hilbert, dynamic population, batched and adjoint)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--legs", default=None,
                    help="comma-separated legs to run (default: all): static_skip, hilbert, sort_cadence, dynamic, "
                         "headline_fp64_state, c1_density_1e7, c2, c3, batched, adjoint")
    ap.add_argument("--json-out", default=None)
    ap.add_argument("--sweep", nargs="?", const=DEFAULT_SWEEP, default=None,
                    help="instead of the headline: agent-steps/s of the plain step on a uniform cube at c2's "
                         "density for each N of a comma-separated list (one JSON line per N)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of 1 GiB five times (scales rocprof byte counters)")
    ap.add_argument("--profile-run", action="store_true",
                    help="only the roofline run, for rocprofv3: one full-build step, then 10 update-build steps")
    ap.add_argument("--summarize-profiles", nargs=6, metavar=("KT", "VALU", "FETCH", "WRITE", "COPY_FETCH",
                                                               "COPY_WRITE"),
                    help="write profiles/k_force_headline_counters.json from rocprofv3 output folders of "
                         "--profile-run (kernel trace, SQ counters, FETCH_SIZE, WRITE_SIZE) and of "
                         "--calibrate-copy (FETCH_SIZE, WRITE_SIZE)")
    args = ap.parse_args()
    if args.summarize_profiles:
        summarize_profiles(*args.summarize_profiles, block_size=args.block_size)
        return
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

    # ------------------------------------------------ headline (roofline run)
    # Section 8(d): the roofline is taken with the static test off (every
    # force evaluated); the static test's speedup is a leg of its own
    log(f"generating headline workload n={args.n}")
    w = workloads.headline(n=args.n)
    pos = torch.from_numpy(w.pos).to(dev)
    diam = torch.from_numpy(w.diam).to(dev)
    # the super-box table sized for the headline's grid (abm_params.super_fraction)
    common = dict(sort_every=args.sort_every, block_size=args.block_size, order=args.order, super_slack=1.2)
    if args.profile_run:
        sim = abm.Sim(pos, diam, detect_static=False, **common)
        sim.step(11)
        sim.sync()
        print(json.dumps({"profile_run": "headline, static test off", "steps": 11}), flush=True)
        return
    sim, el, force_ms = run_plain(pos, diam, args.steps, args.warmup, detect_static=False, **common)
    value = w.n * args.steps / el
    ms_step = 1e3 * el / args.steps
    # the phase breakdown: the next K steps, with events around every kernel
    el_ph, tm_ph = timed_steps(sim, args.steps, timing=1)
    phases = {k: tm_ph[k] / tm_ph["steps"] for k in abm.TIMED_PHASES}
    dominant = max(abm.TIMED_PHASES, key=lambda k: phases[k])
    stats = sim.stats()
    del sim
    prec = w.precision
    alg = STEP_BYTES[prec] * w.n
    ach = alg / (force_ms * 1e-3) / 1e9
    rec = counter_record(args.block_size)
    roof = dict(kernel="k_force (static flags + force + move), static test off", achieved=round(ach, 1),
                peak=HBM_PEAK_GBS, unit="GB/s", frac=round(ach / HBM_PEAK_GBS, 4), traffic=None,
                algorithmic_bytes_per_launch=alg, bytes_per_agent_step=STEP_BYTES[prec],
                avg_launch_ms=round(force_ms, 4),
                step_frac=round(value * STEP_BYTES[prec] / (HBM_PEAK_GBS * 1e9), 4),
                dominant_phase=dominant, phase_ms={k: round(v, 4) for k, v in phases.items()},
                phase_ms_note=f"the K steps after the timed ones, events around every kernel "
                              f"({1e3 * el_ph / args.steps:.4f} ms per step there)")
    bound = None
    if rec is not None:
        traffic = rec["traffic_bytes"]
        valu = rec["per_launch"]["SQ_INSTS_VALU"]
        measured_gbs = traffic / (force_ms * 1e-3) / 1e9
        valu_frac = valu / (force_ms * 1e-3 * VALU_WAVE_INSTR_PEAK)
        bound = "alu" if valu_frac > measured_gbs / HBM_PEAK_GBS else "hbm"
        roof.update(traffic=round(traffic), traffic_unit="HBM bytes per launch (FETCH_SIZE, WRITE_SIZE, scaled)",
                    measured_achieved=round(measured_gbs, 1), measured_frac=round(measured_gbs / HBM_PEAK_GBS, 4),
                    valu=dict(instructions_per_launch=round(valu), achieved=round(valu * 64 / (force_ms * 1e-3) / 1e12, 3),
                              peak=round(VALU_LANE_OPS_PEAK / 1e12, 2), unit="T VALU lane operations/s",
                              frac=round(valu_frac, 4),
                              peak_note="256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz"),
                    counters=os.path.relpath(COUNTERS_FILE, ROOT))
    roof = {"bound": bound or "alu", **roof}
    if roof["bound"] == "alu":
        roof["bound_note"] = ("achieved/peak/frac: the step's algorithmic bytes per launch against the HBM peak; the "
                              "kernel is bound by VALU issue, whose fraction is valu.frac")
    if rec is None:
        roof["bound_note"] = "counter record absent or stale for these kernel sources: bound as last measured"
    log(f"headline {value:.3e} agent-steps/s, {ms_step:.3f} ms/step, force {force_ms:.4f} ms, phases {phases}")

    extras = {}
    only = set(args.legs.split(",")) if args.legs else None
    if not args.no_extras:
        def static_leg():
            s2, el2, f2 = run_plain(pos, diam, args.steps, args.warmup, detect_static=True, **common)
            st = s2.stats()
            return dict(value=w.n * args.steps / el2, unit="agent-steps/s", ms_per_step=round(1e3 * el2 / args.steps, 4),
                        force_ms=round(f2, 4), speedup_vs_static_off=round(el / el2, 3),
                        skip_fraction_last_step=round(st["skip_fraction"], 4),
                        note="the same workload with the static test (Section 5) on; the lattice shell is "
                             "force-free and static from step 1")
        leg(extras, "static_skip", static_leg, only)

        def hilbert_leg():
            sh, elh, fh = run_plain(pos, diam, args.steps, args.warmup, detect_static=False,
                                    **{**common, "order": "hilbert"})
            return dict(value=w.n * args.steps / elh, unit="agent-steps/s", ms_per_step=round(1e3 * elh / args.steps, 4),
                        force_ms=round(fh, 4), speedup_vs_morton=round(el / elh, 3),
                        note="2x2x2 super-boxes along a Hilbert curve, Morton order inside each")
        leg(extras, "hilbert", hilbert_leg, only)

        def cadence_leg():
            # the GPU analog of the paper's agent-sorting frequency study: the
            # step after one that did not re-lay the agents out rebuilds the
            # whole grid, after a re-layout only the changed super-boxes
            out = {}
            for k in (1, 2, 5, 10, 0):
                sk, elk, fk = run_plain(pos, diam, 10, args.warmup, detect_static=False, **{**common, "sort_every": k})
                out[f"sort_every_{k}"] = dict(ms_per_step=round(1e3 * elk / 10, 4), force_ms=round(fk, 4))
                sk.close()
                del sk
            out["note"] = ("the headline workload, static test off, 10 timed steps after the warm-up; sort_every k "
                           "re-lays the agents out every k steps (0: never); a step after one without a re-layout "
                           "is a full grid build")
            return out
        leg(extras, "sort_cadence", cadence_leg, only)

        def dynamic_leg():
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
            return dict(removed=m, added=m, remove_ms=round(1e3 * (t1 - t0), 3), add_ms=round(1e3 * (t2 - t1), 3),
                        next_step_ms=round(1e3 * el_full, 3), following_step_ms=round(1e3 * el_upd, 3),
                        note="calls include their stream synchronisations; the next step's grid is a full build")
        leg(extras, "dynamic", dynamic_leg, only)
        del pos, diam
        torch.cuda.empty_cache()

        def fp64_leg():
            w64 = workloads.headline(n=args.n, dtype=np.float64)
            p64, d64 = torch.from_numpy(w64.pos).to(dev), torch.from_numpy(w64.diam).to(dev)
            s64, el64, f64 = run_plain(p64, d64, args.steps, args.warmup, detect_static=False, **common)
            v = w64.n * args.steps / el64
            return dict(value=v, unit="agent-steps/s", ms_per_step=round(1e3 * el64 / args.steps, 4),
                        force_ms=round(f64, 4), bytes_per_agent_step=STEP_BYTES["f64"],
                        frac=round(STEP_BYTES["f64"] * w64.n / (f64 * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
                        step_frac=round(v * STEP_BYTES["f64"] / (HBM_PEAK_GBS * 1e9), 4),
                        note="the headline workload with FP64 state, static test off")
        leg(extras, "headline_fp64_state", fp64_leg, only)

        def c1_density_leg():
            side = (args.n / workloads.C1_DENSITY) ** (1.0 / 3.0)
            p1, d1 = workloads.uniform_cube(args.n, side, (1, args.n), dtype=np.float32)
            pc, dc = torch.from_numpy(p1).to(dev), torch.from_numpy(d1).to(dev)
            del p1, d1
            k = max(args.steps // 4, 3)
            sc, elc, fc = run_plain(pc, dc, k, 2, detect_static=False, **common)
            return dict(value=args.n * k / elc, unit="agent-steps/s", ms_per_step=round(1e3 * elc / k, 4),
                        force_ms=round(fc, 4), steps=k,
                        note=f"1e7 spheres uniform at c1's density (side {side:.0f}, about 47 candidates and 4 "
                             f"contacts per agent), FP32 state, static test off: bound by VALU, not HBM")
        leg(extras, "c1_density_1e7", c1_density_leg, only)

        def c2_leg():
            w2 = workloads.c2()
            p2, d2 = torch.from_numpy(w2.pos).to(dev), torch.from_numpy(w2.diam).to(dev)
            s2, el2, f2 = run_plain(p2, d2, w2.steps, 3, detect_static=True, sort_every=1, block_size=args.block_size)
            return dict(value=w2.n * w2.steps / el2, unit="agent-steps/s", ms_per_step=round(1e3 * el2 / w2.steps, 4),
                        force_ms=round(f2, 4), steps=w2.steps, skip_fraction_last_step=round(s2.stats()["skip_fraction"], 4),
                        note="c2: 1e6 spheres, FP32, static test on, 100 steps after 3 untimed")
        leg(extras, "c2", c2_leg, only)

        def c3_leg():
            w3 = workloads.c3()
            p3, d3 = torch.from_numpy(w3.pos).to(dev), torch.from_numpy(w3.diam).to(dev)
            s3, el3, f3 = run_plain(p3, d3, 3, 1, detect_static=False, sort_every=10, block_size=args.block_size)
            return dict(value=w3.n * 3 / el3, unit="agent-steps/s", ms_per_step=round(1e3 * el3 / 3, 2),
                        force_ms=round(f3, 2), steps=3,
                        note="c3: 5e7 spheres in 1000 Gaussian blobs, FP32, re-layout every 10 steps; steps 2-4 "
                             "timed; about 5e3 candidates per agent, bound by VALU")
        leg(extras, "c3", c3_leg, only)

        def batched_leg():
            wb = workloads.c4()
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                pb, db = torch.from_numpy(wb.pos).to(dev), torch.from_numpy(wb.diam).to(dev)
                # each trial: 10 steps, then 10 timed, past the first steps' relaxation,
                # when agents change boxes far more often than over the whole run
                tuned = tune.autotune_batched(pb, db, wb.offsets, graph_steps=wb.steps, stream=s, warmup=10, steps=10)
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
                # (i) the same simulations, one plain context each
                kp = 10
                plain_sims = []
                for k in range(len(wb.offsets) - 1):
                    a, e = int(wb.offsets[k]), int(wb.offsets[k + 1])
                    sp = abm.Sim(pb[a:e].contiguous(), db[a:e].contiguous(), stream=s)
                    sp.step(2)
                    sp.graph_capture(kp)
                    sp.graph_launch()
                    plain_sims.append(sp)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for sp in plain_sims:
                    sp.graph_launch()
                torch.cuda.synchronize()
                elc = (time.perf_counter() - t0) / kp
                del plain_sims
            # (ii) one plain simulation of as many agents at volume fraction 0.45
            g = workloads.rng_for((4, 999))
            dd = g.uniform(8.0, 12.0, size=wb.n)
            side = (float(np.sum(np.pi / 6.0 * dd ** 3)) / 0.45) ** (1.0 / 3.0)
            pp = g.uniform(0.0, side, size=(wb.n, 3)).astype(np.float32)
            one, el1, f1 = run_plain(torch.from_numpy(pp).to(dev), torch.from_numpy(dd.astype(np.float32)).to(dev),
                                     10, 3, detect_static=False, sort_every=1, block_size=args.block_size)
            v = wb.n * wb.steps / elb
            return dict(value=v, unit="agent-steps/s", nsims=len(wb.offsets) - 1, agents=int(wb.n), steps=wb.steps,
                        launch="one hipGraph replay of 50 steps", ms_per_step=round(1e3 * elb / wb.steps, 4),
                        plain_contexts_ms_per_step=round(1e3 * elc, 4),
                        speedup_vs_plain_contexts=round(elc / (elb / wb.steps), 3),
                        one_simulation_phi045=dict(value=wb.n * 10 / el1, ms_per_step=round(1e3 * el1 / 10, 4),
                                                   force_ms=round(f1, 4)),
                        ratio_vs_one_simulation=round(v / (wb.n * 10 / el1), 3),
                        ratio_vs_headline=round(v / value, 3),
                        autotuned=tuned.params, tune_trials=len(tuned.trials),
                        untuned_ms_per_step=round(tuned.trials[0][1], 4), tuned_ms_per_step=round(tuned.ms_per_step, 4))
        leg(extras, "batched", batched_leg, only)

        def adjoint_leg():
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
            def fwd_bwd(tapes):
                a2 = abm.Sim(pa, da, sort_every=0)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                a2.forward_record(wa.steps, 10, tapes=tapes)
                xT = a2.positions().double()
                gx, gp = a2.backward(2.0 * (xT - tgt) / (3 * wa.n))
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
                peak = int(a2.ws.numel()) + int(a2.rec.numel()) + 2 * 24 * wa.n
                return el, gp, peak, a2.record_info()
            # contact tapes of every step (the default where they fit), of each
            # recomputed segment, or none (every reverse step walks a grid)
            ela, gp, peak, info = fwd_bwd("all")
            others = {t: fwd_bwd(t) for t in ("segment", "none")}
            same = all(bool(torch.equal(gp, o[1])) for o in others.values())
            del adj, plain
            # the same density with 10x the agents, where fewer kernels are
            # bound by the latency of one wave and a re-layout every step pays:
            # forward + backward (every step's tapes, after an untimed run)
            # against the plain forward, both re-laying out every step
            w6 = workloads.c5(n=1_000_000)
            p6, d6 = torch.from_numpy(w6.pos).to(dev), torch.from_numpy(w6.diam).to(dev)
            t6 = torch.from_numpy(w6.target).to(dev)
            pl6 = abm.Sim(p6, d6, sort_every=1)
            pl6.step(5)
            el6p, _ = timed_steps(pl6, w6.steps)
            del pl6
            el6 = None
            for _ in range(2):
                a6 = abm.Sim(p6, d6, sort_every=1)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                a6.forward_record(w6.steps, 10)
                x6 = a6.positions().double()
                a6.backward(2.0 * (x6 - t6) / (3 * w6.n))
                torch.cuda.synchronize()
                el6 = time.perf_counter() - t0
                info6 = a6.record_info()
                del a6
            at_1e6 = dict(agents=w6.n, value=w6.n * w6.steps / el6, plain_forward=w6.n * w6.steps / el6p,
                          ratio_vs_plain_forward=round(el6p / el6, 3), tapes=info6["tapes"], sort_every=1)
            return dict(value=wa.n * wa.steps / ela, unit="agent-steps/s (forward+backward)", agents=wa.n,
                        steps=wa.steps, ckpt_every=10, plain_forward=wa.n * wa.steps / elp,
                        ratio_vs_plain_forward=round(elp / ela, 3), dL_dk=float(gp[0]), dL_dgamma=float(gp[1]),
                        contact_tapes="every step", record_info=info,
                        by_tapes={t: dict(value=wa.n * wa.steps / o[0], ratio_vs_plain_forward=round(elp / o[0], 3),
                                          peak_device_bytes=o[2])
                                  for t, o in others.items()},
                        plain_forward_note="the plain step and the record both without re-layout (sort_every 0), "
                                           "which is faster at 1e5 agents",
                        same_gradients_all_modes=same, at_1e6_agents=at_1e6, peak_device_bytes=peak,
                        peak_note="workspace + forward record (with every step's contact tape) + dL/dx_T and "
                                  "dL/dx_0 (n x 3 doubles each)")
        leg(extras, "adjoint", adjoint_leg, only)

    cpu = None
    if not args.no_cpu:
        log("cpu baseline")
        cpu = cpu_baseline(False)

    out = {"metric": METRIC, "value": value, "unit": "agent-steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "state_dtype": prec, "data": "synthetic",
           "config": {"workload": "headline: 1e7 spheres, c2 construction (uniform inner cube + jittered "
                                  "force-free lattice shell), side 3387.7, d~U[8,12], seed 2",
                      "n": w.n, "state": prec, "arithmetic": "f64", "detect_static": False,
                      "sort_every": args.sort_every, "block_size": args.block_size, "order": args.order},
           "stats_last_step": {k: (list(v) if isinstance(v, tuple) else v) for k, v in stats.items()},
           "roofline": roof, "cpu_baseline": cpu, **extras}
    line = json.dumps(out)
    print(line, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
