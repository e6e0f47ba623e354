"""Benchmark: EAM copper NVE throughput (atom-steps/s) on one MI355X.

Workload: EAM Cu, fcc 32^3 cells = 131,072 atoms, a = 3.615 A, N(0, 0.05^2) A
displacements, 300 K velocities, dt = 1 fs, skin 0.3 A (r_ns = 5.8 A), 2000-point
spline tables; velocity Verlet with neighbour lists rebuilt every k steps, k taken from a
120-step warm-up on the half-skin threshold (independent of --warmup) and the criterion
verified on every step (a run whose list went stale is void and repeated with a shorter
k); energies and virial reduced every step.  A step is the whole hot path: kick-drift +
displacement check, binning and list build when due, EAM density pass, EAM force pass
with the trailing kick and reductions (the next kick-drift fused into it).

Two GPU paths are timed: FP32-mixed (FP32 pair arithmetic and force sums, FP64
positions/integration/reductions) -- the headline `value` -- and plain FP64.
The timed region is exactly --steps steps, all of them HIP-graph replays: a graph of
whole rebuild periods (about --graph-steps steps) replayed as often as it fits and one
tail graph for the remainder, both captured before the timed region; inputs are resident
in HBM.  Kernel durations for the roofline are taken live with HIP events placed by the
library around single launches (hipExtLaunchKernelGGL).  The NVE drift comes from an
untimed run of --drift-steps steps after the timed one.

`cpu_baseline` times the FP64 O(N^2) oracle (one full step of the same state) on
the host cores; it is the only part of this script that touches the oracle.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 1000; 5000 for al_shock)")
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--graph-steps", type=int, default=50)
    ap.add_argument("--drift-steps", type=int, default=1000,
                    help="NVE steps of the untimed run whose total energy gives the drift")
    ap.add_argument("--lanes", type=int, default=0, help="lanes per atom (0: autotune)")
    ap.add_argument("--kernel-samples", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=["both", "fp32", "fp64"], default="both")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device to device a few times (the known-size "
                         "transfer that scales the FETCH_SIZE/WRITE_SIZE counters)")
    ap.add_argument("--workload", choices=["cu131k", "al_shock", "cold_curve", "force_matching",
                                           "lj13m", "nvt", "bpnn"],
                    default="cu131k",
                    help="cu131k: the headline EAM Cu NVE run; the others are the secondary "
                         "measurements (640k-atom Al shock, 64 batched cold-curve replicas, "
                         "force-matching epochs, the 13M-atom LJ test of Sec. 1.7, Cu with a "
                         "Langevin thermostat, Cu with the network potential)")
    ap.add_argument("--unfused", action="store_true",
                    help="run the kick-drift as its own pass instead of fusing it into the force "
                         "pass")
    ap.add_argument("--rebuild-every", type=int, default=-1,
                    help="rebuild period k (0: on the half-skin threshold every step; "
                         "-1: k chosen from the warm-up's rebuild intervals)")
    return ap.parse_args()


def algorithmic_force_bytes(n_atoms, mean_neigh, force_bytes, fused=False, records=False):
    """EAM force pass, per atom: list length 4 B + list 4 B/entry + own record (x, y, z,
    F') 32 B + force write 3 * force_bytes + velocity read and write 48 B (trailing kick);
    with the next kick-drift fused in, also the displacement reference read 24 B and the
    new position record written 32 B, and when it also writes the next step's FP32
    neighbour records (carried records), 16 B more.  Neighbour records are gathered from
    cache (counted in the traffic measurement)."""
    extra = (56.0 if fused else 0.0) + (16.0 if records else 0.0)
    return n_atoms * (4.0 + 4.0 * mean_neigh + 32.0 + 3.0 * force_bytes + 48.0 + extra)


FORCE_SOURCES = ("paper_2511_22951_amd/csrc/md_force.hip", "paper_2511_22951_amd/csrc/md_internal.h",
                 "paper_2511_22951_amd/csrc/md_tables.h", "include/md.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "eam_cu131k_hbm_traffic.txt")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "eam_cu131k_counters.txt")
# VALU issue ceiling: 256 CUs x 4 SIMDs, one wave64 instruction per SIMD every 4 clocks
# at 2.4 GHz (the 78.6 TFLOP/s vector peak counted per instruction: an FMA is 2 flops on
# each of 64 lanes)
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4


def strip_c_comments(text):
    """C/C++ source without its comments and blank lines (string literals in these sources
    hold no comment markers)."""
    import re
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(l.rstrip() for l in text.splitlines() if l.strip())


def force_source_digest(read=None):
    """SHA-256 of the force-pass sources with comments removed: a counter summary stays
    current while only comments change.  read(name) -> text (default: the working tree)."""
    import hashlib
    h = hashlib.sha256()
    for name in FORCE_SOURCES:
        if read is None:
            with open(os.path.join(ROOT, name)) as f:
                text = f.read()
        else:
            text = read(name)
        h.update(strip_c_comments(text).encode())
    return h.hexdigest()


def _summary_values(path, lanes):
    """The `key = value` lines of a committed counter summary, or None when the summary was
    taken for another lanes-per-atom configuration or the force-pass sources have changed
    since (its source_sha256 differs from force_source_digest())."""
    try:
        kv = {}
        with open(path) as f:
            text = f.read()
        for line in text.splitlines():
            if " = " in line:
                k, v = line.split(" = ", 1)
                kv[k.strip()] = v.strip()
        digest = force_source_digest()
    except OSError:
        return None
    if kv.get("source_sha256") != digest or kv.get("lanes") != str(lanes):
        return None
    return kv


def measured_traffic(prec_name, lanes):
    """HBM bytes per force-pass launch of the given path ("fp32"/"fp64") from the committed
    counter summary (FETCH_SIZE and WRITE_SIZE scaled by a copy calibration), or None when
    the summary was taken for another configuration or the force-pass sources have changed
    since."""
    kv = _summary_values(TRAFFIC_FILE, lanes)
    key = "k_eam_force_traffic_bytes_" + prec_name
    return float(kv[key]) if kv and key in kv else None


def measured_valu(prec_name, lanes):
    """VALU wave-instructions per force-pass launch (SQ_INSTS_VALU over the launch's waves)
    from the committed pipeline-counter summary, under the same conditions as
    measured_traffic."""
    kv = _summary_values(COUNTERS_FILE, lanes)
    key = "valu_wave_instructions_k_eam_force_" + ("f32" if prec_name == "fp32" else "f64")
    return float(kv[key]) if kv and key in kv else None


def time_kernel(md_native, kernel, run_once, samples):
    """Mean duration (ms) of one kernel over `samples` launches, each inside run_once()."""
    L = md_native.lib()
    ms = C.c_float()
    out = []
    for _ in range(samples):
        md_native.check(L.md_timer_arm(md_native.MD_KERNEL[kernel]), "md_timer_arm")
        run_once()
        md_native.check(L.md_timer_read(C.byref(ms)), "md_timer_read")
        out.append(ms.value)
    return float(np.mean(out)), float(np.std(out))


class StaleList(Exception):
    """A timed run with a fixed rebuild period k used a list past the half-skin criterion."""

    def __init__(self, k):
        super().__init__("stale list at rebuild period %d" % k)
        self.k = k


def with_valid_period(run, name=""):
    """run(k_cap) -> result dict, raising StaleList(k) when its timed run used a stale list.
    Such a run is void: it is repeated from its initial state with the period capped at
    k - 1 until one keeps every list valid.  result["retries"] counts the void runs."""
    k_cap, attempt = None, 0
    while True:
        try:
            result = run(k_cap)
            break
        except StaleList as e:
            k_cap, attempt = e.k - 1, attempt + 1
            if k_cap < 1:
                raise RuntimeError("no rebuild period kept the lists valid") from e
            print("[bench] %s: a list went stale at period %d; repeating with period %d"
                  % (name, e.k, k_cap), file=sys.stderr, flush=True)
    result["retries"] = attempt
    return result


PERIOD_WARMUP_STEPS = 120  # threshold-policy steps that choose the rebuild period (untimed)


def rebuild_period(marks, base, k_cap=None):
    """The fixed rebuild period k from a threshold-policy warm-up: marks[s] is the rebuild
    count after warm-up step s + 1, base the count before it (the lists were built just
    before step 1).  k = 4/5 of the shortest interval between builds, at most 20; with no
    threshold rebuild in the warm-up, 4/5 of its length (the lists stayed valid that long).
    k_cap bounds k (void runs).  Returns (k, warm-up steps that rebuilt)."""
    prev = [base] + list(marks[:-1])
    at = [0] + [s + 1 for s in range(len(marks)) if marks[s] > prev[s]]
    gaps = np.diff(at) if len(at) > 1 else np.array([len(marks)])
    k = int(max(1, min(20, np.floor(0.8 * gaps.min()))))
    if k_cap is not None:
        k = max(1, min(k, k_cap))
    return k, at[1:]


def timed_graph_run(sim, steps, graph_steps):
    """Exactly `steps` steps as graph replays only (Simulation.prepare_timed): a main graph
    of whole rebuild periods replayed q times and one tail graph for the remainder.  The
    graphs are captured (and the main one replayed once) before the timed region; events
    bracket every replay on the current stream.  Returns (ms, per-step ms of each replay,
    description); raises if a step ran eagerly inside the timed region."""
    import torch
    from paper_2511_22951_amd.sim import timed_graph_plan
    sim.align()
    G, q, r = timed_graph_plan(steps, sim.rebuild_every, sim.fused, graph_steps)
    plan = sim.prepare_timed(steps, graph_steps)
    if q:  # upload and warm the main graph (keeps the phase and the buffer arrangement)
        plan[0][0].replay()
        sim.n_steps += plan[0][1]
    ev_t = [torch.cuda.Event(enable_timing=True) for _ in range(len(plan) + 1)]
    torch.cuda.synchronize()
    eager0 = sim.eager_steps
    sim.replay_timed(plan, ev_t)
    torch.cuda.synchronize()
    if sim.eager_steps != eager0:
        raise RuntimeError("a step ran outside the graphs in the timed region")
    ms = ev_t[0].elapsed_time(ev_t[-1]) if plan else 0.0
    per = [ev_t[j].elapsed_time(ev_t[j + 1]) / n for j, (_, n) in enumerate(plan)]
    desc = {"graph_steps": G if q else 0, "main_replays": q, "tail_graph_steps": r,
            "eager_steps_timed": 0}
    return ms, per, desc


def run_path(system, prec, lanes, args, k_cap=None):
    import torch
    from paper_2511_22951_amd import _native as N
    from paper_2511_22951_amd.sim import Simulation

    n = system.pos.shape[0]
    cap = (PERIOD_WARMUP_STEPS + args.warmup + args.steps + args.drift_steps
           + args.kernel_samples + 2 * args.graph_steps + 64)
    sim = Simulation(system, precision=prec, lanes=lanes, ev_cap=cap,
                     fused=not args.unfused).setup()
    torch.cuda.synchronize()
    f0 = sim.state.forces()
    epot0 = float(sim.energies([0])[0][0]) / n  # step 0: the initial state
    # A threshold-policy warm-up of fixed length records when rebuilds happen; then lists
    # are rebuilt every k steps.  The half-skin criterion stays verified on every step: a
    # timed run that used a stale list raises MD_ERR_STALE_LIST, and the caller repeats the
    # path with a shorter period (k_cap).
    k = args.rebuild_every
    if k < 0:
        base, marks = sim.state.read_flags()[1]["n_rebuilds"], []
        for _ in range(PERIOD_WARMUP_STEPS):
            sim.step()
            marks.append(sim.state.read_flags()[1]["n_rebuilds"])
        k, at = rebuild_period(marks, base, k_cap)
        print("[bench] %d-step threshold warm-up: rebuilds at steps %s -> rebuild every %d steps"
              % (PERIOD_WARMUP_STEPS, at, k), file=sys.stderr, flush=True)
    sim.set_rebuild_every(k)
    sim.run(args.warmup, graph_steps=args.graph_steps)  # the --warmup steps, at period k
    torch.cuda.synchronize()
    st0 = sim.state.read_flags()[1]
    ms, per_replay, timed_desc = timed_graph_run(sim, args.steps, args.graph_steps)
    status, info = sim.state.read_flags()
    if status == N.MD_ERR_STALE_LIST and args.rebuild_every < 0:
        raise StaleList(k)
    N.check(status, "device flags after the timed run")
    rebuilds = info["n_rebuilds"] - st0["n_rebuilds"]
    # NVE drift over a run of its own (untimed, graphs): total energy per atom against time
    s0 = info["step"]
    sim.run(args.drift_steps, graph_steps=args.graph_steps)
    status, info = sim.state.read_flags()
    if status == N.MD_ERR_STALE_LIST and args.rebuild_every < 0:
        raise StaleList(k)
    N.check(status, "device flags after the drift run")
    steps = list(range(s0, info["step"] + 1))
    ev = sim.energies(steps)
    etot = (ev[:, 0] + ev[:, 7]) / n
    tps = np.array(steps) * system.dt_ps
    slope = float(np.polyfit(tps - tps[0], etot, 1)[0]) if len(steps) > 2 else None
    # live kernel timing of the EAM passes and the kick-drift kernel
    kt = {}
    knames = ("eam_force", "eam_density", "build") + (() if sim.fused else ("kick_drift",))
    for kname in knames:
        if kname == "build":  # one rebuild per sample
            kt[kname] = time_kernel(N, kname, lambda: sim.rebuild(), max(3, args.kernel_samples // 10))
        else:
            kt[kname] = time_kernel(N, kname, lambda: sim.step(), args.kernel_samples)
    nneigh = sim.nl.lengths().double().mean().item()
    rebuild_ms = _gpu_time(lambda: sim.rebuild(), 5) / 5  # binning + list, after the run
    torch.cuda.synchronize()
    return {
        "ms": ms, "steps": args.steps, "rebuilds": rebuilds, "timed": timed_desc,
        "drift_ev_per_atom_ps": slope, "drift_steps": len(steps) - 1, "epot0_per_atom": epot0,
        "energy_span_per_atom": float(np.max(etot) - np.min(etot)),
        "kernels_ms": kt, "mean_neigh": nneigh, "max_nneigh": info["max_nneigh"], "f0": f0,
        "lanes": lanes, "rebuild_every": k, "rebuild_ms": rebuild_ms,
        "replay_ms_per_step": per_replay,
        "records_carried": bool(sim.carry and sim.rebuild_every > 0),
    }


def autotune_lanes(system, prec):
    """Time the EAM force and density kernels for each lanes-per-atom option and keep the
    fastest pair (project autotuner; see paper_2511_22951_amd/tune.py)."""
    from paper_2511_22951_amd import tune
    return tune.best_lanes(system, prec)


def cpu_baseline_one_core(n_full, cells=16):
    """The same FP64 O(N^2) oracle step on one host thread, on a bounded sample: the Cu workload
    at cells^3 fcc cells (16,384 atoms by default), timed whole.  Its pair work per atom is
    m / n_full of the full box's, so the rate per atom-step scales to the full box by m / n_full;
    both figures are reported."""
    import mdinputs as mi
    from oracle import core, integrate
    core.lib()  # loads the oracle and the OpenMP runtime it links
    gomp = C.CDLL("libgomp.so.1")
    prev = core.num_threads()
    small = mi.eam_copper(cells=cells)
    pot = core.EAMPotential.from_table(small.table)
    gomp.omp_set_num_threads(1)
    try:
        threads = core.num_threads()
        x = core.wrap(small.pos, small.box)
        t0 = time.perf_counter()
        r = core.eam(x, small.box, pot)
        v = small.vel + 0.5 * small.dt_ps * r.force / small.mass * integrate.ACCEL
        x = x + small.dt_ps * v
        dt = time.perf_counter() - t0
    finally:
        gomp.omp_set_num_threads(prev)
    m = x.shape[0]
    return {"value": m / dt * m / n_full, "unit": "atom-steps/s", "cores": threads,
            "kind": "oracle", "rate_at_sample": m / dt,
            "sample": "one full FP64 O(N^2) step (density + force + Verlet) of the same Cu "
                      "workload at %d^3 cells (%d atoms) on one thread, %.1f s; the O(N^2) "
                      "work per atom scales the rate to %d atoms by %d/%d"
                      % (cells, m, dt, n_full, m, n_full)}


def cpu_baseline(system, f_gpu):
    """FP64 O(N^2) oracle: one full step (density pass, force pass, velocity Verlet) of the
    same initial state, on all host threads.  Also returns the GPU step-0 force errors."""
    from oracle import core, integrate
    pot = core.EAMPotential.from_table(system.table)
    x = core.wrap(system.pos, system.box)
    t0 = time.perf_counter()
    r = core.eam(x, system.box, pot)
    v = system.vel + 0.5 * system.dt_ps * r.force / system.mass * integrate.ACCEL
    x = x + system.dt_ps * v
    dt = time.perf_counter() - t0
    n = x.shape[0]
    errs = {k: float(np.linalg.norm(f - r.force) / np.linalg.norm(r.force))
            for k, f in f_gpu.items()}
    return {"value": n / dt, "unit": "atom-steps/s", "cores": core.num_threads(),
            "kind": "oracle",
            "sample": "one full FP64 O(N^2) step (density + force + Verlet) of all %d atoms, "
                      "%.1f s" % (n, dt)}, errs, float(r.energy / n)


def device_info():
    """The device's unit counts and memories as the runtime reports them (to confirm the
    figures the rooflines use: 256 CUs, wave64, 4 MB L2 per XCD, 160 KB LDS per CU)."""
    import torch
    p = torch.cuda.get_device_properties(0)
    return {"name": p.name, "arch": getattr(p, "gcnArchName", None),
            "compute_units": p.multi_processor_count, "wavefront": p.warp_size,
            "l2_bytes": getattr(p, "L2_cache_size", None),
            "lds_bytes_per_block": getattr(p, "shared_memory_per_block", None),
            "hbm_bytes": p.total_memory}


def copy_ceiling_gbs(mib=1024, reps=5):
    """Measured device-to-device copy rate (bytes read + written per second), the
    achievable streaming ceiling beside the 8 TB/s peak (outside any timed region)."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = float("inf")
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    return 2.0 * n * 8 / (best * 1e-3) / 1e9


def copy_calibration(mib):
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n * 8, "launches": 3}), flush=True)


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print("bench.py: this benchmark runs on one GPU; --gpus %d is not supported (run with "
              "--gpus 1)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.workload == "cu131k" and args.steps is None:
        args.steps = 1000
    if args.workload != "cu131k":
        {"al_shock": bench_al_shock, "cold_curve": bench_cold_curve,
         "force_matching": bench_force_matching, "lj13m": bench_lj_paper,
         "nvt": bench_nvt, "bpnn": bench_bpnn}[args.workload](args)
        return
    import torch
    import mdinputs as mi
    from paper_2511_22951_amd import _native as N

    N.lib()
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    system = mi.eam_copper(cells=32)
    n = system.pos.shape[0]
    results = {}
    precs = {"both": [("fp32", N.MD_FP32), ("fp64", N.MD_FP64)], "fp32": [("fp32", N.MD_FP32)],
             "fp64": [("fp64", N.MD_FP64)]}[args.precision]
    for name, prec in precs:
        lanes = args.lanes or autotune_lanes(system, prec)
        results[name] = with_valid_period(
            lambda k_cap: run_path(system, prec, lanes, args, k_cap), name)
        print("[bench] %s: %.3f ms/step, lanes %d, force kernel %.2f us" % (
            name, results[name]["ms"] / args.steps, lanes,
            1e3 * results[name]["kernels_ms"]["eam_force"][0]), file=sys.stderr, flush=True)

    head = "fp32" if "fp32" in results else "fp64"
    R = results[head]
    ms_step = R["ms"] / args.steps
    value = n * args.steps / (R["ms"] * 1e-3)

    def roofline(name):
        r = results[name]
        kt = r["kernels_ms"]["eam_force"][0] * 1e-3
        nbytes = algorithmic_force_bytes(n, r["mean_neigh"], 4 if name == "fp32" else 8,
                                         fused=not args.unfused, records=r["records_carried"])
        a = nbytes / kt / 1e9
        vi = measured_valu(name, r["lanes"])
        valu = None if vi is None else {
            "achieved": vi / kt, "peak": VALU_ISSUE_PEAK, "unit": "wave-instructions/s",
            "frac": vi / kt / VALU_ISSUE_PEAK, "instructions_per_launch": vi}
        return {"bound": "hbm", "achieved": a, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": a / HBM_PEAK_GBS, "traffic": measured_traffic(name, r["lanes"]),
                "kernel": "k_eam_force_" + ("f32" if name == "fp32" else "f64"),
                "kernel_us": kt * 1e6, "bytes_per_launch": nbytes, "valu": valu}

    f_gpu = {k: r["f0"] for k, r in results.items()}
    if args.no_cpu_baseline:
        cpu, ferr, e_or, cpu1 = None, {}, None, None
    else:
        cpu, ferr, e_or = cpu_baseline(system, f_gpu)
        cpu1 = cpu_baseline_one_core(n)

    out = {
        "metric": "atom-steps/s (EAM Cu force+Verlet) FP32 vs FP64 at stated force error",
        "value": value,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if head == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": "EAM Cu fcc 32^3 = 131072 atoms, a 3.615, 300 K, dt 1 fs, "
                               "skin 0.3, 2000-point splines, NVE velocity Verlet",
                   "n_atoms": n, "precision": head, "lanes_per_atom": R["lanes"],
                   "timed_region": R["timed"]},
        "roofline": dict(roofline(head), copy_ceiling_GBs=copy_ceiling_gbs()),
        "device": device_info(),
        "cpu_baseline": cpu,
        "cpu_baseline_one_core": cpu1,
    }
    if head != "fp64" and "fp64" in results:
        out["roofline_fp64"] = roofline("fp64")
    paths = {}
    for k, r in results.items():
        paths[k] = {"atom_steps_per_s": n * args.steps / (r["ms"] * 1e-3),
                    "ms_per_step": r["ms"] / args.steps, "lanes": r["lanes"],
                    "rebuilds": r["rebuilds"], "mean_neigh": r["mean_neigh"],
                    "kick_drift": "fused into the force pass" if not args.unfused else "own pass",
                    "records": ("carried: written by the fused kick-drift, no conversion "
                                "between rebuilds" if r["records_carried"] else
                                ("converted every step" if k == "fp32" else "none (FP64)")),
                    "rebuild_policy": ("every %d steps (4/5 of the shortest interval of a %d-step "
                                       "warm-up on the threshold), half-skin criterion verified "
                                       "every step (no violation; %d void runs repeated)"
                                       % (r["rebuild_every"], PERIOD_WARMUP_STEPS,
                                          r.get("retries", 0))
                                       if r["rebuild_every"] > 0 else "on the half-skin threshold"),
                    "timed_region": r["timed"],
                    "ms_per_step_of_each_replay": r["replay_ms_per_step"],
                    "nve_drift_eV_per_atom_ps": r["drift_ev_per_atom_ps"],
                    "nve_drift_steps": r["drift_steps"],
                    "energy_span_eV_per_atom": r["energy_span_per_atom"],
                    "kernel_us": {kk: 1e3 * v[0] for kk, v in r["kernels_ms"].items()},
                    "rebuild_us": 1e3 * r["rebuild_ms"],
                    "epot0_per_atom": r["epot0_per_atom"],
                    "energy_err_per_atom_vs_oracle": (None if e_or is None
                                                      else abs(r["epot0_per_atom"] - e_or)),
                    "force_rel_err_vs_oracle": ferr.get(k)}
    if "fp32" in results and "fp64" in results:
        paths["fp32"]["force_rel_err_vs_fp64_gpu"] = float(
            np.linalg.norm(results["fp32"]["f0"] - results["fp64"]["f0"])
            / np.linalg.norm(results["fp64"]["f0"]))
        paths["speedup_fp32_over_fp64"] = results["fp64"]["ms"] / results["fp32"]["ms"]
    if e_or is not None:
        paths["oracle_epot0_per_atom"] = e_or
    out["paths"] = paths
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------------------
# Secondary measurements (each prints its own JSON line)
# ---------------------------------------------------------------------------
def _gpu_time(fn, reps):
    """Wall time (ms) of `reps` calls of fn() on the current stream, events on that stream."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def _replay_graph(fn, warm=2):
    """Capture fn() once into a HIP graph (after `warm` eager calls) and return replay()."""
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    return g.replay, g


def bench_al_shock(args):
    """640,000-atom Al shock (fcc 20x20x400, piston 1 km/s, top wall), FP32-mixed forces,
    rebuilds on the half-skin threshold (predicated rebuild kernels every step)."""
    import torch
    import mdinputs as mi
    from paper_2511_22951_amd import _native as N
    from paper_2511_22951_amd.sim import Simulation
    N.lib()
    system = mi.eam_aluminum_shock()
    n = system.pos.shape[0]
    steps = args.steps or system.n_steps
    lanes = args.lanes or autotune_lanes(system, N.MD_FP32)
    cap = args.warmup + steps + args.kernel_samples + 2 * args.graph_steps + 64
    sim = Simulation(system, precision=N.MD_FP32, lanes=lanes, max_neigh=160, ev_cap=cap,
                     rebuild_every=0, fused=not args.unfused).setup()
    sim.run(args.warmup, graph_steps=args.graph_steps)
    torch.cuda.synchronize()
    st0 = sim.state.read_flags()[1]
    ms, _, timed_desc = timed_graph_run(sim, steps, args.graph_steps)
    status, info = sim.state.read_flags()
    N.check(status, "device flags after the timed run")
    kt = {}
    for kname in ("eam_force", "eam_density") + (() if sim.fused else ("kick_drift",)):
        kt[kname] = time_kernel(N, kname, lambda: sim.step(), args.kernel_samples)[0]
    nn = sim.nl.lengths().double()
    zc = sim.state.positions()[:, 2]
    # analysis path (Appendix): per-atom energy and virial, then 257 slab profiles along z
    from paper_2511_22951_amd import md
    obs = {}
    obs_ms = _gpu_time(lambda: obs.update(
        zip("ewr", md.md_atom_observables(sim.state, sim.nl, eam=sim.pot))), 5) / 5
    lz, nb = system.box.len[2] + 1.0, 257
    pws = torch.empty(int(N.lib().md_profile_workspace_bytes(nb)), dtype=torch.uint8,
                      device="cuda")
    prof_ms = _gpu_time(lambda: md.md_profiles(sim.state, 2, 0.0, lz / nb, nb, system.mass,
                                               obs["e"], obs["w"], ws=pws), 5) / 5
    rebuild_ms = _gpu_time(lambda: sim.rebuild(), 5) / 5
    kt_force = kt["eam_force"] * 1e-3
    bytes_force = algorithmic_force_bytes(n, nn.mean().item(), 4, fused=sim.fused)
    achieved = bytes_force / kt_force / 1e9
    out = {
        "metric": "atom-steps/s (EAM Al shock, FP32-mixed forces, FP64 integration)",
        "value": n * steps / (ms * 1e-3), "unit": "atom-steps/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": ms / steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "EAM Al fcc 20x20x400 = 640000 atoms, a 4.05, 300 K, piston "
                               "1 km/s at z = 0, top wall, periodic x/y, dt 1 fs, skin 0.3, "
                               "half-skin rebuilds", "n_atoms": n, "lanes_per_atom": lanes,
                   "graph_steps": args.graph_steps},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_eam_force",
                     "kernel_us": kt_force * 1e6, "bytes_per_launch": bytes_force},
        "rebuilds": info["n_rebuilds"] - st0["n_rebuilds"],
        "neighbours": {"mean": nn.mean().item(), "max": int(nn.max().item()),
                       "min": int(nn.min().item())},
        "piston_z_end": float(system.walls["piston_v"] * info["step"] * system.dt_ps),
        "atoms_min_z": float(zc.min()),
        "kernel_us": {k: 1e3 * v for k, v in kt.items()},
        "rebuild_us": 1e3 * rebuild_ms,
        "analysis_us": {"atom_observables_fp64": 1e3 * obs_ms,
                        "profiles_257_slabs": 1e3 * prof_ms},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        from oracle import core, profiles
        o = np.argsort(sim.state.id.cpu().numpy(), kind="stable")
        x, v = sim.state.positions(), sim.state.velocities()
        sample = np.random.default_rng(5).choice(n, 64, replace=False)
        t0 = time.perf_counter()
        core.eam_sampled(x, system.box, core.EAMPotential.from_table(system.table), sample)
        t_f = time.perf_counter() - t0
        e_h, w_h = obs["e"].cpu().numpy()[o], obs["w"].cpu().numpy().T[o]
        t0 = time.perf_counter()
        profiles.profiles(x, v, system.mass, e_h, w_h, system.box, 2, 0.0, lz / nb, nb)
        t_p = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": len(sample) / t_f, "unit": "atom-steps/s (forces only)",
            "cores": core.num_threads(), "kind": "oracle",
            "sample": "FP64 O(N) EAM force sums of %d sampled atoms over all %d atoms, %.1f s; "
                      "the oracle's 257 slab profiles of the same state took %.2f s"
                      % (len(sample), n, t_f, t_p)}
    print(json.dumps(out), flush=True)


def bench_lj_paper(args):
    """The LJ performance test of Sec. 1.7 at its size on one GPU: 12,967,168 Ar atoms
    (periodic fcc 148^3, small perturbations), 300 steps, lists rebuilt every 10 steps;
    FP64 and FP32-mixed paths, both with HIP-graph replay."""
    import torch
    import mdinputs as mi
    from paper_2511_22951_amd import _native as N
    from paper_2511_22951_amd.sim import Simulation
    N.lib()
    system = mi.lj_argon_benchmark()
    n = system.pos.shape[0]
    steps = args.steps or system.n_steps
    k = system.extra["rebuild_every"]
    gs = max(k, args.graph_steps // k * k)
    warm = max(k, args.warmup // k * k)
    sample = np.random.default_rng(7).choice(n, 256, replace=False)
    paths, f_gpu = {}, {}
    from paper_2511_22951_amd import tune
    from paper_2511_22951_amd.sim import fused_grid_fits
    n_tiles = sum((c + 63) // 64 for c in [n])
    for name, prec in (("fp32", N.MD_FP32), ("fp64", N.MD_FP64)):
        if args.precision not in ("both", name):
            continue
        # the fused kick-drift needs a force-pass grid within its displacement slots
        cands = tuple(l for l in tune.CANDIDATES
                      if args.unfused or fused_grid_fits(n_tiles, l))
        lanes = args.lanes or tune.best_lanes(system, prec, candidates=cands)
        cap = warm + steps + args.kernel_samples + 2 * gs + 64
        sim = Simulation(system, precision=prec, lanes=lanes, max_neigh=112, ev_cap=cap,
                         rebuild_every=k, fused=not args.unfused).setup()
        f_gpu[name] = sim.state.forces()[sample]
        sim.run(warm, graph_steps=gs)
        torch.cuda.synchronize()
        st0 = sim.state.read_flags()[1]
        ms, _, timed_desc = timed_graph_run(sim, steps, gs)
        status, info = sim.state.read_flags()
        N.check(status, "device flags after the timed run")
        ev = sim.energies(range(st0["step"], info["step"] + 1))
        etot = (ev[:, 0] + ev[:, 7]) / n
        kt = {kn: 1e3 * time_kernel(N, kn, lambda: sim.step(), args.kernel_samples // 5)[0]
              for kn in ("lj",) + (() if sim.fused else ("kick_drift",))}
        kt["build"] = 1e3 * time_kernel(N, "build", lambda: sim.rebuild(), 3)[0]
        nn = sim.nl.lengths().double()
        force_bytes = 4 if prec == N.MD_FP32 else 8
        # list length 4 + list 4 n + own record 32 + force + v read/write 48; with the next
        # kick-drift fused in, x_ref 24 and the new position record 32
        per_atom = (4.0 + 4.0 * nn.mean().item() + 32.0 + 3.0 * force_bytes + 48.0
                    + (56.0 if sim.fused else 0.0))
        paths[name] = {
            "atom_steps_per_s": n * steps / (ms * 1e-3), "ms_per_step": ms / steps,
            "lanes": lanes, "rebuilds": info["n_rebuilds"] - st0["n_rebuilds"],
            "mean_neigh": nn.mean().item(), "max_neigh": int(nn.max().item()),
            "energy_span_eV_per_atom": float(etot.max() - etot.min()),
            "kernel_us": kt, "lj_bytes_per_launch": n * per_atom,
            "lj_achieved_GBs": n * per_atom / (kt["lj"] * 1e-6) / 1e9,
        }
        del sim
        torch.cuda.empty_cache()
    head = paths.get("fp32") or paths["fp64"]
    out = {
        "metric": "atom-steps/s (LJ, 300 steps, lists rebuilt every 10 steps)",
        "value": head["atom_steps_per_s"], "unit": "atom-steps/s", "n_gpus": 1, "steps": steps,
        "warmup": warm, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if "fp32" in paths else "f64", "data": "synthetic",
        "config": {"workload": "LJ Ar fcc 148^3 = 12967168 atoms, a 5.26, N(0, 0.05^2) "
                               "displacements, 100 K, dt 2 fs, r_c 2.5 sigma, skin 0.5, "
                               "rebuild every 10 steps", "n_atoms": n, "graph_steps": gs},
        "roofline": {"bound": "hbm", "achieved": head["lj_achieved_GBs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": head["lj_achieved_GBs"] / HBM_PEAK_GBS,
                     "traffic": None, "kernel": "k_lj", "kernel_us": head["kernel_us"]["lj"],
                     "bytes_per_launch": head["lj_bytes_per_launch"]},
        "paths": paths,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        from oracle import core
        lj = system.lj
        t0 = time.perf_counter()
        r = core.lj_sampled(system.pos, system.box, lj.eps, lj.sigma, lj.r_cut, sample)
        dt = time.perf_counter() - t0
        for name, f in f_gpu.items():
            paths[name]["force_rel_err_vs_oracle_sampled"] = float(
                np.linalg.norm(f - r.force) / np.linalg.norm(r.force))
        out["cpu_baseline"] = {
            "value": len(sample) / dt, "unit": "atom-steps/s (forces only)",
            "cores": core.num_threads(), "kind": "oracle",
            "sample": "FP64 O(N) force sums of %d sampled atoms over all %d atoms, %.1f s"
                      % (len(sample), n, dt)}
    print(json.dumps(out), flush=True)


def bench_nvt(args):
    """EAM Cu 131,072 atoms, FP32-mixed forces, NVT: the Langevin update of the whole box
    (300 K, stiffness 0.5/ps as in Secs. 3.2-3.3) before every half kick, lists rebuilt
    every 9 steps; beside the same run without the thermostat.  The kick-drift (with the
    Langevin update) is fused into the force pass, as in the NVE benchmark; --unfused runs
    it as its own kernel in both runs."""
    import torch
    import mdinputs as mi
    from paper_2511_22951_amd import _native as N
    from paper_2511_22951_amd.sim import Simulation
    N.lib()
    system = mi.eam_copper(cells=32)
    n = system.pos.shape[0]
    steps = args.steps or 1000
    k = args.rebuild_every if args.rebuild_every > 0 else 9
    fused = not args.unfused
    period = 2 * k if fused and k % 2 else k
    gs = max(2 * period, args.graph_steps // period * period)
    lanes = args.lanes or autotune_lanes(system, N.MD_FP32)
    lang = {"seed": 2511, "regions": [{"T": 300.0, "gamma": 0.5}]}
    res = {}
    kname = "eam_force" if fused else "kick_drift"
    for name, thermo in (("nvt", lang), ("nve", None)):
        cap = args.warmup + steps + args.kernel_samples + 2 * gs + 64
        sim = Simulation(system, precision=N.MD_FP32, lanes=lanes, ev_cap=cap, rebuild_every=k,
                         thermostat=thermo, fused=fused).setup()
        sim.run(args.warmup, graph_steps=gs)
        torch.cuda.synchronize()
        st0 = sim.state.read_flags()[1]
        ms, _, timed_desc = timed_graph_run(sim, steps, gs)
        status, info = sim.state.read_flags()
        N.check(status, "device flags after the timed run")
        ev = sim.energies(range(info["step"] - steps + 1, info["step"] + 1))
        temps = 2.0 * ev[:, 7] / ((3 * n - 3) * 8.617333262e-5)
        kt = time_kernel(N, kname, lambda: sim.step(), args.kernel_samples)[0]
        nn = sim.nl.lengths().double().mean().item()
        res[name] = {"atom_steps_per_s": n * steps / (ms * 1e-3), "ms_per_step": ms / steps,
                     kname + "_us": 1e3 * kt, "mean_T_K": float(temps.mean()),
                     "rebuilds": info["n_rebuilds"] - st0["n_rebuilds"], "mean_neigh": nn,
                     "kick_drift": "fused into the force pass" if fused else "own kernel"}
        del sim
    if fused:
        # the force pass with the kick-drift fused in (and the next step's FP32 records),
        # plus the atom id the thermostat reads
        nbytes = algorithmic_force_bytes(n, res["nvt"]["mean_neigh"], 4, fused=True,
                                         records=True) + 4.0 * n
        kernel = "k_eam_force_f32 (Langevin update and kick-drift fused)"
    else:
        # kick-drift traffic per atom: read v 24, f 12, x 32, x_ref 24 (and id 4 with the
        # thermostat); write v 24, x 32
        nbytes = n * (148.0 + 4.0)
        kernel = "k_kick_drift (Langevin)"
    kus = res["nvt"][kname + "_us"]
    achieved = nbytes / (kus * 1e-6) / 1e9
    out = {
        "metric": "atom-steps/s (EAM Cu NVT, Langevin thermostat)",
        "value": res["nvt"]["atom_steps_per_s"], "unit": "atom-steps/s", "n_gpus": 1,
        "steps": steps, "warmup": args.warmup, "ms_per_step": res["nvt"]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "EAM Cu fcc 32^3 = 131072 atoms, 300 K, dt 1 fs, skin 0.3, "
                               "Langevin 300 K / 0.5 per ps over the whole box, rebuild every "
                               "%d steps" % k, "n_atoms": n, "lanes_per_atom": lanes,
                   "graph_steps": gs, "fused_kick_drift": fused},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": kernel,
                     "kernel_us": kus, "bytes_per_launch": nbytes},
        "paths": res,
        "thermostat_cost": res["nvt"]["ms_per_step"] / res["nve"]["ms_per_step"] - 1.0,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        from oracle import core, thermostat
        sample = np.random.default_rng(6).choice(n, 64, replace=False)
        t0 = time.perf_counter()
        core.eam_sampled(system.pos, system.box, core.EAMPotential.from_table(system.table),
                         sample)
        t_f = time.perf_counter() - t0
        t0 = time.perf_counter()
        thermostat.o_step(system.pos, system.vel, np.arange(n), 1, lang, system.mass,
                          system.dt_ps)
        t_o = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": len(sample) / (t_f + t_o * len(sample) / n),
            "unit": "atom-steps/s (forces and Langevin update)", "cores": core.num_threads(),
            "kind": "oracle",
            "sample": "FP64 O(N) EAM force sums of %d sampled atoms (%.1f s) plus their share of "
                      "the oracle's Langevin update of all %d atoms (%.2f s in all)"
                      % (len(sample), t_f, n, t_o)}
    print(json.dumps(out), flush=True)


FP64_VALU_PEAK_TFLOPS = 78.6


def bench_bpnn(args):
    """Behler-Parrinello network potential (Sec. 2.1) on Cu fcc 32^3 = 131,072 atoms, FP64:
    NVE steps with threshold rebuilds, HIP-graph replay."""
    import torch
    import mdinputs as mi
    from paper_2511_22951_amd import _native as N
    from paper_2511_22951_amd.sim import Simulation
    N.lib()
    system = mi.bpnn_copper(cells=32)
    n = system.pos.shape[0]
    steps = args.steps or 100
    warm = min(args.warmup, 20)
    gs = min(args.graph_steps, 10)
    lanes = args.lanes or 4
    sim = Simulation(system, precision=N.MD_FP64, lanes=lanes, ev_cap=warm + steps + 2 * gs + 64).setup()
    sim.run(warm, graph_steps=gs)
    torch.cuda.synchronize()
    st0 = sim.state.read_flags()[1]
    ms, _, timed_desc = timed_graph_run(sim, steps, gs)
    status, info = sim.state.read_flags()
    N.check(status, "device flags after the timed run")
    ev = sim.energies(range(st0["step"] + 1, info["step"] + 1))
    etot = (ev[:, 0] + ev[:, 7]) / n
    kt = {k: 1e3 * time_kernel(N, k, lambda: sim.step(), 5)[0] for k in ("bpnn_desc", "bpnn_force")}
    # ordered neighbour pairs within r_c (the angular terms' work), counted from the list
    # (which holds the neighbours within r_c + skin) at the final positions
    x = sim.state.pos[:, :3]
    p = system.extra["bpnn"]
    nn = sim.nl.lengths().double().mean().item()
    lst = sim.nl
    raw = lst.neigh.view(lst.max_neigh // lst.lanes, lst.npad, lst.lanes)
    cnt = lst.lengths().long()
    m = torch.arange(lst.max_neigh, device="cuda")
    ent = raw[m // lst.lanes][:, :n, :].gather(2, (m % lst.lanes).view(-1, 1, 1).expand(-1, n, 1))
    ent = ent.squeeze(2).t()  # [n, max_neigh]
    valid = m.view(1, -1) < cnt.view(-1, 1)
    d = x[ent.clamp(min=0).long()] - x.view(n, 1, 3)
    ln = torch.tensor(system.box.len, dtype=torch.float64, device="cuda")
    d -= ln * torch.round(d / ln)
    within = ((d * d).sum(-1) < p["r_cut"] ** 2) & valid
    m_rc = within.sum(1).double()
    pairs = float((m_rc * (m_rc - 1.0)).sum().item())
    grid = len(p["g4_eta"])
    flops = pairs * grid * (2 + 7)  # grid multiply-adds of the two passes per ordered pair
    t_s = (kt["bpnn_desc"] + kt["bpnn_force"]) * 1e-6
    achieved = flops / t_s / 1e12
    out = {
        "metric": "atom-steps/s (Cu, Behler-Parrinello network potential, FP64)",
        "value": n * steps / (ms * 1e-3), "unit": "atom-steps/s", "n_gpus": 1, "steps": steps,
        "warmup": warm, "ms_per_step": ms / steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic (random network weights)",
        "config": {"workload": "Cu fcc 32^3 = 131072 atoms, a 3.615, 300 K, dt 1 fs, r_c 6, "
                               "skin 0.3, 8 G2 + 43 G4, network 51-10-10-1 (tanh)",
                   "n_atoms": n, "lanes_per_atom": lanes, "graph_steps": gs},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VALU_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_VALU_PEAK_TFLOPS,
                     "traffic": None, "kernel": "k_bpnn_desc + k_bpnn_force",
                     "kernel_us": kt["bpnn_desc"] + kt["bpnn_force"],
                     "flops_per_launch": flops},
        "kernel_us": kt, "mean_list_len": nn, "ordered_pairs_per_atom": pairs / n,
        "nve_energy_span_eV_per_atom": float(etot.max() - etot.min()),
        "rebuilds": info["n_rebuilds"] - st0["n_rebuilds"],
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        from oracle import bpnn, core
        small = mi.bpnn_copper(cells=4)
        t0 = time.perf_counter()
        bpnn.forces(small.pos, small.box, small.extra["bpnn"])
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": small.pos.shape[0] / dt, "unit": "atom-steps/s (energy and forces)",
            "cores": 1, "kind": "oracle",
            "sample": "energy and forces of the 256-atom Cu box (4^3 cells, same potential) by "
                      "the numpy oracle, %.1f s" % dt}
    print(json.dumps(out), flush=True)


def _static_batch(reps, prec, lanes, max_neigh=128, block=0):
    from paper_2511_22951_amd import md
    plan = md.Plan([r.box for r in reps], [len(r.pos) for r in reps], 5.8)
    st = md.State(plan, np.concatenate([r.pos for r in reps]), None, prec)
    nl = md.NeighborList(plan.n_atoms, max_neigh, lanes, block=block)
    md.md_bin_cells(st)
    md.md_build_neighbors(st, nl)
    return plan, st, nl


def bench_cold_curve(args):
    """64 perfect Cu replicas (4^3..12^3 cells, a = 3.30..4.20): energy, forces and virial of
    every replica per evaluation.  Batched (one launch per pass over all replicas, HIP graph)
    against a per-replica loop (64 launches per pass, also in a graph); FP32 and FP64."""
    import torch
    import mdinputs as mi
    from paper_2511_22951_amd import _native as N
    from paper_2511_22951_amd import md, tune
    N.lib()
    reps = mi.cold_curve_replicas()
    n_tot = sum(len(r.pos) for r in reps)
    tab = mi.tabulate_eam(mi.EAM_CU)
    pot = md.EAMPotential.from_table(tab)
    reps_per_eval = len(reps)
    evals = max(20, (args.steps or 1000) // 10)
    res = {}
    e_gpu = {}
    for name, prec in (("fp32", N.MD_FP32), ("fp64", N.MD_FP64)):
        table = pot.table(prec)

        def batched(shape):
            plan, st, nl = _static_batch(reps, prec, shape[0], block=shape[1])
            ev = md.ev_buffer(1, len(reps))
            fn = lambda: md.md_eam_forces(st, pot, nl, table=table, ev=ev)
            return fn, (plan, st, nl, ev)

        def timed(shape):
            fn, keep = batched(shape)
            replay, g = _replay_graph(fn)
            return _gpu_time(replay, 10) / 10

        # launch shape: (lanes per atom, workgroup size) from the project's tuner, beside the
        # fixed default shape (4 lanes, 1024 threads)
        fixed = (4, 1024)
        shape = (args.lanes, 1024) if args.lanes else tune.pick(
            ("cold_curve64", name, "shape"), tune.shapes(prec), timed)
        fn, (plan, st, nl, ev) = batched(shape)
        replay, g = _replay_graph(fn)
        t_b = _gpu_time(replay, evals) / evals
        if shape != fixed:
            fn_f, keep_f = batched(fixed)
            replay_f, g_f = _replay_graph(fn_f)
            t_fixed = _gpu_time(replay_f, evals) / evals
            del g_f, keep_f
        else:
            t_fixed = t_b
        lanes = shape[0]
        st.check_flags()
        e = md.ev_values(ev)[0]
        e_gpu[name] = (e[:, 0], st)
        # per-replica loop: one plan/state/list per replica, 64 launches per evaluation
        singles = []
        for r in reps:
            p1, s1, n1 = _static_batch([r], prec, lanes, block=shape[1])
            singles.append((s1, n1, md.ev_buffer(1, 1)))

        def loop():
            for s1, n1, ev1 in singles:
                md.md_eam_forces(s1, pot, n1, table=table, ev=ev1)

        replay_l, g_l = _replay_graph(loop)
        t_l = _gpu_time(replay_l, evals) / evals
        res[name] = {"ms_per_eval_batched": t_b, "ms_per_eval_loop": t_l,
                     "replica_evals_per_s": reps_per_eval / (t_b * 1e-3),
                     "atom_evals_per_s": n_tot / (t_b * 1e-3),
                     "batched_speedup_over_loop": t_l / t_b, "lanes": lanes,
                     "tuned_shape": {"lanes": shape[0], "block": shape[1]},
                     "ms_per_eval_fixed_shape_4x1024": t_fixed,
                     "tuned_speedup_over_fixed_shape": t_fixed / t_b,
                     "max_abs_force": float(np.max(np.abs(st.forces())))}
        del g, g_l
    per_atom = np.array([len(r.pos) for r in reps], np.float64)
    de32 = np.abs(e_gpu["fp32"][0] - e_gpu["fp64"][0]) / per_atom
    res["fp32"]["max_energy_err_vs_fp64_gpu_eV_per_atom"] = float(de32.max())
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import core
        opot = core.EAMPotential.from_table(tab)
        t0 = time.perf_counter()
        e_or = np.array([core.eam(r.pos, r.box, opot).energy for r in reps])
        dt = time.perf_counter() - t0
        cpu = {"value": len(reps) / dt, "unit": "replica-evals/s", "cores": core.num_threads(),
               "kind": "oracle",
               "sample": "one FP64 O(N^2) evaluation of all 64 replicas (%d atoms), %.1f s"
                         % (n_tot, dt)}
        for name in ("fp32", "fp64"):
            res[name]["max_energy_err_vs_oracle_eV_per_atom"] = float(
                np.max(np.abs(e_gpu[name][0] - e_or) / per_atom))
    head = res["fp32"]
    out = {
        "metric": "replica-evals/s (64 batched Cu cold-curve replicas: energy, forces, virial)",
        "value": head["replica_evals_per_s"], "unit": "replica-evals/s", "n_gpus": 1,
        "steps": evals, "warmup": 2, "ms_per_step": head["ms_per_eval_batched"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "64 perfect Cu fcc replicas, n^3 cells with n drawn from "
                               "4..12, a = linspace(3.30, 4.20, 64), EAM Cu 2000-point splines",
                   "n_atoms": n_tot},
        "paths": res,
        "speedup_fp32_over_fp64": res["fp64"]["ms_per_eval_batched"] / head["ms_per_eval_batched"],
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def bench_force_matching(args):
    """Force matching on 1024 Cu snapshots of 500 atoms: forward (forces of the trainable
    splines), loss and hand-written adjoint per epoch; adjoint vs FP64 central differences."""
    import torch
    import mdinputs as mi
    from paper_2511_22951_amd import _native as N
    from paper_2511_22951_amd import fm, md
    N.lib()
    tab = mi.force_matching_tables()
    noise = torch.as_tensor(mi.coefficient_noise(), device="cuda")
    snaps = mi.force_matching_snapshots()
    n_atoms = sum(len(s.pos) for s in snaps)
    fits = [md.md_spline_fit(tf.y, tf.h, tf.dy_lo, tf.dy_hi) for tf in (tab.phi, tab.rho, tab.emb)]
    res = {}
    for name, prec in (("fp64", N.MD_FP64), ("fp32", N.MD_FP32)):
        pot = md.EAMPotential(fits[0] * noise[:64], fits[1] * noise[64:128], fits[2] * noise[128:],
                              tab.rho.x_lo, tab.rho.h, tab.emb.x_lo, tab.emb.h, mi.EAM_CU.r_cut)
        batch = fm.SnapshotBatch(snaps, mi.EAM_CU.r_cut + 0.3, precision=prec)
        ref_pot = md.EAMPotential.from_table(mi.tabulate_eam(mi.EAM_CU))
        f_ref = batch.forces(ref_pot, saved=False).clone()
        coef = torch.cat([c.clone() for c in pot.coef]).requires_grad_(True)

        def epoch():
            coef.grad = None
            loss = fm.force_matching_loss(coef, batch, pot, f_ref)
            loss.backward()
            return loss

        for _ in range(3):
            epoch()
        reps = max(10, (args.steps or 1000) // 50)
        ms = _gpu_time(epoch, reps) / reps
        loss = epoch().item()
        g = coef.grad.detach().cpu().numpy()
        batch.state.check_flags()
        r = {"ms_per_epoch": ms, "epochs_per_s": 1e3 / ms, "atoms_per_s": n_atoms / (ms * 1e-3),
             "loss": loss}
        if prec == N.MD_FP64:
            h = 1e-6
            errs = []
            for k in (5, 20, 40, 64 + 10, 64 + 40, 128 + 20, 128 + 33, 128 + 50):
                cp = coef.detach().clone()
                cm = coef.detach().clone()
                cp[k] += h
                cm[k] -= h
                lp = fm.force_matching_loss(cp, batch, pot, f_ref).item()
                lm = fm.force_matching_loss(cm, batch, pot, f_ref).item()
                errs.append(abs((lp - lm) / (2 * h) - g[k]))
            r["adjoint_vs_fd_max_abs_err"] = float(max(errs))
            r["adjoint_vs_fd_rel_to_max_grad"] = float(max(errs) / np.max(np.abs(g)))
            res["grad_fp64"] = g
        else:
            r["grad_rel_err_vs_fp64_gpu"] = float(np.max(np.abs(g - res["grad_fp64"]))
                                                  / np.max(np.abs(res["grad_fp64"])))
        res[name] = r
    res.pop("grad_fp64")
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import adjoint as oadj
        from oracle import core
        from oracle import spline as osp
        sample = 16
        grids = tuple(oadj.Grid(tf.x_lo, tf.h, tf.K + 2) for tf in (tab.phi, tab.rho, tab.emb))
        nz = noise.cpu().numpy()
        c_or = [osp.fit_table(tf) * nz[64 * b:64 * (b + 1)]
                for b, tf in enumerate((tab.phi, tab.rho, tab.emb))]
        osn = [oadj.Snapshot(s.pos, s.box, mi.EAM_CU.r_cut) for s in snaps[:sample]]
        apot = core.EAMPotential.analytic(mi.EAM_CU)
        t0 = time.perf_counter()
        f_ref_or = [core.eam(s.pos, s.box, apot).force for s in snaps[:sample]]
        oadj.gradient(osn, c_or, grids, f_ref_or)
        dt = time.perf_counter() - t0
        cpu = {"value": sample / len(snaps) / dt, "unit": "epochs/s", "cores": core.num_threads(),
               "kind": "oracle",
               "sample": "reference forces, loss and chain-rule gradient of %d of the %d "
                         "snapshots, %.1f s, scaled to one epoch" % (sample, len(snaps), dt)}
    out = {
        "metric": "force-matching epochs/s (1024 Cu snapshots x 500 atoms, forward + adjoint)",
        "value": res["fp64"]["epochs_per_s"], "unit": "epochs/s", "n_gpus": 1,
        "steps": max(10, (args.steps or 1000) // 50), "warmup": 3, "ms_per_step": res["fp64"]["ms_per_epoch"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "1024 Cu fcc 5^3 snapshots, a ~ U(3.55, 3.68), N(0, 0.1^2) "
                               "displacements; 3 x 64 B-spline coefficients with 5% noise",
                   "n_atoms": n_atoms},
        "paths": res, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
