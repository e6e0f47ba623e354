"""Autotuner for the launch shape of the force passes.

A launch shape is (lanes per atom, workgroup size):
  - lanes (1, 2, 4, 8, 16) sets the neighbour-list layout (strided ELL), how many lanes
    share one atom's list and so the occupancy/gather-parallelism trade-off;
  - block (256, 512 or 1024 threads) sets how many 64-atom tiles one workgroup takes,
    block / (64 lanes): the granularity of the work units the GPU schedules, the analogue
    of the paper's task list with more tasks than workers (Sec. 1.2).  Smaller
    workgroups spread a small batch over more compute units; larger ones stage the
    potential tables into LDS fewer times.
Candidates are timed on the actual system (kernel timer events around single launches, or
graph replays for batches) and the fastest is cached per key -- (device, workload or
potential, precision, atom-count class, neighbour-count class) -- in a JSON file, so a
later run with the same key takes the cached shape without timing.
"""
from __future__ import annotations

import ctypes as C
import json
import math
import os

import numpy as np

from . import _native as N

CACHE = os.environ.get("MD950_TUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "md950", "tune.json"))
LANES = (1, 2, 4, 8, 16)
BLOCKS = (256, 512, 1024)
CANDIDATES = LANES  # lanes-only searches (kept for callers that tune lanes alone)


def shapes(prec, lanes=LANES, blocks=BLOCKS):
    """The valid (lanes, block) pairs: a workgroup holds at least one 64-atom tile
    (block >= 64 lanes); FP32 takes at most 8 lanes per atom."""
    out = []
    for l in lanes:
        if prec == N.MD_FP32 and l > 8:
            continue
        for b in blocks:
            if b >= 64 * l:
                out.append((int(l), int(b)))
    return tuple(out)


def key(workload, prec, n_atoms, mean_neigh):
    """Cache key parts after the device: workload/potential, precision, atom-count class
    (nearest power of two) and neighbour-count class (nearest multiple of 16)."""
    return (workload, "fp32" if prec else "fp64", "n2^%d" % int(round(math.log2(max(1, n_atoms)))),
            "nb%d" % (int(round(mean_neigh / 16.0)) * 16))


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except Exception:
        return {}


def _store(d, path):
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path + ".tmp", "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(path + ".tmp", path)
    except OSError:
        pass


def _norm(c):
    return tuple(c) if isinstance(c, (list, tuple)) else c


def pick(key_parts, candidates, time_fn, use_cache=True, device_name=None, cache_path=None):
    """Generic tuner: time_fn(candidate) -> duration (any unit); returns the fastest
    candidate, cached per (device, key_parts).  A cached choice that is no longer among the
    candidates is ignored and the candidates are timed again."""
    if device_name is None:
        import torch
        device_name = torch.cuda.get_device_name(0)
    path = cache_path or CACHE
    k = "|".join([device_name] + [str(x) for x in key_parts])
    cands = [_norm(c) for c in candidates]
    cache = _load(path) if use_cache else {}
    if k in cache and _norm(cache[k].get("choice")) in cands:
        return _norm(cache[k]["choice"])
    results = {c: float(time_fn(c)) for c in cands}
    best = min(cands, key=lambda c: (results[c], cands.index(c)))
    cache[k] = {"choice": list(best) if isinstance(best, tuple) else best,
                "times": {str(c): v for c, v in results.items()}}
    if use_cache:
        _store(cache, path)
    return best


def time_kernels(sim, kernels, samples=10):
    """Median duration (us) of each named kernel over `samples` force evaluations."""
    L = N.lib()
    ms = C.c_float()
    out = {}
    for kname in kernels:
        acc = []
        for _ in range(samples):
            N.check(L.md_timer_arm(N.MD_KERNEL[kname]), "md_timer_arm")
            sim.forces(kick=False)
            N.check(L.md_timer_read(C.byref(ms)), "md_timer_read")
            acc.append(ms.value)
        out[kname] = 1e3 * float(np.median(acc))
    return out


def best_shape(system, prec, candidates=None, samples=10, use_cache=True, fits=None):
    """(lanes, block) with the shortest force-pass time (density + force for EAM, the LJ pass
    for LJ) on `system` itself; fits(lanes, block) may exclude shapes (e.g. ones whose
    grid exceeds the fused kick-drift's displacement slots)."""
    from .sim import Simulation

    cands = [c for c in (candidates or shapes(prec)) if fits is None or fits(*c)]
    kernels = ("lj",) if system.potential == "lj" else ("eam_density", "eam_force")
    probe = Simulation(system, precision=prec, lanes=cands[0][0], block=cands[0][1],
                       ev_cap=4).setup()
    mean_nb = probe.nl.lengths().double().mean().item()
    k = key(system.potential, prec, probe.plan.n_atoms, mean_nb)
    del probe

    def time_fn(shape):
        sim = Simulation(system, precision=prec, lanes=shape[0], block=shape[1], ev_cap=4).setup()
        return sum(time_kernels(sim, kernels, samples).values())

    return pick(k + ("shape",), cands, time_fn, use_cache=use_cache)


def best_lanes(system, prec, candidates=CANDIDATES, samples=10, use_cache=True):
    """Lanes per atom alone (default workgroups of 1024 threads)."""
    return best_shape(system, prec, [s for s in shapes(prec, candidates, (1024,))], samples,
                      use_cache)[0]
