"""Autotuner for the launch shape of the force passes.

The free parameter is the number of lanes per atom (1, 2, 4, 8, 16): it sets the
neighbour-list layout (strided ELL), the block size (64 atoms x lanes) and the
occupancy/gather parallelism trade-off.  Candidates are timed on the actual
system with the library's kernel timer (events around single launches) and the
fastest is cached per (device, potential, precision, atom-count class,
neighbour-count class) in a JSON file.
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
CANDIDATES = (1, 2, 4, 8, 16)


def _key(device_name, potential, prec, n_atoms, mean_neigh):
    return "%s|%s|%s|n2^%d|nb%d" % (device_name, potential, "fp32" if prec else "fp64",
                                    int(round(math.log2(max(1, n_atoms)))),
                                    int(round(mean_neigh / 16.0)) * 16)


def _load():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except Exception:
        return {}


def _store(d):
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        with open(CACHE + ".tmp", "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(CACHE + ".tmp", CACHE)
    except OSError:
        pass


def time_kernels(sim, kernels, samples=10):
    """Mean duration (us) of each named kernel over `samples` force evaluations."""
    L = N.lib()
    ms = C.c_float()
    out = {}
    for k in kernels:
        acc = []
        for _ in range(samples):
            N.check(L.md_timer_arm(N.MD_KERNEL[k]), "md_timer_arm")
            sim.forces(kick=False)
            N.check(L.md_timer_read(C.byref(ms)), "md_timer_read")
            acc.append(ms.value)
        out[k] = 1e3 * float(np.median(acc))
    return out


def best_lanes(system, prec, candidates=CANDIDATES, samples=10, use_cache=True):
    import torch
    from .sim import Simulation

    name = torch.cuda.get_device_name(0)
    kernels = ("lj",) if system.potential == "lj" else ("eam_density", "eam_force")
    cache = _load() if use_cache else {}
    results = {}
    key = None
    if prec == N.MD_FP32:
        candidates = tuple(c for c in candidates if c <= 8)  # FP32: 1-8 lanes per atom
    for lanes in candidates:
        sim = Simulation(system, precision=prec, lanes=lanes, ev_cap=4).setup()
        if key is None:
            mean_nb = sim.nl.lengths().double().mean().item()
            key = _key(name, system.potential, prec, sim.plan.n_atoms, mean_nb)
            if key in cache and int(cache[key]["lanes"]) in candidates:
                return int(cache[key]["lanes"])
        t = time_kernels(sim, kernels, samples)
        results[lanes] = sum(t.values())
        del sim
    best = min(results, key=results.get)
    cache[key] = {"lanes": int(best), "us": {str(k): v for k, v in results.items()}}
    if use_cache:
        _store(cache)
    return int(best)


def pick(key_parts, candidates, time_fn, use_cache=True):
    """Generic tuner: time_fn(candidate) -> duration (any unit); returns the fastest
    candidate, cached per (device, key_parts)."""
    import torch

    key = "|".join([torch.cuda.get_device_name(0)] + [str(k) for k in key_parts])
    cache = _load() if use_cache else {}
    if key in cache and cache[key].get("choice") in candidates:
        return cache[key]["choice"]
    results = {c: float(time_fn(c)) for c in candidates}
    best = min(results, key=results.get)
    cache[key] = {"choice": best, "times": {str(k): v for k, v in results.items()}}
    if use_cache:
        _store(cache)
    return best
