"""Langevin thermostat (oracle; test infrastructure only).

Sec. 1.5: a Langevin force added to the right-hand side of eq. 1.5 turns the NVE
integration into NVT.  Sec. 3.1 applies it to slabs of the sample, each with a
target temperature T, a mean velocity u and a stiffness (read here as the
friction coefficient gamma, in 1/ps):

    m dv/dt = f - m gamma (v - u) + sqrt(2 m gamma k_B T) eta(t).

The paper gives no discretisation.  This oracle takes the exact solution of the
Ornstein-Uhlenbeck part over one step,

    v <- u + c1 (v - u) + c2 xi,   c1 = exp(-gamma dt),   c2 = sqrt((1 - c1^2) k_B T / m),

applied once per step before the first half kick (the OBABO splitting of Bussi
and Parrinello, Phys. Rev. E 75, 056707 (2007), with its two half-step O parts
merged), followed by the velocity Verlet step of integrate.run_nve.

xi: three standard normals per atom and step.  Their source is a counter-based
generator, so that any implementation can reproduce them from (seed, step, id):
Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC'11) with counter {id, step, 0, 0} and key {seed low 32 bits,
seed high 32 bits}; its four output words w0..w3 give, by the Box-Muller
transform with U_k = (w_k + 1) 2^-32 (k = 0, 2) and U_k = w_k 2^-32 (k = 1, 3),
xi_x = sqrt(-2 ln U0) cos(2 pi U1), xi_y = sqrt(-2 ln U0) sin(2 pi U1),
xi_z = sqrt(-2 ln U2) cos(2 pi U3).  step counts from 1 for the first step.
"""
from __future__ import annotations

import numpy as np

from . import core
from .integrate import ACCEL, apply_walls, kinetic_energy

KB = 8.617333262e-5  # eV/K (CODATA 2018)

_M0, _M1 = 0xD2511F53, 0xCD9E8D57     # Philox4x32 round multipliers
_W0, _W1 = 0x9E3779B9, 0xBB67AE85     # Weyl key increments
_MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds.  ctr: uint array [..., 4], key: uint array [..., 2]
    (broadcast).  Each round: (hi0, lo0) = M0 * c0, (hi1, lo1) = M1 * c2 as 64-bit
    products; c <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); between rounds the key
    gains (W0, W1) modulo 2^32."""
    c = np.array(ctr, dtype=np.uint64) & _MASK
    k = np.array(key, dtype=np.uint64) & _MASK
    c0, c1, c2, c3 = c[..., 0], c[..., 1], c[..., 2], c[..., 3]
    k0, k1 = k[..., 0], k[..., 1]
    for r in range(10):
        if r > 0:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = np.uint64(_M0) * c0
        p1 = np.uint64(_M1) * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(_MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(_MASK)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint64)


def normals(seed, step, ids):
    """[len(ids), 3] standard normals of the given atoms for one step (Box-Muller)."""
    ids = np.asarray(ids, dtype=np.uint64)
    ctr = np.zeros(ids.shape + (4,), dtype=np.uint64)
    ctr[..., 0] = ids & np.uint64(_MASK)
    ctr[..., 1] = np.uint64(step) & np.uint64(_MASK)
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    key = np.array([seed & _MASK, seed >> 32], dtype=np.uint64)
    w = philox4x32_10(ctr, key).astype(np.float64)
    s32 = 2.0 ** -32
    u0, u1 = (w[..., 0] + 1.0) * s32, w[..., 1] * s32
    u2, u3 = (w[..., 2] + 1.0) * s32, w[..., 3] * s32
    r0, r2 = np.sqrt(-2.0 * np.log(u0)), np.sqrt(-2.0 * np.log(u2))
    two_pi = 2.0 * np.pi
    return np.stack([r0 * np.cos(two_pi * u1), r0 * np.sin(two_pi * u1),
                     r2 * np.cos(two_pi * u3)], axis=-1)


def region_of(x, thermostat):
    """Index of the first region with lo <= x[axis] < hi for each atom (-1: none); x is
    taken as given (run_nvt passes positions wrapped into the box)."""
    xa = x[:, thermostat.get("axis", 2)]
    out = np.full(x.shape[0], -1)
    for q in reversed(range(len(thermostat["regions"]))):
        r = thermostat["regions"][q]
        inside = (xa >= r.get("lo", -np.inf)) & (xa < r.get("hi", np.inf))
        out[inside] = q
    return out


def o_step(x, v, ids, step, thermostat, mass, dt):
    """The Ornstein-Uhlenbeck velocity update of one step (returns a new array)."""
    v = np.array(v, np.float64, copy=True)
    reg = region_of(x, thermostat)
    if not np.any(reg >= 0):
        return v
    xi = normals(thermostat.get("seed", 0), step, ids)
    for q, r in enumerate(thermostat["regions"]):
        sel = reg == q
        if not np.any(sel):
            continue
        c1 = np.exp(-r["gamma"] * dt)
        c2 = np.sqrt((1.0 - c1 * c1) * KB * r["T"] / mass * ACCEL)
        u = np.asarray(r.get("u", (0.0, 0.0, 0.0)), np.float64)
        v[sel] = u + c1 * (v[sel] - u) + c2 * xi[sel]
    return v


def run_nvt(x, v, ids, box, mass, dt, n_steps, force_fn, thermostat, walls=None, step0=0,
            record=True):
    """Velocity Verlet with the Langevin update at the start of each step (steps
    step0 + 1 .. step0 + n_steps).  force_fn(x) -> (forces, potential energy).
    Returns final (x, v, f) and per-step (t, PE, KE), step 0 first."""
    x = core.wrap(x, box)
    v = np.array(v, np.float64, copy=True)
    f, pe = force_fn(x)
    t = step0 * dt
    hist = [(t, pe, kinetic_energy(v, mass))]
    for s in range(step0 + 1, step0 + n_steps + 1):
        v = o_step(x, v, ids, s, thermostat, mass, dt)
        v = v + 0.5 * dt * f / mass * ACCEL
        x = x + dt * v
        t = s * dt
        x, v = apply_walls(x, v, t, walls)
        x = core.wrap(x, box)
        f, pe = force_fn(x)
        v = v + 0.5 * dt * f / mass * ACCEL
        if record:
            hist.append((t, pe, kinetic_energy(v, mass)))
    return x, v, f, np.array(hist)
