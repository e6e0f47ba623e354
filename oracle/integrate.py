"""Velocity Verlet integration of Newton's equations (oracle; test infrastructure only).

Sec. 1.5: m_i d^2 r_i/dt^2 = f_i = -grad_i U (eq. 1.5), integrated with the
symplectic Verlet scheme in its velocity (kick-drift-kick) form, NVE:

    v <- v + (dt/2) f/m;   x <- x + dt v;   walls;   wrap;   f <- f(x);   v <- v + (dt/2) f/m

Units: angstrom, ps, u, eV; f/m in eV/(u angstrom) is converted to
angstrom/ps^2 by the factor 9648.5332157.

Walls (Sec. 1.5 mentions hard walls; the piston recipe of the shock workload):
a piston plane z_p(t) = z0 + v_p t moving along +axis reflects atoms
specularly in its own frame (z <- 2 z_p - z, v_z <- 2 v_p - v_z when z < z_p);
a static top wall at z_top reflects (z <- 2 z_top - z, v_z <- -v_z when z > z_top).
"""
from __future__ import annotations

import numpy as np

from . import core

ACCEL = 9648.5332157  # (eV / (u angstrom)) in angstrom / ps^2


def kinetic_energy(v, mass):
    """K = sum_i m v_i^2 / 2, in eV (eq. 1.3)."""
    return 0.5 * mass * float(np.sum(v * v)) / ACCEL


def kinetic_tensor(v, mass):
    """sum_i m v^a v^b in eV, order xx, yy, zz, xy, xz, yz."""
    k = mass * np.array([np.sum(v[:, 0] * v[:, 0]), np.sum(v[:, 1] * v[:, 1]),
                         np.sum(v[:, 2] * v[:, 2]), np.sum(v[:, 0] * v[:, 1]),
                         np.sum(v[:, 0] * v[:, 2]), np.sum(v[:, 1] * v[:, 2])])
    return k / ACCEL


def apply_walls(x, v, t_new, walls):
    if not walls:
        return x, v
    ax = walls["axis"]
    zp = walls["piston_z0"] + walls["piston_v"] * t_new
    vp = walls["piston_v"]
    lo = x[:, ax] < zp
    x[lo, ax] = 2.0 * zp - x[lo, ax]
    v[lo, ax] = 2.0 * vp - v[lo, ax]
    zt = walls["top_z"]
    hi = x[:, ax] > zt
    x[hi, ax] = 2.0 * zt - x[hi, ax]
    v[hi, ax] = -v[hi, ax]
    return x, v


def run_nve(x, v, box, mass, dt, n_steps, force_fn, walls=None, t0=0.0, record=True):
    """Velocity Verlet for n_steps.  force_fn(x) -> (forces [n,3], potential energy).
    Returns final (x, v, f) and per-step (t, PE, KE) after each step (step 0 first)."""
    x = core.wrap(x, box)
    v = np.array(v, np.float64, copy=True)
    f, pe = force_fn(x)
    hist = [(t0, pe, kinetic_energy(v, mass))]
    t = t0
    for _ in range(n_steps):
        v = v + 0.5 * dt * f / mass * ACCEL
        x = x + dt * v
        t = t + dt
        x, v = apply_walls(x, v, t, walls)
        x = core.wrap(x, box)
        f, pe = force_fn(x)
        v = v + 0.5 * dt * f / mass * ACCEL
        if record:
            hist.append((t, pe, kinetic_energy(v, mass)))
    return x, v, f, np.array(hist)


def lj_force_fn(box, p):
    def fn(x):
        r = core.lj(x, box, p.eps, p.sigma, p.r_cut)
        return r.force, r.energy
    return fn


def eam_force_fn(box, pot):
    def fn(x):
        r = core.eam(x, box, pot)
        return r.force, r.energy
    return fn
