"""Closed-form perfect-crystal sums over fcc lattice vectors (independent of any
box, cell list or minimum image): used to pin the oracle."""
import math

import numpy as np


def fcc_shells(a, r_max):
    """[(radius, multiplicity)] of the fcc lattice vectors (a/2)(i, j, k), i+j+k even,
    0 < |v| < r_max."""
    m = int(math.ceil(2.0 * r_max / a)) + 1
    rng = np.arange(-m, m + 1)
    i, j, k = np.meshgrid(rng, rng, rng, indexing="ij")
    even = ((i + j + k) % 2) == 0
    v2 = (i * i + j * j + k * k)[even]
    v2 = v2[v2 > 0]
    out = {}
    for q in v2.tolist():
        r = 0.5 * a * math.sqrt(q)
        if r < r_max:
            out[q] = out.get(q, 0) + 1
    return [(0.5 * a * math.sqrt(q), out[q]) for q in sorted(out)]


def lj_energy_per_atom(a, eps, sigma, r_cut):
    u = lambda r: 4 * eps * ((sigma / r) ** 12 - (sigma / r) ** 6)
    return 0.5 * sum(n * (u(r) - u(r_cut)) for r, n in fcc_shells(a, r_cut))


def eam_per_atom(a, p):
    """(E/atom, rhobar) of the analytic EAM on a perfect fcc lattice."""
    sh = fcc_shells(a, p.r_cut)
    rb = sum(n * math.exp(-p.beta * (r / p.r0 - 1.0)) for r, n in sh)
    ph = sum(n * p.A * math.exp(-p.alpha * (r / p.r0 - 1.0)) for r, n in sh)
    return -math.sqrt(rb) + 0.5 * ph, rb


def eam_dE_da(a, p):
    """Derivative of the per-atom EAM energy with respect to the lattice constant."""
    sh = fcc_shells(a, p.r_cut)
    rb = sum(n * math.exp(-p.beta * (r / p.r0 - 1.0)) for r, n in sh)
    drb = sum(n * (r / a) * (-p.beta / p.r0) * math.exp(-p.beta * (r / p.r0 - 1.0)) for r, n in sh)
    dph = sum(n * (r / a) * (-p.alpha / p.r0) * p.A * math.exp(-p.alpha * (r / p.r0 - 1.0))
              for r, n in sh)
    return -0.5 / math.sqrt(rb) * drb + 0.5 * dph


def count_within(a, r):
    return sum(n for rr, n in fcc_shells(a, r))
