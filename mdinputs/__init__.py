"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module only *generates inputs*: fcc lattices, seeded displacements and
Maxwell-Boltzmann velocities, replica and snapshot recipes, and the tabulated
potential "files" (function values on a uniform grid plus end slopes, the form
in which the paper loads an EAM potential, Sec. 3.3).  It holds none of the
method's arithmetic: no spline fitting or evaluation, no forces, no
integration.  Both sides fit and evaluate their own splines from these samples.

Units are "metal": length in angstrom, energy in eV, time in ps, mass in u,
temperature in K.  Random numbers come from numpy's PCG64 (default_rng), drawn
in a fixed order so that a seed fixes the input bit for bit.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

KB_EV_PER_K = 8.617333262e-5            # Boltzmann constant, eV/K (CODATA 2018)
EV_PER_U_IN_A2_PER_PS2 = 9648.5332157   # 1 eV/u expressed in (angstrom/ps)^2
SEED_BASE = 229510

MASS = {"Ar": 39.948, "Cu": 63.546, "Al": 26.9815385}


# ----------------------------------------------------------------------------
# Boxes and lattices
# ----------------------------------------------------------------------------
@dataclass
class Box:
    """Orthorhombic box [lo, lo+len) per axis; periodic flags per axis."""
    lo: tuple = (0.0, 0.0, 0.0)
    len: tuple = (1.0, 1.0, 1.0)
    periodic: tuple = (1, 1, 1)

    def as_arrays(self):
        return (np.asarray(self.lo, np.float64), np.asarray(self.len, np.float64),
                np.asarray(self.periodic, np.int32))


FCC_BASIS = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])


def fcc_lattice(n1: int, n2: int, n3: int, a: float, z_offset: float = 0.0):
    """fcc positions, order (ix, iy, iz, basis), box [0, n*a) per axis."""
    ix, iy, iz = np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij")
    cells = np.stack([ix, iy, iz], axis=-1).reshape(-1, 1, 3).astype(np.float64)
    pos = (cells + FCC_BASIS[None, :, :]).reshape(-1, 3) * a
    pos[:, 2] += z_offset
    return np.ascontiguousarray(pos), Box((0.0, 0.0, 0.0), (n1 * a, n2 * a, n3 * a), (1, 1, 1))


def thermal_state(pos: np.ndarray, mass: float, temperature: float, sigma_disp: float, seed: int):
    """Gaussian displacements N(0, sigma^2) then Maxwell-Boltzmann velocities (angstrom/ps)
    at `temperature` with the mean velocity removed (zero net momentum, equal masses).
    Draw order: displacements (if sigma_disp > 0), then velocities."""
    rng = np.random.default_rng(seed)
    x = pos.copy()
    if sigma_disp > 0.0:
        x += rng.normal(0.0, sigma_disp, size=x.shape)
    if temperature > 0.0:
        sv = math.sqrt(KB_EV_PER_K * temperature / mass * EV_PER_U_IN_A2_PER_PS2)
        v = rng.normal(0.0, sv, size=x.shape)
        v -= v.mean(axis=0, keepdims=True)
    else:
        v = np.zeros_like(x)
    return np.ascontiguousarray(x), np.ascontiguousarray(v)


def wrap_into_box(pos: np.ndarray, box: Box):
    """Input hygiene for generated states: fold coordinates into [lo, lo+len) on
    periodic axes using a plain modulo (used only when generating inputs)."""
    lo, ln, per = box.as_arrays()
    out = pos.copy()
    for a in range(3):
        if per[a]:
            out[:, a] = lo[a] + np.mod(out[:, a] - lo[a], ln[a])
            out[out[:, a] >= lo[a] + ln[a], a] = lo[a]
    return out


# ----------------------------------------------------------------------------
# Potentials: parameter sets and tabulated "files"
# ----------------------------------------------------------------------------
@dataclass
class LJParams:
    eps: float
    sigma: float
    r_cut: float


@dataclass
class EAMParams:
    """Analytic Finnis-Sinclair-type EAM:
    phi(r) = A exp(-alpha (r/r0 - 1)), rho(r) = exp(-beta (r/r0 - 1)), F(rho) = -sqrt(rho)."""
    A: float
    alpha: float
    beta: float
    r0: float
    r_cut: float


EAM_CU = EAMParams(A=0.2, alpha=9.0, beta=6.0, r0=2.556, r_cut=5.5)
EAM_AL = EAMParams(A=0.15, alpha=8.0, beta=5.5, r0=2.864, r_cut=6.0)
LJ_AR = LJParams(eps=0.0104, sigma=3.405, r_cut=2.5 * 3.405)


@dataclass
class TabulatedFunction:
    """Samples y[k] = f(x_lo + k h), k = 0..K-1, and the end slopes f'(x_lo), f'(x_hi)."""
    x_lo: float
    x_hi: float
    y: np.ndarray
    dy_lo: float
    dy_hi: float

    @property
    def K(self):
        return int(self.y.shape[0])

    @property
    def h(self):
        return (self.x_hi - self.x_lo) / (self.K - 1)


@dataclass
class EAMTable:
    """A tabulated single-element EAM potential: pair phi(r), density rho(r) on
    [r_lo, r_cut], embedding F(rhobar) on [rho_lo, rho_hi]."""
    phi: TabulatedFunction
    rho: TabulatedFunction
    emb: TabulatedFunction
    r_cut: float


def _grid(lo, hi, K):
    k = np.arange(K, dtype=np.float64)
    return lo + k * ((hi - lo) / (K - 1))


def tabulate_eam(p: EAMParams, K: int = 2000, r_lo: float = 1.0, rho_lo: float = 1.0,
                 rho_hi: float = 41.0, r_hi: float | None = None) -> EAMTable:
    """Write the analytic EAM as a table of K samples per function plus end slopes
    (what an EAM potential file holds)."""
    r_hi = p.r_cut if r_hi is None else r_hi
    r = _grid(r_lo, r_hi, K)
    q = _grid(rho_lo, rho_hi, K)
    phi = p.A * np.exp(-p.alpha * (r / p.r0 - 1.0))
    rho = np.exp(-p.beta * (r / p.r0 - 1.0))
    emb = -np.sqrt(q)
    dphi = lambda x: -p.A * p.alpha / p.r0 * math.exp(-p.alpha * (x / p.r0 - 1.0))
    drho = lambda x: -p.beta / p.r0 * math.exp(-p.beta * (x / p.r0 - 1.0))
    demb = lambda x: -0.5 / math.sqrt(x)
    return EAMTable(
        phi=TabulatedFunction(r_lo, r_hi, phi, dphi(r_lo), dphi(r_hi)),
        rho=TabulatedFunction(r_lo, r_hi, rho, drho(r_lo), drho(r_hi)),
        emb=TabulatedFunction(rho_lo, rho_hi, emb, demb(rho_lo), demb(rho_hi)),
        r_cut=p.r_cut,
    )


# ----------------------------------------------------------------------------
# Workload recipes (sizes, distributions, seeds)
# ----------------------------------------------------------------------------
@dataclass
class MDSystem:
    name: str
    pos: np.ndarray
    vel: np.ndarray
    box: Box
    mass: float
    dt_ps: float
    n_steps: int
    skin: float
    potential: str               # "lj", "eam" or "bpnn"
    lj: LJParams | None = None
    eam: EAMParams | None = None
    table: EAMTable | None = None
    walls: dict | None = None
    extra: dict = field(default_factory=dict)


def lj_argon(cells: int = 4, seed: int | None = None) -> MDSystem:
    """LJ argon: fcc cells^3, a = 5.26, eps 0.0104 eV, sigma 3.405, r_c 2.5 sigma
    (energy shift), 100 K, dt 2 fs, 100 steps, skin 0.3."""
    pos, box = fcc_lattice(cells, cells, cells, 5.26)
    x, v = thermal_state(pos, MASS["Ar"], 100.0, 0.0, SEED_BASE + 1 if seed is None else seed)
    return MDSystem("lj_argon_%d" % (4 * cells ** 3), wrap_into_box(x, box), v, box, MASS["Ar"],
                    2e-3, 100, 0.3, "lj", lj=LJ_AR)


def lj_argon_benchmark(cells: int = 148, seed: int | None = None) -> MDSystem:
    """The LJ performance test of Sec. 1.7 at its size: a periodic cube, fcc cells^3
    (148^3 * 4 = 12,967,168 atoms), lattice with small perturbations, 300 steps, the
    lists rebuilt every 10 steps.  The section gives neither the material nor the
    temperature, time step or skin; this reading takes the LJ argon of the small
    system (a = 5.26, eps 0.0104 eV, sigma 3.405, r_c 2.5 sigma), N(0, 0.05^2)
    displacements, 100 K, dt 2 fs, and a 0.5 angstrom skin, wide enough that no atom
    moves half of it in ten steps."""
    pos, box = fcc_lattice(cells, cells, cells, 5.26)
    x, v = thermal_state(pos, MASS["Ar"], 100.0, 0.05, SEED_BASE + 7 if seed is None else seed)
    return MDSystem("lj_argon_%d" % (4 * cells ** 3), wrap_into_box(x, box), v, box, MASS["Ar"],
                    2e-3, 300, 0.5, "lj", lj=LJ_AR, extra={"rebuild_every": 10})


def eam_copper(cells: int = 32, seed: int | None = None, K: int = 2000) -> MDSystem:
    """EAM copper: fcc cells^3, a = 3.615, N(0, 0.05^2) displacements, 300 K,
    dt 1 fs, 1000 steps, skin 0.3, 2000-point tables."""
    pos, box = fcc_lattice(cells, cells, cells, 3.615)
    x, v = thermal_state(pos, MASS["Cu"], 300.0, 0.05, SEED_BASE + 2 if seed is None else seed)
    return MDSystem("eam_cu_%d" % (4 * cells ** 3), wrap_into_box(x, box), v, box, MASS["Cu"],
                    1e-3, 1000, 0.3, "eam", eam=EAM_CU, table=tabulate_eam(EAM_CU, K=K))


def eam_aluminum_shock(nx: int = 20, ny: int = 20, nz: int = 400, seed: int | None = None,
                       K: int = 2000) -> MDSystem:
    """EAM aluminum shock: fcc nx*ny*nz, a = 4.05, lattice shifted by a/4 in z, 300 K,
    periodic in x/y, reflecting piston at z = v_p t (v_p = 10 angstrom/ps = 1 km/s)
    and a static top wall at z = L_z; dt 1 fs, 5000 steps, skin 0.3."""
    a = 4.05
    pos, box = fcc_lattice(nx, ny, nz, a, z_offset=0.25 * a)
    box = Box(box.lo, box.len, (1, 1, 0))
    x, v = thermal_state(pos, MASS["Al"], 300.0, 0.0, SEED_BASE + 3 if seed is None else seed)
    x = wrap_into_box(x, box)
    return MDSystem("eam_al_shock_%d" % (4 * nx * ny * nz), x, v, box, MASS["Al"], 1e-3, 5000, 0.3,
                    "eam", eam=EAM_AL, table=tabulate_eam(EAM_AL, K=K),
                    walls={"axis": 2, "piston_z0": 0.0, "piston_v": 10.0, "top_z": box.len[2]})


@dataclass
class Replica:
    pos: np.ndarray
    box: Box
    a: float
    cells: int


def cold_curve_replicas(n_rep: int = 64, seed: int | None = None, a_lo: float = 3.30,
                        a_hi: float = 4.20, n_min: int = 4, n_max: int = 12):
    """Perfect Cu fcc replicas at rest: cells n_r ~ U{n_min..n_max} from the seed,
    lattice constants linspace(a_lo, a_hi, n_rep)."""
    rng = np.random.default_rng(SEED_BASE + 4 if seed is None else seed)
    ns = rng.integers(n_min, n_max + 1, size=n_rep)
    avals = np.linspace(a_lo, a_hi, n_rep)
    reps = []
    for n, a in zip(ns, avals):
        pos, box = fcc_lattice(int(n), int(n), int(n), float(a))
        reps.append(Replica(pos, box, float(a), int(n)))
    return reps


@dataclass
class Snapshot:
    pos: np.ndarray
    box: Box
    a: float


def force_matching_snapshots(n_snap: int = 1024, cells: int = 5, seed: int | None = None,
                             a_lo: float = 3.55, a_hi: float = 3.68, sigma: float = 0.1):
    """Periodic Cu fcc cells^3 snapshots, a ~ U(a_lo, a_hi), N(0, sigma^2) displacements.
    Draw order per snapshot: a, then the displacement block."""
    rng = np.random.default_rng(SEED_BASE + 5 if seed is None else seed)
    snaps = []
    for _ in range(n_snap):
        a = float(rng.uniform(a_lo, a_hi))
        pos, box = fcc_lattice(cells, cells, cells, a)
        pos = pos + rng.normal(0.0, sigma, size=pos.shape)
        snaps.append(Snapshot(wrap_into_box(pos, box), box, a))
    return snaps


# Trainable-spline grids for force matching: 62 breakpoints -> 64 B-spline
# coefficients per function, 192 in all.
FM_K = 62
FM_R_RANGE = (1.5, 5.5)
FM_RHO_RANGE = (5.0, 25.0)


def force_matching_tables(p: EAMParams = EAM_CU) -> EAMTable:
    """The analytic Cu EAM sampled on the coarse trainable grids."""
    return tabulate_eam(p, K=FM_K, r_lo=FM_R_RANGE[0], r_hi=FM_R_RANGE[1],
                        rho_lo=FM_RHO_RANGE[0], rho_hi=FM_RHO_RANGE[1])


def coefficient_noise(n: int = 3 * (FM_K + 2), seed: int | None = None, scale: float = 0.05):
    """Multiplicative noise factors (1 + scale * xi), xi ~ N(0, 1)."""
    rng = np.random.default_rng(SEED_BASE + 6 if seed is None else seed)
    return 1.0 + scale * rng.normal(0.0, 1.0, size=n)


def random_cotangent(n_atoms: int, seed: int, scale: float = 1.0):
    """Seeded dL/dF cotangent [n_atoms, 3] for vector-Jacobian parity tests."""
    rng = np.random.default_rng(seed)
    return scale * rng.normal(0.0, 1.0, size=(n_atoms, 3))


# ----------------------------------------------------------------------------
# Behler-Parrinello network potential (Sec. 2.1): symmetry-function parameters and
# random network weights (no trained model ships with the paper)
# ----------------------------------------------------------------------------
def bpnn_params(seed: int | None = None, r_cut: float = 6.0, hidden=(10, 10)) -> dict:
    """8 radial G2 functions (shared R_s = 0, eta spread over 0.003-1.0 / A^2) and 43
    angular G4 functions (zeta in {1, 2, 4, 16} x lambda in {+1, -1} x eta in
    {0, 0.003, 0.008, 0.015, 0.03, 0.06} / A^2, the first 43 combinations), as in the
    MAISE-format models the paper describes (8 G2 + 43 G4 per atom type, two hidden
    layers of 10); weights N(0, s^2) with s scaled by the fan-in and a rough input
    magnitude (10 for G2, 100 for G4) so that tanh stays out of saturation."""
    rng = np.random.default_rng(SEED_BASE + 8 if seed is None else seed)
    g2_eta = np.array([0.003, 0.01, 0.03, 0.06, 0.12, 0.25, 0.5, 1.0])
    combos = [(z, l, e) for e in (0.0, 0.003, 0.008, 0.015, 0.03, 0.06)
              for z in (1.0, 2.0, 4.0, 16.0) for l in (1.0, -1.0)][:43]
    g4 = np.array(combos)
    ng = len(g2_eta) + len(g4)
    h1, h2 = hidden
    scale_in = np.concatenate([np.full(len(g2_eta), 10.0), np.full(len(g4), 100.0)])
    w01 = rng.normal(0.0, 1.0, (ng, h1)) / (np.sqrt(ng) * scale_in[:, None])
    return {
        "r_cut": r_cut, "r_s": 0.0, "g2_eta": g2_eta,
        "g4_zeta": g4[:, 0].copy(), "g4_lambda": g4[:, 1].copy(), "g4_eta": g4[:, 2].copy(),
        "w01": w01, "b1": rng.normal(0.0, 0.1, h1),
        "w12": rng.normal(0.0, 1.0 / np.sqrt(h1), (h1, h2)), "b2": rng.normal(0.0, 0.1, h2),
        "w23": rng.normal(0.0, 1.0 / np.sqrt(h2), h2), "b3": -3.5,
    }


def bpnn_copper(cells: int = 8, seed: int | None = None) -> MDSystem:
    """Copper described by the network potential of bpnn_params (r_c 6 A): fcc cells^3,
    a = 3.615, N(0, 0.05^2) displacements, 300 K, dt 1 fs, skin 0.3."""
    pos, box = fcc_lattice(cells, cells, cells, 3.615)
    x, v = thermal_state(pos, MASS["Cu"], 300.0, 0.05, SEED_BASE + 9 if seed is None else seed)
    return MDSystem("bpnn_cu_%d" % (4 * cells ** 3), wrap_into_box(x, box), v, box, MASS["Cu"],
                    1e-3, 100, 0.3, "bpnn", extra={"bpnn": bpnn_params()})
