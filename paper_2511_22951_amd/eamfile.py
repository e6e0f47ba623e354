"""Tabulated EAM potential files (Sec. 3.3: single-element EAM loaded from a tabulated
file, as distributed by the Interatomic Potentials Repository).

Two plain-text layouts are read, single element only:

  setfl   3 comment lines; "1 <element>"; "Nrho drho Nr dr cutoff"; "Z mass a lattice";
          F(rho_k), k < Nrho; rho(r_k), k < Nr; then r_k phi(r_k), k < Nr
  funcfl  1 comment line; "Z mass a lattice"; "Nrho drho Nr dr cutoff"; F(rho_k);
          Z(r_k), with phi(r) = 27.2 x 0.529 Z(r)^2 / r (Hartree Bohr in eV A); rho(r_k)

with rho_k = k drho and r_k = k dr.  Numbers may be split over lines in any way.  The
returned table (samples on uniform grids plus end slopes) is what
md.EAMPotential.from_table fits on the device.  phi and rho start at r = dr (phi is
stored as r phi or through Z(r) and is undefined at r = 0); the files carry no end
slopes, which are taken from the samples by third-order one-sided differences.  Grids
longer than the device fit's limit of 8000 samples are thinned to every m-th sample.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

MAX_SAMPLES = 8000  # the device spline fit's limit (md_spline_fit)
HARTREE_BOHR = 27.2 * 0.529  # eV A, the funcfl convention


@dataclass
class TabFunc:
    """Samples y[k] = f(x_lo + k h) and the end slopes (the fields md.EAMPotential reads)."""
    x_lo: float
    h: float
    y: np.ndarray
    dy_lo: float
    dy_hi: float

    @property
    def K(self):
        return int(self.y.shape[0])

    @property
    def x_hi(self):
        return self.x_lo + (self.K - 1) * self.h


@dataclass
class EAMFile:
    phi: TabFunc
    rho: TabFunc
    emb: TabFunc
    r_cut: float
    element: str
    mass: float
    lattice_constant: float
    lattice: str


def _slopes(y, h):
    lo = (-11.0 * y[0] + 18.0 * y[1] - 9.0 * y[2] + 2.0 * y[3]) / (6.0 * h)
    hi = (11.0 * y[-1] - 18.0 * y[-2] + 9.0 * y[-3] - 2.0 * y[-4]) / (6.0 * h)
    return lo, hi


def _func(x_lo, h, y, max_samples):
    y = np.asarray(y, np.float64)
    if y.shape[0] < 4:
        raise ValueError("a tabulated function needs at least 4 samples")
    m = -(-y.shape[0] // max_samples)  # thinning factor
    if m > 1:
        y = y[::m]
        h = h * m
    lo, hi = _slopes(y, h)
    return TabFunc(float(x_lo), float(h), np.ascontiguousarray(y), float(lo), float(hi))


class _Tokens:
    def __init__(self, lines):
        self.t = " ".join(lines).split()
        self.i = 0

    def take(self, n, conv=float):
        if self.i + n > len(self.t):
            raise ValueError("EAM file ends early")
        out = [conv(x) for x in self.t[self.i:self.i + n]]
        self.i += n
        return out


def read_setfl(path, max_samples=MAX_SAMPLES) -> EAMFile:
    with open(path) as f:
        lines = f.read().splitlines()
    head = lines[3].split()
    if int(head[0]) != 1:
        raise ValueError("only single-element setfl files are supported (%s elements)" % head[0])
    tok = _Tokens(lines[4:])
    nrho, = tok.take(1, int)
    drho, = tok.take(1)
    nr, = tok.take(1, int)
    dr, cut = tok.take(2)
    _z, = tok.take(1, int)
    mass, a = tok.take(2)
    lattice = tok.take(1, str)[0]
    F = np.array(tok.take(nrho))
    rho = np.array(tok.take(nr))
    rphi = np.array(tok.take(nr))
    r = dr * np.arange(nr)
    return EAMFile(phi=_func(dr, dr, rphi[1:] / r[1:], max_samples),
                   rho=_func(dr, dr, rho[1:], max_samples),
                   emb=_func(0.0, drho, F, max_samples),
                   r_cut=float(cut), element=head[1], mass=float(mass),
                   lattice_constant=float(a), lattice=lattice)


def read_funcfl(path, max_samples=MAX_SAMPLES) -> EAMFile:
    with open(path) as f:
        lines = f.read().splitlines()
    tok = _Tokens(lines[1:])
    _z, = tok.take(1, int)
    mass, a = tok.take(2)
    lattice = tok.take(1, str)[0]
    nrho, = tok.take(1, int)
    drho, = tok.take(1)
    nr, = tok.take(1, int)
    dr, cut = tok.take(2)
    F = np.array(tok.take(nrho))
    Z = np.array(tok.take(nr))
    rho = np.array(tok.take(nr))
    r = dr * np.arange(nr)
    phi = HARTREE_BOHR * Z[1:] * Z[1:] / r[1:]
    return EAMFile(phi=_func(dr, dr, phi, max_samples), rho=_func(dr, dr, rho[1:], max_samples),
                   emb=_func(0.0, drho, F, max_samples), r_cut=float(cut), element="",
                   mass=float(mass), lattice_constant=float(a), lattice=lattice)


def read_eam(path, max_samples=MAX_SAMPLES) -> EAMFile:
    """setfl when the fourth line starts with an element count, funcfl otherwise."""
    with open(path) as f:
        lines = [next(f, "") for _ in range(4)]
    parts = lines[3].split()
    is_setfl = len(parts) == 2 and parts[0].isdigit() and not _is_number(parts[1])
    return read_setfl(path, max_samples) if is_setfl else read_funcfl(path, max_samples)


def _is_number(s):
    try:
        float(s)
        return True
    except ValueError:
        return False


def write_setfl(path, F, rho, rphi, drho, dr, r_cut, element="X", z=0, mass=1.0, a=1.0,
                lattice="fcc", comments=("", "", "")):
    """Write a single-element setfl file from samples F(k drho), rho(k dr), r phi(k dr)."""
    def block(v):
        v = np.asarray(v, np.float64)
        return "\n".join(" ".join("%.16e" % x for x in v[i:i + 5]) for i in range(0, len(v), 5))
    with open(path, "w") as f:
        for c in comments:
            f.write(c + "\n")
        f.write("1 %s\n" % element)
        f.write("%d %.16e %d %.16e %.16e\n" % (len(F), drho, len(rho), dr, r_cut))
        f.write("%d %.16e %.16e %s\n" % (z, mass, a, lattice))
        f.write(block(F) + "\n" + block(rho) + "\n" + block(rphi) + "\n")
