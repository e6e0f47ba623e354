"""ctypes front end of the oracle's C core (oracle; test infrastructure only).

Positions are [n, 3] float64 arrays (C order), boxes are mdinputs.Box.  The
potentials are given as spline coefficient arrays (fitted by oracle.spline) or
as the analytic closed forms.  See md_oracle.c for the definitions.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

from . import spline as _spline

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_md_oracle.so")
_lib = None
_lock = threading.Lock()


class _Box(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("len", C.c_double * 3), ("periodic", C.c_int * 3)]


class _Func(C.Structure):
    _fields_ = [("kind", C.c_int), ("ncoef", C.c_int), ("c", C.POINTER(C.c_double)),
                ("x_lo", C.c_double), ("h", C.c_double), ("A", C.c_double),
                ("alpha", C.c_double), ("r0", C.c_double)]


class _EAM(C.Structure):
    _fields_ = [("phi", _Func), ("rho", _Func), ("emb", _Func), ("r_cut", C.c_double)]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(
                    os.path.join(_HERE, "md_oracle.c")):
                from .build_oracle import build
                build()
            L = C.CDLL(_SO)
            dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int)
            bp, ep = C.POINTER(_Box), C.POINTER(_EAM)
            L.or_num_threads.restype = C.c_int
            L.or_wrap.argtypes = [C.c_int, dp, bp]
            L.or_neighbors.argtypes = [C.c_int, dp, bp, C.c_double, C.c_int, ip, ip]
            L.or_neighbors.restype = C.c_int
            L.or_min_gap.argtypes = [C.c_int, dp, bp, C.c_double]
            L.or_min_gap.restype = C.c_double
            L.or_lj.argtypes = [C.c_int, dp, bp, C.c_double, C.c_double, C.c_double, dp, dp, dp]
            L.or_eval_func.argtypes = [C.POINTER(_Func), C.c_int, dp, dp, dp, dp]
            L.or_eval_func.restype = C.c_int
            L.or_eam.argtypes = [C.c_int, dp, bp, ep, dp, dp, dp, dp, dp, dp]
            L.or_eam.restype = C.c_int
            L.or_eam_sampled.argtypes = [C.c_int, dp, bp, ep, C.c_int, ip, dp, dp, dp]
            L.or_eam_sampled.restype = C.c_int
            L.or_lj_sampled.argtypes = [C.c_int, dp, bp, C.c_double, C.c_double, C.c_double,
                                        C.c_int, ip, dp, dp]
            L.or_neighbors_sampled.argtypes = [C.c_int, dp, bp, C.c_double, C.c_int, ip, C.c_int,
                                               ip, ip]
            L.or_pairs.argtypes = [C.c_int, dp, bp, C.c_double, C.c_long, ip, ip, dp]
            L.or_pairs.restype = C.c_long
            _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _pos(pos):
    p = np.ascontiguousarray(np.asarray(pos, np.float64))
    assert p.ndim == 2 and p.shape[1] == 3
    return p


def _box(box):
    b = _Box()
    for a in range(3):
        b.lo[a] = float(box.lo[a])
        b.len[a] = float(box.len[a])
        b.periodic[a] = int(box.periodic[a])
    return b


def num_threads() -> int:
    return int(lib().or_num_threads())


# ----------------------------------------------------------------------------
# Potentials as C structures
# ----------------------------------------------------------------------------
class SplineFunc:
    """A fitted uniform cubic B-spline (coefficients c, grid x_lo, h)."""

    def __init__(self, c, x_lo, h):
        self.c = np.ascontiguousarray(np.asarray(c, np.float64))
        self.x_lo = float(x_lo)
        self.h = float(h)

    @classmethod
    def from_table(cls, tf):
        return cls(_spline.fit_table(tf), tf.x_lo, tf.h)

    def cstruct(self):
        f = _Func()
        f.kind, f.ncoef, f.c = 0, self.c.shape[0], _d(self.c)
        f.x_lo, f.h = self.x_lo, self.h
        return f


class AnalyticFunc:
    """kind 1: A exp(-alpha (x/r0 - 1)); kind 2: -sqrt(x)."""

    def __init__(self, kind, A=0.0, alpha=0.0, r0=1.0):
        self.kind, self.A, self.alpha, self.r0 = kind, A, alpha, r0

    def cstruct(self):
        f = _Func()
        f.kind, f.ncoef, f.c = self.kind, 0, None
        f.A, f.alpha, f.r0 = self.A, self.alpha, self.r0
        return f


class EAMPotential:
    def __init__(self, phi, rho, emb, r_cut):
        self.phi, self.rho, self.emb, self.r_cut = phi, rho, emb, float(r_cut)

    @classmethod
    def from_table(cls, table):
        """Splines fitted to a tabulated EAM (mdinputs.EAMTable)."""
        return cls(SplineFunc.from_table(table.phi), SplineFunc.from_table(table.rho),
                   SplineFunc.from_table(table.emb), table.r_cut)

    @classmethod
    def analytic(cls, p):
        """The closed forms of mdinputs.EAMParams."""
        return cls(AnalyticFunc(1, p.A, p.alpha, p.r0), AnalyticFunc(1, 1.0, p.beta, p.r0),
                   AnalyticFunc(2), p.r_cut)

    def cstruct(self):
        e = _EAM()
        e.phi, e.rho, e.emb = self.phi.cstruct(), self.rho.cstruct(), self.emb.cstruct()
        e.r_cut = self.r_cut
        return e


def eval_func(fn, x):
    """(value, d1, d2, n_out_of_range) of a SplineFunc/AnalyticFunc through the C evaluator."""
    x = np.ascontiguousarray(np.asarray(x, np.float64).ravel())
    v, d1, d2 = np.empty_like(x), np.empty_like(x), np.empty_like(x)
    s = fn.cstruct()
    oor = lib().or_eval_func(C.byref(s), x.shape[0], _d(x), _d(v), _d(d1), _d(d2))
    return v, d1, d2, int(oor)


# ----------------------------------------------------------------------------
# Geometry and neighbour sets
# ----------------------------------------------------------------------------
def wrap(pos, box):
    """x <- x - L floor((x - lo)/L) on periodic axes (a result of lo + L becomes lo)."""
    p = _pos(pos).copy()
    b = _box(box)
    lib().or_wrap(p.shape[0], _d(p), C.byref(b))
    return p


def neighbor_sets(pos, box, r_ns, maxn=512):
    """Brute-force {j != i : r_ij^2 < r_ns^2} with the minimum image (Sec. 1.4, eq. 1.2).
    Returns (counts [n], list of sorted int arrays)."""
    p = _pos(pos)
    n = p.shape[0]
    cnt = np.zeros(n, np.int32)
    lst = np.zeros((n, maxn), np.int32)
    b = _box(box)
    over = lib().or_neighbors(n, _d(p), C.byref(b), float(r_ns), maxn, _i(cnt), _i(lst))
    if over:
        raise ValueError("oracle neighbour capacity %d exceeded" % maxn)
    return cnt, [lst[i, :cnt[i]].copy() for i in range(n)]


def neighbor_sets_sampled(pos, box, r_ns, idx, maxn=512):
    p = _pos(pos)
    idx = np.ascontiguousarray(np.asarray(idx, np.int32))
    cnt = np.zeros(idx.shape[0], np.int32)
    lst = np.zeros((idx.shape[0], maxn), np.int32)
    b = _box(box)
    lib().or_neighbors_sampled(p.shape[0], _d(p), C.byref(b), float(r_ns), idx.shape[0], _i(idx),
                               maxn, _i(cnt), _i(lst))
    if np.any(cnt > maxn):
        raise ValueError("oracle neighbour capacity exceeded")
    return cnt, [lst[s, :cnt[s]].copy() for s in range(idx.shape[0])]


def min_gap(pos, box, r_probe):
    """min over pairs of |r_ij - r_probe|."""
    p = _pos(pos)
    b = _box(box)
    return float(lib().or_min_gap(p.shape[0], _d(p), C.byref(b), float(r_probe)))


def pairs(pos, box, r_cut):
    """All ordered pairs i != j with r < r_c: (i, j, r_ij = x_i - x_j)."""
    p = _pos(pos)
    n = p.shape[0]
    b = _box(box)
    cap = max(1024, n * 128)
    pi = np.empty(cap, np.int32)
    pj = np.empty(cap, np.int32)
    rv = np.empty((cap, 3), np.float64)
    m = lib().or_pairs(n, _d(p), C.byref(b), float(r_cut), cap, _i(pi), _i(pj), _d(rv))
    if m > cap:
        raise ValueError("pair capacity exceeded")
    return pi[:m].copy(), pj[:m].copy(), rv[:m].copy()


# ----------------------------------------------------------------------------
# Potentials
# ----------------------------------------------------------------------------
class Result(dict):
    __getattr__ = dict.__getitem__


def lj(pos, box, eps, sigma, r_cut):
    """Shifted Lennard-Jones: per-atom forces, energies, virials and totals."""
    p = _pos(pos)
    n = p.shape[0]
    f = np.zeros((n, 3))
    e = np.zeros(n)
    w = np.zeros((n, 6))
    b = _box(box)
    lib().or_lj(n, _d(p), C.byref(b), float(eps), float(sigma), float(r_cut), _d(f), _d(e), _d(w))
    return Result(force=f, e_atom=e, w_atom=w, energy=float(np.sum(e)), virial=w.sum(axis=0))


def eam(pos, box, pot: EAMPotential):
    """Embedded-atom energy, forces and virial of all atoms (O(N^2))."""
    p = _pos(pos)
    n = p.shape[0]
    rb, fp, fpp = np.zeros(n), np.zeros(n), np.zeros(n)
    f, e, w = np.zeros((n, 3)), np.zeros(n), np.zeros((n, 6))
    b = _box(box)
    s = pot.cstruct()
    oor = lib().or_eam(n, _d(p), C.byref(b), C.byref(s), _d(rb), _d(fp), _d(fpp), _d(f), _d(e),
                       _d(w))
    return Result(force=f, e_atom=e, w_atom=w, rhobar=rb, fp=fp, fpp=fpp,
                  energy=float(np.sum(e)), virial=w.sum(axis=0), out_of_range=int(oor))


def eam_sampled(pos, box, pot: EAMPotential, idx):
    """EAM force, energy and rhobar of sampled atoms of a large system."""
    p = _pos(pos)
    idx = np.ascontiguousarray(np.asarray(idx, np.int32))
    ns = idx.shape[0]
    rb, f, e = np.zeros(ns), np.zeros((ns, 3)), np.zeros(ns)
    b = _box(box)
    s = pot.cstruct()
    oor = lib().or_eam_sampled(p.shape[0], _d(p), C.byref(b), C.byref(s), ns, _i(idx), _d(rb),
                               _d(f), _d(e))
    return Result(force=f, e_atom=e, rhobar=rb, out_of_range=int(oor))


def lj_sampled(pos, box, eps, sigma, r_cut, idx):
    p = _pos(pos)
    idx = np.ascontiguousarray(np.asarray(idx, np.int32))
    ns = idx.shape[0]
    f, e = np.zeros((ns, 3)), np.zeros(ns)
    b = _box(box)
    lib().or_lj_sampled(p.shape[0], _d(p), C.byref(b), float(eps), float(sigma), float(r_cut), ns,
                        _i(idx), _d(f), _d(e))
    return Result(force=f, e_atom=e)
