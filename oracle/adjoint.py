"""Force matching with EAM splines: loss and exact gradient (oracle; test infrastructure only).

The trainable potential is the single-element EAM of Sec. 1.6 / Sec. 3.3 with
its three tabulated functions phi(r), rho(r), F(rhobar) given as uniform cubic
B-splines (oracle.spline) with coefficient vectors c_phi, c_rho, c_F.

Forces (positions fixed; pairs p = (i, j), i != j, r_p < r_c; r_ij = x_i - x_j,
u_p = r_ij / r_p):
    rhobar_i = sum_{p: i_p = i} rho(r_p)
    F_i      = - sum_{p: i_p = i} [phi'(r_p) + (F'(rhobar_i) + F'(rhobar_j)) rho'(r_p)] u_p
Loss over S snapshots of N atoms:
    L = 1/(S N) sum_s sum_i |F_i - F_ref,i|^2,     G_i = dL/dF_i = 2 (F_i - F_ref,i) / (S N).
Gradient by the forward chain rule, term by term, contracted with G at the end
(g_p = G_{i_p} . u_p, beta_k the B-spline basis function of coefficient k):
    dL/dc_phi_k = - sum_p beta_k'(r_p) g_p
    dL/dc_F_k   = - sum_p [beta_k'(rhobar_i) + beta_k'(rhobar_j)] rho'(r_p) g_p
    dL/dc_rho_k = - sum_p (F'_i + F'_j) beta_k'(r_p) g_p
                  - sum_p (F''_i R_ik + F''_j R_jk) rho'(r_p) g_p,   R_ak = d rhobar_a / d c_rho_k
                                                                     = sum_{p: i_p = a} beta_k(r_p)
This does not use the pair-symmetric adjoint; it differentiates every
dependency directly, so it is an independent check of an adjoint kernel.
"""
from __future__ import annotations

import numpy as np

from . import core
from . import spline as sp


class Grid:
    def __init__(self, x_lo, h, ncoef):
        self.x_lo, self.h, self.ncoef = float(x_lo), float(h), int(ncoef)


class Snapshot:
    """Pairs of one fixed configuration within r_c."""

    def __init__(self, pos, box, r_cut):
        self.n = pos.shape[0]
        self.i, self.j, rv = core.pairs(pos, box, r_cut)
        self.r = np.sqrt(np.sum(rv * rv, axis=1))
        self.u = rv / self.r[:, None]


def _eval(c, g, x, d):
    return sp.evaluate(np.asarray(c, np.float64), g.x_lo, g.h, x, d)[0]


def forces(snap: Snapshot, c, grids):
    """(F [n,3], rhobar, F', F'') for coefficient vectors c = (c_phi, c_rho, c_F)."""
    c_phi, c_rho, c_emb = c
    g_phi, g_rho, g_emb = grids
    rho = _eval(c_rho, g_rho, snap.r, 0)
    drho = _eval(c_rho, g_rho, snap.r, 1)
    dphi = _eval(c_phi, g_phi, snap.r, 1)
    rb = np.bincount(snap.i, weights=rho, minlength=snap.n)
    fp = _eval(c_emb, g_emb, rb, 1)
    fpp = _eval(c_emb, g_emb, rb, 2)
    s = -(dphi + (fp[snap.i] + fp[snap.j]) * drho)
    F = np.stack([np.bincount(snap.i, weights=s * snap.u[:, a], minlength=snap.n)
                  for a in range(3)], axis=1)
    return F, rb, fp, fpp


def loss(snaps, c, grids, f_ref):
    tot, natoms = 0.0, 0
    for s, fr in zip(snaps, f_ref):
        F = forces(s, c, grids)[0]
        tot += float(np.sum((F - fr) ** 2))
        natoms += s.n
    return tot / natoms


def cotangents(snaps, c, grids, f_ref):
    """G_i = dL/dF_i for every snapshot."""
    natoms = sum(s.n for s in snaps)
    return [2.0 * (forces(s, c, grids)[0] - fr) / natoms for s, fr in zip(snaps, f_ref)]


def force_loss(F, f_ref):
    """Loss and cotangents of given per-snapshot forces F (lists of [N_s, 3] arrays):
    L = 1/(S N) sum_s sum_i |F_i - F_ref,i|^2 and G_i = 2 (F_i - F_ref,i) / (S N)."""
    natoms = sum(len(f) for f in F)
    tot = 0.0
    for f, fr in zip(F, f_ref):
        tot += float(np.sum((np.asarray(f, np.float64) - fr) ** 2))
    G = [2.0 * (np.asarray(f, np.float64) - fr) / natoms for f, fr in zip(F, f_ref)]
    return tot / natoms, G


def density_jacobian(snap: Snapshot, g_rho):
    """R [n, ncoef]: R_ak = d rhobar_a / d c_rho_k = sum over the pairs (a, j) of beta_k(r_aj)
    (rhobar is linear in the density coefficients)."""
    idx, W0 = sp.basis_weights(g_rho.ncoef, g_rho.x_lo, g_rho.h, snap.r, 0)
    R = np.zeros((snap.n, g_rho.ncoef))
    np.add.at(R, (np.repeat(snap.i, 4), idx.ravel()), W0.ravel())
    return R


def vjp(snaps, c, grids, G):
    """sum_s sum_i G_i . dF_i/dc for arbitrary cotangents G; returns (g_phi, g_rho, g_F)."""
    c_phi, c_rho, c_emb = c
    g_phi, g_rho, g_emb = grids
    out_phi = np.zeros(g_phi.ncoef)
    out_rho = np.zeros(g_rho.ncoef)
    out_emb = np.zeros(g_emb.ncoef)
    for snap, Gs in zip(snaps, G):
        _, rb, fp, fpp = forces(snap, c, grids)
        drho = _eval(c_rho, g_rho, snap.r, 1)
        g = np.sum(Gs[snap.i] * snap.u, axis=1)
        # phi block
        idx, W = sp.basis_weights(g_phi.ncoef, g_phi.x_lo, g_phi.h, snap.r, 1)
        np.add.at(out_phi, idx, -W * g[:, None])
        # embedding block
        q = drho * g
        idx, W = sp.basis_weights(g_emb.ncoef, g_emb.x_lo, g_emb.h, rb[snap.i], 1)
        np.add.at(out_emb, idx, -W * q[:, None])
        idx, W = sp.basis_weights(g_emb.ncoef, g_emb.x_lo, g_emb.h, rb[snap.j], 1)
        np.add.at(out_emb, idx, -W * q[:, None])
        # density block, direct term
        idx, W = sp.basis_weights(g_rho.ncoef, g_rho.x_lo, g_rho.h, snap.r, 1)
        np.add.at(out_rho, idx, -W * ((fp[snap.i] + fp[snap.j]) * g)[:, None])
        # density block, through rhobar
        R = density_jacobian(snap, g_rho)
        coef_i = fpp[snap.i] * q
        coef_j = fpp[snap.j] * q
        out_rho -= coef_i @ R[snap.i] + coef_j @ R[snap.j]
    return out_phi, out_rho, out_emb


def gradient(snaps, c, grids, f_ref):
    return vjp(snaps, c, grids, cotangents(snaps, c, grids, f_ref))


def fd_gradient(snaps, c, grids, f_ref, h=1e-6, which=None):
    """Central finite differences of the loss in FP64 (step h on each coefficient)."""
    c = [np.array(x, np.float64, copy=True) for x in c]
    out = [np.zeros_like(x) for x in c]
    for b in range(3):
        ks = range(c[b].shape[0]) if which is None else which[b]
        for k in ks:
            old = c[b][k]
            c[b][k] = old + h
            lp = loss(snaps, c, grids, f_ref)
            c[b][k] = old - h
            lm = loss(snaps, c, grids, f_ref)
            c[b][k] = old
            out[b][k] = (lp - lm) / (2 * h)
    return out
