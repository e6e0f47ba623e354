"""Slab profiles of flow and thermodynamic fields (oracle; test infrastructure only).

The Appendix defines, for a volume V_l holding N_l atoms (here: slabs of equal
width along one axis, atoms of equal mass m):

  M_l = sum_i m_i                                     mass of the slab
  u_l = sum_i m_i v_i / M_l                           centre-of-mass velocity
  E_kin^a = sum_i m_i (v_i^a - u_l^a)^2 / 2           kinetic energy per axis, in the
                                                      centre-of-mass frame
  T^a_l = 2 E_kin^a / (k_B N_l),   T_l = (T^x + T^y + T^z) / 3
  P^ab_l = [sum_i m_i (v^a - u^a)(v^b - u^b) + W^ab_l] / V_l,   P_l = trace / 3
  W^ab_l = sum over the slab's atoms of 1/2 sum_j r_ij^a f_ij^b

Readings where the text is garbled: the virial uses the central pair force f_ij on
i due to j with r_ij = x_i - x_j (the printed f_i^b multiplies the total force); the
potential energy per unit mass is sum_i U_i / M_l and the internal energy per unit
mass (sum_i U_i + E_kin) / M_l (the printed form divides by M_l twice); U_i is the
per-atom potential energy (EAM: F(rhobar_i) + 1/2 sum_j phi(r_ij), LJ: 1/2 sum_j U).
Velocities in angstrom/ps, masses in u: kinetic sums are converted to eV by 1/ACCEL.
"""
from __future__ import annotations

import numpy as np

from .integrate import ACCEL
from .thermostat import KB

FIELDS = ("N", "M", "ux", "uy", "uz", "Tx", "Ty", "Tz", "T", "Pxx", "Pyy", "Pzz", "Pxy", "Pxz",
          "Pyz", "P", "Epot_per_mass", "Eint_per_mass")


def slab_index(x, box, axis, lo, width, n_bins):
    """Slab of each atom (-1: outside); x folded into the box on a periodic axis."""
    xa = np.array(x[:, axis], np.float64, copy=True)
    if box.periodic[axis]:
        L, b0 = box.len[axis], box.lo[axis]
        xa = xa - L * np.floor((xa - b0) / L)
        xa[xa >= b0 + L] = b0
    q = np.floor((xa - lo) / width)
    ok = (q >= 0) & (q < n_bins)
    out = np.full(x.shape[0], -1)
    out[ok] = q[ok].astype(int)
    return out


def profiles(x, v, mass, e_atom, w_atom, box, axis, lo, width, n_bins):
    """[n_bins, 18] in the order of FIELDS.  e_atom [n] and w_atom [n, 6] (xx yy zz xy
    xz yz) may be None (their terms are then zero)."""
    area = 1.0
    for a in range(3):
        if a != axis:
            area *= box.len[a]
    vol = width * area
    slab = slab_index(x, box, axis, lo, width, n_bins)
    out = np.zeros((n_bins, len(FIELDS)))
    pairs = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))
    for l in range(n_bins):
        sel = slab == l
        n_l = int(np.count_nonzero(sel))
        if n_l == 0:
            continue
        m_l = mass * n_l
        u = (mass * v[sel]).sum(axis=0) / m_l
        dv = v[sel] - u
        kin = np.array([np.sum(mass * dv[:, a] * dv[:, b]) for a, b in pairs]) / ACCEL  # eV
        w = w_atom[sel].sum(axis=0) if w_atom is not None else np.zeros(6)
        epot = float(np.sum(e_atom[sel])) if e_atom is not None else 0.0
        t_axis = kin[:3] / (KB * n_l)  # T^a = 2 E_kin^a / (k_B N), E_kin^a = kin^aa / 2
        p = (kin + w) / vol
        row = [n_l, m_l, u[0], u[1], u[2], t_axis[0], t_axis[1], t_axis[2], t_axis.mean()]
        row += list(p) + [p[:3].mean(), epot / m_l, (epot + 0.5 * kin[:3].sum()) / m_l]
        out[l] = row
    return out
