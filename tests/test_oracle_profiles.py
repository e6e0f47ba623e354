"""Pins of the oracle's slab profiles (oracle/profiles.py, the Appendix definitions).

  hand example         four atoms in two slabs: centre-of-mass velocity, T per axis,
                       kinetic pressure, energies worked out by hand
  perfect crystal      LJ and EAM lattices at rest: every slab's pressure is the
                       closed-form -dE/dV of the lattice sum; T = 0; E_pot/M = E/atom / m
  Galilean invariance  a uniform velocity shifts u_l only
  ideal-gas identity   with no potential terms P_l = N_l k_B T_l / V_l exactly
  sum rules            slab counts add up to N, slab kinetic tensors plus M u u to the
                       total kinetic tensor; atoms past the box edge fold back in
"""
import numpy as np
import pytest

import mdinputs as mi
from oracle import core, integrate, profiles as pr
from oracle.thermostat import KB
from tests import lattice_sums as ls

F = {k: i for i, k in enumerate(pr.FIELDS)}


def test_hand_worked_example():
    box = mi.Box((0.0, 0.0, 0.0), (2.0, 3.0, 10.0), (1, 1, 0))
    x = np.array([[0.5, 0.5, 1.0], [1.5, 2.5, 2.0], [1.0, 1.0, 4.9], [1.0, 1.0, 7.0]])
    v = np.array([[1.0, 0.0, 0.0], [-1.0, 0.0, 0.0], [0.0, 2.0, 0.0], [3.0, -1.0, 2.0]])
    e = np.array([-1.0, -2.0, -3.0, -4.0])
    w = np.zeros((4, 6))
    w[:, 0] = [0.5, 0.5, 0.5, 1.0]
    m = integrate.ACCEL  # m / ACCEL = 1: kinetic sums in eV are plain sums of dv^2
    out = pr.profiles(x, v, m, e, w, box, axis=2, lo=0.0, width=5.0, n_bins=2)
    s0, s1 = out
    # slab 0 (z < 5): u = (0, 2/3, 0); dv = (1, -2/3, 0), (-1, -2/3, 0), (0, 4/3, 0)
    assert s0[F["N"]] == 3 and np.isclose(s0[F["M"]], 3 * m)
    assert np.allclose(s0[[F["ux"], F["uy"], F["uz"]]], [0.0, 2.0 / 3.0, 0.0])
    kxx, kyy = 2.0, 4.0 / 9 + 4.0 / 9 + 16.0 / 9
    assert np.isclose(s0[F["Tx"]], kxx / (KB * 3)) and np.isclose(s0[F["Ty"]], kyy / (KB * 3))
    assert s0[F["Tz"]] == 0.0
    vol = 5.0 * 2.0 * 3.0
    assert np.isclose(s0[F["Pxx"]], (kxx + 1.5) / vol) and np.isclose(s0[F["Pyy"]], kyy / vol)
    assert np.isclose(s0[F["Pxy"]], 0.0, atol=1e-15)  # 1(-2/3) + (-1)(-2/3) + 0
    assert np.isclose(s0[F["Epot_per_mass"]], -6.0 / (3 * m))
    assert np.isclose(s0[F["Eint_per_mass"]], (-6.0 + 0.5 * (kxx + kyy)) / (3 * m))
    # slab 1: one atom, at rest in its own frame
    assert s1[F["N"]] == 1 and np.allclose(s1[[F["ux"], F["uy"], F["uz"]]], [3.0, -1.0, 2.0])
    assert s1[F["T"]] == 0.0 and np.isclose(s1[F["Pxx"]], 1.0 / vol)


@pytest.mark.parametrize("pot", ["lj", "eam"])
def test_crystal_slab_pressure_is_lattice_derivative(pot):
    if pot == "lj":
        p, a, m = mi.LJ_AR, 5.26, mi.MASS["Ar"]
        pos, box = mi.fcc_lattice(4, 4, 6, a)
        r = core.lj(pos, box, p.eps, p.sigma, p.r_cut)
        e_of = lambda aa: ls.lj_energy_per_atom(aa, p.eps, p.sigma, p.r_cut)
        h = 1e-5
        dEda = (e_of(a + h) - e_of(a - h)) / (2 * h)
        e_atom = e_of(a)
    else:
        p, a, m = mi.EAM_CU, 3.615, mi.MASS["Cu"]
        pos, box = mi.fcc_lattice(4, 4, 6, a)
        r = core.eam(pos, box, core.EAMPotential.analytic(p))
        dEda = ls.eam_dE_da(a, p)
        e_atom = ls.eam_per_atom(a, p)[0]
    # slabs of one cell along z: two atomic planes each
    out = pr.profiles(pos, np.zeros_like(pos), m, r.e_atom, r.w_atom, box, 2, -a / 4, a, 6)
    # P = -dE/dV with V = a^3 / 4 per atom
    p_want = -dEda / (3.0 * a * a / 4.0)
    assert np.allclose(out[:, F["P"]], p_want, rtol=1e-7, atol=0)
    assert np.allclose(out[:, F["Pxx"]], out[:, F["Pzz"]], rtol=1e-12)
    assert np.allclose(out[:, [F["Pxy"], F["Pxz"], F["Pyz"]]], 0.0, atol=1e-12)
    assert np.all(out[:, F["T"]] == 0.0) and np.all(out[:, F["N"]] == 4 * 4 * 4)
    assert np.allclose(out[:, F["Epot_per_mass"]], e_atom / m, rtol=1e-9)


def _thermal_slabs(n=60000, seed=3):
    rng = np.random.default_rng(seed)
    box = mi.Box((0.0, 0.0, 0.0), (30.0, 30.0, 60.0), (1, 1, 1))
    x = rng.uniform(0.0, 1.0, (n, 3)) * np.array(box.len)
    v = rng.normal(0.0, 2.0, (n, 3)) + np.array([0.0, 0.0, 5.0])
    e = rng.normal(-3.0, 0.1, n)
    w = rng.normal(0.0, 0.2, (n, 6))
    return box, x, v, e, w


def test_galilean_invariance():
    box, x, v, e, w = _thermal_slabs()
    c = np.array([3.0, -7.0, 11.0])
    a = pr.profiles(x, v, 26.98, e, w, box, 2, 0.0, 6.0, 10)
    b = pr.profiles(x, v + c, 26.98, e, w, box, 2, 0.0, 6.0, 10)
    u = [F["ux"], F["uy"], F["uz"]]
    assert np.allclose(b[:, u], a[:, u] + c, rtol=0, atol=1e-12)
    rest = [k for k in range(len(pr.FIELDS)) if k not in u]
    assert np.allclose(b[:, rest], a[:, rest], rtol=1e-9, atol=1e-12)


def test_ideal_gas_identity_and_sum_rules():
    box, x, v, _, _ = _thermal_slabs()
    m, width, nb = 39.948, 6.0, 10
    out = pr.profiles(x, v, m, None, None, box, 2, 0.0, width, nb)
    vol = width * box.len[0] * box.len[1]
    assert np.allclose(out[:, F["P"]], out[:, F["N"]] * KB * out[:, F["T"]] / vol, rtol=1e-12)
    assert out[:, F["N"]].sum() == x.shape[0]
    # sum_l (K_l + M_l u_l u_l) = sum_i m v v   (diagonal, eV)
    kin = out[:, [F["Pxx"], F["Pyy"], F["Pzz"]]] * vol
    uu = out[:, [F["ux"], F["uy"], F["uz"]]] ** 2
    tot = (kin + out[:, [F["M"]]] * uu / integrate.ACCEL).sum(axis=0)
    assert np.allclose(tot, m * (v * v).sum(axis=0) / integrate.ACCEL, rtol=1e-12)
    # Maxwell-Boltzmann draw: T per axis near m s^2 / k_B with s = 2 angstrom/ps
    t0 = m * 4.0 / integrate.ACCEL / KB
    assert np.allclose(out[:, [F["Tx"], F["Ty"], F["Tz"]]], t0, rtol=0.05)


def test_periodic_fold_and_outside():
    box = mi.Box((0.0, 0.0, 0.0), (10.0, 10.0, 10.0), (1, 1, 0))
    x = np.array([[10.5, 1.0, 1.0], [-0.5, 1.0, 1.0], [1.0, 1.0, 11.0], [1.0, 1.0, -1.0]])
    assert list(pr.slab_index(x, box, 0, 0.0, 1.0, 10)) == [0, 9, 1, 1]
    assert list(pr.slab_index(x, box, 2, 0.0, 1.0, 10)) == [1, 1, -1, -1]
