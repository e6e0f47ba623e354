"""Pins of the oracle's Behler-Parrinello potential (oracle/bpnn.py, Sec. 2.1).

  cutoff function       f_c(0) = 1, f_c(R_c / 2) = 1/2, f_c(R_c) = 0, f_c' by differences
  dimer                 G2 = exp(-eta (R - R_s)^2) f_c(R) exactly, no angular terms
  equilateral trimer    G4 = 2^(1 - zeta) 2 (1 + lambda / 2)^zeta exp(-3 eta s^2) f_c(s)^3
  network               dE/dG of the backward pass equals central differences
  forces                F = -grad E by central differences; sum F = 0; a constant network
                        gives zero forces
  invariances           translation, rotation (free cluster) and relabelling of atoms
  virial                W^aa = -dE/d(strain_aa) by differences of a strained box
"""
import math

import numpy as np
import pytest

import mdinputs as mi
from oracle import bpnn

P = mi.bpnn_params()


def _cluster(n=14, seed=3):
    """A free cluster (non-periodic box) of n atoms at fcc-like spacings."""
    rng = np.random.default_rng(seed)
    pos, _ = mi.fcc_lattice(2, 2, 2, 3.615)
    x = pos[:n] + rng.normal(0.0, 0.08, (n, 3)) + 20.0
    return x, mi.Box((0.0, 0.0, 0.0), (60.0, 60.0, 60.0), (0, 0, 0))


def test_cutoff_function():
    rc = P["r_cut"]
    fc, dfc = bpnn.cutoff(np.array([0.0, rc / 2, rc, rc + 1.0]), rc)
    assert np.allclose(fc, [1.0, 0.5, 0.0, 0.0], atol=1e-15)
    R = np.array([1.3, 2.9, 4.4, 5.7])
    h = 1e-6
    fd = (bpnn.cutoff(R + h, rc)[0] - bpnn.cutoff(R - h, rc)[0]) / (2 * h)
    assert np.allclose(bpnn.cutoff(R, rc)[1], fd, rtol=1e-8, atol=1e-10)


def test_dimer_radial_closed_form():
    R = 2.7
    a = np.array([[R, 0.0, 0.0]])
    G = bpnn.descriptors_atom(a, np.array([R]), P)
    fc = 0.5 * (math.cos(math.pi * R / P["r_cut"]) + 1.0)
    want = [math.exp(-e * (R - P["r_s"]) ** 2) * fc for e in P["g2_eta"]]
    assert np.allclose(G[:8], want, rtol=1e-14)
    assert np.all(G[8:] == 0.0)


def test_equilateral_trimer_angular_closed_form():
    s = 2.9
    a = np.array([[s, 0.0, 0.0], [s / 2, s * math.sqrt(3.0) / 2, 0.0]])
    G = bpnn.descriptors_atom(a, np.linalg.norm(a, axis=1), P)
    fc = 0.5 * (math.cos(math.pi * s / P["r_cut"]) + 1.0)
    for q in range(len(P["g4_eta"])):
        z, l, e = P["g4_zeta"][q], P["g4_lambda"][q], P["g4_eta"][q]
        want = 2.0 ** (1 - z) * 2.0 * (1 + l * 0.5) ** z * math.exp(-3 * e * s * s) * fc ** 3
        assert math.isclose(G[8 + q], want, rel_tol=1e-12, abs_tol=1e-300)


def test_network_gradient_by_differences():
    rng = np.random.default_rng(9)
    G = np.concatenate([rng.uniform(0, 15, 8), rng.uniform(0, 200, 43)])
    _, dG = bpnn.network(G, P)
    for mu in (0, 3, 7, 8, 20, 50):
        h = 1e-4 * max(1.0, abs(G[mu]))
        gp, gm = G.copy(), G.copy()
        gp[mu] += h
        gm[mu] -= h
        fd = (bpnn.network(gp, P)[0] - bpnn.network(gm, P)[0]) / (2 * h)
        assert abs(fd - dG[mu]) <= 1e-7 * max(abs(dG).max(), 1e-12)


def _fd_force(x, box, i, a, h=1e-4):
    # h = 1e-4: the rounding noise of the total energy (|E| ~ 300 eV) over 2h stays near
    # 1e-10 eV/A, the truncation error (h^2) below it
    xp, xm = x.copy(), x.copy()
    xp[i, a] += h
    xm[i, a] -= h
    return -(bpnn.energy(xp, box, P)[0] - bpnn.energy(xm, box, P)[0]) / (2 * h)


@pytest.mark.parametrize("where", ["cluster", "periodic"])
def test_forces_are_minus_energy_gradient(where):
    if where == "cluster":
        x, box = _cluster()
    else:
        s = mi.bpnn_copper(cells=4)  # L/2 = 7.2 A > r_c: one image per pair
        x, box = s.pos, s.box
    E, e, f, _ = bpnn.forces(x, box, P)
    assert math.isclose(E, e.sum(), rel_tol=1e-14)
    assert math.isclose(E, bpnn.energy(x, box, P)[0], rel_tol=1e-14)
    assert np.abs(f.sum(axis=0)).max() < 1e-12 * max(1.0, np.abs(f).max())
    for i, a in ((0, 0), (5, 2), (11, 1)):
        assert abs(_fd_force(x, box, i, a) - f[i, a]) <= 2e-7 * np.abs(f).max()


def test_constant_network_gives_zero_forces():
    q = dict(P)
    q["w12"] = np.zeros_like(P["w12"])
    x, box = _cluster()
    E, e, f, w = bpnn.forces(x, box, q)
    const = q["b3"] + float(np.tanh(q["b2"]) @ q["w23"])
    assert np.allclose(e, const, rtol=1e-14)
    assert np.all(f == 0.0) and np.all(w == 0.0)


def test_invariances():
    x, box = _cluster()
    E, e, _, _ = bpnn.forces(x, box, P)
    # translation
    E2, _, _, _ = bpnn.forces(x + np.array([1.7, -2.2, 0.9]), box, P)
    assert math.isclose(E, E2, rel_tol=1e-13)
    # rotation about the cluster centre
    t = 0.7
    rot = np.array([[math.cos(t), -math.sin(t), 0.0], [math.sin(t), math.cos(t), 0.0],
                    [0.0, 0.0, 1.0]])
    c = x.mean(axis=0)
    E3, _, _, _ = bpnn.forces((x - c) @ rot.T + c, box, P)
    assert math.isclose(E, E3, rel_tol=1e-12)
    # relabelling permutes the atomic energies
    perm = np.random.default_rng(1).permutation(len(x))
    _, e4, _, _ = bpnn.forces(x[perm], box, P)
    assert np.allclose(e4, e[perm], rtol=1e-13)


def test_virial_is_strain_derivative():
    s = mi.bpnn_copper(cells=4)
    x, box = s.pos, s.box
    _, _, _, w = bpnn.forces(x, box, P)
    h = 1e-6
    for a in range(3):
        es = []
        for sg in (h, -h):
            sc = np.ones(3)
            sc[a] += sg
            b2 = mi.Box(box.lo, tuple(np.array(box.len) * sc), box.periodic)
            es.append(bpnn.energy(x * sc, b2, P)[0])
        assert abs(-(es[0] - es[1]) / (2 * h) - w[a]) < 1e-6 * abs(w[a]) + 1e-9
