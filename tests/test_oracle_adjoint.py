"""Pins of the oracle's force-matching loss and gradient."""
import numpy as np
import pytest

import mdinputs as mi
from oracle import adjoint as adj
from oracle import core
from oracle import spline as sp


@pytest.fixture(scope="module")
def problem():
    tab = mi.force_matching_tables()
    grids = tuple(adj.Grid(tf.x_lo, tf.h, tf.K + 2) for tf in (tab.phi, tab.rho, tab.emb))
    c0 = [sp.fit_table(tf) for tf in (tab.phi, tab.rho, tab.emb)]
    noise = mi.coefficient_noise()
    c = [c0[b] * noise[64 * b:64 * (b + 1)] for b in range(3)]
    snaps_in = mi.force_matching_snapshots(n_snap=2, cells=4)
    snaps = [adj.Snapshot(s.pos, s.box, mi.EAM_CU.r_cut) for s in snaps_in]
    pot = core.EAMPotential.analytic(mi.EAM_CU)
    f_ref = [core.eam(s.pos, s.box, pot).force for s in snaps_in]
    return snaps, snaps_in, c, c0, grids, f_ref


def test_forces_match_core_eam(problem):
    """The pair-list force evaluation equals the O(N^2) EAM on the same splines."""
    snaps, snaps_in, c, c0, grids, f_ref = problem
    pot = core.EAMPotential(*(core.SplineFunc(c[b], grids[b].x_lo, grids[b].h) for b in range(3)),
                            mi.EAM_CU.r_cut)
    for s, si in zip(snaps, snaps_in):
        F = adj.forces(s, c, grids)[0]
        r = core.eam(si.pos, si.box, pot)
        assert np.max(np.abs(F - r.force)) < 1e-11


def test_gradient_matches_central_fd(problem):
    snaps, snaps_in, c, c0, grids, f_ref = problem
    g = adj.gradient(snaps, c, grids, f_ref)
    ks = [np.arange(0, 64, 3), np.arange(1, 64, 3), np.arange(0, 64, 2)]
    fd = adj.fd_gradient(snaps, c, grids, f_ref, h=1e-6, which=ks)
    for b in range(3):
        scale = np.max(np.abs(g[b])) + 1e-300
        err = np.max(np.abs(g[b][ks[b]] - fd[b][ks[b]])) / scale
        assert err < 1e-6, (b, err)


def test_vjp_columns_match_fd_of_forces(problem):
    """G = unit cotangent on one force component: the VJP is a Jacobian row, checked by FD
    of that force component itself."""
    snaps, snaps_in, c, c0, grids, f_ref = problem
    s = snaps[:1]
    G = [np.zeros((s[0].n, 3))]
    G[0][7, 1] = 1.0
    g = adj.vjp(s, c, grids, G)
    h = 1e-6
    for b, k in ((0, 30), (1, 20), (1, 45), (2, 25)):
        cp = [x.copy() for x in c]
        cm = [x.copy() for x in c]
        cp[b][k] += h
        cm[b][k] -= h
        fd = (adj.forces(s[0], cp, grids)[0][7, 1] - adj.forces(s[0], cm, grids)[0][7, 1]) / (2 * h)
        assert abs(fd - g[b][k]) < 1e-6 * max(1.0, abs(fd)), (b, k)


def test_zero_gradient_at_exact_fit(problem):
    snaps, snaps_in, c, c0, grids, f_ref = problem
    f_self = [adj.forces(s, c, grids)[0] for s in snaps]
    assert adj.loss(snaps, c, grids, f_self) == 0.0
    g = adj.gradient(snaps, c, grids, f_self)
    assert all(np.max(np.abs(x)) == 0.0 for x in g)


def test_loss_quadratic_in_phi_block(problem):
    """F is affine in c_phi, so L is quadratic there and central FD is exact for any step."""
    snaps, snaps_in, c, c0, grids, f_ref = problem
    g = adj.gradient(snaps, c, grids, f_ref)
    fd = adj.fd_gradient(snaps, c, grids, f_ref, h=0.5, which=[[10, 40], [], []])
    for k in (10, 40):
        assert abs(fd[0][k] - g[0][k]) < 1e-8 * max(1.0, abs(g[0][k]))


def test_unperturbed_spline_is_close_to_reference(problem):
    snaps, snaps_in, c, c0, grids, f_ref = problem
    assert adj.loss(snaps, c0, grids, f_ref) < 1e-4 * adj.loss(snaps, c, grids, f_ref)


def test_force_loss_pins():
    """force_loss on given forces: zero at F = F_ref; a uniform offset d on every component of
    every atom gives L = 3 d^2 whatever the snapshot sizes; G is the central difference of L in
    each force component (catches the factor 2 and the 1/(S N) normalisation); brute force
    over atoms and components on a tiny input."""
    rng = np.random.default_rng(11)
    f_ref = [rng.normal(size=(5, 3)), rng.normal(size=(2, 3))]
    L0, G0 = adj.force_loss([f.copy() for f in f_ref], f_ref)
    assert L0 == 0.0 and all(np.all(g == 0.0) for g in G0)
    L1, _ = adj.force_loss([f + 0.25 for f in f_ref], f_ref)
    assert abs(L1 - 3 * 0.25 ** 2) < 1e-15
    F = [f + rng.normal(scale=0.3, size=f.shape) for f in f_ref]
    L, G = adj.force_loss(F, f_ref)
    brute = 0.0
    for f, fr in zip(F, f_ref):
        for i in range(len(f)):
            for a in range(3):
                brute += (f[i, a] - fr[i, a]) * (f[i, a] - fr[i, a])
    assert abs(L - brute / 7) < 1e-14
    h = 1e-6
    for s in range(2):
        for i in range(len(F[s])):
            for a in range(3):
                Fp = [f.copy() for f in F]
                Fm = [f.copy() for f in F]
                Fp[s][i, a] += h
                Fm[s][i, a] -= h
                fd = (adj.force_loss(Fp, f_ref)[0] - adj.force_loss(Fm, f_ref)[0]) / (2 * h)
                assert abs(fd - G[s][i, a]) < 1e-8


def test_force_loss_agrees_with_loss_and_cotangents(problem):
    snaps, snaps_in, c, c0, grids, f_ref = problem
    F = [adj.forces(s, c, grids)[0] for s in snaps]
    L, G = adj.force_loss(F, f_ref)
    assert abs(L - adj.loss(snaps, c, grids, f_ref)) <= 1e-15 * L
    for g, g2 in zip(G, adj.cotangents(snaps, c, grids, f_ref)):
        assert np.array_equal(g, g2)


def test_density_jacobian_pins(problem):
    """density_jacobian: R c_rho reproduces rhobar of the force evaluation (rhobar is linear in
    the density coefficients); a unit step in one coefficient changes rhobar by that column;
    each row sums to the number of pairs of the atom inside the grid (partition of unity)."""
    snaps, snaps_in, c, c0, grids, f_ref = problem
    g_rho = grids[1]
    for s in snaps:
        R = adj.density_jacobian(s, g_rho)
        rb = adj.forces(s, c, grids)[1]
        assert np.max(np.abs(R @ c[1] - rb)) <= 1e-12 * np.max(np.abs(rb))
        for k in (15, 30, 45):
            cp = [c[0], c[1].copy(), c[2]]
            cp[1][k] += 1.0
            d = adj.forces(s, cp, grids)[1] - rb
            assert np.max(np.abs(d - R[:, k])) < 1e-11
        npairs = np.bincount(s.i, minlength=s.n)
        assert np.allclose(R.sum(axis=1), npairs, rtol=0, atol=1e-12)
