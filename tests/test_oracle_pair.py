"""Pins of the oracle's geometry, neighbour sets, Lennard-Jones and velocity Verlet."""
import json
import os

import numpy as np
import pytest

import mdinputs as mi
from oracle import core, integrate
from tests import lattice_sums as ls

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.json")


def _disp(pos, box, sigma, seed, r_probe=None, gap=1e-4):
    """Seeded displacement; with r_probe, the first seed from `seed` on whose pairs all stay
    `gap` away from r_probe (so that a finite-difference step never crosses the cutoff)."""
    for s in range(seed, seed + 100):
        rng = np.random.default_rng(s)
        x = core.wrap(pos + rng.normal(0, sigma, pos.shape), box)
        if r_probe is None or core.min_gap(x, box, r_probe) > gap:
            return x
    raise RuntimeError("no configuration clear of the cutoff")


# ----------------------------------------------------------------------------
# wrap and minimum image
# ----------------------------------------------------------------------------
def test_wrap_folds_by_whole_periods():
    pos, box = mi.fcc_lattice(3, 3, 3, 5.26)
    rng = np.random.default_rng(0)
    shift = rng.integers(-3, 4, pos.shape) * np.array(box.len)
    w = core.wrap(pos + shift + 1e-3, box)
    L = np.array(box.len)
    assert np.all(w >= 0) and np.all(w < L)
    k = (pos + shift + 1e-3 - w) / L
    assert np.allclose(k, np.rint(k), atol=1e-9)
    assert np.array_equal(core.wrap(w, box), w)


def test_wrap_boundary_rounding_goes_to_lo():
    pos, box = mi.fcc_lattice(1, 1, 1, 4.0)
    x = np.array([[-1e-17, 0.5, 4.0]])
    w = core.wrap(x, box)
    assert w[0, 0] == 0.0 and w[0, 2] == 0.0


def test_non_periodic_axis_is_not_wrapped():
    box = mi.Box((0, 0, 0), (10, 10, 10), (1, 1, 0))
    x = np.array([[11.0, -1.0, 12.5]])
    w = core.wrap(x, box)
    assert w[0, 2] == 12.5 and w[0, 0] == 1.0 and w[0, 1] == 9.0


# ----------------------------------------------------------------------------
# neighbour sets
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("a,rns,cells", [(5.26, 8.8125, 4), (3.615, 5.8, 5), (3.30, 5.8, 4),
                                         (4.20, 5.8, 4), (4.05, 6.3, 4)])
def test_neighbor_counts_equal_fcc_shell_counts(a, rns, cells):
    pos, box = mi.fcc_lattice(cells, cells, cells, a)
    cnt, _ = core.neighbor_sets(pos, box, rns)
    assert np.all(cnt == ls.count_within(a, rns))


def test_neighbor_sets_symmetric_and_relabel_invariant():
    pos, box = mi.fcc_lattice(4, 4, 4, 3.615)
    x = _disp(pos, box, 0.1, 3)
    cnt, lst = core.neighbor_sets(x, box, 5.8)
    pairs = {(i, j) for i in range(len(x)) for j in lst[i]}
    assert all((j, i) in pairs for i, j in pairs)
    perm = np.random.default_rng(4).permutation(len(x))
    cnt2, lst2 = core.neighbor_sets(x[perm], box, 5.8)
    pairs2 = {(perm[i], perm[j]) for i in range(len(x)) for j in lst2[i]}
    assert pairs2 == pairs


def test_neighbor_set_matches_dense_distance_matrix():
    """Tiny brute force written independently with numpy broadcasting."""
    pos, box = mi.fcc_lattice(3, 3, 3, 5.26)
    x = _disp(pos, box, 0.2, 5)
    L = np.array(box.len)
    d = x[None, :, :] - x[:, None, :]
    d = d - L * np.rint(d / L)
    r2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
    np.fill_diagonal(r2, np.inf)
    cnt, lst = core.neighbor_sets(x, box, 7.5)
    for i in range(len(x)):
        assert np.array_equal(lst[i], np.nonzero(r2[i] < 7.5 ** 2)[0])


def _dense_r2(x, box):
    """All squared minimum-image distances by numpy broadcasting (periodic axes only get the
    image shift), in the same operation order as the definition: (dx dx + dy dy) + dz dz."""
    L = np.array(box.len, np.float64)
    per = np.array(box.periodic, bool)
    d = x[None, :, :] - x[:, None, :]
    d = np.where(per, d - L * np.rint(d / np.where(per, L, 1.0)), d)
    return (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]


@pytest.mark.parametrize("cells,a,rns,periodic", [(3, 5.26, 7.5, (1, 1, 1)),
                                                   (4, 3.615, 5.8, (1, 1, 1)),
                                                   (5, 3.30, 5.8, (1, 1, 0)),
                                                   (3, 4.05, 6.0, (0, 1, 1))])
def test_sampled_neighbor_sets_match_brute_force(cells, a, rns, periodic):
    """The sampled neighbour sets (used to check large systems) against a numpy distance
    matrix and against the full oracle, for an unsorted sample with repeats that includes
    atoms next to every face of the box (eq. 1.2)."""
    pos, _ = mi.fcc_lattice(cells, cells, cells, a)
    box = mi.Box((0.0, 0.0, 0.0), (cells * a,) * 3, periodic)
    x = _disp(pos, box, 0.15, 11)
    n = len(x)
    r2 = _dense_r2(x, box)
    np.fill_diagonal(r2, np.inf)
    L = np.array(box.len)
    near_face = np.nonzero(np.any((x < 0.6) | (x > L - 0.6), axis=1))[0]
    rng = np.random.default_rng(cells)
    idx = np.concatenate([rng.permutation(near_face)[:12], rng.integers(0, n, 20),
                          [n - 1, 0, 0]]).astype(np.int32)
    cnt, lst = core.neighbor_sets_sampled(x, box, rns, idx)
    cnt_all, lst_all = core.neighbor_sets(x, box, rns)
    assert len(lst) == len(idx)
    for s, i in enumerate(idx):
        want = np.nonzero(r2[i] < rns * rns)[0]
        assert cnt[s] == len(want)
        assert np.array_equal(lst[s], want)
        assert np.array_equal(lst[s], lst_all[i])


def test_min_gap_matches_brute_force():
    """min over pairs of |r_ij - r_probe| against numpy's all-pairs distances, for probes
    between, near and on shell radii, periodic and walled boxes."""
    pos, _ = mi.fcc_lattice(3, 3, 3, 3.615)
    for periodic in ((1, 1, 1), (1, 0, 1)):
        box = mi.Box((0.0, 0.0, 0.0), (3 * 3.615,) * 3, periodic)
        x = _disp(pos, box, 0.08, 21)
        r = np.sqrt(_dense_r2(x, box))
        iu = np.triu_indices(len(x), 1)
        n = len(x)
        # probes on the exact distance of chosen pairs (first, adjacent, last atoms) give a
        # gap of zero only if that pair is visited
        exact = [float(r[0, 1]), float(r[7, 8]), float(r[3, n - 1]), float(r[n - 2, n - 1])]
        for probe in [2.556, 3.615 / np.sqrt(2), 4.4, 5.5] + exact:
            want = np.min(np.abs(r[iu] - probe))
            assert core.min_gap(x, box, probe) == pytest.approx(want, rel=0, abs=1e-12)
        for probe in exact:
            assert core.min_gap(x, box, probe) < 1e-12


# ----------------------------------------------------------------------------
# Lennard-Jones
# ----------------------------------------------------------------------------
def test_lj_lattice_energy_closed_form():
    p = mi.LJ_AR
    pos, box = mi.fcc_lattice(4, 4, 4, 5.26)
    r = core.lj(pos, box, p.eps, p.sigma, p.r_cut)
    want = ls.lj_energy_per_atom(5.26, p.eps, p.sigma, p.r_cut)
    assert abs(r.energy / len(pos) - want) < 1e-13
    assert abs(want - (-0.0775879839)) < 1e-10
    assert np.max(np.abs(r.force)) < 1e-12


def test_lj_paper_argon_sample_lattice_energy():
    """The argon basic sample of the moving-window example (Sec. 3.1) on a perfect lattice."""
    g = json.load(open(GOLDEN))
    s = g["argon_basic_sample"]
    eps = s["eps_kj_per_mol"] * g["kj_per_mol_in_eV"]
    pos, box = mi.fcc_lattice(5, 5, 5, s["a_angstrom"])
    r = core.lj(pos, box, eps, s["sigma_angstrom"], s["r_cut_angstrom"])
    want = ls.lj_energy_per_atom(s["a_angstrom"], eps, s["sigma_angstrom"], s["r_cut_angstrom"])
    assert abs(r.energy / len(pos) - want) < 1e-13


def _lj_energy(x, box):
    p = mi.LJ_AR
    return core.lj(x, box, p.eps, p.sigma, p.r_cut).energy


def test_lj_newton_third_law_and_fd_forces():
    p = mi.LJ_AR
    pos, box = mi.fcc_lattice(4, 4, 4, 5.26)
    x = _disp(pos, box, 0.15, 7, r_probe=p.r_cut)
    r = core.lj(x, box, p.eps, p.sigma, p.r_cut)
    assert np.max(np.abs(r.force.sum(axis=0))) < 1e-13
    h = 1e-5
    for i in (0, 17, 200):
        for a in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, a] += h
            xm[i, a] -= h
            fd = -(_lj_energy(xp, box) - _lj_energy(xm, box)) / (2 * h)
            assert abs(fd - r.force[i, a]) <= 1e-7 * max(1.0, np.abs(r.force).max())


def test_lj_virial_is_strain_derivative():
    """W^aa = -dE/d(eps_aa) for a homogeneous strain of positions and box."""
    p = mi.LJ_AR
    pos, box = mi.fcc_lattice(4, 4, 4, 5.26)
    x = _disp(pos, box, 0.15, 8)
    r = core.lj(x, box, p.eps, p.sigma, p.r_cut)
    h = 1e-6
    for a in range(3):
        es = []
        for s in (h, -h):
            sc = np.ones(3)
            sc[a] += s
            b2 = mi.Box(box.lo, tuple(np.array(box.len) * sc), box.periodic)
            es.append(_lj_energy(x * sc, b2))
        assert abs(-(es[0] - es[1]) / (2 * h) - r.virial[a]) < 1e-6 * abs(r.virial[a]) + 1e-9


def test_lj_invariances():
    p = mi.LJ_AR
    pos, box = mi.fcc_lattice(4, 4, 4, 5.26)
    x = _disp(pos, box, 0.15, 9)
    r = core.lj(x, box, p.eps, p.sigma, p.r_cut)
    # translation across the periodic boundary
    xt = core.wrap(x + np.array([7.3, -11.1, 20.9]), box)
    rt = core.lj(xt, box, p.eps, p.sigma, p.r_cut)
    assert np.max(np.abs(rt.force - r.force)) < 1e-12 and abs(rt.energy - r.energy) < 1e-11
    # relabelling
    perm = np.random.default_rng(1).permutation(len(x))
    rp = core.lj(x[perm], box, p.eps, p.sigma, p.r_cut)
    assert np.max(np.abs(rp.force - r.force[perm])) < 1e-12
    # cubic axis permutation (x, y, z) -> (y, z, x)
    rc = core.lj(x[:, [1, 2, 0]], box, p.eps, p.sigma, p.r_cut)
    assert np.max(np.abs(rc.force - r.force[:, [1, 2, 0]])) < 1e-12
    assert np.allclose(rc.virial[:3], r.virial[[1, 2, 0]], atol=1e-11)


# ----------------------------------------------------------------------------
# velocity Verlet
# ----------------------------------------------------------------------------
def test_verlet_free_particle_and_constant_force():
    """Closed forms: x(t) = x0 + v0 t + a t^2 / 2 for a constant force."""
    box = mi.Box((0, 0, 0), (100, 100, 100), (0, 0, 0))
    x0 = np.array([[10.0, 20.0, 30.0]])
    v0 = np.array([[1.0, -2.0, 0.5]])
    fconst = np.array([[0.3, 0.0, -0.1]])
    m, dt, n = 12.0, 1e-3, 50
    x, v, f, _ = integrate.run_nve(x0, v0, box, m, dt, n, lambda x: (fconst, 0.0))
    t = n * dt
    acc = fconst / m * integrate.ACCEL
    assert np.allclose(x, x0 + v0 * t + 0.5 * acc * t * t, atol=1e-12)
    assert np.allclose(v, v0 + acc * t, atol=1e-12)


def test_verlet_time_reversible_and_conserves_energy():
    s = mi.lj_argon()
    fn = integrate.lj_force_fn(s.box, s.lj)
    x, v, f, h = integrate.run_nve(s.pos, s.vel, s.box, s.mass, s.dt_ps, 100, fn)
    e = h[:, 1] + h[:, 2]
    assert np.max(np.abs(e - e[0])) / len(s.pos) < 2e-5
    xb, vb, _, _ = integrate.run_nve(x, -v, s.box, s.mass, s.dt_ps, 100, fn)
    d = xb - s.pos
    L = np.array(s.box.len)
    d -= L * np.rint(d / L)
    assert np.max(np.abs(d)) < 1e-9


def test_verlet_second_order_energy_error():
    s = mi.lj_argon()
    fn = integrate.lj_force_fn(s.box, s.lj)
    spread = []
    for dt, n in ((4e-3, 50), (2e-3, 100)):
        _, _, _, h = integrate.run_nve(s.pos, s.vel, s.box, s.mass, dt, n, fn)
        e = h[:, 1] + h[:, 2]
        spread.append(np.sqrt(np.mean((e - e.mean()) ** 2)))
    assert 3.0 < spread[0] / spread[1] < 5.0


def test_piston_and_top_wall_reflection():
    walls = {"axis": 2, "piston_z0": 0.0, "piston_v": 10.0, "top_z": 50.0}
    x = np.array([[0.0, 0.0, 0.005], [0.0, 0.0, 49.999], [0.0, 0.0, 25.0]])
    v = np.array([[0.0, 0.0, -3.0], [0.0, 0.0, 4.0], [0.0, 0.0, 1.0]])
    x2, v2 = integrate.apply_walls(x.copy(), v.copy(), 1e-3, walls)
    zp = 0.01
    assert abs(x2[0, 2] - (2 * zp - 0.005)) < 1e-15 and v2[0, 2] == 2 * 10.0 + 3.0
    x3, v3 = integrate.apply_walls(np.array([[0, 0, 50.002]]), np.array([[0, 0, 4.0]]), 0.0,
                                   walls)
    assert abs(x3[0, 2] - 49.998) < 1e-12 and v3[0, 2] == -4.0
    assert x2[2, 2] == 25.0 and v2[2, 2] == 1.0
