"""Pins of the oracle's EAM (tabulated splines and analytic forms)."""
import json
import os

import numpy as np
import pytest

import mdinputs as mi
from oracle import core
from tests import lattice_sums as ls

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.json")


@pytest.fixture(scope="module")
def cu_spline():
    return core.EAMPotential.from_table(mi.tabulate_eam(mi.EAM_CU))


def _disp(pos, box, sigma, seed, r_probe=None, gap=1e-4):
    """Seeded displacement; with r_probe, the first seed from `seed` on whose pairs all stay
    `gap` away from r_probe (so that a finite-difference step never crosses the cutoff)."""
    for s in range(seed, seed + 100):
        rng = np.random.default_rng(s)
        x = core.wrap(pos + rng.normal(0, sigma, pos.shape), box)
        if r_probe is None or core.min_gap(x, box, r_probe) > gap:
            return x
    raise RuntimeError("no configuration clear of the cutoff")


@pytest.mark.parametrize("a", [3.30, 3.55, 3.615, 3.68, 4.20])
def test_eam_lattice_energy_closed_form(a, cu_spline):
    p = mi.EAM_CU
    n = 4 if a < 3.5 else 5
    pos, box = mi.fcc_lattice(n, n, n, a)
    e_want, rb_want = ls.eam_per_atom(a, p)
    ra = core.eam(pos, box, core.EAMPotential.analytic(p))
    assert abs(ra.energy / len(pos) - e_want) < 1e-12
    assert np.max(np.abs(ra.rhobar - rb_want)) < 1e-11
    rs = core.eam(pos, box, cu_spline)
    assert abs(rs.energy / len(pos) - e_want) < 1e-9 and rs.out_of_range == 0
    assert np.max(np.abs(rs.rhobar - rb_want)) < 1e-9
    assert np.max(np.abs(rs.force)) < 1e-11


def test_eam_cu_reference_values():
    """Cu at a = 3.615: E/atom = -2.363525746 eV, rhobar = 12.82053654 (closed form)."""
    e, rb = ls.eam_per_atom(3.615, mi.EAM_CU)
    assert abs(e + 2.363525746) < 1e-9 and abs(rb - 12.82053654) < 1e-8


@pytest.mark.parametrize("lattice", ["Zhakhovsky", "Mishin", "WKG"])
def test_eam_al_table1_lattices(lattice):
    """Al toy EAM at the Table 1 lattice parameters (Sec. 3.3), closed form vs oracle."""
    a = json.load(open(GOLDEN))["aluminum_lattice_parameters"][lattice] * 10.0
    pot = core.EAMPotential.from_table(mi.tabulate_eam(mi.EAM_AL))
    pos, box = mi.fcc_lattice(4, 4, 4, a)
    r = core.eam(pos, box, pot)
    e_want, rb_want = ls.eam_per_atom(a, mi.EAM_AL)
    assert abs(r.energy / len(pos) - e_want) < 1e-9
    assert np.max(np.abs(r.rhobar - rb_want)) < 1e-9


def test_eam_virial_equals_minus_dE_dV_on_lattice(cu_spline):
    """tr W / (3V) = -dE/dV with V = N a^3 / 4 (closed-form derivative of the shell sum)."""
    a = 3.615
    pos, box = mi.fcc_lattice(5, 5, 5, a)
    r = core.eam(pos, box, core.EAMPotential.analytic(mi.EAM_CU))
    n = len(pos)
    dEdV = n * ls.eam_dE_da(a, mi.EAM_CU) / (3 * n * a * a / 4)
    V = n * a ** 3 / 4
    assert abs((r.virial[:3].sum()) / (3 * V) + dEdV) < 1e-12


def _E(x, box, pot):
    return core.eam(x, box, pot).energy


def test_eam_fd_forces_newton_and_virial(cu_spline):
    pos, box = mi.fcc_lattice(4, 4, 4, 3.615)
    x = _disp(pos, box, 0.1, 11, r_probe=mi.EAM_CU.r_cut)
    r = core.eam(x, box, cu_spline)
    assert r.out_of_range == 0
    assert np.max(np.abs(r.force.sum(axis=0))) < 1e-12
    h = 1e-5
    for i in (0, 31, 255):
        for a in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, a] += h
            xm[i, a] -= h
            fd = -(_E(xp, box, cu_spline) - _E(xm, box, cu_spline)) / (2 * h)
            assert abs(fd - r.force[i, a]) <= 1e-7 * max(1.0, np.abs(r.force).max())
    hs = 1e-6
    for a in range(3):
        es = []
        for s in (hs, -hs):
            sc = np.ones(3)
            sc[a] += s
            b2 = mi.Box(box.lo, tuple(np.array(box.len) * sc), box.periodic)
            es.append(_E(x * sc, b2, cu_spline))
        assert abs(-(es[0] - es[1]) / (2 * hs) - r.virial[a]) < 1e-6 * abs(r.virial[a]) + 1e-8


def test_eam_invariances(cu_spline):
    pos, box = mi.fcc_lattice(4, 4, 4, 3.615)
    x = _disp(pos, box, 0.1, 12)
    r = core.eam(x, box, cu_spline)
    xt = core.wrap(x + np.array([3.3, 7.7, -5.1]), box)
    rt = core.eam(xt, box, cu_spline)
    assert np.max(np.abs(rt.force - r.force)) < 1e-11 and abs(rt.energy - r.energy) < 1e-10
    perm = np.random.default_rng(2).permutation(len(x))
    rp = core.eam(x[perm], box, cu_spline)
    assert np.max(np.abs(rp.force - r.force[perm])) < 1e-12
    assert np.max(np.abs(rp.rhobar - r.rhobar[perm])) < 1e-12
    rc = core.eam(x[:, [2, 0, 1]], box, cu_spline)
    assert np.max(np.abs(rc.force - r.force[:, [2, 0, 1]])) < 1e-12


def test_eam_spline_vs_analytic_forces(cu_spline):
    pos, box = mi.fcc_lattice(4, 4, 4, 3.615)
    x = _disp(pos, box, 0.1, 13)
    rs = core.eam(x, box, cu_spline)
    ra = core.eam(x, box, core.EAMPotential.analytic(mi.EAM_CU))
    assert np.linalg.norm(rs.force - ra.force) / np.linalg.norm(ra.force) < 1e-8
    assert abs(rs.energy - ra.energy) / abs(ra.energy) < 1e-10


def test_eam_sampled_equals_full(cu_spline):
    pos, box = mi.fcc_lattice(4, 4, 4, 3.615)
    x = _disp(pos, box, 0.1, 14)
    r = core.eam(x, box, cu_spline)
    idx = np.array([0, 5, 77, 130, 255])
    s = core.eam_sampled(x, box, cu_spline, idx)
    assert np.max(np.abs(s.force - r.force[idx])) < 1e-12
    assert np.max(np.abs(s.rhobar - r.rhobar[idx])) < 1e-12
    assert np.max(np.abs(s.e_atom - r.e_atom[idx])) < 1e-12
    sl = core.lj_sampled(x, box, 0.01, 2.3, 5.0, idx)
    rl = core.lj(x, box, 0.01, 2.3, 5.0)
    assert np.max(np.abs(sl.force - rl.force[idx])) < 1e-13


def test_eam_reduces_to_pair_potential_when_embedding_linear():
    """With F(rhobar) = k rhobar the EAM is a pair potential phi + 2 k rho: check the force
    against a numpy pair sum written from eq. 1.6."""
    p = mi.EAM_CU
    tab = mi.tabulate_eam(p)
    k = -0.3
    q = tab.emb.x_lo + tab.emb.h * np.arange(tab.emb.K)
    lin = mi.TabulatedFunction(tab.emb.x_lo, tab.emb.x_hi, k * q, k, k)
    pot = core.EAMPotential(core.SplineFunc.from_table(tab.phi), core.SplineFunc.from_table(tab.rho),
                            core.SplineFunc.from_table(lin), p.r_cut)
    pos, box = mi.fcc_lattice(3, 3, 4, 3.7)
    x = _disp(pos, box, 0.1, 15)
    r = core.eam(x, box, pot)
    L = np.array(box.len)
    d = x[:, None, :] - x[None, :, :]
    d -= L * np.rint(d / L)
    rr = np.sqrt((d ** 2).sum(-1))
    np.fill_diagonal(rr, np.inf)
    m = rr < p.r_cut
    dV = np.where(m, -p.A * p.alpha / p.r0 * np.exp(-p.alpha * (rr / p.r0 - 1))
                  + 2 * k * (-p.beta / p.r0) * np.exp(-p.beta * (rr / p.r0 - 1)), 0.0)
    f = -(dV[..., None] * d / np.where(m, rr, 1.0)[..., None]).sum(1)
    assert np.max(np.abs(f - r.force)) < 1e-8
