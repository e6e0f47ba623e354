"""GPU parity at the full benchmark sizes, in the launch configuration bench.py times
(2 lanes per atom, the next kick-drift fused into the force pass, HIP-graph replay):
sampled atoms against the oracle's per-atom routines, plus properties that hold at any
size.

  neighbour sets of sampled atoms (after a rebuild at the evolved positions)   bit-exact
  forces of sampled atoms, FP64 / FP32-mixed (norm over the sample)           1e-11 / 1e-5
  net force over all atoms, relative to the sum of |F_i|, FP64 / FP32          1e-10 / 1e-5
  force-matching adjoint (1024 snapshots), cotangent on 16 sampled snapshots   1e-10
"""
import numpy as np
import pytest

import mdinputs as mi
from oracle import core

pytestmark = pytest.mark.gpu


def _lists_of(nl, cur):
    """Neighbour lists (current order) of the atoms at current-order positions `cur`."""
    from paper_2511_22951_amd import _native as N
    nn = nl.nneigh.cpu().numpy() & (N.MD_NN_IMG - 1)
    raw = nl.neigh.cpu().numpy().reshape(nl.max_neigh // nl.lanes, nl.npad, nl.lanes)
    out = []
    for i in cur:
        k = np.arange(nn[i])
        out.append(raw[k // nl.lanes, i, k % nl.lanes])
    return out


def _check_sets(sim, s, sample):
    sim.rebuild()
    ids = sim.state.id.cpu().numpy()
    cur_of = np.empty_like(ids)
    cur_of[ids] = np.arange(len(ids))
    x = sim.state.positions()
    cnt, want = core.neighbor_sets_sampled(x, s.box, sim.r_ns, sample)
    got = _lists_of(sim.nl, cur_of[sample])
    for a, g, w in zip(sample, got, want):
        assert np.array_equal(np.sort(ids[g]), np.sort(w)), a


def _check_forces(sim, s, sample, tol, tol_net):
    x = sim.previous_positions()  # the positions the last force pass saw
    f = sim.state.forces()
    r = core.eam_sampled(x, s.box, core.EAMPotential.from_table(s.table), sample)
    assert r.out_of_range == 0
    err = np.linalg.norm(f[sample] - r.force) / np.linalg.norm(r.force)
    assert err < tol, err
    net = np.abs(f.sum(axis=0)).max() / np.abs(f).sum()
    assert net < tol_net, net


@pytest.mark.parametrize("prec", [1, 0])
def test_cu131k_bench_configuration(prec):
    """EAM Cu fcc 32^3 (131,072 atoms): 360 steps, rebuilds every 12 steps, 18-step graphs."""
    from paper_2511_22951_amd.sim import Simulation
    s = mi.eam_copper(cells=32)
    sim = Simulation(s, precision=prec, lanes=2, ev_cap=64, rebuild_every=12, fused=True).setup()
    n0 = sim.state.check_flags()["n_rebuilds"]
    sim.run(360, graph_steps=18)
    assert sim.state.check_flags()["n_rebuilds"] - n0 == 30  # steps 12, 24, .., 360
    rng = np.random.default_rng(2024 + prec)
    sample = rng.choice(s.pos.shape[0], 256, replace=False)
    _check_forces(sim, s, sample, 1e-5 if prec else 1e-11, 1e-5 if prec else 1e-10)
    _check_sets(sim, s, sample)


def test_al640k_shock_configuration():
    """EAM Al shock (640,000 atoms, piston, top wall), FP32-mixed, threshold rebuilds,
    40 steps with 20-step graphs."""
    from paper_2511_22951_amd import _native as N
    from paper_2511_22951_amd.sim import Simulation
    s = mi.eam_aluminum_shock()
    sim = Simulation(s, precision=N.MD_FP32, lanes=2, max_neigh=160, ev_cap=64,
                     rebuild_every=0, fused=True).setup()
    sim.run(40, graph_steps=20)
    sim.state.check_flags()
    rng = np.random.default_rng(2025)
    # atoms near the piston (first 2 %) and elsewhere
    n = s.pos.shape[0]
    order = np.argsort(s.pos[:, 2])
    sample = np.concatenate([order[rng.choice(n // 50, 64, replace=False)],
                             rng.choice(n, 128, replace=False)])
    _check_forces(sim, s, sample, 1e-5, 1e-4)
    _check_sets(sim, s, sample)


def test_lj13m_paper_configuration():
    """The LJ test of Sec. 1.7 at its size: 12,967,168 Ar atoms, lists rebuilt every 10
    steps (the list holds over 2^30 entries, so the passes take 64-bit entry offsets), the
    next kick-drift fused into the LJ pass; FP64 and FP32-mixed, 20 steps with 10-step
    graphs."""
    from paper_2511_22951_amd import _native as N
    from paper_2511_22951_amd.sim import Simulation
    s = mi.lj_argon_benchmark()
    n = s.pos.shape[0]
    sample = np.random.default_rng(2026).choice(n, 128, replace=False)
    for prec, tol, tol_net in ((N.MD_FP64, 1e-11, 1e-10), (N.MD_FP32, 1e-5, 1e-5)):
        sim = Simulation(s, precision=prec, lanes=2, max_neigh=112, ev_cap=64,
                         rebuild_every=10, fused=True).setup()
        assert sim.nl.max_neigh * sim.nl.npad >= 1 << 30
        n0 = sim.state.check_flags()["n_rebuilds"]
        sim.run(20, graph_steps=10)
        assert sim.state.check_flags()["n_rebuilds"] - n0 == 2
        x = sim.previous_positions()  # the positions the last force pass saw
        f = sim.state.forces()
        lj = s.lj
        r = core.lj_sampled(x, s.box, lj.eps, lj.sigma, lj.r_cut, sample)
        err = np.linalg.norm(f[sample] - r.force) / np.linalg.norm(r.force)
        assert err < tol, (prec, err)
        net = np.abs(f.sum(axis=0)).max() / np.abs(f).sum()
        assert net < tol_net, (prec, net)
        if prec == N.MD_FP64:
            _check_sets(sim, s, sample)
        del sim


def test_force_matching_1024_snapshots_vjp_sampled():
    """The force-matching batch at its size (1024 Cu snapshots x 500 atoms, 192 spline
    coefficients, FP64, 4 lanes per atom as bench.py runs it): the adjoint of a cotangent that
    is nonzero on 16 sampled snapshots only equals the oracle's chain-rule VJP over those
    snapshots alone (the VJP is linear in the cotangent and snapshots do not interact), to
    1e-10 of its largest entry."""
    from paper_2511_22951_amd import md
    from oracle import adjoint as oadj
    from tests.test_gpu_batch_adjoint import _fm_problem
    snaps, osnaps, grids, c_or, pot, batch = _fm_problem(md, n_snap=1024)
    assert sum(len(s.pos) for s in snaps) == 512000
    pick = np.sort(np.random.default_rng(2027).choice(len(snaps), 16, replace=False))
    G = [np.zeros((len(s.pos), 3)) for s in snaps]
    for k in pick:
        G[k] = mi.random_cotangent(len(snaps[k].pos), seed=100 + int(k))
    want = np.concatenate(oadj.vjp([osnaps[k] for k in pick], c_or, grids, [G[k] for k in pick]))
    batch.forces(pot, saved=True)
    got = batch.backward(pot, batch.to_current_order(np.concatenate(G))).cpu().numpy()
    batch.state.check_flags()
    assert np.max(np.abs(got - want)) < 1e-10 * np.max(np.abs(want))
