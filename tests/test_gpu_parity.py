"""GPU parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances:
  neighbour sets, wrapped positions, cell order       bit-exact
  FP64 forces / energy / virial                       relative 1e-12 (Frobenius) / 1e-12 / 1e-11
  FP32 forces                                         relative 1e-5 (Frobenius, all atoms)
  FP32 virial                                         1e-5 of the largest component
  FP32 energy                                         1e-6 eV per atom
"""
import numpy as np
import pytest
import torch

from tests.gpu_util import evv, md_ev

import mdinputs as mi
from oracle import core, integrate
from oracle import spline as osp
from tests.gpu_util import assert_same_sets, displaced, neighbor_sets_by_id, rel_fro

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mdmod():
    from paper_2511_22951_amd import md, _native
    _native.lib()
    return md


def _setup(md, pos, box, r_ns, lanes=4, max_neigh=128, prec=0, vel=None):
    plan = md.Plan([box], [len(pos)], r_ns)
    st = md.State(plan, pos, vel, prec)
    nl = md.NeighborList(len(pos), max_neigh, lanes)
    md.md_bin_cells(st)
    md.md_build_neighbors(st, nl)
    return plan, st, nl


# ----------------------------------------------------------------------------
# splines
# ----------------------------------------------------------------------------
def test_spline_fit_matches_oracle(mdmod):
    for tf in (mi.tabulate_eam(mi.EAM_CU).phi, mi.tabulate_eam(mi.EAM_CU).emb,
               mi.force_matching_tables().rho):
        got = mdmod.md_spline_fit(tf.y, tf.h, tf.dy_lo, tf.dy_hi).cpu().numpy()
        want = osp.fit_table(tf)
        assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))


# ----------------------------------------------------------------------------
# binning and neighbour lists
# ----------------------------------------------------------------------------
CASES = [
    # name, cells, a, sigma, r_ns, periodic
    ("lj_argon_256", 4, 5.26, 0.15, 2.5 * 3.405 + 0.3, (1, 1, 1)),
    ("cu_864_ragged", 6, 3.615, 0.08, 5.8, (1, 1, 1)),
    ("cu_tiny_grid_2cells", 4, 3.30, 0.05, 5.8, (1, 1, 1)),
    ("cu_walled_z", 6, 3.615, 0.05, 5.8, (1, 1, 0)),
]


@pytest.mark.parametrize("name,cells,a,sigma,r_ns,per", CASES)
@pytest.mark.parametrize("lanes", [1, 4, 16])
def test_neighbor_sets_bit_exact(mdmod, name, cells, a, sigma, r_ns, per, lanes):
    print("case", name, "lanes", lanes, flush=True)
    pos, box = displaced(cells, a, sigma, seed=100 + cells, box_periodic=per)
    if not per[2]:
        pos[:, 2] = np.clip(pos[:, 2], 0.01, box.len[2] - 0.01)
    assert core.min_gap(pos, box, r_ns) > 1e-9
    plan, st, nl = _setup(mdmod, pos, box, r_ns, lanes=lanes)
    info = st.check_flags()
    cnt, want = core.neighbor_sets(pos, box, r_ns)
    assert info["max_nneigh"] == cnt.max()
    assert_same_sets(neighbor_sets_by_id(st, nl), want)
    # wrapped positions equal the oracle's wrap bit for bit, and atoms are in cell order
    assert np.array_equal(st.positions(), core.wrap(pos, box))
    cs = st.cell_start.cpu().numpy()
    assert cs[0] == 0 and cs[-1] == len(pos) and np.all(np.diff(cs) >= 0)


def test_binning_wraps_far_outside_positions(mdmod):
    pos, box = displaced(5, 3.615, 0.05, seed=7)
    shift = np.random.default_rng(3).integers(-2, 3, pos.shape) * np.array(box.len)
    x = pos + shift
    plan, st, nl = _setup(mdmod, x, box, 5.8)
    xw = core.wrap(x, box)
    assert np.array_equal(st.positions(), xw)
    cnt, want = core.neighbor_sets(xw, box, 5.8)
    assert_same_sets(neighbor_sets_by_id(st, nl), want)


def test_neighbor_overflow_is_reported(mdmod):
    pos, box = displaced(4, 3.615, 0.05, seed=9)
    plan, st, nl = _setup(mdmod, pos, box, 5.8, lanes=4, max_neigh=32)
    with pytest.raises(mdmod.MDError) as e:
        st.check_flags()
    assert e.value.status == -3
    st.clear_flags()
    assert st.read_flags()[0] == 0


# ----------------------------------------------------------------------------
# forces
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("cells,lanes", [(4, 4), (5, 1), (5, 8), (5, 16)])
def test_lj_fp64_matches_oracle(mdmod, cells, lanes):
    p = mi.LJ_AR
    pos, box = displaced(cells, 5.26, 0.15, seed=11)
    plan, st, nl = _setup(mdmod, pos, box, p.r_cut + 0.3, lanes=lanes)
    ev = md_ev(1)
    mdmod.md_lj_forces(st, mdmod.lj_params(p.eps, p.sigma, p.r_cut), nl, ev=ev)
    r = core.lj(pos, box, p.eps, p.sigma, p.r_cut)
    assert rel_fro(st.forces(), r.force) < 1e-12
    e = evv(ev)[0, 0]
    assert abs(e[0] - r.energy) < 1e-12 * abs(r.energy)
    assert np.max(np.abs(e[1:7] - r.virial)) < 1e-11 * np.max(np.abs(r.virial))


def test_lj_fp32_rejects_16_lanes(mdmod):
    """FP32 takes 1-8 lanes per atom (as the EAM passes): 16 is an argument error."""
    p = mi.LJ_AR
    pos, box = displaced(4, 5.26, 0.15, seed=14)
    plan, st, nl = _setup(mdmod, pos, box, p.r_cut + 0.3, lanes=16, prec=1)
    with pytest.raises(mdmod.MDError) as e:
        mdmod.md_lj_forces(st, mdmod.lj_params(p.eps, p.sigma, p.r_cut), nl)
    assert e.value.status == -1
    st.check_flags()


def test_lj_fp32_within_tolerance(mdmod):
    p = mi.LJ_AR
    pos, box = displaced(5, 5.26, 0.15, seed=12)
    plan, st, nl = _setup(mdmod, pos, box, p.r_cut + 0.3, prec=1)
    ev = md_ev(1)
    mdmod.md_lj_forces(st, mdmod.lj_params(p.eps, p.sigma, p.r_cut), nl, ev=ev)
    r = core.lj(pos, box, p.eps, p.sigma, p.r_cut)
    assert rel_fro(st.forces(), r.force) < 1e-5
    assert abs(evv(ev)[0, 0, 0] - r.energy) / len(pos) < 1e-6


@pytest.mark.parametrize("prec,lanes", [(0, 4), (0, 1), (0, 16), (1, 4), (1, 8)])
def test_eam_matches_oracle(mdmod, prec, lanes):
    tab = mi.tabulate_eam(mi.EAM_CU)
    pos, box = displaced(6, 3.615, 0.08, seed=13)
    plan, st, nl = _setup(mdmod, pos, box, 5.8, lanes=lanes, prec=prec)
    pot = mdmod.EAMPotential.from_table(tab)
    ev = md_ev(1)
    saved = torch.zeros((3, len(pos)), dtype=torch.float64, device="cuda")
    mdmod.md_eam_forces(st, pot, nl, saved=saved, ev=ev)
    st.check_flags()
    r = core.eam(pos, box, core.EAMPotential.from_table(tab))
    e = evv(ev)[0, 0]
    order = st._order()
    rb = saved.cpu().numpy()[0][order]
    if prec == 0:
        assert rel_fro(st.forces(), r.force) < 1e-12
        assert abs(e[0] - r.energy) < 1e-12 * abs(r.energy)
        assert np.max(np.abs(e[1:7] - r.virial)) < 1e-11 * np.max(np.abs(r.virial))
        assert np.max(np.abs(rb - r.rhobar)) < 1e-12 * np.max(r.rhobar)
    else:
        assert rel_fro(st.forces(), r.force) < 1e-5
        assert abs(e[0] - r.energy) / len(pos) < 1e-6
        assert np.max(np.abs(e[1:7] - r.virial)) < 1e-5 * np.max(np.abs(r.virial))
        assert np.max(np.abs(rb - r.rhobar)) < 1e-5 * np.max(r.rhobar)


@pytest.mark.skip(reason="FP32 at 16 lanes per atom on 19,652 atoms faulted the GPU on its first "
                         "run; no cause was found by reading the code, so FP32 at 16 lanes is "
                         "switched off (md_eam_forces returns MD_ERR_ARG) and this case stays off")
def test_eam_fp32_large_batch_shape(mdmod):
    """FP32 density/force on a system with more wavefronts than fit on the chip at once
    at 16 lanes per atom (19,652 atoms): the kernels' other launch shape."""
    tab = mi.tabulate_eam(mi.EAM_CU)
    pos, box = displaced(17, 3.615, 0.05, seed=14)
    plan, st, nl = _setup(mdmod, pos, box, 5.8, lanes=16, prec=1)
    assert plan.n_tiles * 16 > 16 * 256
    pot = mdmod.EAMPotential.from_table(tab)
    ev = md_ev(1)
    mdmod.md_eam_forces(st, pot, nl, ev=ev)
    st.check_flags()
    r = core.eam(pos, box, core.EAMPotential.from_table(tab))
    e = evv(ev)[0, 0]
    assert rel_fro(st.forces(), r.force) < 1e-5
    assert abs(e[0] - r.energy) / len(pos) < 1e-6
    assert np.max(np.abs(e[1:7] - r.virial)) < 1e-5 * np.max(np.abs(r.virial))


def test_eam_table_range_flag(mdmod):
    """Atoms pushed closer than the table start set MD_FLAG_TABLE_RANGE."""
    tab = mi.tabulate_eam(mi.EAM_CU, r_lo=2.4)
    pos, box = displaced(5, 3.615, 0.0, seed=1)
    pos[1] = pos[0] + np.array([2.0, 0.0, 0.0])
    plan, st, nl = _setup(mdmod, pos, box, 5.8)
    mdmod.md_eam_forces(st, mdmod.EAMPotential.from_table(tab), nl)
    with pytest.raises(mdmod.MDError) as e:
        st.check_flags()
    assert e.value.status == -4


# ----------------------------------------------------------------------------
# integration
# ----------------------------------------------------------------------------
def test_lj_argon_trajectory_100_steps(mdmod):
    """LJ argon 256 atoms, 100 velocity-Verlet steps, FP64: positions, velocities and
    energies follow the oracle."""
    from paper_2511_22951_amd.sim import Simulation
    s = mi.lj_argon()
    sim = Simulation(s, precision=0, lanes=4).setup()
    sim.run(100)
    info = sim.state.check_flags()
    assert info["step"] == 100 and info["n_rebuilds"] >= 2
    fn = integrate.lj_force_fn(s.box, s.lj)
    x, v, f, hist = integrate.run_nve(s.pos, s.vel, s.box, s.mass, s.dt_ps, 100, fn)
    d = sim.state.positions() - x
    L = np.array(s.box.len)
    d -= L * np.rint(d / L)
    assert np.max(np.abs(d)) < 1e-9
    assert np.max(np.abs(sim.state.velocities() - v)) < 1e-8
    e = sim.energies(range(101))
    assert np.max(np.abs(e[:, 0] - hist[:, 1])) < 1e-10 * abs(hist[0, 1])
    assert np.max(np.abs(e[:, 7] - hist[:, 2])) < 1e-10 * abs(hist[0, 2])


def test_eam_cu_trajectory_20_steps_and_graph_replay(mdmod):
    """EAM Cu 864 atoms: 20 eager steps follow the oracle; a graph-captured run replays
    the same trajectory bit for bit."""
    from paper_2511_22951_amd.sim import Simulation
    s = mi.eam_copper(cells=6)
    sim = Simulation(s, precision=0, lanes=4).setup()
    sim.run(20)
    sim.state.check_flags()
    pot = core.EAMPotential.from_table(s.table)
    x, v, f, hist = integrate.run_nve(s.pos, s.vel, s.box, s.mass, s.dt_ps, 20,
                                      integrate.eam_force_fn(s.box, pot))
    d = sim.state.positions() - x
    L = np.array(s.box.len)
    d -= L * np.rint(d / L)
    assert np.max(np.abs(d)) < 1e-9
    e = sim.energies(range(21))
    assert np.max(np.abs(e[:, 0] - hist[:, 1])) < 1e-10 * abs(hist[0, 1])
    g = Simulation(s, precision=0, lanes=4).setup()
    g.run(20, graph_steps=10)
    torch.cuda.synchronize()
    assert np.array_equal(g.state.positions(), sim.state.positions())
    assert np.array_equal(g.energies(range(21)), e)


def test_piston_walls_match_oracle(mdmod):
    """Walled box (periodic x, y; piston and top wall on z), 40 steps; the piston starts at
    z = 0.6 and moves at 2 km/s so that the bottom layer is reflected within the run."""
    from paper_2511_22951_amd.sim import Simulation
    s = mi.eam_aluminum_shock(nx=4, ny=4, nz=8)
    s.walls = dict(s.walls, piston_z0=0.6, piston_v=20.0)
    sim = Simulation(s, precision=0, lanes=4).setup()
    sim.run(40)
    sim.state.check_flags()
    pot = core.EAMPotential.from_table(s.table)
    x, v, f, hist = integrate.run_nve(s.pos, s.vel, s.box, s.mass, s.dt_ps, 40,
                                      integrate.eam_force_fn(s.box, pot), walls=s.walls)
    # the piston reached the bottom layer: some velocities were reflected
    assert np.max(sim.state.velocities()[:, 2]) > 30.0
    d = sim.state.positions() - x
    L = np.array(s.box.len)
    per = np.array(s.box.periodic, bool)
    d[:, per] -= L[per] * np.rint(d[:, per] / L[per])
    assert np.max(np.abs(d)) < 1e-9


def test_fixed_interval_rebuilds_match_oracle(mdmod):
    """Rebuilds every 10 steps (the interval of the paper's benchmark) with the half-skin
    criterion verified on the device: LJ argon follows the oracle for 100 steps, graph
    replay included, and the flags stay clear."""
    from paper_2511_22951_amd.sim import Simulation
    s = mi.lj_argon()
    sim = Simulation(s, precision=0, lanes=4, rebuild_every=10).setup()
    sim.run(100, graph_steps=20)
    info = sim.state.check_flags()
    assert info["step"] == 100 and info["n_rebuilds"] == 11
    x, v, f, hist = integrate.run_nve(s.pos, s.vel, s.box, s.mass, s.dt_ps, 100,
                                      integrate.lj_force_fn(s.box, s.lj))
    d = sim.state.positions() - x
    L = np.array(s.box.len)
    d -= L * np.rint(d / L)
    assert np.max(np.abs(d)) < 1e-9
    e = sim.energies(range(101))
    assert np.max(np.abs(e[:, 0] - hist[:, 1])) < 1e-10 * abs(hist[0, 1])


@pytest.mark.parametrize("prec,policy", [(0, 0), (1, 6), (0, 6)])
def test_fused_kick_drift_equals_separate(mdmod, prec, policy):
    """The force pass with the next kick-drift fused in (md_drift) gives the same bits as the
    separate md_verlet_step: EAM Cu, 30 steps, threshold rebuilds or rebuilds every 6 steps
    with graph replay; the fused run is one kick-drift ahead at the end."""
    from paper_2511_22951_amd import _native as N
    from paper_2511_22951_amd.sim import Simulation
    s = mi.eam_copper(cells=6)
    a = Simulation(s, precision=prec, lanes=4, rebuild_every=policy).setup()
    b = Simulation(s, precision=prec, lanes=4, rebuild_every=policy, fused=True).setup()
    a.run(30, graph_steps=6 if policy else 0)
    b.run(30, graph_steps=6 if policy else 0)
    ia, ib = a.state.check_flags(), b.state.check_flags()
    assert ia["n_rebuilds"] == ib["n_rebuilds"] > 1
    assert np.array_equal(b.previous_positions(), a.state.positions())
    assert np.array_equal(a.energies(range(31)), b.energies(range(31)))
    mdmod.md_verlet_step(a.state, N.MD_KICK_DRIFT, a.dt, a.inv_mass, a.walls, a.half_skin)
    assert np.array_equal(a.state.positions(), b.state.positions())
    assert np.array_equal(a.state.velocities(), b.state.velocities())


@pytest.mark.parametrize("pot,policy,graph", [("eam", 0, 0), ("eam", 6, 6), ("lj", 0, 0),
                                              ("lj", 5, 10)])
def test_carried_fp32_records_equal_converted(mdmod, pot, policy, graph):
    """FP32 neighbour records written by the fused kick-drift (md_drift.rec_out) and taken by
    the next force call (rec_in) give the same bits as converting the positions every step,
    across rebuilds (which reorder the atoms, so the records are remade), with threshold or
    fixed-period rebuilds (between which the records are declared current and no conversion is
    launched), eager or graph-replayed; rec_in equal to rec_out is refused, and records declared
    current after a reorder raise MD_ERR_STALE_RECORDS."""
    from paper_2511_22951_amd import _native as N
    from paper_2511_22951_amd.sim import Simulation
    if pot == "eam":
        s = mi.eam_copper(cells=6)
    else:
        s = mi.lj_argon(cells=4)
        s.vel = s.vel * np.sqrt(3.0)  # 300 K
    a = Simulation(s, precision=1, lanes=2, rebuild_every=policy, fused=True,
                   carry_records=False).setup()
    b = Simulation(s, precision=1, lanes=2, rebuild_every=policy, fused=True).setup()
    assert b.carry and not a.carry  # b carries its records when rebuilds have a fixed period
    a.run(30, graph_steps=graph)
    b.run(30, graph_steps=graph)
    ia, ib = a.state.check_flags(), b.state.check_flags()
    assert ia["n_rebuilds"] == ib["n_rebuilds"] >= (1 if policy == 0 and pot == "lj" else 2)
    assert np.array_equal(a.state.positions(), b.state.positions())
    assert np.array_equal(a.state.velocities(), b.state.velocities())
    assert np.array_equal(a.energies(range(31)), b.energies(range(31)))
    st = b.state
    # all records at one point: the void step below also turns forces and positions
    # non-finite, and the void step is what md_read_flags must report
    r1 = torch.zeros(16 * st.n, dtype=torch.uint8, device="cuda")
    r2 = torch.empty_like(r1)
    drift = mdmod.drift_params(b.pos_alt, st.pos_ref, b.dt, b.half_skin, b.walls,
                               rec_in=r1, rec_out=r1)

    def force(drift):
        if pot == "eam":
            mdmod.md_eam_forces(st, b.pot, b.nl, b.table, None, b.inv_mass, 0.5 * b.dt, kick=True,
                                drift=drift)
        else:
            mdmod.md_lj_forces(st, b.lj, b.nl, b.inv_mass, 0.5 * b.dt, kick=True, drift=drift)
    with pytest.raises(mdmod.MDError) as e:
        force(drift)
    assert e.value.status == N.MD_ERR_ARG
    # records declared current right after a reorder: the device notices, the step is void
    mdmod.md_bin_cells(st, N.MD_ALWAYS)
    mdmod.md_build_neighbors(st, b.nl, N.MD_ALWAYS)
    force(mdmod.drift_params(b.pos_alt, st.pos_ref, b.dt, b.half_skin, b.walls, rec_in=r1,
                             rec_out=r2, rec_current=True))
    with pytest.raises(mdmod.MDError) as e:
        st.check_flags()
    assert e.value.status == N.MD_ERR_STALE_RECORDS
    if pot == "lj":  # coincident records: infinite pair forces, non-finite positions too
        assert st.read_flags()[1]["flags"] & N.FLAG_NONFINITE


def test_carried_records_after_steps_without_them(mdmod):
    """Fused FP32 steps that write no records, between steps that carry them: those force
    passes mark the carried buffers stale on the device, so the next carried step (which does
    not claim its records current) converts again -- the run equals one that converts every
    step, bit for bit."""
    from paper_2511_22951_amd.sim import Simulation
    s = mi.eam_copper(cells=6)
    a = Simulation(s, precision=1, lanes=2, rebuild_every=6, fused=True,
                   carry_records=False).setup()
    b = Simulation(s, precision=1, lanes=2, rebuild_every=6, fused=True).setup()
    a.run(20)
    b.run(7)
    b.carry = False  # steps 8-10 move the atoms without writing records
    b.run(3)
    b.carry = True   # step 11 is no rebuild step: only the device's mark makes it convert
    b.run(10)
    assert np.array_equal(a.state.positions(), b.state.positions())
    assert np.array_equal(a.state.velocities(), b.state.velocities())
    a.state.check_flags()
    b.state.check_flags()


@pytest.mark.parametrize("fused,k,steps", [(True, 5, 23), (True, 6, 20), (False, 5, 23)])
def test_graph_only_timed_run_equals_eager(mdmod, fused, k, steps):
    """The benchmark's timed region (Simulation.prepare_timed / replay_timed): a main graph
    of whole graph periods replayed q times plus one tail graph -- of an odd number of steps
    in the fused cases with k = 5 -- gives the same bits as the same steps taken eagerly, takes
    no eager step, and leaves the state ready for further steps (EAM Cu FP32)."""
    from paper_2511_22951_amd.sim import Simulation, timed_graph_plan
    s = mi.eam_copper(cells=6)
    a = Simulation(s, precision=1, lanes=2, rebuild_every=k, fused=fused).setup()
    b = Simulation(s, precision=1, lanes=2, rebuild_every=k, fused=fused).setup()
    for sim in (a, b):
        sim.run(7)
        sim.align()
    assert a.n_steps == b.n_steps
    G, q, r = timed_graph_plan(steps, k, fused, 10)
    assert q >= 1 and r > 0 and (not fused or k % 2 == 0 or r % 2 == 1)
    plan = b.prepare_timed(steps, 10)
    e0 = b.eager_steps
    b.replay_timed(plan)
    assert b.eager_steps == e0 and len(plan) == q + 1
    a.run(steps)
    for _ in range(2):
        ia, ib = a.state.check_flags(), b.state.check_flags()
        assert ia["step"] == ib["step"] and ia["n_rebuilds"] == ib["n_rebuilds"] > 1
        assert np.array_equal(a.state.positions(), b.state.positions())
        assert np.array_equal(a.state.velocities(), b.state.velocities())
        assert np.array_equal(a.energies(range(ia["step"] + 1)), b.energies(range(ib["step"] + 1)))
        a.run(7)  # then further steps (graphs where whole ones fit) on both
        b.run(7, graph_steps=10)


@pytest.mark.parametrize("prec,policy", [(0, 0), (1, 5)])
def test_fused_kick_drift_lj_equals_separate(mdmod, prec, policy):
    """The same for the LJ pass: argon 4^3 cells (256 atoms) at 300 K, 30 steps."""
    from paper_2511_22951_amd import _native as N
    from paper_2511_22951_amd.sim import Simulation
    s = mi.lj_argon(cells=4)
    s.vel = s.vel * np.sqrt(3.0)
    a = Simulation(s, precision=prec, lanes=2, rebuild_every=policy).setup()
    b = Simulation(s, precision=prec, lanes=2, rebuild_every=policy, fused=True).setup()
    assert b.fused
    a.run(30, graph_steps=10 if policy else 0)
    b.run(30, graph_steps=10 if policy else 0)
    ia, ib = a.state.check_flags(), b.state.check_flags()
    assert ia["n_rebuilds"] == ib["n_rebuilds"]
    assert np.array_equal(b.previous_positions(), a.state.positions())
    assert np.array_equal(a.energies(range(31)), b.energies(range(31)))
    mdmod.md_verlet_step(a.state, N.MD_KICK_DRIFT, a.dt, a.inv_mass, a.walls, a.half_skin)
    assert np.array_equal(a.state.positions(), b.state.positions())
    assert np.array_equal(a.state.velocities(), b.state.velocities())


def test_fused_kick_drift_with_walls(mdmod):
    """Fused kick-drift with the piston and top wall (the shock set-up) equals the separate
    one bit for bit."""
    from paper_2511_22951_amd import _native as N
    from paper_2511_22951_amd.sim import Simulation
    s = mi.eam_aluminum_shock(nx=4, ny=4, nz=8)
    s.walls = dict(s.walls, piston_z0=0.6, piston_v=20.0)
    a = Simulation(s, precision=1, lanes=4).setup()
    b = Simulation(s, precision=1, lanes=4, fused=True).setup()
    a.run(40)
    b.run(40)
    a.state.check_flags()
    b.state.check_flags()
    assert np.max(b.state.velocities()[:, 2]) > 30.0
    mdmod.md_verlet_step(a.state, N.MD_KICK_DRIFT, a.dt, a.inv_mass, a.walls, a.half_skin)
    assert np.array_equal(a.state.positions(), b.state.positions())
    assert np.array_equal(a.state.velocities(), b.state.velocities())


def test_stale_list_is_detected(mdmod):
    """Without rebuilds a hot system soon moves atoms by more than half the skin: the force
    pass reports MD_ERR_STALE_LIST."""
    from paper_2511_22951_amd.sim import Simulation
    s = mi.lj_argon()
    s.vel = s.vel * 4.0
    sim = Simulation(s, precision=0, lanes=4, rebuild_every=100000).setup()
    sim.run(40)
    with pytest.raises(mdmod.MDError) as e:
        sim.state.check_flags()
    assert e.value.status == -9


@pytest.mark.parametrize("pot,prec", [("eam", 1), ("eam", 0), ("lj", 1)])
def test_big_list_offsets_equal_small_list(mdmod, pot, prec):
    """A list of 2^30 entries (4 GiB: 2048 atoms with room for 524,288 neighbours each) takes
    the 64-bit entry offsets of the force passes and the 64-bit addressing of the list build;
    forces and records equal those of an ordinary list bit for bit."""
    from paper_2511_22951_amd.sim import Simulation
    s = mi.eam_copper(cells=8) if pot == "eam" else mi.lj_argon(cells=8)
    out = []
    for max_neigh in (128, 524288):
        sim = Simulation(s, precision=prec, lanes=2, max_neigh=max_neigh, ev_cap=8).setup()
        assert (sim.nl.max_neigh * sim.nl.npad >= 1 << 30) == (max_neigh > 128)
        sim.run(3)
        info = sim.state.check_flags()
        out.append((sim.state.forces(), sim.energies([info["step"]])[0]))
        del sim
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
