"""GPU parity of the batched path (many uneven boxes in one launch) and of the EAM
adjoint (md_eam_backward) with the oracle.

Tolerances: per-box FP64 energies 1e-12 relative to the oracle and 1e-9 eV/atom to the
closed-form lattice sum (spline interpolation error); FP32 energies 1e-6 eV/atom;
perfect-lattice forces |F| < 1e-10 eV/A (FP64); adjoint vs the oracle's chain-rule
gradient 1e-10 relative (FP64 throughout).
"""
import numpy as np
import pytest
import torch

from tests.gpu_util import evv, md_ev

import mdinputs as mi
from oracle import adjoint as oadj
from oracle import core
from oracle import spline as osp
from tests import lattice_sums as ls
from tests.gpu_util import assert_same_sets, neighbor_sets_by_id

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def md():
    from paper_2511_22951_amd import md as m
    m.N.lib()
    return m


def _batch(md, reps, prec=0, lanes=4):
    boxes = [r.box for r in reps]
    counts = [len(r.pos) for r in reps]
    plan = md.Plan(boxes, counts, 5.8)
    st = md.State(plan, np.concatenate([r.pos for r in reps]), None, prec)
    nl = md.NeighborList(plan.n_atoms, 128, lanes)
    md.md_bin_cells(st)
    md.md_build_neighbors(st, nl)
    return plan, st, nl


def test_batched_replicas_match_closed_form_and_single_calls(md):
    reps = mi.cold_curve_replicas(n_rep=8, seed=31, n_min=4, n_max=7)
    tab = mi.tabulate_eam(mi.EAM_CU)
    pot = md.EAMPotential.from_table(tab)
    plan, st, nl = _batch(md, reps)
    ev = md_ev(len(reps))
    md.md_eam_forces(st, pot, nl, ev=ev)
    st.check_flags()
    e = evv(ev)[0]
    assert np.max(np.abs(st.forces())) < 1e-10
    opot = core.EAMPotential.from_table(tab)
    sets = neighbor_sets_by_id(st, nl)
    off = 0
    for r, rep in enumerate(reps):
        n = len(rep.pos)
        e_cf, _ = ls.eam_per_atom(rep.a, mi.EAM_CU)
        assert abs(e[r, 0] / n - e_cf) < 1e-9, (r, rep.a)
        ro = core.eam(rep.pos, rep.box, opot)
        assert abs(e[r, 0] - ro.energy) < 1e-12 * abs(ro.energy)
        assert np.max(np.abs(e[r, 1:7] - ro.virial)) < 1e-11 * np.max(np.abs(ro.virial))
        cnt, want = core.neighbor_sets(rep.pos, rep.box, 5.8)
        for i in range(n):
            assert np.array_equal(sets[off + i] - off, want[i])
        # the same box alone
        p1, s1, n1 = _batch(md, [rep])
        ev1 = md_ev(1)
        md.md_eam_forces(s1, pot, n1, ev=ev1)
        assert abs(evv(ev1)[0, 0, 0] - e[r, 0]) < 1e-12 * abs(e[r, 0])
        off += n


@pytest.mark.parametrize("prec", [0, 1])
def test_cold_curve_64_replicas(md, prec):
    reps = mi.cold_curve_replicas()
    pot = md.EAMPotential.from_table(mi.tabulate_eam(mi.EAM_CU))
    plan, st, nl = _batch(md, reps, prec=prec)
    ev = md_ev(len(reps))
    md.md_eam_forces(st, pot, nl, ev=ev)
    st.check_flags()
    e = evv(ev)[0]
    tol = 1e-9 if prec == 0 else 1e-6
    for r, rep in enumerate(reps):
        e_cf, _ = ls.eam_per_atom(rep.a, mi.EAM_CU)
        assert abs(e[r, 0] / len(rep.pos) - e_cf) < tol, (r, rep.a, e[r, 0] / len(rep.pos), e_cf)
        # pressure from the virial equals -dE/dV of the closed form (T = 0); the splines'
        # first derivatives carry the O(h^3) interpolation error (~2e-8 relative to the
        # individual pair and embedding terms, which are ~0.1 eV/A^3 per unit volume even
        # where they cancel near equilibrium)
        V = len(rep.pos) * rep.a ** 3 / 4
        p_cf = -len(rep.pos) * ls.eam_dE_da(rep.a, mi.EAM_CU) / (3 * len(rep.pos) * rep.a ** 2 / 4)
        ptol = (1e-7 if prec == 0 else 1e-5) * (abs(p_cf) + 0.1)
        assert abs(e[r, 1:4].sum() / (3 * V) - p_cf) < ptol


def test_batched_graph_replay_equals_eager(md):
    reps = mi.cold_curve_replicas(n_rep=16, seed=33, n_min=4, n_max=6)
    pot = md.EAMPotential.from_table(mi.tabulate_eam(mi.EAM_CU))
    plan, st, nl = _batch(md, reps)
    ev = md_ev(len(reps))
    table = pot.table(0)
    md.md_eam_forces(st, pot, nl, table=table, ev=ev)
    torch.cuda.synchronize()
    eager = ev.clone()
    f_eager = st.force.clone()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(g, stream=s):
        md.md_eam_forces(st, pot, nl, table=table, ev=ev)
    torch.cuda.current_stream().wait_stream(s)
    for _ in range(3):
        ev.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(ev, eager) and torch.equal(st.force, f_eager)


# ----------------------------------------------------------------------------
# adjoint
# ----------------------------------------------------------------------------
def _fm_problem(md, n_snap=3, cells=5, prec=0, lanes=4, jac=True):
    from paper_2511_22951_amd import fm
    tab = mi.force_matching_tables()
    noise = mi.coefficient_noise()
    snaps = mi.force_matching_snapshots(n_snap=n_snap, cells=cells)
    # oracle side
    grids = tuple(oadj.Grid(tf.x_lo, tf.h, tf.K + 2) for tf in (tab.phi, tab.rho, tab.emb))
    c_or = [osp.fit_table(tf) * noise[64 * b:64 * (b + 1)]
            for b, tf in enumerate((tab.phi, tab.rho, tab.emb))]
    osnaps = [oadj.Snapshot(s.pos, s.box, mi.EAM_CU.r_cut) for s in snaps]
    # GPU side: its own fit of the same samples, times the same noise
    fits = [md.md_spline_fit(tf.y, tf.h, tf.dy_lo, tf.dy_hi) for tf in (tab.phi, tab.rho, tab.emb)]
    nz = torch.as_tensor(noise, device="cuda")
    pot = md.EAMPotential(fits[0] * nz[:64], fits[1] * nz[64:128], fits[2] * nz[128:],
                          tab.rho.x_lo, tab.rho.h, tab.emb.x_lo, tab.emb.h, mi.EAM_CU.r_cut)
    batch = fm.SnapshotBatch(snaps, mi.EAM_CU.r_cut + 0.3, precision=prec, lanes=lanes,
                             density_jacobian=jac)
    return snaps, osnaps, grids, c_or, pot, batch


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n", [0, 1, 1000, 300000])
def test_force_loss_matches_oracle(md, prec, n):
    """md_force_loss on seeded forces (one block, a ragged block and a grid that strides
    over the atoms): the loss within 1e-14 relative of the oracle's, the cotangent within
    1e-15 of its largest entry, both bitwise reproducible; n = 0 gives loss 0."""
    rng = np.random.default_rng(500 + n)
    F = rng.normal(size=(n, 3))
    Fr = rng.normal(size=(n, 3))
    if prec == 1:
        F = F.astype(np.float32)
    dt = torch.float32 if prec == 1 else torch.float64
    force = torch.as_tensor(np.ascontiguousarray(F.T), dtype=dt, device="cuda")
    f_ref = torch.as_tensor(np.ascontiguousarray(Fr.T), device="cuda")
    G = torch.full((3, n), 7.0, dtype=torch.float64, device="cuda")
    loss = md.md_force_loss(force, f_ref, prec, grad_force=G)
    if n == 0:
        assert loss.item() == 0.0
        return
    want_L, want_G = oadj.force_loss([F.astype(np.float64)], [Fr])
    assert abs(loss.item() - want_L) <= 1e-14 * want_L
    got_G = G.t().cpu().numpy()
    assert np.max(np.abs(got_G - want_G[0])) <= 1e-15 * np.max(np.abs(want_G[0]))
    G2 = torch.empty_like(G)
    assert torch.equal(md.md_force_loss(force, f_ref, prec, grad_force=G2), loss)
    assert torch.equal(G2, G)
    assert torch.equal(md.md_force_loss(force, f_ref, prec), loss)  # loss only


@pytest.mark.parametrize("prec", [0, 1])
def test_fused_loss_equals_force_path(md, prec):
    """force_matching_loss (forces, loss and cotangent in the library) against EAMForces with
    the loss written in torch: same loss to 1e-13 and same gradient to 1e-12, FP64 and FP32."""
    from paper_2511_22951_amd import fm
    snaps, osnaps, grids, c_or, pot, batch = _fm_problem(md, n_snap=2, prec=prec)
    ref_pot = md.EAMPotential.from_table(mi.tabulate_eam(mi.EAM_CU))
    f_ref = batch.forces(ref_pot, saved=False).clone()
    c1 = torch.cat([c.clone() for c in pot.coef]).requires_grad_(True)
    l1 = fm.force_matching_loss(c1, batch, pot, f_ref)
    l1.backward()
    c2 = torch.cat([c.clone() for c in pot.coef]).requires_grad_(True)
    f = fm.EAMForces.apply(c2, batch, pot)
    l2 = ((f - f_ref) ** 2).sum() / batch.n
    l2.backward()
    assert abs(l1.item() - l2.item()) <= 1e-13 * l2.item()
    g1, g2 = c1.grad.cpu().numpy(), c2.grad.cpu().numpy()
    assert np.max(np.abs(g1 - g2)) <= 1e-12 * np.max(np.abs(g2))


def test_adjoint_vjp_matches_oracle(md):
    snaps, osnaps, grids, c_or, pot, batch = _fm_problem(md)
    G = [mi.random_cotangent(len(s.pos), seed=40 + k) for k, s in enumerate(snaps)]
    want = np.concatenate(oadj.vjp(osnaps, c_or, grids, G))
    batch.forces(pot, saved=True)
    got = batch.backward(pot, batch.to_current_order(np.concatenate(G))).cpu().numpy()
    batch.state.check_flags()
    assert np.max(np.abs(got - want)) < 1e-10 * np.max(np.abs(want))
    got2 = batch.backward(pot, batch.to_current_order(np.concatenate(G))).cpu().numpy()
    assert np.array_equal(got, got2)  # run-to-run bitwise reproducible


@pytest.mark.parametrize("jac", [False, True])
@pytest.mark.parametrize("lanes", [1, 2, 4, 8, 16])
def test_adjoint_vjp_every_lane_count(md, lanes, jac):
    """The adjoint at every lane count the list allows (a different number of bin copies
    per wavefront fits the LDS at each: 8, 8, 8, 4, 2 with the second list visit, 4, 4, 4, 4,
    2 with the density Jacobian; 16 lanes leave about five list entries per lane) against the
    oracle's chain-rule VJP, 1e-10 relative."""
    snaps, osnaps, grids, c_or, pot, batch = _fm_problem(md, n_snap=2, lanes=lanes, jac=jac)
    G = [mi.random_cotangent(len(s.pos), seed=60 + k) for k, s in enumerate(snaps)]
    want = np.concatenate(oadj.vjp(osnaps, c_or, grids, G))
    batch.forces(pot, saved=True)
    got = batch.backward(pot, batch.to_current_order(np.concatenate(G))).cpu().numpy()
    batch.state.check_flags()
    assert np.max(np.abs(got - want)) < 1e-10 * np.max(np.abs(want))


@pytest.mark.parametrize("lanes", [1, 4, 16])
def test_density_jacobian_matches_oracle(md, lanes):
    """md_eam_density_jacobian against the oracle's d rhobar / d c_rho (rows in the batch's
    current order), 1e-12 of the largest entry, and bitwise reproducible."""
    snaps, osnaps, grids, c_or, pot, batch = _fm_problem(md, lanes=lanes)
    jac = md.md_eam_density_jacobian(batch.state, pot, batch.nl)
    batch.state.check_flags()
    want = np.concatenate([oadj.density_jacobian(s, grids[1]) for s in osnaps])
    got = jac.cpu().numpy()[np.argsort(batch.order_ids.cpu().numpy())]
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    assert torch.equal(md.md_eam_density_jacobian(batch.state, pot, batch.nl), jac)


@pytest.mark.parametrize("prec", [0, 1])
def test_forces_with_jacobian_match_pair_pass(md, prec):
    """md_eam_forces_jac (density as jac c_rho) against md_eam_forces on the same batch and
    against the oracle.  FP64: forces within 1e-12 and {rhobar, F', F''} within 1e-13 of their
    largest entries, forces within 1e-10 of the oracle's.  FP32 (the force pass's resampled
    r^2 tables of these 64-coefficient splines): both forms within 5e-5 (Frobenius) of the
    oracle's forces, rhobar within 1e-5 of the pair pass's (the pair pass sums the resampled
    FP32 density table, the Jacobian form evaluates the spline in FP64)."""
    snaps, osnaps, grids, c_or, pot, batch = _fm_problem(md, prec=prec, jac=False)
    st, nl = batch.state, batch.nl
    s0 = torch.empty((3, batch.n), dtype=torch.float64, device="cuda")
    md.md_eam_forces(st, pot, nl, saved=s0)
    f0 = st.force.double().clone()
    jac = md.md_eam_density_jacobian(st, pot, nl)
    s1 = torch.empty_like(s0)
    md.md_eam_forces_jac(st, pot, nl, jac, saved=s1)
    f1 = st.force.double().clone()
    st.check_flags()
    order = np.argsort(batch.order_ids.cpu().numpy())
    want = np.concatenate([oadj.forces(s, c_or, grids)[0] for s in osnaps])
    got0 = f0.t().cpu().numpy()[order]
    got1 = f1.t().cpu().numpy()[order]
    if prec == 0:
        fmax = f0.abs().max().item()
        assert (f1 - f0).abs().max().item() <= 1e-12 * fmax
        for r in range(3):
            assert (s1[r] - s0[r]).abs().max().item() <= 1e-13 * s0[r].abs().max().item()
        assert np.max(np.abs(got1 - want)) <= 1e-10 * np.max(np.abs(want))
    else:
        e0, e1 = (np.linalg.norm(g - want) / np.linalg.norm(want) for g in (got0, got1))
        assert e0 <= 5e-5 and e1 <= 5e-5, (e0, e1)
        assert (s1[0] - s0[0]).abs().max().item() <= 1e-5 * s0[0].abs().max().item()


@pytest.mark.parametrize("lanes", [2, 4])
def test_uneven_snapshots_jacobian_paths_match_oracle(md, lanes):
    """Snapshots of 4^3, 6^3 and 5^3 cells (256, 864 and 500 atoms: ragged last tiles) in one
    batch: the Jacobian density pass's forces and {rhobar} against the oracle's, and the
    adjoint with and without the Jacobian against the oracle's VJP (1e-10 relative)."""
    from paper_2511_22951_amd import fm
    tab = mi.force_matching_tables()
    noise = mi.coefficient_noise()
    snaps = (mi.force_matching_snapshots(n_snap=1, cells=4, seed=901)
             + mi.force_matching_snapshots(n_snap=1, cells=6, seed=902)
             + mi.force_matching_snapshots(n_snap=1, cells=5, seed=903))
    grids = tuple(oadj.Grid(tf.x_lo, tf.h, tf.K + 2) for tf in (tab.phi, tab.rho, tab.emb))
    c_or = [osp.fit_table(tf) * noise[64 * b:64 * (b + 1)]
            for b, tf in enumerate((tab.phi, tab.rho, tab.emb))]
    osnaps = [oadj.Snapshot(s.pos, s.box, mi.EAM_CU.r_cut) for s in snaps]
    fits = [md.md_spline_fit(tf.y, tf.h, tf.dy_lo, tf.dy_hi) for tf in (tab.phi, tab.rho, tab.emb)]
    nz = torch.as_tensor(noise, device="cuda")
    pot = md.EAMPotential(fits[0] * nz[:64], fits[1] * nz[64:128], fits[2] * nz[128:],
                          tab.rho.x_lo, tab.rho.h, tab.emb.x_lo, tab.emb.h, mi.EAM_CU.r_cut)
    G = [mi.random_cotangent(len(s.pos), seed=70 + k) for k, s in enumerate(snaps)]
    want_vjp = np.concatenate(oadj.vjp(osnaps, c_or, grids, G))
    want_f = np.concatenate([oadj.forces(s, c_or, grids)[0] for s in osnaps])
    want_rb = np.concatenate([oadj.forces(s, c_or, grids)[1] for s in osnaps])
    for jac in (False, True):
        batch = fm.SnapshotBatch(snaps, mi.EAM_CU.r_cut + 0.3, lanes=lanes, density_jacobian=jac)
        f = batch.forces(pot, saved=True)
        order = np.argsort(batch.order_ids.cpu().numpy())
        got_f = f.t().cpu().numpy()[order]
        got_rb = batch.saved[0].cpu().numpy()[order]
        assert np.max(np.abs(got_f - want_f)) <= 1e-10 * np.max(np.abs(want_f))
        assert np.max(np.abs(got_rb - want_rb)) <= 1e-12 * np.max(np.abs(want_rb))
        got = batch.backward(pot, batch.to_current_order(np.concatenate(G))).cpu().numpy()
        batch.state.check_flags()
        assert np.max(np.abs(got - want_vjp)) < 1e-10 * np.max(np.abs(want_vjp)), jac


def test_jacobian_paths_with_100_coefficient_splines(md):
    """Splines of 100 coefficients (the density pass's 8-loads-per-lane form, 51 KB Jacobian
    rows in LDS, 200 phi|rho bins per copy): the Jacobian against the oracle's (1e-12), the
    Jacobian forward's forces (1e-10) and both adjoint forms (1e-10) against the oracle."""
    from paper_2511_22951_amd import fm
    rr, qr = mi.FM_R_RANGE, mi.FM_RHO_RANGE
    tab = mi.tabulate_eam(mi.EAM_CU, K=98, r_lo=rr[0], r_hi=rr[1], rho_lo=qr[0], rho_hi=qr[1])
    snaps = mi.force_matching_snapshots(n_snap=2, cells=5, seed=911)
    grids = tuple(oadj.Grid(tf.x_lo, tf.h, tf.K + 2) for tf in (tab.phi, tab.rho, tab.emb))
    c_or = [osp.fit_table(tf) for tf in (tab.phi, tab.rho, tab.emb)]
    assert all(len(c) == 100 for c in c_or)
    osnaps = [oadj.Snapshot(s.pos, s.box, mi.EAM_CU.r_cut) for s in snaps]
    pot = md.EAMPotential.from_table(tab)
    G = [mi.random_cotangent(len(s.pos), seed=75 + k) for k, s in enumerate(snaps)]
    want_vjp = np.concatenate(oadj.vjp(osnaps, c_or, grids, G))
    want_f = np.concatenate([oadj.forces(s, c_or, grids)[0] for s in osnaps])
    want_j = np.concatenate([oadj.density_jacobian(s, grids[1]) for s in osnaps])
    for jac in (False, True):
        batch = fm.SnapshotBatch(snaps, mi.EAM_CU.r_cut + 0.3, density_jacobian=jac)
        order = np.argsort(batch.order_ids.cpu().numpy())
        if jac:
            J = batch.jacobian(pot).cpu().numpy()[order]
            assert np.max(np.abs(J - want_j)) <= 1e-12 * np.max(np.abs(want_j))
        f = batch.forces(pot, saved=True)
        assert np.max(np.abs(f.t().cpu().numpy()[order] - want_f)) <= 1e-10 * np.max(np.abs(want_f))
        got = batch.backward(pot, batch.to_current_order(np.concatenate(G))).cpu().numpy()
        batch.state.check_flags()
        assert np.max(np.abs(got - want_vjp)) < 1e-10 * np.max(np.abs(want_vjp)), jac


def test_backward_with_jacobian_equals_second_visit(md):
    """Both forms of the adjoint on the same forward state and cotangent: equal to 1e-13 of
    the largest gradient entry."""
    snaps, osnaps, grids, c_or, pot, batch = _fm_problem(md, jac=False)
    G = batch.to_current_order(np.concatenate(
        [mi.random_cotangent(len(s.pos), seed=80 + k) for k, s in enumerate(snaps)]))
    batch.forces(pot, saved=True)
    a = batch.backward(pot, G).cpu().numpy()
    jac = md.md_eam_density_jacobian(batch.state, pot, batch.nl)
    b = md.md_eam_backward(batch.state, pot, batch.nl, batch.saved, G, jac=jac).cpu().numpy()
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))


def test_force_matching_gradient_matches_oracle_and_fd(md):
    from paper_2511_22951_amd import fm
    snaps, osnaps, grids, c_or, pot, batch = _fm_problem(md)
    # reference forces: oracle from the analytic EAM; GPU from the 2000-point table
    apot = core.EAMPotential.analytic(mi.EAM_CU)
    f_ref_or = [core.eam(s.pos, s.box, apot).force for s in snaps]
    want = np.concatenate(oadj.gradient(osnaps, c_or, grids, f_ref_or))
    ref_pot = md.EAMPotential.from_table(mi.tabulate_eam(mi.EAM_CU))
    f_ref = batch.forces(ref_pot, saved=False).clone()
    coef = torch.cat([c.clone() for c in pot.coef]).requires_grad_(True)
    loss = fm.force_matching_loss(coef, batch, pot, f_ref)
    loss.backward()
    got = coef.grad.cpu().numpy()
    l_or = oadj.loss(osnaps, c_or, grids, f_ref_or)
    assert abs(loss.item() - l_or) < 1e-6 * l_or
    assert np.max(np.abs(got - want)) < 1e-6 * np.max(np.abs(want))
    # FP64 central differences of the GPU loss, h = 1e-6
    h = 1e-6
    for k in (5, 20, 64 + 10, 64 + 40, 128 + 20, 128 + 33):
        cp = coef.detach().clone()
        cm = coef.detach().clone()
        cp[k] += h
        cm[k] -= h
        lp = fm.force_matching_loss(cp, batch, pot, f_ref).item()
        lm = fm.force_matching_loss(cm, batch, pot, f_ref).item()
        fd = (lp - lm) / (2 * h)
        assert abs(fd - got[k]) < 1e-5 * np.max(np.abs(got)), (k, fd, got[k])


def test_force_matching_fp32_forward_gradient_near_fp64(md):
    """The FP32-mixed forward (records and r^2 tables, Jacobian density pass) with the FP64
    adjoint: loss within 1e-5 and gradient within 1e-5 of the largest entry of the all-FP64
    epoch's, for the same snapshots, coefficients and reference forces."""
    from paper_2511_22951_amd import fm
    out = {}
    for prec in (0, 1):
        snaps, osnaps, grids, c_or, pot, batch = _fm_problem(md, n_snap=2, prec=prec)
        ref_pot = md.EAMPotential.from_table(mi.tabulate_eam(mi.EAM_CU))
        f_ref = batch.forces(ref_pot, saved=False).clone() if prec == 0 else out[0][2]
        coef = torch.cat([c.clone() for c in pot.coef]).requires_grad_(True)
        loss = fm.force_matching_loss(coef, batch, pot, f_ref)
        loss.backward()
        batch.state.check_flags()
        out[prec] = (loss.item(), coef.grad.cpu().numpy(), f_ref)
    (l64, g64, _), (l32, g32, _) = out[0], out[1]
    assert abs(l32 - l64) <= 1e-5 * l64
    assert np.max(np.abs(g32 - g64)) <= 1e-5 * np.max(np.abs(g64))


def test_force_matching_backward_after_another_forward(md):
    """Two losses at different coefficients, then backward of the first: its gradient equals
    that of a forward-backward at the first coefficients alone, bit for bit."""
    from paper_2511_22951_amd import fm
    snaps, osnaps, grids, c_or, pot, batch = _fm_problem(md, n_snap=2)
    ref_pot = md.EAMPotential.from_table(mi.tabulate_eam(mi.EAM_CU))
    f_ref = batch.forces(ref_pot, saved=False).clone()
    c1 = torch.cat([c.clone() for c in pot.coef])
    c2 = c1 * 1.01
    a = c1.clone().requires_grad_(True)
    fm.force_matching_loss(a, batch, pot, f_ref).backward()
    want = a.grad.clone()
    b1 = c1.clone().requires_grad_(True)
    b2 = c2.clone().requires_grad_(True)
    l1 = fm.force_matching_loss(b1, batch, pot, f_ref)
    l2 = fm.force_matching_loss(b2, batch, pot, f_ref)
    l1.backward()
    assert torch.equal(b1.grad, want)
    assert torch.equal(torch.cat(pot.coef), c2)  # the later coefficients are back in place
    l2.backward()
    b2_alone = c2.clone().requires_grad_(True)
    fm.force_matching_loss(b2_alone, batch, pot, f_ref).backward()
    assert torch.equal(b2.grad, b2_alone.grad)


def test_launch_shapes_and_tuner(md, tmp_path):
    """Every launch shape the tuner may pick -- (lanes per atom, workgroup size) -- gives the
    fixed default shape's per-replica records and forces on the 64 uneven cold-curve
    replicas, displaced (FP64, 1e-12 relative); the tuner times each shape once, takes the
    fastest, and reuses the cached choice for the same key without timing."""
    from paper_2511_22951_amd import tune
    from tests.gpu_util import rel_fro
    reps = mi.cold_curve_replicas()
    rng = np.random.default_rng(77)
    for r in reps:
        r.pos = r.pos + rng.normal(0.0, 0.05, r.pos.shape)
    pot = md.EAMPotential.from_table(mi.tabulate_eam(mi.EAM_CU))
    table = pot.table(0)

    def run(shape, calls=1):
        plan, st, nl = _batch(md, reps, 0, shape[0])
        nl.set_block(shape[1])
        ev = md_ev(len(reps))
        for _ in range(calls):
            md.md_eam_forces(st, pot, nl, table=table, ev=ev)
        st.check_flags()
        return evv(ev)[0], st.forces(), st

    e0, f0, _ = run((4, 1024))
    # per replica: 1e-12 of the record's largest component, plus one fixed-point quantum
    # (2^-36 eV) per tile, since a different workgroup size rounds differently grouped tile
    # partials into the fixed-point record
    tiles = np.array([(len(r.pos) + 63) // 64 for r in reps], np.float64)
    tol = 1e-12 * np.max(np.abs(e0), axis=1) + tiles * 2.0 ** -36
    assert np.max(np.abs(f0)) > 0.1
    for shape in tune.shapes(0):
        e, f, _ = run(shape)
        assert np.all(np.abs(e - e0) <= tol[:, None]), shape
        assert rel_fro(f, f0) < 1e-12, shape

    calls = []

    def time_fn(shape):
        calls.append(shape)
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        plan, st, nl = _batch(md, reps, 0, shape[0])
        nl.set_block(shape[1])
        t0.record()
        for _ in range(3):
            md.md_eam_forces(st, pot, nl, table=table)
        t1.record()
        torch.cuda.synchronize()
        return t0.elapsed_time(t1)

    path = str(tmp_path / "tune.json")
    best = tune.pick(("cold_curve_test", "fp64"), tune.shapes(0), time_fn, cache_path=path)
    assert best in tune.shapes(0) and sorted(calls) == sorted(tune.shapes(0))
    n = len(calls)
    assert tune.pick(("cold_curve_test", "fp64"), tune.shapes(0), time_fn, cache_path=path) == best
    assert len(calls) == n
