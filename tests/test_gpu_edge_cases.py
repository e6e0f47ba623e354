"""Degenerate inputs of the HIP path, through the C ABI.

  empty box in a batch     a box without atoms between two Cu boxes: the others' lists,
                           forces and records equal single-box calls (forces bit for bit,
                           records to the fixed-point rounding of per-block sums); the
                           empty box's record is exactly zero; EAM and LJ, FP64 and FP32
  empty batch              n_atoms = 0: every entry point returns MD_OK and writes nothing
                           (md_profiles, both adjoints and md_force_loss write zeros)
  lone atom                no neighbours: LJ force and energy exactly zero; EAM density 0
                           lies below the embedding table, so MD_ERR_TABLE_RANGE is reported
                           (the oracle flags the same atom)
  pairs past the cutoff    listed pairs with r_c < r < r_ns (the FP32 tables' zero row, the
                           FP64 mask) add exactly nothing: an EAM dimer's forces are bit for
                           bit those with the second dimer far away
  dimer                    LJ force and energy equal the closed form of eq. 1.6 (FP64 to
                           1e-14, FP32 to 1e-6); virial equal to the oracle's.  EAM: energy
                           2 F(rho(r)) + phi(r) and the pair force with both atoms' F' from the
                           analytic forms, within the tables' interpolation error
"""
import ctypes as C

import numpy as np
import pytest
import torch

import mdinputs as mi
from oracle import core
from tests.gpu_util import displaced, evv, md_ev, neighbor_sets_by_id

pytestmark = pytest.mark.gpu

R_NS = 5.8


def _run(md, systems, pot, prec, lanes=4):
    """Bin, list and one force pass for a batch of (pos, box) systems."""
    plan = md.Plan([b for _, b in systems], [len(p) for p, _ in systems], R_NS)
    pos = np.concatenate([p for p, _ in systems]) if plan.n_atoms else np.zeros((0, 3))
    st = md.State(plan, pos, None, prec)
    nl = md.NeighborList(plan.n_atoms, 128, lanes)
    md.md_bin_cells(st)
    md.md_build_neighbors(st, nl)
    ev = md_ev(len(systems))
    if pot == "eam":
        md.md_eam_forces(st, md.EAMPotential.from_table(mi.tabulate_eam(mi.EAM_CU)), nl, ev=ev)
    else:
        p = mi.LJ_AR
        md.md_lj_forces(st, md.lj_params(p.eps, p.sigma, 5.5), nl, ev=ev)
    st.check_flags()
    return st, nl, evv(ev)[0]


@pytest.mark.parametrize("pot,prec", [("eam", 0), ("eam", 1), ("lj", 0), ("lj", 1)])
def test_empty_box_in_batch_equals_single_boxes(pot, prec):
    from paper_2511_22951_amd import md
    print("case", pot, prec, flush=True)
    a = displaced(4, 3.615, 0.06, seed=31)
    c = displaced(5, 3.615, 0.06, seed=32)
    empty = (np.zeros((0, 3)), mi.Box((0.0, 0.0, 0.0), (15.0, 16.0, 17.0), (1, 1, 1)))
    st, nl, rec = _run(md, [a, empty, c], pot, prec)
    assert np.all(rec[1] == 0.0)
    f = st.forces()
    sets = neighbor_sets_by_id(st, nl)
    na = len(a[0])
    for k, (sysk, part) in enumerate([(a, slice(0, na)), (c, slice(na, None))]):
        s1, nl1, rec1 = _run(md, [sysk], pot, prec)
        assert np.array_equal(f[part], s1.forces())
        sets1 = neighbor_sets_by_id(s1, nl1)
        off = 0 if k == 0 else na
        for i, js in sets1.items():
            assert np.array_equal(sets[i + off] - off, js)
        want = rec1[0]
        assert np.allclose(rec[2 * k], want, rtol=1e-12, atol=1e-9)


def test_empty_batch_entry_points_write_nothing():
    from paper_2511_22951_amd import _native as N
    from paper_2511_22951_amd import md
    L = N.lib()
    box = mi.Box((0.0, 0.0, 0.0), (15.0, 15.0, 15.0), (1, 1, 1))
    plan = md.Plan([box], [0], R_NS)
    assert plan.n_atoms == 0 and plan.n_tiles == 0
    b = C.byref(plan.c)
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    sentinel = 12345.0
    buf = {k: torch.full((256,), sentinel, dtype=torch.float64, device="cuda")
           for k in ("pos", "vel", "force", "pos_ref", "saved", "e", "w", "rf", "grad", "out")}
    ibuf = {k: torch.full((256,), 777, dtype=torch.int32, device="cuda")
            for k in ("id", "cell_start", "neigh", "nneigh")}
    ws = torch.zeros(1 << 16, dtype=torch.uint8, device="cuda")
    ctl = torch.zeros(int(L.md_ctl_bytes()), dtype=torch.uint8, device="cuda")
    assert L.md_ctl_init(md._ptr(ctl), s) == N.MD_OK
    ev = torch.full((1, 1, N.MD_EV_LEN), 99, dtype=torch.int64, device="cuda")
    P = lambda t: md._ptr(t)
    nl = N.NList(ibuf["neigh"].data_ptr(), ibuf["nneigh"].data_ptr(), 128, 4)
    pot = md.EAMPotential.from_table(mi.tabulate_eam(mi.EAM_CU))
    p = mi.LJ_AR
    lj = md.lj_params(p.eps, p.sigma, p.r_cut)
    ok = N.MD_OK
    assert L.md_bin_cells(b, N.MD_ALWAYS, P(buf["pos"]), P(buf["vel"]), P(ibuf["id"]),
                          P(buf["pos_ref"]), P(ibuf["cell_start"]), P(ws), P(ctl), s) == ok
    assert L.md_build_neighbors(b, N.MD_ALWAYS, P(buf["pos"]), P(ibuf["cell_start"]),
                                C.byref(nl), P(ctl), s) == ok
    for prec in (N.MD_FP64, N.MD_FP32):
        assert L.md_eam_forces(b, C.byref(pot.c), prec, P(pot.table(prec)), P(buf["pos"]),
                               C.byref(nl), P(buf["force"]), P(buf["saved"]), P(buf["vel"]),
                               1.0, 0.0005, None, P(ev), 1, P(ws), P(ctl), s) == ok
        assert L.md_lj_forces(b, C.byref(lj), prec, P(buf["pos"]), C.byref(nl),
                              P(buf["force"]), P(buf["vel"]), 1.0, 0.0005, None, P(ev), 1,
                              P(ws), P(ctl), s) == ok
        for phase in (N.MD_KICK_DRIFT, N.MD_KICK):
            assert L.md_verlet_step(b, phase, 0.001, P(buf["pos"]), P(buf["vel"]),
                                    P(buf["force"]), prec, 1.0, None, None, P(buf["pos_ref"]),
                                    0.15, P(ctl), s) == ok
    assert L.md_atom_observables(b, None, C.byref(lj), P(buf["pos"]), C.byref(nl), P(buf["e"]),
                                 P(buf["w"]), P(buf["rf"]), P(ctl), s) == ok
    bp = md.BPNNPotential(mi.bpnn_params())
    assert L.md_bpnn_forces(b, C.byref(bp.c), P(buf["pos"]), C.byref(nl), P(buf["force"]),
                            P(buf["e"]), None, 0.0, 0.0, P(ev), 1, P(ws), P(ctl), s) == ok
    torch.cuda.synchronize()
    for k, t in buf.items():
        assert torch.all(t == sentinel), k
    for k, t in ibuf.items():
        assert torch.all(t == 777), k
    assert torch.all(ev == 99)
    # reductions over no atoms: zeros
    n_bins = 8
    pw = torch.zeros(int(L.md_profile_workspace_bytes(n_bins)), dtype=torch.uint8, device="cuda")
    assert L.md_profiles(b, 2, 0.0, 15.0 / n_bins, n_bins, P(buf["pos"]), P(buf["vel"]), 63.546,
                         None, None, P(buf["out"]), P(pw), s) == ok
    fm = md.EAMPotential.from_table(mi.force_matching_tables())  # 3 x 64 coefficients
    ncoef = fm.c.phi.ncoef + fm.c.rho.ncoef + fm.c.emb.ncoef
    assert ncoef == 192
    assert L.md_eam_backward(b, C.byref(fm.c), N.MD_FP64, P(buf["pos"]), C.byref(nl),
                             P(buf["saved"]), P(buf["force"]), P(buf["grad"]), P(ws), P(ctl),
                             s) == ok
    assert L.md_eam_density_jacobian(b, C.byref(fm.c), P(buf["pos"]), C.byref(nl),
                                     P(buf["out"]), P(ctl), s) == ok
    for prec in (N.MD_FP64, N.MD_FP32):
        assert L.md_eam_forces_jac(b, C.byref(fm.c), prec, P(fm.table(prec)), P(buf["pos"]),
                                   C.byref(nl), P(buf["out"]), P(buf["force"]), P(buf["saved"]),
                                   P(ws), P(ctl), s) == ok
    g2 = torch.full((ncoef + 4,), sentinel, dtype=torch.float64, device="cuda")
    assert L.md_eam_backward_jac(b, C.byref(fm.c), N.MD_FP64, P(buf["pos"]), C.byref(nl),
                                 P(buf["saved"]), P(buf["out"]), P(buf["force"]), P(g2), P(ws),
                                 P(ctl), s) == ok
    lo = torch.full((2,), sentinel, dtype=torch.float64, device="cuda")
    assert ws.numel() >= L.md_force_loss_workspace_bytes(0)
    for prec in (N.MD_FP64, N.MD_FP32):
        assert L.md_force_loss(0, prec, None, None, P(lo), None, P(ws), s) == ok
    torch.cuda.synchronize()
    assert lo[0].item() == 0.0 and lo[1].item() == sentinel
    assert torch.all(buf["out"][:n_bins * N.MD_PROF_LEN] == 0.0)
    assert torch.all(buf["out"][n_bins * N.MD_PROF_LEN:] == sentinel)
    assert torch.all(buf["grad"][:ncoef] == 0.0) and torch.all(buf["grad"][ncoef:] == sentinel)
    assert torch.all(g2[:ncoef] == 0.0) and torch.all(g2[ncoef:] == sentinel)
    flags = (C.c_int * 4)()
    assert L.md_read_flags(P(ctl), flags, s) == ok
    assert list(flags) == [0, 0, 0, 0]  # flags, step, rebuilds, longest list


def test_lone_atom():
    from paper_2511_22951_amd import md
    box = mi.Box((0.0, 0.0, 0.0), (15.0, 15.0, 15.0), (1, 1, 1))
    x = np.array([[3.0, 4.0, 5.0]])
    for prec in (0, 1):
        st, nl, rec = _run(md, [(x, box)], "lj", prec)
        assert int(nl.lengths().cpu()[0]) == 0
        assert np.all(st.forces() == 0.0) and np.all(rec[0, :7] == 0.0)
    # EAM: rhobar = 0 is below the embedding table (which starts at 1), as in the oracle
    o = core.eam(x, box, core.EAMPotential.from_table(mi.tabulate_eam(mi.EAM_CU)))
    assert o.out_of_range == 1
    with pytest.raises(md.MDError) as e:
        _run(md, [(x, box)], "eam", 0)
    assert e.value.status == -4


@pytest.mark.parametrize("prec,tol", [(0, 1e-14), (1, 1e-6)])
def test_lj_dimer_closed_form(prec, tol):
    from paper_2511_22951_amd import md
    p = mi.LJ_AR
    box = mi.Box((0.0, 0.0, 0.0), (30.0, 30.0, 30.0), (1, 1, 1))
    r = 3.7
    d = np.array([0.6, -0.48, 0.64]) * r  # a unit vector times r
    x = np.array([[10.0, 11.0, 12.0], [10.0, 11.0, 12.0] + d])
    plan = md.Plan([box], [2], p.r_cut + 0.3)
    st = md.State(plan, x, None, prec)
    nl = md.NeighborList(2, 128, 4)
    md.md_bin_cells(st)
    md.md_build_neighbors(st, nl)
    ev = md_ev(1)
    md.md_lj_forces(st, md.lj_params(p.eps, p.sigma, p.r_cut), nl, ev=ev)
    st.check_flags()
    sr6, sc6 = (p.sigma / r) ** 6, (p.sigma / p.r_cut) ** 6
    fmag = 24.0 * p.eps * (2.0 * sr6 * sr6 - sr6) / r  # > 0: repulsive at 3.7 A
    u = 4.0 * p.eps * (sr6 * sr6 - sr6) - 4.0 * p.eps * (sc6 * sc6 - sc6)
    f = st.forces()
    unit = d / r
    assert np.max(np.abs(f[1] - fmag * unit)) <= tol * abs(fmag)
    assert np.max(np.abs(f[0] + fmag * unit)) <= tol * abs(fmag)
    rec = evv(ev)[0, 0]
    assert abs(rec[0] - u) <= tol * abs(u) + 2e-11
    o = core.lj(x, box, p.eps, p.sigma, p.r_cut)
    assert np.max(np.abs(rec[1:7] - o.virial)) <= tol * np.max(np.abs(o.virial)) + 2e-11


@pytest.mark.parametrize("prec,tol_e", [(0, 1e-8), (1, 1e-6)])
def test_eam_dimer_closed_form(prec, tol_e):
    """Two Cu atoms 2.5 A apart: E = 2 F(rho(r)) + phi(r), and the force on each is
    [phi'(r) + 2 F'(rho(r)) rho'(r)] along the pair (both atoms' F' enter the pair term),
    from the analytic forms the tables sample.  Tolerances: the 2000-point splines'
    interpolation error (about 1e-9 on E, a few 1e-7 on F' near rho = 1)."""
    from paper_2511_22951_amd import md
    p = mi.EAM_CU
    box = mi.Box((0.0, 0.0, 0.0), (30.0, 30.0, 30.0), (1, 1, 1))
    r = 2.5
    unit = np.array([0.48, 0.6, -0.64])
    x = np.array([[10.0, 11.0, 12.0], [10.0, 11.0, 12.0] + r * unit])
    st, nl, rec = _run(md, [(x, box)], "eam", prec)
    phi = p.A * np.exp(-p.alpha * (r / p.r0 - 1.0))
    rho = np.exp(-p.beta * (r / p.r0 - 1.0))
    dphi, drho = -p.alpha / p.r0 * phi, -p.beta / p.r0 * rho
    e = 2.0 * -np.sqrt(rho) + phi
    dedr = dphi + 2.0 * (-0.5 / np.sqrt(rho)) * drho
    f = st.forces()
    assert abs(rec[0, 0] - e) <= tol_e * abs(e)
    assert np.max(np.abs(f[1] + dedr * unit)) <= 5e-6 * abs(dedr)
    assert np.max(np.abs(f[0] - dedr * unit)) <= 5e-6 * abs(dedr)


@pytest.mark.parametrize("prec", [0, 1])
def test_eam_listed_pairs_past_the_cutoff_add_nothing(prec):
    """Two Cu dimers (2.5 A bonds) whose atoms face each other at 5.6 A, between r_c = 5.5 and
    r_ns = 5.8: the cross pairs are listed but lie past the cutoff, so the first dimer's forces
    equal, bit for bit, those with the second dimer moved far away, and the energy is twice
    the lone dimer's."""
    from paper_2511_22951_amd import md
    box = mi.Box((0.0, 0.0, 0.0), (40.0, 40.0, 40.0), (1, 1, 1))
    a, b = np.array([10.0, 10.0, 10.0]), np.array([12.5, 10.0, 10.0])
    near = np.array([a, b, a + [0.0, 0.0, 5.6], b + [0.0, 0.0, 5.6]])
    far = np.array([a, b, a + [0.0, 0.0, 15.6], b + [0.0, 0.0, 15.6]])
    got = {}
    for name, x in (("near", near), ("far", far)):
        st, nl, rec = _run(md, [(x, box)], "eam", prec)
        ids = st.id.cpu().numpy()
        nn = nl.lengths().cpu().numpy()
        f = st.forces()  # by original id
        got[name] = (f, rec[0, 0], {int(ids[k]): int(nn[k]) for k in range(len(ids))})
    assert got["near"][2][0] == 2 and got["far"][2][0] == 1  # the cross pair is listed
    assert np.array_equal(got["near"][0][:2], got["far"][0][:2])
    assert abs(got["near"][1] - got["far"][1]) <= 1e-9
