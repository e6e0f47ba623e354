"""md_eam_forces_noalloc (the allocation-free entry point, scratch in a static device array)
against md_eam_forces on the same inputs, through the C ABI: two calls in a row, the second
on a smaller system, FP64 and FP32, with the trailing kick, the fused next kick-drift, the
saved {rhobar, F', F''} and the per-box records.  The two entry points run the same kernels
on the same inputs, so every output must agree bit for bit."""
import numpy as np
import pytest
import torch

import mdinputs as mi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def md():
    from paper_2511_22951_amd import _native, md
    _native.lib()
    return md


def _state(md, system, prec, lanes):
    plan = md.Plan([system.box], [len(system.pos)], system.eam.r_cut + system.skin)
    st = md.State(plan, system.pos, system.vel, prec)
    nl = md.NeighborList(plan.n_atoms, 128, lanes)
    md.md_bin_cells(st)
    md.md_build_neighbors(st, nl)
    return st, nl


@pytest.mark.parametrize("prec,lanes", [(0, 2), (1, 2), (1, 4)])
def test_noalloc_equals_workspace_entry_point(md, prec, lanes):
    for cells in (8, 5):  # the second call on a smaller system
        system = mi.eam_copper(cells=cells)
        pot = md.EAMPotential.from_table(system.table)
        out = []
        for fn in (md.md_eam_forces, md.md_eam_forces_noalloc):
            st, nl = _state(md, system, prec, lanes)
            n = st.n
            saved = torch.zeros((3, n), dtype=torch.float64, device="cuda")
            ev = md.ev_buffer(4, 1, "cuda")
            pos_out = torch.empty_like(st.pos)
            drift = md.drift_params(pos_out, st.pos_ref, system.dt_ps, 0.5 * system.skin, None)
            fn(st, pot, nl, saved=saved, inv_mass=1.0 / system.mass, half_dt=0.5 * system.dt_ps,
               kick=True, ev=ev, ev_cap=4, drift=drift)
            st.check_flags()
            torch.cuda.synchronize()
            out.append([st.force.clone(), st.vel.clone(), st.pos.clone(), pos_out.clone(),
                        saved.clone(), ev.clone()])
        for a, b in zip(*out):
            assert torch.equal(a, b)
        assert torch.count_nonzero(out[0][0]) > 0 and torch.count_nonzero(out[0][5]) > 0


def test_noalloc_at_its_maximum_size(md):
    """At exactly MD_NOALLOC_MAX_ATOMS atoms (Cu fcc 64^3 = 2^20, 16,384 tiles) the static
    scratch is filled to its end: FP32 (whose neighbour records use the whole record region),
    bit for bit against md_eam_forces, then a small system on the same scratch."""
    from paper_2511_22951_amd import _native as N
    for cells in (64, 5):
        system = mi.eam_copper(cells=cells)
        if cells == 64:
            assert len(system.pos) == N.MD_NOALLOC_MAX_ATOMS
        pot = md.EAMPotential.from_table(system.table)
        out = []
        for fn in (md.md_eam_forces, md.md_eam_forces_noalloc):
            st, nl = _state(md, system, 1, 2)
            ev = md.ev_buffer(4, 1, "cuda")
            fn(st, pot, nl, inv_mass=1.0 / system.mass, half_dt=0.5 * system.dt_ps, kick=True,
               ev=ev, ev_cap=4)
            st.check_flags()
            torch.cuda.synchronize()
            out.append([st.force.clone(), st.vel.clone(), ev.clone()])
        for a, b in zip(*out):
            assert torch.equal(a, b)
        assert torch.count_nonzero(out[0][0]) > 0
