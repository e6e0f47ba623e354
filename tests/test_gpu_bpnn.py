"""GPU parity of the Behler-Parrinello potential (md_bpnn_forces) with the oracle
(oracle/bpnn.py), through the C ABI.

  forces / atomic energies / E / virial   Cu 256 atoms, displaced, 300 K       1e-10 / 1e-11
  NVE steps                               4 velocity-Verlet steps, positions     1e-10
  perfect crystal at any size             E/atom of 4^3 and 12^3 cells agree, forces vanish
  argument checks                         malformed md_bpnn -> MD_ERR_ARG
"""
import ctypes as C

import numpy as np
import pytest

import mdinputs as mi
from oracle import bpnn, integrate

pytestmark = pytest.mark.gpu


def _rel_fro(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_bpnn_matches_oracle():
    import torch
    from paper_2511_22951_amd import _native as N
    from paper_2511_22951_amd import md
    from paper_2511_22951_amd.sim import Simulation
    s = mi.bpnn_copper(cells=4)
    p = s.extra["bpnn"]
    sim = Simulation(s, precision=N.MD_FP64, lanes=4, ev_cap=4).setup()
    st = sim.state
    e_atom = torch.empty(st.n, dtype=torch.float64, device="cuda")
    md.md_bpnn_forces(st, sim.bpnn, sim.nl, ev=sim.ev, ev_cap=sim.ev_cap, e_atom=e_atom)
    st.check_flags()
    rec = md.ev_values(sim.ev)[st.read_flags()[1]["step"] % sim.ev_cap, 0]
    E, e, f, w = bpnn.forces(s.pos, s.box, p)
    order = np.argsort(st.id.cpu().numpy(), kind="stable")
    assert _rel_fro(st.forces(), f) < 1e-10
    assert np.abs(e_atom.cpu().numpy()[order] - e).max() < 1e-11 * np.abs(e).max()
    assert abs(rec[0] - E) < 1e-11 * abs(E)
    assert np.abs(rec[1:7] - w).max() < 1e-10 * np.abs(w).max()


def test_bpnn_nve_steps_match_oracle():
    from paper_2511_22951_amd import _native as N
    from paper_2511_22951_amd.sim import Simulation
    s = mi.bpnn_copper(cells=4)
    p = s.extra["bpnn"]
    sim = Simulation(s, precision=N.MD_FP64, lanes=2, ev_cap=8).setup()
    sim.run(4)
    sim.state.check_flags()
    fn = lambda x: (lambda r: (r[2], r[0]))(bpnn.forces(x, s.box, p))
    xo, vo, _, _ = integrate.run_nve(s.pos, s.vel, s.box, s.mass, s.dt_ps, 4, fn)
    d = sim.state.positions() - xo
    d -= np.asarray(s.box.len) * np.rint(d / np.asarray(s.box.len))
    assert np.abs(d).max() < 1e-10
    assert np.abs(sim.state.velocities() - vo).max() < 1e-8


def test_bpnn_perfect_crystal_any_size():
    from paper_2511_22951_amd import _native as N
    from paper_2511_22951_amd.sim import Simulation
    out = []
    for cells in (4, 12):
        pos, box = mi.fcc_lattice(cells, cells, cells, 3.615)
        s = mi.bpnn_copper(cells=cells)
        s.pos, s.vel = pos, np.zeros_like(pos)
        sim = Simulation(s, precision=N.MD_FP64, lanes=4, ev_cap=4).setup()
        info = sim.state.check_flags()
        rec = sim.energies([info["step"]])[0]
        out.append(rec[0] / pos.shape[0])
        assert np.abs(sim.state.forces()).max() < 1e-12
    assert abs(out[0] - out[1]) < 1e-12 * abs(out[0])


def test_bpnn_rejects_malformed_parameters():
    from paper_2511_22951_amd import _native as N
    from paper_2511_22951_amd import md
    from paper_2511_22951_amd.sim import Simulation
    s = mi.bpnn_copper(cells=4)
    sim = Simulation(s, precision=N.MD_FP64, lanes=4, ev_cap=4).setup()
    st = sim.state
    ws = md.md_bpnn_forces(st, sim.bpnn, sim.nl)
    L = N.lib()

    def call(c):
        return L.md_bpnn_forces(C.byref(st.plan.c), C.byref(c), md._ptr(st.pos), C.byref(sim.nl.c),
                                md._ptr(st.force), None, None, 0.0, 0.0, None, 1, md._ptr(ws),
                                md._ptr(st.ctl), md._stream())

    def fresh():
        c = N.BPNN()
        C.memmove(C.addressof(c), C.addressof(sim.bpnn.c), C.sizeof(c))
        return c

    assert call(fresh()) == N.MD_OK
    bad = fresh()
    bad.n_g4 = 60  # 8 + 60 inputs > 64
    assert call(bad) == N.MD_ERR_ARG
    bad = fresh()
    bad.g4_zeta[0] = 0.5
    assert call(bad) == N.MD_ERR_ARG
    bad = fresh()
    bad.g4_lambda[3] = 0.5
    assert call(bad) == N.MD_ERR_ARG
    bad = fresh()
    for q in range(9):  # nine distinct eta values
        bad.g4_eta[q] = 0.001 * (q + 1)
    assert call(bad) == N.MD_ERR_ARG
    bad = fresh()
    bad.weights = None
    assert call(bad) == N.MD_ERR_ARG
    st.check_flags()


def test_bpnn_batch_equals_single_boxes():
    """Two boxes of different size in one batch give each box's own forces and records."""
    import torch
    from paper_2511_22951_amd import _native as N
    from paper_2511_22951_amd import md
    p = mi.bpnn_params()
    pot = md.BPNNPotential(p)
    systems = [mi.bpnn_copper(cells=4, seed=11), mi.bpnn_copper(cells=5, seed=12)]
    r_ns = p["r_cut"] + 0.3

    def run(sys_list):
        plan = md.Plan([s.box for s in sys_list], [s.pos.shape[0] for s in sys_list], r_ns)
        st = md.State(plan, np.concatenate([s.pos for s in sys_list]), None, N.MD_FP64)
        nl = md.NeighborList(plan.n_atoms, 128, 4)
        md.md_bin_cells(st)
        md.md_build_neighbors(st, nl)
        ev = md.ev_buffer(1, len(sys_list))
        md.md_bpnn_forces(st, pot, nl, ev=ev, ev_cap=1)
        st.check_flags()
        return st.forces(), md.ev_values(ev)[0]

    fb, eb = run(systems)
    n0 = systems[0].pos.shape[0]
    for k, s in enumerate(systems):
        f1, e1 = run([s])
        part = fb[:n0] if k == 0 else fb[n0:]
        assert np.abs(part - f1).max() <= 1e-13 * np.abs(f1).max()
        assert np.allclose(eb[k], e1[0], rtol=1e-12, atol=1e-9)
