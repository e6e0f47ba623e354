"""An EAM potential read from a setfl file (Sec. 3.3) runs through the GPU path: a file
written from the analytic Cu form on a typical repository grid (3000 r samples of
0.002 A, 3000 rho samples of 0.015) gives the oracle's analytic energies and forces
within the cubic-interpolation error (about 3e-11 relative for these grids)."""
import numpy as np
import pytest

import mdinputs as mi
from oracle import core

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,tol_f,tol_e", [(0, 1e-7, 1e-8), (1, 1e-5, 1e-6)])
def test_setfl_potential_matches_analytic_oracle(tmp_path, prec, tol_f, tol_e):
    from paper_2511_22951_amd import eamfile
    from paper_2511_22951_amd.sim import Simulation
    p = mi.EAM_CU
    r = 0.002 * np.arange(3000)
    q = 0.015 * np.arange(3000)
    phi = p.A * np.exp(-p.alpha * (r / p.r0 - 1.0))
    rho = np.exp(-p.beta * (r / p.r0 - 1.0))
    path = tmp_path / "Cu.eam.alloy"
    eamfile.write_setfl(path, -np.sqrt(q), rho, r * phi, 0.015, 0.002, p.r_cut, element="Cu",
                        z=29, mass=63.546, a=3.615)
    table = eamfile.read_eam(path)
    s = mi.eam_copper(cells=6)
    sim = Simulation(s, precision=prec, lanes=4, ev_cap=4, table=table).setup()
    info = sim.state.check_flags()
    e = sim.energies([info["step"]])[0]
    want = core.eam(s.pos, s.box, core.EAMPotential.analytic(p))
    f = sim.state.forces()
    assert np.linalg.norm(f - want.force) / np.linalg.norm(want.force) < tol_f
    assert abs(e[0] - want.energy) < tol_e * abs(want.energy)
