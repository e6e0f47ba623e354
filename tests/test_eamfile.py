"""Reading tabulated EAM files (setfl, funcfl): round trips of files written from the
analytic Cu form, end slopes against the analytic derivatives, thinning of long grids and
malformed files (host logic, no GPU)."""
import math

import numpy as np
import pytest

import mdinputs as mi
from paper_2511_22951_amd import eamfile

P = mi.EAM_CU


def _cu_samples(nr=3000, dr=0.002, nrho=3000, drho=0.015):
    r = dr * np.arange(nr)
    q = drho * np.arange(nrho)
    phi = P.A * np.exp(-P.alpha * (r / P.r0 - 1.0))
    rho = np.exp(-P.beta * (r / P.r0 - 1.0))
    F = -np.sqrt(q)
    return r, q, phi, rho, F


def test_setfl_round_trip(tmp_path):
    r, q, phi, rho, F = _cu_samples()
    path = tmp_path / "Cu.eam.alloy"
    eamfile.write_setfl(path, F, rho, r * phi, 0.015, 0.002, 5.5, element="Cu", z=29,
                        mass=63.546, a=3.615)
    t = eamfile.read_eam(path)
    assert t.element == "Cu" and t.mass == 63.546 and t.lattice == "fcc" and t.r_cut == 5.5
    assert t.phi.x_lo == 0.002 and t.phi.h == 0.002 and t.phi.K == 2999
    assert np.allclose(t.phi.y, phi[1:], rtol=1e-15) and np.allclose(t.rho.y, rho[1:], rtol=1e-15)
    assert t.emb.x_lo == 0.0 and np.allclose(t.emb.y, F, rtol=0, atol=1e-15)
    # end slopes from third-order one-sided differences: for exp(-k r) the relative error
    # is (k h)^3 / 4 = 8.7e-8 at k = alpha / r0 = 3.52 / A, h = 0.002 A
    dphi = lambda x: -P.A * P.alpha / P.r0 * math.exp(-P.alpha * (x / P.r0 - 1.0))
    assert math.isclose(t.phi.dy_lo, dphi(t.phi.x_lo), rel_tol=2e-7)
    assert math.isclose(t.phi.dy_hi, dphi(t.phi.x_hi), rel_tol=2e-7)


def test_funcfl_round_trip(tmp_path):
    nr, dr, nrho, drho = 500, 0.012, 400, 0.1
    r = dr * np.arange(nr)
    Z = 3.0 * np.exp(-r)
    rho = np.exp(-r)
    F = -np.sqrt(drho * np.arange(nrho))
    vals = lambda v: "\n".join(" ".join("%.16e" % x for x in v[i:i + 5]) for i in range(0, len(v), 5))
    path = tmp_path / "X.eam"
    path.write_text("made-up funcfl\n29 63.546 3.615 fcc\n%d %.16e %d %.16e 5.5\n%s\n%s\n%s\n"
                    % (nrho, drho, nr, dr, vals(F), vals(Z), vals(rho)))
    t = eamfile.read_eam(path)
    assert t.lattice == "fcc" and t.r_cut == 5.5 and t.phi.K == nr - 1
    assert np.allclose(t.phi.y, 27.2 * 0.529 * Z[1:] ** 2 / r[1:], rtol=1e-15)
    assert np.allclose(t.rho.y, rho[1:], rtol=1e-15)


def test_long_grids_are_thinned(tmp_path):
    r, q, phi, rho, F = _cu_samples(nr=10001, dr=0.0006, nrho=10000, drho=0.0045)
    path = tmp_path / "long.eam.alloy"
    eamfile.write_setfl(path, F, rho, r * phi, 0.0045, 0.0006, 5.5, element="Cu")
    t = eamfile.read_eam(path)
    assert t.phi.K <= eamfile.MAX_SAMPLES and t.emb.K <= eamfile.MAX_SAMPLES
    assert t.phi.h == 2 * 0.0006 and t.emb.h == 2 * 0.0045
    assert np.allclose(t.phi.y, phi[1::2], rtol=1e-15)


def test_malformed_files(tmp_path):
    p2 = tmp_path / "two.eam.alloy"
    p2.write_text("a\nb\nc\n2 Cu Ni\n10 0.1 10 0.1 5.0\n")
    with pytest.raises(ValueError):
        eamfile.read_eam(p2)
    r, q, phi, rho, F = _cu_samples(nr=100, nrho=100)
    p3 = tmp_path / "short.eam.alloy"
    eamfile.write_setfl(p3, F, rho, r * phi, 0.015, 0.002, 0.19, element="Cu")
    text = p3.read_text().split("\n")
    p3.write_text("\n".join(text[:-10]))
    with pytest.raises(ValueError):
        eamfile.read_eam(p3)
