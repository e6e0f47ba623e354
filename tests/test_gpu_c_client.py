"""The C ABI from plain C: tests/c_client/lj_nve.c (a C program with no Python or torch in
its process, using only include/md.h and the HIP runtime's memory API) runs LJ argon 256
atoms for 100 velocity-Verlet steps with threshold rebuilds; its positions, velocities and
per-step energies follow the oracle integrator (1e-9 A, 1e-8 A/ps, 1e-10 relative).
"""
import os
import struct
import subprocess

import numpy as np
import pytest

import mdinputs as mi
from oracle import integrate

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_client", "lj_nve")


def test_c_client_lj_nve_matches_oracle(tmp_path):
    assert os.path.exists(EXE), "the C client is not built (__graft_entry__.build())"
    s = mi.lj_argon()
    assert tuple(s.box.lo) == (0.0, 0.0, 0.0) and all(s.box.periodic)
    n, steps = len(s.pos), 100
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(inp, "wb") as f:
        f.write(struct.pack("<i", n))
        f.write(np.array(list(s.box.len) + [s.lj.eps, s.lj.sigma, s.lj.r_cut, s.skin, s.mass,
                                            s.dt_ps], np.float64).tobytes())
        f.write(np.ascontiguousarray(s.pos, np.float64).tobytes())
        f.write(np.ascontiguousarray(s.vel, np.float64).tobytes())
    print("C client:", EXE, n, "atoms", steps, "steps", flush=True)
    r = subprocess.run([EXE, str(inp), str(out), str(steps)], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    raw = open(out, "rb").read()
    assert len(raw) == 16 * (steps + 1) + 48 * n + 16
    rec = np.frombuffer(raw, np.float64, 2 * (steps + 1)).reshape(steps + 1, 2)
    off = 16 * (steps + 1)
    x = np.frombuffer(raw, np.float64, 3 * n, off).reshape(n, 3)
    v = np.frombuffer(raw, np.float64, 3 * n, off + 24 * n).reshape(n, 3)
    status, step, rebuilds, longest = np.frombuffer(raw, np.int32, 4, off + 48 * n)
    assert status == 0 and step == steps and rebuilds >= 2 and 0 < longest <= 128
    xo, vo, _, hist = integrate.run_nve(s.pos, s.vel, s.box, s.mass, s.dt_ps, steps,
                                        integrate.lj_force_fn(s.box, s.lj))
    d = x - xo
    L = np.array(s.box.len)
    d -= L * np.rint(d / L)
    assert np.max(np.abs(d)) < 1e-9
    assert np.max(np.abs(v - vo)) < 1e-8
    assert np.max(np.abs(rec[:, 0] - hist[:, 1])) < 1e-10 * abs(hist[0, 1])
    assert np.max(np.abs(rec[:, 1] - hist[:, 2])) < 1e-10 * abs(hist[0, 2])
