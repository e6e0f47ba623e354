"""Pins of the oracle's Langevin thermostat (oracle/thermostat.py).

  Philox4x32-10          the published known-answer vectors (tests/golden)
  Box-Muller normals     moments, tail masses and independence of the draws
  O update, T = 0        v_n - u = exp(-gamma n dt) (v_0 - u) exactly (free particles)
  O update, one step     from rest: mean (1 - c1) u, variance (1 - c1^2) k_B T / m
  gamma = 0              the thermostat step reduces to plain velocity Verlet
  regions                first matching slab wins; atoms outside keep NVE
  NVT                    a 256-atom LJ crystal relaxes to the target temperature
"""
import json
import math
import os

import numpy as np
import pytest

import mdinputs as mi
from oracle import integrate, thermostat as th

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.json")) as f:
        kat = json.load(f)["vectors"]
    for v in kat:
        ctr = [int(x, 16) for x in v["ctr"]]
        key = [int(x, 16) for x in v["key"]]
        out = [int(x) for x in th.philox4x32_10(ctr, key)]
        assert out == [int(x, 16) for x in v["out"]]


def test_philox_vectorised_equals_single():
    rng = np.random.default_rng(5)
    ctr = rng.integers(0, 2 ** 32, size=(50, 4), dtype=np.uint64)
    key = rng.integers(0, 2 ** 32, size=(50, 2), dtype=np.uint64)
    batch = th.philox4x32_10(ctr, key)
    for i in range(50):
        assert np.array_equal(batch[i], th.philox4x32_10(ctr[i], key[i]))


def test_normals_moments_and_tails():
    z = th.normals(20251202, 3, np.arange(300000))
    n = z.size
    assert np.all(np.isfinite(z))
    # mean 0 (sd 1/sqrt(n) per component), variance 1 (sd sqrt(2/n))
    assert np.abs(z.mean(axis=0)).max() < 5.0 / math.sqrt(n / 3)
    assert np.abs(z.var(axis=0) - 1.0).max() < 5.0 * math.sqrt(2.0 / (n / 3))
    # tail masses of the standard normal: P(|z| < 1) = 0.682689, P(|z| < 2) = 0.954500
    for a, p in ((1.0, 0.6826894921), (2.0, 0.9544997361)):
        frac = np.mean(np.abs(z) < a)
        assert abs(frac - p) < 5.0 * math.sqrt(p * (1 - p) / n)
    # components, neighbouring ids and consecutive steps are uncorrelated
    c = np.corrcoef(z.T)
    assert np.abs(c[np.triu_indices(3, 1)]).max() < 0.01
    z2 = th.normals(20251202, 4, np.arange(300000))
    assert abs(np.corrcoef(z[:, 0], z2[:, 0])[0, 1]) < 0.01
    assert abs(np.corrcoef(z[:-1, 0], z[1:, 0])[0, 1]) < 0.01
    # the seed's high word matters
    z3 = th.normals(20251202 + (1 << 32), 3, np.arange(1000))
    assert not np.allclose(z3, z[:1000])


def _free(n, seed=1):
    rng = np.random.default_rng(seed)
    box = mi.Box((0.0, 0.0, 0.0), (50.0, 50.0, 50.0), (1, 1, 1))
    x = rng.uniform(0.0, 50.0, (n, 3))
    v = rng.normal(0.0, 3.0, (n, 3))
    zero = lambda y: (np.zeros_like(y), 0.0)
    return box, x, v, zero


def test_zero_temperature_is_exponential_decay():
    box, x, v0, zero = _free(500)
    u = (1.0, -2.0, 0.5)
    lang = {"seed": 1, "axis": 2, "regions": [{"T": 0.0, "gamma": 3.0, "u": u}]}
    dt, n = 2e-3, 40
    _, v, _, _ = th.run_nvt(x, v0, np.arange(500), box, 39.948, dt, n, zero, lang)
    want = np.asarray(u) + math.exp(-3.0 * n * dt) * (v0 - np.asarray(u))
    assert np.allclose(v, want, rtol=0, atol=1e-13)


def test_one_update_has_the_ou_mean_and_variance():
    n, mass, T, gamma, dt = 200000, 26.98, 450.0, 40.0, 1e-3
    x = np.zeros((n, 3))
    v0 = np.zeros((n, 3))
    u = np.array([0.3, 0.0, -1.2])
    lang = {"seed": 77, "regions": [{"T": T, "gamma": gamma, "u": tuple(u)}]}
    v = th.o_step(x, v0, np.arange(n), 9, lang, mass, dt)
    c1 = math.exp(-gamma * dt)
    var = (1.0 - c1 * c1) * th.KB * T / mass * integrate.ACCEL
    assert np.abs(v.mean(axis=0) - (1.0 - c1) * u).max() < 5.0 * math.sqrt(var / n)
    assert np.abs(v.var(axis=0) / var - 1.0).max() < 5.0 * math.sqrt(2.0 / n)


def test_zero_friction_is_velocity_verlet():
    s = mi.lj_argon(cells=3)
    fn = integrate.lj_force_fn(s.box, s.lj)
    lang = {"seed": 3, "regions": [{"T": 500.0, "gamma": 0.0}]}
    ids = np.arange(s.pos.shape[0])
    xa, va, _, ha = th.run_nvt(s.pos, s.vel, ids, s.box, s.mass, s.dt_ps, 20, fn, lang)
    xb, vb, _, hb = integrate.run_nve(s.pos, s.vel, s.box, s.mass, s.dt_ps, 20, fn)
    assert np.allclose(xa, xb, rtol=0, atol=1e-11)
    assert np.allclose(va, vb, rtol=0, atol=1e-11)
    assert np.allclose(ha, hb, rtol=1e-12, atol=1e-12)


def test_regions_first_match_and_outside():
    n = 3000
    rng = np.random.default_rng(4)
    x = rng.uniform(0.0, 30.0, (n, 3))
    v = rng.normal(0.0, 1.0, (n, 3))
    lang = {"seed": 11, "axis": 1, "regions": [
        {"lo": 0.0, "hi": 10.0, "T": 0.0, "gamma": 1e9, "u": (1.0, 0.0, 0.0)},
        {"lo": 5.0, "hi": 20.0, "T": 0.0, "gamma": 1e9, "u": (0.0, 2.0, 0.0)}]}
    out = th.o_step(x, v, np.arange(n), 1, lang, 10.0, 1e-3)
    y = x[:, 1]
    a, b, c = y < 10.0, (y >= 10.0) & (y < 20.0), y >= 20.0
    assert np.allclose(out[a], [1.0, 0.0, 0.0], atol=1e-12)   # includes the overlap 5..10
    assert np.allclose(out[b], [0.0, 2.0, 0.0], atol=1e-12)
    assert np.array_equal(out[c], v[c])


@pytest.mark.parametrize("target", [60.0, 160.0])
def test_lj_crystal_relaxes_to_target_temperature(target):
    """256 Ar atoms from 100 K: the mean temperature over the second half of 1200
    steps (dt 2 fs, gamma 5/ps) is the target within 8 % (about 5 standard errors)."""
    s = mi.lj_argon(cells=4)
    n = s.pos.shape[0]
    fn = integrate.lj_force_fn(s.box, s.lj)
    lang = {"seed": 2024, "regions": [{"T": target, "gamma": 5.0}]}
    _, _, _, h = th.run_nvt(s.pos, s.vel, np.arange(n), s.box, s.mass, s.dt_ps, 1200, fn, lang)
    temps = 2.0 * h[:, 2] / ((3 * n - 3) * th.KB)
    assert abs(temps[600:].mean() / target - 1.0) < 0.08
