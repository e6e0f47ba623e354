"""Pins of the oracle's uniform cubic B-spline (fit and evaluation)."""
import numpy as np
import pytest
from scipy.interpolate import make_interp_spline

import mdinputs as mi
from oracle import core
from oracle import spline as sp


def _tables():
    return [("cu", mi.tabulate_eam(mi.EAM_CU)), ("al", mi.tabulate_eam(mi.EAM_AL)),
            ("fm", mi.force_matching_tables())]


@pytest.mark.parametrize("name,tab", _tables())
def test_fit_equals_scipy_clamped_interpolant(name, tab):
    """The clamped interpolating cubic is unique; scipy builds it in another basis."""
    rng = np.random.default_rng(1)
    for tf in (tab.phi, tab.rho, tab.emb):
        c = sp.fit_table(tf)
        x = tf.x_lo + tf.h * np.arange(tf.K)
        ref = make_interp_spline(x, tf.y, k=3, bc_type=([(1, tf.dy_lo)], [(1, tf.dy_hi)]))
        xs = rng.uniform(tf.x_lo, tf.x_hi, 4000)
        for d in range(3):
            got = sp.evaluate(c, tf.x_lo, tf.h, xs, d)[0]
            want = ref(xs, d)
            scale = np.max(np.abs(want)) + 1e-300
            # s'' = (c_i - 2 c_{i+1} + c_{i+2}) / h^2 amplifies coefficient rounding by
            # ~|c| / (h^2 max|s''|): the tolerance grows with the derivative order.
            tol = (1e-13, 1e-11, 1e-8)[d]
            assert np.max(np.abs(got - want)) / scale < tol, (name, d)


def test_interpolation_conditions_exact():
    tf = mi.tabulate_eam(mi.EAM_CU).rho
    c = sp.fit_table(tf)
    x = tf.x_lo + tf.h * np.arange(tf.K)
    v = sp.evaluate(c, tf.x_lo, tf.h, x, 0)[0]
    assert np.max(np.abs(v - tf.y) / np.abs(tf.y)) < 1e-14
    d = sp.evaluate(c, tf.x_lo, tf.h, np.array([tf.x_lo, x[-1]]), 1)[0]
    assert abs(d[0] - tf.dy_lo) < 1e-11 * abs(tf.dy_lo) and abs(d[1] - tf.dy_hi) < 1e-9


def test_spline_vs_analytic_within_interpolation_bound():
    """Cubic interpolation error (5/384) h^4 max|f''''|: ~1e-10 relative for phi, rho on
    the 2000-point grid and ~2e-9 for F near rhobar = 1."""
    p = mi.EAM_CU
    tab = mi.tabulate_eam(p)
    xs = np.linspace(1.0, p.r_cut, 20011)[:-1]
    phi = p.A * np.exp(-p.alpha * (xs / p.r0 - 1))
    rho = np.exp(-p.beta * (xs / p.r0 - 1))
    for tf, f in ((tab.phi, phi), (tab.rho, rho)):
        c = sp.fit_table(tf)
        v = sp.evaluate(c, tf.x_lo, tf.h, xs, 0)[0]
        assert np.max(np.abs(v - f) / np.abs(f)) < 1e-9
    q = np.linspace(1.0, 41.0, 20011)
    c = sp.fit_table(tab.emb)
    v = sp.evaluate(c, tab.emb.x_lo, tab.emb.h, q, 0)[0]
    assert np.max(np.abs(v + np.sqrt(q))) < 5e-9
    d1 = sp.evaluate(c, tab.emb.x_lo, tab.emb.h, q[q > 4], 1)[0]
    assert np.max(np.abs(d1 + 0.5 / np.sqrt(q[q > 4]))) < 1e-8


def test_c_evaluator_equals_numpy_definition():
    tab = mi.tabulate_eam(mi.EAM_CU)
    f = core.SplineFunc.from_table(tab.phi)
    x = np.random.default_rng(2).uniform(1.0, 5.5, 1000)
    v, d1, d2, oor = core.eval_func(f, x)
    assert oor == 0
    for d, got in enumerate((v, d1, d2)):
        want = sp.evaluate(f.c, f.x_lo, f.h, x, d)[0]
        # same definition, different operation order: rounding grows with the order
        assert np.max(np.abs(got - want)) <= (1e-14, 1e-12, 1e-9)[d] * np.max(np.abs(want))


def test_out_of_range_flag_and_end_polynomial():
    tab = mi.tabulate_eam(mi.EAM_CU)
    f = core.SplineFunc.from_table(tab.emb)
    v, d1, d2, oor = core.eval_func(f, np.array([0.5, 1.0, 41.0, 45.0]))
    assert oor == 2
    # below the range the first interval's cubic is continued
    i, t, _ = sp._interval(f.c, f.x_lo, f.h, np.array([0.5]))
    assert i[0] == 0 and t[0] < 0


def test_basis_partition_of_unity_and_weights():
    t = np.linspace(0, 1, 101)
    assert np.allclose(sp.basis(t).sum(-1), 1.0, atol=1e-15)
    assert np.allclose(sp.basis_d1(t).sum(-1), 0.0, atol=1e-15)
    assert np.allclose(sp.basis_d2(t).sum(-1), 0.0, atol=1e-15)
    # derivative with respect to a coefficient equals the basis function (linearity)
    tf = mi.force_matching_tables().rho
    c = sp.fit_table(tf)
    x = np.array([2.0, 3.3, 4.9])
    idx, W = sp.basis_weights(c.shape[0], tf.x_lo, tf.h, x, 0)
    for k in range(c.shape[0]):
        e = np.zeros_like(c)
        e[k] = 1.0
        want = sp.evaluate(e, tf.x_lo, tf.h, x, 0)[0]
        got = np.where(idx == k, W, 0.0).sum(-1)
        assert np.allclose(got, want, atol=1e-15)
