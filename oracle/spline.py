"""Uniform cubic B-splines, written from the definition (oracle; test infrastructure only).

A tabulated potential (Sec. 3.3: EAM loaded from a table) is represented as a
uniform cubic B-spline on K breakpoints x_k = x_lo + k h, k = 0..K-1, with K + 2
coefficients c_0..c_{K+1}.  On interval i (x_i <= x < x_{i+1}), t = (x - x_i)/h:

    s(x) = c_i b0(t) + c_{i+1} b1(t) + c_{i+2} b2(t) + c_{i+3} b3(t)
    b0 = (1-t)^3/6, b1 = (3t^3 - 6t^2 + 4)/6, b2 = (-3t^3 + 3t^2 + 3t + 1)/6, b3 = t^3/6.

The coefficients interpolate the table values at every breakpoint and match
the end slopes (complete/clamped cubic interpolation):

    (c_k + 4 c_{k+1} + c_{k+2}) / 6 = y_k,     k = 0..K-1
    (c_2 - c_0) / (2h) = y'(x_lo),   (c_{K+1} - c_{K-1}) / (2h) = y'(x_hi).

Outside [x_lo, x_{K-1}] the end interval's polynomial is used and the point is
reported as out of range.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_banded


def fit_clamped(y: np.ndarray, dy_lo: float, dy_hi: float, h: float) -> np.ndarray:
    """Coefficients c[0..K+1] of the clamped interpolating uniform cubic B-spline."""
    y = np.asarray(y, np.float64)
    K = y.shape[0]
    n = K + 2
    # Banded storage for solve_banded with (l, u) = (2, 2): ab[2 + r - col, col] = A[r, col].
    ab = np.zeros((5, n))
    rhs = np.zeros(n)
    # row 0: -c0 + c2 = 2 h y'_lo
    ab[2 + 0 - 0, 0] = -1.0
    ab[2 + 0 - 2, 2] = 1.0
    rhs[0] = 2.0 * h * dy_lo
    # rows 1..K: c_{r-1} + 4 c_r + c_{r+1} = 6 y_{r-1}
    for r in range(1, K + 1):
        ab[2 + 1, r - 1] = 1.0
        ab[2 + 0, r] = 4.0
        ab[2 - 1, r + 1] = 1.0
        rhs[r] = 6.0 * y[r - 1]
    # row K+1: -c_{K-1} + c_{K+1} = 2 h y'_hi
    r = K + 1
    ab[2 + 2, K - 1] = -1.0
    ab[2 + 0, K + 1] = 1.0
    rhs[r] = 2.0 * h * dy_hi
    return solve_banded((2, 2), ab, rhs)


def fit_table(tf) -> np.ndarray:
    """Fit a mdinputs.TabulatedFunction."""
    return fit_clamped(tf.y, tf.dy_lo, tf.dy_hi, tf.h)


def _interval(c: np.ndarray, x_lo: float, h: float, x):
    K = c.shape[0] - 2
    u = (np.asarray(x, np.float64) - x_lo) / h
    fl = np.floor(u)
    i = np.clip(fl, 0, K - 2).astype(np.int64)
    t = u - i
    oor = (u < 0.0) | (u > K - 1)
    return i, t, oor


def basis(t):
    s = 1.0 - t
    return np.stack([s ** 3 / 6.0, (3 * t ** 3 - 6 * t ** 2 + 4) / 6.0,
                     (-3 * t ** 3 + 3 * t ** 2 + 3 * t + 1) / 6.0, t ** 3 / 6.0], axis=-1)


def basis_d1(t):
    """d b_m / dt."""
    s = 1.0 - t
    return np.stack([-0.5 * s ** 2, (3 * t ** 2 - 4 * t) / 2.0, (-3 * t ** 2 + 2 * t + 1) / 2.0,
                     0.5 * t ** 2], axis=-1)


def basis_d2(t):
    """d^2 b_m / dt^2."""
    return np.stack([1.0 - t, 3 * t - 2.0, 1.0 - 3 * t, t], axis=-1)


def evaluate(c: np.ndarray, x_lo: float, h: float, x, deriv: int = 0):
    """s(x), s'(x) or s''(x); returns (values, out_of_range_mask)."""
    i, t, oor = _interval(c, x_lo, h, x)
    B = (basis, basis_d1, basis_d2)[deriv](t) / h ** deriv
    idx = i[..., None] + np.arange(4)
    return np.sum(c[idx] * B, axis=-1), oor


def basis_weights(c_len: int, x_lo: float, h: float, x, deriv: int = 0):
    """For each x the 4 coefficient indices it touches and the basis weights
    d^deriv beta_k(x)/dx^deriv on them (the derivative of s with respect to c_k)."""
    K = c_len - 2
    u = (np.asarray(x, np.float64) - x_lo) / h
    i = np.clip(np.floor(u), 0, K - 2).astype(np.int64)
    t = u - i
    B = (basis, basis_d1, basis_d2)[deriv](t) / h ** deriv
    return i[..., None] + np.arange(4), B
