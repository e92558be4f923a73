"""Certification of oracle results with extended-precision residuals.

Test infrastructure only (see ``oracle/__init__``).

The quantities of Sect. 2.4.1 are defined for the exact normal matrix
``A = H^T W H`` of the given float64 inputs.  An assembled float64 ``A``
already carries rounding, so the residual here is formed from ``H`` directly,
``r = H^T W (y - H x)``, with every product and sum in ``np.longdouble``
(64-bit significand on x86).  A few steps of iterative refinement with a
float64 factorisation then converge to the solution of the exact problem up
to a tiny multiple of the extended unit roundoff.
"""
from __future__ import annotations

import numpy as np

LD = np.longdouble


def _rows(rowptr):
    return np.repeat(np.arange(len(rowptr) - 1), np.diff(rowptr))


def normal_residual_ld(rowptr, col, val, w, y, x):
    """``H^T W (y - H x)`` evaluated in long double (returned as long double)."""
    rows = _rows(rowptr)
    m = len(rowptr) - 1
    n = len(x)
    v = np.asarray(val).astype(LD)
    hx = np.zeros(m, dtype=LD)
    np.add.at(hx, rows, v * np.asarray(x).astype(LD)[col])
    t = np.asarray(w).astype(LD) * (np.asarray(y).astype(LD) - hx)
    r = np.zeros(n, dtype=LD)
    np.add.at(r, col, v * t[rows])
    return r


def apply_normal_ld(rowptr, col, val, w, z):
    """``H^T W H z`` in long double."""
    rows = _rows(rowptr)
    m = len(rowptr) - 1
    v = np.asarray(val).astype(LD)
    hz = np.zeros(m, dtype=LD)
    np.add.at(hz, rows, v * np.asarray(z).astype(LD)[col])
    t = np.asarray(w).astype(LD) * hz
    r = np.zeros(len(z), dtype=LD)
    np.add.at(r, col, v * t[rows])
    return r


def refine_solution(prob, solve, x0, steps: int = 3, residual=None):
    """Refine ``x`` for ``H^T W H x = H^T W y``; ``solve`` is a float64 solver.

    ``residual`` (default :func:`normal_residual_ld`) takes the arguments of
    that function; the pins substitute deliberately wrong variants of it."""
    res = normal_residual_ld if residual is None else residual
    x = np.asarray(x0).astype(LD)
    for _ in range(steps):
        r = res(prob.rowptr, prob.col, prob.val, prob.w, prob.y, x)
        x = x + np.asarray(solve(r.astype(np.float64))).astype(LD)
    return x


def refine_inverse_column(prob, solve, j: int, steps: int = 3):
    """Column j of ``A^-1`` (``A z = e_j``) refined with long-double residuals."""
    n = prob.n
    e = np.zeros(n, dtype=LD)
    e[j] = 1
    z = np.asarray(solve(e.astype(np.float64))).astype(LD)
    for _ in range(steps):
        r = e - apply_normal_ld(prob.rowptr, prob.col, prob.val, prob.w, z)
        z = z + np.asarray(solve(r.astype(np.float64))).astype(LD)
    return z
