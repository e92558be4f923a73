"""Symmetric indefinite normal matrices (oracle).

Test infrastructure only (see ``oracle/__init__``).

With weights of either sign, ``A = H^T W H`` is symmetric but may be
indefinite.  Sect. 5 reports that the SPI matrices are numerically
indefinite and need two-by-two pivots, and Sect. 3.2.2 and Sect. 4.3 that
the factorisation must pivot to stay accurate.  What is computed does not
change: ``x`` solves ``A x = b`` and the variances are the diagonal entries
of ``A^-1`` (Sect. 2.4.1).  Both have plain definitions, which this module
writes out: ``A`` assembled densely from its definition
(:func:`oracle.normal_eq.normal_equations`), a general LU factorisation with
row pivoting (LAPACK ``getrf`` through scipy, a library step that assumes
no symmetry or definiteness) as the float64 solver, and iterative
refinement with long-double residuals formed from ``H`` itself
(:mod:`oracle.certify`), for ``x`` and for every column of ``A^-1`` whose
diagonal entry is asked for.  The pivot order any factorisation chooses does
not enter: ``x`` and ``diag(A^-1)`` are unique for a nonsingular ``A``.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .certify import refine_solution, refine_inverse_column
from .normal_eq import normal_equations


class _LU:
    """float64 solves with an LU factorisation of the dense matrix."""

    def __init__(self, A):
        self.lu = sla.lu_factor(A, check_finite=True)

    def solve(self, r):
        return sla.lu_solve(self.lu, np.asarray(r, dtype=np.float64))


def indefinite_solve(prob, diag_idx=None, want_diag: bool = True,
                     refine_steps: int = 3):
    """``x = A^-1 b`` and ``diag(A^-1)`` (entries ``diag_idx``, all if None)
    for ``A = H^T W H`` with weights of either sign.

    Returns a dict with ``x``, ``diag``, ``diag_idx``, ``A`` (dense) and
    ``b``.  Dense: meant for test sizes (a few thousand unknowns at most).
    """
    As, b = normal_equations(prob.rowptr, prob.col, prob.val, prob.w, prob.y,
                             prob.n)
    A = As.toarray()
    f = _LU(A)
    x = refine_solution(prob, f.solve, f.solve(b), refine_steps).astype(np.float64)
    out = {"x": x, "A": A, "b": np.asarray(b, dtype=np.float64)}
    if want_diag:
        idx = np.arange(prob.n) if diag_idx is None else np.asarray(diag_idx)
        out["diag"] = np.array([
            float(refine_inverse_column(prob, f.solve, int(j), refine_steps)[j])
            for j in idx])
        out["diag_idx"] = idx
    return out
