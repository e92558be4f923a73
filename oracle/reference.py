"""End-to-end oracle: x = A^-1 b and diag(A^-1) for one problem.

Test infrastructure only (see ``oracle/__init__``).

Paper, Sect. 2.4.1: ``A = H^T Sigma^-2 H``, ``b = H^T Sigma^-2 y``,
``x = A^-1 b`` and ``Var(x_i) ~ (A^-1)_ii``.  Tiny problems use the dense
factorisation of :mod:`oracle.dense`; larger ones the two-block factorisation
of :mod:`oracle.blockchol`.  Optionally the solution is certified by
refinement with long-double residuals formed from H (:mod:`oracle.certify`).
"""
from __future__ import annotations

import numpy as np

from .normal_eq import normal_equations
from .dense import cholesky, forward_subst, backward_subst, diag_inv_colnorms
from .blockchol import BlockCholesky
from .certify import refine_solution, refine_inverse_column

DENSE_MAX = 1500


class _DenseFactor:
    def __init__(self, A):
        self.L = cholesky(A)

    def solve(self, b):
        return backward_subst(self.L, forward_subst(self.L, b))

    def diag_inv(self, idx=None):
        d = diag_inv_colnorms(self.L)
        return d if idx is None else d[np.asarray(idx)]


def factor_problem(prob, force_block: bool = False):
    A, b = normal_equations(prob.rowptr, prob.col, prob.val, prob.w, prob.y,
                            prob.n)
    if prob.n <= DENSE_MAX and not force_block:
        f = _DenseFactor(A.toarray())
    else:
        f = BlockCholesky(A, prob.n_bg)
    return A, b, f


def oracle_solve(prob, diag_idx=None, want_diag: bool = True,
                 refine_steps: int = 2, certify_diag: bool = False,
                 force_block: bool = False):
    """Returns a dict with ``x``, ``diag`` (for ``diag_idx``, all if None),
    ``A`` (scipy CSR), ``b`` and the factor object."""
    A, b, f = factor_problem(prob, force_block)
    x = f.solve(b)
    if refine_steps:
        x = refine_solution(prob, f.solve, x, refine_steps).astype(np.float64)
    out = {"x": x, "A": A, "b": b, "factor": f}
    if want_diag:
        idx = np.arange(prob.n) if diag_idx is None else np.asarray(diag_idx)
        if certify_diag:
            d = np.array([float(refine_inverse_column(prob, f.solve, int(j))[j])
                          for j in idx])
        else:
            d = f.diag_inv(idx)
        out["diag"] = d
        out["diag_idx"] = idx
    return out
