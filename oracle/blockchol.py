"""Two-block Cholesky of the normal matrix (oracle, medium/large cases).

Test infrastructure only (see ``oracle/__init__``).

The unknowns are split as in the paper's expanded transfer matrix, Sect.
2.2.3 (``H(1:M, 1:K0)`` background, the rest sky): ``A = [[A_bb, A_sb^T],
[A_sb, A_ss]]`` with the first ``n_b`` (background) unknowns eliminated
first.  This is the oracle's *own* ordering (background first, then the
remaining unknowns in their natural order); it need not match the ordering
the product chooses.

Factorisation ``A = L L^T`` (Sect. 3.2.2 with D folded into L):
``L_bb = chol(A_bb)``, ``L_sb = A_sb L_bb^-T``, and the remaining block is the
Cholesky factor of the Schur complement ``S = A_ss - L_sb L_sb^T``.

Solution (Sect. 3.2.3): forward ``z = L^-1 b`` then backward ``x = L^-T z``.

The product ``L_sb L_sb^T`` is taken with a sparse product, or with a dense
BLAS product of the same formula when ``L_sb`` is more than 10% dense (wide
fields of view: the sparse product is then about 100 times slower).

Variances (Sect. 2.4.1) ``(A^-1)_ii = ||L^-1 e_i||^2`` (the left-looking
formula of Sect. 4.3 with D = I).  Column i of ``L^-1`` is
``[u; -L_ss^-1 L_sb u]`` with ``u = L_bb^-1 e_i`` for a background unknown
and ``[0; L_ss^-1 e_i']`` for a sky unknown.  Requested entries are computed
in blocks of right-hand sides (128 at a time, as in Sect. 3.3.1 / Table 6).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


class BlockCholesky:
    # L_sb is kept dense above this fraction of structural non-zeros
    DENSE_FRACTION = 0.1

    def __init__(self, A, n_b: int):
        A = sp.csr_matrix(A)
        n = A.shape[0]
        self.n, self.n_b = n, n_b
        Abb = A[:n_b, :n_b].tocsr()
        Asb = A[n_b:, :n_b].tocsc()
        Ass = A[n_b:, n_b:]
        off = Abb - sp.diags(Abb.diagonal())
        self.bb_diagonal = off.count_nonzero() == 0
        if n_b == 0:
            self.Lbb = np.zeros((0, 0))
            self.Lsb = sp.csr_matrix((n - n_b, 0))
        elif self.bb_diagonal:
            d = Abb.diagonal()
            if np.any(~(d > 0)):
                raise ValueError("background block not positive definite")
            self.Lbb = np.sqrt(d)                       # diagonal factor
            self.Lsb = (Asb @ sp.diags(1.0 / self.Lbb)).tocsr()
            if self.Lsb.nnz > self.DENSE_FRACTION * max(
                    1, self.Lsb.shape[0] * self.Lsb.shape[1]):
                self.Lsb = self.Lsb.toarray()           # dense products below
        else:
            self.Lbb = np.linalg.cholesky(Abb.toarray())
            self.Lsb = sp.csr_matrix(
                sla.solve_triangular(self.Lbb, Asb.toarray().T, lower=True).T)
        S = Ass.toarray()
        if n_b:
            LLt = self.Lsb @ self.Lsb.T
            S -= LLt.toarray() if sp.issparse(LLt) else LLt
        self.Lss = np.linalg.cholesky(S)

    # -- triangular solves with the block factor ------------------------------
    def _lbb_solve(self, v, trans=False):
        if self.n_b == 0:
            return v
        if self.bb_diagonal:
            return v / (self.Lbb[:, None] if v.ndim == 2 else self.Lbb)
        return sla.solve_triangular(self.Lbb, v, lower=True,
                                    trans="T" if trans else "N")

    def forward(self, b):
        """z = L^-1 b."""
        b = np.asarray(b, dtype=np.float64)
        zb = self._lbb_solve(b[:self.n_b])
        zs = sla.solve_triangular(self.Lss, b[self.n_b:] - self.Lsb @ zb,
                                  lower=True)
        return np.concatenate([zb, zs])

    def backward(self, z):
        """x = L^-T z."""
        zb, zs = z[:self.n_b], z[self.n_b:]
        xs = sla.solve_triangular(self.Lss, zs, lower=True, trans="T")
        xb = self._lbb_solve(zb - self.Lsb.T @ xs, trans=True)
        return np.concatenate([xb, xs])

    def solve(self, b):
        return self.backward(self.forward(b))

    # -- variances -------------------------------------------------------------
    def diag_inv(self, idx=None, block: int = 128):
        """``(A^-1)_ii`` for the requested unknowns (all by default)."""
        idx = np.arange(self.n) if idx is None else np.asarray(idx)
        out = np.empty(len(idx))
        nb, ns = self.n_b, self.n - self.n_b
        for k0 in range(0, len(idx), block):
            sel = idx[k0:k0 + block]
            E = np.zeros((self.n, len(sel)))
            E[sel, np.arange(len(sel))] = 1.0
            U = self._lbb_solve(E[:nb])                    # L_bb^-1 part
            # L_sb U with U taken as sparse when L_sb is (U has at most one
            # non-zero per column on the diagonal branch)
            LU = self.Lsb @ (sp.csc_matrix(U) if sp.issparse(self.Lsb) else U)
            LU = LU.toarray() if sp.issparse(LU) else LU
            V = sla.solve_triangular(self.Lss, E[nb:] - LU,
                                     lower=True)          # L_ss^-1 part
            out[k0:k0 + block] = (U * U).sum(axis=0) + (V * V).sum(axis=0)
            del E
        return out

    # -- general entries of A^-1 (covariances) -------------------------------
    def inverse_entries(self, rows, cols, block: int = 128):
        """``(A^-1)_ij`` for the pairs (rows[k], cols[k]): column j of A^-1
        solves A z = e_j (forward then backward substitution with the block
        factor, Sect. 3.3.1), taken for up to ``block`` distinct columns at a
        time (blocked right-hand sides, Sect. 4.3)."""
        rows = np.asarray(rows)
        cols = np.asarray(cols)
        out = np.empty(len(rows))
        uniq = np.unique(cols)
        for k0 in range(0, len(uniq), block):
            sel = uniq[k0:k0 + block]
            E = np.zeros((self.n, len(sel)))
            E[sel, np.arange(len(sel))] = 1.0
            Z = self.solve(E)
            where = {int(c): q for q, c in enumerate(sel)}
            for k in np.nonzero(np.isin(cols, sel))[0]:
                out[k] = Z[rows[k], where[int(cols[k])]]
        return out
