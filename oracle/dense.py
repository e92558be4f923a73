"""Dense Cholesky, substitutions and inverse entries (oracle, tiny cases).

Test infrastructure only (see ``oracle/__init__``).

* Factorisation ``A = L L^T`` (Sect. 3.2: a symmetric matrix is factored into
  triangular factors; the paper uses ``L D L^T``, here D is folded into L,
  which gives the same x and the same entries of A^-1 in exact arithmetic).
* Solution by forward substitution ``z = L^-1 b`` then backward substitution
  ``x = L^-T z`` (Sect. 3.2.3).
* ``(A^-1)_ii = sum_k (L^-1)_ki^2`` (Sect. 4.3, the left-looking formula
  with d_kk = 1), computed one column of ``L^-T`` (row of ``L^-1``) at a time.
* A single entry ``(A^-1)_ij = (A^-1 e_j)_i`` with the forward solve on the
  sparse right-hand side e_j restricted to the path j -> root and the
  backward solve restricted to the path root -> i (Sect. 3.3.1).
"""
from __future__ import annotations

import numpy as np

from .etree import ancestors


def cholesky(A):
    """Right-looking column Cholesky ``A = L L^T`` in float64 (own loop).

    Raises ``ValueError`` at the first non-positive pivot.
    """
    A = np.array(A, dtype=np.float64, copy=True)
    n = A.shape[0]
    L = np.zeros_like(A)
    for k in range(n):
        d = A[k, k]
        if not d > 0.0:
            raise ValueError(f"matrix not positive definite at column {k}")
        lkk = np.sqrt(d)
        L[k, k] = lkk
        col = A[k + 1:, k] / lkk
        L[k + 1:, k] = col
        # Schur complement update of the trailing block (both triangles)
        A[k + 1:, k + 1:] -= np.outer(col, col)
    return L


def forward_subst(L, b):
    """Solve ``L z = b`` (L lower triangular)."""
    L = np.asarray(L)
    b = np.array(b, dtype=np.float64, copy=True)
    n = L.shape[0]
    z = np.zeros_like(b)
    for i in range(n):
        z[i] = (b[i] - L[i, :i] @ z[:i]) / L[i, i]
    return z


def backward_subst(L, z):
    """Solve ``L^T x = z`` (L lower triangular)."""
    L = np.asarray(L)
    z = np.asarray(z, dtype=np.float64)
    n = L.shape[0]
    x = np.zeros_like(z)
    for i in range(n - 1, -1, -1):
        x[i] = (z[i] - L[i + 1:, i] @ x[i + 1:]) / L[i, i]
    return x


def solve_dense(A, b):
    L = cholesky(A)
    return backward_subst(L, forward_subst(L, b)), L


def inverse_from_cholesky(L):
    """Full ``A^-1 = L^-T L^-1``; column j solves ``A z = e_j``."""
    n = L.shape[0]
    Z = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        Z[:, j] = backward_subst(L, forward_subst(L, e))
    return Z


def diag_inv_colnorms(L):
    """``(A^-1)_ii = sum_k (L^-1)_ki^2`` (Sect. 4.3 with D = I)."""
    n = L.shape[0]
    out = np.zeros(n)
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        col = forward_subst(L, e)       # column i of L^-1
        out[i] = col @ col
    return out


def selected_entry_pruned(L, parent, i, j):
    """``(A^-1)_ij`` with the two pruned traversals of Sect. 3.3.1.

    ``parent`` is the elimination tree of L (parent[v] = -1 at the root).
    Forward: ``L z = e_j``; z is non-zero only on j and its ancestors, so
    only those nodes are visited, in bottom-up order.  Backward: component i
    of ``L^-T z`` depends only on the components of i's ancestors, so the
    solve runs top-down along the path root -> i.  Returns (value, visited
    forward nodes, visited backward nodes).
    """
    L = np.asarray(L)
    fwd = [j] + ancestors(parent, j)
    z = {}
    for v in fwd:                       # bottom-up along j -> root
        s = 1.0 if v == j else 0.0
        for u, zu in z.items():
            s -= L[v, u] * zu
        z[v] = s / L[v, v]
    bwd = list(reversed([i] + ancestors(parent, i)))
    x = {}
    for v in bwd:                       # top-down along root -> i
        s = z.get(v, 0.0)
        for u, xu in x.items():
            s -= L[u, v] * xu
        x[v] = s / L[v, v]
    return x[i], fwd, bwd
