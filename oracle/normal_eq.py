"""Normal equations of the weighted least-squares problem (oracle).

Test infrastructure only (see ``oracle/__init__``).

Paper, Sect. 2.4.1: minimising chi^2 = sum_i ((y_i - sum_j h_ij x_j)/sigma_i)^2
gives ``(H^T [Sigma^-2] H) x = H^T [Sigma^-2] y``, i.e. ``A x = b`` with
``A_ij = sum_r h_ri w_r h_rj`` and ``b_i = sum_r h_ri w_r y_r`` where
``w_r = sigma_r^-2``.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def normal_equations_bruteforce(rowptr, col, val, w, y, n):
    """The definition written out with Python loops (tiny inputs only).

    Returns dense ``A`` (n x n) and ``b`` (n).
    """
    A = np.zeros((n, n))
    b = np.zeros(n)
    m = len(rowptr) - 1
    for r in range(m):
        lo, hi = int(rowptr[r]), int(rowptr[r + 1])
        for p in range(lo, hi):
            i = int(col[p])
            b[i] += val[p] * w[r] * y[r]
            for q in range(lo, hi):
                j = int(col[q])
                A[i, j] += val[p] * w[r] * val[q]
    return A, b


def normal_equations(rowptr, col, val, w, y, n):
    """``A = H^T diag(w) H`` (scipy CSR, both triangles) and ``b = H^T (w*y)``.

    The sparse matrix product is the library primitive for the sum over rows.
    """
    m = len(rowptr) - 1
    H = sp.csr_matrix((np.asarray(val, dtype=np.float64),
                       np.asarray(col), np.asarray(rowptr)), shape=(m, n))
    w = np.asarray(w, dtype=np.float64)
    A = (H.T @ sp.diags(w) @ H).tocsr()
    A.sort_indices()
    b = H.T @ (w * np.asarray(y, dtype=np.float64))
    return A, np.asarray(b).ravel()
