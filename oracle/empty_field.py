"""Empty-field (detector pattern) loop of App. A.4-A.5: oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Model (Sect. 2.2.3, background term B_dp = I^bg_p U^d t_dp): the
background column of row i = (pointing p, detector d) holds U_{u(i)} t_i,
where u(i) is the pattern unit of the row (its detector d, or with the
per-interval variant of App. A.4 the pair (d, interval of p)) and x_j of
that column is the background intensity I^bg of the time bin.  With the
solution x fixed, the counts due to the sources D^S_i are the sky part of
(H x)_i, and the pattern that minimises chi^2 for each unit is the closed
form U^LSQ (App. A.4):

    U^LSQ_u = sum_{i in u} (y_i - D^S_i) g_i / sigma_i^2
              / sum_{i in u} g_i^2 / sigma_i^2,      g_i = I_i t_i

with sigma_i^-2 = w_i; the likelihood version U^MLE_u = sum (y_i - D^S_i) /
sum g_i.  (The per-interval LSQ formula of App. A.4 prints (I t^2)^2 in its
denominator; it is read as (I t)^2, the same form as the whole-dataset
formula, of which it is the restriction to the interval.)

Algorithm 1 (App. A.5), as read here: starting from U_0, each pass
  (a) sets the background entries of H to U_u t_i,
  (b) solves the LSQ problem for x (normal equations, Sect. 2.4.1),
  (c) takes chi^2 = sum_i w_i (y_i - (H x)_i)^2 of that x and H,
  (d) updates U by the closed form from that x;
passes stop once chi^2 decreases by no more than rtol (relative) from the
previous pass, or after itermax passes.  The result is the last pass's x
with its U, and diag(A^-1) of that pass's A (the Hessian at the solution).
"""
from __future__ import annotations

import numpy as np

from .reference import oracle_solve


def row_parts(rowptr, col, val, x, bg_pos):
    """(e, s, I): e_i = (H x)_i, s_i = D^S_i (its sky part, the background
    entry left out), I_i = x at the row's background column (0 if none)."""
    m = len(rowptr) - 1
    e = np.zeros(m)
    s = np.zeros(m)
    I = np.zeros(m)
    for i in range(m):
        lo, hi = rowptr[i], rowptr[i + 1]
        prod = val[lo:hi] * x[col[lo:hi]]
        e[i] = prod.sum()
        b = bg_pos[i]
        if b >= 0:
            s[i] = e[i] - val[b] * x[col[b]]
            I[i] = x[col[b]]
        else:
            s[i] = e[i]
    return e, s, I


def pattern_update(rowptr, col, val, w, y, x, bg_pos, t, grp_ptr, grp_rows,
                   U_old, stat="lsq"):
    """Closed-form pattern of every unit (App. A.4) for the solution x."""
    _, s, I = row_parts(rowptr, col, val, x, bg_pos)
    U = np.array(U_old, dtype=np.float64, copy=True)
    for u in range(len(grp_ptr) - 1):
        rows = grp_rows[grp_ptr[u]:grp_ptr[u + 1]]
        rows = rows[bg_pos[rows] >= 0]
        g = I[rows] * t[rows]
        if stat == "lsq":
            num = np.sum((y[rows] - s[rows]) * g * w[rows])
            den = np.sum(g * g * w[rows])
        else:
            num = np.sum(y[rows] - s[rows])
            den = np.sum(g)
        if den != 0.0:
            U[u] = num / den
    return U


def chi2(rowptr, col, val, w, y, x):
    e, _, _ = row_parts(rowptr, col, val, x, np.full(len(rowptr) - 1, -1))
    return float(np.sum(w * (y - e) ** 2))


def set_background(val, bg_pos, t, unit_of_row, U):
    """H's background entries U_{u(i)} t_i (a copy of val)."""
    out = np.array(val, dtype=np.float64, copy=True)
    has = bg_pos >= 0
    out[bg_pos[has]] = U[unit_of_row[has]] * t[has]
    return out


def empty_field_loop(prob, U0, grp_ptr, grp_rows, unit_of_row, t, bg_pos,
                     itermax=10, rtol=1e-6, stat="lsq"):
    """Algorithm 1.  Returns a dict with the passes (list of dicts with x,
    U (the pattern the pass used), chi2) and the final x, U, diag."""
    import dataclasses
    U = np.array(U0, dtype=np.float64)
    passes = []
    prev = None
    for _ in range(itermax):
        val = set_background(prob.val, bg_pos, t, unit_of_row, U)
        q = dataclasses.replace(prob, val=val)
        o = oracle_solve(q, want_diag=False)
        x = o["x"]
        c = chi2(q.rowptr, q.col, q.val, q.w, q.y, x)
        passes.append({"x": x, "U": U.copy(), "chi2": c, "factor": o["factor"]})
        if prev is not None and prev - c <= rtol * prev:
            break
        prev = c
        U = pattern_update(q.rowptr, q.col, q.val, q.w, q.y, x, bg_pos, t,
                           grp_ptr, grp_rows, U, stat)
    last = passes[-1]
    d = last["factor"].diag_inv()
    return {"passes": passes, "x": last["x"], "U": last["U"], "diag": d}
