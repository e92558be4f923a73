"""Poisson maximum-likelihood solution by Newton's method (App. A.1-A.2):
oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

With the model e = H x and the counts d (the data y), the likelihood of
App. A.1 is L = -2 sum_i (e_i - d_i ln e_i); the fit maximises it, i.e.
minimises C = -L = 2 sum_i (e_i - d_i ln e_i) (a row with d_i = 0 adds
2 e_i).  Its gradient and half Hessian (App. A.2):

    G_j = dC/dx_j = 2 sum_i H_ij (1 - d_i / e_i),     Hess = H^T [d/e^2] H.

Newton's step solves Hess delta = -G / 2 = H^T (d/e - 1): the normal
equations of Sect. 2.4.1 with the weights w_i = d_i / e_i^2 and a new
right-hand side.  The start is the LSQ solution (App. A.2).  As read here:
the step x + a delta takes a = 1, halved while some e_i <= 0 or while C
does not fall by at least 1e-4 a |G . delta| (a sufficient-decrease rule),
except once the predicted decrease |G . delta| is below 1e-12 |C| (below
what C resolves, so a decrease test would only see rounding): then the
whole step is taken.  Iterations stop after a step with max|delta| <= tol
max|x|, or after itermax steps.  The
variances are diag(Hess^-1) at the solution (App. A.2: the Hessian's
inverse, as for the LSQ case; its weights d/e^2 tend to 1/d = 1/sigma^2 as
e -> d).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .reference import oracle_solve


def model(rowptr, col, val, x):
    m = len(rowptr) - 1
    e = np.zeros(m)
    for i in range(m):
        lo, hi = rowptr[i], rowptr[i + 1]
        e[i] = np.sum(val[lo:hi] * x[col[lo:hi]])
    return e


def cash(e, d):
    """C = 2 sum (e - d ln e); +inf if some e_i <= 0 where d_i > 0 (and
    where d_i = 0 a negative e_i is not a valid model either)."""
    if np.any(e <= 0.0):
        return np.inf
    pos = d > 0
    return 2.0 * (np.sum(e) - np.sum(d[pos] * np.log(e[pos])))


def gradient(prob, x):
    """G_j = 2 sum_i H_ij (1 - d_i / e_i)."""
    e = model(prob.rowptr, prob.col, prob.val, x)
    r = 1.0 - prob.y / e
    H = prob.scipy_csr()
    return 2.0 * (H.T @ r)


def hessian_weights(prob, x):
    e = model(prob.rowptr, prob.col, prob.val, x)
    return prob.y / (e * e)


def newton(prob, itermax=20, tol=1e-10, x0=None):
    """Returns a dict: iterates (list of dicts x, C, alpha), final x, C,
    diag (variances), and the LSQ start."""
    if x0 is None:
        x0 = oracle_solve(prob, want_diag=False)["x"]
    x = np.array(x0, dtype=np.float64)
    H = prob.scipy_csr()
    e = model(prob.rowptr, prob.col, prob.val, x)
    C = cash(e, prob.y)
    its = [{"x": x.copy(), "C": C, "alpha": 0.0}]
    for _ in range(itermax):
        w = prob.y / (e * e)
        rhs = H.T @ (prob.y / e - 1.0)            # -G / 2
        q = dataclasses.replace(prob, w=w, y=np.zeros(prob.m))
        f = oracle_solve(q, want_diag=False, refine_steps=0)["factor"]
        delta = f.solve(rhs)
        dec = float(delta @ rhs)                  # -(G . delta) / 2 >= 0
        small = 2.0 * dec <= 1e-12 * abs(C)
        a = 1.0
        while True:
            xt = x + a * delta
            et = model(prob.rowptr, prob.col, prob.val, xt)
            Ct = cash(et, prob.y)
            if np.isfinite(Ct) and (small or Ct <= C - 1e-4 * a * 2.0 * dec):
                break
            a *= 0.5
            if a < 1e-10:
                raise RuntimeError("line search failed")
        x, e, C = xt, et, Ct
        its.append({"x": x.copy(), "C": C, "alpha": a})
        if np.max(np.abs(a * delta)) <= tol * np.max(np.abs(x)):
            break
    q = dataclasses.replace(prob, w=prob.y / (e * e))
    d = oracle_solve(q, refine_steps=0)["diag"]
    return {"iterates": its, "x": x, "C": C, "diag": d, "x_lsq": np.asarray(x0)}
