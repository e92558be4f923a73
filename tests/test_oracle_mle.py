"""Pins of the Poisson maximum-likelihood oracle (App. A.1-A.2), CPU only.

* The gradient matches central finite differences of C = 2 sum(e - d ln e);
  the half Hessian H^T [d/e^2] H matches finite differences of the
  gradient (planted mistakes: d/e in place of d/e^2, a sign flip).
* Where the model equals the data (e = d), the Hessian is the chi-square
  normal matrix with weights 1/d (App. A.2's limit).
* One unknown, e_i = h_i x: the MLE is sum d / sum h (closed form), which
  Newton reaches.
* Newton from the LSQ start lowers C, ends with a zero gradient, and its
  variances are those of the final Hessian (positive, at least 1/Hess_jj).
"""
import dataclasses

import numpy as np
import pytest
import scipy.sparse as sp

import spi_synth as synth
from oracle import mle


@pytest.fixture(scope="module")
def prob():
    return synth.make_config(0)


def _C(p, x):
    return mle.cash(mle.model(p.rowptr, p.col, p.val, x), p.y)


def test_gradient_matches_finite_differences(prob):
    p = prob
    x = p.x_true * (1.0 + 0.05 * np.random.default_rng(0).standard_normal(p.n))
    g = mle.gradient(p, x)
    rng = np.random.default_rng(1)
    for j in rng.choice(p.n, 12, replace=False):
        h = 1e-5 * x[j]
        xp, xm = x.copy(), x.copy()
        xp[j] += h
        xm[j] -= h
        fd = (_C(p, xp) - _C(p, xm)) / (2 * h)
        assert abs(fd - g[j]) <= 1e-5 * max(1.0, abs(g[j])), (j, fd, g[j])


def _hess_vec(p, x, v, w_fn):
    H = p.scipy_csr()
    return H.T @ (w_fn(p, x) * (H @ v))


def test_hessian_matches_gradient_differences(prob):
    p = prob
    x = p.x_true * 1.02
    rng = np.random.default_rng(2)
    v = rng.standard_normal(p.n)
    h = 1e-6
    fd = (mle.gradient(p, x + h * v) - mle.gradient(p, x - h * v)) / (2 * h)
    hv = 2.0 * _hess_vec(p, x, v, mle.hessian_weights)
    assert np.max(np.abs(fd - hv)) <= 1e-5 * np.max(np.abs(hv))
    # planted: d/e instead of d/e^2
    bad = 2.0 * _hess_vec(p, x, v, lambda q, z: q.y / mle.model(q.rowptr, q.col,
                                                                  q.val, z))
    assert np.max(np.abs(fd - bad)) > 1e-2 * np.max(np.abs(hv))
    # planted: sign of the gradient
    g = mle.gradient(p, x)
    j = int(np.argmax(np.abs(g)))
    xp, xm = x.copy(), x.copy()
    xp[j] += 1e-5 * x[j]
    xm[j] -= 1e-5 * x[j]
    fd_j = (_C(p, xp) - _C(p, xm)) / (2e-5 * x[j])
    assert abs(fd_j + g[j]) > 1e-3 * abs(g[j])


def test_hessian_limit_is_chi_square_matrix(prob):
    p = prob
    H = p.scipy_csr()
    q = dataclasses.replace(p, y=H @ p.x_true)           # e = d at x_true
    w = mle.hessian_weights(q, p.x_true)
    assert np.allclose(w, 1.0 / q.y, rtol=1e-14)
    from oracle import normal_equations
    A1, _ = normal_equations(q.rowptr, q.col, q.val, w, q.y, q.n)
    A2, _ = normal_equations(q.rowptr, q.col, q.val, 1.0 / q.y, q.y, q.n)
    assert np.allclose(A1.toarray(), A2.toarray(), rtol=1e-13, atol=0)


def test_one_unknown_closed_form():
    rng = np.random.default_rng(3)
    m = 40
    h = 0.2 + rng.random(m)
    d = rng.poisson(30.0 * h).astype(float)
    rowptr = np.arange(m + 1, dtype=np.int64)
    p = synth.Problem(m=m, n=1, n_bg=0, rowptr=rowptr, col=np.zeros(m, np.int32),
                      val=h, w=1.0 / np.maximum(d, 1.0), y=d, x_true=np.array([30.0]))
    out = mle.newton(p, itermax=30)
    assert abs(out["x"][0] - d.sum() / h.sum()) <= 1e-13 * out["x"][0]


def test_newton_from_lsq_start(prob):
    p = prob
    out = mle.newton(p, itermax=20)
    its = out["iterates"]
    C = [it["C"] for it in its]
    # (the last, small step changes C only by rounding)
    assert all(b <= a + 1e-15 * abs(a) for a, b in zip(C, C[1:]))
    assert C[-1] < C[0]
    g = mle.gradient(p, out["x"])
    scale = 2.0 * np.abs(p.scipy_csr()).T @ np.ones(p.m)
    assert np.max(np.abs(g) / scale) <= 1e-10
    assert len(its) <= 8
    H = p.scipy_csr()
    e = H @ out["x"]
    hjj = np.asarray((H.multiply(H)).T @ (p.y / e ** 2)).ravel()
    assert np.all(out["diag"] > 0) and np.all(out["diag"] * hjj >= 1 - 1e-12)
