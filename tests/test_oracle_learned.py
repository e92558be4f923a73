"""Pins of the learned-preconditioner oracle (CPU, FP64).

* The analytic gradient matches central finite differences. A planted
  mistake (a dropped term of the chain rule) fails the same check.
* Closed form: when the band is an exact rescaling ``A_b = S A_r S``, the
  parameters ``g = -f0 / 2`` make ``M_b^-1 = A_b^-1``. The loss is then 0 and
  one preconditioned step solves the system.
* The tanh layers reproduce a hand-evaluated constant network.
* PCG with the exact inverse as preconditioner converges in one step, and
  in general it converges to the direct solution.
"""
import numpy as np
import pytest

import spi_synth as synth
from oracle import learned as L
from oracle import normal_equations

HID = 8


def _dense(p):
    A, b = normal_equations(p.rowptr, p.col, p.val, p.w, p.y, p.n)
    A = A.toarray() if hasattr(A, "toarray") else np.asarray(A)
    return A, np.asarray(b)


def _pair(seed=3, pure_scale=False):
    """A reference band and a later band on one small pattern."""
    base = synth.make_random_leafy(6, 4, 30, 3, 8, 10, seed=seed)
    rng = np.random.default_rng(seed)
    Ar, _ = _dense(base)
    if pure_scale:
        s = np.exp(rng.uniform(-0.3, 0.3, base.n))
        val = base.val * s[base.col]
        w = base.w
    else:
        val = base.val * np.exp(rng.uniform(-0.2, 0.2, base.n))[base.col]
        w = base.w * np.exp(rng.uniform(-0.1, 0.1, base.m))
    band = synth.Problem(m=base.m, n=base.n, n_bg=base.n_bg, rowptr=base.rowptr,
                         col=base.col, val=val, w=w, y=base.y,
                         x_true=base.x_true, seed=seed)
    Ab, rhs = _dense(band)
    # leaf unknowns of make_random_leafy come first (n_bg of them)
    is_root = (np.arange(base.n) >= base.n_bg).astype(np.float64)
    phi = L.features(np.diag(Ab), np.diag(Ar), is_root)
    return Ar, Ab, rhs, phi


def _ops(Ar, Ab):
    Ari = np.linalg.inv(Ar)
    return (lambda v: Ari @ v), (lambda v: Ab @ v)


def test_gradient_matches_finite_differences():
    Ar, Ab, rhs, phi = _pair()
    x = np.linalg.solve(Ab, rhs)
    M, A = _ops(Ar, Ab)
    params = synth.lp_init_params(HID, seed=1).astype(np.float64)
    params[-3:] = [-0.3, 0.1, 0.05]
    loss, grad = L.loss_grad(params, phi, rhs, x, M, A, HID)
    assert loss > 0
    h = 1e-6
    rng = np.random.default_rng(0)
    for k in rng.choice(params.size, 40, replace=False):
        pp, pm = params.copy(), params.copy()
        pp[k] += h
        pm[k] -= h
        fd = (L.loss_grad(pp, phi, rhs, x, M, A, HID)[0] -
              L.loss_grad(pm, phi, rhs, x, M, A, HID)[0]) / (2 * h)
        assert abs(fd - grad[k]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (k, fd, grad[k])


def test_planted_gradient_mistake_is_caught():
    """Dropping the second chain-rule term of dL/dd (the path through the
    inner D) must break the finite-difference agreement."""
    Ar, Ab, rhs, phi = _pair()
    x = np.linalg.solve(Ab, rhs)
    M, A = _ops(Ar, Ab)
    params = synth.lp_init_params(HID, seed=1).astype(np.float64)
    params[-3:] = [-0.3, 0.1, 0.05]

    def bad_loss_grad(params):
        g, cache = L.mlp_forward(params, phi, HID)
        d = np.exp(g)
        v = M(d * rhs)
        e = d * v - x
        q = A(e)
        xr = float(x @ rhs)
        dLdd = (q / xr) * v                       # planted: term missing
        return L.mlp_backward(params, cache, dLdd * d, HID)
    gb = bad_loss_grad(params)
    k = params.size - 3                           # the skip weight of f0
    h = 1e-6
    pp, pm = params.copy(), params.copy()
    pp[k] += h
    pm[k] -= h
    fd = (L.loss_grad(pp, phi, rhs, x, M, A, HID)[0] -
          L.loss_grad(pm, phi, rhs, x, M, A, HID)[0]) / (2 * h)
    assert abs(fd - gb[k]) > 1e-3 * abs(fd)


def test_pure_rescaling_is_corrected_exactly():
    Ar, Ab, rhs, phi = _pair(pure_scale=True)
    x = np.linalg.solve(Ab, rhs)
    M, A = _ops(Ar, Ab)
    params = np.zeros(L.param_count(HID))
    params[-3:] = [-0.5, 0.0, 0.0]
    loss, grad = L.loss_grad(params, phi, rhs, x, M, A, HID)
    assert loss <= 1e-24
    g, _ = L.mlp_forward(params, phi, HID)
    xs = L.precond_apply(np.exp(g), M, rhs)
    assert np.allclose(xs, x, rtol=1e-10, atol=0)
    # and the uncorrected base preconditioner is clearly worse
    loss0, _ = L.loss_grad(np.zeros_like(params), phi, rhs, x, M, A, HID)
    assert loss0 > 1e-4


def test_tanh_layers_constant_network():
    phi = np.random.default_rng(0).standard_normal((5, 3))
    W1, b1, W2, b2, w3, b3, wl = (np.zeros((HID, 3)), np.full(HID, np.arctanh(0.5)),
                                  np.zeros((HID, HID)), np.full(HID, np.arctanh(0.25)),
                                  np.ones(HID), 0.1, np.zeros(3))
    params = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, w3, [b3], wl])
    g, (ph, h1, h2) = L.mlp_forward(params, phi, HID)
    assert np.allclose(h1, 0.5) and np.allclose(h2, 0.25)
    assert np.allclose(g, 0.25 * HID + 0.1)


def test_pcg_reference():
    Ar, Ab, rhs, phi = _pair()
    x = np.linalg.solve(Ab, rhs)
    A = lambda v: Ab @ v
    Ai = np.linalg.inv(Ab)
    xs, it = L.pcg(A, rhs, lambda r: Ai @ r, 1e-12, 50)
    assert it == 1 and np.linalg.norm(xs - x) <= 1e-10 * np.linalg.norm(x)
    Ari = np.linalg.inv(Ar)
    xs, it = L.pcg(A, rhs, lambda r: Ari @ r, 1e-12, 200)
    assert it > 1 and np.linalg.norm(xs - x) <= 1e-9 * np.linalg.norm(x)


def test_features_hand_worked_fixture():
    """Features against a hand-worked fixture; a mean over all unknowns in
    place of the per-kind mean f2 fails it."""
    import os
    fx = {}
    with open(os.path.join(os.path.dirname(__file__), "golden",
                           "lp_features_6.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                k, *v = line.split()
                fx[k] = np.array([float(x) for x in v])
    phi = L.features(fx["diag_band"], fx["diag_ref"], fx["is_root"])
    assert phi.shape == (6, 3)
    for c, key in enumerate(("f0", "f1", "f2")):
        assert np.allclose(phi[:, c], fx[key], rtol=1e-15, atol=1e-15), key
    assert not np.allclose(np.full(6, phi[:, 0].mean()), fx["f2"], rtol=1e-6)
