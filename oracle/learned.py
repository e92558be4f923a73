"""Learned preconditioner: FP64 CPU reference of the network, its training
loss and gradient, and of preconditioned conjugate gradients.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper solves each system directly. It names iterative solvers with
preconditioners as the alternative for large sparse systems, and notes that
they need a good preconditioner to converge (Sect. 3.1). This module is the
plain definition of the extension built on that remark. Many energy bands
share the pattern of H (Sect. 2.2.3). The direct factor of one reference band
serves as the base preconditioner for later bands. A small network predicts
a per-unknown diagonal correction ``D = diag(d)`` of it:

    M_b^-1 = D A_ref^-1 D

Features of unknown j, for band ``b`` against the reference ``r``:
  f0 = log(A_b,jj / A_r,jj)     (diagonal drift of the normal matrix)
  f1 = 1 for a root-front unknown, 0 for a leaf unknown
  f2 = mean of f0 over the unknowns of the same kind
Network, with hidden width ``H``, applied to every unknown with shared weights:
  h1 = tanh(W1 f + b1),  h2 = tanh(W2 h1 + b2),
  g  = w3 . h2 + b3 + wl . f,        d = exp(g)
The linear skip ``wl . f`` lets the correction extrapolate beyond the drift
seen in training. For a pure rescaling ``A_b = S A_r S``, ``g = -f0 / 2`` gives
``D = S^-1`` and hence ``M_b^-1 = A_b^-1`` exactly.

Flat parameter layout (float32 on the device):
  [W1 (H x 3, row-major), b1 (H), W2 (H x H, row-major), b2 (H),
   w3 (H), b3 (1), wl (3)]

Training loss on a band with direct solution ``x = A_b^-1 rhs``:
  e = M_b^-1 rhs - x,   L = (e^T A_b e) / (2 x^T rhs)
This is the squared energy-norm error of one preconditioned step, relative
to ``||x||_A^2 = x^T rhs``.
"""
from __future__ import annotations

import numpy as np

N_FEAT = 3


def param_count(hidden: int) -> int:
    H = hidden
    return H * N_FEAT + H + H * H + H + H + 1 + N_FEAT


def unpack(params, hidden: int):
    H = hidden
    p = np.asarray(params, dtype=np.float64)
    assert p.size == param_count(H)
    o = 0

    def take(k):
        nonlocal o
        v = p[o:o + k]
        o += k
        return v
    W1 = take(H * N_FEAT).reshape(H, N_FEAT)
    b1 = take(H)
    W2 = take(H * H).reshape(H, H)
    b2 = take(H)
    w3 = take(H)
    b3 = take(1)[0]
    wl = take(N_FEAT)
    return W1, b1, W2, b2, w3, b3, wl


def features(diag_band, diag_ref, is_root):
    """Per-unknown features (n x 3) from the diagonals of the two normal
    matrices and the root/leaf flag."""
    f0 = np.log(np.asarray(diag_band, np.float64) / np.asarray(diag_ref, np.float64))
    f1 = np.asarray(is_root, np.float64)
    f2 = np.empty_like(f0)
    for kind in (0.0, 1.0):
        m = f1 == kind
        if m.any():
            f2[m] = f0[m].mean()
    return np.stack([f0, f1, f2], axis=1)


def mlp_forward(params, phi, hidden: int):
    W1, b1, W2, b2, w3, b3, wl = unpack(params, hidden)
    a1 = phi @ W1.T + b1
    h1 = np.tanh(a1)
    a2 = h1 @ W2.T + b2
    h2 = np.tanh(a2)
    g = h2 @ w3 + b3 + phi @ wl
    return g, (phi, h1, h2)


def mlp_backward(params, cache, dg, hidden: int):
    """Gradient of sum_j dg_j g_j with respect to the flat parameters."""
    W1, b1, W2, b2, w3, b3, wl = unpack(params, hidden)
    phi, h1, h2 = cache
    g_w3 = h2.T @ dg
    g_b3 = dg.sum()
    g_wl = phi.T @ dg
    d2 = np.outer(dg, w3) * (1.0 - h2 * h2)          # dL/da2
    g_W2 = d2.T @ h1
    g_b2 = d2.sum(axis=0)
    d1 = (d2 @ W2) * (1.0 - h1 * h1)                 # dL/da1
    g_W1 = d1.T @ phi
    g_b1 = d1.sum(axis=0)
    return np.concatenate([g_W1.ravel(), g_b1, g_W2.ravel(), g_b2, g_w3,
                           [g_b3], g_wl])


def precond_apply(d, apply_ref_inv, r):
    """M_b^-1 r = D A_ref^-1 D r."""
    return d * apply_ref_inv(d * r)


def loss_grad(params, phi, rhs, x, apply_ref_inv, apply_A, hidden: int):
    """Training loss of one band and its gradient (FP64)."""
    g, cache = mlp_forward(params, phi, hidden)
    d = np.exp(g)
    v = apply_ref_inv(d * rhs)
    f = d * v
    e = f - x
    q = apply_A(e)
    xr = float(x @ rhs)
    loss = 0.5 * float(e @ q) / xr
    dLdf = q / xr
    dLdd = dLdf * v + rhs * apply_ref_inv(d * dLdf)
    grad = mlp_backward(params, cache, dLdd * d, hidden)
    return loss, grad


def pcg(apply_A, b, apply_Minv, tol: float, maxit: int, x0=None):
    """Preconditioned conjugate gradients in FP64 (reference iteration):
    stops when ||b - A x|| <= tol ||b||.  Returns (x, iterations)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply_A(x)
    nb = np.linalg.norm(b)
    if np.linalg.norm(r) <= tol * nb:
        return x, 0
    z = apply_Minv(r)
    p = z.copy()
    rz = float(r @ z)
    for it in range(1, maxit + 1):
        q = apply_A(p)
        alpha = rz / float(p @ q)
        x += alpha * p
        r -= alpha * q
        if np.linalg.norm(r) <= tol * nb:
            return x, it
        z = apply_Minv(r)
        rz_new = float(r @ z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, maxit
