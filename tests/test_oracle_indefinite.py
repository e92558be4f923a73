"""Pins of the indefinite-matrix oracle (x = A^-1 b and diag(A^-1) for
A = H^T W H with weights of either sign; Sect. 5, Sect. 2.4.1).

Each pin fixes the result by something other than the oracle's own route
(LU with row pivoting plus long-double refinement): a closed form, an
eigen-decomposition built into H and W, the positive-definite oracle, and
the Sherman-Morrison formula for a flipped weight.
"""
import numpy as np
import pytest

import spi_synth as synth
from oracle import oracle_solve
from oracle.indefinite import indefinite_solve
from oracle.normal_eq import normal_equations


def _problem(H, w, y, name="pin"):
    H = np.asarray(H, dtype=np.float64)
    m, n = H.shape
    rows_c = [np.nonzero(H[r])[0] for r in range(m)]
    rowptr = np.zeros(m + 1, dtype=np.int64)
    rowptr[1:] = np.cumsum([len(c) for c in rows_c])
    col = np.concatenate(rows_c).astype(np.int32)
    val = np.concatenate([H[r, rows_c[r]] for r in range(m)])
    return synth.Problem(m=m, n=n, n_bg=0, rowptr=rowptr, col=col, val=val,
                         w=np.asarray(w, dtype=np.float64),
                         y=np.asarray(y, dtype=np.float64), x_true=np.zeros(n),
                         name=name)


def test_two_unknowns_closed_form():
    """H = [e1; e2; e1 + e2], w = (1, 1, -2): A = [[-1, -2], [-2, -1]]
    (det -3), A^-1 = [[1, -2], [-2, 1]] / 3; y = H (1, 2) gives x = (1, 2)."""
    p = _problem([[1, 0], [0, 1], [1, 1]], [1.0, 1.0, -2.0], [1.0, 2.0, 3.0])
    o = indefinite_solve(p)
    assert np.allclose(o["A"], [[-1.0, -2.0], [-2.0, -1.0]], rtol=0, atol=0)
    assert np.allclose(o["x"], [1.0, 2.0], rtol=1e-15, atol=1e-15)
    assert np.allclose(o["diag"], [1.0 / 3.0, 1.0 / 3.0], rtol=1e-15)


def test_eigen_construction():
    """H = diag(sqrt|lam|) Q^T, W = sign(lam) gives A = Q diag(lam) Q^T, so
    A^-1 = Q diag(1/lam) Q^T: diag(A^-1)_i = sum_k Q_ik^2 / lam_k."""
    rng = np.random.default_rng(4)
    n = 9
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.array([3.0, -2.0, 0.5, -0.25, 7.0, -5.0, 1.5, 2.5, -0.75])
    H = np.diag(np.sqrt(np.abs(lam))) @ Q.T
    y = rng.standard_normal(n)
    p = _problem(H, np.sign(lam), y)
    o = indefinite_solve(p)
    d_ref = (Q * Q / lam).sum(axis=1)
    b = H.T @ (np.sign(lam) * y)
    x_ref = Q @ ((Q.T @ b) / lam)
    assert np.max(np.abs(o["diag"] - d_ref)) <= 1e-12 * np.max(np.abs(d_ref))
    assert np.linalg.norm(o["x"] - x_ref) <= 1e-12 * np.linalg.norm(x_ref)


def test_agrees_with_the_positive_definite_oracle():
    """With positive weights the LU route and the Cholesky route of the
    positive-definite oracle give the same x and variances."""
    p = synth.make_random_leafy(6, 4, 60, 3, 8, 20, seed=11)
    o1 = indefinite_solve(p)
    o2 = oracle_solve(p)
    assert np.linalg.norm(o1["x"] - o2["x"]) <= 1e-13 * np.linalg.norm(o2["x"])
    assert np.max(np.abs(o1["diag"] - o2["diag"]) / o2["diag"]) <= 1e-12


def test_flipped_weight_sherman_morrison():
    """Flipping the sign of row r's weight: A' = A - 2 w_r h h^T, and
    A'^-1 = A^-1 + 2 w_r (A^-1 h)(A^-1 h)^T / (1 - 2 w_r h^T A^-1 h)
    (A^-1 from the positive-definite oracle's dense inverse)."""
    p = synth.make_random_leafy(4, 3, 30, 3, 6, 10, seed=5)
    A, _ = normal_equations(p.rowptr, p.col, p.val, p.w, p.y, p.n)
    Ainv = np.linalg.inv(A.toarray())
    r = 2  # 2 w_r h^T A^-1 h = 1.96 > 1: the flipped matrix is indefinite
    h = np.zeros(p.n)
    h[p.col[p.rowptr[r]:p.rowptr[r + 1]]] = p.val[p.rowptr[r]:p.rowptr[r + 1]]
    z = Ainv @ h
    s = 2.0 * p.w[r] * (h @ z)
    assert s > 1.5
    w2 = p.w.copy()
    w2[r] *= -1.0
    q = synth.Problem(m=p.m, n=p.n, n_bg=p.n_bg, rowptr=p.rowptr, col=p.col,
                      val=p.val, w=w2, y=p.y, x_true=p.x_true, name="flip")
    o = indefinite_solve(q)
    d_ref = np.diag(Ainv) + 2.0 * p.w[r] * z * z / (1.0 - s)
    assert np.min(np.linalg.eigvalsh(o["A"])) < 0.0
    assert np.max(np.abs(o["diag"] - d_ref)) <= 1e-9 * np.max(np.abs(d_ref))


def test_generator_zero_diagonal_entries_are_exact():
    """The zero-diagonal unknowns of the indefinite generator: A_zz = 0 and
    A_zk = 2 exactly, and A is indefinite."""
    p = synth.make_indefinite(4, 3, 60, 3, 6, 20, 4, seed=2)
    A, _ = normal_equations(p.rowptr, p.col, p.val, p.w, p.y, p.n)
    A = A.toarray()
    deg = np.diff(p.rowptr)
    zero = [j for j in range(p.n_bg, p.n) if A[j, j] == 0.0]
    assert len(zero) == 4
    for z in zero:
        nz = A[z][A[z] != 0.0]
        assert np.all(nz == 2.0)
    assert np.min(np.linalg.eigvalsh(A)) < 0.0
    assert deg.min() >= 1
    o = indefinite_solve(p)
    assert np.max(np.abs(A @ o["x"] - o["b"])) <= 1e-12 * np.max(np.abs(o["b"]))


@pytest.mark.parametrize("seed", [1, 3])
def test_indefinite_residuals(seed):
    """x solves A x = b and the diagonal entries are those of the refined
    inverse columns: A z_j = e_j to working accuracy for sampled j."""
    p = synth.make_indefinite(8, 4, 150, 3, 8, 80, 3, seed=seed)
    o = indefinite_solve(p)
    A = o["A"]
    assert np.min(np.linalg.eigvalsh(A)) < 0.0
    assert np.linalg.norm(A @ o["x"] - o["b"]) <= 1e-13 * np.linalg.norm(o["b"])
    Ainv = np.linalg.inv(A)
    cond = np.linalg.cond(A)
    assert np.max(np.abs(o["diag"] - np.diag(Ainv))) <= \
        50 * cond * 1e-16 * np.max(np.abs(np.diag(Ainv)))
