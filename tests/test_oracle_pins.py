"""Pins for the CPU oracle against facts the paper and mathematics fix.

Every test here runs on the CPU.  The oracle is checked against exact
rational arithmetic, hand-worked fixtures, the paper's worked elimination-tree
example, closed forms, invariants and a statistical property of the
variances -- never against itself alone.
"""
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

import spi_synth as synth
from oracle import (normal_equations, normal_equations_bruteforce, cholesky,
                    forward_subst, backward_subst, solve_dense,
                    inverse_from_cholesky, diag_inv_colnorms,
                    selected_entry_pruned, BlockCholesky, oracle_solve)
from oracle import etree as et
from oracle.certify import (normal_residual_ld, refine_inverse_column,
                            refine_solution, LD)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- exact helpers
def _frac_matrix(A):
    return [[Fraction(int(v)) if float(v).is_integer() else Fraction(float(v))
             for v in row] for row in np.asarray(A)]


def _exact_inverse(A):
    """Gauss-Jordan elimination in exact rational arithmetic."""
    n = len(A)
    M = [row[:] + [Fraction(int(i == j)) for j in range(n)]
         for i, row in enumerate(_frac_matrix(A))]
    for k in range(n):
        piv = next(r for r in range(k, n) if M[r][k] != 0)
        M[k], M[piv] = M[piv], M[k]
        pk = M[k][k]
        M[k] = [v / pk for v in M[k]]
        for r in range(n):
            if r != k and M[r][k] != 0:
                f = M[r][k]
                M[r] = [a - f * b for a, b in zip(M[r], M[k])]
    return [row[n:] for row in M]


def _exact_ldl(A):
    """A = Lt D Lt^T with unit lower Lt, exact rationals."""
    n = len(A)
    F = _frac_matrix(A)
    Lt = [[Fraction(int(i == j)) for j in range(n)] for i in range(n)]
    D = [Fraction(0)] * n
    for j in range(n):
        D[j] = F[j][j] - sum(Lt[j][k] ** 2 * D[k] for k in range(j))
        for i in range(j + 1, n):
            Lt[i][j] = (F[i][j] - sum(Lt[i][k] * Lt[j][k] * D[k]
                                      for k in range(j))) / D[j]
    return Lt, D


def _integer_spd(n, seed, extra_rows=None):
    rng = np.random.default_rng(seed)
    m = extra_rows or 2 * n
    H = rng.integers(-3, 4, size=(m, n)).astype(float)
    H[rng.random((m, n)) < 0.5] = 0.0
    H = np.vstack([H, 2 * np.eye(n)])
    return H.T @ H, H


# ------------------------------------------------------------ normal equations
def _read_fixture(name):
    rows = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            rows.setdefault(key, []).append([float(v) for v in vals])
    return rows


def test_normal_equations_hand_worked_fixture():
    fx = _read_fixture("normal_eq_3x2.txt")
    H = np.array(fx["H"])
    w, y = np.array(fx["w"][0]), np.array(fx["y"][0])
    Hs = sp.csr_matrix(H)
    Hs.eliminate_zeros()
    A, b = normal_equations(Hs.indptr, Hs.indices, Hs.data, w, y, 2)
    assert np.array_equal(A.toarray(), np.array(fx["A"]))
    assert np.array_equal(b, np.array(fx["b"][0]))
    Ab, bb = normal_equations_bruteforce(Hs.indptr, Hs.indices, Hs.data, w, y, 2)
    assert np.array_equal(Ab, np.array(fx["A"]))
    assert np.array_equal(bb, np.array(fx["b"][0]))


def test_normal_equations_identity_transfer_matrix():
    n = 7
    w = np.arange(1, n + 1, dtype=float)
    y = np.arange(10, 10 + n, dtype=float)
    I = sp.identity(n, format="csr")
    A, b = normal_equations(I.indptr, I.indices, I.data, w, y, n)
    assert np.array_equal(A.toarray(), np.diag(w))
    assert np.array_equal(b, w * y)


def test_normal_equations_bruteforce_matches_sparse_exactly():
    p = synth.make_random(40, 15, 4, seed=3, integer=True)
    A, b = normal_equations(p.rowptr, p.col, p.val, p.w, p.y, p.n)
    Ab, bb = normal_equations_bruteforce(p.rowptr, p.col, p.val, p.w, p.y, p.n)
    assert np.array_equal(A.toarray(), Ab)       # integers: exact in binary64
    assert np.array_equal(b, bb)
    # symmetric, and the diagonal equals the weighted column sums of squares
    assert np.array_equal(Ab, Ab.T)
    H = p.scipy_csr().toarray()
    assert np.array_equal(np.diag(Ab), (H * H * p.w[:, None]).sum(axis=0))


# ---------------------------------------------------------- elimination tree
def _paper_tree():
    fx = _read_fixture("etree_6node.txt")
    parent = {int(a): int(b) for a, b in fx["parent"]}
    return fx, [parent[v] - 1 for v in range(1, 7)]  # 0-based, root -> -1


# A pattern whose elimination tree is the paper's tree, with one fill entry
# (eliminating node 2 connects 3 and 6).  1-based pairs.
_PAPER_PATTERN = [(1, 4), (1, 5), (2, 3), (2, 6), (3, 5), (4, 5), (5, 6)]


def test_etree_paper_example():
    fx, parent = _paper_tree()
    edges = [(a - 1, b - 1) for a, b in _PAPER_PATTERN]
    struct = et.symbolic_cholesky(6, edges)
    assert et.etree_from_struct(struct) == parent
    assert struct[1] == [2, 5]                     # fill (6, 3) from node 2
    assert et.roots(parent) == [5]
    assert sorted(et.leaves(parent)) == [v - 1 for v in fx["leaves"][0]]
    assert et.descendants(parent, 4) == [v - 1 for v in fx["descendants"][0][1:]]
    assert set(et.children(parent)[4]) == {2, 3}
    assert et.ancestors(parent, 3) == [4, 5]
    order = [int(v) - 1 for v in fx["postorder"][0]]
    assert et.is_postorder(order, parent)
    assert et.is_postorder(et.postorder(parent), parent)
    assert not et.is_postorder([0, 1, 3, 2, 4, 5], parent)   # 4's subtree split


def test_etree_matches_numerical_cholesky_pattern():
    """Parents from the symbolic code equal those read off a numerical L."""
    rng = np.random.default_rng(0)
    for trial in range(20):
        n = int(rng.integers(5, 25))
        pairs = [(i, j) for i in range(n) for j in range(i)
                 if rng.random() < 0.15]
        A = np.eye(n) * (n + 1.0)
        for i, j in pairs:
            A[i, j] = A[j, i] = rng.uniform(0.5, 1.0)
        Ln = np.linalg.cholesky(A)
        par_num = []
        for j in range(n):
            nz = np.nonzero(np.abs(Ln[j + 1:, j]) > 1e-300)[0]
            par_num.append(int(nz[0]) + j + 1 if len(nz) else -1)
        assert et.etree_from_struct(et.symbolic_cholesky(n, pairs)) == par_num


def test_pruned_inverse_entry_paper_example():
    fx, parent = _paper_tree()
    n = 6
    A = np.eye(n) * 6.0
    for a, b in _PAPER_PATTERN:
        A[a - 1, b - 1] = A[b - 1, a - 1] = 1.0
    L = cholesky(A)
    i, j = (int(v) - 1 for v in fx["entry"][0])
    val, fwd, bwd = selected_entry_pruned(L, parent, i, j)
    assert fwd == [int(v) - 1 for v in fx["forward"][0]]
    assert bwd == [int(v) - 1 for v in fx["backward"][0]]
    skipped = {int(v) - 1 for v in fx["skipped"][0]}
    assert not skipped & set(fwd + bwd)
    Zx = _exact_inverse(A)
    assert abs(val - float(Zx[i][j])) <= 1e-15 * abs(float(Zx[i][j]))


# --------------------------------------------------------- dense factorisation
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_dense_cholesky_matches_exact_ldl(seed):
    A, _ = _integer_spd(8, seed)
    Lt, D = _exact_ldl(A)
    L_exact = np.array([[float(Lt[i][j]) * np.sqrt(float(D[j])) for j in range(8)]
                        for i in range(8)])
    L = cholesky(A)
    assert np.allclose(L, L_exact, rtol=1e-13, atol=1e-13 * np.abs(L_exact).max())
    assert np.array_equal(L, np.tril(L))


@pytest.mark.parametrize("seed", [0, 1])
def test_dense_solve_inverse_and_colnorms_match_exact(seed):
    A, H = _integer_spd(9, seed)
    Zx = np.array([[float(v) for v in row] for row in _exact_inverse(A)])
    b = np.arange(1, 10, dtype=float)
    x, L = solve_dense(A, b)
    assert np.allclose(x, Zx @ b, rtol=1e-12, atol=0)
    assert np.allclose(inverse_from_cholesky(L), Zx, rtol=1e-12, atol=1e-15)
    assert np.allclose(diag_inv_colnorms(L), np.diag(Zx), rtol=1e-13, atol=0)
    # forward/backward separately: L z = b and L^T x = z
    z = forward_subst(L, b)
    assert np.allclose(L @ z, b, rtol=1e-14, atol=1e-13)
    assert np.allclose(L.T @ backward_subst(L, z), z, rtol=1e-14, atol=1e-13)


def test_pruned_entries_match_exact_inverse_random_pattern():
    A, _ = _integer_spd(10, 5)
    n = A.shape[0]
    pairs = [(i, j) for i in range(n) for j in range(i) if A[i, j] != 0]
    parent = et.etree_from_struct(et.symbolic_cholesky(n, pairs))
    L = cholesky(A)
    Zx = _exact_inverse(A)
    for i in range(n):
        for j in range(n):
            val, _, _ = selected_entry_pruned(L, parent, i, j)
            ref = float(Zx[i][j])
            assert abs(val - ref) <= 1e-12 * max(abs(ref), 1e-3)


def test_not_spd_is_reported():
    A = np.array([[4.0, 2.0], [2.0, 1.0 - 1e-3]])
    with pytest.raises(ValueError):
        cholesky(A)


# ------------------------------------------------------------- closed forms
def test_two_unknown_closed_form():
    """1 background unknown (coefficient 1) + 1 sky pixel with responses h."""
    h = np.array([0.3, 0.9, 0.5, 0.7])
    w = np.array([0.01, 0.02, 0.015, 0.005])
    y = np.array([40.0, 61.0, 52.0, 48.0])
    rowptr = np.arange(0, 9, 2, dtype=np.int64)
    col = np.tile(np.array([0, 1], dtype=np.int32), 4)
    val = np.ravel(np.column_stack([np.ones(4), h]))
    a11, a12, a22 = w.sum(), (w * h).sum(), (w * h * h).sum()
    b1, b2 = (w * y).sum(), (w * h * y).sum()
    det = a11 * a22 - a12 * a12
    x_ref = np.array([(a22 * b1 - a12 * b2) / det, (a11 * b2 - a12 * b1) / det])
    d_ref = np.array([a22 / det, a11 / det])
    A, b = normal_equations(rowptr, col, val, w, y, 2)
    x, L = solve_dense(A.toarray(), b)
    assert np.allclose(x, x_ref, rtol=1e-13)
    assert np.allclose(diag_inv_colnorms(L), d_ref, rtol=1e-13)
    f = BlockCholesky(A, 1)
    assert np.allclose(f.solve(b), x_ref, rtol=1e-13)
    assert np.allclose(f.diag_inv(), d_ref, rtol=1e-13)


def test_block_diagonal_problem_splits():
    """Two problems with no shared row: diag(A^-1) is the per-block diagonal."""
    p1 = synth.make_random(30, 8, 3, seed=11)
    p2 = synth.make_random(25, 6, 3, seed=12)
    rowptr = np.concatenate([p1.rowptr, p1.rowptr[-1] + p2.rowptr[1:]])
    col = np.concatenate([p1.col, p2.col + p1.n]).astype(np.int32)
    val = np.concatenate([p1.val, p2.val])
    w = np.concatenate([p1.w, p2.w])
    y = np.concatenate([p1.y, p2.y])
    A, b = normal_equations(rowptr, col, val, w, y, p1.n + p2.n)
    x, L = solve_dense(A.toarray(), b)
    d = diag_inv_colnorms(L)
    for p, sl in ((p1, slice(0, p1.n)), (p2, slice(p1.n, None))):
        Ai, bi = normal_equations(p.rowptr, p.col, p.val, p.w, p.y, p.n)
        Zi = np.linalg.inv(Ai.toarray())          # textbook inverse (LAPACK)
        assert np.allclose(d[sl], np.diag(Zi), rtol=1e-12)
        assert np.allclose(x[sl], Zi @ bi, rtol=1e-11)


# ----------------------------------------------- block factorisation (tiny workload)
@pytest.fixture(scope="module")
def tiny():
    p = synth.make_config(0)
    A, b = normal_equations(p.rowptr, p.col, p.val, p.w, p.y, p.n)
    return p, A, b


def test_block_factor_matches_dense_and_invariants(tiny):
    p, A, b = tiny
    Ad = A.toarray()
    x_d, L = solve_dense(Ad, b)
    d_d = diag_inv_colnorms(L)
    f = BlockCholesky(A, p.n_bg)
    assert f.bb_diagonal                      # background unknowns share no row
    x_b = f.solve(b)
    d_b = f.diag_inv()
    assert np.linalg.norm(x_b - x_d) / np.linalg.norm(x_d) < 1e-12
    assert np.max(np.abs(d_b - d_d) / d_d) < 1e-12
    # residual and Cauchy-Schwarz lower bound diag(A^-1)_i >= 1/A_ii > 0
    assert np.linalg.norm(Ad @ x_b - b) / np.linalg.norm(b) < 1e-14
    assert np.all(d_b * np.diag(Ad) >= 1.0 - 1e-12)
    # against LAPACK's inverse (a textbook routine, not the oracle's code)
    Z = np.linalg.inv(Ad)
    assert np.max(np.abs(d_b - np.diag(Z)) / np.diag(Z)) < 1e-10


def test_block_factor_sparse_and_dense_products_agree(tiny, monkeypatch):
    """The coupling block is dense on the tiny workload (dense products);
    forced sparse, the same factor gives the same x and variances, and both
    match the dense oracle's own loop."""
    p, A, b = tiny
    fd = BlockCholesky(A, p.n_bg)
    assert not sp.issparse(fd.Lsb)
    monkeypatch.setattr(BlockCholesky, "DENSE_FRACTION", 2.0)
    fs = BlockCholesky(A, p.n_bg)
    assert sp.issparse(fs.Lsb)
    x_d, L = solve_dense(A.toarray(), b)
    d_d = diag_inv_colnorms(L)
    for f in (fd, fs):
        assert np.linalg.norm(f.solve(b) - x_d) / np.linalg.norm(x_d) < 1e-12
        assert np.max(np.abs(f.diag_inv() - d_d) / d_d) < 1e-12


def test_block_factor_general_pivot_block():
    """Leading block that is not diagonal goes through the general branch."""
    p = synth.make_random(60, 12, 4, seed=4)
    A, b = normal_equations(p.rowptr, p.col, p.val, p.w, p.y, p.n)
    f = BlockCholesky(A, 5)
    assert not f.bb_diagonal
    Z = np.linalg.inv(A.toarray())
    assert np.allclose(f.solve(b), Z @ b, rtol=1e-10)
    assert np.allclose(f.diag_inv(), np.diag(Z), rtol=1e-10)


def test_certified_solution_and_inverse_column(tiny):
    p, A, b = tiny
    out = oracle_solve(p, diag_idx=[0, 5, 400, 779], refine_steps=2)
    r = normal_residual_ld(p.rowptr, p.col, p.val, p.w, p.y, out["x"])
    assert float(np.max(np.abs(r))) <= 1e-13 * float(np.max(np.abs(b)))
    f = out["factor"]
    for j, dj in zip(out["diag_idx"], out["diag"]):
        zc = refine_inverse_column(p, f.solve, int(j))
        assert abs(float(zc[j]) - dj) <= 1e-13 * dj


def _exact_lsq(p):
    """Exact rational solution of H^T W H x = H^T W y for integer H, W, y."""
    H = p.scipy_csr().toarray()
    A = H.T @ (p.w[:, None] * H)            # integers: exact in binary64
    b = H.T @ (p.w * p.y)
    assert np.array_equal(A, np.round(A)) and np.array_equal(b, np.round(b))
    Zx = _exact_inverse(A)
    bx = [Fraction(int(v)) for v in b]
    n = len(bx)
    return A, b, [sum(Zx[i][k] * bx[k] for k in range(n)) for i in range(n)]


def _rel_err_exact(x, xe):
    """max_i |x_i - xe_i| / max_i |xe_i| in exact arithmetic."""
    num = max(abs(Fraction(*LD(v).as_integer_ratio()) - e) for v, e in zip(x, xe))
    return float(num / max(abs(e) for e in xe))


def _residual_sign_flip(rowptr, col, val, w, y, x):
    """Planted mistake: H^T W (y + H x) instead of H^T W (y - H x)."""
    return normal_residual_ld(rowptr, col, val, w, y, -np.asarray(x, dtype=LD))


def _residual_wrong_row(rowptr, col, val, w, y, x):
    """Planted mistake: the weights and data of the next row (shifted index)."""
    return normal_residual_ld(rowptr, col, val, np.roll(w, 1), np.roll(y, 1), x)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_refined_solution_matches_exact_rational(seed):
    """The long-double refinement that certifies every reference x reaches
    the exact rational solution of an integer problem far below binary64
    resolution; a residual with a sign error or a shifted row index, fed to
    the same refinement, misses it."""
    p = synth.make_random(30, 10, 4, seed=seed, integer=True)
    A, b, xe = _exact_lsq(p)
    solve = lambda r: np.linalg.solve(A, r)        # binary64 LAPACK solve
    x0 = solve(b)
    assert _rel_err_exact(x0, xe) > 1e-17          # binary64 alone is not exact
    x = refine_solution(p, solve, x0, steps=3)
    assert x.dtype == LD
    assert _rel_err_exact(x, xe) <= 1e-18
    for bad in (_residual_sign_flip, _residual_wrong_row):
        xb = refine_solution(p, solve, x0, steps=3, residual=bad)
        assert _rel_err_exact(xb, xe) > 1e-6, bad.__name__


def test_refined_solution_agrees_with_block_solve(tiny):
    """On the tiny workload the certified x equals the block factor's plain
    binary64 solution to within that solution's own rounding."""
    p, A, b = tiny
    f = BlockCholesky(A, p.n_bg)
    xb = f.solve(b)
    xr = refine_solution(p, f.solve, xb, steps=2).astype(np.float64)
    assert np.linalg.norm(xr - xb) / np.linalg.norm(xr) <= 1e-13


def test_inverse_entries_match_exact_and_pruned(tiny):
    """General entries of A^-1 (covariances) by blocked solves with the
    block factor: the exact rational inverse of an integer problem (both
    branches of the factor), the paper's pruned traversal on the tiny
    workload (Sect. 3.3.1), and symmetry."""
    A, _ = _integer_spd(11, 7)
    Zx = _exact_inverse(A)
    for nb in (4, 0):
        f = BlockCholesky(sp.csr_matrix(A), nb)
        r, c = np.meshgrid(np.arange(11), np.arange(11), indexing="ij")
        v = f.inverse_entries(r.ravel(), c.ravel(), block=5)
        ref = np.array([float(Zx[i][j]) for i, j in zip(r.ravel(), c.ravel())])
        assert np.max(np.abs(v - ref)) <= 1e-13 * np.max(np.abs(ref))
    p, A, b = tiny
    f = BlockCholesky(A, p.n_bg)
    L = cholesky(A.toarray())
    pairs = [(i, j) for i in range(L.shape[0]) for j in range(i + 1)
             if A[i, j] != 0 or i == j]
    parent = et.etree_from_struct(et.symbolic_cholesky(L.shape[0], pairs))
    rng = np.random.default_rng(4)
    rr = rng.integers(0, p.n, 40)
    cc = rng.integers(0, p.n, 40)
    v = f.inverse_entries(rr, cc)
    vt = f.inverse_entries(cc, rr)
    assert np.max(np.abs(v - vt)) <= 1e-13 * np.max(np.abs(v))
    for k in range(0, 40, 4):
        ref, _, _ = selected_entry_pruned(L, parent, int(rr[k]), int(cc[k]))
        assert abs(v[k] - ref) <= 1e-12 * max(abs(ref), 1e-3)


def test_pulls_have_unit_scale():
    """Unscaled diag(A^-1) is the variance: pulls (x - x_true)/sd ~ N(0, 1).

    Catches a wrong variance scale (a factor 2 moves the std to 0.71 or
    1.41), a wrong sign or index in the solve (mean drifts away from 0).
    """
    pulls = []
    for seed in range(6):
        p = synth.make_config(0, seed=seed)
        A, b = normal_equations(p.rowptr, p.col, p.val, p.w, p.y, p.n)
        f = BlockCholesky(A, p.n_bg)
        x = f.solve(b)
        d = f.diag_inv()
        pulls.append((x - p.x_true) / np.sqrt(d))
    pulls = np.concatenate(pulls)
    assert abs(pulls.mean()) < 0.15
    assert abs(pulls.std() - 1.0) < 0.06


# --------------------------------------------------- planted oracle mistakes
def test_planted_mistakes_are_caught(tiny):
    """Variants with a dropped term, a sign flip and a transposed operand
    must fail the same checks the real oracle passes."""
    p, A, b = tiny
    Ad = A.toarray()
    f = BlockCholesky(A, p.n_bg)
    # (1) dropped Schur-complement term: factor A_ss instead of S
    bad = BlockCholesky(A, p.n_bg)
    bad.Lss = np.linalg.cholesky(A[p.n_bg:, p.n_bg:].toarray())
    xb = bad.solve(b)
    assert np.linalg.norm(Ad @ xb - b) / np.linalg.norm(b) > 1e-6
    # (2) sign flip in the coupling block
    bad2 = BlockCholesky(A, p.n_bg)
    bad2.Lsb = -bad2.Lsb
    assert np.linalg.norm(Ad @ bad2.solve(b) - b) / np.linalg.norm(b) > 1e-6
    # (3) transposed factor in the backward substitution (L x = z, not L^T)
    As, bs = Ad[-40:, -40:], b[-40:]          # sky block: L is not diagonal
    L = cholesky(As)
    z = forward_subst(L, bs)
    x_wrong = forward_subst(L, z)
    assert np.linalg.norm(As @ x_wrong - bs) / np.linalg.norm(bs) > 1e-6
    x_right = backward_subst(L, z)
    assert np.linalg.norm(As @ x_right - bs) / np.linalg.norm(bs) < 1e-14
    # (4) a missing diagonal term in the variances: norm of the sky part only
    d_ok = f.diag_inv(np.arange(5))
    U = 1.0 / f.Lbb[:5]
    assert np.all(np.abs(d_ok - (d_ok - U * U)) / d_ok > 1e-3)
