"""GPU parity for symmetric indefinite matrices (opts.indefinite = 1):
weights of either sign, Bunch-Kaufman 1 x 1 and 2 x 2 pivots inside the
root front's 64-column pivot blocks (Sect. 5: the SPI matrices need 2 x 2
pivots; Sect. 3.2.2 and 4.3).  Against the indefinite oracle (LU with row
pivoting plus long-double refinement).

Tolerances: x is refined with double-double residuals, so
``||x - x_o|| / ||x_o|| <= 1e-11``; the diagonal of A^-1 is not refined and
its entries may be near zero or negative, so it is compared normwise:
``max|d - d_o| <= 1e-10 max|d_o|`` (the systems here have condition numbers
up to about 1e5).  Mixed precision (binary32 products in the root sweeps'
bulk, variances not refined): 1e-10 for x, and 1e-5 normwise for d, the
unit roundoff of binary32 (6e-8) times the condition number of these
systems (1e4..1e5) with a margin of ten below that product (measured:
1.4e-6).
"""
import sys

import numpy as np
import pytest

import spi_synth as synth
from oracle.indefinite import indefinite_solve

pytestmark = pytest.mark.gpu

TOL_X, TOL_D = 1e-11, 1e-10
TOL_X_MIXED, TOL_D_MIXED = 1e-10, 1e-5


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(p, block=None, **opts):
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver
    dev = torch.device("cuda")
    s = SpiSolver(p.m, p.n, p.rowptr, p.col, **opts)
    if block:
        s.potrf_block = block
    s.set_values(torch.from_numpy(p.val).to(dev), torch.from_numpy(p.w).to(dev))
    s.factor()
    b = s.rhs(torch.from_numpy(p.y).to(dev))
    x = s.solve(b)
    d = s.diag_inv()
    torch.cuda.synchronize()
    out = {"x": x.cpu().numpy(), "d": d.cpu().numpy(), "info": s.info()}
    s.close()
    return out


def _check(g, o, tol_x=TOL_X, tol_d=TOL_D):
    ex = np.linalg.norm(g["x"] - o["x"]) / np.linalg.norm(o["x"])
    ed = np.max(np.abs(g["d"] - o["diag"])) / np.max(np.abs(o["diag"]))
    _say(f"  err_x={ex:.2e} err_d={ed:.2e} refine={g['info']['refine_steps_done']}")
    assert ex <= tol_x
    assert ed <= tol_d


# (groups, leaf/group, root, rows/leaf, root/row, negative rows, zero-diagonal
# unknowns, seed, outer block)
CASES = [
    (8, 4, 150, 3, 8, 80, 0, 1, None),    # negative weights only
    (8, 4, 150, 3, 8, 0, 6, 2, None),     # zero diagonal: 2 x 2 pivots
    (10, 5, 700, 3, 10, 300, 12, 3, 128),  # several bands of 128 (padded 768)
    (10, 5, 700, 3, 10, 300, 12, 4, 512),  # two bands of 512
    (10, 5, 1300, 3, 10, 500, 12, 5, 1024),  # bands of 1024 and 384
]


def _leaf_work(c):
    # the leaf unknowns' work; every root unknown's is at least n_root
    return c[3] * (1 + c[4])


@pytest.mark.parametrize("case", CASES, ids=[f"indef{i}" for i in range(len(CASES))])
def test_indefinite_parity(case):
    ng, lpg, nr, rpl, rpr, neg, zd, seed, block = case
    p = synth.make_indefinite(ng, lpg, nr, rpl, rpr, neg, zd, seed)
    o = indefinite_solve(p)
    assert np.min(np.linalg.eigvalsh(o["A"])) < 0.0
    _say(f"case indefinite seed={seed} m={p.m} n={p.n} block={block}")
    g = _run(p, block, indefinite=1, leaf_max_work=_leaf_work(case))
    assert g["info"]["n_leaf"] == ng * lpg
    _check(g, o)


def test_indefinite_mixed_precision():
    c = CASES[2]
    p = synth.make_indefinite(*c[:8])
    o = indefinite_solve(p)
    _say(f"case indefinite mixed m={p.m} n={p.n}")
    g = _run(p, 256, indefinite=1, precision=1, leaf_max_work=_leaf_work(c))
    assert g["info"]["precision"] == 1
    _check(g, o, TOL_X_MIXED, TOL_D_MIXED)


def test_indefinite_route_on_a_definite_system():
    """Positive weights: the indefinite route gives the definite results."""
    from oracle import oracle_solve
    p = synth.make_random_leafy(10, 5, 300, 3, 10, 100, seed=6)
    o = oracle_solve(p)
    _say(f"case indefinite route, definite system n={p.n}")
    g = _run(p, 128, indefinite=1)
    assert np.linalg.norm(g["x"] - o["x"]) / np.linalg.norm(o["x"]) <= 1e-12
    assert np.max(np.abs(g["d"] - o["diag"]) / o["diag"]) <= 1e-12


def test_definite_route_reports_an_indefinite_root():
    """Without indefinite = 1 a root pivot that is not positive is reported,
    as for any matrix that is not positive definite."""
    from paper_1305_5683_amd import SpiError
    c = CASES[1]
    p = synth.make_indefinite(*c[:8])
    _say("case definite route on an indefinite root")
    with pytest.raises(SpiError):
        _run(p, leaf_max_work=_leaf_work(c))


def test_singular_root_block_is_reported():
    """A root unknown whose coefficients are all zero (its structure kept)
    leaves a zero row and column in A: reported, not pivoted."""
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver, SpiError
    c = CASES[0]
    p = synth.make_indefinite(*c[:8])
    j = p.n_bg + 5
    val = p.val.copy()
    val[p.col == j] = 0.0
    dev = torch.device("cuda")
    _say(f"case singular root unknown j={j}")
    s = SpiSolver(p.m, p.n, p.rowptr, p.col, indefinite=1,
                  leaf_max_work=_leaf_work(c))
    s.set_values(torch.from_numpy(val).to(dev), torch.from_numpy(p.w).to(dev))
    with pytest.raises(SpiError):
        s.factor()
    s.close()
