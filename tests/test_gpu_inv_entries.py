"""GPU: general entries of A^-1 (covariances) through the C ABI, against
the oracle's blocked solves with its block factor (pinned against the exact
inverse and the paper's pruned traversal) at the FP64 bar, 1e-12 of the
largest entry of A^-1 compared: pairs of two root unknowns, a leaf and a
root unknown either way round, two leaves of one front and of two fronts,
and diagonal entries (which must equal spi_diag_inv)."""
import sys

import numpy as np
import pytest

import spi_synth as synth
from oracle import BlockCholesky, normal_equations

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _pairs(p, front, rng, k):
    """k pairs of each kind, from the analysis' column-to-front map (index
    bookkeeping only)."""
    leaf = np.nonzero(front >= 0)[0]
    root = np.nonzero(front < 0)[0]
    out = []
    if len(root):
        out.append((rng.choice(root, k), rng.choice(root, k)))
    if len(root) and len(leaf):
        a, b = rng.choice(leaf, k), rng.choice(root, k)
        out += [(a, b), (b, a)]
    if len(leaf):
        a = rng.choice(leaf, k)
        same = np.array([rng.choice(np.nonzero(front == front[x])[0]) for x in a])
        out += [(a, same), (rng.choice(leaf, k), rng.choice(leaf, k))]
    d = rng.choice(p.n, k)
    out.append((d, d))
    return np.concatenate([o[0] for o in out]), np.concatenate([o[1] for o in out])


CASES = [("tiny", None, {}), ("tiny-cholesky", None, {"root_inverse": 0}),
         ("leafy", (30, 3, 200, 4, 30, 0, 2), {}), ("medium", 1, {})]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_inverse_entries_match_oracle(case):
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver, symbolic
    name, shape, opts = case
    if shape is None:
        p = synth.make_config(0)
    elif isinstance(shape, int):
        p = synth.make_config(shape)
    else:
        p = synth.make_random_leafy(*shape)
    _, _, _, front = symbolic(p.m, p.n, p.rowptr, p.col)
    rng = np.random.default_rng(11)
    rows, cols = _pairs(p, front, rng, 40 if name == "medium" else 60)
    _say(f"case inverse entries {name} n={p.n}: {len(rows)} pairs")
    s = SpiSolver(p.m, p.n, p.rowptr, p.col, **opts)
    s.set_values(torch.from_numpy(p.val).cuda(), torch.from_numpy(p.w).cuda())
    s.factor()
    g = s.inv_entries(torch.from_numpy(rows.astype(np.int32)).cuda(),
                      torch.from_numpy(cols.astype(np.int32)).cuda()).cpu().numpy()
    d = s.diag_inv().cpu().numpy()
    A, _ = normal_equations(p.rowptr, p.col, p.val, p.w, p.y, p.n)
    f = BlockCholesky(A, p.n_bg)
    o = f.inverse_entries(rows, cols)
    err = np.max(np.abs(g - o)) / np.max(np.abs(o))
    _say(f"  max err {err:.2e} of max |entry| {np.max(np.abs(o)):.3e}")
    assert err <= 1e-12
    diag = rows == cols
    assert np.max(np.abs(g[diag] - d[rows[diag]]) / d[rows[diag]]) <= 1e-13
    s.close()


def test_inverse_entries_argument_checks():
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver, SpiError
    p = synth.make_config(0)
    s = SpiSolver(p.m, p.n, p.rowptr, p.col)
    r = torch.tensor([0, 1], dtype=torch.int32, device="cuda")
    with pytest.raises(SpiError) as ei:       # no factor yet
        s.inv_entries(r, r)
    assert ei.value.status == 2
    s.set_values(torch.from_numpy(p.val).cuda(), torch.from_numpy(p.w).cuda())
    s.factor()
    bad = torch.tensor([0, p.n], dtype=torch.int32, device="cuda")
    with pytest.raises(SpiError) as ei:
        s.inv_entries(r, bad)
    assert ei.value.status == 1
    assert s.inv_entries(r[:0], r[:0]).numel() == 0
    s.close()
