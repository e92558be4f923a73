"""GPU: the allocation-free variances call (spi_diag_inv_noalloc).

It runs the kernels of spi_diag_inv with the selected inversion's partial
sums in the library's fixed device array, so on the same factor it must
give the same variances as spi_diag_inv, bit for bit (same kernels, same
order of every sum).  Two calls in a row, the second on a smaller system,
check that the shared array carries nothing from one call to the next; a
system that needs more scratch than the array holds is refused with
SPI_E_ARG; both also against the FP64 oracle at 1e-12.
"""
import sys

import numpy as np
import pytest

import spi_synth as synth
from oracle import oracle_solve

pytestmark = pytest.mark.gpu

SCRATCH_DOUBLES = 1 << 23


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _factored(p, **opts):
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver
    s = SpiSolver(p.m, p.n, p.rowptr, p.col, **opts)
    s.set_values(torch.from_numpy(p.val).cuda(), torch.from_numpy(p.w).cuda())
    s.factor()
    return s


def _part_doubles(p, **opts):
    """Partial sums the selected inversion needs: for every leaf front,
    (tasks = T (T + 1) / 2 over T = ceil(|U| / 64) blocks) x (its columns),
    counted on the host from the analysis' column-to-front map."""
    import scipy.sparse as sp
    from paper_1305_5683_amd import symbolic
    info, _, _, front = symbolic(p.m, p.n, p.rowptr, p.col, **opts)
    Hb = sp.csr_matrix((np.ones(p.nnz), p.col, p.rowptr), shape=(p.m, p.n))
    leaf = front >= 0
    G = sp.csr_matrix((np.ones(int(leaf.sum())), (front[leaf], np.nonzero(leaf)[0])),
                      shape=(info["n_groups"], p.n))
    widths = np.diff(((G @ Hb.T) @ Hb[:, ~leaf]).tocsr().indptr)
    cols = np.bincount(front[leaf], minlength=info["n_groups"])
    t = -(-widths // 64)
    return int(np.sum(t * (t + 1) // 2 * cols))


def test_noalloc_variances_match_diag_inv_twice():
    torch = _torch()
    cases = [("large-shape", synth.make_problem(
                 synth.SkyConfig("noalloc-s40", 40, 700, 31, 0), seed=5)),
             ("tiny", synth.make_config(0))]
    for name, p in cases:
        need = _part_doubles(p)
        _say(f"case noalloc {name} m={p.m} n={p.n} scratch {need} doubles")
        assert 0 < need <= SCRATCH_DOUBLES
        s = _factored(p)
        d_ref = s.diag_inv().cpu().numpy()
        out = torch.full((p.n,), float("nan"), dtype=torch.float64, device="cuda")
        s.diag_inv_noalloc(out)
        torch.cuda.synchronize()
        d = out.cpu().numpy()
        assert np.array_equal(d, d_ref)
        o = oracle_solve(p)
        assert np.max(np.abs(d - o["diag"]) / o["diag"]) <= 1e-12
        s.close()


def test_noalloc_refuses_more_than_its_array():
    from paper_1305_5683_amd import SpiError
    p = synth.make_config(1)
    opts = {"max_group": 64, "amalg_density": 0.0}
    need = _part_doubles(p, **opts)
    _say(f"case noalloc refusal medium max_group=64: {need} doubles")
    assert need > SCRATCH_DOUBLES
    s = _factored(p, **opts)
    torch = _torch()
    out = torch.empty(p.n, dtype=torch.float64, device="cuda")
    with pytest.raises(SpiError) as ei:
        s.diag_inv_noalloc(out)
    assert ei.value.status == 1
    s.close()
