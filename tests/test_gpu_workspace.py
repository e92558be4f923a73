"""Workspace hygiene and repeatability.

* Poisoned workspaces: every device work buffer of a handle is overwritten
  with NaN bytes right after the analysis (`spi_debug_poison`); the results
  of each route must still match the oracle at its usual tolerance, so no
  result depends on a buffer's earlier contents (uninitialised memory,
  stale padding, a flag not reset).
* Repeatability: two runs on the same handle (the second after poisoning
  again).  b = H^T W y is a fixed-order sum and must agree bit for bit; x
  and the variances pass through the root assembly, whose LDS additions
  come in no fixed order, so they agree to rounding (1e-13), not bitwise.
"""
import sys

import numpy as np
import pytest

import spi_synth as synth
from oracle import oracle_solve
from oracle.indefinite import indefinite_solve

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _pipeline(s, p, torch):
    dev = torch.device("cuda")
    s.set_values(torch.from_numpy(p.val).to(dev), torch.from_numpy(p.w).to(dev))
    s.factor()
    b = s.rhs(torch.from_numpy(p.y).to(dev))
    x = s.solve(b)
    d = s.diag_inv()
    torch.cuda.synchronize()
    return b.cpu().numpy(), x.cpu().numpy(), d.cpu().numpy()


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


ROUTES = [
    ("fp64", {}, 1e-12, 1e-12),
    ("mixed", {"precision": 1}, 1e-10, 1e-6),
    ("cholesky", {"root_inverse": 0}, 1e-12, 1e-12),
    ("tile128", {"asm_tile": 128}, 1e-12, 1e-12),
]


@pytest.mark.parametrize("route", ROUTES, ids=[r[0] for r in ROUTES])
def test_poisoned_workspace(route):
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver
    name, opts, tx, td = route
    p = synth.make_random_leafy(12, 7, 600, 3, 25, 50, seed=5)
    o = oracle_solve(p)
    _say(f"case poisoned workspace route={name} n={p.n}")
    s = SpiSolver(p.m, p.n, p.rowptr, p.col, **opts)
    s.debug_poison()
    b, x, d = _pipeline(s, p, torch)
    s.close()
    ex, ed = _rel(x, o["x"]), np.max(np.abs(d - o["diag"]) / o["diag"])
    _say(f"  err_x={ex:.2e} err_d={ed:.2e}")
    assert np.all(np.isfinite(x)) and np.all(np.isfinite(d))
    assert ex <= tx and ed <= td


def test_poisoned_workspace_indefinite():
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver
    p = synth.make_indefinite(10, 5, 700, 3, 10, 300, 12, 3)
    o = indefinite_solve(p)
    _say(f"case poisoned workspace, indefinite n={p.n}")
    s = SpiSolver(p.m, p.n, p.rowptr, p.col, indefinite=1, leaf_max_work=33)
    s.potrf_block = 128
    s.debug_poison()
    _, x, d = _pipeline(s, p, torch)
    s.close()
    ex = _rel(x, o["x"])
    ed = np.max(np.abs(d - o["diag"])) / np.max(np.abs(o["diag"]))
    _say(f"  err_x={ex:.2e} err_d={ed:.2e}")
    assert ex <= 1e-11 and ed <= 1e-10


def test_poisoned_workspace_incremental_reassembly():
    """keep_root_sum: the kept A_RR is poisoned too; the first factorisation
    must rebuild it before a leaf-only update reuses it."""
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver
    p = synth.make_random_leafy(12, 7, 600, 3, 25, 50, seed=8)
    dev = torch.device("cuda")
    s = SpiSolver(p.m, p.n, p.rowptr, p.col, keep_root_sum=1)
    s.debug_poison()
    _pipeline(s, p, torch)
    # new leaf values (columns of the leaf unknowns only)
    val2 = p.val.copy()
    leaf = p.col < p.n_bg
    val2[leaf] *= 1.25
    q = synth.Problem(m=p.m, n=p.n, n_bg=p.n_bg, rowptr=p.rowptr, col=p.col,
                      val=val2, w=p.w, y=p.y, x_true=p.x_true, name="leaf2")
    s.set_leaf_values(torch.from_numpy(val2).to(dev))
    s.factor()
    assert s.info()["root_assembly_mode"] == 2
    b = s.rhs(torch.from_numpy(q.y).to(dev))
    x = s.solve(b).cpu().numpy()
    d = s.diag_inv().cpu().numpy()
    s.close()
    o = oracle_solve(q)
    _say(f"case poisoned workspace, leaf update: err_x={_rel(x, o['x']):.2e}")
    assert _rel(x, o["x"]) <= 1e-12
    assert np.max(np.abs(d - o["diag"]) / o["diag"]) <= 1e-12


def test_repeatability():
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver
    p = synth.make_config(0)
    s = SpiSolver(p.m, p.n, p.rowptr, p.col)
    b1, x1, d1 = _pipeline(s, p, torch)
    s.debug_poison()
    b2, x2, d2 = _pipeline(s, p, torch)
    s.close()
    _say(f"case repeatability: x {_rel(x2, x1):.1e}, d "
         f"{np.max(np.abs(d2 - d1) / d1):.1e}")
    assert np.array_equal(b1, b2)
    assert _rel(x2, x1) <= 1e-13
    assert np.max(np.abs(d2 - d1) / d1) <= 1e-13


def test_device_memory_cap():
    """opts.device_mem_cap: a handle that needs more device memory than the
    cap is refused with SPI_E_OOM (nothing allocated beyond it, nothing
    left); at exactly what spi_info.device_bytes reports it is built and
    matches the oracle."""
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver, SpiError
    p = synth.make_random_leafy(12, 7, 600, 3, 25, 50, seed=5)
    s = SpiSolver(p.m, p.n, p.rowptr, p.col)
    need = s.info()["device_bytes"]
    s.close()
    # the root front alone (n_pad^2 doubles) is part of it
    assert need >= 8 * 640 * 640
    _say(f"case device memory cap: the handle holds {need} bytes")
    for cap in (need - 1, need // 2, 1):
        with pytest.raises(SpiError) as ei:
            SpiSolver(p.m, p.n, p.rowptr, p.col, device_mem_cap=cap)
        assert ei.value.status == 4 and "cap" in str(ei.value)
    s = SpiSolver(p.m, p.n, p.rowptr, p.col, device_mem_cap=need)
    assert s.info()["device_bytes"] == need
    _, x, d = _pipeline(s, p, torch)
    s.close()
    o = oracle_solve(p)
    assert _rel(x, o["x"]) <= 1e-12
    assert np.max(np.abs(d - o["diag"]) / o["diag"]) <= 1e-12


def test_handle_from_an_analysis_file(tmp_path):
    """A handle read from an analysis file (spi_save_analysis, or the
    host-only spi_symbolic_save, then spi_analyze_load) gives the fresh
    handle's results: b bit for bit, x and the variances to rounding (1e-13:
    the root assembly's additions come in no fixed order).  The file's
    analysis options replace the caller's; the caller's others (mixed
    precision here) apply."""
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver, symbolic_save
    p = synth.make_random_leafy(12, 7, 600, 3, 25, 50, seed=5)
    s = SpiSolver(p.m, p.n, p.rowptr, p.col, max_group=8)
    i0 = s.info()
    b1, x1, d1 = _pipeline(s, p, torch)
    f1 = tmp_path / "saved.spia"
    s.save_analysis(f1)
    s.close()
    _say(f"case analysis file: {f1.stat().st_size} bytes, {i0['n_groups']} fronts")
    t = SpiSolver.from_analysis(f1)  # default options: max_group from the file
    i1 = t.info()
    for k in ("n_groups", "n_root", "n_root_padded", "nnz_l", "asm_tile"):
        assert i1[k] == i0[k], k
    b2, x2, d2 = _pipeline(t, p, torch)
    t.close()
    assert np.array_equal(b1, b2)
    assert _rel(x2, x1) <= 1e-13
    assert np.max(np.abs(d2 - d1) / d1) <= 1e-13
    f2 = tmp_path / "symbolic.spia"
    symbolic_save(p.m, p.n, p.rowptr, p.col, f2, max_group=8)
    u = SpiSolver.from_analysis(f2, precision=1)
    assert u.info()["precision"] == 1 and u.info()["n_groups"] == i0["n_groups"]
    _, x3, d3 = _pipeline(u, p, torch)
    u.close()
    o = oracle_solve(p)
    assert _rel(x3, o["x"]) <= 1e-10
    assert np.max(np.abs(d3 - o["diag"]) / o["diag"]) <= 1e-6
