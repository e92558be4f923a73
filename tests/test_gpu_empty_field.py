"""GPU: the empty-field loop (App. A.4-A.5) and the incremental
re-assembly of the root front after a change confined to the background
(leaf) columns (Sect. 4.1, modified columns of H).

* Every pass of Algorithm 1 driven through the C ABI (pattern update,
  spi_set_leaf_values, factor, solve) matches the oracle's passes: x, the
  pattern U and chi^2.  Tolerance: each pass's FP64 solve is within 1e-12
  of the oracle's, the pattern update (a ratio of two sums over about a
  tenth of the rows) and the next pass's matrix carry that error forward,
  and the passes contract; 1e-10 relative bounds the chain with a margin
  (the errors are printed).
* The loop call gives the oracle's pass count, chi^2 history, final x and
  U and the final variances.
* With keep_root_sum the factorisation after spi_set_leaf_values starts
  from the kept A_RR (assembly mode 2) and gives the full assembly's x and
  variances; if a root entry changed as well, it assembles everything.
"""
import dataclasses
import sys

import numpy as np
import pytest

import spi_synth as synth
from oracle import empty_field as ef
from oracle import oracle_solve

pytestmark = pytest.mark.gpu

TOL_CHAIN = 1e-10
# small enough for the oracle, and every sky pixel seen in enough rows that
# the analysis makes exactly the background (bin) columns leaves
CFG_TINY = synth.SkyConfig("ef-tiny", 14, 300, 9, 3)
CFG_MEDIUM = synth.CONFIGS[1]


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _setup(p, **opts):
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver, EmptyField, symbolic
    ptr, rows, unit = synth.empty_field_groups(p)
    _, _, _, front = symbolic(p.m, p.n, p.rowptr, p.col)
    assert np.array_equal(front >= 0, np.arange(p.n) < p.n_bg)
    s = SpiSolver(p.m, p.n, p.rowptr, p.col, keep_root_sum=1, **opts)
    val = torch.from_numpy(p.val.copy()).cuda()
    s.set_values(val, torch.from_numpy(p.w).cuda())
    e = EmptyField(s, p.meta["bg_pos"], p.meta["t"], ptr, rows)
    return s, e, val, torch.from_numpy(p.y).cuda(), (ptr, rows, unit)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("which,passes", [("tiny", 6), ("medium", 3)])
def test_passes_match_oracle(which, passes):
    torch = _torch()
    cfg = CFG_TINY if which == "tiny" else CFG_MEDIUM
    p = synth.make_empty_field(cfg, seed=4)
    _say(f"case empty-field passes {which} m={p.m} n={p.n} passes={passes}")
    s, e, val, y, (ptr, rows, unit) = _setup(p)
    t, bg = p.meta["t"], p.meta["bg_pos"]
    U = torch.ones(len(ptr) - 1, dtype=torch.float64, device="cuda")
    Uo = np.ones(len(ptr) - 1)
    for i in range(passes):
        # oracle pass with its own pattern
        q = dataclasses.replace(p, val=ef.set_background(p.val, bg, t, unit, Uo))
        xo = oracle_solve(q, want_diag=False)["x"]
        co = ef.chi2(q.rowptr, q.col, q.val, q.w, q.y, xo)
        # GPU pass: the values val carry U (set by the previous update)
        s.set_leaf_values(val)
        s.factor()
        mode = s.info()["root_assembly_mode"]
        x = s.solve(s.rhs(y))
        Ug = U.cpu().numpy().copy()
        c = e.update(val, y, x, U)
        ex, eu, ec = _rel(x.cpu().numpy(), xo), _rel(Ug, Uo), abs(c - co) / co
        _say(f"  pass {i}: assembly mode {mode} err_x={ex:.2e} err_U={eu:.2e} "
             f"err_chi2={ec:.2e} chi2={c:.6e}")
        assert mode == (1 if i == 0 else 2)
        assert ex <= TOL_CHAIN and eu <= TOL_CHAIN and ec <= TOL_CHAIN
        Uo = ef.pattern_update(q.rowptr, q.col, q.val, q.w, q.y, xo, bg, t, ptr,
                               rows, Uo)
    vv = val.cpu().numpy()
    assert _rel(vv[bg], (Uo[unit] * t)) <= TOL_CHAIN   # background entries U t
    s.close()


@pytest.mark.timeout(900)
def test_loop_call_matches_oracle_loop():
    torch = _torch()
    p = synth.make_empty_field(CFG_TINY, seed=5)
    _say(f"case empty-field loop call tiny m={p.m} n={p.n}")
    s, e, val, y, (ptr, rows, unit) = _setup(p)
    t, bg = p.meta["t"], p.meta["bg_pos"]
    o = ef.empty_field_loop(p, np.ones(len(ptr) - 1), ptr, rows, unit, t, bg,
                            itermax=25, rtol=1e-9)
    U = torch.ones(len(ptr) - 1, dtype=torch.float64, device="cuda")
    x, d, hist = e.loop(val, y, U, itermax=25, rtol=1e-9)
    co = np.array([ps["chi2"] for ps in o["passes"]])
    _say(f"  passes gpu {len(hist)} oracle {len(co)}; chi2 {hist[-1]:.6e}; "
         f"err_x={_rel(x.cpu().numpy(), o['x']):.2e} "
         f"err_U={_rel(U.cpu().numpy(), o['U']):.2e} "
         f"err_d={_rel(d.cpu().numpy(), o['diag']):.2e}")
    assert len(hist) == len(co)
    assert np.max(np.abs(hist - co) / co) <= TOL_CHAIN
    assert _rel(x.cpu().numpy(), o["x"]) <= TOL_CHAIN
    assert _rel(U.cpu().numpy(), o["U"]) <= TOL_CHAIN
    assert np.max(np.abs(d.cpu().numpy() - o["diag"]) / o["diag"]) <= TOL_CHAIN
    s.close()


def test_incremental_reassembly_matches_full():
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver
    p = synth.make_empty_field(CFG_TINY, seed=6)
    _say(f"case incremental re-assembly tiny m={p.m} n={p.n}")
    bg = p.meta["bg_pos"]
    val2 = p.val.copy()
    val2[bg] *= np.exp(np.random.default_rng(1).uniform(-0.3, 0.3, len(bg)))
    w = torch.from_numpy(p.w).cuda()
    y = torch.from_numpy(p.y).cuda()
    from paper_1305_5683_amd import symbolic
    _, _, _, front = symbolic(p.m, p.n, p.rowptr, p.col)
    assert np.array_equal(front >= 0, np.arange(p.n) < p.n_bg)
    s = SpiSolver(p.m, p.n, p.rowptr, p.col, keep_root_sum=1)
    s.set_values(torch.from_numpy(p.val).cuda(), w)
    s.factor()
    assert s.info()["root_assembly_mode"] == 1
    s.set_leaf_values(torch.from_numpy(val2).cuda())
    s.factor()
    assert s.info()["root_assembly_mode"] == 2
    x = s.solve(s.rhs(y)).cpu().numpy()
    d = s.diag_inv().cpu().numpy()
    o = oracle_solve(dataclasses.replace(p, val=val2))
    ex, ed = _rel(x, o["x"]), np.max(np.abs(d - o["diag"]) / o["diag"])
    _say(f"  incremental vs oracle: err_x={ex:.2e} err_d={ed:.2e}")
    assert ex <= 1e-12 and ed <= 1e-12
    # a root (sky) entry changed too: everything is assembled again
    val3 = val2.copy()
    val3[bg[5] + 1] *= 1.5
    s.set_leaf_values(torch.from_numpy(val3).cuda())
    s.factor()
    assert s.info()["root_assembly_mode"] == 1
    x = s.solve(s.rhs(y)).cpu().numpy()
    o = oracle_solve(dataclasses.replace(p, val=val3), want_diag=False)
    assert _rel(x, o["x"]) <= 1e-12
    s.close()
