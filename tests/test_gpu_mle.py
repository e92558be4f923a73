"""GPU: the Poisson likelihood fit by Newton's method (App. A.1-A.2).

* The likelihood terms through the C ABI (C, the Newton weights y/e^2 and
  the right-hand side H^T (y/e - 1)) match the oracle's at the LSQ start.
* Every Newton iterate of the library's loop matches the oracle's (the
  likelihood C after each step, the final x and the variances from the
  final Hessian).  Tolerance: each step is an FP64 solve within 1e-12 of
  the oracle's and Newton contracts the errors of earlier steps; 1e-10
  relative bounds x and the variances, and C (about 1e7, summed over the
  rows) is compared at 1e-13 relative.
"""
import sys

import numpy as np
import pytest

import spi_synth as synth
from oracle import mle, oracle_solve

pytestmark = pytest.mark.gpu


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


def _gpu_lsq(p):
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver
    s = SpiSolver(p.m, p.n, p.rowptr, p.col)
    val = torch.from_numpy(p.val).cuda()
    y = torch.from_numpy(p.y).cuda()
    s.set_values(val, torch.from_numpy(p.w).cuda())
    s.factor()
    x = s.solve(s.rhs(y))
    return s, val, y, x


def test_terms_match_oracle():
    from paper_1305_5683_amd import mle_terms
    p = synth.make_config(0)
    _say(f"case likelihood terms tiny m={p.m} n={p.n}")
    s, val, y, x = _gpu_lsq(p)
    xo = oracle_solve(p, want_diag=False)["x"]
    C, w, g = mle_terms(s, val, y, x)
    e = mle.model(p.rowptr, p.col, p.val, xo)
    Co = mle.cash(e, p.y)
    go = -0.5 * mle.gradient(p, xo)
    wo = mle.hessian_weights(p, xo)
    ec, ew, eg = abs(C - Co) / abs(Co), _rel(w.cpu().numpy(), wo), \
        _rel(g.cpu().numpy(), go)
    _say(f"  err_C={ec:.2e} err_w={ew:.2e} err_g={eg:.2e} (|g| {np.max(np.abs(go)):.2e})")
    assert ec <= 1e-13 and ew <= 1e-10
    # g is a sum with cancellation (H^T of y/e - 1): its error is relative to
    # the size of the summed terms, not of g
    H = p.scipy_csr()
    scale = np.max(np.abs(H).T @ np.abs(p.y / e - 1.0))
    assert np.max(np.abs(g.cpu().numpy() - go)) <= 1e-10 * scale
    s.close()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("which", ["tiny", "medium"])
def test_newton_matches_oracle(which):
    from paper_1305_5683_amd import mle_newton
    p = synth.make_config(0 if which == "tiny" else 1)
    _say(f"case likelihood Newton {which} m={p.m} n={p.n}")
    o = mle.newton(p)
    s, val, y, x = _gpu_lsq(p)
    x, d, hist = mle_newton(s, val, y, x)
    Co = np.array([it["C"] for it in o["iterates"]])
    ex, ed = _rel(x.cpu().numpy(), o["x"]), \
        float(np.max(np.abs(d.cpu().numpy() - o["diag"]) / o["diag"]))
    _say(f"  steps gpu {len(hist) - 1} oracle {len(Co) - 1}; "
         f"err_C={np.max(np.abs(hist - Co) / np.abs(Co)):.2e} err_x={ex:.2e} "
         f"err_d={ed:.2e}; C {Co[0]:.10e} -> {Co[-1]:.10e}")
    assert len(hist) == len(Co)
    assert np.max(np.abs(hist - Co) / np.abs(Co)) <= 1e-13
    assert ex <= 1e-10 and ed <= 1e-10
    s.close()
