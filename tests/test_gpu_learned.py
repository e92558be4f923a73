"""GPU: learned preconditioner and FP32 PCG through the C ABI.

* The loss and gradient of the network come from the library's own forward
  and backward kernels. They must match the FP64 CPU oracle
  (``oracle.learned``). The oracle is written from the definitions and
  pinned by finite differences. Tolerances follow from binary32 network
  arithmetic: 1e-5 relative on the loss, 1e-3 of the largest gradient
  component on each component.
* PCG (binary32 inner iterations, binary64 residual passes) reaches a
  relative residual of 1e-10, and x matches the oracle's direct solution at
  that level.
* An iteration cap forces the multifrontal fallback, whose result is FP64
  exact.
* Gain: a network trained on early bands cuts the PCG iterations on later,
  drifted bands compared with the same PCG and base preconditioner without
  the correction.
"""
import sys

import numpy as np
import pytest

import spi_synth as synth
from oracle import learned as L
from oracle import normal_equations, oracle_solve

pytestmark = pytest.mark.gpu

HID = 16


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _solver(p, **opts):
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver
    dev = torch.device("cuda")
    s = SpiSolver(p.m, p.n, p.rowptr, p.col, **opts)
    s.set_values(torch.from_numpy(p.val).to(dev), torch.from_numpy(p.w).to(dev))
    return s


def _band(base, b, n_bands=256):
    rs, bs = synth.band_scales_drift(b, n_bands)
    return synth.make_band(base, rs, bs, seed=1000 + b)


def _dense(p):
    A, rhs = normal_equations(p.rowptr, p.col, p.val, p.w, p.y, p.n)
    A = A.toarray() if hasattr(A, "toarray") else np.asarray(A)
    return A, np.asarray(rhs)


@pytest.mark.parametrize("eq", [1, 0])
def test_loss_and_gradient_match_oracle(eq):
    torch = _torch()
    from paper_1305_5683_amd import SpiLearnedPrecond, symbolic
    # a small coded-mask system: its background unknowns (the first n_bg
    # columns) are the leaves of both the oracle's own ordering and the
    # library's analysis, the sky pixels the root
    base = synth.make_problem(synth.SkyConfig("lp-grad", 10, 60, 5, 4), seed=11)
    ref_p, band_p = _band(base, 0), _band(base, 96)
    _say(f"case lp-grad eq={eq} n={base.n}")
    ref = _solver(ref_p, equilibrate=eq)
    ref.factor()
    band = _solver(band_p, equilibrate=eq)
    band.factor()
    rhs = band.rhs(torch.from_numpy(band_p.y).cuda())
    x = band.solve(rhs)
    params = synth.lp_init_params(HID, seed=2)
    params[-3:] = [-0.3, 0.05, 0.1]
    lp = SpiLearnedPrecond(HID, params)
    loss, grad = lp.loss_grad(band, ref, rhs, x)
    # oracle, from its own normal equations, right-hand side and kinds
    Ar, _ = _dense(ref_p)
    Ab, rhs_o = _dense(band_p)
    is_root = (np.arange(base.n) >= base.n_bg).astype(np.float64)
    _, _, _, front = symbolic(base.m, base.n, base.rowptr, base.col)
    assert np.array_equal(front < 0, is_root > 0)    # the library's split agrees
    assert np.max(np.abs(rhs.cpu().numpy() - rhs_o)) <= 1e-14 * np.max(np.abs(rhs_o))
    phi = L.features(np.diag(Ab), np.diag(Ar), is_root)
    Ari = np.linalg.inv(Ar)
    x_o = np.linalg.solve(Ab, rhs_o)
    loss_o, grad_o = L.loss_grad(params.astype(np.float64), phi, rhs_o, x_o,
                                 lambda v: Ari @ v, lambda v: Ab @ v, HID)
    gs = np.max(np.abs(grad_o))
    _say(f"  loss {loss:.6e} oracle {loss_o:.6e}; max grad diff "
         f"{np.max(np.abs(grad - grad_o)) / gs:.2e} of max|grad|")
    assert abs(loss - loss_o) <= 1e-5 * loss_o
    assert np.max(np.abs(grad - grad_o)) <= 1e-3 * gs
    lp.close()
    ref.close()
    band.close()


def test_pcg_reaches_tolerance_and_matches_oracle():
    torch = _torch()
    from paper_1305_5683_amd import SpiLearnedPrecond, pcg_solve
    base = synth.make_config(0)
    ref_p, band_p = _band(base, 31), _band(base, 160)
    _say(f"case pcg tiny n={base.n}")
    ref = _solver(ref_p)
    ref.factor()
    band = _solver(band_p)
    rhs = band.rhs(torch.from_numpy(band_p.y).cuda())
    o = oracle_solve(band_p, want_diag=False)
    for lp in (None, SpiLearnedPrecond(HID, synth.lp_init_params(HID, 0))):
        x, info = pcg_solve(band, ref, rhs, lp=lp, tol=1e-10, maxit=300)
        ex = np.linalg.norm(x.cpu().numpy() - o["x"]) / np.linalg.norm(o["x"])
        _say(f"  lp={'yes' if lp else 'no '} {info} err_x={ex:.2e}")
        assert info["fell_back"] == 0
        assert info["rel_residual"] <= 1e-10
        assert ex <= 1e-9
    ref.close()
    band.close()


def test_pcg_fallback_is_direct_and_exact():
    torch = _torch()
    from paper_1305_5683_amd import pcg_solve
    base = synth.make_config(0)
    ref_p, band_p = _band(base, 31), _band(base, 200)
    _say("case pcg fallback tiny")
    ref = _solver(ref_p)
    ref.factor()
    band = _solver(band_p)
    rhs = band.rhs(torch.from_numpy(band_p.y).cuda())
    x, info = pcg_solve(band, ref, rhs, tol=1e-10, maxit=1)
    o = oracle_solve(band_p, want_diag=False)
    ex = np.linalg.norm(x.cpu().numpy() - o["x"]) / np.linalg.norm(o["x"])
    _say(f"  {info} err_x={ex:.2e}")
    assert info["fell_back"] == 1
    assert ex <= 1e-12 and info["rel_residual"] <= 1e-13
    # a tolerance even the direct fallback cannot meet: SPI_E_NOCONV
    from paper_1305_5683_amd import SpiError
    _say("case pcg fallback misses tol=1e-30")
    with pytest.raises(SpiError) as ei:
        pcg_solve(band, ref, rhs, tol=1e-30, maxit=1)
    assert ei.value.status == 6
    ref.close()
    band.close()


def test_trained_network_reduces_iterations():
    """Train on bands 0..30 against the factor of band 31 (GPU kernels),
    then compare PCG iterations on drifted later bands with and without the
    correction."""
    torch = _torch()
    from paper_1305_5683_amd import SpiLearnedPrecond, pcg_solve
    cfg = synth.SkyConfig("lp-small", 30, 600, 11, 4)
    base = synth.make_problem(cfg, seed=5)
    _say(f"case lp-gain m={base.m} n={base.n}")
    ref_p = _band(base, 31)
    ref = _solver(ref_p)
    ref.factor()
    work = _solver(ref_p)
    lp = SpiLearnedPrecond(HID, synth.lp_init_params(HID, 0))
    data = []
    for b in range(0, 31, 3):
        bp = _band(base, b)
        work.set_values(torch.from_numpy(bp.val).cuda(), torch.from_numpy(bp.w).cuda())
        work.factor()
        rhs = work.rhs(torch.from_numpy(bp.y).cuda())
        data.append((bp, rhs, work.solve(rhs).clone()))
    losses = []
    for epoch in range(40):
        tot = 0.0
        for bp, rhs, x in data:
            work.set_values(torch.from_numpy(bp.val).cuda(),
                            torch.from_numpy(bp.w).cuda())
            tot += lp.train_step(work, ref, rhs, x, lr=0.02)
        losses.append(tot / len(data))
    _say(f"  train loss {losses[0]:.3e} -> {losses[-1]:.3e}")
    assert losses[-1] < 0.5 * losses[0]
    it0 = it1 = 0
    for b in (64, 128, 192, 240):
        bp = _band(base, b)
        work.set_values(torch.from_numpy(bp.val).cuda(), torch.from_numpy(bp.w).cuda())
        rhs = work.rhs(torch.from_numpy(bp.y).cuda())
        _, i0 = pcg_solve(work, ref, rhs, lp=None, tol=1e-10, maxit=400)
        _, i1 = pcg_solve(work, ref, rhs, lp=lp, tol=1e-10, maxit=400)
        _say(f"  band {b}: iterations without {i0['iterations']} with {i1['iterations']}")
        assert i0["fell_back"] == 0 and i1["fell_back"] == 0
        it0 += i0["iterations"]
        it1 += i1["iterations"]
    _say(f"  total iterations without {it0} with {it1}")
    assert it1 <= 0.8 * it0
    lp.close()
    ref.close()
    work.close()


def test_trained_network_reduces_iterations_on_the_medium_pattern():
    """The learned workload's recipe on its pattern: bands on the medium
    configuration (33,750 unknowns), trained on bands 0..30 for 20 epochs
    against the factor of band 31; the correction reduces the PCG
    iterations on later, drifted bands (64, 128, 192) by at least a fifth,
    with no fallback."""
    torch = _torch()
    from paper_1305_5683_amd import SpiLearnedPrecond, pcg_solve
    base = synth.make_config(1)
    _say(f"case lp-gain, medium pattern m={base.m} n={base.n}")
    ref_p = _band(base, 31)
    ref = _solver(ref_p)
    ref.factor()
    work = _solver(ref_p)
    lp = SpiLearnedPrecond(HID, synth.lp_init_params(HID, 0))
    data = []
    for b in range(31):
        bp = _band(base, b)
        work.set_values(torch.from_numpy(bp.val).cuda(), torch.from_numpy(bp.w).cuda())
        work.factor()
        rhs = work.rhs(torch.from_numpy(bp.y).cuda())
        data.append((bp, rhs, work.solve(rhs).clone()))
    vals = [(torch.from_numpy(bp.val).cuda(), torch.from_numpy(bp.w).cuda())
            for bp, _, _ in data]
    losses = []
    for epoch in range(20):
        tot = 0.0
        for (val, w), (_, rhs, x) in zip(vals, data):
            work.set_values(val, w)
            tot += lp.train_step(work, ref, rhs, x, lr=0.02)
        losses.append(tot / len(data))
    _say(f"  train loss {losses[0]:.3e} -> {losses[-1]:.3e}")
    assert losses[-1] < 0.5 * losses[0]
    it0 = it1 = 0
    for b in (64, 128, 192):
        bp = _band(base, b)
        work.set_values(torch.from_numpy(bp.val).cuda(), torch.from_numpy(bp.w).cuda())
        rhs = work.rhs(torch.from_numpy(bp.y).cuda())
        _, i0 = pcg_solve(work, ref, rhs, lp=None, tol=1e-10, maxit=400)
        _, i1 = pcg_solve(work, ref, rhs, lp=lp, tol=1e-10, maxit=400)
        _say(f"  band {b}: iterations without {i0['iterations']} with {i1['iterations']}")
        assert i0["fell_back"] == 0 and i1["fell_back"] == 0
        it0 += i0["iterations"]
        it1 += i1["iterations"]
    _say(f"  total iterations without {it0} with {it1}")
    assert it1 <= 0.8 * it0
    lp.close()
    ref.close()
    work.close()
