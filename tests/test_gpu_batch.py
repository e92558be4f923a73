"""GPU: batches of systems, shared analyses and the POTRF autotuner.

Every system of a batch must give what it gives alone: x and diag(A^-1)
against the FP64 oracle at the FP64 tolerance (1e-12), for both eager and
graph runs, with graphs replayed on new values.  A failing pivot in one
system is reported for that system only.
"""
import sys

import numpy as np
import pytest

import spi_synth as synth
from oracle import oracle_solve

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _set(s, p):
    torch = _torch()
    s.set_values(torch.from_numpy(p.val).cuda(), torch.from_numpy(p.w).cuda())


def _systems():
    base = synth.make_config(0)
    bands = [synth.make_band(base, *synth.band_scales_drift(b, 64), seed=2000 + b)
             for b in (0, 21, 42)]
    subs = [synth.make_problem(c, seed=7 + i) for i, c in
            enumerate(synth.subproblem_configs(3, seed=3, side_lo=12, side_hi=24))]
    return base, bands, subs


def test_analyze_like_matches_fresh_analysis():
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver
    p = synth.make_config(0)
    _say("case analyze_like tiny")
    a = SpiSolver(p.m, p.n, p.rowptr, p.col)
    b = SpiSolver.like(a)
    out = []
    for s in (a, b):
        _set(s, p)
        s.factor()
        rhs = s.rhs(torch.from_numpy(p.y).cuda())
        out.append((s.solve(rhs).cpu().numpy(), s.diag_inv().cpu().numpy()))
    # the root assembly sums with LDS atomics, so two runs agree to
    # rounding, not bit for bit
    assert _rel(out[0][0], out[1][0]) <= 1e-13
    assert np.max(np.abs(out[0][1] - out[1][1]) / out[1][1]) <= 1e-13
    a.close()
    b.close()


@pytest.mark.parametrize("graphs", [0, 1])
def test_batch_matches_oracle(graphs):
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver, SpiBatch
    base, bands, subs = _systems()
    _say(f"case batch graphs={graphs}: 3 bands + 3 sub-problems")
    first = SpiSolver(base.m, base.n, base.rowptr, base.col,
                      stream=torch.cuda.Stream())
    solvers = [first] + [SpiSolver.like(first, stream=torch.cuda.Stream())
                         for _ in bands[1:]]
    solvers += [SpiSolver(q.m, q.n, q.rowptr, q.col, stream=torch.cuda.Stream())
                for q in subs]
    probs = bands + subs
    batch = SpiBatch(solvers, use_graphs=bool(graphs))
    y = [torch.from_numpy(q.y).cuda() for q in probs]
    rhs = [torch.empty(q.n, dtype=torch.float64, device="cuda") for q in probs]
    x = [torch.empty_like(r) for r in rhs]
    d = [torch.empty_like(r) for r in rhs]
    for rnd in range(2):
        if rnd == 1:   # new values on the same buffers: graphs are replayed
            probs = [synth.make_band(base, *synth.band_scales_drift(b, 64),
                                     seed=3000 + b) for b in (5, 26, 47)] + subs
            for i, q in enumerate(probs[:3]):
                y[i].copy_(torch.from_numpy(q.y))
        for s, q in zip(solvers, probs):
            _set(s, q)
        torch.cuda.synchronize()
        st = batch.run(y, rhs, x, d)
        assert st == [0] * len(probs)
        for i, q in enumerate(probs):
            o = oracle_solve(q)
            ex = _rel(x[i].cpu().numpy(), o["x"])
            ed = np.max(np.abs(d[i].cpu().numpy() - o["diag"]) / o["diag"])
            _say(f"  round {rnd} system {i} n={q.n}: err_x={ex:.2e} err_d={ed:.2e}")
            assert ex <= TOL and ed <= TOL
    batch.close()
    for s in solvers:
        s.close()


def test_batch_reports_failing_system_only():
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver, SpiBatch
    base, bands, subs = _systems()
    _say("case batch with one non-SPD system")
    solvers = [SpiSolver(q.m, q.n, q.rowptr, q.col, stream=torch.cuda.Stream())
               for q in (bands[0], subs[0])]
    _set(solvers[0], bands[0])
    bad = subs[0]
    solvers[1].set_values(torch.from_numpy(bad.val).cuda(),
                          torch.from_numpy(-bad.w).cuda())
    batch = SpiBatch(solvers, use_graphs=True)
    y = [torch.from_numpy(q.y).cuda() for q in (bands[0], bad)]
    rhs = [torch.empty(q.n, dtype=torch.float64, device="cuda") for q in (bands[0], bad)]
    x = [torch.empty_like(r) for r in rhs]
    st = batch.run(y, rhs, x)
    assert st[0] == 0 and st[1] == 3
    o = oracle_solve(bands[0], want_diag=False)
    assert _rel(x[0].cpu().numpy(), o["x"]) <= TOL
    batch.close()
    for s in solvers:
        s.close()


def test_autotune_picks_a_block_and_factor_stays_exact():
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver
    p = synth.make_random_leafy(10, 5, 700, 3, 30, 40, seed=9)
    _say(f"case autotune n={p.n}")
    s = SpiSolver(p.m, p.n, p.rowptr, p.col)
    _set(s, p)
    blk = s.autotune()
    _say(f"  chosen block {blk}, bulk tile {s.bulk_tile}")
    assert blk in (128, 256, 512, 1024) and s.potrf_block == blk
    assert s.bulk_tile in (64, 128)
    rhs = s.rhs(torch.from_numpy(p.y).cuda())
    x = s.solve(rhs).cpu().numpy()
    d = s.diag_inv().cpu().numpy()
    o = oracle_solve(p)
    assert _rel(x, o["x"]) <= TOL
    assert np.max(np.abs(d - o["diag"]) / o["diag"]) <= TOL
    for blk, tile in ((128, 64), (512, 128)):
        s.potrf_block, s.bulk_tile = blk, tile
        s.factor()
        x2 = s.solve(rhs).cpu().numpy()
        assert _rel(x2, o["x"]) <= TOL
    from paper_1305_5683_amd import SpiError
    with pytest.raises(SpiError):
        s.bulk_tile = 96
    s.close()


def test_batch_graphs_with_multiband_sweeps():
    """Outer block 128: the root sweeps run 2-4 bands (4 on the 400-pixel
    sky of the bands) with the side-stream lookahead, and the batch
    captures that fork and join in its graphs; replays on new values stay
    exact."""
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver, SpiBatch
    base, bands, subs = _systems()
    _say("case batch graphs, block 128: 3 bands + 3 sub-problems")
    first = SpiSolver(base.m, base.n, base.rowptr, base.col,
                      stream=torch.cuda.Stream())
    solvers = [first] + [SpiSolver.like(first, stream=torch.cuda.Stream())
                         for _ in bands[1:]]
    solvers += [SpiSolver(q.m, q.n, q.rowptr, q.col, stream=torch.cuda.Stream())
                for q in subs]
    for s in solvers:
        s.potrf_block = 128
        assert s.info()["n_root_padded"] >= 256
    probs = bands + subs
    batch = SpiBatch(solvers, use_graphs=True)
    y = [torch.from_numpy(q.y).cuda() for q in probs]
    rhs = [torch.empty(q.n, dtype=torch.float64, device="cuda") for q in probs]
    x = [torch.empty_like(r) for r in rhs]
    d = [torch.empty_like(r) for r in rhs]
    for rnd in range(3):
        for s, q in zip(solvers, probs):
            _set(s, q)
        torch.cuda.synchronize()
        assert batch.run(y, rhs, x, d) == [0] * len(probs)
        for i, q in enumerate(probs):
            o = oracle_solve(q)
            ex = _rel(x[i].cpu().numpy(), o["x"])
            ed = np.max(np.abs(d[i].cpu().numpy() - o["diag"]) / o["diag"])
            _say(f"  round {rnd} system {i} n={q.n}: err_x={ex:.2e} err_d={ed:.2e}")
            assert ex <= TOL and ed <= TOL
    batch.close()
    for s in solvers:
        s.close()


@pytest.mark.parametrize("graphs", [0, 1])
def test_mixed_batch_matches_oracle(graphs):
    """Mixed precision in a batch (binary32 root products, three fixed
    refinement steps, no read-back between them): x within 1e-10 and the
    variances within 1e-6 of the FP64 oracle, and the convergence check at
    the batch's synchronisation passes."""
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver, SpiBatch
    base, bands, subs = _systems()
    _say(f"case mixed batch graphs={graphs}: 3 bands + 3 sub-problems")
    opts = dict(precision=1, refine_tol=1e-14, refine_steps=3)
    first = SpiSolver(base.m, base.n, base.rowptr, base.col,
                      stream=torch.cuda.Stream(), **opts)
    solvers = [first] + [SpiSolver.like(first, stream=torch.cuda.Stream())
                         for _ in bands[1:]]
    solvers += [SpiSolver(q.m, q.n, q.rowptr, q.col, stream=torch.cuda.Stream(), **opts)
                for q in subs]
    probs = bands + subs
    batch = SpiBatch(solvers, use_graphs=bool(graphs))
    y = [torch.from_numpy(q.y).cuda() for q in probs]
    rhs = [torch.empty(q.n, dtype=torch.float64, device="cuda") for q in probs]
    x = [torch.empty_like(r) for r in rhs]
    d = [torch.empty_like(r) for r in rhs]
    for rnd in range(2):
        for s, q in zip(solvers, probs):
            _set(s, q)
        torch.cuda.synchronize()
        assert batch.run(y, rhs, x, d) == [0] * len(probs)
        for i, q in enumerate(probs):
            o = oracle_solve(q)
            ex = _rel(x[i].cpu().numpy(), o["x"])
            ed = np.max(np.abs(d[i].cpu().numpy() - o["diag"]) / o["diag"])
            info = solvers[i].info()
            _say(f"  round {rnd} system {i} n={q.n}: err_x={ex:.2e} err_d={ed:.2e} "
                 f"last correction {info['last_refine_norm']:.1e}")
            assert ex <= 1e-10 and ed <= 1e-6
            assert info["refine_steps_done"] == 3
    batch.close()
    for s in solvers:
        s.close()


def test_batch_reports_unconverged_refinement():
    """One refinement step cannot meet a refine_tol of 1e-300: the batch
    reports SPI_E_NOCONV for that system (x is still written) and SPI_OK
    for the others."""
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver, SpiBatch
    base, bands, subs = _systems()
    _say("case batch with an unreachable refine_tol")
    s0 = SpiSolver(base.m, base.n, base.rowptr, base.col, stream=torch.cuda.Stream())
    s1 = SpiSolver(base.m, base.n, base.rowptr, base.col, stream=torch.cuda.Stream(),
                   refine_tol=1e-300, refine_steps=1)
    for s in (s0, s1):
        _set(s, bands[0])
    batch = SpiBatch([s0, s1], use_graphs=False)
    y = [torch.from_numpy(bands[0].y).cuda()] * 2
    rhs = [torch.empty(base.n, dtype=torch.float64, device="cuda") for _ in range(2)]
    x = [torch.empty_like(r) for r in rhs]
    assert batch.run(y, rhs, x) == [0, 6]
    o = oracle_solve(bands[0], want_diag=False)
    for xi in x:
        assert _rel(xi.cpu().numpy(), o["x"]) <= TOL
    batch.close()
    s0.close()
    s1.close()


def test_batch_reports_nonfinite_input():
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver, SpiBatch
    base, bands, subs = _systems()
    _say("case batch with a NaN weight")
    s0 = SpiSolver(base.m, base.n, base.rowptr, base.col, stream=torch.cuda.Stream())
    s1 = SpiSolver.like(s0, stream=torch.cuda.Stream())
    _set(s0, bands[0])
    w = bands[1].w.copy()
    w[5] = np.nan
    s1.set_values(torch.from_numpy(bands[1].val).cuda(), torch.from_numpy(w).cuda())
    batch = SpiBatch([s0, s1], use_graphs=True)
    y = [torch.from_numpy(q.y).cuda() for q in bands[:2]]
    rhs = [torch.empty(base.n, dtype=torch.float64, device="cuda") for _ in range(2)]
    x = [torch.empty_like(r) for r in rhs]
    assert batch.run(y, rhs, x) == [0, 1]
    batch.close()
    s0.close()
    s1.close()


def test_mixed_batch_at_config_scale():
    """The batch workload's shapes: two energy bands on the medium pattern
    (33,750 unknowns, a 10,000-pixel root; drifted response and background
    scales, fresh counts) sharing one analysis, and two sub-problems of sky
    side 30 and 60, in one graph-replayed mixed-precision batch.  Against
    the FP64 oracle: x in full at 1e-10, the variances at 1e-6 on 96 sampled
    unknowns of each band (every one on the sub-problems)."""
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver, SpiBatch
    base = synth.make_config(1)
    bands = [synth.make_band(base, *synth.band_scales_drift(b, 64), seed=3000 + b)
             for b in (0, 40)]
    subs = [synth.make_problem(synth.SkyConfig(f"sub-s{s}", s, 4 * -(-s * s // 10), 17, 4),
                               seed=40 + s) for s in (30, 60)]
    _say(f"case mixed batch at config scale: bands n={base.n}, sub-problems "
         f"n={[q.n for q in subs]}")
    opts = dict(precision=1, refine_tol=1e-14, refine_steps=3)
    first = SpiSolver(base.m, base.n, base.rowptr, base.col,
                      stream=torch.cuda.Stream(), **opts)
    solvers = [first, SpiSolver.like(first, stream=torch.cuda.Stream())]
    solvers += [SpiSolver(q.m, q.n, q.rowptr, q.col, stream=torch.cuda.Stream(), **opts)
                for q in subs]
    probs = bands + subs
    for s, q in zip(solvers, probs):
        _set(s, q)
    batch = SpiBatch(solvers, use_graphs=True)
    y = [torch.from_numpy(q.y).cuda() for q in probs]
    rhs = [torch.empty(q.n, dtype=torch.float64, device="cuda") for q in probs]
    x = [torch.empty_like(r) for r in rhs]
    d = [torch.empty_like(r) for r in rhs]
    torch.cuda.synchronize()
    assert batch.run(y, rhs, x, d) == [0] * len(probs)
    rng = np.random.default_rng(7)
    for i, q in enumerate(probs):
        idx = None
        if q.n == base.n:
            idx = np.sort(np.concatenate([rng.choice(q.n_bg, 48, replace=False),
                                          q.n_bg + rng.choice(q.n - q.n_bg, 48,
                                                              replace=False)]))
        o = oracle_solve(q, diag_idx=idx)
        di = d[i].cpu().numpy()
        if idx is not None:
            di = di[idx]
        ex = _rel(x[i].cpu().numpy(), o["x"])
        ed = np.max(np.abs(di - o["diag"]) / o["diag"])
        _say(f"  system {i} n={q.n}: err_x={ex:.2e} err_d={ed:.2e}")
        assert ex <= 1e-10 and ed <= 1e-6
    batch.close()
    for s in solvers:
        s.close()


@pytest.mark.parametrize("graphs", [1, 0])
def test_mixed_batch_falls_back_to_fp64(graphs):
    """opts.fp64_fallback in a batch.  Beside a well-conditioned band, the
    near-collinear system of the parity tests (cond(A) about 5.6e8, root in
    its original order, bands of 128), whose mixed refinement stalls far
    above refine_tol = 1e-10, is redone alone in binary64 after the batch's
    synchronisation: both report SPI_OK; its x within 1e-9 of the oracle and
    its variances within 1e-6 of a plain FP64 handle's; spi_info counts one
    switch for it and none for the band.  A second run replays the band's
    graph and recaptures the other in binary64.  Without the option the same
    batch reports SPI_E_NOCONV for that system only."""
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver, SpiBatch
    from test_gpu_parity import _near_collinear
    base, bands, _ = _systems()
    q = _near_collinear(far=1)
    o = oracle_solve(q)
    ob = oracle_solve(bands[0])
    qopts = dict(keep_root_order=1, refine_tol=1e-10, refine_steps=10)
    dev = torch.device("cuda")

    def near(stream=None, **more):
        s = SpiSolver(q.m, q.n, q.rowptr, q.col, stream=stream, **qopts, **more)
        s.potrf_block = 128
        return s

    ref = near(precision=0)       # plain FP64 on the current stream
    _set(ref, q)
    ref.factor()
    ref.solve(ref.rhs(torch.from_numpy(q.y).to(dev)))
    d_ref = ref.diag_inv().cpu().numpy()
    ref.close()
    probs = [bands[0], q]
    y = [torch.from_numpy(p.y).to(dev) for p in probs]
    rhs = [torch.empty(p.n, dtype=torch.float64, device=dev) for p in probs]
    x = [torch.empty_like(r) for r in rhs]
    d = [torch.empty_like(r) for r in rhs]
    for fallback in (0, 1):
        _say(f"case mixed batch fallback={fallback} graphs={graphs}")
        band = SpiSolver(base.m, base.n, base.rowptr, base.col, stream=torch.cuda.Stream(),
                         precision=1, refine_tol=1e-12, refine_steps=4,
                         fp64_fallback=fallback)
        s = near(stream=torch.cuda.Stream(), precision=1, fp64_fallback=fallback)
        for h, p in zip((band, s), probs):
            _set(h, p)
        torch.cuda.synchronize()
        batch = SpiBatch([band, s], use_graphs=bool(graphs))
        for rnd in range(2 if fallback else 1):
            st = batch.run(y, rhs, x, d)
            ex = _rel(x[1].cpu().numpy(), o["x"])
            ed = np.max(np.abs(d[1].cpu().numpy() - d_ref) / d_ref)
            eb = _rel(x[0].cpu().numpy(), ob["x"])
            _say(f"  run {rnd}: status {st}; near-collinear err_x={ex:.2e} "
                 f"err_d={ed:.2e} switches {s.info()['fp64_fallbacks']}; band "
                 f"err_x={eb:.2e} switches {band.info()['fp64_fallbacks']}")
            assert eb <= 1e-10 and band.info()["fp64_fallbacks"] == 0
            if not fallback:
                assert st == [0, 6]
                continue
            assert st == [0, 0]
            assert ex <= 1e-9 and ed <= 1e-6
            assert s.info()["fp64_fallbacks"] == 1
        batch.close()
        band.close()
        s.close()


def test_handle_on_its_own_stream():
    """A handle on a stream of its own, its inputs computed by torch on the
    current stream right before each call, behind a long fill kernel: the
    binding makes the handle's stream wait for them, keeps the tensors'
    memory from reuse, and after the current stream waits for the handle's
    stream x and diag(A^-1) match the FP64 oracle (three rounds)."""
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver
    _, bands, _ = _systems()
    p = bands[1]
    o = oracle_solve(p)
    _say(f"case handle on its own stream n={p.n}")
    st = torch.cuda.Stream()
    s = SpiSolver(p.m, p.n, p.rowptr, p.col, stream=st)
    val0 = torch.from_numpy(p.val).cuda()
    w0 = torch.from_numpy(p.w).cuda()
    y0 = torch.from_numpy(p.y).cuda()
    torch.cuda.synchronize()
    for rnd in range(3):
        busy = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        busy.fill_(1.0)                    # keeps the current stream busy
        val = val0 * 2.0 / 2.0             # exact, produced behind the fill
        w = w0 * 4.0 / 4.0
        y = y0 * 0.5 * 2.0
        s.set_values(val, w)
        s.factor()
        x = s.solve(s.rhs(y))
        d = s.diag_inv()
        del val, w, y, busy
        torch.cuda.current_stream().wait_stream(st)
        ex = _rel(x.cpu().numpy(), o["x"])
        ed = np.max(np.abs(d.cpu().numpy() - o["diag"]) / o["diag"])
        _say(f"  round {rnd}: err_x={ex:.2e} err_d={ed:.2e}")
        assert ex <= TOL and ed <= TOL
    s.close()
