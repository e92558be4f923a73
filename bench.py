"""Seconds per system for x = A^-1 b plus diag(A^-1) on one MI355X.

A step is one whole system: set the band's values (H, W already in HBM),
assemble + factor, b = H^T W y, solve with refinement, and all variances.
The workload is the medium coded-mask configuration (100x100 sky, 5000
pointings x 19 detectors, 17x17 field of view, background per detector per
4-pointing time bin: 95,000 rows, 33,750 unknowns), synthetic and seeded.

Prints one JSON line.  ``--gpus`` above 1 is refused: this build runs on
one GPU.

Other workloads (``--workload``), each printing its own JSON line:
  batch    64 energy bands on the medium pattern (response scale
           U(0.5, 1.5) per band, fresh Poisson counts) plus 32 independent
           sub-problems of uneven size (sky 30..120), mixed precision: each
           system alone, one after the other, against batched runs
           (concurrent streams, HIP graphs);
  learned  256 drifting bands on the medium pattern (+-20% response and
           background scale): direct solves of bands 0..31, the network
           trained on them, then FP32 PCG on a sample of bands 32..255 with
           and without the learned correction.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
# HBM bytes moved by one launch of the reported mixed-precision kernel (the
# root W^T W GEMM) on the medium workload: rocprofv3 FETCH_SIZE + WRITE_SIZE, each scaled by
# what the same counter reads for a copy kernel of known size (fetch x2.0,
# write x1.0).  Taken on the current GEMM kernel; None for other workloads.
LAUUM_HBM_BYTES_MEDIUM = 19.306e9 + 0.409e9
# The same for the reported FP64 kernel, the bulk update of the root sweeps
# (average per launch, outer block 512).
BULK_HBM_BYTES_MEDIUM = 1.2546e9 + 0.3683e9


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=("medium", "batch", "learned", "copy"),
                    default="medium")
    ap.add_argument("--bands", type=int, default=64,
                    help="batch: number of bands; learned: PCG sample size")
    ap.add_argument("--subproblems", type=int, default=32)
    ap.add_argument("--potrf-block", type=int, default=0, choices=(0, 128, 256, 512),
                    help="root POTRF outer block; 0 = the library's autotuner")
    ap.add_argument("--precision", choices=("fp64", "mixed", "both"), default="fp64",
                    help="fp64: every stage in binary64; mixed: binary32 "
                         "matrix-core products on the root front, binary64 "
                         "elsewhere, refinement to convergence")
    return ap.parse_args()


def cpu_baseline(p):
    """Time the CPU oracle, stage by stage, on a bounded sample of the same
    workload and scale each stage to one whole system."""
    import scipy.sparse as sp
    import scipy.linalg as sla
    from threadpoolctl import threadpool_limits
    from oracle.normal_eq import normal_equations
    from oracle.blockchol import BlockCholesky

    cores = len(os.sched_getaffinity(0))
    t = {}
    with threadpool_limits(limits=cores):
        # (1) normal equations on 10% of the rows, scaled by the row count
        rows = np.arange(0, p.m, 10)
        rp = np.concatenate([[0], np.cumsum(np.diff(p.rowptr)[rows])])
        sel = np.concatenate([np.arange(p.rowptr[r], p.rowptr[r + 1]) for r in rows])
        t0 = time.perf_counter()
        normal_equations(rp, p.col[sel], p.val[sel], p.w[rows], p.y[rows], p.n)
        t["normal_eq"] = (time.perf_counter() - t0) * (p.m / len(rows))
        # full A for the factor stages (not timed: already counted above)
        A, b = normal_equations(p.rowptr, p.col, p.val, p.w, p.y, p.n)
        nb = p.n_bg
        # (2) Schur complement update on 10% of the background columns
        Asb = A[nb:, :nb].tocsc()
        d = A.diagonal()[:nb]
        cols = np.arange(0, nb, 10)
        Lsb = (Asb[:, cols] @ sp.diags(1.0 / np.sqrt(d[cols]))).tocsr()
        t0 = time.perf_counter()
        (Lsb @ Lsb.T).toarray()
        t["schur"] = (time.perf_counter() - t0) * (nb / len(cols))
        # (3) dense Cholesky of the root block at full size (same order and
        #     cost as the Schur complement the oracle factors)
        Ass = A[nb:, nb:].toarray()
        t0 = time.perf_counter()
        Lss = np.linalg.cholesky(Ass)
        t["root_cholesky"] = time.perf_counter() - t0
        # (4) solve: two triangular solves with the root factor + leaf parts
        f = BlockCholesky.__new__(BlockCholesky)
        f.n, f.n_b, f.bb_diagonal = p.n, nb, True
        f.Lbb = np.sqrt(A.diagonal()[:nb])
        f.Lsb = (Asb @ sp.diags(1.0 / f.Lbb)).tocsr()
        f.Lss = Lss
        t0 = time.perf_counter()
        f.solve(b)
        t["solve"] = time.perf_counter() - t0
        # (5) variances: 2 blocks of 128 right-hand sides of each kind,
        #     scaled to all unknowns of that kind
        ib = np.arange(0, 256)
        isk = nb + np.arange(0, 256)
        t0 = time.perf_counter()
        f.diag_inv(ib)
        t["diag_bg"] = (time.perf_counter() - t0) * (nb / 256)
        t0 = time.perf_counter()
        f.diag_inv(isk)
        t["diag_sky"] = (time.perf_counter() - t0) * ((p.n - nb) / 256)
    total = sum(t.values())
    return {"value": total, "unit": "s/system", "cores": cores, "kind": "oracle",
            "sample": ("normal equations on 10% of rows and Schur update on 10% "
                       "of background columns, each scaled linearly; root "
                       "Cholesky and solve at full size; variances for 256 "
                       "background + 256 sky unknowns (RHS blocks of 128) "
                       "scaled to all unknowns"),
            "stages_s": {k: round(v, 3) for k, v in t.items()}}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "this build has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        return run_batch(args)
    if args.workload == "learned":
        return run_learned(args)
    if args.workload == "copy":
        return run_copy(args)
    import torch
    import spi_synth
    from paper_1305_5683_amd import SpiSolver

    print(f"# generating workload config {args.config}", file=sys.stderr, flush=True)
    p = spi_synth.make_config(args.config, progress=lambda f: print(
        f"#   pattern {100 * f:.0f}%", file=sys.stderr, flush=True))
    torch.cuda.set_device(torch.device("cuda:0"))
    precisions = ["fp64", "mixed"] if args.precision == "both" else [args.precision]
    results = {}
    for prec in precisions:
        out, x, d = measure(p, prec, args)
        results[prec] = (out, x, d)
    if len(precisions) == 2:
        # mixed against the FP64 GPU path on the same system
        _, x64, d64 = results["fp64"]
        out, xm, dm = results["mixed"]
        out["mixed_vs_fp64"] = {
            "x_rel": float(torch.linalg.norm(xm - x64) / torch.linalg.norm(x64)),
            "d_max_rel": float(torch.max(torch.abs(dm - d64) / d64)),
            "fp64_s_per_system": results["fp64"][0]["value"]}
        print(json.dumps(results["fp64"][0]))
        print(json.dumps(out))
        return
    out = results[precisions[0]][0]
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle, bounded sample)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(p)
    print(json.dumps(out))


def sweep_bulk_launches(np_pad, blk):
    """Bulk updates of one root inversion by sweeps: one per band that
    leaves lower-triangle entries outside its rows and columns and outside
    the next band's pivot block."""
    nb = min(blk, np_pad, 512)
    widths = [min(nb, np_pad - k) for k in range(0, np_pad, nb)]
    cnt = 0
    for k, w in enumerate(widths):
        kn = widths[k + 1] if k + 1 < len(widths) else 0
        R = np_pad - w
        cnt += R * (R + 1) // 2 - kn * (kn + 1) // 2 > 0
    return cnt


def measure(p, prec, args):
    """Time `args.steps` whole systems at one precision; returns the JSON
    object and the last x and diag(A^-1) (device tensors)."""
    import torch
    from paper_1305_5683_amd import SpiSolver
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    mixed = prec == "mixed"
    s = SpiSolver(p.m, p.n, p.rowptr, p.col, stream=stream, timing=1,
                  precision=1 if mixed else 0)
    t_an = time.perf_counter() - t0
    val = torch.from_numpy(p.val).to(dev)
    w = torch.from_numpy(p.w).to(dev)
    y = torch.from_numpy(p.y).to(dev)
    bbuf = torch.empty(p.n, dtype=torch.float64, device=dev)
    xbuf = torch.empty_like(bbuf)
    dbuf = torch.empty_like(bbuf)

    def step():
        s.set_values(val, w)
        s.factor()
        s.rhs(y, out=bbuf)
        s.solve(bbuf, out=xbuf)
        s.diag_inv(out=dbuf)

    # the library's autotuner picks the root POTRF block on this system
    # (unless one is given, as in profiling runs)
    s.set_values(val, w)
    if args.potrf_block:
        s.potrf_block = args.potrf_block
        blk = args.potrf_block
    else:
        blk = s.autotune()
    print(f"# {prec}: analysis {t_an:.2f}s; POTRF block {blk}; warmup {args.warmup}",
          file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    i0 = s.info()
    print(f"# timing {args.steps} steps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    i1 = s.info()
    K = args.steps
    ms = (t1 - t0) * 1e3 / K
    ph = {k: (i1[k] - i0[k]) / K for k in
          ("t_leaf_ms", "t_extend_ms", "t_potrf_ms", "t_solve_ms", "t_trtri_ms",
           "t_lauum_ms", "t_selinv_ms")}
    nR = i1["n_root"]
    refine = i1["refine_steps_done"]
    flops = (i1["flops_factor"] + i1["flops_selinv"] +
             i1["flops_solve"] * (1 + refine) + i1["flops_assembly"])
    peak = PEAK_FP64_TFLOPS
    bulk_s = (i1["t_sweep_bulk_ms"] - i0["t_sweep_bulk_ms"]) / 1e3
    if bulk_s > 0:
        # the root inverse by block sweeps; reported kernel = the bulk update
        # (one MFMA GEMM per band, FP64, or FP32 for mixed precision with
        # binary32 sums of at most 256 terms added in FP64: the lower
        # triangle outside the band's rows and columns and outside the next
        # band's pivot block, rank = the block; time and flops from the
        # library's timers)
        bulk_flops = i1["flops_sweep_bulk"] - i0["flops_sweep_bulk"]
        launches = sweep_bulk_launches(i1["n_root_padded"], blk)
        if mixed:
            peak = PEAK_FP32_TFLOPS
        roof = {"bound": "mfma",
                "kernel": ("k_gemm<128,128,XC,XC,float> (root sweep bulk update)"
                           if mixed else
                           "k_gemm<128,128,XC,XC> (root sweep bulk update)"),
                "achieved": bulk_flops / bulk_s / 1e12, "peak": peak,
                "unit": "TFLOP/s", "frac": bulk_flops / bulk_s / 1e12 / peak,
                "traffic": (BULK_HBM_BYTES_MEDIUM
                            if args.config == 1 and blk == 512 and not mixed
                            else None),
                "launches_per_system": launches,
                "flops_per_launch": bulk_flops / (K * launches),
                "avg_launch_us": bulk_s * 1e6 / (K * launches)}
    else:
        # mixed: the root inverse product Z = W^T W (an FP64 MFMA GEMM,
        # n_R^3 / 3 algorithmic flops, one launch)
        lauum_s = ph["t_lauum_ms"] / 1e3
        ach = (nR ** 3 / 3.0) / lauum_s / 1e12 if lauum_s > 0 else 0.0
        roof = {"bound": "mfma", "kernel": "k_gemm<128,128,KC,KC> (root W^T W)",
                "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                "frac": ach / peak,
                "traffic": LAUUM_HBM_BYTES_MEDIUM if args.config == 1 else None}
    out = {
        "metric": "s/system for solve+diag(A^-1)",
        "value": ms / 1e3,
        "unit": "s/system",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": f"coded-mask config {args.config}: sky {p.meta['sky']}x{p.meta['sky']}, "
                               f"{p.meta['n_point']} pointings x 19 detectors, FoV {p.meta['fov']}, "
                               f"M={p.m}, N={p.n}",
                   "m": p.m, "n": p.n, "nnz_h": int(p.nnz), "n_root": nR,
                   "n_leaf": i1["n_leaf"], "n_fronts": i1["n_groups"],
                   "nnz_a": i1["nnz_a"], "nnz_l": i1["nnz_l"],
                   "precision": prec, "parallelism": "1 GPU"},
        "gflops_per_s": flops / (ms / 1e3) / 1e9,
        "frac_fp64_peak_path": flops / (ms / 1e3) / (PEAK_FP64_TFLOPS * 1e12),
        "algorithmic_flops": flops,
        "analysis_s": t_an,
        "phases_ms": {k[2:-3]: round(v, 4) for k, v in ph.items()},
        "refine_steps": refine,
        "potrf_block": blk,
        "roofline": roof,
    }
    s.close()
    return out, xbuf, dbuf




def _say(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def _mixed_opts():
    # binary32 root products, 3 fixed refinement steps (batches do not read
    # norms back)
    return dict(precision=1, refine_tol=1e-14, refine_steps=3)


def run_batch(args):
    import torch
    import spi_synth
    from paper_1305_5683_amd import SpiSolver, SpiBatch
    torch.cuda.set_device(0)
    base = spi_synth.make_config(1)
    rng = np.random.default_rng(3000)
    nb, ns = args.bands, args.subproblems
    _say(f"generating {nb} bands")
    bands = [spi_synth.make_band(base, float(rng.uniform(0.5, 1.5)), 1.0,
                                 seed=3000 + b) for b in range(nb)]
    _say(f"generating {ns} sub-problems")
    subs = [spi_synth.make_problem(c, seed=3500 + i) for i, c in
            enumerate(spi_synth.subproblem_configs(ns, seed=3500))]
    opts = _mixed_opts()
    slots = 4
    streams = [torch.cuda.Stream() for _ in range(slots + ns)]
    _say("analysis")
    first = SpiSolver(base.m, base.n, base.rowptr, base.col, stream=streams[0], **opts)
    bslots = [first] + [SpiSolver.like(first, stream=streams[i]) for i in range(1, slots)]
    sub_s = [SpiSolver(q.m, q.n, q.rowptr, q.col, stream=streams[slots + i], **opts)
             for i, q in enumerate(subs)]
    dev = torch.device("cuda")
    bvals = [(torch.from_numpy(q.val).to(dev), torch.from_numpy(q.w).to(dev),
              torch.from_numpy(q.y).to(dev)) for q in bands]
    svals = [(torch.from_numpy(q.val).to(dev), torch.from_numpy(q.w).to(dev),
              torch.from_numpy(q.y).to(dev)) for q in subs]

    def outs(n):
        return [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(3)]
    bout = [outs(base.n) for _ in range(slots)]
    sout = [outs(q.n) for q in subs]

    def alone(s, v, o):
        s.set_values(v[0], v[1])
        s.factor()
        s.rhs(v[2], out=o[0])
        s.solve(o[0], out=o[1])
        s.diag_inv(out=o[2])
    def sequential():
        for b in range(nb):
            alone(bslots[0], bvals[b], bout[0])
        for s, v, o in zip(sub_s, svals, sout):
            alone(s, v, o)
        torch.cuda.synchronize()
    bb = SpiBatch(bslots, use_graphs=True)
    sb = SpiBatch(sub_s, use_graphs=True)
    def batched():
        for c in range(0, nb, slots):
            grp = list(range(c, min(nb, c + slots)))
            for k, b in enumerate(grp):
                bslots[k].set_values(bvals[b][0], bvals[b][1])
            ys = [bvals[b][2] for b in grp] + [bvals[grp[0]][2]] * (slots - len(grp))
            st = bb.run(ys, [o[0] for o in bout], [o[1] for o in bout],
                        [o[2] for o in bout])
            assert st == [0] * slots, st
        for s, v in zip(sub_s, svals):
            s.set_values(v[0], v[1])
        st = sb.run([v[2] for v in svals], [o[0] for o in sout],
                    [o[1] for o in sout], [o[2] for o in sout])
        assert st == [0] * ns, st
        torch.cuda.synchronize()
    _say("warm-up")
    sequential()
    batched()
    _say("timing sequential")
    t0 = time.perf_counter()
    sequential()
    t_seq = time.perf_counter() - t0
    _say("timing batched")
    t0 = time.perf_counter()
    batched()
    t_bat = time.perf_counter() - t0
    k = nb + ns
    # plain FP64 on the same systems, one at a time (the reference point)
    _say("timing plain FP64 sequential")
    s64 = SpiSolver(base.m, base.n, base.rowptr, base.col, stream=streams[0])
    sub64 = [SpiSolver(q.m, q.n, q.rowptr, q.col, stream=streams[slots + i])
             for i, q in enumerate(subs)]

    def sequential64():
        for b in range(nb):
            alone(s64, bvals[b], bout[0])
        for s, v, o in zip(sub64, svals, sout):
            alone(s, v, o)
        torch.cuda.synchronize()
    sequential64()
    t0 = time.perf_counter()
    sequential64()
    t_64 = time.perf_counter() - t0
    for s in [s64] + sub64:
        s.close()
    flops = 0.0
    for s, cnt in [(bslots[0], nb)] + [(x, 1) for x in sub_s]:
        i = s.info()
        flops += cnt * (i["flops_factor"] + i["flops_selinv"] +
                        4 * i["flops_solve"] + i["flops_assembly"])
    out = {
        "metric": "s/system for solve+diag(A^-1)", "value": t_bat / k,
        "unit": "s/system", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": t_bat * 1e3, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"batch: {nb} bands on the medium pattern + {ns} "
                               "sub-problems (sky 30..120), mixed precision",
                   "systems": k, "sub_problem_n": [q.n for q in subs]},
        "sequential_s_per_system": t_seq / k,
        "batched_s_per_system": t_bat / k,
        "speedup": t_seq / t_bat,
        "fp64_sequential_s_per_system": t_64 / k,
        "speedup_vs_fp64_sequential": t_64 / t_bat,
        "gflops_per_s": flops / t_bat / 1e9,
    }
    bb.close()
    sb.close()
    print(json.dumps(out))


def run_copy(args):
    """A plain streaming kernel of known size (y = 1.0 * x over 2^27 doubles,
    1 GiB read and 1 GiB written per launch): the reference that scales the
    HBM counters (FETCH_SIZE, WRITE_SIZE) of the other kernels."""
    import torch
    torch.cuda.set_device(0)
    n = 1 << 27
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(args.steps):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"workload": "copy", "bytes_read": 8 * n, "bytes_written": 8 * n,
                      "launches": args.steps}))


def run_learned(args):
    import torch
    import spi_synth
    from paper_1305_5683_amd import SpiSolver, SpiLearnedPrecond, pcg_solve
    torch.cuda.set_device(0)
    dev = torch.device("cuda")
    base = spi_synth.make_config(1)
    n_bands = 256

    def band(b):
        rs, bs = spi_synth.band_scales_drift(b, n_bands)
        return spi_synth.make_band(base, rs, bs, seed=4000 + b)
    _say("analysis")
    ref = SpiSolver(base.m, base.n, base.rowptr, base.col)
    work = SpiSolver.like(ref)
    # direct solves of bands 0..31 (training data), reference = band 31
    _say("direct solves of bands 0..31")
    data, t_direct = [], []
    for b in range(32):
        q = band(b)
        v = (torch.from_numpy(q.val).to(dev), torch.from_numpy(q.w).to(dev),
             torch.from_numpy(q.y).to(dev))
        s = ref if b == 31 else work
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.set_values(v[0], v[1])
        s.factor()
        rhs = s.rhs(v[2])
        x = s.solve(rhs)
        torch.cuda.synchronize()
        t_direct.append(time.perf_counter() - t0)
        if b < 31:
            data.append((v, rhs, x))
    hid = 16
    lp = SpiLearnedPrecond(hid, spi_synth.lp_init_params(hid, 0))
    _say("training")
    t0 = time.perf_counter()
    losses = []
    for epoch in range(20):
        tot = 0.0
        for v, rhs, x in data:
            work.set_values(v[0], v[1])
            tot += lp.train_step(work, ref, rhs, x, lr=0.02)
        losses.append(tot / len(data))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    sample = np.linspace(32, 255, args.bands).round().astype(int)
    res = {"with": [], "without": []}
    _say(f"PCG on {len(sample)} bands")
    for b in sample:
        q = band(int(b))
        v = (torch.from_numpy(q.val).to(dev), torch.from_numpy(q.w).to(dev),
             torch.from_numpy(q.y).to(dev))
        work.set_values(v[0], v[1])
        rhs = work.rhs(v[2])
        for key, model in (("without", None), ("with", lp)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, info = pcg_solve(work, ref, rhs, lp=model, tol=1e-10, maxit=300)
            torch.cuda.synchronize()
            res[key].append((time.perf_counter() - t0, info["iterations"],
                             info["fell_back"], info["rel_residual"]))
    def summ(r):
        a = np.array([x[:3] for x in r], dtype=float)
        return {"s_per_band": float(a[:, 0].mean()), "iterations_mean": float(a[:, 1].mean()),
                "fallbacks": int(a[:, 2].sum()),
                "max_rel_residual": float(max(x[3] for x in r))}
    out = {
        "metric": "s/band for x = A^-1 b (learned-preconditioned FP32 PCG)",
        "value": summ(res["with"])["s_per_band"], "unit": "s/band", "n_gpus": 1,
        "higher_is_better": False, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "learned: 256 drifting bands on the medium pattern",
                   "pcg_bands": [int(b) for b in sample], "hidden": hid},
        "direct_s_per_band": float(np.median(t_direct)),
        "train_s": t_train, "train_loss_first_last": [losses[0], losses[-1]],
        "pcg_with_network": summ(res["with"]),
        "pcg_without_network": summ(res["without"]),
    }
    lp.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
