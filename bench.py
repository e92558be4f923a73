"""Seconds per system for x = A^-1 b plus diag(A^-1) on one MI355X.

A step is one whole system: set the band's values (H, W already in HBM),
assemble + factor, b = H^T W y, solve with refinement, and all variances.
The default workload is the large coded-mask configuration (180x180 sky,
40,000 pointings x 19 detectors, 31x31 field of view, background per
detector per time bin of random length 1..10 pointings: 760,000 rows,
170,853 unknowns, a dense root front of order 32,400), synthetic and
seeded, timed in FP64 (the line's value) and then in mixed precision
(binary32 root products, FP64 refinement), whose x and variances are
compared with the FP64 GPU result.  ``--config 1`` times the medium
configuration (100x100 sky, 5000 pointings, 17x17 field of view, bins of 4
pointings: 95,000 rows, 33,750 unknowns) instead.

Prints one JSON line.  ``--gpus`` above 1 is refused: the solver runs on
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
           and without the learned correction;
  copy     a streaming copy of known size, the reference that scales the
           HBM counters of the other kernels.
"""
from __future__ import annotations

import argparse
import hashlib
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
CSRC = os.path.join(ROOT, "paper_1305_5683_amd", "csrc")

# HBM bytes per launch of the reported kernels, from rocprofv3 --pmc runs
# (FETCH_SIZE, then WRITE_SIZE; each scaled by what the same counter reads
# for the copy workload of known size).  Keyed by (config, kernel, outer
# block or None, precision); "src" names the source file and the section of
# it that holds the kernel (between two marker lines) with the SHA-256 prefix
# of that section's text when the counters were taken: once it changes the
# figure no longer applies and `traffic` is reported as null.
HBM_COUNTERS = {
    # large coded-mask system, FP64, outer block 512 (profiles/hbm_counters.txt)
    (2, "bulk", 512, "fp64"): {"bytes": 12.812e9 + 4.0965e9, "src": "6291710c77d9dd5a"},
    (2, "bulk", 1024, "fp64"): {"bytes": 28.628e9 + 3.9645e9, "src": "6291710c77d9dd5a"},
    (2, "assembly", None, "fp64"): {"bytes": 2969.4e9 + 4.2286e9, "src": "db0047727ae4bf4a"},
    (2, "assembly", None, "mixed"): {"bytes": 2969.4e9 + 4.2286e9, "src": "db0047727ae4bf4a"},
    # medium coded-mask system, FP64, outer block 512
    (1, "bulk", 512, "fp64"): {"bytes": 1.2486e9 + 0.3683e9, "src": "6291710c77d9dd5a"},
    (1, "assembly", None, "fp64"): {"bytes": 16.516e9 + 0.4092e9, "src": "db0047727ae4bf4a"},
    (1, "assembly", None, "mixed"): {"bytes": 16.516e9 + 0.4092e9, "src": "db0047727ae4bf4a"},
}


def src_hash(parts):
    """SHA-256 prefix of the concatenated source sections: (file, first
    marker line or None for the whole file, end marker or None)."""
    h = hashlib.sha256()
    for name, begin, end in parts:
        with open(os.path.join(CSRC, name), encoding="utf-8") as fh:
            text = fh.read()
        if begin is not None:
            i = text.index(begin)
            j = text.index(end, i) if end is not None else len(text)
            text = text[i:j]
        h.update(text.encode())
    return h.hexdigest()[:16]


# the sources the counters depend on: the kernel and the code that decides
# its launch order or its shapes
SRC_SECTIONS = {
    "bulk": [("k_gemm.hip", None, None),
             ("k_dense.hip", "hipError_t root_sweep(Handle& h) {", "\n}\n")],
    "assembly": [("k_sparse.hip",
                  "// --------------------------------------------------------- root assembly",
                  "// ------------------------------------------------------------ equilibration"),
                 ("analysis.cpp", "  // ---- amalgamate consecutive leaves", '  phase("incidences");')],
}


def counter_traffic(config, kernel, blk, prec):
    c = HBM_COUNTERS.get((config, kernel, blk if kernel == "bulk" else None, prec))
    if c is None:
        return None
    return c["bytes"] if src_hash(SRC_SECTIONS[kernel]) == c["src"] else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2, choices=(1, 2))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--slots", type=int, default=4,
                    help="batch workload: band systems run concurrently")
    ap.add_argument("--hw-queues", type=int, default=16,
                    help="batch workload: hardware queues of the process "
                         "(GPU_MAX_HW_QUEUES, 1..32; 0 = leave as set)")
    ap.add_argument("--workload", choices=("medium", "batch", "learned", "copy"),
                    default="medium")
    ap.add_argument("--bands", type=int, default=64,
                    help="batch: number of bands; learned: PCG sample size")
    ap.add_argument("--subproblems", type=int, default=32)
    ap.add_argument("--potrf-block", type=int, default=0, choices=(0, 128, 256, 512, 1024),
                    help="root POTRF outer block; 0 = the library's autotuner")
    ap.add_argument("--precision", choices=("fp64", "mixed", "both"), default="both",
                    help="fp64: every stage in binary64; mixed: binary32 "
                         "matrix-core products on the root front, binary64 "
                         "elsewhere, refinement to convergence")
    return ap.parse_args()


def cpu_baseline(p):
    """Time the CPU oracle, stage by stage, on a bounded sample of the same
    workload (about 10-30 s of CPU work) and scale each stage to one whole
    system by its operation count."""
    import scipy.sparse as sp
    import scipy.linalg as sla
    from threadpoolctl import threadpool_limits
    from oracle.normal_eq import normal_equations
    from oracle.blockchol import BlockCholesky

    cores = len(os.sched_getaffinity(0))
    t = {}
    nb, ns = p.n_bg, p.n - p.n_bg
    with threadpool_limits(limits=cores):
        # (1) normal equations on the rows of every k-th background column
        #     (about 2,500 columns, 500 for a root above 16,384), scaled by
        #     the row count; every coupling entry of those columns comes
        #     from these rows
        kc = max(1, nb // (2500 if ns <= 16384 else 500))
        cols = np.arange(0, nb, kc)
        H = p.scipy_csr()
        crow = np.unique(H[:, cols].tocsc().indices)
        Hr = H[crow]
        del H
        t0 = time.perf_counter()
        Ab, _ = normal_equations(Hr.indptr, Hr.indices, Hr.data, p.w[crow],
                                 p.y[crow], p.n)
        t["normal_eq"] = (time.perf_counter() - t0) * (p.m / len(crow))
        # (2) Schur complement update by the oracle's block factor on those
        #     columns, scaled by the column count; where the block factor
        #     takes a dense product, the sample is also cut to the first
        #     4,096 root rows (a 4,096^2 block of the product, scaled by
        #     (n_root / 4096)^2 as well)
        Ab = Ab.tocsc()
        As = Ab
        Asb = Ab[nb:, cols]
        Lsb = Asb @ sp.diags(1.0 / np.sqrt(Ab.diagonal()[cols]))
        rows_scale = 1.0
        if Lsb.nnz > BlockCholesky.DENSE_FRACTION * Lsb.shape[0] * Lsb.shape[1]:
            kr2 = min(ns, 4096)
            Ld = Lsb[:kr2].toarray()
            rows_scale = (ns / kr2) ** 2
            t0 = time.perf_counter()
            _ = Ld @ Ld.T
        else:
            t0 = time.perf_counter()
            _ = (Lsb @ Lsb.T).toarray()
        t["schur"] = (time.perf_counter() - t0) * (nb / len(cols)) * rows_scale
        del Ab, Asb, Lsb
        # (3) dense Cholesky of the root (LAPACK through NumPy, as the
        #     block factor calls it) at order k = min(n_root, 8192), on the
        #     sampled rows' sky block plus a diagonal shift (positive
        #     definite), scaled by (n_root / k)^3
        k = min(ns, 8192)
        M = As[nb:nb + k, nb:nb + k].toarray()
        M[np.diag_indices(k)] += np.abs(M).sum(axis=1) + 1.0
        t0 = time.perf_counter()
        Lk = np.linalg.cholesky(M)
        t["root_cholesky"] = (time.perf_counter() - t0) * (ns / k) ** 3
        # (4) solve: forward and backward substitution with that factor,
        #     scaled by (n_root / k)^2
        v = np.ones(k)
        t0 = time.perf_counter()
        sla.solve_triangular(Lk, sla.solve_triangular(Lk, v, lower=True),
                             lower=True, trans="T")
        t["solve"] = (time.perf_counter() - t0) * (ns / k) ** 2
        # (5) variances: the block factor's blocks of 128 right-hand sides
        #     cost a triangular solve with the root factor each; two blocks
        #     timed, scaled by (n_root / k)^2 and by n / 256
        E = np.zeros((k, 128))
        E[np.arange(128), np.arange(128)] = 1.0
        t0 = time.perf_counter()
        for _ in range(2):
            V = sla.solve_triangular(Lk, E, lower=True)
            (V * V).sum(axis=0)
        t["diag"] = (time.perf_counter() - t0) * (ns / k) ** 2 * (p.n / 256)
    total = sum(t.values())
    return {"value": total, "unit": "s/system", "cores": cores, "kind": "oracle",
            "sample": (f"normal equations on the rows of every {kc}th "
                       f"background column and the Schur update on those "
                       f"columns, each scaled linearly (the Schur product on its first 4096 root rows "
                       f"when it is dense, scaled by (n_root/4096)^2); root "
                       f"Cholesky, substitutions and 2 variance "
                       f"blocks of 128 right-hand sides at order {k}, scaled by "
                       f"(n_root/{k})^3, (n_root/{k})^2 and (n_root/{k})^2 * n/256"),
            "stages_s": {k_: round(v_, 3) for k_, v_ in t.items()}}


def main():
    args = parse()
    if not 0 <= args.hw_queues <= 32:
        print("--hw-queues takes 0..32", file=sys.stderr)
        sys.exit(2)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the solver has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        return run_batch(args)
    if args.workload == "learned":
        return run_learned(args)
    if args.workload == "copy":
        return run_copy(args)
    import torch
    import spi_synth

    print(f"# generating workload config {args.config}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    p = spi_synth.make_config(args.config, progress=lambda f: print(
        f"#   pattern {100 * f:.0f}%", file=sys.stderr, flush=True))
    print(f"# generated in {time.perf_counter() - t0:.1f} s: m={p.m} n={p.n} "
          f"nnz={p.nnz}", file=sys.stderr, flush=True)
    torch.cuda.set_device(torch.device("cuda:0"))
    precisions = ["fp64", "mixed"] if args.precision == "both" else [args.precision]
    results = {}
    src = None   # the first handle's analysis is copied for the second
    for prec in precisions:
        results[prec] = measure(p, prec, args, src)
        src = results[prec][3]
    out = results[precisions[0]][0]
    if len(precisions) == 2:
        # mixed precision on the same system, against the FP64 GPU result
        _, x64, d64, _ = results["fp64"]
        om, xm, dm, _ = results["mixed"]
        out["mixed"] = {
            "s_per_system": om["value"], "ms_per_step": om["ms_per_step"],
            "speedup_vs_fp64": out["value"] / om["value"],
            "x_rel_vs_fp64": float(torch.linalg.norm(xm - x64) / torch.linalg.norm(x64)),
            "d_max_rel_vs_fp64": float(torch.max(torch.abs(dm - d64) / d64)),
            "refine_steps": om["refine_steps"], "potrf_block": om["potrf_block"],
            "phases_ms": om["phases_ms"], "roofline": om["roofline"]}
    for r in results.values():
        r[3].close()
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle, bounded sample)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(p)
    print(json.dumps(out))


def sweep_bulk_launches(np_pad, blk):
    """Bulk updates of one root inversion by sweeps: one per band that
    leaves lower-triangle entries outside its rows and columns and outside
    the next band's pivot block."""
    nb = min(blk, np_pad)
    widths = [min(nb, np_pad - k) for k in range(0, np_pad, nb)]
    cnt = 0
    for k, w in enumerate(widths):
        kn = widths[k + 1] if k + 1 < len(widths) else 0
        R = np_pad - w
        cnt += R * (R + 1) // 2 - kn * (kn + 1) // 2 > 0
    return cnt


def measure(p, prec, args, src=None):
    """Time `args.steps` whole systems at one precision; returns the JSON
    object, the last x and diag(A^-1) (device tensors) and the handle.
    With `src`, the handle copies src's analysis (spi_analyze_like) and the
    reported analysis time is src's."""
    import torch
    from paper_1305_5683_amd import SpiSolver
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    mixed = prec == "mixed"
    if src is None:
        s = SpiSolver(p.m, p.n, p.rowptr, p.col, stream=stream, timing=1,
                      precision=1 if mixed else 0)
        t_an = time.perf_counter() - t0
    else:
        s = SpiSolver.like(src.solver, stream=stream, timing=1,
                           precision=1 if mixed else 0)
        t_an = src.t_an
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

    # the library's autotuner picks the root's outer block on this system
    # (unless one is given, as in profiling runs)
    s.set_values(val, w)
    if args.potrf_block:
        s.potrf_block = args.potrf_block
        blk = args.potrf_block
    else:
        blk = s.autotune()
    print(f"# {prec}: analysis {t_an:.2f}s; outer block {blk}, bulk tile "
          f"{s.bulk_tile}; warmup {args.warmup}",
          file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    i0 = s.info()
    print(f"# {prec}: timing {args.steps} steps", file=sys.stderr, flush=True)
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
    # the kernels that dominate a step, timed live with HIP events on the
    # handle's stream by the library: the root assembly (one launch per
    # step) and the sweeps' bulk updates (one launch per band)
    peak = PEAK_FP32_TFLOPS if mixed else PEAK_FP64_TFLOPS
    bulk_ms = (i1["t_sweep_bulk_ms"] - i0["t_sweep_bulk_ms"]) / K
    bulk_flops = (i1["flops_sweep_bulk"] - i0["flops_sweep_bulk"]) / K
    launches = sweep_bulk_launches(i1["n_root_padded"], blk)
    tile = s.bulk_tile
    asm_ms = ph["t_extend_ms"]
    kernels = {
        "assembly": {"kernel": f"k_assemble_root<{i1['asm_tile']}> (root front assembly)",
                     "ms_per_step": asm_ms, "launches_per_step": 1,
                     "flops_per_launch": i1["flops_root_assembly"],
                     "peak": PEAK_FP64_TFLOPS, "key": "assembly"},
        "bulk": {"kernel": (f"k_gemm<{tile},{tile},XC,XC,float> (root sweep bulk update)"
                            if mixed else
                            f"k_gemm<{tile},{tile},XC,XC> (root sweep bulk update)"),
                 "ms_per_step": bulk_ms, "launches_per_step": launches,
                 "flops_per_launch": bulk_flops / max(1, launches),
                 "peak": peak, "key": "bulk"},
    }
    dom = max(kernels.values(), key=lambda k: k["ms_per_step"])
    avg_s = dom["ms_per_step"] / 1e3 / dom["launches_per_step"]
    ach = dom["flops_per_launch"] / avg_s / 1e12 if avg_s > 0 else 0.0
    roof = {"bound": "mfma", "kernel": dom["kernel"], "achieved": ach,
            "peak": dom["peak"], "unit": "TFLOP/s", "frac": ach / dom["peak"],
            "traffic": counter_traffic(args.config, dom["key"], blk, prec),
            "launches_per_step": dom["launches_per_step"],
            "flops_per_launch": dom["flops_per_launch"],
            "avg_launch_us": avg_s * 1e6}
    kernel_ms = {k: round(v["ms_per_step"], 4) for k, v in kernels.items()}
    cfgs = {1: "medium", 2: "large"}
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
        "config": {"workload": f"coded-mask {cfgs[args.config]} system: sky "
                               f"{p.meta['sky']}x{p.meta['sky']}, {p.meta['n_point']} "
                               f"pointings x 19 detectors, FoV {p.meta['fov']}, "
                               f"M={p.m}, N={p.n}",
                   "m": p.m, "n": p.n, "nnz_h": int(p.nnz), "n_root": nR,
                   "n_leaf": i1["n_leaf"], "n_fronts": i1["n_groups"],
                   "nnz_a": i1["nnz_a"], "nnz_l": i1["nnz_l"],
                   "precision": prec, "parallelism": "1 GPU"},
        "gflops_per_s": flops / (ms / 1e3) / 1e9,
        "frac_fp64_peak_path": flops / (ms / 1e3) / (PEAK_FP64_TFLOPS * 1e12),
        "algorithmic_flops": flops,
        "executed_flops_assembly_selinv": (i1["flops_exec_assembly"] +
                                           i1["flops_exec_selinv"]),
        "analysis_s": t_an,
        "s_per_system_with_analysis": ms / 1e3 + t_an,
        "phases_ms": {k[2:-3]: round(v, 4) for k, v in ph.items()},
        "kernels_ms_per_step": kernel_ms,
        "refine_steps": refine,
        "potrf_block": blk,
        "bulk_tile": tile,
        "roofline": roof,
    }

    class _Kept:
        pass
    kept = _Kept()
    kept.solver, kept.t_an = s, t_an
    kept.close = s.close
    return out, xbuf, dbuf, kept




def _say(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def _mixed_opts():
    # binary32 root products, 3 fixed refinement steps (batches do not read
    # norms back)
    return dict(precision=1, refine_tol=1e-14, refine_steps=3)


def run_batch(args):
    # Hardware queues of this process: HIP maps streams onto 4 by default,
    # which serialises the concurrent systems of a batch; 16 lets the band
    # slots and sub-problems run side by side.  HIP reads it at start-up, so
    # it is set before torch first touches the GPU.
    if args.hw_queues:
        os.environ["GPU_MAX_HW_QUEUES"] = str(args.hw_queues)
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
    slots = args.slots
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
    # launch shapes: the library's autotuner on the first band (shared by
    # every band slot) and on each sub-problem
    _say("autotuning")
    first.set_values(bvals[0][0], bvals[0][1])
    first.autotune()
    for s in bslots[1:]:
        s.potrf_block, s.bulk_tile = first.potrf_block, first.bulk_tile
    for s, v in zip(sub_s, svals):
        s.set_values(v[0], v[1])
        s.autotune()

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
    for s, v in [(s64, bvals[0])] + list(zip(sub64, svals)):
        s.set_values(v[0], v[1])
        s.autotune()

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
                   "systems": k, "sub_problem_n": [q.n for q in subs],
                   "band_potrf_block": first.potrf_block,
                   "band_bulk_tile": first.bulk_tile,
                   "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES")},
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
