"""Seconds per system for x = A^-1 b plus diag(A^-1) on one MI355X.

A step is one whole system: set the band's values (H, W already in HBM),
assemble + factor, b = H^T W y, solve with refinement, and all variances.
The workload is the medium coded-mask configuration (100x100 sky, 5000
pointings x 19 detectors, 17x17 field of view, background per detector per
4-pointing time bin: 95,000 rows, 33,750 unknowns), synthetic and seeded.

Prints one JSON line.  ``--gpus`` above 1 is refused: this build runs on
one GPU.
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="fp64",
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
    import torch
    import spi_synth
    from paper_1305_5683_amd import SpiSolver

    print(f"# generating workload config {args.config}", file=sys.stderr, flush=True)
    p = spi_synth.make_config(args.config)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    mixed = args.precision == "mixed"
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

    print(f"# analysis {t_an:.2f}s; warmup {args.warmup}", file=sys.stderr, flush=True)
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
    # reported kernel: the root inverse product Z = W^T W (an FP64 MFMA GEMM
    # in both precisions; n_R^3 / 3 algorithmic flops)
    peak = PEAK_FP64_TFLOPS
    lauum_flops = nR ** 3 / 3.0
    lauum_s = ph["t_lauum_ms"] / 1e3
    ach = lauum_flops / lauum_s / 1e12 if lauum_s > 0 else 0.0
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
                   "precision": args.precision, "parallelism": "1 GPU"},
        "gflops_per_s": flops / (ms / 1e3) / 1e9,
        "frac_fp64_peak_path": flops / (ms / 1e3) / (PEAK_FP64_TFLOPS * 1e12),
        "algorithmic_flops": flops,
        "analysis_s": t_an,
        "phases_ms": {k[2:-3]: round(v, 4) for k, v in ph.items()},
        "refine_steps": refine,
        "roofline": {"bound": "mfma", "kernel": "k_gemm<128,128,KC,KC> (root W^T W)",
                     "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                     "frac": ach / peak, "traffic": None},
    }
    s.close()
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle, bounded sample)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(p)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
