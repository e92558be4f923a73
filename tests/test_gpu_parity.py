"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Tolerances (plain FP64 path): solution ``||x - x_o|| / ||x_o|| <= 1e-12``
and variances ``max_i |d_i - d_o,i| / d_o,i <= 1e-12``; the oracle's x is
certified by refinement with long-double residuals, so its own error is far
below the bound.  Integer-valued inputs make ``b = H^T W y`` exact, so it is
compared bit for bit.  Mixed precision (FP32 matrix-core products on the
root front, FP64 elsewhere, refinement to convergence): ``<= 1e-10`` for x
and ``<= 1e-6`` for the variances, the errors printed per case.
"""
import functools
import os
import sys

import numpy as np
import pytest

import spi_synth as synth
from oracle import oracle_solve, normal_equations_bruteforce
from oracle.certify import refine_inverse_column, apply_normal_ld

pytestmark = pytest.mark.gpu

TOL_X = 1e-12
TOL_D = 1e-12
TOL_X_MIXED = 1e-10
TOL_D_MIXED = 1e-6


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_gpu(p, want_diag=True, y=None, **opts):
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver
    dev = torch.device("cuda")
    s = SpiSolver(p.m, p.n, p.rowptr, p.col, **opts)
    s.set_values(torch.from_numpy(p.val).to(dev), torch.from_numpy(p.w).to(dev))
    s.factor()
    yy = torch.from_numpy(p.y if y is None else y).to(dev)
    b = s.rhs(yy)
    x = s.solve(b)
    d = s.diag_inv() if want_diag else None
    torch.cuda.synchronize()
    out = {"b": b.cpu().numpy(), "x": x.cpu().numpy(),
           "d": None if d is None else d.cpu().numpy(), "info": s.info()}
    s.close()
    return out


def rel_x(x, xo):
    return np.linalg.norm(x - xo) / np.linalg.norm(xo)


def rel_d(d, do):
    return np.max(np.abs(d - do) / np.abs(do))


def _check(p, g, o, idx=None, tol_x=TOL_X, tol_d=TOL_D):
    ex = rel_x(g["x"], o["x"])
    bo = o["b"]
    eb = np.max(np.abs(g["b"] - bo)) / np.max(np.abs(bo))
    dg = g["d"] if idx is None else g["d"][idx]
    ed = rel_d(dg, o["diag"])
    _say(f"  {p.name}: n={p.n} err_x={ex:.2e} err_d={ed:.2e} err_b={eb:.2e} "
         f"refine={g['info']['refine_steps_done']}")
    assert eb <= 1e-14
    assert ex <= tol_x
    assert ed <= tol_d
    assert np.all(g["d"] > 0)


@functools.lru_cache(maxsize=1)
def _medium():
    """The medium workload and its oracle, x and every variance."""
    p = synth.make_config(1)
    return p, None, oracle_solve(p)


# A large-workload shape at a size the oracle finishes in seconds: the
# large configuration's 31x31 field of view and random time-bin lengths
# U{1..10} on a 60x60 sky with 1500 pointings (28,500 rows, 8,711 unknowns).
# Its leaf fronts see up to the whole 3,600-pixel root, wider than the 2,048
# positions the leaf assembly accumulates on chip, so the in-place leaf
# assembly runs.
LARGE_SHAPE = synth.SkyConfig("large-shape-s60", 60, 1500, 31, 0)


@functools.lru_cache(maxsize=1)
def _large_shape():
    p = synth.make_problem(LARGE_SHAPE, seed=22)
    return p, oracle_solve(p)


def _front_widths(p):
    """Root positions of every leaf front, from the analysis' column-to-front
    map and the pattern of H (host-side counting, no arithmetic of the
    method)."""
    from paper_1305_5683_amd import symbolic
    import scipy.sparse as sp
    info, _, _, front = symbolic(p.m, p.n, p.rowptr, p.col)
    Hb = sp.csr_matrix((np.ones(p.nnz), p.col, p.rowptr), shape=(p.m, p.n))
    leaf = front >= 0
    G = sp.csr_matrix((np.ones(int(leaf.sum())), (front[leaf], np.nonzero(leaf)[0])),
                      shape=(info["n_groups"], p.n))
    FU = (G @ Hb.T) @ Hb[:, ~leaf]
    return np.diff(FU.tocsr().indptr), info


def test_tiny_config_parity():
    p = synth.make_config(0)
    _say(f"case tiny config seed={p.seed} m={p.m} n={p.n}")
    g = run_gpu(p)
    o = oracle_solve(p)
    _check(p, g, o)
    assert g["info"]["n_leaf"] == 380 and g["info"]["n_root"] == 400


LEAFY = [
    # (groups, leaf/group, root, rows/leaf, root/row, extra rows, seed, opts)
    (9, 5, 70, 3, 8, 12, 0, {}),            # ragged U, row-only fronts, pad 128
    (4, 23, 150, 2, 20, 40, 1, {}),         # fronts wider than 16 columns
    (30, 3, 200, 4, 30, 0, 2, {}),          # U spanning several 64-tiles
    (6, 4, 260, 2, 60, 300, 3, {"max_group": 1}),  # one pivot per front
    (5, 6, 90, 3, 10, 20, 4, {"leaf_max_work": 0.0}),  # no leaves: dense root
    (12, 7, 600, 3, 25, 50, 5, {"root_inverse": 0}),   # substitution solves
    (12, 7, 600, 3, 25, 50, 5, {"refine_steps": 0}),   # no refinement
]


@pytest.mark.parametrize("case", LEAFY, ids=[f"leafy{i}" for i in range(len(LEAFY))])
def test_leafy_structure_parity(case):
    ng, lpg, nr, rpl, rpr, ex, seed, opts = case
    p = synth.make_random_leafy(ng, lpg, nr, rpl, rpr, ex, seed)
    _say(f"case leafy seed={seed} m={p.m} n={p.n} opts={opts}")
    g = run_gpu(p, **opts)
    o = oracle_solve(p)
    _check(p, g, o)


def test_all_leaves_no_root():
    """Every unknown has rows of its own: A is diagonal, no root front."""
    rng = np.random.default_rng(5)
    n, k = 37, 3
    rowptr = np.arange(n * k + 1, dtype=np.int64)
    col = np.repeat(np.arange(n, dtype=np.int32), k)
    val = 0.1 + rng.random(n * k)
    w = 0.5 + rng.random(n * k)
    y = rng.random(n * k) * 10
    p = synth.Problem(m=n * k, n=n, n_bg=n, rowptr=rowptr, col=col, val=val,
                      w=w, y=y, x_true=np.ones(n), name="diag")
    _say("case all-leaves n=37")
    g = run_gpu(p)
    assert g["info"]["n_root"] == 0
    a = np.bincount(col, weights=w * val * val, minlength=n)
    bb = np.bincount(col, weights=w * val * y, minlength=n)
    assert np.allclose(g["x"], bb / a, rtol=1e-14)
    assert np.allclose(g["d"], 1.0 / a, rtol=1e-14)


def test_rhs_is_exact_on_integer_inputs():
    p = synth.make_random_leafy(6, 4, 40, 2, 6, 10, seed=7, integer=True)
    _say(f"case integer rhs m={p.m} n={p.n}")
    g = run_gpu(p, want_diag=False)
    _, bb = normal_equations_bruteforce(p.rowptr, p.col, p.val, p.w, p.y, p.n)
    assert np.array_equal(g["b"], bb)


def test_multiple_right_hand_sides():
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver
    p = synth.make_random_leafy(8, 5, 80, 3, 9, 15, seed=8)
    _say(f"case multi-rhs m={p.m} n={p.n}")
    o = oracle_solve(p, want_diag=False, refine_steps=0)
    f = o["factor"]
    rng = np.random.default_rng(0)
    B = rng.standard_normal((3, p.n))
    s = SpiSolver(p.m, p.n, p.rowptr, p.col)
    dev = torch.device("cuda")
    s.set_values(torch.from_numpy(p.val).to(dev), torch.from_numpy(p.w).to(dev))
    s.factor()
    X = s.solve(torch.from_numpy(B).to(dev)).cpu().numpy()
    s.close()
    for c in range(3):
        xo = f.solve(B[c]).astype(np.longdouble)
        for _ in range(2):     # certify with long-double residuals from H
            r = B[c].astype(np.longdouble) - apply_normal_ld(
                p.rowptr, p.col, p.val, p.w, xo)
            xo = xo + f.solve(r.astype(np.float64))
        assert rel_x(X[c], xo.astype(np.float64)) <= TOL_X


def test_not_spd_is_reported_with_column():
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver, SpiError
    p = synth.make_config(0)
    dev = torch.device("cuda")
    # a negative weight on every row of background unknown 7: pivot < 0
    w = p.w.copy()
    w[p.col[p.rowptr[:-1]] == 7] = -1.0
    s = SpiSolver(p.m, p.n, p.rowptr, p.col)
    s.set_values(torch.from_numpy(p.val).to(dev), torch.from_numpy(w).to(dev))
    _say("case not-spd leaf")
    with pytest.raises(SpiError) as ei:
        s.factor()
    assert ei.value.status == 3 and s.info()["failed_col"] == 7
    with pytest.raises(SpiError) as ei:       # no factor: state error
        s.diag_inv()
    assert ei.value.status == 2
    # root: weights scaled negative on all rows -> first root pivot fails
    s.set_values(torch.from_numpy(p.val).to(dev),
                 torch.from_numpy(-p.w).to(dev))
    _say("case not-spd all")
    with pytest.raises(SpiError) as ei:
        s.factor()
    assert ei.value.status == 3
    s.close()


def test_state_errors():
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver, SpiError
    p = synth.make_config(0)
    s = SpiSolver(p.m, p.n, p.rowptr, p.col)
    with pytest.raises(SpiError) as ei:
        s.factor()
    assert ei.value.status == 2
    s.close()


@pytest.mark.timeout(900)
def test_medium_config_parity():
    """The medium workload (100x100 sky, 5000 pointings, 33,750 unknowns):
    all of x against the certified oracle, and every variance against the
    oracle's block factor; a few variances also against certified inverse
    columns."""
    p, _, o = _medium()
    _say(f"case medium config m={p.m} n={p.n}")
    g = run_gpu(p)
    _check(p, g, o)
    f = o["factor"]
    rng = np.random.default_rng(1)
    for j in np.concatenate([rng.choice(p.n_bg, 4, replace=False),
                             p.n_bg + rng.choice(p.n - p.n_bg, 4, replace=False)]):
        zc = refine_inverse_column(p, f.solve, int(j))
        assert abs(g["d"][j] - float(zc[j])) <= TOL_D * float(zc[j])


def test_medium_config_parity_tile64():
    """The medium workload with 64 x 64 root assembly tiles (the analysis
    takes 128 x 128 at this order): same parity bar."""
    p, _, o = _medium()
    _say(f"case medium config, assembly tile 64, m={p.m} n={p.n}")
    g = run_gpu(p, asm_tile=64)
    assert g["info"]["asm_tile"] == 64
    _check(p, g, o)


@pytest.mark.parametrize("case", LEAFY, ids=[f"leafy{i}" for i in range(len(LEAFY))])
def test_leafy_structure_parity_tile128(case):
    """The planted-structure cases with 128 x 128 root assembly tiles (the
    analysis takes 64 x 64 at these orders): runs spanning tiles, ragged
    tails and padded roots in the 16-wave kernel."""
    ng, lpg, nr, rpl, rpr, ex, seed, opts = case
    p = synth.make_random_leafy(ng, lpg, nr, rpl, rpr, ex, seed)
    _say(f"case leafy tile128 seed={seed} m={p.m} n={p.n} opts={opts}")
    g = run_gpu(p, asm_tile=128, **opts)
    assert g["info"]["asm_tile"] == 128 or g["info"]["n_root"] == 0
    _check(p, g, oracle_solve(p))


@pytest.mark.timeout(900)
def test_large_shape_parity_fp64():
    """The large workload's field of view (31x31) and random bin lengths:
    all of x and every variance at 1e-12.  Its fronts are wider than the
    on-chip accumulation cap (in-place leaf assembly), a chunk of 50,000
    tasks splits the leaf selected inversion into several launches, and the
    root is assembled in 128 x 128 tiles as the large workload's is."""
    p, o = _large_shape()
    widths, info = _front_widths(p)
    nt = -(-widths // 64)
    n_tasks = int(np.sum(nt * (nt + 1) // 2))
    _say(f"case large-shape fp64 m={p.m} n={p.n} root={info['n_root']} "
         f"widest front {widths.max()}, {n_tasks} selected-inversion tasks")
    assert widths.max() > 2048 and n_tasks > 3 * 50000
    g = run_gpu(p, selinv_chunk=50000, asm_tile=128)
    assert g["info"]["asm_tile"] == 128
    _check(p, g, o)


@pytest.mark.timeout(900)
def test_large_shape_parity_mixed():
    p, o = _large_shape()
    _say(f"case large-shape mixed m={p.m} n={p.n}")
    g = run_gpu(p, precision=1)
    _check(p, g, o, tol_x=TOL_X_MIXED, tol_d=TOL_D_MIXED)


FORCED = [
    # (case, opts): leaf panels accumulated in place (cap below every front
    # width) and the selected inversion in launches of a few tasks
    ((30, 3, 200, 4, 30, 0, 2), {"leaf_lds_cap": 16, "selinv_chunk": 7}),
    ((4, 23, 150, 2, 20, 40, 1), {"leaf_lds_cap": 1, "selinv_chunk": 1}),
    ((12, 7, 600, 3, 25, 50, 5), {"leaf_lds_cap": 64, "selinv_chunk": 100,
                                  "precision": 1}),
]


@pytest.mark.parametrize("case", FORCED, ids=[f"forced{i}" for i in range(len(FORCED))])
def test_inplace_leaf_assembly_and_chunked_selinv(case):
    shape, opts = case
    p = synth.make_random_leafy(*shape)
    _say(f"case forced paths m={p.m} n={p.n} opts={opts}")
    g = run_gpu(p, **opts)
    o = oracle_solve(p)
    mixed = opts.get("precision", 0) == 1
    _check(p, g, o, tol_x=TOL_X_MIXED if mixed else TOL_X,
           tol_d=TOL_D_MIXED if mixed else TOL_D)


def test_nonfinite_values_are_rejected():
    """A NaN value or an infinite weight is caught on the device and
    reported by the factorisation as SPI_E_ARG; good values afterwards
    factor normally."""
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver, SpiError
    p = synth.make_config(0)
    dev = torch.device("cuda")
    s = SpiSolver(p.m, p.n, p.rowptr, p.col)
    val, w = p.val.copy(), p.w.copy()
    val[1234] = np.nan
    w[77] = np.inf
    for v, ww, what in ((val, p.w, "nan value"), (p.val, w, "inf weight")):
        _say(f"case non-finite input: {what}")
        s.set_values(torch.from_numpy(v).to(dev), torch.from_numpy(ww).to(dev))
        with pytest.raises(SpiError) as ei:
            s.factor()
        assert ei.value.status == 1
        with pytest.raises(SpiError) as ei:
            s.diag_inv()
        assert ei.value.status == 2
    s.set_values(torch.from_numpy(p.val).to(dev), torch.from_numpy(p.w).to(dev))
    s.factor()
    d = s.diag_inv().cpu().numpy()
    o = oracle_solve(p)
    assert rel_d(d, o["diag"]) <= TOL_D
    s.close()


# ------------------------------------------------------------ equilibration
def test_equilibration_changes_no_rounding():
    """Power-of-two scaling is exact: FP64 results with and without it agree
    to the last bits (the pivots' rsqrt seed is the only scale-sensitive
    step, and Newton refinement removes it)."""
    p = synth.make_config(0)
    _say("case equilibration on/off tiny")
    g1 = run_gpu(p, equilibrate=1)
    g0 = run_gpu(p, equilibrate=0)
    dx = rel_x(g1["x"], g0["x"])
    dd = rel_d(g1["d"], g0["d"])
    _say(f"  on vs off: dx={dx:.2e} dd={dd:.2e}")
    assert dx <= 1e-14 and dd <= 1e-14


def _badly_scaled(p, seed=0):
    """Columns of H multiplied by powers of two spanning 2^-90 .. 2^90: A's
    entries then overflow binary32 unless the matrix is equilibrated."""
    rng = np.random.default_rng(seed)
    e = rng.integers(-90, 91, size=p.n).astype(np.float64)
    q = synth.Problem(**{k: getattr(p, k) for k in
                         ("m", "n", "n_bg", "rowptr", "col", "w", "y",
                          "x_true", "seed")},
                      val=p.val * np.exp2(e)[p.col], name=p.name + "-scaled")
    return q


def test_fp64_badly_scaled_columns():
    p = _badly_scaled(synth.make_config(0))
    _say("case fp64 badly scaled tiny")
    g = run_gpu(p)
    o = oracle_solve(p)
    _check(p, g, o)


# ---------------------------------------------------------- mixed precision
MIXED = [
    ("tiny", None, {}),
    ("leafy-tiles", (30, 3, 200, 4, 30, 0, 2), {}),
    ("leafy-600", (12, 7, 600, 3, 25, 50, 5), {}),
    ("leafy-600-subst", (12, 7, 600, 3, 25, 50, 5), {"root_inverse": 0}),
    ("leafy-dense-root", (5, 6, 90, 3, 10, 20, 4), {"leaf_max_work": 0.0}),
]


@pytest.mark.parametrize("case", MIXED, ids=[c[0] for c in MIXED])
def test_mixed_parity(case):
    name, shape, opts = case
    p = synth.make_config(0) if shape is None else synth.make_random_leafy(*shape)
    _say(f"case mixed {name} m={p.m} n={p.n} opts={opts}")
    g = run_gpu(p, precision=1, **opts)
    o = oracle_solve(p)
    assert g["info"]["precision"] == 1
    _check(p, g, o, tol_x=TOL_X_MIXED, tol_d=TOL_D_MIXED)


def test_mixed_badly_scaled_columns():
    p = _badly_scaled(synth.make_config(0), seed=1)
    _say("case mixed badly scaled tiny")
    g = run_gpu(p, precision=1)
    o = oracle_solve(p)
    _check(p, g, o, tol_x=TOL_X_MIXED, tol_d=TOL_D_MIXED)


@pytest.mark.timeout(900)
def test_mixed_medium_config_parity():
    p, _, o = _medium()
    _say(f"case mixed medium config m={p.m} n={p.n}")
    g = run_gpu(p, precision=1)
    _check(p, g, o, tol_x=TOL_X_MIXED, tol_d=TOL_D_MIXED)


# ------------------------------------------------------------- edge cases
def _problem_from_rows(rows, n, seed=0, name="edge"):
    """CSR problem from a list of (cols, vals) rows; y drawn around H x."""
    rng = np.random.default_rng(seed)
    rowptr = np.zeros(len(rows) + 1, dtype=np.int64)
    rowptr[1:] = np.cumsum([len(c) for c, _ in rows])
    col = np.concatenate([np.asarray(c, np.int32) for c, _ in rows]) if rows else \
        np.zeros(0, np.int32)
    val = np.concatenate([np.asarray(v, np.float64) for _, v in rows]) if rows else \
        np.zeros(0)
    m = len(rows)
    w = 0.5 + rng.random(m)
    y = rng.random(m) * 10 + 1
    return synth.Problem(m=m, n=n, n_bg=0, rowptr=rowptr, col=col, val=val, w=w,
                         y=y, x_true=np.ones(n), name=name)


def test_single_unknown():
    p = _problem_from_rows([([0], [2.0]), ([0], [0.5]), ([0], [1.5])], 1)
    _say("case edge n=1")
    g = run_gpu(p)
    a = np.sum(p.w * p.val ** 2)
    assert abs(g["x"][0] - np.sum(p.w * p.val * p.y) / a) <= 1e-14 * abs(g["x"][0])
    assert abs(g["d"][0] - 1.0 / a) <= 1e-14 / a


def test_empty_rows_and_single_root_unknown():
    """Rows with no entries contribute nothing; a root of order 1 is padded
    to a full tile."""
    rows = [([], []), ([0, 3], [1.0, 0.3]), ([1, 3], [0.7, 0.2]), ([], []),
            ([2, 3], [0.4, 0.9]), ([3], [0.6]), ([0], [0.2]), ([1], [0.8]),
            ([2], [0.5]), ([], [])]
    p = _problem_from_rows(rows, 4)
    _say("case edge empty rows, root order 1")
    g = run_gpu(p)
    o = oracle_solve(p)
    _check(p, g, o)
    assert g["info"]["n_root"] >= 1


def test_ragged_root_sizes_across_tile_edges():
    """Dense roots (no leaves) of order 127, 128, 129 and 257: identity
    padding and ragged last tiles of the 64/128/256 blocks."""
    for nr in (127, 128, 129, 257):
        p = synth.make_random(3 * nr, nr, 12, seed=nr)
        _say(f"case edge dense root {nr}")
        g = run_gpu(p, leaf_max_work=0.0)
        assert g["info"]["n_root"] == nr
        o = oracle_solve(p)
        _check(p, g, o)


def _run_blocks(p, block, tile=128, **opts):
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver
    dev = torch.device("cuda")
    s = SpiSolver(p.m, p.n, p.rowptr, p.col, **opts)
    s.potrf_block = block
    s.bulk_tile = tile
    assert s.bulk_tile == tile
    s.set_values(torch.from_numpy(p.val).to(dev), torch.from_numpy(p.w).to(dev))
    s.factor()
    b = s.rhs(torch.from_numpy(p.y).to(dev))
    x = s.solve(b)
    d = s.diag_inv()
    torch.cuda.synchronize()
    out = {"b": b.cpu().numpy(), "x": x.cpu().numpy(), "d": d.cpu().numpy(),
           "info": s.info()}
    s.close()
    return out


def test_sweep_bulk_timers_count_the_bulk_flops():
    """With timing on, the library times the sweeps' bulk updates and sums
    their algorithmic flops: 2 kb per lower-triangle entry outside the band's
    rows and columns and outside the next band's pivot block, i.e.
    2 kb (R(R+1)/2 - kn(kn+1)/2) with R = n - kb rows outside the band and kn
    the next band's width (the roofline figure of the benchmark)."""
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver
    p = synth.make_random(2100, 700, 14, seed=77)
    dev = torch.device("cuda")
    s = SpiSolver(p.m, p.n, p.rowptr, p.col, leaf_max_work=0.0, timing=1)
    s.potrf_block = 128
    s.set_values(torch.from_numpy(p.val).to(dev), torch.from_numpy(p.w).to(dev))
    s.factor()
    i = s.info()
    npad, nb = i["n_root_padded"], 128
    widths = [min(nb, npad - k) for k in range(0, npad, nb)]
    want = 0.0
    for k, w in enumerate(widths):
        kn = widths[k + 1] if k + 1 < len(widths) else 0
        R = npad - w
        cells = R * (R + 1) / 2 - kn * (kn + 1) / 2
        if cells > 0:
            want += 2.0 * w * cells
    _say(f"case bulk timers: {i['flops_sweep_bulk']:.4e} flops in {i['t_sweep_bulk_ms']:.3f} ms")
    assert i["flops_sweep_bulk"] == want
    assert i["t_sweep_bulk_ms"] > 0.0
    s.close()


@pytest.mark.parametrize("tile", [128, 64])
@pytest.mark.parametrize("block", [128, 256, 512])
def test_mixed_sweeps_over_several_bands(block, tile):
    """Mixed precision on a dense root of order 700 (padded 768) with 6, 3 or
    2 bands: bands of 128 and 256 take one binary32 sum per launch, bands of
    512 two sums of 256 terms added in binary64 (the split kernel), for the
    bulk and for the next pivot block's update alike; bulk tiles of 128 and
    64."""
    p = synth.make_random(2100, 700, 14, seed=77)
    o = oracle_solve(p)
    _say(f"case mixed sweeps block={block} tile={tile}")
    g = _run_blocks(p, block, tile, leaf_max_work=0.0, precision=1)
    assert g["info"]["n_root"] == 700 and g["info"]["precision"] == 1
    _check(p, g, o, tol_x=TOL_X_MIXED, tol_d=TOL_D_MIXED)


@pytest.mark.parametrize("tile", [128, 64])
@pytest.mark.parametrize("block", [128, 256, 512])
def test_root_sweeps_over_several_bands(block, tile):
    """Dense root of order 700 (padded 768): 6, 3 or 2 bands, so the
    lookahead band update, the bulk outside both bands and the negated last
    band all run, with bulk tiles of 128 and 64; also the Cholesky route
    (root_inverse=0) on the same system with the same outer block."""
    p = synth.make_random(2100, 700, 14, seed=77)
    o = oracle_solve(p)
    for ri in (1, 0):
        _say(f"case sweeps block={block} tile={tile} root_inverse={ri}")
        g = _run_blocks(p, block, tile, leaf_max_work=0.0, root_inverse=ri)
        assert g["info"]["n_root"] == 700
        _check(p, g, o)


def test_root_sweeps_with_1024_column_bands():
    """FP64 sweeps take bands of up to 1024 columns (the large root's
    autotuned choice): a dense root of order 2300 (padded 2304) in bands of
    1024, 1024 and 256, so a 16-step pivot chain, the lookahead update of a
    1024 pivot block and the negated last band all run.  Mixed precision
    and the Cholesky route refuse the block (their bands stay at 512)."""
    from paper_1305_5683_amd import SpiSolver, SpiError
    p = synth.make_random(6900, 2300, 14, seed=78)
    o = oracle_solve(p)
    _say("case sweeps block=1024 n_root=2300")
    g = _run_blocks(p, 1024, 128, leaf_max_work=0.0)
    assert g["info"]["n_root"] == 2300
    _check(p, g, o)
    for opts in ({"precision": 1}, {"root_inverse": 0}):
        s = SpiSolver(p.m, p.n, p.rowptr, p.col, leaf_max_work=0.0, **opts)
        with pytest.raises(SpiError):
            s.potrf_block = 1024
        s.close()


def test_root_pivot_failure_same_column_both_routes():
    """A dense root made indefinite by strongly negative weights on a few
    rows: the sweeps and the Cholesky factorisation pivot on the same Schur
    complements, so both report the same first failing column."""
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver, SpiError
    p = synth.make_random(1200, 400, 10, seed=5)
    w = p.w.copy()
    w[[300, 301, 302]] = -1e3
    dev = torch.device("cuda")
    cols = []
    for ri in (1, 0):
        s = SpiSolver(p.m, p.n, p.rowptr, p.col, leaf_max_work=0.0, root_inverse=ri)
        s.potrf_block = 128
        s.set_values(torch.from_numpy(p.val).to(dev), torch.from_numpy(w).to(dev))
        _say(f"case root pivot failure root_inverse={ri}")
        with pytest.raises(SpiError) as ei:
            s.factor()
        assert ei.value.status == 3
        cols.append(s.info()["failed_col"])
        s.close()
    _say(f"  failed columns {cols}")
    assert cols[0] == cols[1] and cols[0] >= 0


def test_root_order_original_and_locality_agree():
    """The locality numbering of the root (default) and the original order
    give the same solution and variances (an internal permutation of the
    dense root)."""
    p = synth.make_problem(synth.SkyConfig("order-s24", 24, 300, 9, 4), seed=3)
    o = oracle_solve(p)
    for keep in (0, 1):
        _say(f"case root order keep_root_order={keep}")
        g = run_gpu(p, keep_root_order=keep)
        _check(p, g, o)


def _near_collinear(seed=3, delta=1e-3, far=279):
    """A leafy system whose sky columns 10 and 10 + far are nearly collinear
    (the second = the first times 1 + delta N(0, 1) per row): cond(A) about
    5.6e8 for delta = 1e-3 (measured with numpy)."""
    import scipy.sparse as sp
    p = synth.make_random_leafy(8, 4, 300, 3, 20, 60, seed=seed)
    H = sp.csr_matrix((p.val, p.col, p.rowptr), shape=(p.m, p.n)).toarray()
    rng = np.random.default_rng(seed)
    j1, j2 = p.n_bg + 10, p.n_bg + 10 + far
    nz = H[:, j1] != 0
    H[:, j2] = 0.0
    H[nz, j2] = H[nz, j1] * (1.0 + delta * rng.standard_normal(int(nz.sum())))
    Hs = sp.csr_matrix(H)
    Hs.sort_indices()
    return synth.Problem(m=p.m, n=p.n, n_bg=p.n_bg,
                         rowptr=Hs.indptr.astype(np.int64),
                         col=Hs.indices.astype(np.int32), val=Hs.data.copy(),
                         w=p.w, y=p.y, x_true=p.x_true, name="near-collinear")


def test_mixed_precision_falls_back_to_fp64():
    """cond(A) about 5.6e8 (two nearly collinear sky columns), the root in
    its original order and bands of 128, so the binary32 bulk products
    carry the near-null direction: the mixed refinement stalls far above
    refine_tol = 1e-10 (its corrections stay near 1e-3), while binary64
    reaches it in two steps (measured).  Without opts.fp64_fallback the
    mixed handle reports SPI_E_NOCONV; with it the work is redone in
    binary64: x within 1e-9 of the oracle (the refinement's floor on this
    system is about 1e-11), the variances within 1e-6 of a plain FP64
    handle's (unrefined: about cond(A) times the unit roundoff), spi_info
    reporting the switch; new values bring the handle back to mixed
    precision."""
    torch = _torch()
    from paper_1305_5683_amd import SpiSolver, SpiError
    dev = torch.device("cuda")
    q = _near_collinear(far=1)
    o = oracle_solve(q)
    val = torch.from_numpy(q.val).to(dev)
    w = torch.from_numpy(q.w).to(dev)
    y = torch.from_numpy(q.y).to(dev)
    opts = dict(keep_root_order=1, refine_tol=1e-10, refine_steps=10)

    def handle(**more):
        s = SpiSolver(q.m, q.n, q.rowptr, q.col, **opts, **more)
        s.potrf_block = 128
        s.set_values(val, w)
        return s

    _say(f"case mixed precision fallback n={q.n}")
    s = handle(precision=1)
    s.factor()
    with pytest.raises(SpiError) as ei:
        s.solve(s.rhs(y))
    _say(f"  without the fallback: status {ei.value.status}, last correction "
         f"{s.info()['last_refine_norm']:.1e}")
    assert ei.value.status == 6
    s.close()
    s = handle(precision=0)
    s.factor()
    s.solve(s.rhs(y))
    d_ref = s.diag_inv().cpu().numpy()
    s.close()
    s = handle(precision=1, fp64_fallback=1)
    s.factor()
    x = s.solve(s.rhs(y))
    d = s.diag_inv()
    torch.cuda.synchronize()
    info = s.info()
    x, d = x.cpu().numpy(), d.cpu().numpy()
    ex = np.linalg.norm(x - o["x"]) / np.linalg.norm(o["x"])
    ed = np.max(np.abs(d - d_ref) / d_ref)
    _say(f"  with it: switches {info['fp64_fallbacks']}, err_x {ex:.2e}, d vs FP64 {ed:.2e}")
    assert info["fp64_fallbacks"] == 1 and info["precision"] == 0
    assert ex <= 1e-9
    assert ed <= 1e-6
    # values of a well-conditioned system on the same pattern: mixed again
    val2 = q.val.copy()
    sel = q.col == q.n_bg + 11
    val2[sel] = np.random.default_rng(5).uniform(0.5, 1.0, int(sel.sum()))
    s.set_values(torch.from_numpy(val2).to(dev), w)
    assert s.info()["precision"] == 1
    s.factor()
    s.solve(s.rhs(y))
    info = s.info()
    s.close()
    assert info["precision"] == 1 and info["fp64_fallbacks"] == 1
