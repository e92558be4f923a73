"""Seeded synthetic coded-mask spectrometer workloads.

This module only *draws inputs*.  It holds none of the solver's arithmetic
(no normal equations, no factorisation, no inversion), so that both the CPU
oracle (``oracle/``) and the HIP path (``paper_1305_5683_amd``) can take their
inputs from it without sharing any of the method's code.

Data model (paper, Sect. 2.2.3 "Problem formulation", eqs. for D^raw and the
background model B = I^bg * U^d * t, and the time-bin expansion H0 -> H):

* ``n_det`` detectors (19), ``n_point`` pointings; one measurement row per
  (pointing p, detector d), row index ``r = p * n_det + d``.
* The sky is an ``S x S`` pixel grid; pixel (x, y) is one constant-intensity
  unknown.  Each pointing sees an ``F x F`` patch centred on a random dither
  position (centre uniform over all pixels, patch clipped at the sky edge).
  Every (row, pixel-in-patch) response is independently non-zero with
  probability ``mask_p`` (coded-mask zeroing) and then ``U(resp_lo, 1)``.
* Background: one unknown per (detector d, time-bin t) with coefficient 1;
  time-bins are runs of consecutive pointings (fixed length, or random
  lengths U{1..10} with the last bin truncated).
* Column order: background columns first (index ``t * n_det + d``), then the
  sky pixels in row-major order (``n_bg + y * S + x``), as in the paper where
  H(1:M, 1:K0) is the background block.
* ``x_true ~ U(1, 50)``, counts ``D ~ Poisson(H x_true)``, weights
  ``W = 1 / max(D, 1)`` (sigma^2 = D), data ``y = D``.

All randomness comes from ``numpy.random.default_rng(seed)`` (PCG64) in a
fixed draw order, so every array is reproducible from ``(config, seed)``.
If some unknown is never observed (an empty column, which would make the
normal matrix singular) the draw is repeated with ``seed + 10**6``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

__all__ = [
    "SkyConfig", "Problem", "CONFIGS", "make_problem", "make_config",
    "make_band", "band_scales_drift", "make_random", "make_random_leafy",
    "make_empty_field", "empty_field_groups",
]

_CHUNK = 256  # pointings per generation chunk (part of the draw order)


@dataclass(frozen=True)
class SkyConfig:
    name: str
    sky: int            # S: the sky is S x S pixels
    n_point: int        # number of pointings
    fov: int            # F: odd side of the observed sky patch
    bin_len: int        # > 0: fixed time-bin length; 0: random U{1..10}
    n_det: int = 19
    mask_p: float = 0.5
    resp_lo: float = 0.05
    x_lo: float = 1.0
    x_hi: float = 50.0


# Workload shapes: tiny, medium and large coded-mask systems (fixed or
# random time-bin lengths).
CONFIGS = {
    0: SkyConfig("tiny-fp64", sky=20, n_point=200, fov=9, bin_len=10),
    1: SkyConfig("medium-fp64", sky=100, n_point=5000, fov=17, bin_len=4),
    2: SkyConfig("large-mixed", sky=180, n_point=40000, fov=31, bin_len=0),
}


@dataclass
class Problem:
    """A weighted least-squares instance ``min ||W^(1/2) (H x - y)||``.

    ``H`` is M x N in CSR form with sorted, unique column indices per row.
    """
    m: int
    n: int
    n_bg: int
    rowptr: np.ndarray   # int64, m + 1
    col: np.ndarray      # int32, nnz
    val: np.ndarray      # float64, nnz
    w: np.ndarray        # float64, m
    y: np.ndarray        # float64, m
    x_true: np.ndarray   # float64, n
    seed: int = 0
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def scipy_csr(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.rowptr),
                             shape=(self.m, self.n))


def _bin_lengths(cfg: SkyConfig, rng: np.random.Generator) -> np.ndarray:
    if cfg.bin_len > 0:
        nb = -(-cfg.n_point // cfg.bin_len)
        lens = np.full(nb, cfg.bin_len, dtype=np.int64)
        lens[-1] = cfg.n_point - cfg.bin_len * (nb - 1)
        return lens
    lens = []
    total = 0
    while total < cfg.n_point:
        draw = rng.integers(1, 11, size=4096)
        for v in draw:
            v = int(min(v, cfg.n_point - total))
            lens.append(v)
            total += v
            if total >= cfg.n_point:
                break
    return np.asarray(lens, dtype=np.int64)


def _pattern_and_values(cfg: SkyConfig, rng: np.random.Generator, progress=None):
    S, F, nd, npnt = cfg.sky, cfg.fov, cfg.n_det, cfg.n_point
    lens = _bin_lengths(cfg, rng)
    n_bins = len(lens)
    bin_of_point = np.repeat(np.arange(n_bins, dtype=np.int64), lens)
    n_bg = n_bins * nd
    cx = rng.integers(0, S, size=npnt)
    cy = rng.integers(0, S, size=npnt)
    h = F // 2
    off = np.arange(-h, h + 1)
    dy_grid, dx_grid = np.meshgrid(off, off, indexing="ij")  # dy outer, dx inner
    dy_flat, dx_flat = dy_grid.ravel(), dx_grid.ravel()

    rowptr = np.zeros(npnt * nd + 1, dtype=np.int64)
    cols_chunks, vals_chunks = [], []
    pos = 0
    n_chunks = -(-npnt // _CHUNK)
    for ci, p0 in enumerate(range(0, npnt, _CHUNK)):
        if progress is not None and ci % max(1, n_chunks // 10) == 0:
            progress(ci / n_chunks)
        p1 = min(npnt, p0 + _CHUNK)
        cnt = p1 - p0
        u_mask = rng.random((cnt, nd, F * F))
        u_val = rng.random((cnt, nd, F * F))
        yy = cy[p0:p1, None] + dy_flat[None, :]          # cnt x F*F
        xx = cx[p0:p1, None] + dx_flat[None, :]
        inside = (yy >= 0) & (yy < S) & (xx >= 0) & (xx < S)
        keep = (u_mask < cfg.mask_p) & inside[:, None, :]  # cnt x nd x F*F
        pix = (yy * S + xx)                               # cnt x F*F
        pix_b = np.broadcast_to(pix[:, None, :], keep.shape)
        sky_cols = (n_bg + pix_b[keep]).astype(np.int32)
        sky_vals = (cfg.resp_lo + (1.0 - cfg.resp_lo) * u_val[keep])
        per_row = keep.reshape(cnt * nd, F * F).sum(axis=1)
        # each row: one background entry (coefficient 1) then its sky entries
        bg_cols = (bin_of_point[p0:p1, None] * nd + np.arange(nd)[None, :]).ravel()
        row_len = per_row + 1
        starts = np.concatenate([[0], np.cumsum(row_len)[:-1]])
        tot = int(row_len.sum())
        c = np.empty(tot, dtype=np.int32)
        v = np.empty(tot, dtype=np.float64)
        c[starts] = bg_cols
        v[starts] = 1.0
        sky_slot = np.ones(tot, dtype=bool)
        sky_slot[starts] = False
        c[sky_slot] = sky_cols
        v[sky_slot] = sky_vals
        cols_chunks.append(c)
        vals_chunks.append(v)
        r0 = p0 * nd
        rowptr[r0 + 1: r0 + cnt * nd + 1] = pos + np.cumsum(row_len)
        pos += tot
    col = np.concatenate(cols_chunks)
    val = np.concatenate(vals_chunks)
    return rowptr, col, val, n_bg, n_bins, lens


def _draw_counts(rowptr, col, val, x_true, rng):
    m = len(rowptr) - 1
    rows = np.repeat(np.arange(m), np.diff(rowptr))
    lam = np.bincount(rows, weights=val * x_true[col], minlength=m)
    d = rng.poisson(lam).astype(np.float64)
    w = 1.0 / np.maximum(d, 1.0)
    return d, w


def make_problem(cfg: SkyConfig, seed: int = 0, progress=None) -> Problem:
    """Draw one coded-mask least-squares instance of shape ``cfg``.
    ``progress(fraction)`` (optional) is called as the pattern is drawn."""
    s = seed
    for _ in range(8):
        rng = np.random.default_rng(s)
        rowptr, col, val, n_bg, n_bins, lens = _pattern_and_values(cfg, rng, progress)
        n = n_bg + cfg.sky * cfg.sky
        counts = np.bincount(col, minlength=n)
        if np.all(counts > 0):
            break
        s += 10**6
    else:  # pragma: no cover - practically unreachable for the shipped shapes
        raise RuntimeError("could not draw a problem with every unknown observed")
    x_true = cfg.x_lo + (cfg.x_hi - cfg.x_lo) * rng.random(n)
    d, w = _draw_counts(rowptr, col, val, x_true, rng)
    m = len(rowptr) - 1
    return Problem(m=m, n=n, n_bg=n_bg, rowptr=rowptr, col=col, val=val, w=w,
                   y=d, x_true=x_true, seed=s, name=cfg.name,
                   meta={"n_bins": n_bins, "sky": cfg.sky, "fov": cfg.fov,
                         "n_point": cfg.n_point, "n_det": cfg.n_det})


def make_config(i: int, seed: int | None = None, progress=None) -> Problem:
    """Workload ``i`` (0 tiny, 1 medium, 2 large); default seed is ``i``."""
    return make_problem(CONFIGS[i], i if seed is None else seed, progress)


def band_scales_drift(b: int, n_bands: int = 256):
    """Smoothly drifting (response, background) scales for band ``b`` (+-20%)."""
    t = 2.0 * np.pi * b / n_bands
    return 1.0 + 0.2 * np.sin(t), 1.0 + 0.2 * np.cos(t)


def make_band(base: Problem, resp_scale: float, bg_scale: float,
              seed: int) -> Problem:
    """Another energy band on ``base``'s sparsity pattern.

    Sky responses are multiplied by ``resp_scale``, background coefficients
    by ``bg_scale``; ``x_true`` is shared; counts are a fresh Poisson draw.
    """
    rng = np.random.default_rng(seed)
    val = base.val.copy()
    is_bg = base.col < base.n_bg
    val[is_bg] *= bg_scale
    val[~is_bg] *= resp_scale
    d, w = _draw_counts(base.rowptr, base.col, val, base.x_true, rng)
    return Problem(m=base.m, n=base.n, n_bg=base.n_bg, rowptr=base.rowptr,
                   col=base.col, val=val, w=w, y=d, x_true=base.x_true,
                   seed=seed, name=base.name + f"-band{seed}",
                   meta=dict(base.meta, resp_scale=resp_scale,
                             bg_scale=bg_scale))


def _csr_from_lists(rows_cols, rows_vals, n):
    rowptr = np.zeros(len(rows_cols) + 1, dtype=np.int64)
    rowptr[1:] = np.cumsum([len(c) for c in rows_cols])
    col = np.concatenate(rows_cols).astype(np.int32) if rows_cols else np.zeros(0, np.int32)
    val = np.concatenate(rows_vals).astype(np.float64) if rows_vals else np.zeros(0)
    return rowptr, col, val


def make_random(m: int, n: int, per_row: int, seed: int,
                integer: bool = False) -> Problem:
    """Unstructured random sparse H (every column observed, full rank w.p. 1).

    ``integer=True`` draws small integer entries and unit weights, so that
    every product and sum in ``H^T W H`` is exact in binary64.
    """
    rng = np.random.default_rng(seed)
    rows_c, rows_v = [], []
    for r in range(m):
        k = int(min(n, max(1, rng.integers(1, 2 * per_row))))
        c = np.sort(rng.choice(n, size=k, replace=False))
        if integer:
            v = rng.integers(1, 5, size=k).astype(np.float64)
        else:
            v = 0.05 + 0.95 * rng.random(k)
        rows_c.append(c)
        rows_v.append(v)
    # guarantee every column is observed: append a diagonal-ish block of rows
    for j in range(n):
        rows_c.append(np.array([j]))
        rows_v.append(np.array([2.0 if integer else 0.5 + rng.random()]))
    rowptr, col, val = _csr_from_lists(rows_c, rows_v, n)
    mm = len(rows_c)
    x_true = 1.0 + 49.0 * rng.random(n)
    if integer:
        w = np.ones(mm)
        y = rng.integers(0, 100, size=mm).astype(np.float64)
    else:
        y, w = _draw_counts(rowptr, col, val, x_true, rng)
    return Problem(m=mm, n=n, n_bg=0, rowptr=rowptr, col=col, val=val, w=w,
                   y=y, x_true=x_true, seed=seed, name=f"random{m}x{n}")


def make_random_leafy(n_groups: int, leaf_per_group: int, n_root: int,
                      rows_per_leaf: int, root_per_row: int, extra_rows: int,
                      seed: int, integer: bool = False) -> Problem:
    """Random problem with private ("leaf") unknowns and shared ("root") ones.

    Each leaf unknown owns ``rows_per_leaf`` rows of its own (no other leaf
    unknown appears in them); each such row also touches ``root_per_row``
    random root unknowns drawn from a window, so leaves within a group have
    overlapping root structure.  ``extra_rows`` rows touch root unknowns
    only.  Leaf columns come first.  Used to exercise general structure:
    ragged groups, rows with no leaf, windows of varying overlap.
    """
    rng = np.random.default_rng(seed)
    n_leaf = n_groups * leaf_per_group
    n = n_leaf + n_root
    rows_c, rows_v = [], []

    def vals(k):
        if integer:
            return rng.integers(1, 5, size=k).astype(np.float64)
        return 0.05 + 0.95 * rng.random(k)

    for g in range(n_groups):
        lo = int(rng.integers(0, max(1, n_root - 1)))
        span = int(min(n_root, max(root_per_row + 1, rng.integers(root_per_row, 4 * root_per_row + 2))))
        lo = min(lo, n_root - span)
        for q in range(leaf_per_group):
            j = g * leaf_per_group + q
            for _ in range(rows_per_leaf):
                k = int(min(span, root_per_row))
                rc = n_leaf + lo + np.sort(rng.choice(span, size=k, replace=False))
                c = np.concatenate([[j], rc])
                rows_c.append(c)
                rows_v.append(vals(len(c)))
    for _ in range(extra_rows):
        k = int(min(n_root, root_per_row))
        c = n_leaf + np.sort(rng.choice(n_root, size=k, replace=False))
        rows_c.append(c)
        rows_v.append(vals(k))
    for j in range(n_leaf, n):  # every root unknown observed
        rows_c.append(np.array([j]))
        rows_v.append(vals(1))
    rowptr, col, val = _csr_from_lists(rows_c, rows_v, n)
    mm = len(rows_c)
    x_true = 1.0 + 49.0 * rng.random(n)
    if integer:
        w = np.ones(mm)
        y = rng.integers(0, 100, size=mm).astype(np.float64)
    else:
        y, w = _draw_counts(rowptr, col, val, x_true, rng)
    return Problem(m=mm, n=n, n_bg=n_leaf, rowptr=rowptr, col=col, val=val,
                   w=w, y=y, x_true=x_true, seed=seed,
                   name=f"leafy{n_groups}x{leaf_per_group}+{n_root}")


def make_indefinite(n_groups: int, leaf_per_group: int, n_root: int,
                    rows_per_leaf: int, root_per_row: int, neg_rows: int,
                    zero_diag: int, seed: int, neg_scale: float = 1.0,
                    partners: int = 8) -> Problem:
    """Random problem whose ``H^T W H`` is symmetric indefinite while the
    leaf unknowns keep positive pivots.

    * Leaf unknowns as in :func:`make_random_leafy` (each owns
      ``rows_per_leaf`` rows that also touch ``root_per_row`` root unknowns
      from a window), with weights U(0.5, 1.5); every root unknown also has
      one row of its own, weight U(0.5, 1.5).
    * ``neg_rows`` rows touch 2..4 random root unknowns (outside the ones
      below) with weights ``-neg_scale`` U(0.5, 1.5).
    * ``zero_diag`` root unknowns z have a zero diagonal: each is seen only by
      row pairs ``e_z + e_k`` (weight +1) and ``e_z - e_k`` (weight -1) with
      ``partners`` other root unknowns k, all values 1, so their entries in
      ``H^T W H`` are exact: ``A_zz = 0`` and ``A_zk = 2``.
    * One row of weight 0 touches every root unknown (structure only: it
      adds exact zeros to ``H^T W H``), so that an analysis with
      ``leaf_max_work = rows_per_leaf (1 + root_per_row)`` takes exactly the
      leaf unknowns as leaves and keeps every root unknown in the root.
    Only random draws and structure here; ``y`` is U(0, 10).
    """
    rng = np.random.default_rng(seed)
    n_leaf = n_groups * leaf_per_group
    n = n_leaf + n_root
    rows_c, rows_v, rows_w = [], [], []
    zcols = n_leaf + np.sort(rng.choice(n_root, size=zero_diag, replace=False)) \
        if zero_diag else np.zeros(0, dtype=np.int64)
    normal = np.setdiff1d(np.arange(n_leaf, n), zcols)
    zset = set(int(z) for z in zcols)

    def add(c, v, w):
        rows_c.append(np.asarray(c))
        rows_v.append(np.asarray(v, dtype=np.float64))
        rows_w.append(float(w))

    for g in range(n_groups):
        span = int(min(len(normal), max(root_per_row + 1,
                                         rng.integers(root_per_row, 4 * root_per_row + 2))))
        lo = int(rng.integers(0, max(1, len(normal) - span + 1)))
        for q in range(leaf_per_group):
            j = g * leaf_per_group + q
            for _ in range(rows_per_leaf):
                k = int(min(span, root_per_row))
                rc = np.sort(normal[lo + rng.choice(span, size=k, replace=False)])
                add(np.concatenate([[j], rc]), 0.05 + 0.95 * rng.random(k + 1),
                    0.5 + rng.random())
    for j in normal:
        add([j], [0.05 + 0.95 * rng.random()], 0.5 + rng.random())
    for _ in range(neg_rows):
        k = int(rng.integers(2, 5))
        c = np.sort(rng.choice(normal, size=min(k, len(normal)), replace=False))
        add(c, 0.05 + 0.95 * rng.random(len(c)), -neg_scale * (0.5 + rng.random()))
    for z in zcols:
        ks = rng.choice(normal, size=min(partners, len(normal)), replace=False)
        for kk in ks:
            c = np.sort(np.array([z, kk]))
            add(c, [1.0, 1.0], 1.0)
            add(c, [1.0, -1.0] if c[0] == z else [-1.0, 1.0], -1.0)
    add(np.arange(n_leaf, n), 0.05 + 0.95 * rng.random(n_root), 0.0)
    rowptr, col, val = _csr_from_lists(rows_c, rows_v, n)
    mm = len(rows_c)
    w = np.array(rows_w)
    y = 10.0 * rng.random(mm)
    assert not (zset & set(range(n_leaf)))
    return Problem(m=mm, n=n, n_bg=n_leaf, rowptr=rowptr, col=col, val=val,
                   w=w, y=y, x_true=np.zeros(n), seed=seed,
                   name=f"indef{n_groups}x{leaf_per_group}+{n_root}")


def lp_init_params(hidden: int, seed: int = 0) -> np.ndarray:
    """Seeded initial weights of the learned-preconditioner network (float32,
    flat layout [W1 (H x 3), b1, W2 (H x H), b2, w3, b3, wl (3)]):
    Gaussian weights scaled by 1/sqrt(fan-in), zero biases, zero skip.
    Only random draws: the network itself is defined elsewhere."""
    rng = np.random.default_rng(seed)
    H, F = hidden, 3
    W1 = rng.standard_normal((H, F)) / np.sqrt(F)
    W2 = rng.standard_normal((H, H)) / np.sqrt(H)
    w3 = rng.standard_normal(H) / np.sqrt(H) * 0.1
    p = np.concatenate([W1.ravel(), np.zeros(H), W2.ravel(), np.zeros(H), w3,
                        [0.0], np.zeros(F)])
    return p.astype(np.float32)


def subproblem_configs(k: int, seed: int = 0, side_lo: int = 30,
                       side_hi: int = 120) -> list:
    """Shapes of ``k`` independent sub-problems of uneven size: sky side
    s ~ U{side_lo..side_hi}, FoV 17, 50% mask, bins of 4 pointings and
    4 * ceil(0.1 s^2) pointings (about 2.9 s^2 unknowns)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(k):
        s = int(rng.integers(side_lo, side_hi + 1))
        n_p = 4 * int(np.ceil(0.1 * s * s))
        out.append(SkyConfig(f"sub{i}-s{s}", s, n_p, 17, 4))
    return out


def make_empty_field(cfg: SkyConfig, seed: int = 0, u_spread: float = 0.25,
                     t_lo: float = 0.8, t_hi: float = 1.2) -> Problem:
    """A coded-mask instance with the paper's background model, for the
    empty-field loop: one background unknown per time bin (its intensity,
    shared by the detectors) whose coefficient in row (pointing p, detector
    d) is ``U^d t_dp``, with the detector pattern ``U`` unknown.

    The same sky draw as :func:`make_problem` (patches, masks, responses),
    then, in this order: the true pattern ``U_true[d] ~ 1 + u_spread
    U(-1, 1)``, effective times ``t_dp ~ U(t_lo, t_hi)`` per row, ``x_true``
    (sky pixels and bin intensities ~ U(1, 50)) and Poisson counts from the
    true model.  The returned values ``val`` hold the background entries for
    ``U = 1`` (the starting pattern, entries ``t_dp``); ``meta`` holds
    ``U_true``, ``t`` (per row), ``bg_pos`` (CSR position of each row's
    background entry: the first of the row) and ``val_true``.
    """
    base = make_problem(cfg, seed)
    nd = cfg.n_det
    rng = np.random.default_rng(seed + 7919)
    m = base.m
    rows = np.repeat(np.arange(m), np.diff(base.rowptr))
    det = np.arange(m) % nd
    old_nbg = base.n_bg
    n_bins = old_nbg // nd
    col = base.col.astype(np.int64)
    is_bg = col < old_nbg
    # background columns: (bin, detector) -> bin; sky columns shift down
    col = np.where(is_bg, col // nd, col - old_nbg + n_bins).astype(np.int32)
    n = base.n - old_nbg + n_bins
    U_true = 1.0 + u_spread * (2.0 * rng.random(nd) - 1.0)
    t = t_lo + (t_hi - t_lo) * rng.random(m)
    x_true = cfg.x_lo + (cfg.x_hi - cfg.x_lo) * rng.random(n)
    val_true = base.val.copy()
    val_true[is_bg] = (U_true[det] * t)[rows[is_bg]]
    d, w = _draw_counts(base.rowptr, col, val_true, x_true, rng)
    val0 = base.val.copy()
    val0[is_bg] = t[rows[is_bg]]
    bg_pos = base.rowptr[:-1].copy()
    return Problem(m=m, n=n, n_bg=n_bins, rowptr=base.rowptr, col=col, val=val0,
                   w=w, y=d, x_true=x_true, seed=seed, name=cfg.name + "-ef",
                   meta=dict(base.meta, U_true=U_true, t=t, bg_pos=bg_pos,
                             val_true=val_true, n_det=nd))


def empty_field_groups(p: Problem, interval: int = 0):
    """Rows grouped by detector pattern unit: by detector (``interval = 0``,
    one unit per detector) or by (detector, interval of ``interval``
    consecutive pointings).  Returns (grp_ptr int64[n_u + 1], grp_rows
    int32, unit_of_row int32[m]): index bookkeeping only."""
    nd = p.meta["n_det"]
    r = np.arange(p.m)
    det = r % nd
    if interval > 0:
        k = (r // nd) // interval
        unit = k * nd + det
    else:
        unit = det
    order = np.argsort(unit, kind="stable")
    n_u = int(unit.max()) + 1
    ptr = np.zeros(n_u + 1, dtype=np.int64)
    ptr[1:] = np.cumsum(np.bincount(unit, minlength=n_u))
    return ptr, order.astype(np.int32), unit.astype(np.int32)
