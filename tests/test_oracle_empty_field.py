"""Pins of the empty-field oracle (App. A.4-A.5), CPU only.

* The LSQ pattern update is the minimiser of chi^2 over each unit's pattern
  with x fixed: the derivative of chi^2 (evaluated from the whole model by
  the oracle's own chi2) vanishes there and any step away raises chi^2.
* The MLE update preserves each unit's total counts and, with no source
  counts, is the stationary point of the unit's likelihood.
* One interval covering all pointings gives the whole-dataset update.
* Noise-free data: from the true pattern the first pass returns the true
  intensities and keeps the pattern; from U = 1 the loop drives chi^2 to
  zero with a pattern proportional to the true one (the model fixes U only
  up to a common scale of U and the bin intensities).
* chi^2 does not increase from pass to pass.
* Planted mistakes (a sign error in the source counts, the (I t^2)^2
  denominator printed in the per-interval formula) fail the first check.
"""
import dataclasses

import numpy as np
import pytest

import spi_synth as synth
from oracle import empty_field as ef

CFG = synth.SkyConfig("ef-tiny", 16, 150, 7, 5)


@pytest.fixture(scope="module")
def prob():
    p = synth.make_empty_field(CFG, seed=3)
    ptr, rows, unit = synth.empty_field_groups(p)
    return p, ptr, rows, unit


def _x_of(p, val):
    from oracle import oracle_solve
    return oracle_solve(dataclasses.replace(p, val=val), want_diag=False)["x"]


def test_lsq_update_minimises_chi2(prob):
    p, ptr, rows, unit = prob
    t, bg = p.meta["t"], p.meta["bg_pos"]
    U0 = np.ones(len(ptr) - 1)
    x = _x_of(p, p.val)
    U = ef.pattern_update(p.rowptr, p.col, p.val, p.w, p.y, x, bg, t, ptr, rows, U0)

    def c2(Uv):
        return ef.chi2(p.rowptr, p.col, ef.set_background(p.val, bg, t, unit, Uv),
                       p.w, p.y, x)
    base = c2(U)
    for u in (0, 7, 18):
        h = 1e-4 * abs(U[u])
        Up, Um = U.copy(), U.copy()
        Up[u] += h
        Um[u] -= h
        cp, cm = c2(Up), c2(Um)
        assert cp > base and cm > base
        assert abs(cp - cm) / (2 * h) <= 1e-6 * base / abs(U[u])   # derivative ~ 0
    assert base < c2(U0)


def _bad_sign_update(p, x, bg, t, ptr, rows, U0):
    """Planted: source counts added instead of subtracted."""
    _, s, I = ef.row_parts(p.rowptr, p.col, p.val, x, bg)
    U = U0.copy()
    for u in range(len(ptr) - 1):
        r = rows[ptr[u]:ptr[u + 1]]
        g = I[r] * t[r]
        U[u] = np.sum((p.y[r] + s[r]) * g * p.w[r]) / np.sum(g * g * p.w[r])
    return U


def _t_squared_update(p, x, bg, t, ptr, rows, U0):
    """Planted: the (I t^2)^2 denominator."""
    _, s, I = ef.row_parts(p.rowptr, p.col, p.val, x, bg)
    U = U0.copy()
    for u in range(len(ptr) - 1):
        r = rows[ptr[u]:ptr[u + 1]]
        g = I[r] * t[r]
        U[u] = np.sum((p.y[r] - s[r]) * g * p.w[r]) / np.sum((I[r] * t[r] ** 2) ** 2 * p.w[r])
    return U


def test_planted_update_mistakes_are_caught(prob):
    p, ptr, rows, unit = prob
    t, bg = p.meta["t"], p.meta["bg_pos"]
    U0 = np.ones(len(ptr) - 1)
    x = _x_of(p, p.val)

    def c2(Uv):
        return ef.chi2(p.rowptr, p.col, ef.set_background(p.val, bg, t, unit, Uv),
                       p.w, p.y, x)
    for bad in (_bad_sign_update, _t_squared_update):
        U = bad(p, x, bg, t, ptr, rows, U0)
        Up = U.copy()
        Up[3] *= 1.0 + 1e-4
        Um = U.copy()
        Um[3] *= 1.0 - 1e-4
        assert not (c2(Up) > c2(U) and c2(Um) > c2(U)), bad.__name__


def test_mle_update_counts_and_stationarity(prob):
    p, ptr, rows, unit = prob
    t, bg = p.meta["t"], p.meta["bg_pos"]
    U0 = np.ones(len(ptr) - 1)
    x = _x_of(p, p.val)
    U = ef.pattern_update(p.rowptr, p.col, p.val, p.w, p.y, x, bg, t, ptr, rows,
                          U0, stat="mle")
    _, s, I = ef.row_parts(p.rowptr, p.col, p.val, x, bg)
    for u in range(len(ptr) - 1):
        r = rows[ptr[u]:ptr[u + 1]]
        assert abs(np.sum(s[r] + U[u] * I[r] * t[r]) - np.sum(p.y[r])) <= \
            1e-10 * np.sum(p.y[r])
    # no source counts: the unit's likelihood -2 sum(e - y ln e), e = U g,
    # is stationary at the update
    x0 = x.copy()
    x0[p.n_bg:] = 0.0
    U = ef.pattern_update(p.rowptr, p.col, p.val, p.w, p.y, x0, bg, t, ptr, rows,
                          U0, stat="mle")
    _, _, I = ef.row_parts(p.rowptr, p.col, p.val, x0, bg)
    for u in (0, 9):
        r = rows[ptr[u]:ptr[u + 1]]
        g = I[r] * t[r]

        def L(Uu):
            e = Uu * g
            return -2.0 * np.sum(e - p.y[r] * np.log(e))
        h = 1e-5 * U[u]
        assert abs(L(U[u] + h) - L(U[u] - h)) / (2 * h) <= 1e-6 * abs(L(U[u])) / U[u]


def test_single_interval_equals_whole_dataset(prob):
    p, ptr, rows, unit = prob
    t, bg = p.meta["t"], p.meta["bg_pos"]
    x = _x_of(p, p.val)
    U1 = ef.pattern_update(p.rowptr, p.col, p.val, p.w, p.y, x, bg, t, ptr, rows,
                           np.ones(len(ptr) - 1))
    pi, ri, ui = synth.empty_field_groups(p, interval=CFG.n_point)
    assert len(pi) == len(ptr)
    Ui = ef.pattern_update(p.rowptr, p.col, p.val, p.w, p.y, x, bg, t, pi, ri,
                           np.ones(len(pi) - 1))
    assert np.allclose(Ui, U1, rtol=1e-14)
    # several intervals: each unit sees only its own rows
    pk, rk, uk = synth.empty_field_groups(p, interval=50)
    assert len(pk) - 1 == 19 * 3
    assert np.all(uk[rk[pk[5]:pk[6]]] == 5)


def test_noise_free_recovery(prob):
    p, ptr, rows, unit = prob
    t, bg = p.meta["t"], p.meta["bg_pos"]
    Ut = p.meta["U_true"]
    vt = p.meta["val_true"]
    H = dataclasses.replace(p, val=vt).scipy_csr()
    q = dataclasses.replace(p, y=H @ p.x_true, w=np.ones(p.m))
    # from the true pattern: exact intensities, pattern kept
    x = _x_of(q, vt)
    assert np.max(np.abs(x - p.x_true) / p.x_true) <= 1e-10
    U = ef.pattern_update(q.rowptr, q.col, vt, q.w, q.y, x, bg, t, ptr, rows, Ut)
    assert np.max(np.abs(U - Ut) / Ut) <= 1e-10
    # from U = 1: chi^2 falls towards zero, the pattern up to a common scale
    out = ef.empty_field_loop(q, np.ones(len(Ut)), ptr, rows, unit, t, bg,
                              itermax=40, rtol=0.0)
    c = [ps["chi2"] for ps in out["passes"]]
    # (down to the rounding floor of the residual, about 1e-28 of the start)
    assert all(b <= a * (1 + 1e-12) + 1e-24 * c[0] for a, b in zip(c, c[1:]))
    assert c[-1] <= 1e-20 * c[0]
    ratio = out["U"] / Ut
    assert np.std(ratio) / np.mean(ratio) <= 1e-3


def test_chi2_does_not_increase_and_loop_stops(prob):
    p, ptr, rows, unit = prob
    t, bg = p.meta["t"], p.meta["bg_pos"]
    out = ef.empty_field_loop(p, np.ones(len(ptr) - 1), ptr, rows, unit, t, bg,
                              itermax=30, rtol=1e-6)
    c = [ps["chi2"] for ps in out["passes"]]
    assert 2 <= len(c) < 30
    assert all(b <= a * (1 + 1e-12) for a, b in zip(c, c[1:]))
    assert c[-2] - c[-1] <= 1e-6 * c[-2]
    assert np.all(out["diag"] > 0)
