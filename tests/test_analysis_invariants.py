"""Host analysis: structural invariants of everything it hands to the kernels.

The analysis is written to a file (``symbolic_save``) and read back here
field by field, then checked against definitions computed directly from the
pattern of H in numpy:

* every unknown is a leaf or a root unknown, once; the root numbering and
  the leaf list are inverse maps;
* leaves share no row (the leaf block of A is diagonal);
* fronts partition the leaves; a front's U is exactly the set of root
  unknowns in the rows of its columns; its panel holds p x |U| values;
  the slots (a leaf's rows) point at the leaf's entry of H and at each
  root entry of the row with its position in U;
* row panels hold every row with root entries exactly once, and a panel's
  U is exactly the set of root unknowns of its rows; each panel row's
  entries point at H's root entries with their positions in U, and its
  column of the dense panel starts where the panel layout says;
* the selected-inversion tasks of a front are its 64 x 64 blocks (I, J),
  J <= I, each once, their launch order a permutation, their partial sums
  laid out pivot-major without overlap;
* the root tiles are launched column by column, each once;
* every tile lists exactly the (update, run, run) incidences that the
  updates' U sets define, in increasing update order, leaf fronts first.

No GPU is needed.
"""
import os
import struct

import numpy as np
import pytest

import spi_synth as synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1305_5683_amd", "libspi.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libspi.so not built")

KET = 64  # edge of a selected-inversion block

INT = {"rptr": np.int64, "col ": np.int32, "cptr": np.int64, "crow": np.int32,
       "lcol": np.int32, "lgrp": np.int32, "gcol": np.int64, "gU  ": np.int64,
       "U   ": np.int32, "gpan": np.int64, "rcol": np.int32, "rofc": np.int32,
       "lofc": np.int32, "task": np.int32, "gtsk": np.int64, "tpof": np.int64,
       "sord": np.int32, "tord": np.int32, "iptr": np.int64, "ispl": np.int64,
       "inc ": np.int32, "rprp": np.int64, "rprw": np.int32, "rpUp": np.int64,
       "rpvo": np.int64, "upUo": np.int64, "upQo": np.int64, "upnU": np.int32,
       "upk ": np.int32, "cpos": np.int64, "lslp": np.int64, "gslp": np.int64,
       "srow": np.int32, "srrp": np.int64, "slsr": np.int64, "rrlp": np.int32,
       "rrsr": np.int64, "rprb": np.int64, "rpep": np.int64, "rpeq": np.int32,
       "rpes": np.int64}
SCALAR = {"m   ", "n   ", "nnz ", "ngrp", "nrp ", "rpUb", "nup ", "asmt", "ntil",
          "nrt ", "npad"}


def _read(path):
    """The analysis file's fields by tag (format: magic, version, size, then
    (tag, element size, count, bytes) items, then a 64-bit checksum)."""
    data = open(path, "rb").read()
    assert data[:8] == b"SPIANL01"
    pos, out = 16, {}
    while pos < len(data) - 8:
        tag = data[pos:pos + 4].decode()
        es, cnt = struct.unpack_from("<IQ", data, pos + 4)
        pos += 16
        if tag in INT:
            assert np.dtype(INT[tag]).itemsize == es, tag
            out[tag] = np.frombuffer(data, INT[tag], cnt, pos)
        elif tag in SCALAR:
            assert es in (4, 8) and cnt == 1, tag
            out[tag] = struct.unpack_from("<q" if es == 8 else "<i", data, pos)[0]
        pos += es * cnt
    assert pos == len(data) - 8
    return out


def _runs(U, tile):
    """(tile, first, end) of each maximal run of U (sorted) inside one tile."""
    out, a = [], 0
    while a < len(U):
        t, b = U[a] // tile, a + 1
        while b < len(U) and U[b] // tile == t:
            b += 1
        out.append((int(t), a, b))
        a = b
    return out


def _cases():
    tiny = synth.make_config(0)
    leafy = synth.make_random_leafy(12, 7, 600, 3, 25, 50, seed=5)
    sub = synth.make_problem(synth.subproblem_configs(1, seed=9, side_lo=14, side_hi=14)[0],
                             seed=4)
    return [("tiny", tiny, {}),
            ("tiny-original-order-tile128", tiny, {"keep_root_order": 1, "asm_tile": 128}),
            ("leafy-small-groups", leafy, {"max_group": 3, "asm_tile": 64}),
            ("sub-problem", sub, {})]


@pytest.mark.parametrize("name,p,opts", _cases(), ids=[c[0] for c in _cases()])
def test_analysis_invariants(name, p, opts, tmp_path):
    from paper_1305_5683_amd import symbolic_save
    f = tmp_path / "a.spia"
    symbolic_save(p.m, p.n, p.rowptr, p.col, str(f), **opts)
    a = _read(f)
    m, n = a["m   "], a["n   "]
    rp, col = a["rptr"], a["col "]
    assert np.array_equal(rp, p.rowptr) and np.array_equal(col, p.col)
    rows_of = np.repeat(np.arange(m), np.diff(rp))

    # leaves and root
    rcol, lcol, rofc, lofc = a["rcol"], a["lcol"], a["rofc"], a["lofc"]
    nr = a["nrt "]
    assert len(rcol) == nr and len(rcol) + len(lcol) == n
    assert np.array_equal(np.sort(np.concatenate([rcol, lcol])), np.arange(n))
    assert np.array_equal(rofc[rcol], np.arange(nr))
    assert np.array_equal(lofc[lcol], np.arange(len(lcol)))
    assert np.all(rofc[lcol] < 0) and np.all(lofc[rcol] < 0)
    assert a["npad"] >= nr and (a["npad"] - nr) < 128 and a["npad"] % 128 == 0
    is_leaf = lofc[col] >= 0
    assert np.bincount(rows_of[is_leaf], minlength=m).max(initial=0) <= 1

    # transpose
    cptr, crow = a["cptr"], a["crow"]
    order = np.lexsort((rows_of, col))
    assert np.array_equal(cptr, np.concatenate([[0], np.cumsum(np.bincount(col, minlength=n))]))
    assert np.array_equal(crow, rows_of[order])
    assert np.array_equal(a["cpos"], order)

    def root_entries(r, Ulist):
        """H positions of row r's root entries and their positions in U."""
        e = np.arange(rp[r], rp[r + 1])
        e = e[rofc[col[e]] >= 0]
        return e, np.searchsorted(Ulist, rofc[col[e]])

    # root unknowns of each row
    rroot = [np.unique(rofc[col[rp[r]:rp[r + 1]]]) for r in range(m)]
    rroot = [x[x >= 0] for x in rroot]

    # fronts
    ng, gcol, gU, U, gpan, lgrp = a["ngrp"], a["gcol"], a["gU  "], a["U   "], a["gpan"], a["lgrp"]
    assert gcol[0] == 0 and gcol[-1] == len(lcol) and np.all(np.diff(gcol) >= 1)
    assert np.array_equal(lgrp, np.repeat(np.arange(ng), np.diff(gcol)))
    for g in range(ng):
        Ug = U[gU[g]:gU[g + 1]]
        rows = np.concatenate([crow[cptr[c]:cptr[c + 1]] for c in lcol[gcol[g]:gcol[g + 1]]])
        want = np.unique(np.concatenate([rroot[r] for r in rows] + [np.zeros(0, np.int32)]))
        assert np.array_equal(Ug, want), (name, g)
        assert gpan[g + 1] - gpan[g] == (gcol[g + 1] - gcol[g]) * len(Ug)
        # slots of the front's leaves
        for l in range(gcol[g], gcol[g + 1]):
            c = lcol[l]
            sl = np.arange(a["lslp"][l], a["lslp"][l + 1])
            assert np.array_equal(a["srow"][sl], crow[cptr[c]:cptr[c + 1]])
            assert np.array_equal(a["slsr"][sl], order[cptr[c]:cptr[c + 1]])
            for s_ in sl:
                e, pos = root_entries(a["srow"][s_], Ug)
                q = np.arange(a["srrp"][s_], a["srrp"][s_ + 1])
                assert np.array_equal(a["rrsr"][q], e)
                assert np.array_equal(a["rrlp"][q], pos)
                assert np.array_equal(Ug[pos], rofc[col[e]])
    assert np.array_equal(a["gslp"], a["lslp"][gcol])

    # row panels
    nrp, rprp, rprw, rpUp, rpUb = a["nrp "], a["rprp"], a["rprw"], a["rpUp"], a["rpUb"]
    with_root = [r for r in range(m) if len(rroot[r])]
    assert np.array_equal(np.sort(rprw), with_root)
    assert np.all(np.diff(rprw) > 0)   # panels of consecutive rows, in order
    for q in range(nrp):
        Uq = U[rpUb + rpUp[q]:rpUb + rpUp[q + 1]]
        want = np.unique(np.concatenate([rroot[r] for r in rprw[rprp[q]:rprp[q + 1]]]))
        assert np.array_equal(Uq, want), (name, q)
        rpvo = a["rpvo"]
        assert rpvo[q + 1] - rpvo[q] == len(Uq) * (rprp[q + 1] - rprp[q])
        for i in range(rprp[q], rprp[q + 1]):
            assert a["rprb"][i] == rpvo[q] + (i - rprp[q]) * len(Uq)
            e, pos = root_entries(rprw[i], Uq)
            z = np.arange(a["rpep"][i], a["rpep"][i + 1])
            assert np.array_equal(a["rpes"][z], e)
            assert np.array_equal(a["rpeq"][z], pos)
            assert np.array_equal(Uq[pos], rofc[col[e]])

    # selected-inversion tasks
    task, gtsk, tpof, sord = a["task"].reshape(-1, 3), a["gtsk"], a["tpof"], a["sord"]
    assert len(task) == gtsk[-1] == len(sord)
    assert np.array_equal(np.sort(sord), np.arange(len(task)))
    for g in range(ng):
        nb = -(-(gU[g + 1] - gU[g]) // KET)
        pg = gcol[g + 1] - gcol[g]
        tg = task[gtsk[g]:gtsk[g + 1]]
        assert np.all(tg[:, 0] == g)
        want = {(I, J) for I in range(nb) for J in range(I + 1)}
        got = [(int(I), int(J)) for I, J in tg[:, 1:]]
        assert len(got) == len(want) and set(got) == want
        # pivot-major partial sums: task t of the front owns p entries from
        # tpof[t], consecutive tasks one entry apart
        assert np.array_equal(np.diff(tpof[gtsk[g]:gtsk[g + 1] + 1]),
                              np.full(len(tg), pg))

    # root tiles and incidences
    if not nr:
        return
    tile, ntil, tord = a["asmt"], a["ntil"], a["tord"]
    T = a["npad"] // tile
    assert ntil == T * (T + 1) // 2
    assert np.array_equal(tord, [I * (I + 1) // 2 + J for J in range(T) for I in range(J, T)])
    upUo, upnU, upk, nup = a["upUo"], a["upnU"], a["upk "], a["nup "]
    assert nup == ng + nrp
    want = {}
    for u in range(nup):
        if upk[u] == 0:
            continue
        runs = _runs(U[upUo[u]:upUo[u] + upnU[u]], tile)
        for x in range(len(runs)):
            for y in range(x + 1):
                (I, x0, x1), (J, y0, y1) = runs[x], runs[y]
                want.setdefault(I * (I + 1) // 2 + J, []).append(
                    (u, x0, y0, (x1 - x0) | ((y1 - y0) << 16)))
    iptr, inc, ispl = a["iptr"], a["inc "].reshape(-1, 4), a["ispl"]
    for t in range(ntil):
        got = [tuple(int(v) for v in e) for e in inc[iptr[t]:iptr[t + 1]]]
        assert got == want.get(t, []), (name, t)   # same entries, update order
        us = [e[0] for e in got]
        k = ispl[t] - iptr[t]
        assert all(u < ng for u in us[:k]) and all(u >= ng for u in us[k:])
