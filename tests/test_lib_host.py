"""Host-side tests of libspi: exported symbols, argument checks and the
symbolic analysis (no GPU needed).

The elimination tree of the library's ordering is checked against the
oracle's brute-force symbolic factorisation of the permuted pattern.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

import spi_synth as synth
from oracle import etree as et

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1305_5683_amd", "libspi.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB),
                                reason="libspi.so not built")


def _declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"\b(spi_\w+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(LIB)
    names = _declared_functions()
    assert "spi_analyze" in names and "spi_diag_inv" in names
    for name in names:
        assert hasattr(lib, name), name


def test_binding_exports_match_header():
    from paper_1305_5683_amd import spi
    assert sorted(spi.EXPORTED) == _declared_functions()


def _symbolic(p, **kw):
    from paper_1305_5683_amd import symbolic
    return symbolic(p.m, p.n, p.rowptr, p.col, **kw)


def test_symbolic_rejects_malformed_patterns():
    from paper_1305_5683_amd import symbolic, SpiError
    ok_rp = np.array([0, 2, 3], dtype=np.int64)
    with pytest.raises(SpiError, match="strictly increasing"):
        symbolic(2, 3, ok_rp, np.array([1, 0, 2], dtype=np.int32))
    with pytest.raises(SpiError, match="out of range"):
        symbolic(2, 3, ok_rp, np.array([0, 3, 2], dtype=np.int32))
    with pytest.raises(SpiError, match="appears in no row"):
        symbolic(2, 4, ok_rp, np.array([0, 1, 2], dtype=np.int32))
    with pytest.raises(SpiError, match="rowptr"):
        symbolic(2, 3, np.array([0, 3, 2], dtype=np.int64),
                 np.array([0, 1, 2], dtype=np.int32))
    with pytest.raises(SpiError, match="strictly increasing"):
        symbolic(2, 3, ok_rp, np.array([1, 1, 2], dtype=np.int32))


def _rows_of(p):
    return [p.col[p.rowptr[r]:p.rowptr[r + 1]] for r in range(p.m)]


def _check_structure(p, order, parent, front, info):
    n = p.n
    assert sorted(order.tolist()) == list(range(n))
    nl = info["n_leaf"]
    leaves = set(order[:nl].tolist())
    assert info["n_root"] == n - nl
    # leaves are pairwise uncoupled: no row holds two leaf unknowns
    for cols in _rows_of(p):
        assert sum(c in leaves for c in cols) <= 1
    assert np.all(front[order[:nl]] >= 0) and np.all(front[order[nl:]] < 0)
    # fronts are contiguous in the elimination order
    f = front[order[:nl]]
    assert np.all(np.diff(f) >= 0)
    # etree of the permuted pattern (oracle, brute force) for the leaves;
    # the root front is stored dense, a chain
    pos = np.empty(n, dtype=np.int64)
    pos[order] = np.arange(n)
    edges = set()
    for cols in _rows_of(p):
        pc = sorted(pos[c] for c in cols)
        for a in range(len(pc)):
            for b in range(a):
                edges.add((pc[a], pc[b]))
    par_perm = et.etree_from_struct(et.symbolic_cholesky(n, sorted(edges)))
    for k in range(nl):
        want = par_perm[k]
        got = parent[order[k]]
        assert (order[want] if want >= 0 else -1) == got
    for k in range(nl, n):
        got = parent[order[k]]
        assert got == (order[k + 1] if k + 1 < n else -1)


def test_symbolic_tiny_config_structure():
    p = synth.make_config(0)
    info, order, parent, front = _symbolic(p)
    assert info["n_leaf"] == p.n_bg == 380      # background unknowns first
    assert info["n_root"] == 400
    assert info["n_root_padded"] % 128 == 0
    assert info["nnz_a"] > 0
    _check_structure(p, order, parent, front, info)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_symbolic_leafy_structure(seed):
    p = synth.make_random_leafy(n_groups=7, leaf_per_group=5, n_root=50,
                                rows_per_leaf=3, root_per_row=6, extra_rows=9,
                                seed=seed)
    info, order, parent, front = _symbolic(p)
    _check_structure(p, order, parent, front, info)
    assert info["n_leaf"] >= 20    # the private unknowns (and possibly others)


def test_symbolic_unstructured_is_still_valid():
    p = synth.make_random(30, 20, 5, seed=4)
    info, order, parent, front = _symbolic(p)
    _check_structure(p, order, parent, front, info)


def test_symbolic_max_group_and_density_options():
    p = synth.make_config(0)
    i1, _, _, f1 = _symbolic(p, max_group=1)
    assert i1["n_groups"] == i1["n_leaf"]
    i2, _, _, f2 = _symbolic(p, leaf_max_work=0.0)
    assert i2["n_leaf"] == 0 and i2["n_root"] == p.n
