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


def _root_tiles_per_row(p, order, n_leaf):
    """Mean number of lower 64 x 64 tiles of the dense root that a row's
    root columns touch, for the root numbering in `order`."""
    pos = np.full(p.n, -1, dtype=np.int64)
    pos[order[n_leaf:]] = np.arange(p.n - n_leaf)
    tot = 0.0
    for cols in _rows_of(p):
        r = pos[cols]
        b = np.unique(r[r >= 0] // 64)
        tot += len(b) * (len(b) + 1) / 2
    return tot / p.m


def test_root_numbering_original_order_option():
    p = synth.make_config(0)
    info, order, _, _ = _symbolic(p, keep_root_order=1)
    nl = info["n_leaf"]
    assert np.all(np.diff(order[nl:]) > 0)   # root columns in original order


def test_root_locality_numbering_is_deterministic_and_local():
    """The default root numbering is a permutation of the same root set,
    the same on every call, and puts a row's root columns into fewer
    64-column tiles than the original (row-major sky) order."""
    p = synth.make_problem(synth.SkyConfig("order-s40", 40, 800, 17, 4), seed=1)
    i0, o0, _, _ = _symbolic(p, keep_root_order=1)
    i1, o1, _, _ = _symbolic(p)
    _, o2, _, _ = _symbolic(p)
    nl = i0["n_leaf"]
    assert i1["n_leaf"] == nl and np.array_equal(o0[:nl], o1[:nl])
    assert sorted(o1[nl:].tolist()) == sorted(o0[nl:].tolist())
    assert np.array_equal(o1, o2)
    t_orig = _root_tiles_per_row(p, o0, nl)
    t_loc = _root_tiles_per_row(p, o1, nl)
    print(f"lower root tiles per row: original {t_orig:.1f}, locality {t_loc:.1f}")
    assert t_loc <= 0.75 * t_orig


def test_root_order_option_is_validated():
    from paper_1305_5683_amd import SpiError
    p = synth.make_config(0)
    with pytest.raises(SpiError, match="invalid options"):
        _symbolic(p, keep_root_order=2)


def test_device_memory_cap_option_is_validated():
    from paper_1305_5683_amd import SpiError
    p = synth.make_config(0)
    info, _, _, _ = _symbolic(p, device_mem_cap=1 << 30)
    assert info["device_bytes"] == 0  # host-only analysis holds no device memory
    with pytest.raises(SpiError, match="invalid options"):
        _symbolic(p, device_mem_cap=-1)
    with pytest.raises(SpiError, match="invalid options"):
        _symbolic(p, fp64_fallback=2)


def test_indefinite_needs_the_root_sweeps():
    """opts.indefinite = 1 with the Cholesky route is refused by the
    analysis (host-only check)."""
    import spi_synth as synth
    from paper_1305_5683_amd import symbolic, SpiError
    p = synth.make_indefinite(4, 3, 40, 3, 6, 10, 2, seed=1)
    symbolic(p.m, p.n, p.rowptr, p.col, indefinite=1)
    with pytest.raises(SpiError):
        symbolic(p.m, p.n, p.rowptr, p.col, indefinite=1, root_inverse=0)


def test_analysis_does_not_depend_on_the_thread_count(tmp_path):
    """The analysis runs its phases on host threads (fixed chunks of leaves
    and rows where decisions are sequential, counting sorts over contiguous
    ranges where lists are filled): 1, 3 and 7 threads give the same fronts,
    elimination order and counts, and the same analysis files byte for
    byte (every array of the analysis)."""
    from paper_1305_5683_amd import symbolic_save
    import os
    from paper_1305_5683_amd import symbolic
    p = synth.make_config(0)
    q = synth.make_random_leafy(30, 6, 300, 3, 20, 200, seed=4)
    outs, files = [], []
    old = os.environ.get("SPI_ANALYSIS_THREADS")
    try:
        for nt in ("1", "3", "7"):
            os.environ["SPI_ANALYSIS_THREADS"] = nt
            outs.append([symbolic(r.m, r.n, r.rowptr, r.col) for r in (p, q)])
            blobs = []
            for k, r in enumerate((p, q)):
                f = tmp_path / f"t{nt}_{k}.spia"
                symbolic_save(r.m, r.n, r.rowptr, r.col, f)
                blobs.append(f.read_bytes())
            files.append(blobs)
    finally:
        if old is None:
            os.environ.pop("SPI_ANALYSIS_THREADS", None)
        else:
            os.environ["SPI_ANALYSIS_THREADS"] = old
    assert files[1] == files[0] and files[2] == files[0]
    for other in outs[1:]:
        for (i0, o0, p0, f0), (i1, o1, p1, f1) in zip(outs[0], other):
            assert np.array_equal(o0, o1) and np.array_equal(p0, p1)
            assert np.array_equal(f0, f1)
            for k in ("n_leaf", "n_groups", "n_root", "nnz_l", "asm_tile"):
                assert i0[k] == i1[k]
            assert i0["flops_exec_assembly"] == i1["flops_exec_assembly"]


def test_analysis_file_round_trip(tmp_path):
    """spi_symbolic_save / spi_analysis_file_info: a file gives back the
    counters of the analysis it holds, the same pattern and options write
    the same bytes, and a missing, foreign, truncated or corrupted file is
    refused (host only)."""
    from paper_1305_5683_amd import (symbolic, symbolic_save, analysis_file_info,
                                     SpiError)
    for p, opts in ((synth.make_config(0), {}),
                    (synth.make_random_leafy(12, 7, 600, 3, 25, 50, seed=5),
                     {"max_group": 8, "asm_tile": 128})):
        f1, f2 = tmp_path / "a1.spia", tmp_path / "a2.spia"
        symbolic_save(p.m, p.n, p.rowptr, p.col, f1, **opts)
        symbolic_save(p.m, p.n, p.rowptr, p.col, f2, **opts)
        assert f1.read_bytes() == f2.read_bytes()
        info, _, _, _ = symbolic(p.m, p.n, p.rowptr, p.col, **opts)
        got = analysis_file_info(f1)
        for k in ("m", "n", "nnz_h", "nnz_a", "nnz_l", "n_leaf", "n_groups", "n_root",
                  "n_root_padded", "flops_factor", "flops_selinv", "flops_solve",
                  "flops_assembly", "flops_exec_assembly", "flops_exec_selinv",
                  "flops_root_assembly", "asm_tile"):
            assert got[k] == info[k], k
    data = f1.read_bytes()
    bad = tmp_path / "bad.spia"
    k = len(data) // 3  # inside one of the arrays
    cases = [(data[: len(data) // 2], "truncated"),
             (data[:k] + bytes([data[k] ^ 1]) + data[k + 1:], "corrupted"),
             (b"not an analysis" * 10, "not an analysis file"),
             (data + b"\0", "too long")]
    for blob, why in cases:
        bad.write_bytes(blob)
        with pytest.raises(SpiError, match=why):
            analysis_file_info(bad)
    with pytest.raises(SpiError, match="cannot open"):
        analysis_file_info(tmp_path / "missing.spia")


def test_binding_structs_match_the_c_header(tmp_path):
    """The ctypes mirrors of spi_opts, spi_info_t and spi_pcg_info have the
    C header's size and every field at the C header's offset (a C99 program
    compiled against include/spi.h prints them)."""
    import ctypes as C
    import shutil
    import subprocess
    from paper_1305_5683_amd.spi import spi_opts, spi_info_t, spi_pcg_info
    structs = (("spi_opts", spi_opts), ("spi_info_t", spi_info_t),
               ("spi_pcg_info", spi_pcg_info))
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc is missing")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "spi.h"',
             "int main(void) {"]
    for cname, py in structs:
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-std=c99", "-I", os.path.join(root, "include"), str(src),
                    "-o", str(exe)], check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        s, f, v = line.split()
        got[(s, f)] = int(v)
    for cname, py in structs:
        assert got[(cname, "size")] == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_missing_library_fails_loudly(tmp_path):
    """Without libspi.so the binding raises on first use: there is no CPU
    fallback to route the solver through.  Run in a fresh interpreter so the
    library this process already loaded does not answer."""
    import subprocess
    import sys
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "import paper_1305_5683_amd.spi as spi\n"
        "spi.LIB_PATH = %r\n"
        "try:\n"
        "    spi.load_library(spi.LIB_PATH)\n"
        "except RuntimeError as e:\n"
        "    print('raised:', e)\n"
        "    sys.exit(0)\n"
        "sys.exit(3)\n" % (ROOT, str(tmp_path / "libspi.so")))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "not found" in r.stdout


def test_one_hip_runtime_whatever_the_import_order():
    """Loading the library before torch must not bring a second HIP runtime
    into the process (libspi.so's own dependency next to torch's bundled
    copy): the binding imports torch first.  Checked from the process's
    memory map in a fresh interpreter."""
    import subprocess
    import sys
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_1305_5683_amd import load_library\n"
        "load_library()\n"
        "import torch\n"
        "maps = open('/proc/self/maps').read().splitlines()\n"
        "libs = sorted({l.split()[-1] for l in maps if 'libamdhip64' in l})\n"
        "print(libs)\n"
        "sys.exit(0 if len(libs) == 1 else 3)\n" % ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr


def test_unknown_option_names_are_refused():
    """A misspelt option must not be dropped silently (ctypes structures
    accept any attribute name)."""
    from paper_1305_5683_amd import default_opts
    assert default_opts(precision=1).precision == 1
    with pytest.raises(TypeError):
        default_opts(presicion=1)
