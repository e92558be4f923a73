"""Thin ctypes binding of libspi (include/spi.h).

Argument marshalling only: every step of the solve runs in the library's
HIP kernels.  PyTorch supplies device memory (tensors) and the HIP stream.
There is no CPU fallback: if ``libspi.so`` is missing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libspi.so")

SPI_OK, SPI_E_ARG, SPI_E_STATE, SPI_E_NOT_SPD, SPI_E_OOM, SPI_E_HIP, SPI_E_NOCONV = range(7)
SPI_FP64, SPI_MIXED = 0, 1
_STATUS = {0: "SPI_OK", 1: "SPI_E_ARG", 2: "SPI_E_STATE", 3: "SPI_E_NOT_SPD",
           4: "SPI_E_OOM", 5: "SPI_E_HIP", 6: "SPI_E_NOCONV"}

EXPORTED = ["spi_default_opts", "spi_analyze", "spi_set_values", "spi_factor",
            "spi_rhs", "spi_solve", "spi_diag_inv", "spi_symbolic", "spi_info",
            "spi_last_error", "spi_destroy", "spi_lp_param_count",
            "spi_lp_create", "spi_lp_get_params", "spi_lp_loss_grad",
            "spi_lp_train_step", "spi_lp_destroy", "spi_pcg_solve",
            "spi_analyze_like", "spi_batch_create", "spi_batch_run",
            "spi_batch_destroy", "spi_autotune", "spi_get_potrf_block",
            "spi_set_potrf_block", "spi_diag_inv_noalloc", "spi_set_leaf_values",
            "spi_empty_field_update", "spi_empty_field_loop", "spi_mle_terms",
            "spi_mle_newton", "spi_inv_entries", "spi_get_bulk_tile",
            "spi_set_bulk_tile", "spi_debug_poison", "spi_save_analysis",
            "spi_symbolic_save", "spi_analysis_file_info", "spi_analyze_load"]


class spi_opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("max_group", C.c_int32),
                ("leaf_max_work", C.c_double), ("amalg_density", C.c_double),
                ("refine_steps", C.c_int32), ("timing", C.c_int32),
                ("root_inverse", C.c_int32), ("equilibrate", C.c_int32),
                ("refine_tol", C.c_double), ("keep_root_order", C.c_int32),
                ("leaf_lds_cap", C.c_int32), ("selinv_chunk", C.c_int32),
                ("keep_root_sum", C.c_int32), ("indefinite", C.c_int32),
                ("asm_tile", C.c_int32), ("device_mem_cap", C.c_int64),
                ("fp64_fallback", C.c_int32)]


class spi_info_t(C.Structure):
    _fields_ = [("m", C.c_int64), ("n", C.c_int64), ("nnz_h", C.c_int64),
                ("nnz_a", C.c_int64), ("nnz_l", C.c_int64),
                ("n_leaf", C.c_int64), ("n_groups", C.c_int64),
                ("n_root", C.c_int64), ("n_root_padded", C.c_int64),
                ("failed_col", C.c_int64), ("flops_factor", C.c_double),
                ("flops_selinv", C.c_double), ("flops_solve", C.c_double),
                ("flops_assembly", C.c_double), ("t_analyze_ms", C.c_double),
                ("precision", C.c_int32), ("refine_steps_done", C.c_int32),
                ("last_refine_norm", C.c_double), ("t_leaf_ms", C.c_double),
                ("t_extend_ms", C.c_double), ("t_potrf_ms", C.c_double),
                ("t_solve_ms", C.c_double), ("t_trtri_ms", C.c_double),
                ("t_lauum_ms", C.c_double), ("t_selinv_ms", C.c_double),
                ("t_sweep_bulk_ms", C.c_double), ("flops_sweep_bulk", C.c_double),
                ("flops_exec_assembly", C.c_double), ("flops_exec_selinv", C.c_double),
                ("flops_root_assembly", C.c_double),
                ("root_assembly_mode", C.c_int32), ("asm_tile", C.c_int32),
                ("device_bytes", C.c_int64), ("fp64_fallbacks", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class spi_pcg_info(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("outer", C.c_int32),
                ("fell_back", C.c_int32), ("reserved", C.c_int32),
                ("rel_residual", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class SpiError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libspi.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with "
                           "`python -m paper_1305_5683_amd.build`")
    # torch first: libspi.so's HIP and HSA runtime dependencies then resolve
    # to the copies torch has already loaded.  Loaded the other way round,
    # the process holds two HIP runtimes, and the one libspi.so calls finds
    # no device.
    import torch  # noqa: F401
    lib = C.CDLL(path)
    P, I64, I32, D = C.c_void_p, C.c_int64, C.c_int32, C.c_double
    lib.spi_default_opts.argtypes = [C.POINTER(spi_opts)]
    lib.spi_default_opts.restype = None
    lib.spi_analyze.argtypes = [C.POINTER(C.c_void_p), I64, I64, P, P,
                                C.POINTER(spi_opts), P]
    lib.spi_set_values.argtypes = [P, P, P]
    lib.spi_set_leaf_values.argtypes = [P, P]
    lib.spi_empty_field_update.argtypes = [P, P, P, P, P, P, P, P, I32, I32, P,
                                           C.POINTER(D)]
    lib.spi_empty_field_loop.argtypes = [P, P, P, P, P, P, P, I32, I32, I32, D, P,
                                         P, P, P, C.POINTER(I32)]
    lib.spi_mle_terms.argtypes = [P, P, P, P, P, P, C.POINTER(D)]
    lib.spi_mle_newton.argtypes = [P, P, P, P, I32, D, P, P, C.POINTER(I32)]
    lib.spi_factor.argtypes = [P]
    lib.spi_rhs.argtypes = [P, P, P]
    lib.spi_solve.argtypes = [P, P, P, I32, I64]
    lib.spi_diag_inv.argtypes = [P, P]
    lib.spi_diag_inv_noalloc.argtypes = [P, P]
    lib.spi_inv_entries.argtypes = [P, I64, P, P, P]
    lib.spi_symbolic.argtypes = [I64, I64, P, P, C.POINTER(spi_opts),
                                 C.POINTER(spi_info_t), P, P, P]
    lib.spi_info.argtypes = [P, C.POINTER(spi_info_t)]
    lib.spi_last_error.argtypes = [P]
    lib.spi_last_error.restype = C.c_char_p
    lib.spi_destroy.argtypes = [P]
    lib.spi_destroy.restype = None
    lib.spi_lp_param_count.argtypes = [I32]
    lib.spi_lp_create.argtypes = [C.POINTER(C.c_void_p), I32, P]
    lib.spi_lp_get_params.argtypes = [P, P]
    lib.spi_lp_loss_grad.argtypes = [P, P, P, P, P, C.POINTER(D), P]
    lib.spi_lp_train_step.argtypes = [P, P, P, P, P, D, C.POINTER(D)]
    lib.spi_lp_destroy.argtypes = [P]
    lib.spi_lp_destroy.restype = None
    lib.spi_pcg_solve.argtypes = [P, P, P, P, P, D, I32, C.POINTER(spi_pcg_info)]
    lib.spi_analyze_like.argtypes = [C.POINTER(C.c_void_p), P,
                                     C.POINTER(spi_opts), P]
    lib.spi_batch_create.argtypes = [C.POINTER(C.c_void_p), P, I32, I32]
    lib.spi_batch_run.argtypes = [P, P, P, P, P, P]
    lib.spi_batch_destroy.argtypes = [P]
    lib.spi_batch_destroy.restype = None
    lib.spi_autotune.argtypes = [P, C.POINTER(I32)]
    lib.spi_get_potrf_block.argtypes = [P]
    lib.spi_set_potrf_block.argtypes = [P, I32]
    lib.spi_get_bulk_tile.argtypes = [P]
    lib.spi_debug_poison.argtypes = [P]
    lib.spi_set_bulk_tile.argtypes = [P, I32]
    lib.spi_save_analysis.argtypes = [P, C.c_char_p]
    lib.spi_symbolic_save.argtypes = [I64, I64, P, P, C.POINTER(spi_opts), C.c_char_p]
    lib.spi_analysis_file_info.argtypes = [C.c_char_p, C.POINTER(spi_info_t)]
    lib.spi_analyze_load.argtypes = [C.POINTER(C.c_void_p), C.c_char_p,
                                     C.POINTER(spi_opts), P]
    for name in EXPORTED:
        if name not in ("spi_default_opts", "spi_last_error", "spi_destroy",
                        "spi_lp_destroy", "spi_lp_param_count",
                        "spi_batch_destroy"):
            getattr(lib, name).restype = C.c_int
    lib.spi_lp_param_count.restype = C.c_int64
    del I64, I32, D
    _lib = lib
    return lib


def default_opts(**kw) -> spi_opts:
    lib = load_library()
    o = spi_opts()
    lib.spi_default_opts(C.byref(o))
    names = {f[0] for f in spi_opts._fields_}
    for k, v in kw.items():
        if k not in names:   # a ctypes structure would take it silently
            raise TypeError(f"unknown solver option {k!r}")
        setattr(o, k, v)
    return o


def _pattern(rowptr, col):
    rp = np.ascontiguousarray(rowptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    return rp, cl


def symbolic(m, n, rowptr, col, **opts):
    """Host-only analysis: (info dict, elim_order, col_parent, front_of)."""
    lib = load_library()
    rp, cl = _pattern(rowptr, col)
    info = spi_info_t()
    order = np.empty(n, dtype=np.int32)
    parent = np.empty(n, dtype=np.int32)
    front = np.empty(n, dtype=np.int32)
    o = default_opts(**opts)
    st = lib.spi_symbolic(m, n, rp.ctypes.data, cl.ctypes.data, C.byref(o),
                          C.byref(info), order.ctypes.data, parent.ctypes.data,
                          front.ctypes.data)
    if st != SPI_OK:
        raise SpiError(st, lib.spi_last_error(None).decode())
    return info.as_dict(), order, parent, front


def symbolic_save(m, n, rowptr, col, path, **opts):
    """Host-only analysis written to ``path`` (see ``SpiSolver.from_analysis``)."""
    lib = load_library()
    rp, cl = _pattern(rowptr, col)
    o = default_opts(**opts)
    st = lib.spi_symbolic_save(m, n, rp.ctypes.data, cl.ctypes.data, C.byref(o),
                               os.fsencode(path))
    if st != SPI_OK:
        raise SpiError(st, lib.spi_last_error(None).decode())


def analysis_file_info(path) -> dict:
    """Read and check an analysis file; its counters as ``symbolic`` gives them."""
    lib = load_library()
    info = spi_info_t()
    st = lib.spi_analysis_file_info(os.fsencode(path), C.byref(info))
    if st != SPI_OK:
        raise SpiError(st, lib.spi_last_error(None).decode())
    return info.as_dict()


def _ptr(t, n=None, dtype=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device (cuda/hip) torch tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if n is not None and t.numel() < n:
        raise ValueError(f"tensor too small: {t.numel()} < {n}")
    return C.c_void_p(t.data_ptr())


class SpiSolver:
    """One analysed pattern; values, factor and results live on the GPU."""

    def __init__(self, m, n, rowptr, col, stream=None, **opts):
        import torch
        self.lib = load_library()
        self.m, self.n = int(m), int(n)
        rp, cl = _pattern(rowptr, col)
        self.nnz = int(rp[-1])
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.opts = dict(opts)
        h = C.c_void_p()
        o = default_opts(**opts)
        st = self.lib.spi_analyze(C.byref(h), self.m, self.n, rp.ctypes.data,
                                  cl.ctypes.data, C.byref(o),
                                  C.c_void_p(stream.cuda_stream))
        if st != SPI_OK:
            raise SpiError(st, self.lib.spi_last_error(None).decode())
        self.h = h

    @classmethod
    def like(cls, src: "SpiSolver", stream=None, **opts):
        """A handle on ``src``'s pattern with a copy of its analysis; its
        options are ``src``'s, with ``opts`` replacing some of them."""
        import torch
        self = cls.__new__(cls)
        self.lib = src.lib
        self.m, self.n, self.nnz = src.m, src.n, src.nnz
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.opts = {**src.opts, **opts}
        h = C.c_void_p()
        o = default_opts(**self.opts) if opts else None
        st = self.lib.spi_analyze_like(C.byref(h), src.h,
                                       None if o is None else C.byref(o),
                                       C.c_void_p(self.stream.cuda_stream))
        if st != SPI_OK:
            raise SpiError(st, self.lib.spi_last_error(None).decode())
        self.h = h
        return self

    @classmethod
    def from_analysis(cls, path, stream=None, **opts):
        """A handle from an analysis file (``save_analysis`` or
        ``symbolic_save``); ``opts`` as for the constructor, whose analysis
        options the file's replace."""
        import torch
        self = cls.__new__(cls)
        self.lib = load_library()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.opts = dict(opts)
        h = C.c_void_p()
        o = default_opts(**opts)
        st = self.lib.spi_analyze_load(C.byref(h), os.fsencode(path), C.byref(o),
                                       C.c_void_p(self.stream.cuda_stream))
        if st != SPI_OK:
            raise SpiError(st, self.lib.spi_last_error(None).decode())
        self.h = h
        i = self.info()
        self.m, self.n, self.nnz = int(i["m"]), int(i["n"]), int(i["nnz_h"])
        return self

    def save_analysis(self, path):
        """Write this handle's analysis to ``path``."""
        self._check(self.lib.spi_save_analysis(self.h, os.fsencode(path)))

    def _check(self, st):
        if st != SPI_OK:
            raise SpiError(st, self.lib.spi_last_error(self.h).decode())

    def _enter(self, *tensors):
        """Stream order of a call on the handle's stream when that is not the
        current stream: the handle's stream first waits for the current
        stream's work (whatever produced the inputs there), and the tensors'
        memory is kept from reuse until the handle's stream has used it.
        Results are ready in the handle's stream order."""
        import torch
        cur = torch.cuda.current_stream()
        if self.stream == cur:
            return
        self.stream.wait_stream(cur)
        for t in tensors:
            if t is not None:
                t.record_stream(self.stream)

    def autotune(self) -> int:
        """Pick the root POTRF outer block by timing; returns it."""
        c = C.c_int32()
        self._check(self.lib.spi_autotune(self.h, C.byref(c)))
        return c.value

    @property
    def potrf_block(self) -> int:
        return int(self.lib.spi_get_potrf_block(self.h))

    @potrf_block.setter
    def potrf_block(self, v):
        self._check(self.lib.spi_set_potrf_block(self.h, int(v)))

    def debug_poison(self):
        """Fill the handle's device work buffers with NaN bytes (test aid)."""
        self._check(self.lib.spi_debug_poison(self.h))

    @property
    def bulk_tile(self) -> int:
        return int(self.lib.spi_get_bulk_tile(self.h))

    @bulk_tile.setter
    def bulk_tile(self, v):
        self._check(self.lib.spi_set_bulk_tile(self.h, int(v)))

    def set_values(self, val, w):
        import torch
        self._enter(val, w)
        self._check(self.lib.spi_set_values(
            self.h, _ptr(val, self.nnz, torch.float64),
            _ptr(w, self.m, torch.float64)))

    def set_leaf_values(self, val):
        """New values in the leaf-front (background) columns only."""
        import torch
        self._enter(val)
        self._check(self.lib.spi_set_leaf_values(
            self.h, _ptr(val, self.nnz, torch.float64)))

    def factor(self):
        self._enter()
        self._check(self.lib.spi_factor(self.h))

    def rhs(self, y, out=None):
        import torch
        b = out if out is not None else torch.empty(self.n, dtype=torch.float64,
                                                    device=y.device)
        self._enter(y, b)
        self._check(self.lib.spi_rhs(self.h, _ptr(y, self.m, torch.float64),
                                     _ptr(b, self.n, torch.float64)))
        return b

    def solve(self, b, out=None):
        """x = A^-1 b; ``b`` of shape (n,) or (nrhs, n) (column-major n x nrhs)."""
        import torch
        nrhs = 1 if b.dim() == 1 else b.shape[0]
        x = out if out is not None else torch.empty_like(b)
        self._enter(b, x)
        self._check(self.lib.spi_solve(self.h, _ptr(b, nrhs * self.n, torch.float64),
                                       _ptr(x, nrhs * self.n, torch.float64),
                                       nrhs, self.n))
        return x

    def diag_inv(self, out=None):
        import torch
        d = out if out is not None else torch.empty(
            self.n, dtype=torch.float64, device=torch.device("cuda"))
        self._enter(d)
        self._check(self.lib.spi_diag_inv(self.h, _ptr(d, self.n, torch.float64)))
        return d

    def inv_entries(self, rows, cols):
        """(A^-1)_{rows[q], cols[q]} (device int32 tensors) as a device tensor."""
        import torch
        k = int(rows.numel())
        if cols.numel() != k:
            raise ValueError("rows and cols differ in length")
        out = torch.empty(k, dtype=torch.float64, device=rows.device)
        self._enter(rows, cols, out)
        if k:
            self._check(self.lib.spi_inv_entries(
                self.h, k, _ptr(rows, k, torch.int32), _ptr(cols, k, torch.int32),
                _ptr(out, k, torch.float64)))
        else:
            self._check(self.lib.spi_inv_entries(self.h, 0, None, None, None))
        return out

    def diag_inv_noalloc(self, out):
        """diag(A^-1) into ``out`` with the library's fixed scratch array
        (no device allocation; see spi_diag_inv_noalloc)."""
        import torch
        self._enter(out)
        self._check(self.lib.spi_diag_inv_noalloc(
            self.h, _ptr(out, self.n, torch.float64)))
        return out

    def info(self) -> dict:
        i = spi_info_t()
        self._check(self.lib.spi_info(self.h, C.byref(i)))
        return i.as_dict()

    def close(self):
        if getattr(self, "h", None):
            self.lib.spi_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class EmptyField:
    """Device arrays of the empty-field loop (App. A.4-A.5) for one handle:
    background positions, effective times and the rows of each pattern
    unit (see spi_empty_field_update in spi.h)."""

    def __init__(self, solver: "SpiSolver", bg_pos, t, grp_ptr, grp_rows, stat=0):
        import torch
        dev = torch.device("cuda")
        self.s = solver
        self.bg_pos = torch.as_tensor(np.asarray(bg_pos, np.int64), device=dev)
        self.t = torch.as_tensor(np.asarray(t, np.float64), device=dev)
        self.grp_ptr = torch.as_tensor(np.asarray(grp_ptr, np.int64), device=dev)
        self.grp_rows = torch.as_tensor(np.asarray(grp_rows, np.int32), device=dev)
        self.n_u = int(len(grp_ptr) - 1)
        self.stat = int(stat)

    def _args(self):
        import torch
        s = self.s
        return (_ptr(self.bg_pos, s.m, torch.int64), _ptr(self.t, s.m, torch.float64),
                _ptr(self.grp_ptr, self.n_u + 1, torch.int64),
                _ptr(self.grp_rows, None, torch.int32), self.n_u, self.stat)

    def update(self, val, y, x, U):
        """One closed-form pattern update (U and val's background entries
        in place); returns chi^2 of x with the values before the update."""
        import torch
        s = self.s
        c = C.c_double()
        bg, t, gp, gr, nu, st = self._args()
        s._enter(val, y, x, U, self.bg_pos, self.t, self.grp_ptr, self.grp_rows)
        s._check(s.lib.spi_empty_field_update(
            s.h, _ptr(val, s.nnz, torch.float64), _ptr(y, s.m, torch.float64),
            _ptr(x, s.n, torch.float64), bg, t, gp, gr, nu, st,
            _ptr(U, nu, torch.float64), C.byref(c)))
        return c.value

    def loop(self, val, y, U, itermax=20, rtol=1e-6, want_diag=True):
        """Algorithm 1; returns (x, d or None, chi^2 per pass)."""
        import torch
        s = self.s
        x = torch.empty(s.n, dtype=torch.float64, device=y.device)
        d = torch.empty_like(x) if want_diag else None
        hist = np.zeros(itermax)
        npass = C.c_int32()
        bg, t, gp, gr, nu, st = self._args()
        s._enter(val, y, U, x, d, self.bg_pos, self.t, self.grp_ptr, self.grp_rows)
        s._check(s.lib.spi_empty_field_loop(
            s.h, _ptr(val, s.nnz, torch.float64), _ptr(y, s.m, torch.float64),
            bg, t, gp, gr, nu, st, int(itermax), float(rtol),
            _ptr(U, nu, torch.float64), _ptr(x, s.n, torch.float64),
            None if d is None else _ptr(d, s.n, torch.float64),
            hist.ctypes.data, C.byref(npass)))
        return x, d, hist[:npass.value]


def mle_terms(s: "SpiSolver", val, y, x):
    """Likelihood terms at x: (C, weights y/e^2, H^T (y/e - 1))."""
    import torch
    w = torch.empty(s.m, dtype=torch.float64, device=x.device)
    g = torch.empty(s.n, dtype=torch.float64, device=x.device)
    c = C.c_double()
    s._enter(val, y, x, w, g)
    s._check(s.lib.spi_mle_terms(s.h, _ptr(val, s.nnz, torch.float64),
                                 _ptr(y, s.m, torch.float64),
                                 _ptr(x, s.n, torch.float64),
                                 _ptr(w, s.m, torch.float64),
                                 _ptr(g, s.n, torch.float64), C.byref(c)))
    return c.value, w, g


def mle_newton(s: "SpiSolver", val, y, x, itermax=20, tol=1e-10, want_diag=True):
    """Newton's method from x (in place); returns (x, d or None, C per step)."""
    import torch
    d = torch.empty(s.n, dtype=torch.float64, device=x.device) if want_diag else None
    hist = np.zeros(itermax + 1)
    steps = C.c_int32()
    s._enter(val, y, x, d)
    s._check(s.lib.spi_mle_newton(
        s.h, _ptr(val, s.nnz, torch.float64), _ptr(y, s.m, torch.float64),
        _ptr(x, s.n, torch.float64), int(itermax), float(tol),
        None if d is None else _ptr(d, s.n, torch.float64), hist.ctypes.data,
        C.byref(steps)))
    return x, d, hist[:steps.value + 1]


class SpiLearnedPrecond:
    """The learned diagonal correction of a reference factor (see spi.h):
    a small network on the GPU, trained by the library's own kernels."""

    def __init__(self, hidden, params):
        self.lib = load_library()
        self.hidden = int(hidden)
        self.P = int(self.lib.spi_lp_param_count(self.hidden))
        if self.P < 0:
            raise ValueError("hidden width must be 8, 16 or 32")
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != self.P:
            raise ValueError(f"expected {self.P} parameters, got {p.size}")
        h = C.c_void_p()
        st = self.lib.spi_lp_create(C.byref(h), self.hidden, p.ctypes.data)
        if st != SPI_OK:
            raise SpiError(st, "spi_lp_create failed")
        self.h = h

    def params(self):
        out = np.empty(self.P, dtype=np.float32)
        st = self.lib.spi_lp_get_params(self.h, out.ctypes.data)
        if st != SPI_OK:
            raise SpiError(st, "spi_lp_get_params failed")
        return out

    def loss_grad(self, band: "SpiSolver", ref: "SpiSolver", rhs, x, grad=True):
        import torch
        loss = C.c_double()
        g = np.empty(self.P, dtype=np.float64) if grad else None
        band._enter(rhs, x)
        ref._enter()
        band._check(self.lib.spi_lp_loss_grad(
            self.h, band.h, ref.h, _ptr(rhs, band.n, torch.float64),
            _ptr(x, band.n, torch.float64), C.byref(loss),
            None if g is None else g.ctypes.data))
        return loss.value, g

    def train_step(self, band: "SpiSolver", ref: "SpiSolver", rhs, x, lr):
        import torch
        loss = C.c_double()
        band._enter(rhs, x)
        ref._enter()
        band._check(self.lib.spi_lp_train_step(
            self.h, band.h, ref.h, _ptr(rhs, band.n, torch.float64),
            _ptr(x, band.n, torch.float64), float(lr), C.byref(loss)))
        return loss.value

    def close(self):
        if getattr(self, "h", None):
            self.lib.spi_lp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pcg_solve(band: "SpiSolver", ref: "SpiSolver", b, lp=None, tol=1e-10,
              maxit=500, out=None):
    """x = A_band^-1 b by FP32 PCG with the reference factor (and the learned
    correction ``lp``, if given), FP64 outer residuals, direct fallback.
    Returns (x, info dict)."""
    import torch
    lib = load_library()
    x = out if out is not None else torch.empty_like(b)
    info = spi_pcg_info()
    band._enter(b, x)
    ref._enter()
    band._check(lib.spi_pcg_solve(
        band.h, ref.h, None if lp is None else lp.h,
        _ptr(b, band.n, torch.float64), _ptr(x, band.n, torch.float64),
        float(tol), int(maxit), C.byref(info)))
    return x, info.as_dict()


class SpiBatch:
    """Several handles run together (see spi_batch_run in spi.h)."""

    def __init__(self, solvers, use_graphs=True):
        self.lib = load_library()
        self.solvers = list(solvers)
        arr = (C.c_void_p * len(self.solvers))(*[s.h.value for s in self.solvers])
        h = C.c_void_p()
        st = self.lib.spi_batch_create(C.byref(h), arr, len(self.solvers),
                                       1 if use_graphs else 0)
        if st != SPI_OK:
            raise SpiError(st, "spi_batch_create failed")
        self.h = h

    def run(self, y, rhs, x, d=None):
        """Lists of device tensors, one per system; returns per-system status."""
        import torch
        k = len(self.solvers)

        def arr(ts, cnt, allow_none=False):
            a = (C.c_void_p * k)()
            for i, (t, s) in enumerate(zip(ts, self.solvers)):
                if t is None and allow_none:
                    a[i] = None
                else:
                    a[i] = _ptr(t, cnt(s), torch.float64).value
            return a
        st = (C.c_int32 * k)()
        for i, s in enumerate(self.solvers):
            s._enter(y[i], rhs[i], x[i], None if d is None else d[i])
        ya = arr(y, lambda s: s.m)
        ra = arr(rhs, lambda s: s.n)
        xa = arr(x, lambda s: s.n)
        da = None if d is None else arr(d, lambda s: s.n, allow_none=True)
        self.lib.spi_batch_run(self.h, ya, ra, xa, da, st)
        return [int(v) for v in st]

    def close(self):
        if getattr(self, "h", None):
            self.lib.spi_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
