"""MI355X (gfx950) sparse weighted least-squares solver with variances.

``SpiSolver`` wraps the C ABI of ``libspi.so`` (see ``include/spi.h``):
analysis on the host, assembly of ``A = H^T W H``, multifrontal Cholesky,
triangular solves and selected inversion for ``diag(A^-1)`` in HIP kernels.
"""
from .spi import (SpiSolver, SpiError, load_library, symbolic,  # noqa: F401
                  default_opts, SPI_FP64, SPI_MIXED, SpiLearnedPrecond,
                  pcg_solve, SpiBatch, EmptyField, mle_terms, mle_newton,
                  symbolic_save, analysis_file_info)
