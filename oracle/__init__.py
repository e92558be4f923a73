"""FP64 CPU oracle for the weighted least-squares solve and its variances.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or
calls this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path: the two only take their inputs from ``spi_synth``.

What it computes (Bouchet et al., "Simultaneous analysis of large
INTEGRAL/SPI datasets", Sect. 2.4.1 and Sect. 3):

* the normal equations ``A = H^T Sigma^-2 H``, ``b = H^T Sigma^-2 y``
  (Sect. 2.4.1, normal equation) -- :mod:`oracle.normal_eq`;
* the solution ``x = A^-1 b`` by a Cholesky factorisation ``A = L L^T``
  followed by forward and backward substitution (Sect. 3.2.2-3.2.3) --
  :mod:`oracle.dense` (tiny cases) and :mod:`oracle.blockchol` (two-block
  factorisation with the background block eliminated first);
* the variances ``Var(x_i) ~ (A^-1)_ii`` (Sect. 2.4.1) as squared column
  norms of ``L^-1`` -- the left-looking formula of Sect. 4.3 with ``D = I``
  -- and, for single entries, by the pruned sparse-right-hand-side solves of
  Sect. 3.3.1 (:func:`oracle.dense.selected_entry_pruned`);
* the elimination-tree notions of Sect. 3.2.1 (:mod:`oracle.etree`);
* certification of results by residuals in extended precision
  (:mod:`oracle.certify`).
"""
from .normal_eq import normal_equations, normal_equations_bruteforce  # noqa: F401
from .dense import (cholesky, forward_subst, backward_subst, solve_dense,  # noqa: F401
                    inverse_from_cholesky, diag_inv_colnorms,
                    selected_entry_pruned)
from .blockchol import BlockCholesky  # noqa: F401
from .reference import oracle_solve  # noqa: F401
