"""Consistency of the paper's printed tables (CPU; sanity checks of the
figures the design notes quote, not parity of this code).

* Table `sparsity`: the density of A times N^2 gives nz(A) of Table
  `fillin` within the rounding of the printed density (two decimals of a
  percent).
* Its footnote: the density of H times M N gives nz(H) within the same
  rounding.
* Sect. 3.2.2: storing A densely takes N^2 x 8 bytes, 23 GB for N = 55,333
  and 167 GB for N = 149,526 (binary gigabytes).
* Table `fillin`: the factor has at least as many non-zeros as the lower
  triangle of A, (nz(A) + N) / 2, for every matrix.
"""
import os

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_tables.txt")


def _rows(kind):
    out = []
    with open(GOLDEN) as f:
        for line in f:
            p = line.split()
            if p and p[0] == kind:
                out.append([float(v) for v in p[1:]])
    return out


def _within_rounding(count, total, rho_pct):
    # rho printed with two decimals of a percent: +-0.005 %
    lo = (rho_pct - 0.005) / 100.0 * total
    hi = (rho_pct + 0.005) / 100.0 * total
    return lo <= count <= hi


def test_density_of_A_matches_nz_of_A():
    rho_a = {int(n): ra for n, _, ra in _rows("sparsity")}
    checked = 0
    for n, nz_a, _ in _rows("fillin"):
        assert _within_rounding(nz_a, n * n, rho_a[int(n)]), n
        checked += 1
    assert checked == 5


def test_density_of_H_matches_nz_of_H():
    rho_h = {int(n): rh for n, rh, _ in _rows("sparsity")}
    for n, m, nz_h in _rows("nzH"):
        assert _within_rounding(nz_h, m * n, rho_h[int(n)]), n


def test_dense_storage_figures():
    for n, gb in _rows("dense"):
        assert round(n * n * 8 / 2**30) == gb


def test_factor_holds_the_lower_triangle():
    for n, nz_a, nz_l in _rows("fillin"):
        assert nz_l >= (nz_a + n) / 2
