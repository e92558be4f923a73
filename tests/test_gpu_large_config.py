"""GPU: the large coded-mask workload at full size (180 x 180 sky, 40,000
pointings x 19 detectors, 31 x 31 field of view: 760,000 rows, 170,853
unknowns, a dense root of order 32,400), in the launch configuration the
benchmark times there (FP64, root sweeps in bands of 1024 as the autotuner
picks them, 128 x 128 assembly tiles).

The oracle cannot factor a system of this size in seconds, so the checks
are properties that hold at any size, with the oracle's long-double
residuals evaluated on samples (the rows of H that touch the sampled
unknowns, so the sampled entries are exact):

* x: componentwise backward error of 12 background and 12 sky equations,
  ``|r_j| <= 1e-13 (|H|^T W (|y| + |H| |x|))_j`` with
  ``r = H^T W (y - H x)``;
* diag(A^-1): every ``d_j >= 1 / A_jj`` (Cauchy-Schwarz: for SPD A,
  ``(e_j^T A^-1 e_j)(e_j^T A e_j) >= 1``), and for one background and one
  sky unknown, ``d_j`` equals entry j of the solve of ``A z = e_j`` (the
  substitution path through the root inverse and the leaf panels, a route
  independent of the selected inversion) to 1e-10, with that ``z``'s
  sampled backward error checked as for x.
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

import spi_synth as synth
from oracle.certify import apply_normal_ld, normal_residual_ld

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rows_touching(Hc, cols):
    """CSR sub-matrix of the rows of H with a non-zero in one of `cols`."""
    rows = np.unique(Hc[:, cols].tocoo().row)
    return rows


def _sub(H, rows):
    S = H[rows]
    S.sort_indices()
    return S


@pytest.mark.timeout(900)
def test_large_config_full_size_properties():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1305_5683_amd import SpiSolver
    p = synth.make_config(2)
    _say(f"case large config m={p.m} n={p.n} nnz={p.nnz}")
    dev = torch.device("cuda")
    s = SpiSolver(p.m, p.n, p.rowptr, p.col)
    s.potrf_block = 1024
    s.set_values(torch.from_numpy(p.val).to(dev), torch.from_numpy(p.w).to(dev))
    s.factor()
    b = s.rhs(torch.from_numpy(p.y).to(dev))
    x = s.solve(b).cpu().numpy()
    d = s.diag_inv().cpu().numpy()
    i = s.info()
    assert i["asm_tile"] == 128 and i["n_root"] == 32400
    rng = np.random.default_rng(2)
    jb = rng.choice(p.n_bg, 12, replace=False)
    js = p.n_bg + rng.choice(p.n - p.n_bg, 12, replace=False)
    J = np.sort(np.concatenate([jb, js]))
    H = sp.csr_matrix((p.val, p.col, p.rowptr), shape=(p.m, p.n))
    Hc = H.tocsc()
    # diag(A^-1) >= 1 / A_jj for every unknown (A_jj = sum_r w_r h_rj^2)
    a_diag = np.asarray(Hc.multiply(Hc).T @ p.w).ravel()
    assert np.all(d * a_diag >= 1.0 - 1e-12)
    # x: sampled backward error, long-double residual on the touching rows
    R = _rows_touching(Hc, J)
    S = _sub(H, R)
    _say(f"  sampled equations: {len(J)} unknowns, {len(R)} rows, {S.nnz} entries")
    r = normal_residual_ld(S.indptr.astype(np.int64), S.indices, S.data, p.w[R], p.y[R], x)
    Sa = abs(S)
    bound = Sa.T @ (p.w[R] * (np.abs(p.y[R]) + Sa @ np.abs(x)))
    be = np.abs(r[J].astype(np.float64)) / bound[J]
    _say(f"  x: max sampled backward error {be.max():.2e}")
    assert be.max() <= 1e-13
    # variances against inverse columns from the solve path
    for j in (int(jb[0]), int(js[0])):
        e = torch.zeros(p.n, dtype=torch.float64, device=dev)
        e[j] = 1.0
        z = s.solve(e).cpu().numpy()
        Rj = _rows_touching(Hc, [j])
        Sj = _sub(H, Rj)
        Az = apply_normal_ld(Sj.indptr.astype(np.int64), Sj.indices, Sj.data, p.w[Rj], z)
        Sja = abs(Sj)
        bj = (Sja.T @ (p.w[Rj] * (Sja @ np.abs(z))))[j] + 1.0
        be_z = abs(float(1.0 - Az[j])) / bj
        rel = abs(d[j] - z[j]) / z[j]
        _say(f"  d[{j}] = {d[j]:.6e}, z_j = {z[j]:.6e}, rel {rel:.1e}, "
             f"backward error {be_z:.1e}")
        assert be_z <= 1e-13
        assert rel <= 1e-10
    s.close()
