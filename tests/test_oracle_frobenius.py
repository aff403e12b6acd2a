"""Pins of the oracle's Frobenius loss (equation loss_A) and its gradient."""
import numpy as np

import oracle as O
import pdegen as g
from oracle import gnn


def _pattern_vals(A, seed):
    pat = O.Pattern(A)
    rng = np.random.default_rng(seed)
    lv = rng.uniform(-0.5, 0.5, pat.nnz_l)
    row = np.repeat(np.arange(A.n), np.diff(pat.lrowptr))
    d = pat.lcol == row
    lv[d] = rng.uniform(1.0, 2.0, d.sum())
    return pat, lv


def test_matches_dense_definition():
    A = g.fem_p1_delaunay(9, 1, 2)[0]
    pat, lv = _pattern_vals(A, 0)
    loss, gr = gnn.frobenius_loss(A, lv, pat.lrowptr, pat.lcol)
    L = g.CSR(A.n, pat.lrowptr, pat.lcol, lv).to_dense()
    D = A.to_dense()
    s = np.mean(np.diag(D))
    ref = np.sum((L @ L.T - D) ** 2) / s ** 2
    assert abs(loss - ref) <= 1e-12 * ref
    # dense gradient 4 (L L^T - A) L on the pattern
    Gd = 4 * (L @ L.T - D) @ L / s ** 2
    row = np.repeat(np.arange(A.n), np.diff(pat.lrowptr))
    np.testing.assert_allclose(gr, Gd[row, pat.lcol], rtol=1e-10, atol=1e-12 * np.abs(Gd).max())


def test_gradient_finite_differences():
    A = g.heat_system_3d(4, 1e-2, 1, 2)[0]
    pat, lv = _pattern_vals(A, 1)
    _, gr = gnn.frobenius_loss(A, lv, pat.lrowptr, pat.lcol)
    rng = np.random.default_rng(2)
    v = rng.standard_normal(lv.shape)
    eps = 1e-6
    fp = gnn.frobenius_loss(A, lv + eps * v, pat.lrowptr, pat.lcol)[0]
    fm = gnn.frobenius_loss(A, lv - eps * v, pat.lrowptr, pat.lcol)[0]
    fd = (fp - fm) / (2 * eps)
    assert abs(fd - gr @ v) <= 1e-7 * max(1.0, abs(fd))


def test_zero_at_exact_cholesky():
    A = g.tridiag_1d(40)  # no fill: IC(0) is the exact Cholesky factor
    pat = O.Pattern(A)
    l, _ = O.ic0(pat, A)
    loss, gr = gnn.frobenius_loss(A, l, pat.lrowptr, pat.lcol)
    assert loss <= 1e-26 and np.abs(gr).max() <= 1e-12


def test_diagonal_factor_closed_form():
    """L = c I: ||c^2 I - A||_F^2 = sum_i (c^2 - A_ii)^2 + sum_{i != j} A_ij^2."""
    A = g.poisson_grid(5, 2)
    pat = O.Pattern(A)
    row = np.repeat(np.arange(A.n), np.diff(pat.lrowptr))
    c = 1.7
    lv = np.where(pat.lcol == row, c, 0.0)
    loss, _ = gnn.frobenius_loss(A, lv, pat.lrowptr, pat.lcol)
    D = A.to_dense()
    s = np.mean(np.diag(D))
    off = D - np.diag(np.diag(D))
    ref = (np.sum((c * c - np.diag(D)) ** 2) + np.sum(off ** 2)) / s ** 2
    assert abs(loss - ref) <= 1e-12 * ref
