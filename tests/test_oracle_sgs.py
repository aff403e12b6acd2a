"""Pins of the symmetric Gauss-Seidel factor (Experiments, baseline methods,
in its symmetric form): L L^T applied as two triangular solves must equal one
forward Gauss-Seidel sweep from zero followed by one backward sweep, written
out from the definition of the method (CPU only)."""
import numpy as np
import pytest

import oracle as O
import pdegen as g


def _sweeps(A, r):
    """z = M^-1 r for symmetric Gauss-Seidel: forward sweep from x = 0 over
    rows 0..n-1 with the latest values, then the backward sweep n-1..0."""
    D = A.to_dense()
    n = A.n
    x = np.zeros(n)
    for i in range(n):
        x[i] = (r[i] - D[i, :] @ x + D[i, i] * x[i]) / D[i, i]
    for i in reversed(range(n)):
        x[i] = (r[i] - D[i, :] @ x + D[i, i] * x[i]) / D[i, i]
    return x


@pytest.mark.parametrize("A", [g.poisson_grid(7, 2), g.heat_system_3d(4, 1e-3, 1, 2)[0],
                               g.fem_p1_delaunay(12, 0, 1)[0], g.random_spd(60, 0.1, 2)],
                         ids=["poisson2d", "heat3d", "fem", "random"])
def test_sgs_factor_equals_two_sweeps(A):
    pat = O.Pattern(A)
    lval = O.sgs_factor(pat, A)
    r = np.random.default_rng(0).standard_normal(A.n)
    z = O.trsv_upper(pat, lval, O.trsv_lower(pat, lval, r))
    ref = _sweeps(A, r)
    np.testing.assert_allclose(z, ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max())


def test_sgs_diagonal_matrix_is_exact():
    """For diagonal A the sweeps solve exactly: P = A, one PCG iteration."""
    A = g.csr_from_dense(np.diag([2.0, 5.0, 0.5, 9.0]))
    pat = O.Pattern(A)
    lval = O.sgs_factor(pat, A)
    np.testing.assert_allclose(lval, np.sqrt([2.0, 5.0, 0.5, 9.0]), rtol=1e-15)
    res = O.pcg(A, np.array([1.0, -2.0, 3.0, 0.5]), pat=pat, lval=lval, tol=1e-12)
    assert res["iters"] == 1 and res["status"] == O.OK


def test_sgs_planted_mistake_fails():
    """A dropped off-diagonal scale (L_ij = A_ij instead of A_ij / sqrt(A_jj))
    breaks the sweep identity, so the pin above can see it."""
    A = g.poisson_grid(5, 2)
    pat = O.Pattern(A)
    wrong = O.sgs_factor(pat, A).copy()
    row = np.repeat(np.arange(A.n), np.diff(pat.lrowptr))
    off = pat.lcol != row
    wrong[off] = np.asarray(A.val)[pat.lsrc][off]
    r = np.random.default_rng(1).standard_normal(A.n)
    z = O.trsv_upper(pat, wrong, O.trsv_lower(pat, wrong, r))
    assert np.linalg.norm(z - _sweeps(A, r)) > 1e-3 * np.linalg.norm(z)
