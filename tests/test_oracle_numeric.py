"""Pins for the oracle's floating-point routines: SpMV, triangular
substitution, IC(0), PCG (Appendix algorithm) and the data loss gradient.

References used (none of them is the oracle): NumPy dense products and
Cholesky, SciPy's triangular solver, closed-form eigenpairs of the Dirichlet
Laplacian, the closed-form Cholesky factor of tridiag(-1,2,-1), Higham's
componentwise backward-error bound for substitution, the CG finite
termination / A-orthogonality / A-norm monotonicity / iteration bound
properties, and central finite differences.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
import pdegen as g


# ------------------------------------------------------------------ SpMV
def test_spmv_matches_dense():
    A = g.random_spd(64, 0.2, seed=1)
    x = np.random.default_rng(0).standard_normal(64)
    np.testing.assert_allclose(O.spmv(A, x), A.to_dense() @ x, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("d,m", [(2, 12), (3, 7)])
def test_spmv_closed_form_eigenpairs(d, m):
    """A u_pq = lambda_pq u_pq for the Dirichlet Laplacian, u = prod sin(p pi x h)."""
    A = g.poisson_grid(m, d)
    h = 1.0 / (m + 1)
    rng = np.random.default_rng(d)
    for _ in range(4):
        ks = rng.integers(1, m + 1, size=d)
        coords = np.indices((m,) * d).reshape(d, -1)[::-1] + 1  # x fastest, 1-based
        u = np.prod([np.sin(ks[a] * np.pi * coords[a] * h) for a in range(d)], axis=0)
        lam = sum((2.0 - 2.0 * np.cos(ks[a] * np.pi * h)) for a in range(d)) / h ** 2
        np.testing.assert_allclose(O.spmv(A, u), lam * u, rtol=0, atol=1e-9 * lam)


# ------------------------------------------------------------------ SpTRSV
def _random_lower(seed, n=50):
    A = g.random_spd(n, 0.15, seed=seed)
    pat = O.Pattern(A)
    rng = np.random.default_rng(seed)
    lval = rng.uniform(-1, 1, pat.nnz_l)
    dmask = pat.lcol == np.repeat(np.arange(n), np.diff(pat.lrowptr))
    lval[dmask] = rng.uniform(1.0, 2.0, dmask.sum())
    Ld = np.zeros((n, n))
    Ld[np.repeat(np.arange(n), np.diff(pat.lrowptr)), pat.lcol] = lval
    return A, pat, lval, Ld


def test_trsv_lower_and_upper_match_scipy():
    for seed in range(5):
        A, pat, lval, Ld = _random_lower(seed)
        r = np.random.default_rng(seed + 100).standard_normal(A.n)
        y = O.trsv_lower(pat, lval, r)
        np.testing.assert_allclose(y, sla.solve_triangular(Ld, r, lower=True), rtol=1e-11, atol=1e-12)
        z = O.trsv_upper(pat, lval, y)
        np.testing.assert_allclose(z, sla.solve_triangular(Ld.T, y, lower=False), rtol=1e-11, atol=1e-12)


def test_trsv_componentwise_backward_error_bound():
    """|r - L y| <= gamma_k |L| |y| with gamma_k = k u / (1 - k u) (Higham,
    Accuracy and Stability of Numerical Algorithms, Thm 8.5)."""
    A = g.heat_step_3d(10, 1e-3, np.exp(g.grf((10, 10, 10), 1 / 11, 1.0, 0.1, 5)))
    pat = O.Pattern(A)
    lval, st = O.ic0(pat, A)
    assert st == 0
    r = np.random.default_rng(1).standard_normal(A.n)
    y = O.trsv_lower(pat, lval, r)
    Ld = np.zeros((A.n, A.n))
    Ld[np.repeat(np.arange(A.n), np.diff(pat.lrowptr)), pat.lcol] = lval
    u = 2.0 ** -53
    k = np.diff(pat.lrowptr).max()
    gamma = k * u / (1 - k * u)
    lhs = np.abs(r - Ld @ y)
    rhs = gamma * (np.abs(Ld) @ np.abs(y))
    assert np.all(lhs <= 4 * rhs + 1e-300)


# ------------------------------------------------------------------ IC(0)
def test_ic0_tridiagonal_closed_form():
    """tridiag(-1,2,-1) has no fill: IC(0) is the exact Cholesky factor with
    L_ii = sqrt((i+1)/i), L_{i,i-1} = -sqrt((i-1)/i) (1-based i)."""
    n = 40
    A = g.tridiag_1d(n)
    pat = O.Pattern(A)
    lval, st = O.ic0(pat, A)
    assert st == 0
    i = np.arange(1, n + 1, dtype=float)
    diag = np.sqrt((i + 1) / i)
    sub = -np.sqrt((i[1:] - 1) / i[1:])
    Ld = np.zeros((n, n))
    Ld[np.repeat(np.arange(n), np.diff(pat.lrowptr)), pat.lcol] = lval
    np.testing.assert_allclose(np.diag(Ld), diag, rtol=1e-15)
    np.testing.assert_allclose(np.diag(Ld, -1), sub, rtol=1e-14)
    np.testing.assert_allclose(Ld @ Ld.T, A.to_dense(), atol=1e-14)


def test_ic0_no_fill_pattern_equals_cholesky():
    """Arrow pattern with the hub last: the Cholesky factor has no fill, so
    IC(0) equals numpy.linalg.cholesky."""
    n = 30
    rng = np.random.default_rng(2)
    D = np.diag(rng.uniform(3, 4, n))
    D[-1, :-1] = D[:-1, -1] = rng.uniform(-0.5, 0.5, n - 1)
    D[-1, -1] = 40.0
    A = g.csr_from_dense(D)
    pat = O.Pattern(A)
    lval, st = O.ic0(pat, A)
    assert st == 0
    Lc = np.linalg.cholesky(D)
    np.testing.assert_allclose(lval, Lc[np.repeat(np.arange(n), np.diff(pat.lrowptr)), pat.lcol],
                               rtol=1e-13, atol=1e-15)


def _pattern_product_error(A, pat, lval):
    n = A.n
    Ld = np.zeros((n, n))
    Ld[np.repeat(np.arange(n), np.diff(pat.lrowptr)), pat.lcol] = lval
    P = Ld @ Ld.T
    row = A.row_of_entry()
    return np.max(np.abs(P[row, A.colind] - A.val)) / np.max(np.abs(A.val))


def test_ic0_pattern_invariant():
    """(L L^T)_ij = A_ij on the pattern of A (definition of IC(0))."""
    A = g.poisson_grid(16, 2)
    pat = O.Pattern(A)
    lval, st = O.ic0(pat, A)
    assert st == 0 and _pattern_product_error(A, pat, lval) < 1e-15
    A3 = g.heat_step_3d(9, 1e-3, np.exp(g.grf((9, 9, 9), 0.1, 1.0, 0.1, 2)))
    pat3 = O.Pattern(A3)
    l3, st = O.ic0(pat3, A3)
    assert st == 0 and _pattern_product_error(A3, pat3, l3) < 1e-15
    F = g.fem_p1_delaunay(16, 0, 1)[0]
    patf = O.Pattern(F)
    lf, st = O.ic0(patf, F)
    assert st == 0 and _pattern_product_error(F, patf, lf) < 1e-14


def test_ic0_reports_breakdown_and_shift_recovers():
    D = np.array([[1.0, 2.0, 0.0], [2.0, 1.0, 0.5], [0.0, 0.5, 3.0]])  # indefinite
    A = g.csr_from_dense(D)
    pat = O.Pattern(A)
    _, st = O.ic0(pat, A)
    assert st == 2  # 1-based row of the first non-positive pivot
    _, st = O.ic0(pat, A, shift=4.0)
    assert st == 0


# ------------------------------------------------------------------ PCG
def _spd_dense_csr(n, seed):
    rng = np.random.default_rng(seed)
    Q = rng.standard_normal((n, n))
    D = Q @ Q.T / n + 0.25 * np.eye(n)
    return g.csr_from_dense(D), D


def test_cg_finite_termination_distinct_eigenvalues():
    """P = I: CG terminates after as many steps as A has distinct eigenvalues
    (Krylov space dimension).  n <= 64 with 5 distinct eigenvalues: exactly 5
    iterations reach 1e-12, and x agrees with a dense solve to kappa * 1e-12."""
    for seed, n in ((0, 16), (1, 40), (2, 64)):
        rng = np.random.default_rng(seed)
        Qm, _ = np.linalg.qr(rng.standard_normal((n, n)))
        lam = rng.choice([1.0, 2.0, 3.5, 5.0, 8.0], size=n)
        lam[:5] = [1.0, 2.0, 3.5, 5.0, 8.0]
        D = (Qm * lam) @ Qm.T
        D = 0.5 * (D + D.T)
        A = g.csr_from_dense(D)
        b = np.random.default_rng(seed + 7).standard_normal(n)
        res = O.pcg(A, b, O.PC_NONE, tol=1e-12, maxit=4 * n)
        assert res["status"] == O.OK and res["iters"] == 5
        x = np.linalg.solve(D, b)
        assert np.linalg.norm(res["x"] - x) / np.linalg.norm(x) <= 8.0 * 1e-12


def test_cg_well_conditioned_small_within_n_plus_slack():
    """n <= 64, kappa ~ 15: 1e-12 is reached within n + 2 iterations (finite
    termination up to the orthogonality loss of floating point)."""
    for seed, n in ((0, 16), (1, 40), (2, 64)):
        A, D = _spd_dense_csr(n, seed)
        b = np.random.default_rng(seed + 7).standard_normal(n)
        res = O.pcg(A, b, O.PC_NONE, tol=1e-12, maxit=4 * n)
        assert res["status"] == O.OK and res["iters"] <= n + 2
        x = np.linalg.solve(D, b)
        assert np.linalg.norm(res["x"] - x) / np.linalg.norm(x) <= np.linalg.cond(D) * 1e-12


def test_pcg_exact_preconditioner_one_iteration():
    """On a full pattern IC(0) is the exact Cholesky factor: P = A, so one
    iteration solves the system."""
    A, D = _spd_dense_csr(24, 3)
    pat = O.Pattern(A)
    lval, st = O.ic0(pat, A)
    assert st == 0
    b = np.random.default_rng(4).standard_normal(24)
    res = O.pcg(A, b, O.PC_LLT, pat, lval, tol=1e-10)
    assert res["iters"] == 1
    np.testing.assert_allclose(res["x"], np.linalg.solve(D, b), rtol=1e-9)


@pytest.mark.parametrize("kind", [O.PC_NONE, O.PC_JACOBI, O.PC_LLT])
def test_pcg_a_orthogonality_and_a_norm_monotone(kind):
    A = g.heat_step_3d(6, 1e-2, np.exp(g.grf((6, 6, 6), 1 / 7, 1.0, 0.2, 1)))
    pat = O.Pattern(A)
    lval, _ = O.ic0(pat, A)
    D = A.to_dense()
    b = np.random.default_rng(5).standard_normal(A.n)
    res = O.pcg(A, b, kind, pat, lval, tol=1e-13, keep_p=True)
    Pm = res["P"]
    k = min(8, Pm.shape[0])
    G = Pm[:k] @ D @ Pm[:k].T
    nrm = np.sqrt(np.diag(G))
    off = np.abs(G) / np.outer(nrm, nrm) - np.eye(k)
    assert np.max(np.abs(off)) < 1e-10
    xs = np.linalg.solve(D, b)
    errs = []
    for it in range(1, res["iters"] + 1):
        r = O.pcg(A, b, kind, pat, lval, tol=0.0, maxit=it)
        e = r["x"] - xs
        errs.append(np.sqrt(e @ D @ e))
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-12) for i in range(len(errs) - 1))


def test_pcg_scale_invariance_of_preconditioner():
    A = g.poisson_grid(12, 2)
    pat = O.Pattern(A)
    lval, _ = O.ic0(pat, A)
    b = np.random.default_rng(6).standard_normal(A.n)
    r1 = O.pcg(A, b, O.PC_LLT, pat, lval, tol=1e-10)
    r2 = O.pcg(A, b, O.PC_LLT, pat, 3.7 * lval, tol=1e-10)
    assert r1["iters"] == r2["iters"]
    np.testing.assert_allclose(r1["x"], r2["x"], rtol=1e-9, atol=1e-12)


def test_cg_iteration_bound_c0():
    """k <= ceil(sqrt(kappa)/2 * ln(2/eps)) with the closed-form
    kappa = cot^2(pi h / 2) of the 2D Dirichlet Laplacian, h = 1/33."""
    A = g.poisson_grid(32, 2)
    h = 1 / 33
    kappa = 1.0 / np.tan(np.pi * h / 2) ** 2
    b = np.random.default_rng(0).standard_normal(A.n)
    eps = 1e-8
    res = O.pcg(A, b, O.PC_NONE, tol=eps)
    # relative residual <= sqrt(kappa) * relative A-norm error: tighten eps
    bound = int(np.ceil(0.5 * np.sqrt(kappa) * np.log(2 * np.sqrt(kappa) / eps)))
    assert res["status"] == O.OK and res["iters"] <= bound


def test_jacobi_equals_cg_on_symmetrically_scaled_system():
    A = g.heat_step_3d(6, 1e-2, np.exp(g.grf((6, 6, 6), 1 / 7, 1.0, 0.2, 3)))
    d = O.diag(A)
    S = g.csr_from_dense(A.to_dense() / np.sqrt(np.outer(d, d)), keep_pattern=A.to_dense() != 0)
    b = np.random.default_rng(2).standard_normal(A.n)
    for k in (1, 3, 6):
        rj = O.pcg(A, b, O.PC_JACOBI, tol=0.0, maxit=k)
        rs = O.pcg(S, b / np.sqrt(d), O.PC_NONE, tol=0.0, maxit=k)
        np.testing.assert_allclose(rj["x"], rs["x"] / np.sqrt(d), rtol=1e-10, atol=1e-13)


def test_pcg_zero_rhs_returns_immediately():
    A = g.poisson_grid(8, 2)
    res = O.pcg(A, np.zeros(A.n), O.PC_JACOBI, tol=1e-6)
    assert res["iters"] == 0 and np.all(res["x"] == 0)


# ------------------------------------------------------------------ loss
def test_llt_loss_gradient_finite_differences():
    A = g.poisson_grid(6, 2)
    pat = O.Pattern(A)
    rng = np.random.default_rng(8)
    lval = rng.uniform(-1, 1, pat.nnz_l)
    x = rng.standard_normal(A.n)
    b = rng.standard_normal(A.n)
    loss, grad = O.llt_loss(pat, lval, x, b)
    for _ in range(4):
        v = rng.standard_normal(pat.nnz_l)
        eps = 1e-6
        lp, _ = O.llt_loss(pat, lval + eps * v, x, b, grad=False)
        lm, _ = O.llt_loss(pat, lval - eps * v, x, b, grad=False)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - grad @ v) <= 1e-7 * max(1.0, abs(fd))
    # dense definition of the loss
    Ld = np.zeros((A.n, A.n))
    Ld[np.repeat(np.arange(A.n), np.diff(pat.lrowptr)), pat.lcol] = lval
    assert np.isclose(loss, np.sum((Ld @ Ld.T @ x - b) ** 2), rtol=1e-13)


def test_llt_loss_zero_at_exact_factor():
    """L = chol(A) (IC(0) of a no-fill matrix) and b = A x: loss and gradient vanish."""
    A = g.tridiag_1d(30)
    pat = O.Pattern(A)
    lval, _ = O.ic0(pat, A)
    x = np.random.default_rng(1).standard_normal(A.n)
    b = A.to_dense() @ x
    loss, grad = O.llt_loss(pat, lval, x, b)
    assert loss < 1e-26 and np.max(np.abs(grad)) < 1e-12
