"""Pins of the condition-number estimate from PCG's coefficients (appendix
"Condition Number Comparison"): on small systems run to a full Krylov space
the Lanczos extremes equal the extreme eigenvalues of the preconditioned
operator (dense eigenvalues of L^-1 A L^-T, D^-1/2 A D^-1/2 or A); after fewer
steps they lie inside the spectrum (Ritz values interlace)."""
import numpy as np
import pytest

import oracle as O
import pdegen as g


def _precond_spectrum(A, kind, pat, lval):
    D = A.to_dense()
    if kind == O.PC_NONE:
        M = D
    elif kind == O.PC_JACOBI:
        s = 1.0 / np.sqrt(np.diag(D))
        M = D * s[:, None] * s[None, :]
    else:
        L = g.CSR(A.n, pat.lrowptr, pat.lcol, lval).to_dense()
        Li = np.linalg.inv(L)
        M = Li @ D @ Li.T
    ev = np.linalg.eigvalsh((M + M.T) / 2)
    return ev[0], ev[-1]


@pytest.mark.parametrize("kind", [O.PC_NONE, O.PC_JACOBI, O.PC_LLT])
@pytest.mark.parametrize("make", [lambda: g.poisson_grid(6, 2), lambda: g.heat_system_3d(4, 1e-2, 1, 2)[0],
                                  lambda: g.fem_p1_delaunay(8, 0, 1)[0]])
def test_lanczos_extremes_match_dense_spectrum(make, kind):
    A = make()
    pat = O.Pattern(A)
    lval = O.ic0(pat, A)[0] if kind == O.PC_LLT else None
    lo, hi = _precond_spectrum(A, kind, pat, lval)
    b = np.random.default_rng(0).standard_normal(A.n)
    # run to 1e-14: the extremes converge first; with IC(0) the spectrum
    # clusters and PCG stops before the top Ritz value is exact (2e-5 off on
    # 6x6 Poisson), so the bars are 1e-3 / 1e-2 -- a wrong tridiagonal (an
    # index shift, a missing beta/alpha term) is off by O(1)
    r = O.pcg(A, b, kind, pat, lval, tol=1e-14, maxit=A.n)
    lmin, lmax = O.lanczos_extremes(r["alpha"], r["beta"])
    assert lo * (1 - 1e-10) <= lmin <= lmax <= hi * (1 + 1e-10)  # Ritz values interlace
    assert abs(lmax - hi) <= 1e-3 * hi
    assert abs(lmin - lo) <= 1e-2 * lo


def test_ritz_values_inside_spectrum_and_kappa_grows():
    A = g.poisson_grid(12, 2)
    pat = O.Pattern(A)
    lo, hi = _precond_spectrum(A, O.PC_NONE, pat, None)
    b = np.random.default_rng(1).standard_normal(A.n)
    prev = 1.0
    for k in (3, 6, 12, 24):
        r = O.pcg(A, b, O.PC_NONE, tol=1e-30, maxit=k)
        lmin, lmax = O.lanczos_extremes(r["alpha"], r["beta"])
        assert lo * (1 - 1e-10) <= lmin <= lmax <= hi * (1 + 1e-10)
        assert lmax / lmin >= prev * (1 - 1e-12)  # extremes move outwards with k
        prev = lmax / lmin


def test_exact_preconditioner_gives_kappa_one():
    A = g.tridiag_1d(30)  # IC(0) = exact Cholesky: P^-1 A = I
    pat = O.Pattern(A)
    l, _ = O.ic0(pat, A)
    r = O.pcg(A, np.ones(A.n), O.PC_LLT, pat, l, tol=1e-30, maxit=1)
    lmin, lmax = O.lanczos_extremes(r["alpha"], r["beta"])
    assert abs(lmin - 1) <= 1e-12 and abs(lmax - 1) <= 1e-12
