"""FP64 CPU oracle for learned-preconditioner PCG -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The product library neither imports nor links it,
and this package imports nothing from the product: the two share no code.
The only common dependency is the seeded input generator module `pdegen`,
which holds no arithmetic of the method.

Contents (each follows the cited part of the paper):
  * C routines (csrc/lpcg_oracle.c) wrapped here with ctypes: lower pattern,
    transpose, reverse-edge map, forward/backward levels and level sets,
    greedy multicolour ordering and the symmetric permutation, SpMV,
    forward/backward substitution, IC(0), PCG (Appendix algorithm), data loss
    and its gradient (equation loss_Ab); in Python: the symmetric
    Gauss-Seidel factor and the Lanczos extremes of the PCG coefficients.
  * oracle.gnn: the encoder-processor-decoder GNN (technical-details appendix)
    forward and its hand-written reverse-mode derivative, NumPy float64.

Parity status of every function is listed in oracle/gnn.py and below; all are
pinned by the `-m "not gpu"` tests in tests/test_oracle_*.py.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIB, build

_lib = None

PC_NONE, PC_JACOBI, PC_LLT = 0, 1, 2
OK, NOTCONV, BREAKDOWN = 0, 1, 2


class _Prec(C.Structure):
    _fields_ = [("kind", C.c_int), ("diag", C.c_void_p),
                ("lrowptr", C.c_void_p), ("lcol", C.c_void_p), ("lval", C.c_void_p),
                ("urowptr", C.c_void_p), ("ucol", C.c_void_p), ("uval", C.c_void_p)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = C.CDLL(LIB)
        _lib.orc_llt_loss.restype = C.c_double
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- patterns
def lower_pattern(n, rowptr, col):
    """(lrowptr, lcol, src): tril pattern incl. diagonal; src = A-position."""
    rowptr, col = _i32(rowptr), _i32(col)
    lrowptr = np.zeros(n + 1, np.int32)
    lcol = np.zeros(col.shape[0], np.int32)
    src = np.zeros(col.shape[0], np.int32)
    k = lib().orc_lower_pattern(C.c_int(n), _p(rowptr), _p(col), _p(lrowptr), _p(lcol), _p(src))
    return lrowptr, lcol[:k].copy(), src[:k].copy()


def transpose(n, rowptr, col):
    """(trowptr, tcol, tsrc) of the explicit transpose."""
    rowptr, col = _i32(rowptr), _i32(col)
    nnz = int(rowptr[n])
    trowptr = np.zeros(n + 1, np.int32)
    tcol = np.zeros(nnz, np.int32)
    tsrc = np.zeros(nnz, np.int32)
    lib().orc_transpose(C.c_int(n), _p(rowptr), _p(col), _p(trowptr), _p(tcol), _p(tsrc))
    return trowptr, tcol, tsrc


def rev(n, rowptr, col):
    rowptr, col = _i32(rowptr), _i32(col)
    out = np.zeros(col.shape[0], np.int32)
    missing = lib().orc_rev(C.c_int(n), _p(rowptr), _p(col), _p(out))
    return out, int(missing)


def levels_lower(n, lrowptr, lcol):
    lrowptr, lcol = _i32(lrowptr), _i32(lcol)
    lev = np.zeros(n, np.int32)
    nlev = lib().orc_levels_lower(C.c_int(n), _p(lrowptr), _p(lcol), _p(lev))
    return lev, int(nlev)


def levels_upper(n, urowptr, ucol):
    urowptr, ucol = _i32(urowptr), _i32(ucol)
    lev = np.zeros(n, np.int32)
    nlev = lib().orc_levels_upper(C.c_int(n), _p(urowptr), _p(ucol), _p(lev))
    return lev, int(nlev)


def level_sets(level, nlev):
    level = _i32(level)
    n = level.shape[0]
    ptr = np.zeros(nlev + 1, np.int32)
    rows = np.zeros(n, np.int32)
    lib().orc_level_sets(C.c_int(n), _p(level), C.c_int(nlev), _p(ptr), _p(rows))
    return ptr, rows


def greedy_colors(n, lrowptr, lcol):
    """(colour per row, number of colours): first-fit colouring in row order
    on the lower-triangle graph."""
    lrowptr, lcol = _i32(lrowptr), _i32(lcol)
    color = np.zeros(n, np.int32)
    nc = lib().orc_greedy_colors(C.c_int(n), _p(lrowptr), _p(lcol), _p(color))
    return color, int(nc)


def color_order(A, sys_rowptr=None):
    """Multicolour ordering of A: perm[new] = old row, sorting rows by
    (system of the batch, greedy colour) and keeping ascending row order within
    a colour.  Returns (perm, colour per original row, number of colours)."""
    lrowptr, lcol, _ = lower_pattern(A.n, A.rowptr, A.colind)
    color, nc = greedy_colors(A.n, lrowptr, lcol)
    srp = np.array([0, A.n]) if sys_rowptr is None else np.asarray(sys_rowptr)
    row_sys = np.repeat(np.arange(len(srp) - 1), np.diff(srp))
    perm = np.lexsort((np.arange(A.n), color, row_sys)).astype(np.int32)
    return perm, color, nc


def permute_sym(A, perm):
    """P A P^T as a CSR with ascending columns: entry (r, c) of the result is
    A[perm[r], perm[c]].  Every stored entry of A (explicit zeros included)
    is kept."""
    from pdegen.csr import CSR
    perm = np.asarray(perm, np.int64)
    iperm = np.empty_like(perm)
    iperm[perm] = np.arange(A.n)
    erow = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    r, c = iperm[erow], iperm[np.asarray(A.colind, np.int64)]
    order = np.lexsort((c, r))
    rowptr = np.zeros(A.n + 1, np.int64)
    np.add.at(rowptr, r + 1, 1)
    return CSR(A.n, np.cumsum(rowptr).astype(np.int32), c[order].astype(np.int32),
               np.asarray(A.val, np.float64)[order])


class Pattern:
    """Everything the oracle derives from a sparsity pattern."""

    def __init__(self, A):
        self.n = A.n
        self.rowptr, self.col = _i32(A.rowptr), _i32(A.colind)
        self.lrowptr, self.lcol, self.lsrc = lower_pattern(A.n, self.rowptr, self.col)
        self.urowptr, self.ucol, self.usrc = transpose(A.n, self.lrowptr, self.lcol)
        self.rev, self.rev_missing = rev(A.n, self.rowptr, self.col)
        self.flevel, self.nlev_f = levels_lower(A.n, self.lrowptr, self.lcol)
        self.blevel, self.nlev_b = levels_upper(A.n, self.urowptr, self.ucol)
        self.flev_ptr, self.flev_rows = level_sets(self.flevel, self.nlev_f)
        self.blev_ptr, self.blev_rows = level_sets(self.blevel, self.nlev_b)

    @property
    def nnz_l(self):
        return int(self.lrowptr[-1])

    def upper_values(self, lval):
        """Values of U = L^T in U's CSR order."""
        return _f64(lval)[self.usrc]


# ------------------------------------------------------------ numerics
def spmv(A, x):
    y = np.zeros(A.n)
    lib().orc_spmv(C.c_int(A.n), _p(_i32(A.rowptr)), _p(_i32(A.colind)), _p(_f64(A.val)),
                   _p(_f64(x)), _p(y))
    return y


def trsv_lower(pat, lval, r):
    y = np.zeros(pat.n)
    lval, r = _f64(lval), _f64(r)
    lib().orc_trsv_lower(C.c_int(pat.n), _p(pat.lrowptr), _p(pat.lcol), _p(lval), _p(r), _p(y))
    return y


def trsv_upper(pat, lval, y):
    """Solve L^T z = y (built as the explicit transpose of L)."""
    z = np.zeros(pat.n)
    uval = pat.upper_values(lval)
    y = _f64(y)
    lib().orc_trsv_upper(C.c_int(pat.n), _p(pat.urowptr), _p(pat.ucol), _p(uval), _p(y), _p(z))
    return z


def ic0(pat, A, shift=0.0):
    """(lval, status): status 0, or 1-based row of the first bad pivot."""
    aval = _f64(A.val)[pat.lsrc]
    lval = np.zeros(pat.nnz_l)
    st = lib().orc_ic0(C.c_int(pat.n), _p(pat.lrowptr), _p(pat.lcol), _p(aval),
                       C.c_double(shift), _p(lval))
    return lval, int(st)


def diag(A):
    r = A.row_of_entry()
    return _f64(A.val)[A.colind == r]


def sgs_factor(pat, A):
    """Symmetric Gauss-Seidel as a factor P = L L^T (Experiments, baseline
    methods: the triangles are taken from A itself; CG needs a symmetric
    preconditioner, so the forward sweep is followed by the backward one):
    P = (D + A_<) D^-1 (D + A_<)^T, i.e. L = (D + A_<) D^-1/2 on the pattern
    of tril(A): L_ij = A_ij / sqrt(A_jj) (which gives sqrt(A_ii) on the
    diagonal)."""
    aval = _f64(A.val)[pat.lsrc]
    return aval / np.sqrt(diag(A)[pat.lcol])


def pcg(A, b, kind=PC_LLT, pat=None, lval=None, tol=1e-6, maxit=None, x0=None,
        keep_p=False):
    """Appendix PCG.  Returns dict(x, iters, relres, status, hist[, P])."""
    n = A.n
    if maxit is None:
        maxit = n
    x = np.zeros(n) if x0 is None else _f64(x0).copy()
    b = _f64(b)
    P = _Prec()
    P.kind = kind
    keep = []
    if kind == PC_JACOBI:
        d = diag(A)
        keep.append(d)
        P.diag = _p(d).value
    elif kind == PC_LLT:
        if pat is None:
            pat = Pattern(A)
        lv = _f64(lval)
        uv = pat.upper_values(lv)
        keep += [lv, uv]
        P.lrowptr, P.lcol, P.lval = _p(pat.lrowptr).value, _p(pat.lcol).value, _p(lv).value
        P.urowptr, P.ucol, P.uval = _p(pat.urowptr).value, _p(pat.ucol).value, _p(uv).value
    hist = np.zeros(maxit + 1)
    coef = np.zeros(2 * (maxit + 1))
    pv = np.zeros((maxit, n)) if keep_p else None
    iters = C.c_int(0)
    relres = C.c_double(0)
    st = lib().orc_pcg(C.c_int(n), _p(_i32(A.rowptr)), _p(_i32(A.colind)), _p(_f64(A.val)),
                       _p(b), _p(x), C.byref(P), C.c_double(tol), C.c_int(maxit),
                       C.byref(iters), C.byref(relres), _p(hist),
                       _p(pv) if keep_p else None, _p(coef))
    k = iters.value
    out = dict(x=x, iters=k, relres=relres.value, status=int(st),
               hist=hist[:k + 1].copy(), alpha=coef[2:2 * k + 2:2].copy(),
               beta=coef[3:2 * k + 1:2].copy())
    if keep_p:
        out["P"] = pv[:iters.value].copy()
    return out


def lanczos_extremes(alpha, beta):
    """Extreme eigenvalues of the Lanczos tridiagonal of the preconditioned
    operator built from PCG's coefficients (Golub & Van Loan, CG-Lanczos
    connection): T_kk = 1/alpha_k + beta_{k-1}/alpha_{k-1},
    T_k,k+1 = sqrt(beta_k)/alpha_k.  Returns (lambda_min, lambda_max)."""
    from scipy.linalg import eigvalsh_tridiagonal
    a = np.asarray(alpha, np.float64)
    bt = np.asarray(beta, np.float64)[: len(a) - 1]
    d = 1.0 / a
    d[1:] += bt / a[:-1]
    e = np.sqrt(bt) / a[:-1]
    ev = eigvalsh_tridiagonal(d, e)
    return float(ev[0]), float(ev[-1])


def llt_loss(pat, lval, x, b, grad=True):
    """(loss, dloss/dL) of ||L L^T x - b||^2 on L's stored entries."""
    g = np.zeros(pat.nnz_l) if grad else None
    lval, x, b = _f64(lval), _f64(x), _f64(b)
    loss = lib().orc_llt_loss(C.c_int(pat.n), _p(pat.lrowptr), _p(pat.lcol), _p(lval),
                              _p(x), _p(b), _p(g) if grad else None)
    return float(loss), g


def true_relres(A, b, x):
    r = _f64(b) - spmv(A, x)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(r) / (nb if nb > 0 else 1.0))
