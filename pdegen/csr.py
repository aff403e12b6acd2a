"""Canonical CSR container and assembly helpers (host, NumPy)."""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass
class CSR:
    """Square sparse matrix in canonical CSR.

    rowptr: int32[n+1], colind: int32[nnz] (ascending per row, diagonal
    present), val: float64[nnz].
    """
    n: int
    rowptr: np.ndarray
    colind: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.colind, self.rowptr), shape=(self.n, self.n))

    def to_dense(self) -> np.ndarray:
        return self.to_scipy().toarray()

    def row_of_entry(self) -> np.ndarray:
        return np.repeat(np.arange(self.n, dtype=np.int32), np.diff(self.rowptr))


def canonical_csr(m, n: int | None = None) -> CSR:
    """Canonicalise any scipy sparse matrix: sum duplicates, sort columns,
    make every diagonal entry structurally present (explicit zero if absent).
    Explicit zeros already in m are kept as structural entries."""
    c = sp.coo_matrix(m)
    if n is None:
        n = c.shape[0]
    assert c.shape == (n, n)
    d = np.arange(n, dtype=np.int64)
    rows = np.concatenate([c.row.astype(np.int64), d])
    cols = np.concatenate([c.col.astype(np.int64), d])
    vals = np.concatenate([c.data.astype(np.float64), np.zeros(n)])
    key = rows * n + cols
    order = np.argsort(key, kind="stable")
    key = key[order]
    uniq, start = np.unique(key, return_index=True)
    summed = np.add.reduceat(vals[order], start)
    r = (uniq // n).astype(np.int64)
    col = (uniq % n).astype(np.int32)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, r + 1, 1)
    rowptr = np.cumsum(rowptr)
    assert rowptr[-1] < 2**31
    return CSR(n, rowptr.astype(np.int32), col, summed.astype(np.float64))


def csr_from_dense(d: np.ndarray, keep_pattern: np.ndarray | None = None) -> CSR:
    """Dense -> canonical CSR.  keep_pattern (bool mask) keeps structural zeros."""
    d = np.asarray(d, dtype=np.float64)
    n = d.shape[0]
    mask = d != 0
    if keep_pattern is not None:
        mask = mask | keep_pattern
    mask = mask | np.eye(n, dtype=bool)
    rows, cols = np.nonzero(mask)
    rowptr = np.zeros(n + 1, dtype=np.int32)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int32)
    return CSR(n, rowptr, cols.astype(np.int32), d[rows, cols].copy())


def block_diag_csr(mats: list[CSR]) -> tuple[CSR, np.ndarray]:
    """Stack systems into one block-diagonal CSR.  Returns (csr, sys_rowptr)
    with sys_rowptr[s] the first row of system s."""
    n = sum(m.n for m in mats)
    sys_rowptr = np.zeros(len(mats) + 1, dtype=np.int32)
    rp = [np.zeros(1, dtype=np.int64)]
    cols, vals = [], []
    roff = 0
    eoff = 0
    for s, m in enumerate(mats):
        sys_rowptr[s + 1] = sys_rowptr[s] + m.n
        rp.append(m.rowptr[1:].astype(np.int64) + eoff)
        cols.append(m.colind.astype(np.int64) + roff)
        vals.append(m.val)
        roff += m.n
        eoff += m.nnz
    rowptr = np.concatenate(rp)
    assert rowptr[-1] < 2**31
    return CSR(n, rowptr.astype(np.int32), np.concatenate(cols).astype(np.int32),
               np.concatenate(vals)), sys_rowptr


def permute_csr(a: CSR, perm: np.ndarray) -> CSR:
    """Symmetric relabelling B = P A P^T with new index q holding old index perm[q]."""
    m = a.to_scipy()
    p = np.asarray(perm)
    return canonical_csr(m[p][:, p])
