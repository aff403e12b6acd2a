"""Pins for the oracle's integer pattern work: lower triangle, transpose,
reverse-edge map, forward/backward levels and level sets.

Each check is against something other than the oracle: SciPy's tril/transpose,
closed-form level numbers of natural-order grids, and brute-force longest
paths on tiny random DAGs.
"""
import functools
from math import comb

import numpy as np
import scipy.sparse as sp

import oracle as O
import pdegen as g


def test_lower_pattern_matches_scipy_tril():
    A = g.random_spd(60, 0.1, seed=3)
    pat = O.Pattern(A)
    T = sp.tril(A.to_scipy()).tocsr()
    T.sort_indices()
    assert np.array_equal(pat.lrowptr, T.indptr)
    assert np.array_equal(pat.lcol, T.indices)
    assert np.array_equal(A.val[pat.lsrc], T.data)


def test_transpose_matches_scipy():
    A = g.random_spd(50, 0.12, seed=4)
    pat = O.Pattern(A)
    L = sp.csr_matrix((np.arange(pat.nnz_l, dtype=float) + 1, pat.lcol, pat.lrowptr), shape=(A.n, A.n))
    U = L.T.tocsr()
    U.sort_indices()
    assert np.array_equal(pat.urowptr, U.indptr)
    assert np.array_equal(pat.ucol, U.indices)
    assert np.array_equal(pat.usrc + 1, U.data.astype(int))


def test_rev_is_involution_and_swaps_indices():
    A = g.fem_p1_delaunay(12, 0, 1)[0]
    pat = O.Pattern(A)
    assert pat.rev_missing == 0
    k = np.arange(A.nnz)
    assert np.array_equal(pat.rev[pat.rev], k)
    row = A.row_of_entry()
    assert np.array_equal(row[pat.rev], A.colind)
    assert np.array_equal(A.colind[pat.rev], row)


def test_rev_reports_unsymmetric_pattern():
    A = g.csr_from_dense(np.array([[2.0, 1.0, 0.0], [0.0, 2.0, 0.0], [0.0, 0.0, 1.0]]))
    _, missing = O.rev(A.n, A.rowptr, A.colind)
    assert missing == 1


def _grid_levels_closed_form(m, d):
    """Natural order grid: level(i,j,k) = i+j+k (forward), the mirror backward."""
    coords = np.indices((m,) * d).reshape(d, -1)[::-1]  # x fastest
    return coords.sum(axis=0), (m - 1 - coords).sum(axis=0)


def test_grid_levels_closed_form_2d_c0():
    A = g.poisson_grid(32, 2)
    pat = O.Pattern(A)
    fwd, bwd = _grid_levels_closed_form(32, 2)
    assert np.array_equal(pat.flevel, fwd)
    assert np.array_equal(pat.blevel, bwd)
    assert pat.nlev_f == pat.nlev_b == 2 * 31 + 1 == 63


def _level_size_3d(s, m):
    # number of (i,j,k) in [0,m)^3 with i+j+k = s (inclusion-exclusion)
    def c2(x):
        return comb(x, 2) if x >= 2 else 0
    return c2(s + 2) - 3 * c2(s - m + 2) + 3 * c2(s - 2 * m + 2) - c2(s - 3 * m + 2)


def test_grid_levels_closed_form_3d_c3():
    m = 64
    a, _ = g.heat_system_3d(m, 1e-3, k_seed=0, u0_seed=1)
    pat = O.Pattern(a)
    fwd, bwd = _grid_levels_closed_form(m, 3)
    assert pat.nlev_f == 3 * (m - 1) + 1 == 190
    assert np.array_equal(pat.flevel, fwd)
    assert np.array_equal(pat.blevel, bwd)
    sizes = np.diff(pat.flev_ptr)
    assert all(sizes[s] == _level_size_3d(s, m) for s in range(190))
    assert sizes.max() == 3072
    assert pat.nnz_l == 1036288


def _brute_levels(n, lower_adj):
    @functools.lru_cache(maxsize=None)
    def depth(i):
        # longest path ending at i, by exhaustive recursion over predecessors
        preds = lower_adj[i]
        return 0 if not preds else 1 + max(depth(j) for j in preds)
    return np.array([depth(i) for i in range(n)])


def _brute_levels_paths(n, lower_adj):
    """Longest path by enumerating every path (only for tiny n)."""
    best = [0] * n

    def walk(i, length):
        best[i] = max(best[i], length)
        for k in range(i + 1, n):
            if i in lower_adj[k]:
                walk(k, length + 1)
    for i in range(n):
        if not lower_adj[i]:
            walk(i, 0)
    return np.array(best)


def test_levels_brute_force_random_dags():
    for seed in range(12):
        n = 10 + seed % 5
        A = g.random_lower_dag(n, 0.3, seed)
        pat = O.Pattern(A)
        d = A.to_dense() != 0
        lower_adj = tuple(tuple(j for j in range(i) if d[i, j]) for i in range(n))
        upper_adj = tuple(tuple(n - 1 - j for j in range(n) if j > i and d[i, j]) for i in range(n))
        assert np.array_equal(pat.flevel, _brute_levels_paths(n, lower_adj))
        assert np.array_equal(pat.flevel, _brute_levels(n, lower_adj))
        # backward DAG = forward DAG of the reversed numbering
        rev_lower = tuple(upper_adj[n - 1 - i] for i in range(n))
        assert np.array_equal(pat.blevel[::-1], _brute_levels_paths(n, rev_lower))


def test_level_sets_partition_and_order():
    A = g.random_spd(200, 0.03, seed=9)
    pat = O.Pattern(A)
    for lev, ptr, rows, nlev in ((pat.flevel, pat.flev_ptr, pat.flev_rows, pat.nlev_f),
                                 (pat.blevel, pat.blev_ptr, pat.blev_rows, pat.nlev_b)):
        assert np.array_equal(np.sort(rows), np.arange(A.n))
        for s in range(nlev):
            seg = rows[ptr[s]:ptr[s + 1]]
            assert len(seg) > 0
            assert np.all(lev[seg] == s)
            assert np.all(np.diff(seg) > 0)
