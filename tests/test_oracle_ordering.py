"""Pins of the oracle's multicolour ordering (greedy first-fit colouring in
row order, rows sorted by (system, colour)) and of its symmetric permutation,
against closed forms, graph invariants and dense linear algebra."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import pdegen as g


def _grid_parity(shape):
    idx = np.indices(shape[::-1]).reshape(len(shape), -1)  # natural order: first axis fastest
    return idx.sum(axis=0) % 2


@pytest.mark.parametrize("make,shape", [
    (lambda: g.tridiag_1d(37), (37,)),
    (lambda: g.poisson_grid(9, 2), (9, 9)),
    (lambda: g.heat_system_3d(6, 1e-3, 1, 2)[0], (6, 6, 6)),
    (lambda: g.poisson_grid(5, 3), (5, 5, 5)),
])
def test_grid_greedy_colouring_is_red_black(make, shape):
    """A grid graph in natural order is bipartite by the parity of i+j(+k);
    first-fit in row order gives colour = parity (induction over rows: every
    earlier neighbour has the opposite parity)."""
    A = make()
    perm, color, nc = O.color_order(A)
    assert nc == 2
    np.testing.assert_array_equal(color, _grid_parity(shape))
    # stable: the even rows first, ascending, then the odd rows
    ev = np.flatnonzero(color == 0)
    od = np.flatnonzero(color == 1)
    np.testing.assert_array_equal(perm, np.concatenate([ev, od]))


def test_complete_graph_needs_n_colours():
    n = 9
    A = g.csr_from_dense(np.eye(n) * n + np.ones((n, n)))
    perm, color, nc = O.color_order(A)
    assert nc == n
    np.testing.assert_array_equal(color, np.arange(n))
    np.testing.assert_array_equal(perm, np.arange(n))


@pytest.mark.parametrize("center_last", [False, True])
def test_star_graph(center_last):
    n = 7
    c = n - 1 if center_last else 0
    D = np.eye(n) * 4.0
    for j in range(n):
        if j != c:
            D[c, j] = D[j, c] = -1.0
    _, color, nc = O.color_order(g.csr_from_dense(D))
    assert nc == 2
    exp = np.zeros(n, int) if center_last else np.ones(n, int)
    exp[c] = 1 if center_last else 0
    np.testing.assert_array_equal(color, exp)


@pytest.mark.parametrize("name", ["fem", "random", "heat"])
def test_colouring_is_proper_and_bounded(name):
    if name == "fem":
        A = g.fem_p1_delaunay(30, 0, 1)[0]
    elif name == "random":
        A = g.random_spd(300, 0.03, seed=4)
    else:
        A = g.heat_system_3d(7, 1e-3, 3, 4)[0]
    perm, color, nc = O.color_order(A)
    erow = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    off = erow != A.colind
    assert np.all(color[erow[off]] != color[A.colind[off]])
    lower_deg = np.bincount(erow[off & (A.colind < erow)], minlength=A.n)
    assert nc <= lower_deg.max() + 1
    assert np.all(color <= lower_deg)  # first-fit never exceeds the number of earlier neighbours
    assert sorted(perm.tolist()) == list(range(A.n))
    # permuted lower triangle: a row depends only on rows of smaller colour
    Ap = O.permute_sym(A, perm)
    pat = O.Pattern(Ap)
    assert len(pat.flev_ptr) - 1 <= nc


def test_permute_sym_matches_dense_and_preserves_solution():
    A = g.fem_p1_delaunay(12, 2, 3)[0]
    perm, _, _ = O.color_order(A)
    Ap = O.permute_sym(A, perm)
    D = A.to_dense()
    np.testing.assert_array_equal(Ap.to_dense(), D[np.ix_(perm, perm)])
    assert np.all(np.diff(Ap.colind)[np.diff(Ap.row_of_entry()) == 0] > 0)  # ascending columns
    rng = np.random.default_rng(0)
    b = rng.standard_normal(A.n)
    x = np.linalg.solve(D, b)
    xp = np.linalg.solve(Ap.to_dense(), b[perm])
    np.testing.assert_allclose(xp, x[perm], rtol=1e-10, atol=1e-12)


def test_permute_keeps_explicit_zeros():
    perm = np.array([2, 0, 1])
    # explicit zeros at (0,1) and (1,0) are structural entries
    M = sp.coo_matrix((np.array([2.0, 0.0, 1.0, 0.0, 3.0, 1.0, 4.0]),
                       (np.array([0, 0, 0, 1, 1, 2, 2]), np.array([0, 1, 2, 0, 1, 0, 2]))), shape=(3, 3))
    B = g.canonical_csr(M)
    assert B.nnz == 7
    Bp = O.permute_sym(B, perm)
    assert Bp.nnz == 7
    np.testing.assert_array_equal(Bp.to_dense(), B.to_dense()[np.ix_(perm, perm)])


def test_batch_order_keeps_systems_contiguous():
    mats = [g.poisson_grid(5, 2), g.heat_system_3d(4, 1e-3, 1, 2)[0], g.fem_p1_delaunay(9, 0, 1)[0]]
    B, srp = g.block_diag_csr(mats)
    perm, color, _ = O.color_order(B, srp)
    row_sys = np.repeat(np.arange(len(mats)), np.diff(srp))
    assert np.all(np.diff(row_sys[perm]) >= 0)
    for s, m in enumerate(mats):
        sub = perm[srp[s]:srp[s + 1]] - srp[s]
        ps, cs, _ = O.color_order(m)
        np.testing.assert_array_equal(sub, ps)  # block-diagonal: colouring is per block
        np.testing.assert_array_equal(color[srp[s]:srp[s + 1]], cs)


def test_ic0_pcg_on_red_black_order():
    """PCG with IC(0) on the red-black ordered 3D heat system converges to the
    same solution as on the natural order (the permutation changes the
    preconditioner, not the system)."""
    A, b = g.heat_system_3d(10, 1e-3, 5, 6)
    perm, _, nc = O.color_order(A)
    Ap = O.permute_sym(A, perm)
    pat = O.Pattern(Ap)
    l, st = O.ic0(pat, Ap)
    r = O.pcg(Ap, b[perm], O.PC_LLT, pat, l, tol=1e-10)
    assert r["status"] == O.OK
    x = np.empty(A.n)
    x[perm] = r["x"]
    assert O.true_relres(A, b, x) <= 1e-9
    # red-black IC(0): the first colour's rows of L are diagonal only
    n0 = int((O.color_order(A)[1] == 0).sum())
    assert np.all(np.diff(pat.lrowptr)[:n0] == 1)
