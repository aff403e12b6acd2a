"""Sparse SPD systems from discretised second-order PDEs (inputs only).

* tridiag_1d      : 1D Dirichlet Laplacian stencil tridiag(-1, 2, -1), unscaled.
* poisson_grid    : 2D 5-point / 3D 7-point Dirichlet Laplacian on an m^d
                    interior grid, h = 1/(m+1), scaled by 1/h^2.
* heat_step_3d    : one implicit-Euler step of the variable-coefficient heat
                    equation on an m^3 interior grid:  A = I + dt/h^2 * K,
                    K the 7-point finite-volume operator of -div(k grad u) with
                    nodal k, harmonic-mean face coefficients and homogeneous
                    Dirichlet walls whose face coefficient is the nodal k.
* bipartite_grid  : a 2D grid stencil with odd-sum offsets only (bipartite,
                    rows of up to 13 entries), diagonally dominant.
* fem_p1_delaunay : P1 Galerkin stiffness of -div(k grad u) = f on a Delaunay
                    mesh of a jittered point grid in the unit square, k
                    constant per triangle, boundary nodes eliminated
                    (homogeneous Dirichlet), load = lumped mass * f.

Node numbering on grids is natural (x fastest, then y, then z).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .csr import CSR, canonical_csr
from .grf import grf


def tridiag_1d(n: int) -> CSR:
    main = np.full(n, 2.0)
    off = np.full(n - 1, -1.0)
    return canonical_csr(sp.diags([off, main, off], [-1, 0, 1], shape=(n, n)))


def _grid_index(shape):
    return np.arange(int(np.prod(shape))).reshape(shape[::-1]).transpose()


def poisson_grid(m: int, d: int) -> CSR:
    """Dirichlet Laplacian (2d on the diagonal, -1 to each grid neighbour) / h^2."""
    h = 1.0 / (m + 1)
    n = m ** d
    idx = _grid_index((m,) * d)
    rows, cols, vals = [np.arange(n)], [np.arange(n)], [np.full(n, 2.0 * d / h ** 2)]
    for ax in range(d):
        a = np.take(idx, np.arange(m - 1), axis=ax).ravel()
        b = np.take(idx, np.arange(1, m), axis=ax).ravel()
        for u, v in ((a, b), (b, a)):
            rows.append(u)
            cols.append(v)
            vals.append(np.full(u.shape[0], -1.0 / h ** 2))
    coo = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                        shape=(n, n))
    return canonical_csr(coo)


def bipartite_grid(m: int) -> CSR:
    """2D m x m grid whose stencil couples each node to the nodes at offsets
    (+-1, 0), (0, +-1), (+-1, +-2) and (+-2, +-1): every offset has an odd
    coordinate sum, so the graph is bipartite (a red-black colouring has two
    colours) while interior rows hold 13 entries.  Off-diagonal -1, diagonal
    1 + the row's neighbour count: a strictly diagonally dominant M-matrix."""
    offs = [(1, 0), (-1, 0), (0, 1), (0, -1), (1, 2), (1, -2), (-1, 2), (-1, -2), (2, 1), (2, -1), (-2, 1), (-2, -1)]
    idx = _grid_index((m, m))
    rows, cols = [], []
    deg = np.zeros(m * m)
    for di, dj in offs:
        a = idx[max(0, -di):m - max(0, di), max(0, -dj):m - max(0, dj)].ravel()
        b = idx[max(0, di):m - max(0, -di), max(0, dj):m - max(0, -dj)].ravel()
        rows.append(a)
        cols.append(b)
        np.add.at(deg, a, 1.0)
    r = np.concatenate(rows + [np.arange(m * m)])
    c = np.concatenate(cols + [np.arange(m * m)])
    v = np.concatenate([np.full(sum(len(x) for x in rows), -1.0), 1.0 + deg])
    return canonical_csr(sp.coo_matrix((v, (r, c)), shape=(m * m, m * m)))


def heat_step_3d(m: int, dt: float, k: np.ndarray) -> CSR:
    """A = I + dt/h^2 K for nodal coefficient field k of shape (m, m, m),
    indexed k[x, y, z]."""
    assert k.shape == (m, m, m)
    h = 1.0 / (m + 1)
    n = m ** 3
    idx = _grid_index((m, m, m))
    kf = k.ravel(order="F")  # natural order: x fastest
    diag = np.zeros(n)
    rows, cols, vals = [], [], []
    for ax in range(3):
        a = np.take(idx, np.arange(m - 1), axis=ax).ravel()
        b = np.take(idx, np.arange(1, m), axis=ax).ravel()
        face = 2.0 * kf[a] * kf[b] / (kf[a] + kf[b])
        np.add.at(diag, a, face)
        np.add.at(diag, b, face)
        rows += [a, b]
        cols += [b, a]
        vals += [-face, -face]
        # Dirichlet walls: the two boundary faces along this axis
        lo = np.take(idx, [0], axis=ax).ravel()
        hi = np.take(idx, [m - 1], axis=ax).ravel()
        np.add.at(diag, lo, kf[lo])
        np.add.at(diag, hi, kf[hi])
    c = dt / (h * h)
    rows.append(np.arange(n))
    cols.append(np.arange(n))
    vals.append(np.zeros(n))
    coo = sp.coo_matrix((c * np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                        shape=(n, n))
    a = canonical_csr(coo)
    # add identity + scaled diagonal on the (sorted) diagonal slots
    r = a.row_of_entry()
    dmask = a.colind == r
    a.val[dmask] += 1.0 + c * diag
    return a


def heat_system_3d(m: int, dt: float = 1e-3, k_seed: int = 0, u0_seed: int = 1,
                   sigma: float = 1.0, ell: float = 0.1, rhs: str = "grf"):
    """The 3D implicit heat step with k = exp(GRF(sigma, ell)) and b = u0, a
    smooth zero-mean GRF ("grf") or white noise N(0,1) ("white")."""
    h = 1.0 / (m + 1)
    k = np.exp(grf((m, m, m), h, sigma, ell, seed=k_seed))
    a = heat_step_3d(m, dt, k)
    if rhs == "grf":
        b = grf((m, m, m), h, 1.0, ell, seed=u0_seed).ravel(order="F")
    else:
        b = np.random.default_rng(u0_seed).standard_normal(m ** 3)
    return a, b


def fem_p1_delaunay(side: int = 128, k_seed: int = 0, f_seed: int = 1,
                    sigma: float = 1.0, ell: float = 0.1, jitter: float = 0.3):
    """P1 FEM system on a Delaunay triangulation of a side x side jittered grid.

    Returns (A, b, info) with A the stiffness restricted to interior nodes.
    """
    from scipy.spatial import Delaunay

    rng = np.random.default_rng(k_seed + 7919)
    hs = 1.0 / (side - 1)
    gx, gy = np.meshgrid(np.arange(side) * hs, np.arange(side) * hs, indexing="xy")
    pts = np.stack([gx.ravel(), gy.ravel()], axis=1)
    ii, jj = np.meshgrid(np.arange(side), np.arange(side), indexing="xy")
    ii, jj = ii.ravel(), jj.ravel()
    bnd = (ii == 0) | (jj == 0) | (ii == side - 1) | (jj == side - 1)
    inner = ~bnd
    pts[inner] += rng.uniform(-jitter, jitter, size=(inner.sum(), 2)) / side
    tri = Delaunay(pts).simplices
    p0, p1, p2 = pts[tri[:, 0]], pts[tri[:, 1]], pts[tri[:, 2]]
    det = (p1[:, 0] - p0[:, 0]) * (p2[:, 1] - p0[:, 1]) - (p2[:, 0] - p0[:, 0]) * (p1[:, 1] - p0[:, 1])
    area = 0.5 * np.abs(det)
    keep = area > 1e-14 * hs * hs
    tri, p0, p1, p2, det, area = tri[keep], p0[keep], p1[keep], p2[keep], det[keep], area[keep]
    # k per triangle: exp(GRF) sampled at the grid node nearest the centroid
    field = grf((side, side), hs, sigma, ell, seed=k_seed)
    cen = (p0 + p1 + p2) / 3.0
    ci = np.clip(np.rint(cen[:, 0] / hs).astype(int), 0, side - 1)
    cj = np.clip(np.rint(cen[:, 1] / hs).astype(int), 0, side - 1)
    kt = np.exp(field[ci, cj])
    # barycentric gradients: grad phi_a = rot(p_b - p_c) / (2 * signed area)
    P = [p0, p1, p2]
    grads = []
    for a in range(3):
        pb, pc = P[(a + 1) % 3], P[(a + 2) % 3]
        e = pc - pb
        grads.append(np.stack([-e[:, 1], e[:, 0]], axis=1) / det[:, None])
    rows, cols, vals = [], [], []
    for a in range(3):
        for b in range(3):
            rows.append(tri[:, a])
            cols.append(tri[:, b])
            vals.append(kt * area * np.sum(grads[a] * grads[b], axis=1))
    npt = pts.shape[0]
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(npt, npt)).tocsr()
    lump = np.zeros(npt)
    for a in range(3):
        np.add.at(lump, tri[:, a], area / 3.0)
    interior = np.nonzero(inner)[0]
    Ki = K[interior][:, interior]
    f = np.random.default_rng(f_seed).standard_normal(interior.shape[0])
    b = lump[interior] * f
    info = {"points": pts[interior], "n_triangles": int(tri.shape[0]), "k_tri": kt}
    return canonical_csr(Ki), b, info


def random_spd(n: int, density: float, seed: int, dominance: float = 1.0) -> CSR:
    """Random sparse symmetric matrix with a structurally symmetric pattern,
    made SPD by diagonal dominance: A_ii = dominance * sum_j |A_ij| + 1."""
    rng = np.random.default_rng(seed)
    m = sp.random(n, n, density=density, random_state=rng, data_rvs=lambda s: -rng.uniform(0.1, 1.0, s))
    m = sp.triu(m, 1)
    m = (m + m.T).tocsr()
    rs = np.asarray(abs(m).sum(axis=1)).ravel()
    m = m + sp.diags(dominance * rs + 1.0)
    return canonical_csr(m)


def random_lower_dag(n: int, p: float, seed: int) -> CSR:
    """Random structurally symmetric pattern (values: unit-diagonally dominant)
    whose strictly-lower part is a random DAG with edge probability p."""
    rng = np.random.default_rng(seed)
    lower = np.tril(rng.random((n, n)) < p, -1)
    pat = lower | lower.T
    d = np.where(pat, -rng.uniform(0.1, 1.0, (n, n)), 0.0)
    d = np.triu(d, 1)
    d = d + d.T
    d = d + np.diag(np.abs(d).sum(axis=1) + 1.0)
    return canonical_csr(sp.csr_matrix(np.where(pat | np.eye(n, dtype=bool), d, 0.0)))


def mixed_batch_member(seed: int, i: int, n: float):
    """System i of a mixed batch: P1 FEM on a jittered Delaunay grid (side ~
    sqrt(n) + 2, boundary eliminated) for even i, the 3D heat step on a cube
    of side ceil(n^(1/3)) for odd i; k fields and right-hand sides seeded per
    system (b = u0 GRF for the 3D systems, the lumped FEM load for the 2D
    ones).  Returns (A, b)."""
    if i % 2 == 0:
        side = max(4, int(round(np.sqrt(n))) + 2)
        A, b, _ = fem_p1_delaunay(side, k_seed=seed * 1000 + i, f_seed=seed * 1000 + i + 500)
    else:
        m = max(2, int(np.ceil(n ** (1.0 / 3.0))))
        A, b = heat_system_3d(m, 1e-3, k_seed=seed * 1000 + i, u0_seed=seed * 1000 + i + 500)
    return A, b


def mixed_batch_sizes(nsys: int, n_min: int, n_max: int, seed: int) -> np.ndarray:
    """Target sizes of a mixed batch: log-uniform in [n_min, n_max], seeded."""
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(np.log(n_min), np.log(n_max), nsys))


def mixed_batch(nsys: int, n_min: int, n_max: int, seed: int):
    """Uneven batch of independent systems (mixed_batch_member for each of the
    sizes of mixed_batch_sizes).  Returns a list of (A, b)."""
    sizes = mixed_batch_sizes(nsys, n_min, n_max, seed)
    return [mixed_batch_member(seed, i, n) for i, n in enumerate(sizes)]


def _member(args):
    from threadpoolctl import threadpool_limits
    seed, i, n = args
    with threadpool_limits(1):
        return mixed_batch_member(seed, i, n)


def mixed_batch_parallel(nsys: int, n_min: int, n_max: int, seed: int, workers: int = 8):
    """mixed_batch generated by `workers` processes started fresh ("spawn":
    they import neither torch nor any GPU library, so a caller that has
    initialised a GPU hands nothing of it to them).  Same systems, same order."""
    import multiprocessing as mp
    sizes = mixed_batch_sizes(nsys, n_min, n_max, seed)
    with mp.get_context("spawn").Pool(workers) as pool:
        return pool.map(_member, [(seed, i, float(n)) for i, n in enumerate(sizes)], chunksize=4)
