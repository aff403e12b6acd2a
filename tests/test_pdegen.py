"""Checks of the seeded input generators (closed forms and structure)."""
import numpy as np

import pdegen as g


def test_heat_step_constant_k_eigenpairs():
    """k = 1: A = I + dt/h^2 K with K the 7-point Laplacian stencil, so
    A u = (1 + dt/h^2 * sum_a (2 - 2 cos(p_a pi h))) u for u = prod sin(p_a pi x_a h)."""
    m, dt = 6, 1e-2
    A = g.heat_step_3d(m, dt, np.ones((m, m, m)))
    h = 1.0 / (m + 1)
    coords = np.indices((m, m, m)).reshape(3, -1)[::-1] + 1
    D = A.to_dense()
    for ks in ((1, 1, 1), (2, 5, 3), (6, 1, 4)):
        u = np.prod([np.sin(ks[a] * np.pi * coords[a] * h) for a in range(3)], axis=0)
        lam = 1 + dt / h ** 2 * sum(2 - 2 * np.cos(k * np.pi * h) for k in ks)
        np.testing.assert_allclose(D @ u, lam * u, atol=1e-12 * lam)


def test_systems_symmetric_positive_diagonal_spd():
    for A in (g.poisson_grid(7, 2), g.heat_system_3d(5, 1e-3, 0, 1)[0],
              g.fem_p1_delaunay(12, 0, 1)[0], g.random_spd(40, 0.1, 0)):
        D = A.to_dense()
        assert np.array_equal(D, D.T)
        assert np.all(np.diag(D) > 0)
        np.linalg.cholesky(D)
        rows = A.row_of_entry()
        for i in range(A.n):
            seg = A.colind[A.rowptr[i]:A.rowptr[i + 1]]
            assert np.all(np.diff(seg) > 0) and i in seg
        del rows


def test_fem_constant_k_reproduces_linear_functions():
    """With k = 1 (sigma = 0) the P1 stiffness annihilates linear fields on
    interior rows: A u_interior = -K_(interior, boundary) u_boundary, checked
    through the row sums of the assembled interior block for u = 1 being
    nonnegative (diagonal dominance of the Laplacian stiffness)."""
    A, b, info = g.fem_p1_delaunay(10, 0, 1, sigma=0.0)
    D = A.to_dense()
    assert np.all(D.sum(axis=1) >= -1e-12)


def test_grf_variance_and_correlation():
    m, h, ell = 48, 1.0 / 49, 0.1
    vals = np.stack([g.grf((m, m), h, 1.0, ell, seed=s) for s in range(20)])
    assert abs(vals.var() - 1.0) < 0.15
    lag = int(round(ell / h))
    c = np.mean(vals[:, :-lag, :] * vals[:, lag:, :])
    assert abs(c - np.exp(-0.5 * (lag * h / ell) ** 2)) < 0.15
