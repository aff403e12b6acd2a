"""The oracle's training triples: x solves A x = b to the stated 1e-12
(checked against a sparse direct solve, not the oracle), the file holds
every system bit for bit as pdegen made it, and the training script's
reader returns the same arrays as the oracle-side reader."""
import numpy as np
import scipy.sparse.linalg as spla

import pdegen as g
from oracle import triples as T


def _rows(family, size, seeds):
    return [T._one((family, size, s)) for s in seeds]


def test_triples_solutions_and_roundtrip(tmp_path):
    for family, size, maker in (("fem2d", 14, lambda s: g.fem_p1_delaunay(14, s, 20000 + s)[:2]),
                                ("heat3d", 6, lambda s: g.heat_system_3d(6, 1e-3, s, 10000 + s))):
        rows = _rows(family, size, [0, 1, 2])
        path = str(tmp_path / f"{family}.npz")
        rel = T.write(path, family, size, rows)
        assert np.all(rel <= 1e-12)
        back = T.load(path)
        from paper_2305_16432_amd.train import load_triples, shared_pattern
        tr, fam, sz = load_triples(path)
        assert fam == family and sz == size
        assert shared_pattern(tr) == (family == "heat3d")
        for s, ((A, b, x), (rp, ci, v, bt, xt)) in enumerate(zip(back, tr)):
            A0, b0 = maker(s)
            assert np.array_equal(A.rowptr, A0.rowptr) and np.array_equal(A.colind, A0.colind)
            assert np.array_equal(A.val, A0.val) and np.array_equal(b, b0)
            assert np.array_equal(rp, A.rowptr) and np.array_equal(ci, A.colind)
            assert np.array_equal(v, A.val) and np.array_equal(bt, b) and np.array_equal(xt, x)
            xd = spla.spsolve(A0.to_scipy().tocsc(), b0)
            # x within the residual bound times a condition estimate of the
            # small system
            kappa = np.linalg.cond(A0.to_dense())
            assert np.linalg.norm(x - xd) <= 10 * kappa * 1e-12 * np.linalg.norm(xd)


def test_triples_restart_reaches_tolerance():
    # an ill-conditioned FEM system (sigma 2 coefficients): the true residual
    # still meets 1e-12 after the FP64 restarts
    A, b, _ = g.fem_p1_delaunay(24, 3, 4, sigma=2.0)
    x, its, rel, kind = T.solve_oracle(A, b)
    r = b - A.to_scipy() @ x
    assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(b) * 1.0001
    assert rel <= 1e-12 and its > 0 and kind in ("ic0", "jacobi")
