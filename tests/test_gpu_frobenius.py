"""GPU parity of the Frobenius loss (equation loss_A, the ablation of the
loss-function section) against the oracle: per system loss to 1e-10 relative
(FP64 on the same FP32 factor values) and the FP32 gradient to 1e-6."""
import numpy as np
import pytest
import torch

import oracle as O
import pdegen as g
from oracle import gnn as ognn
from paper_2305_16432_amd import lpcg
from tests.gpu_util import cuda_f32, gpu_system, host

pytestmark = pytest.mark.gpu


def _rand_lower(pat, seed):
    rng = np.random.default_rng(seed)
    lv = rng.uniform(-0.5, 0.5, pat.nnz_l)
    row = np.repeat(np.arange(len(pat.lrowptr) - 1), np.diff(pat.lrowptr))
    d = pat.lcol == row
    lv[d] = rng.uniform(1.0, 3.0, d.sum())
    return lv.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("ordering", [0, 1])
def test_frobenius_loss_batch_parity(ordering):
    mats = [g.poisson_grid(8, 2), g.heat_system_3d(6, 1e-3, 1, 2)[0], g.fem_p1_delaunay(12, 0, 1)[0],
            g.random_spd(120, 0.05, 2)]
    B, srp = g.block_diag_csr(mats)
    if ordering:
        perm, _, _ = O.color_order(B, srp)
        Bi = O.permute_sym(B, perm)
    else:
        Bi = B
    pat = O.Pattern(Bi)
    lv = _rand_lower(pat, 3)
    S = gpu_system(B, srp, ordering)
    loss, dl = lpcg.frob_loss(S, cuda_f32(lv))
    loss, dl = host(loss), host(dl).astype(np.float64)
    ref_g = np.zeros(pat.nnz_l)
    for s in range(len(mats)):
        r0, r1 = srp[s], srp[s + 1]
        sub = g.canonical_csr(Bi.to_scipy()[r0:r1, r0:r1])
        sp = O.Pattern(sub)
        ls, gs = ognn.frobenius_loss(sub, lv[pat.lrowptr[r0]:pat.lrowptr[r1]], sp.lrowptr, sp.lcol)
        assert abs(loss[s] - ls) <= 1e-10 * ls, (s, loss[s], ls)
        ref_g[pat.lrowptr[r0]:pat.lrowptr[r1]] = gs
    np.testing.assert_allclose(dl, ref_g, rtol=1e-6, atol=1e-6 * np.abs(ref_g).max())


def test_frobenius_loss_zero_for_exact_factor_and_c3():
    A = g.tridiag_1d(500)  # IC(0) = exact Cholesky
    S = gpu_system(A)
    l, _, _ = lpcg.ic0(S)
    loss, dl = lpcg.frob_loss(S, l)
    assert float(host(loss)[0]) <= 1e-9 and float(torch.abs(dl).max()) <= 1e-5
    # full size: 64^3 heat step with its IC(0) factor, against the oracle
    A, _ = g.heat_system_3d(64, 1e-3, 1000, 2000)
    pat = O.Pattern(A)
    S = gpu_system(A)
    l, _, _ = lpcg.ic0(S)
    loss, dl = lpcg.frob_loss(S, l)
    ls, gs = ognn.frobenius_loss(A, host(l).astype(np.float64), pat.lrowptr, pat.lcol)
    assert abs(float(host(loss)[0]) - ls) <= 1e-10 * ls
    np.testing.assert_allclose(host(dl), gs, rtol=1e-5, atol=1e-6 * np.abs(gs).max())
