"""GPU parity: the symmetric Gauss-Seidel factor (Experiments, baseline
methods, symmetric form) against the FP64 oracle.  The library forms
A_ij / sqrt(A_jj) in FP64 and rounds once to FP32, so every entry matches the
oracle's value rounded to FP32 within one FP32 ulp (2^-23 relative); U = L^T
carries the same values in U order."""
import numpy as np
import pytest
import torch

import oracle as O
import pdegen as g
from paper_2305_16432_amd import lpcg
from tests.gpu_util import gpu_system, host, matrices_small

pytestmark = pytest.mark.gpu


def _check(A, S):
    l, ut = lpcg.sgs(S)
    torch.cuda.synchronize()
    lg, ug = host(l).astype(np.float64), host(ut).astype(np.float64)
    pat = O.Pattern(A)
    ref = O.sgs_factor(pat, A).astype(np.float32).astype(np.float64)
    np.testing.assert_allclose(lg, ref, rtol=2.0 ** -23, atol=0)
    np.testing.assert_array_equal(ug, lg[pat.usrc])


@pytest.mark.parametrize("name", ["one", "tridiag_1000", "poisson2d_32", "heat3d_13", "fem_40", "random_777"])
def test_sgs_values(name):
    A = matrices_small()[name]
    _check(A, gpu_system(A))


def test_sgs_batch_and_new_values():
    mats = [g.poisson_grid(9, 2), g.heat_system_3d(5, 1e-3, 1, 2)[0]]
    B, srp = g.block_diag_csr(mats)
    S = gpu_system(B, srp)
    _check(B, S)
    # swap in new values on the same pattern (the factor follows them)
    B2 = g.CSR(B.n, B.rowptr, B.colind, np.asarray(B.val) * 3.0)
    lpcg.update_values(S, torch.as_tensor(np.asarray(B2.val)).cuda())
    _check(B2, S)


def test_sgs_colour_order_internal_numbering():
    """In colour order the factor lives on tril(P A P^T)."""
    A = matrices_small()["heat3d_13"]
    S = gpu_system(A, ordering=lpcg.ORDER_COLOR)
    perm = host(lpcg.export_perm(S))
    _check(O.permute_sym(A, perm), S)
