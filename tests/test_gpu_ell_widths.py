"""The ELL kernels for every slot count 1..8 (each a template instance):
Dirichlet Laplacians on product grids of shape (2, 2, ..., m), whose nodes
have one neighbour per size-2 axis and up to two along the long axis, give
rows of every width; all are bipartite, so their red-black orders take the
two-level pair with (width - 1) slots per half.

Bars: the ELL SpMV within the per-row FP32 bound 2 k u32 (|A||x|)_i of the
FP64 oracle; Jacobi-PCG and red-black IC(0)-PCG reach the FP64 tolerance
with the oracle's iteration count within max(2, 10%)."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import pdegen as g
from paper_2305_16432_amd import lpcg
from tests.gpu_util import U32, cuda_f32, cuda_f64, gpu_system, host

pytestmark = pytest.mark.gpu


def _laplacian(shape):
    """sum_d I x .. x T_d x .. x I with T = tridiag(-1, 2, -1) (diagonal 1 for
    a single point), plus the identity: SPD, rows of 1 + 2 (axes) entries."""
    mats = [sp.diags([-np.ones(k - 1), 2 * np.ones(k), -np.ones(k - 1)], [-1, 0, 1]) if k > 1
            else sp.identity(1) for k in shape]
    n = int(np.prod(shape))
    A = sp.identity(n, format="csr")
    for d, Td in enumerate(mats):
        left = sp.identity(int(np.prod(shape[:d])))
        right = sp.identity(int(np.prod(shape[d + 1:])))
        A = A + sp.kron(sp.kron(left, Td), right)
    return g.canonical_csr(A.tocsr())


# A's widths 1..8 (one shape each) for the product; the pair's slot counts
# 1..8 (width minus one) for the red-black application, the last with rows of
# 9 entries, so that its product takes a CSR form beside the ELL pair
SHAPES = [(1,), (2,), (64,), (2, 256), (2, 2, 128), (2, 2, 2, 64), (2, 2, 2, 2, 32), (2, 2, 2, 2, 2, 16)]
PAIR_SHAPES = [(2,), (64,), (2, 256), (2, 2, 128), (2, 2, 2, 64), (2, 2, 2, 2, 32), (2, 2, 2, 2, 2, 16),
               (2, 2, 2, 2, 2, 2, 8)]


def _width(A):
    return int(np.diff(A.rowptr).max())


def test_shapes_cover_every_width():
    assert [_width(_laplacian(s)) for s in SHAPES] == [1, 2, 3, 4, 5, 6, 7, 8]
    assert [_width(_laplacian(s)) - 1 for s in PAIR_SHAPES] == [1, 2, 3, 4, 5, 6, 7, 8]


@pytest.mark.parametrize("shape", SHAPES)
def test_ell_spmv_every_width(shape):
    A = _laplacian(shape)
    w = _width(A)
    print(f"[ell widths] shape {shape} n={A.n} width {w}", flush=True)
    assert w <= 8
    S = gpu_system(A)
    lpcg.set_trsv_cfg(S, 2, 1)
    assert lpcg.get_trsv_cfg(S, 2)["mode"] == 1
    x = np.random.default_rng(w).standard_normal(A.n).astype(np.float32)
    y = host(lpcg.spmv(S, cuda_f32(x)))
    ref = O.spmv(A, x.astype(np.float64))
    bound = O.spmv(g.CSR(A.n, A.rowptr, A.colind, np.abs(A.val)), np.abs(x.astype(np.float64)))
    k = np.diff(A.rowptr)
    assert np.all(np.abs(y - ref) <= 2 * k * U32 * bound + 1e-30)
    b = np.random.default_rng(w + 100).standard_normal(A.n)
    xs, res = lpcg.pcg_solve(S, lpcg.PC_JACOBI, cuda_f64(b), tol=1e-6, max_restarts=2)
    ref = O.pcg(A, b, O.PC_JACOBI, tol=1e-6)
    assert res["status"] == 0 and O.true_relres(A, b, host(xs)) <= 1e-6
    assert abs(res["iters"] - ref["iters"]) <= max(2, int(0.1 * ref["iters"])), (res["iters"], ref["iters"])


@pytest.mark.parametrize("shape", PAIR_SHAPES)
def test_ell_pair_every_width(shape):
    """Red-black IC(0)-PCG through the pair's ELL form (slots per half = the
    width minus the diagonal) with the update in the pair, against the oracle
    on the same ordering."""
    A = _laplacian(shape)
    w = _width(A)
    print(f"[ell pair] shape {shape} n={A.n} width {w}", flush=True)
    S = gpu_system(A, None, lpcg.ORDER_COLOR)
    assert S.info["nlev_fwd"] == 2 and S.info["ncolors"] == 2
    l, ut, _ = lpcg.ic0(S)
    b = np.random.default_rng(w + 200).standard_normal(A.n)
    xs, res = lpcg.pcg_solve(S, lpcg.PC_LLT, cuda_f64(b), l_val=l, ut_val=ut, tol=1e-6, max_restarts=2)
    perm, _, _ = O.color_order(A)
    Ap = O.permute_sym(A, perm)
    pat = O.Pattern(Ap)
    lref, _ = O.ic0(pat, Ap)
    ref = O.pcg(Ap, b[perm], O.PC_LLT, pat, lref, tol=1e-6)
    assert res["status"] == 0 and O.true_relres(A, b, host(xs)) <= 1e-6
    assert abs(res["iters"] - ref["iters"]) <= max(2, int(0.1 * ref["iters"])), (res["iters"], ref["iters"])
