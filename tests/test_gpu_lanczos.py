"""GPU parity of the condition-number estimate: the PCG coefficients the
library records (FP32 vectors, FP64 scalars) give Lanczos extremes close to
the FP64 oracle's, and the library's Sturm-bisection eigenvalues of a given
coefficient sequence equal the oracle's tridiagonal eigenvalues.

Bars: for the same coefficients, eigenvalues to 1e-10 relative; GPU vs oracle
coefficients (different rounding in the recurrences), lambda_max to 1% and
kappa to 10% (the lambda_min Ritz value converges last)."""
import numpy as np
import pytest
import torch

import oracle as O
import pdegen as g
from paper_2305_16432_amd import lpcg
from tests.gpu_util import cuda_f64, gpu_system

pytestmark = pytest.mark.gpu


def test_lanczos_extremes_same_coefficients():
    A = g.fem_p1_delaunay(20, 1, 2)[0]
    pat = O.Pattern(A)
    l, _ = O.ic0(pat, A)
    r = O.pcg(A, np.random.default_rng(0).standard_normal(A.n), O.PC_LLT, pat, l, tol=1e-10)
    k = r["iters"]
    coef = np.zeros(2 * (k + 1))
    coef[2:2 * k + 2:2] = r["alpha"]
    coef[3:2 * k + 1:2] = r["beta"]
    lo, hi = lpcg.lanczos_extremes(coef, k)
    rlo, rhi = O.lanczos_extremes(r["alpha"], r["beta"])
    assert abs(lo - rlo) <= 1e-10 * rlo and abs(hi - rhi) <= 1e-10 * rhi


@pytest.mark.parametrize("kind", ["ic0", "jacobi"])
@pytest.mark.parametrize("m", [13, 64])
def test_kappa_estimate_vs_oracle(m, kind):
    A, b = g.heat_system_3d(m, 1e-3, 1000, 2000)
    pat = O.Pattern(A)
    S = gpu_system(A)
    maxit = 400
    coef = torch.zeros(2 * (maxit + 1), dtype=torch.float64, device="cuda")
    if kind == "ic0":
        l, ut, _ = lpcg.ic0(S)
        _, res = lpcg.pcg_solve(S, lpcg.PC_LLT, cuda_f64(b), l_val=l, ut_val=ut, tol=1e-6, maxit=maxit, coef=coef)
        lo_, _ = O.ic0(pat, A)
        r = O.pcg(A, b, O.PC_LLT, pat, lo_, tol=1e-6)
    else:
        _, res = lpcg.pcg_solve(S, lpcg.PC_JACOBI, cuda_f64(b), tol=1e-6, maxit=maxit, coef=coef)
        r = O.pcg(A, b, O.PC_JACOBI, tol=1e-6)
    k = min(res["iters"], r["iters"])
    lo, hi = lpcg.lanczos_extremes(coef, k)
    rlo, rhi = O.lanczos_extremes(r["alpha"][:k], r["beta"][:k - 1])
    print(f"[kappa] {m}^3 {kind}: gpu {hi / lo:.2f} ({lo:.4g}, {hi:.4g})  oracle {rhi / rlo:.2f}", flush=True)
    assert abs(hi - rhi) <= 0.01 * rhi
    assert abs(hi / lo - rhi / rlo) <= 0.1 * (rhi / rlo)
