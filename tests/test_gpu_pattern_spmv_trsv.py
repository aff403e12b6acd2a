"""GPU parity: pattern analysis (bit-exact), SpMV, triangular solves, IC(0),
Jacobi -- HIP library vs the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle as O
import pdegen as g
from paper_2305_16432_amd import lpcg
from tests.gpu_util import U32, U64, cuda_f32, cuda_f64, gpu_system, host, matrices_small

pytestmark = pytest.mark.gpu

PATTERN_KEYS = [("lrowptr", "lrowptr"), ("lcol", "lcol"), ("lsrc", "lsrc"), ("urowptr", "urowptr"),
                ("ucol", "ucol"), ("u2l", "usrc"), ("rev", "rev"), ("flevel", "flevel"),
                ("flev_ptr", "flev_ptr"), ("flev_rows", "flev_rows"), ("blevel", "blevel"),
                ("blev_ptr", "blev_ptr"), ("blev_rows", "blev_rows")]


def _check_pattern(A, sys_rowptr=None):
    ref = O.Pattern(A)
    S = gpu_system(A, sys_rowptr)
    assert S.info["nnz_l"] == ref.nnz_l
    assert S.info["nlev_fwd"] == ref.nlev_f and S.info["nlev_bwd"] == ref.nlev_b
    got = lpcg.export_pattern(S)
    torch.cuda.synchronize()
    for gk, rk in PATTERN_KEYS:
        assert np.array_equal(host(got[gk]), getattr(ref, rk)), gk
    return S, ref


@pytest.mark.parametrize("name", list(matrices_small()))
def test_pattern_bitexact_small(name):
    print(f"[pattern] {name}", flush=True)
    _check_pattern(matrices_small()[name])


def test_pattern_bitexact_c3_full_size():
    print("[pattern] heat3d_64", flush=True)
    A, _ = g.heat_system_3d(64, 1e-3, 1000, 2000)
    S, ref = _check_pattern(A)
    assert S.info["nlev_fwd"] == 190 and S.info["max_width_fwd"] == 3072


def test_pattern_block_diagonal_batch():
    mats = [g.poisson_grid(7, 2), g.heat_system_3d(5, 1e-3, 1, 2)[0], g.fem_p1_delaunay(11, 0, 1)[0]]
    B, srp = g.block_diag_csr(mats)
    _check_pattern(B, srp)


def test_pattern_rejects_bad_input():
    A = g.csr_from_dense(np.array([[2.0, 1.0], [0.0, 2.0]]))  # unsymmetric pattern
    with pytest.raises(lpcg.LpcgError) as e:
        gpu_system(A)
    assert e.value.code == lpcg.EINVAL
    rp = np.array([0, 1, 2], np.int32)
    ci = np.array([1, 0], np.int32)  # no diagonal
    with pytest.raises(lpcg.LpcgError):
        lpcg.analyze(rp, ci, np.ones(2))
    B, srp = g.block_diag_csr([g.poisson_grid(3, 2), g.poisson_grid(3, 2)])
    with pytest.raises(lpcg.LpcgError):  # system boundary through a row
        gpu_system(B, np.array([0, 5, 18]))


def _spmv_bound(A, x, u):
    absA = np.abs(A.to_scipy())
    k = np.diff(A.rowptr)
    return 2.0 * k * u * (absA @ np.abs(x)) + 1e-300


@pytest.mark.parametrize("name", ["tridiag_1000", "heat3d_13", "fem_40", "random_777", "one"])
def test_spmv_fp64_fp32(name):
    A = matrices_small()[name]
    S = gpu_system(A)
    x = np.random.default_rng(1).standard_normal(A.n)
    y64 = host(lpcg.spmv(S, cuda_f64(x)))
    ref = O.spmv(A, x)
    assert np.all(np.abs(y64 - ref) <= _spmv_bound(A, x, U64))
    x32 = x.astype(np.float32)
    y32 = host(lpcg.spmv(S, cuda_f32(x32))).astype(np.float64)
    A32 = g.CSR(A.n, A.rowptr, A.colind, A.val.astype(np.float32).astype(np.float64))
    ref32 = O.spmv(A32, x32.astype(np.float64))
    assert np.all(np.abs(y32 - ref32) <= _spmv_bound(A32, x32, U32))


def test_spmv_c3_full_size():
    A, b = g.heat_system_3d(64, 1e-3, 1000, 2000)
    S = gpu_system(A)
    y = host(lpcg.spmv(S, cuda_f64(b)))
    assert np.all(np.abs(y - O.spmv(A, b)) <= _spmv_bound(A, b, U64))


def _lower_values(A, pat, seed):
    rng = np.random.default_rng(seed)
    lval = rng.uniform(-0.3, 0.3, pat.nnz_l)
    row = np.repeat(np.arange(A.n), np.diff(pat.lrowptr))
    d = pat.lcol == row
    lval[d] = rng.uniform(1.0, 2.0, d.sum())
    return lval.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("name", ["tridiag_1000", "poisson2d_32", "heat3d_13", "fem_40", "random_777",
                                  "dag_60", "one"])
def test_sptrsv_forward_backward(name):
    """Componentwise backward error |rhs - T y| <= c k u32 |T| |y| (Higham's
    substitution bound, FP32 arithmetic; c = 4 covers FMA and the division)."""
    A = matrices_small()[name]
    print(f"[sptrsv] {name}", flush=True)
    pat = O.Pattern(A)
    S = gpu_system(A)
    lval = _lower_values(A, pat, 7)
    utv = lval[pat.usrc]
    rhs = np.random.default_rng(8).standard_normal(A.n).astype(np.float32).astype(np.float64)
    L = g.CSR(A.n, pat.lrowptr, pat.lcol, lval).to_scipy()
    k = np.diff(pat.lrowptr).max()
    y = host(lpcg.sptrsv(S, False, cuda_f32(lval), cuda_f32(utv), cuda_f32(rhs))).astype(np.float64)
    assert np.all(np.abs(rhs - L @ y) <= 4 * k * U32 * (abs(L) @ np.abs(y)) + 1e-30)
    yref = O.trsv_lower(pat, lval, rhs)
    np.testing.assert_allclose(y, yref, rtol=1e-3, atol=1e-5 * np.abs(yref).max())
    z = host(lpcg.sptrsv(S, True, cuda_f32(lval), cuda_f32(utv), cuda_f32(rhs))).astype(np.float64)
    assert np.all(np.abs(rhs - L.T @ z) <= 4 * k * U32 * (abs(L.T) @ np.abs(z)) + 1e-30)
    zref = O.trsv_upper(pat, lval, rhs)
    np.testing.assert_allclose(z, zref, rtol=1e-3, atol=1e-5 * np.abs(zref).max())


def test_sptrsv_c3_full_size_and_deterministic():
    A, b = g.heat_system_3d(64, 1e-3, 1000, 2000)
    pat = O.Pattern(A)
    S = gpu_system(A)
    l, ut, _ = lpcg.ic0(S)
    lval = host(l).astype(np.float64)
    rhs = b.astype(np.float32).astype(np.float64)
    y1 = lpcg.sptrsv(S, False, l, ut, cuda_f32(rhs))
    y2 = lpcg.sptrsv(S, False, l, ut, cuda_f32(rhs))
    assert torch.equal(y1, y2)
    y = host(y1).astype(np.float64)
    L = g.CSR(A.n, pat.lrowptr, pat.lcol, lval).to_scipy()
    assert np.all(np.abs(rhs - L @ y) <= 4 * 4 * U32 * (abs(L) @ np.abs(y)))
    z = host(lpcg.sptrsv(S, True, l, ut, cuda_f32(rhs))).astype(np.float64)
    assert np.all(np.abs(rhs - L.T @ z) <= 4 * 4 * U32 * (abs(L.T) @ np.abs(z)))


@pytest.mark.parametrize("name", ["tridiag_1000", "poisson2d_32", "heat3d_13", "fem_40", "random_777",
                                  "one"])
def test_ic0_matches_oracle(name):
    """GPU IC(0) runs in FP64 and rounds to FP32: |l - fl32(l_ref)| <= u32 |l_ref|
    up to FP64 reordering noise."""
    A = matrices_small()[name]
    pat = O.Pattern(A)
    ref, st = O.ic0(pat, A)
    assert st == 0
    S = gpu_system(A)
    l, ut, shift = lpcg.ic0(S)
    assert shift == 0.0
    lg = host(l).astype(np.float64)
    assert np.all(np.abs(lg - ref) <= 1.0001 * U32 * np.abs(ref) + 1e-300)
    assert np.array_equal(host(ut), host(l)[pat.usrc])


def test_ic0_c3_full_size():
    A, _ = g.heat_system_3d(64, 1e-3, 1000, 2000)
    pat = O.Pattern(A)
    ref, _ = O.ic0(pat, A)
    S = gpu_system(A)
    l, _, _ = lpcg.ic0(S)
    lg = host(l).astype(np.float64)
    assert np.all(np.abs(lg - ref) <= 1.0001 * U32 * np.abs(ref))


def test_ic0_breakdown_shift_retry():
    D = np.array([[1.0, 2.0, 0.0], [2.0, 1.0, 0.5], [0.0, 0.5, 3.0]])
    A = g.csr_from_dense(D)
    S = gpu_system(A)
    with pytest.raises(lpcg.LpcgError) as e:
        lpcg.ic0(S, 0.0, 0)
    assert e.value.code == lpcg.EBREAKDOWN
    l, _, shift = lpcg.ic0(S, 0.0, 20)
    assert shift > 0
    ref, st = O.ic0(O.Pattern(A), A, shift=shift)
    assert st == 0
    assert np.all(np.abs(host(l) - ref) <= 1.0001 * U32 * np.abs(ref))


def test_jacobi():
    A = matrices_small()["fem_40"]
    S = gpu_system(A)
    d = host(lpcg.jacobi(S))
    np.testing.assert_array_equal(d, (1.0 / O.diag(A)).astype(np.float32))
