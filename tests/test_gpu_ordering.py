"""GPU parity of the multicolour ordering: the permutation and the whole
derived structure bit-exact against the oracle's (its colouring, then its
analysis of P A P^T), and every numeric entry point of a reordered system
against the oracle run on P A P^T, with vectors in the caller's numbering.

Tolerances are those of the natural-order tests: SpMV per row
2 nnz_i u32 (|A||x|)_i, substitution backward error 4 k u32, IC(0) 1.0001 u32
relative, PCG iterations within max(2, 10%) of the oracle's, GNN split bars (tests/parity_bars.py)
relative Frobenius, loss 1e-10 relative."""
import numpy as np
import pytest
import torch

import oracle as O
import pdegen as g
from oracle import gnn as ognn
from paper_2305_16432_amd import lpcg
from tests import parity_bars as PB
from tests.gpu_util import U32, cuda_f32, cuda_f64, gpu_system, host, matrices_small
from tests.test_gpu_pattern_spmv_trsv import PATTERN_KEYS

pytestmark = pytest.mark.gpu

COLOR = lpcg.ORDER_COLOR


def _ref(A, srp=None):
    perm, color, nc = O.color_order(A, srp)
    Ap = O.permute_sym(A, perm)
    return perm, nc, Ap, O.Pattern(Ap)


def _check_structure(A, srp=None):
    perm, nc, Ap, pat = _ref(A, srp)
    S = gpu_system(A, srp, COLOR)
    assert S.info["ordering"] == COLOR and S.info["ncolors"] == nc
    assert np.array_equal(host(lpcg.export_perm(S)), perm)
    assert S.info["nlev_fwd"] == pat.nlev_f and S.info["nlev_bwd"] == pat.nlev_b
    assert S.info["nlev_fwd"] <= nc
    got = lpcg.export_pattern(S)
    torch.cuda.synchronize()
    for gk, rk in PATTERN_KEYS:
        if gk == "lsrc":  # positions in the internal CSR, which is Ap's
            continue
        assert np.array_equal(host(got[gk]), getattr(pat, rk)), gk
    assert np.array_equal(host(got["lsrc"]), pat.lsrc)
    return S, perm, Ap, pat


@pytest.mark.parametrize("name", list(matrices_small()))
def test_color_structure_bitexact_small(name):
    print(f"[order] {name}", flush=True)
    _check_structure(matrices_small()[name])


def test_color_structure_c3_full_size_is_red_black():
    print("[order] heat3d_64", flush=True)
    A, _ = g.heat_system_3d(64, 1e-3, 1000, 2000)
    S, perm, _, _ = _check_structure(A)
    assert S.info["ncolors"] == 2 and S.info["nlev_fwd"] == 2 and S.info["nlev_bwd"] == 2


def test_color_structure_batch():
    mats = [g.poisson_grid(7, 2), g.heat_system_3d(5, 1e-3, 1, 2)[0], g.fem_p1_delaunay(11, 0, 1)[0]]
    B, srp = g.block_diag_csr(mats)
    _check_structure(B, srp)


def test_color_rejects_unknown_ordering():
    A = g.poisson_grid(4, 2)
    with pytest.raises(lpcg.LpcgError) as e:
        gpu_system(A, None, 7)
    assert e.value.code == lpcg.EINVAL


@pytest.mark.parametrize("name", ["fem_40", "heat3d_13", "random_777"])
def test_color_spmv_trsv_ic0_in_caller_numbering(name):
    A = matrices_small()[name]
    perm, _, Ap, pat = _ref(A)
    S = gpu_system(A, None, COLOR)
    rng = np.random.default_rng(0)
    # SpMV, original numbering
    x = rng.standard_normal(A.n).astype(np.float32).astype(np.float64)
    y = host(lpcg.spmv(S, cuda_f32(x))).astype(np.float64)
    ref = O.spmv(A, x)
    absAx = O.spmv(g.CSR(A.n, A.rowptr, A.colind, np.abs(A.val)), np.abs(x))
    nnz_row = np.diff(A.rowptr)
    assert np.all(np.abs(y - ref) <= 2 * nnz_row * U32 * absAx + 1e-300)
    y64 = host(lpcg.spmv(S, cuda_f64(x)))
    np.testing.assert_allclose(y64, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    # IC(0) of P A P^T
    l, ut, _ = lpcg.ic0(S)
    lref, st = O.ic0(pat, Ap)
    assert st == 0
    lg = host(l).astype(np.float64)
    assert np.all(np.abs(lg - lref) <= 1.0001 * U32 * np.abs(lref))
    # forward solve with the GPU factor, rhs and result in the original numbering
    r = rng.standard_normal(A.n).astype(np.float32)
    yf = host(lpcg.sptrsv(S, False, l, ut, cuda_f32(r))).astype(np.float64)
    yi = yf[perm]  # internal order
    res = O.spmv(g.CSR(A.n, pat.lrowptr, pat.lcol, lg), yi) - r[perm]
    absL = O.spmv(g.CSR(A.n, pat.lrowptr, pat.lcol, np.abs(lg)), np.abs(yi))
    k = np.diff(pat.lrowptr)
    assert np.all(np.abs(res) <= 4 * k * U32 * absL + 1e-30)


@pytest.mark.parametrize("kind", ["ic0", "jacobi"])
@pytest.mark.parametrize("name", ["fem_40", "heat3d_13", "poisson2d_32"])
def test_color_pcg_matches_oracle(name, kind):
    A = matrices_small()[name]
    b = np.random.default_rng(3).standard_normal(A.n)
    perm, _, Ap, pat = _ref(A)
    S = gpu_system(A, None, COLOR)
    bd = cuda_f64(b)
    if kind == "ic0":
        l, ut, _ = lpcg.ic0(S)
        x, res = lpcg.pcg_solve(S, lpcg.PC_LLT, bd, l_val=l, ut_val=ut, tol=1e-6, max_restarts=2)
        lref, _ = O.ic0(pat, Ap)
        ro = O.pcg(Ap, b[perm], O.PC_LLT, pat, lref, tol=1e-6)
    else:
        x, res = lpcg.pcg_solve(S, lpcg.PC_JACOBI, bd, tol=1e-6, max_restarts=2)
        ro = O.pcg(Ap, b[perm], O.PC_JACOBI, pat, None, tol=1e-6)
    assert res["status"] == 0 and res["relres_true"] <= 1e-6
    xh = host(x)
    assert O.true_relres(A, b, xh) <= 1e-6  # original system, original numbering
    assert abs(res["iters"] - ro["iters"]) <= max(2, 0.1 * ro["iters"]), (res["iters"], ro["iters"])
    xo = np.empty(A.n)
    xo[perm] = ro["x"]
    assert np.linalg.norm(xh - xo) / np.linalg.norm(xo) <= 1e-3


def test_color_pcg_c3_full_size():
    print("[order] pcg heat3d_64 red-black", flush=True)
    A, b = g.heat_system_3d(64, 1e-3, 1000, 2000)
    perm, _, Ap, pat = _ref(A)
    S = gpu_system(A, None, COLOR)
    l, ut, _ = lpcg.ic0(S)
    x, res = lpcg.pcg_solve(S, lpcg.PC_LLT, cuda_f64(b), l_val=l, ut_val=ut, tol=1e-6, max_restarts=2)
    lref, _ = O.ic0(pat, Ap)
    ro = O.pcg(Ap, b[perm], O.PC_LLT, pat, lref, tol=1e-6)
    print(f"iters gpu {res['iters']} oracle {ro['iters']}")
    assert res["status"] == 0 and O.true_relres(A, b, host(x)) <= 1e-6
    assert abs(res["iters"] - ro["iters"]) <= max(2, 0.1 * ro["iters"])


@pytest.mark.parametrize("diag_mode", [0, 1, 2])
def test_color_gnn_and_loss(diag_mode):
    A = matrices_small()["fem_40"]
    b = np.random.default_rng(5).standard_normal(A.n)
    perm, _, Ap, pat = _ref(A)
    S = gpu_system(A, None, COLOR)
    h, n_mp = 32, 3
    P = g.init_gnn_params(h, n_mp, seed=8)
    params = lpcg.pack_params(P, h, n_mp).cuda()
    ws = lpcg.gnn_workspace(S, h, n_mp)
    lv = torch.empty(pat.nnz_l, dtype=torch.float32, device="cuda")
    ut = torch.empty_like(lv)
    lpcg.gnn_predict_L(S, params, h, n_mp, cuda_f64(b), ws, lv, ut, diag_mode=diag_mode)
    ref, _ = ognn.forward(Ap, b[perm], P, h, n_mp, rev=pat.rev, diag_mode=diag_mode)
    lg = host(lv).astype(np.float64)
    PB.check_factor(pat, lg, ref, diag_mode)
    # data loss with x, b in the original numbering
    x = np.linalg.solve(A.to_dense(), b)
    loss, dl = lpcg.llt_loss(S, lv, cuda_f64(x), cuda_f64(b))
    ls, gs = ognn.training_loss(Ap, b[perm], x[perm], lg, pat.lrowptr, pat.lcol,
                                lambda lvv, xx, bb: O.llt_loss(pat, lvv, xx, bb))
    assert abs(float(host(loss)[0]) - ls) <= 1e-10 * abs(ls)
    gg = host(dl).astype(np.float64)
    np.testing.assert_allclose(gg, gs, rtol=1e-6, atol=1e-6 * np.abs(gs).max())


def test_color_update_values():
    A1, _ = g.heat_system_3d(9, 1e-3, 1, 2)
    A2, _ = g.heat_system_3d(9, 1e-3, 3, 4)  # same pattern, other k field
    perm, _, _, pat = _ref(A1)
    S = gpu_system(A1, None, COLOR)
    lpcg.update_values(S, cuda_f64(A2.val))
    l, _, _ = lpcg.ic0(S)
    lref, _ = O.ic0(pat, O.permute_sym(A2, perm))
    assert np.all(np.abs(host(l) - lref) <= 1.0001 * U32 * np.abs(lref))


@pytest.mark.parametrize("name", ["heat3d_13", "poisson2d_32", "bipartite_24"])
def test_two_level_pcg_matches_per_level_launches(name):
    """On a red-black system the PCG applies L L^T with the two-level pair:
    its ELL form (rows of at most 8 entries: the 7- and 5-point grids) or its
    CSR form (the bipartite 13-entry stencil); forcing the backward direction
    to the dependency-driven mode takes the per-level path.  Both reach the
    FP64 tolerance with the oracle's iteration count, and their iterates
    agree to FP32 rounding."""
    A = matrices_small()[name]
    b = np.random.default_rng(5).standard_normal(A.n)
    perm, _, Ap, pat = _ref(A)
    S = gpu_system(A, None, COLOR)
    assert S.info["nlev_fwd"] == 2 and S.info["ncolors"] == 2
    l, ut, _ = lpcg.ic0(S)
    bd = cuda_f64(b)
    x2, r2 = lpcg.pcg_solve(S, lpcg.PC_LLT, bd, l_val=l, ut_val=ut, tol=1e-6, max_restarts=2)
    lpcg.set_trsv_cfg(S, 1, 0)
    x1, r1 = lpcg.pcg_solve(S, lpcg.PC_LLT, bd, l_val=l, ut_val=ut, tol=1e-6, max_restarts=2)
    lref, _ = O.ic0(pat, Ap)
    ro = O.pcg(Ap, b[perm], O.PC_LLT, pat, lref, tol=1e-6)
    for res in (r1, r2):
        assert res["status"] == 0 and res["relres_true"] <= 1e-6
        assert abs(res["iters"] - ro["iters"]) <= max(2, 0.1 * ro["iters"]), (res["iters"], ro["iters"])
    assert abs(r1["iters"] - r2["iters"]) <= 2, (r1["iters"], r2["iters"])
    xa, xb = host(x1), host(x2)
    assert np.linalg.norm(xa - xb) / np.linalg.norm(xa) <= 1e-3
