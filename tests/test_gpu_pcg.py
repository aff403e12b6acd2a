"""GPU parity: PCG (Appendix algorithm) with IC(0), symmetric Gauss-Seidel,
Jacobi and no preconditioner -- HIP library vs the FP64 oracle.

Several results are correct (any x with FP64 true relative residual <= tol),
so the comparisons are: the FP64 true residual (hard), x against the
oracle's x within kappa * tol, and the iteration count (FP32 apply: within
max(2, 10%) of the FP64 oracle)."""
import numpy as np
import pytest
import torch

import oracle as O
import pdegen as g
from paper_2305_16432_amd import lpcg
from tests.gpu_util import cuda_f64, gpu_system, host, matrices_small

pytestmark = pytest.mark.gpu


def _iters_close(got, ref, slack=0.1):
    """FP32 vectors vs the FP64 oracle: finite-precision CG loses
    orthogonality and converges later (Greenbaum), increasingly so with the
    condition number, so the band is relative; unpreconditioned solves of the
    kappa ~ 1e4 FEM systems get a wider one."""
    return abs(got - ref) <= max(2, int(slack * ref))


def _kappa_bound(A):
    """lambda_min >= min_i (A_ii - sum_{j!=i} |A_ij|) when positive (Gershgorin),
    lambda_max <= max_i sum_j |A_ij|; fallback to a dense estimate for small n."""
    D = None
    if A.n <= 2000:
        D = A.to_dense()
        ev = np.linalg.eigvalsh(D)
        return ev[-1] / ev[0]
    S = A.to_scipy()
    r = np.asarray(abs(S).sum(axis=1)).ravel()
    d = O.diag(A)
    lo = np.min(2 * d - r)
    assert lo > 0
    return r.max() / lo


def _run(A, kind, tol, b, use_graph=False, pat=None):
    S = gpu_system(A)
    l = ut = None
    pk = {"ic0": lpcg.PC_LLT, "sgs": lpcg.PC_LLT, "jacobi": lpcg.PC_JACOBI, "none": lpcg.PC_NONE}[kind]
    if kind == "ic0":
        l, ut, _ = lpcg.ic0(S)
    elif kind == "sgs":
        l, ut = lpcg.sgs(S)
    x, res, hist = lpcg.pcg_solve(S, pk, cuda_f64(b), l_val=l, ut_val=ut, tol=tol, hist=True,
                                  use_graph=use_graph, max_restarts=3)
    return S, host(x), res, host(hist), l


def _oracle(A, kind, tol, b):
    pat = O.Pattern(A)
    if kind == "ic0":
        lval, _ = O.ic0(pat, A)
        return O.pcg(A, b, O.PC_LLT, pat, lval, tol=tol)
    if kind == "sgs":
        return O.pcg(A, b, O.PC_LLT, pat, O.sgs_factor(pat, A), tol=tol)
    return O.pcg(A, b, O.PC_JACOBI if kind == "jacobi" else O.PC_NONE, tol=tol)


@pytest.mark.parametrize("kind", ["ic0", "sgs", "jacobi", "none"])
@pytest.mark.parametrize("name", ["poisson2d_32", "heat3d_13", "fem_40", "random_777"])
def test_pcg_small(name, kind):
    print(f"[pcg] {name} {kind}", flush=True)
    A = matrices_small()[name]
    b = np.random.default_rng(0).standard_normal(A.n)
    tol = 1e-6
    _, x, res, hist, _ = _run(A, kind, tol, b)
    ref = _oracle(A, kind, tol, b)
    assert res["status"] == lpcg.OK
    assert res["relres_true"] <= tol
    assert np.isclose(res["relres_true"], O.true_relres(A, b, x), rtol=1e-6)
    assert _iters_close(res["iters"], ref["iters"], 0.1 if kind != "none" else 0.25), \
        (res["iters"], ref["iters"])
    kap = _kappa_bound(A)
    assert np.linalg.norm(x - ref["x"]) / np.linalg.norm(ref["x"]) <= kap * tol
    # residual history tracks the oracle's to FP32-level agreement early on
    if res["restarts"] == 0:
        k = min(len(hist), len(ref["hist"]), 5)
        np.testing.assert_allclose(hist[:k], ref["hist"][:k], rtol=1e-3)


def test_pcg_c0_ic0_vs_dense_cholesky():
    """C0: 2D Poisson 32x32, IC(0), tol 1e-8, checked against a dense solve."""
    A = g.poisson_grid(32, 2)
    b = np.random.default_rng(0).standard_normal(A.n)
    _, x, res, _, _ = _run(A, "ic0", 1e-8, b)
    xs = np.linalg.solve(A.to_dense(), b)
    assert res["status"] == lpcg.OK and res["relres_true"] <= 1.5e-8
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= _kappa_bound(A) * 1.5e-8


@pytest.mark.parametrize("kind", ["ic0", "sgs", "jacobi"])
def test_pcg_c3_full_size(kind):
    """3D 64^3 heat step, tol 1e-6: FP64 true residual, iterations and sampled
    entries of x against the oracle."""
    print(f"[pcg] heat3d_64 {kind}", flush=True)
    A, b = g.heat_system_3d(64, 1e-3, 1000, 2000)
    tol = 1e-6
    _, x, res, _, _ = _run(A, kind, tol, b, use_graph=True)
    ref = _oracle(A, kind, tol, b)
    assert res["status"] == lpcg.OK and res["relres_true"] <= tol
    assert _iters_close(res["iters"], ref["iters"]), (res["iters"], ref["iters"])
    kap = _kappa_bound(A)
    idx = np.random.default_rng(3).choice(A.n, 2000, replace=False)
    err = np.abs(x[idx] - ref["x"][idx])
    assert np.linalg.norm(x - ref["x"]) / np.linalg.norm(ref["x"]) <= kap * tol
    assert err.max() <= kap * tol * np.abs(ref["x"]).max()


def test_pcg_graph_equals_eager_and_deterministic():
    A = matrices_small()["heat3d_13"]
    b = np.random.default_rng(1).standard_normal(A.n)
    S = gpu_system(A)
    l, ut, _ = lpcg.ic0(S)
    outs = []
    for use_graph in (False, True, True, False):
        x, res = lpcg.pcg_solve(S, lpcg.PC_LLT, cuda_f64(b), l_val=l, ut_val=ut, tol=1e-8,
                                use_graph=use_graph, check_every=3)
        torch.cuda.synchronize()
        outs.append((host(x), res["iters"]))
    for x, it in outs[1:]:
        assert it == outs[0][1]
        assert np.array_equal(x, outs[0][0])


def test_pcg_maxit_notconv_and_zero_rhs():
    A = matrices_small()["poisson2d_32"]
    S = gpu_system(A)
    b = np.random.default_rng(2).standard_normal(A.n)
    x, res = lpcg.pcg_solve(S, lpcg.PC_JACOBI, cuda_f64(b), tol=1e-12, maxit=5)
    assert res["status"] == lpcg.ENOTCONV and res["iters"] == 5
    ref = O.pcg(A, b, O.PC_JACOBI, tol=1e-12, maxit=5)
    assert ref["status"] == O.NOTCONV
    np.testing.assert_allclose(host(x), ref["x"], rtol=1e-4, atol=1e-5 * np.abs(ref["x"]).max())
    x, res = lpcg.pcg_solve(S, lpcg.PC_JACOBI, cuda_f64(np.zeros(A.n)), tol=1e-6)
    assert res["status"] == lpcg.OK and res["iters"] == 0 and not np.any(host(x))


def test_pcg_breakdown_on_indefinite():
    A = g.csr_from_dense(np.array([[1.0, 0.0], [0.0, -1.0]]))
    S = gpu_system(A)
    x, res = lpcg.pcg_solve(S, lpcg.PC_NONE, cuda_f64(np.array([1.0, 1.0])), tol=1e-8)
    assert res["status"] == lpcg.EBREAKDOWN
    ref = O.pcg(A, np.array([1.0, 1.0]), O.PC_NONE, tol=1e-8)
    assert ref["status"] == O.BREAKDOWN and ref["iters"] == res["iters"]


def test_pcg_nonzero_initial_guess_and_restart():
    A = matrices_small()["fem_40"]
    b = np.random.default_rng(4).standard_normal(A.n)
    S = gpu_system(A)
    x0 = np.random.default_rng(5).standard_normal(A.n)
    x, res = lpcg.pcg_solve(S, lpcg.PC_JACOBI, cuda_f64(b), x=cuda_f64(x0), tol=1e-10,
                            max_restarts=3)
    assert res["status"] == lpcg.OK and res["relres_true"] <= 1e-10


@pytest.mark.parametrize("ordering", [0, 1])
def test_time_pcg_kernels_parts(ordering):
    """The timing aid runs the iteration's three parts and returns positive
    durations; with Jacobi the application part is empty (0), and so is the
    update part in the red-black order, whose two-level pair (ELL form)
    performs the update.  A solve afterwards on the same system is
    unaffected (it resets its own state)."""
    A, b = g.heat_system_3d(16, 1e-3, 3, 4)
    S = gpu_system(A, None, ordering)
    bd = cuda_f64(b)
    l, ut, _ = lpcg.ic0(S)
    t = lpcg.time_pcg_kernels(S, lpcg.PC_LLT, bd, l_val=l, ut_val=ut, reps=5)
    if ordering == 1:
        assert t[0] > 0 and t[1] > 0 and t[2] == 0, t
    else:
        assert all(v > 0 for v in t), t
    tj = lpcg.time_pcg_kernels(S, lpcg.PC_JACOBI, bd, reps=5)
    assert tj[0] == 0 and tj[1] > 0 and tj[2] > 0, tj
    x, res = lpcg.pcg_solve(S, lpcg.PC_LLT, bd, l_val=l, ut_val=ut, tol=1e-6, max_restarts=2)
    assert res["status"] == 0 and O.true_relres(A, b, host(x)) <= 1e-6


def test_pcg_color_fused_update():
    """Red-black order: the two-level pair's ELL form performs the x, r
    update (three launches per iteration).  Graph replay equals eager bit for
    bit and repeats bit for bit; an iteration cap ends with ENOTCONV after
    exactly maxit products at the oracle's iterate (same IC(0) in FP64); the
    residual history follows the per-level path's (separate update kernel)
    to FP32 rounding, with the same iteration count."""
    A = matrices_small()["heat3d_13"]
    b = np.random.default_rng(11).standard_normal(A.n)
    S = gpu_system(A, None, 1)
    assert S.info["nlev_fwd"] == 2
    l, ut, _ = lpcg.ic0(S)
    outs = []
    for use_graph in (False, True, True, False):
        x, res = lpcg.pcg_solve(S, lpcg.PC_LLT, cuda_f64(b), l_val=l, ut_val=ut, tol=1e-8,
                                use_graph=use_graph, check_every=3)
        torch.cuda.synchronize()
        outs.append((host(x), res["iters"]))
    for x, it in outs[1:]:
        assert it == outs[0][1]
        assert np.array_equal(x, outs[0][0])
    # the cap: 5 products, x after the 5th update
    x, res = lpcg.pcg_solve(S, lpcg.PC_LLT, cuda_f64(b), l_val=l, ut_val=ut, tol=1e-12, maxit=5)
    assert res["status"] == lpcg.ENOTCONV and res["iters"] == 5
    perm, _, _ = O.color_order(A)
    Ap = O.permute_sym(A, perm)
    pat = O.Pattern(Ap)
    lref, _ = O.ic0(pat, Ap)
    ref = O.pcg(Ap, b[perm], O.PC_LLT, pat, lref, tol=1e-12, maxit=5)
    assert ref["status"] == O.NOTCONV
    xr = np.empty(A.n)
    xr[perm] = ref["x"]
    np.testing.assert_allclose(host(x), xr, rtol=1e-4, atol=1e-5 * np.abs(xr).max())
    # history against the per-level path (k_xr)
    _, r1, h1 = lpcg.pcg_solve(S, lpcg.PC_LLT, cuda_f64(b), l_val=l, ut_val=ut, tol=1e-8, hist=True)
    lpcg.set_trsv_cfg(S, 1, 0)
    _, r2, h2 = lpcg.pcg_solve(S, lpcg.PC_LLT, cuda_f64(b), l_val=l, ut_val=ut, tol=1e-8, hist=True)
    assert r1["status"] == 0 and r2["status"] == 0 and r1["iters"] == r2["iters"], (r1, r2)
    k = r1["iters"] + 1
    h1, h2 = host(h1)[:k], host(h2)[:k]
    assert np.all(np.abs(h1 - h2) <= 1e-3 * h2), np.max(np.abs(h1 - h2) / h2)


def test_pcg_color_fused_breakdown():
    """Red-black order, where the product's p.w is reduced by the next
    application: a negative definite A (the factor of the SPD -A) breaks down
    at the first product, as the oracle does, with the iteration counted and
    x left at x0."""
    A = matrices_small()["heat3d_13"]
    b = np.random.default_rng(12).standard_normal(A.n)
    S = gpu_system(A, None, 1)
    l, ut, _ = lpcg.ic0(S)
    neg = g.CSR(A.n, A.rowptr, A.colind, -A.val)
    lpcg.update_values(S, cuda_f64(neg.val))
    x, res = lpcg.pcg_solve(S, lpcg.PC_LLT, cuda_f64(b), l_val=l, ut_val=ut, tol=1e-8)
    perm, _, _ = O.color_order(A)
    Ap = O.permute_sym(A, perm)
    pat = O.Pattern(Ap)
    lref, _ = O.ic0(pat, Ap)
    ref = O.pcg(O.permute_sym(neg, perm), b[perm], O.PC_LLT, pat, lref, tol=1e-8)
    assert ref["status"] == O.BREAKDOWN
    assert res["status"] == lpcg.EBREAKDOWN and res["iters"] == ref["iters"] == 1, (res, ref["iters"])
    assert not np.any(host(x))


@pytest.mark.parametrize("case", ["natural_ic0", "color_ic0", "jacobi"])
def test_pcg_adaptive_chunks_equal_fixed(case):
    """When the host looks at the done flag changes nothing on the device:
    chunks sized from the residual's decay (check_every = 0), fixed chunks of
    8 and of 1, and graph replay give the same iterate bit for bit, the same
    iteration count, status and residual history; also when the cap ends the
    solve (tol = 0) and with a cap below the first chunk."""
    print(f"[pcg] adaptive chunks {case}", flush=True)
    A = matrices_small()["heat3d_13"]
    b = np.random.default_rng(21).standard_normal(A.n)
    S = gpu_system(A, None, 1 if case == "color_ic0" else 0)
    if case == "jacobi":
        kind, kw = lpcg.PC_JACOBI, {}
    else:
        l, ut, _ = lpcg.ic0(S)
        kind, kw = lpcg.PC_LLT, dict(l_val=l, ut_val=ut)
    for tol, maxit, status in ((1e-8, 0, lpcg.OK), (0.0, 23, lpcg.ENOTCONV), (1e-12, 3, lpcg.ENOTCONV)):
        outs = []
        for check_every, use_graph in ((0, False), (8, False), (1, False), (5, True)):
            x, res, h = lpcg.pcg_solve(S, kind, cuda_f64(b), tol=tol, maxit=maxit, check_every=check_every,
                                       use_graph=use_graph, hist=True, **kw)
            torch.cuda.synchronize()
            outs.append((host(x), res["iters"], res["status"], host(h)))
        assert outs[0][2] == status, (tol, maxit, outs[0][1:3])
        if maxit:
            assert outs[0][1] == maxit
        for x, it, st, h in outs[1:]:
            assert (it, st) == outs[0][1:3], (tol, maxit, it, st, outs[0][1:3])
            assert np.array_equal(x, outs[0][0])
            assert np.array_equal(h, outs[0][3], equal_nan=True)
