"""GPU parity: the preconditioner GNN forward (BF16 MFMA, FP32 accumulation)
against the FP64 oracle.

Bars (tests/parity_bars.py): the strictly lower entries, which are the
network's decoded pair averages, and the diagonal are checked separately,
each by relative Frobenius <= 2e-2 and entry by entry within 3e-2 of
(|ref| + rms of the part); in diag_mode 1 the diagonal sqrt(A_ii) carries
no network output and must match to two FP32 ulps.  The bars sit 2.3-5x
above the error of a BF16 emulation of the same arithmetic
(tests/bf16_emul.py).  Every diagonal entry must be positive and finite."""
import numpy as np
import pytest
import torch

import oracle as O
import pdegen as g
from oracle import gnn as ognn
from paper_2305_16432_amd import lpcg
from tests import parity_bars as PB
from tests.gpu_util import cuda_f64, gpu_system, host, matrices_small

pytestmark = pytest.mark.gpu


def _gpu_L(S, A, b, P, h, n_mp, diag_mode=0):
    params = lpcg.pack_params(P, h, n_mp).cuda()
    ws = lpcg.gnn_workspace(S, h, n_mp)
    nl = S.info["nnz_l"]
    lv = torch.empty(nl, dtype=torch.float32, device="cuda")
    ut = torch.empty(nl, dtype=torch.float32, device="cuda")
    lpcg.gnn_predict_L(S, params, h, n_mp, cuda_f64(b), ws, lv, ut, diag_mode=diag_mode)
    torch.cuda.synchronize()
    return host(lv).astype(np.float64), host(ut).astype(np.float64)


def _check(A, b, h, n_mp, seed, sys_rowptr=None, diag_mode=0, P=None):
    pat = O.Pattern(A)
    if P is None:
        P = g.init_gnn_params(h, n_mp, seed=seed)
    S = gpu_system(A, sys_rowptr)
    lg, ut = _gpu_L(S, A, b, P, h, n_mp, diag_mode)
    if sys_rowptr is None:
        ref, _ = ognn.forward(A, b, P, h, n_mp, rev=pat.rev, diag_mode=diag_mode)
    else:  # per-system normalisation: the oracle runs each block separately
        ref = _blockwise_ref(A, b, P, h, n_mp, sys_rowptr, pat, diag_mode)
    st = PB.check_factor(pat, lg, ref, diag_mode)
    print("bars:", {k: f"{v:.2e}" for k, v in st.items()}, flush=True)
    np.testing.assert_array_equal(ut, lg[pat.usrc])
    return st


def _blockwise_ref(A, b, P, h, n_mp, srp, pat, diag_mode=0):
    out = np.zeros(pat.nnz_l)
    for s in range(len(srp) - 1):
        r0, r1 = srp[s], srp[s + 1]
        sub = g.canonical_csr(A.to_scipy()[r0:r1, r0:r1])
        lsub, _ = ognn.forward(sub, b[r0:r1], P, h, n_mp, diag_mode=diag_mode)
        out[pat.lrowptr[r0]:pat.lrowptr[r1]] = lsub
    return out


@pytest.mark.parametrize("diag_mode", [0, 1, 2, 3])
@pytest.mark.parametrize("h,n_mp", [(32, 3), (64, 2), (64, 5)])
@pytest.mark.parametrize("name", ["poisson2d_32", "heat3d_13", "fem_40", "random_777", "tridiag_1000",
                                  "one"])
def test_gnn_forward_parity(name, h, n_mp, diag_mode):
    print(f"[gnn] {name} h={h} n_mp={n_mp} diag_mode={diag_mode}", flush=True)
    A = matrices_small()[name]
    b = np.random.default_rng(1).standard_normal(A.n)
    _check(A, b, h, n_mp, seed=5, diag_mode=diag_mode)


@pytest.mark.parametrize("diag_mode", [0, 1, 2, 3])
def test_gnn_forward_batch_per_system_normalisation(diag_mode):
    mats = [g.poisson_grid(9, 2), g.heat_system_3d(6, 1e-3, 1, 2)[0], g.fem_p1_delaunay(13, 0, 1)[0]]
    B, srp = g.block_diag_csr(mats)
    rng = np.random.default_rng(3)
    b = np.concatenate([rng.standard_normal(m.n) * (10.0 ** s) for s, m in enumerate(mats)])
    _check(B, b, 32, 3, seed=7, sys_rowptr=srp, diag_mode=diag_mode)


@pytest.mark.parametrize("diag_mode", [0, 1, 2, 3])
def test_gnn_forward_c3_full_size(diag_mode):
    print(f"[gnn] heat3d_64 h=32 n_mp=3 diag_mode={diag_mode}", flush=True)
    A, b = g.heat_system_3d(64, 1e-3, 1000, 2000)
    _check(A, b, 32, 3, seed=11, diag_mode=diag_mode)


@pytest.mark.parametrize("wfile", ["heat3d_h32_mp3_ft64.npz", "heat3d_h32_mp3.npz"])
def test_gnn_forward_trained_c3_full_size(wfile):
    """The shipped networks, whose decoded values vary from edge to edge, on
    the full 64^3 benchmark system."""
    import os
    W = np.load(os.path.join(os.path.dirname(lpcg.__file__), "weights", wfile))
    h, n_mp, dm = int(W["h"]), int(W["n_mp"]), int(W["diag_mode"])
    P = {k: np.asarray(v, np.float64) for k, v in
         lpcg.unpack_params(torch.as_tensor(W["params"].astype(np.float32)), h, n_mp).items()}
    print(f"[gnn] heat3d_64 trained {wfile}", flush=True)
    A, b = g.heat_system_3d(64, 1e-3, 1000, 2000)
    _check(A, b, h, n_mp, seed=0, diag_mode=dm, P=P)


@pytest.mark.parametrize("diag_mode", [0, 1])
def test_gnn_forward_c1_full_size(diag_mode):
    """The 2D FEM configuration: 128 x 128 jittered points (15,876 unknowns),
    h = 64 with 5 message-passing layers (the appendix's depth for its 2D
    problems), softplus diagonal (mode 0) and the fixed-diagonal form."""
    print(f"[gnn] fem_128 h=64 n_mp=5 diag_mode={diag_mode}", flush=True)
    A, b, _ = g.fem_p1_delaunay(128, 0, 1)
    _check(A, b, 64, 5, seed=13, diag_mode=diag_mode)


def test_gnn_zero_weights_closed_form():
    """All-zero weights: d = dec.b1 on every edge, so L_ij = sqrt(s) dec.b1 and
    L_ii = sqrt(s) softplus(dec.b1) exactly up to FP32 rounding."""
    A, b = g.heat_system_3d(7, 1e-3, 3, 4)
    P = g.init_gnn_params(32, 2, seed=1, zero=True)
    S = gpu_system(A)
    lg, _ = _gpu_L(S, A, b, P, 32, 2)
    pat = O.Pattern(A)
    c = float(np.float32(P["dec.b1"][0]))
    s = np.mean(O.diag(A))
    row = np.repeat(np.arange(A.n), np.diff(pat.lrowptr))
    diag = pat.lcol == row
    np.testing.assert_allclose(lg[~diag], np.sqrt(s) * c, rtol=1e-6)
    np.testing.assert_allclose(lg[diag], np.sqrt(s) * np.log1p(np.exp(c)), rtol=1e-6)


def test_gnn_deterministic_and_workspace_check():
    A = matrices_small()["fem_40"]
    b = np.random.default_rng(2).standard_normal(A.n)
    P = g.init_gnn_params(32, 3, seed=2)
    S = gpu_system(A)
    l1, _ = _gpu_L(S, A, b, P, 32, 3)
    l2, _ = _gpu_L(S, A, b, P, 32, 3)
    assert np.array_equal(l1, l2)
    params = lpcg.pack_params(P, 32, 3).cuda()
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(lpcg.LpcgError) as e:
        lpcg.gnn_predict_L(S, params, 32, 3, cuda_f64(b), small)
    assert e.value.code == lpcg.ENOMEM
    with pytest.raises(lpcg.LpcgError) as e:
        lpcg.gnn_predict_L(S, params, 48, 3, cuda_f64(b), lpcg.gnn_workspace(S, 32, 3))
    assert e.value.code == lpcg.EINVAL


def test_learned_pcg_c1_full_size():
    """Learned-L PCG on the 2D FEM configuration (15,876 unknowns, h = 64,
    five layers, fixed-diagonal form): the GPU's factor in the GPU's PCG and
    the oracle's factor in the oracle's PCG reach 1e-6 in the same number of
    iterations, give or take max(2, 10%), and the FP64 residual is met."""
    print("[gnn] fem_128 learned-L PCG", flush=True)
    A, b, _ = g.fem_p1_delaunay(128, 0, 1)
    pat = O.Pattern(A)
    h, n_mp, dm = 64, 5, 1
    P = g.init_gnn_params(h, n_mp, seed=13)
    S = gpu_system(A)
    params = lpcg.pack_params(P, h, n_mp).cuda()
    ws = lpcg.gnn_workspace(S, h, n_mp)
    lv = torch.empty(pat.nnz_l, dtype=torch.float32, device="cuda")
    ut = torch.empty_like(lv)
    bd = cuda_f64(b)
    lpcg.gnn_predict_L(S, params, h, n_mp, bd, ws, lv, ut, diag_mode=dm)
    x, r = lpcg.pcg_solve(S, lpcg.PC_LLT, bd, l_val=lv, ut_val=ut, tol=1e-6, max_restarts=2)
    lref, _ = ognn.forward(A, b, P, h, n_mp, rev=pat.rev, diag_mode=dm)
    ro = O.pcg(A, b, O.PC_LLT, pat, lref, tol=1e-6)
    print(f"iters gpu {r['iters']} oracle {ro['iters']}", flush=True)
    assert r["status"] == 0 and O.true_relres(A, b, host(x)) <= 1e-6
    assert abs(r["iters"] - ro["iters"]) <= max(2, 0.1 * ro["iters"])


@pytest.mark.parametrize("n_mp", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("name", ["heat3d_13", "fem_40", "poisson2d_32"])
def test_gnn_fused_inference_parity(name, n_mp):
    """Inference at width 32 and up to four layers runs the fused pass (edge
    latents recomputed, never stored); five layers, and training, run the
    stored form.  Both against the oracle, and the fused factor against the
    training forward's (stored form) on the same weights, by the same bars."""
    print(f"[gnn] fused {name} h=32 n_mp={n_mp}", flush=True)
    A = matrices_small()[name]
    b = np.random.default_rng(2).standard_normal(A.n)
    P = g.init_gnn_params(32, n_mp, seed=17)
    st = _check(A, b, 32, n_mp, seed=17, diag_mode=1, P=P)
    S = gpu_system(A)
    params = lpcg.pack_params(P, 32, n_mp).cuda()
    ws = lpcg.gnn_workspace(S, 32, n_mp, train=True)
    lt = host(lpcg.gnn_forward_train(S, params, 32, n_mp, cuda_f64(b), ws, diag_mode=1)).astype(np.float64)
    lf, _ = _gpu_L(S, A, b, P, 32, n_mp, 1)
    pat = O.Pattern(A)
    st2 = PB.check_factor(pat, lf, lt, 1)
    print("fused vs stored:", {k: f"{v:.2e}" for k, v in st2.items()}, "oracle:", st["off_rel"], flush=True)


def test_gnn_row_longer_than_a_tile():
    """A row with more than 32 stored entries (a star graph joined to a grid)
    has no row-aligned tile: inference falls back to the stored form."""
    import scipy.sparse as sp
    base = g.poisson_grid(8, 2).to_scipy().tolil()
    n = base.shape[0]
    for j in range(1, 40):
        base[0, j] = base[j, 0] = -0.01
    base[0, 0] = base[0, 0] + 1.0
    A = g.canonical_csr(sp.csr_matrix(base))
    assert np.max(np.diff(A.rowptr)) > 32
    b = np.random.default_rng(4).standard_normal(n)
    _check(A, b, 32, 3, seed=19, diag_mode=0)
