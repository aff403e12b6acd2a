"""GPU parity of the training side: data loss and its gradient, the
hand-written GNN reverse mode, Adam, and the autograd wiring.

Tolerances: the loss runs in FP64 on FP32 factor values, so it matches the
oracle on the same (FP32-rounded) values to 1e-10 relative and the FP32
gradient to 1e-6.  The GNN backward rounds GEMM operands to BF16 (relative
rounding 2^-9) like the forward.  The whole flattened gradient must have
cosine similarity >= 0.999 with the FP64 oracle's and relative error <= 0.05.
Per tensor, both the relative error and 1 - cosine must stay within 6 times
those of a BF16 emulation of the same arithmetic on the same inputs
(tests/bf16_emul.py; floors 0.05 and 0.01; tests/parity_bars.py).  The
emulation sets each tensor's scale: the first-layer encoder weights
([1 x h]) sum n signed terms whose cancellation costs digits, while a tensor
such as dec.b1 is accurate to 1e-3; a tensor off by a factor of 2 fails."""
import numpy as np
import pytest
import torch

import oracle as O
import pdegen as g
from oracle import gnn as ognn
from paper_2305_16432_amd import lpcg
from tests import bf16_emul as EMU
from tests import parity_bars as PB
from tests.gpu_util import cuda_f32, cuda_f64, gpu_system, host, matrices_small

pytestmark = pytest.mark.gpu


def test_llt_loss_parity_batch():
    mats = [g.poisson_grid(8, 2), g.heat_system_3d(5, 1e-3, 1, 2)[0], g.fem_p1_delaunay(11, 0, 1)[0]]
    B, srp = g.block_diag_csr(mats)
    pat = O.Pattern(B)
    rng = np.random.default_rng(0)
    lval = rng.uniform(-0.5, 0.5, pat.nnz_l).astype(np.float32).astype(np.float64)
    row = np.repeat(np.arange(B.n), np.diff(pat.lrowptr))
    lval[pat.lcol == row] = rng.uniform(1, 2, (pat.lcol == row).sum()).astype(np.float32)
    x = rng.standard_normal(B.n)
    b = rng.standard_normal(B.n) * 3.0
    S = gpu_system(B, srp)
    loss, dl = lpcg.llt_loss(S, cuda_f32(lval), cuda_f64(x), cuda_f64(b))
    loss, dl = host(loss), host(dl).astype(np.float64)
    ref_g = np.zeros(pat.nnz_l)
    for s in range(len(mats)):
        r0, r1 = srp[s], srp[s + 1]
        sub = g.canonical_csr(B.to_scipy()[r0:r1, r0:r1])
        sp = O.Pattern(sub)
        lsub = lval[pat.lrowptr[r0]:pat.lrowptr[r1]]
        ls, gs = ognn.training_loss(sub, b[r0:r1], x[r0:r1], lsub, sp.lrowptr, sp.lcol,
                                    lambda lv, xx, bb: O.llt_loss(sp, lv, xx, bb))
        assert abs(loss[s] - ls) <= 1e-10 * abs(ls)
        ref_g[pat.lrowptr[r0]:pat.lrowptr[r1]] = gs
    np.testing.assert_allclose(dl, ref_g, rtol=1e-6, atol=1e-6 * np.abs(ref_g).max())


def _grad_check(A, b, h, n_mp, seed, sys_rowptr=None, diag_mode=0):
    P = g.init_gnn_params(h, n_mp, seed=seed)
    pat = O.Pattern(A)
    S = gpu_system(A, sys_rowptr)
    params = lpcg.pack_params(P, h, n_mp).cuda()
    ws = lpcg.gnn_workspace(S, h, n_mp, train=True)
    gl = np.random.default_rng(seed + 1).standard_normal(pat.nnz_l).astype(np.float32)
    lpcg.gnn_forward_train(S, params, h, n_mp, cuda_f64(b), ws, diag_mode=diag_mode)
    d1 = lpcg.gnn_backward(S, params, h, n_mp, ws, cuda_f32(gl), diag_mode=diag_mode)
    d2 = lpcg.gnn_backward(S, params, h, n_mp, ws, cuda_f32(gl), diag_mode=diag_mode)
    assert torch.equal(d1, d2), "backward not bit-reproducible"
    G = lpcg.unpack_params(d1, h, n_mp)
    _, cache = ognn.forward(A, b, P, h, n_mp, rev=pat.rev, keep=True, diag_mode=diag_mode)
    R = ognn.backward(P, cache, gl.astype(np.float64))
    _, ce = EMU.forward(A, b, P, h, n_mp, pat.rev, diag_mode=diag_mode, keep=True)
    Em = EMU.backward(P, ce, gl.astype(np.float64))
    keys = [k for k, _ in lpcg.param_layout(h, n_mp)]
    worst = PB.check_grads({k: np.asarray(G[k], np.float64) for k in keys}, R, Em, keys)
    return worst


@pytest.mark.parametrize("diag_mode", [0, 1, 2, 3])
@pytest.mark.parametrize("h,n_mp", [(32, 3), (64, 2), (64, 5)])
@pytest.mark.parametrize("name", ["poisson2d_32", "heat3d_13", "fem_40"])
def test_gnn_backward_parity(name, h, n_mp, diag_mode):
    print(f"[gnn bwd] {name} h={h} n_mp={n_mp} diag_mode={diag_mode}", flush=True)
    A = matrices_small()[name]
    b = np.random.default_rng(4).standard_normal(A.n)
    worst = _grad_check(A, b, h, n_mp, seed=6, diag_mode=diag_mode)
    print("bars", worst, flush=True)


@pytest.mark.parametrize("diag_mode", [0, 1])
def test_gnn_backward_c1_full_size(diag_mode):
    """The 2D FEM configuration at full size: 15,876 unknowns, h = 64, five
    message-passing layers."""
    print(f"[gnn bwd] fem_128 h=64 n_mp=5 diag_mode={diag_mode}", flush=True)
    A, b, _ = g.fem_p1_delaunay(128, 0, 1)
    worst = _grad_check(A, b, 64, 5, seed=13, diag_mode=diag_mode)
    print("bars", worst, flush=True)


def test_gnn_backward_batch():
    mats = [g.poisson_grid(9, 2), g.heat_system_3d(6, 1e-3, 1, 2)[0], g.fem_p1_delaunay(13, 0, 1)[0]]
    B, srp = g.block_diag_csr(mats)
    b = np.random.default_rng(3).standard_normal(B.n)
    P = g.init_gnn_params(32, 2, seed=9)
    pat = O.Pattern(B)
    S = gpu_system(B, srp)
    params = lpcg.pack_params(P, 32, 2).cuda()
    ws = lpcg.gnn_workspace(S, 32, 2, train=True)
    gl = np.random.default_rng(10).standard_normal(pat.nnz_l).astype(np.float32)
    lpcg.gnn_forward_train(S, params, 32, 2, cuda_f64(b), ws)
    G = host(lpcg.gnn_backward(S, params, 32, 2, ws, cuda_f32(gl))).astype(np.float64)
    # the batch gradient is the sum of the per-system gradients
    R = None
    for s in range(len(mats)):
        r0, r1 = srp[s], srp[s + 1]
        sub = g.canonical_csr(B.to_scipy()[r0:r1, r0:r1])
        _, cache = ognn.forward(sub, b[r0:r1], P, 32, 2, keep=True)
        Rs = ognn.backward(P, cache, gl[pat.lrowptr[r0]:pat.lrowptr[r1]].astype(np.float64))
        flat = np.concatenate([Rs[k].ravel() for k, _ in lpcg.param_layout(32, 2)])
        R = flat if R is None else R + flat
    cos = G @ R / (np.linalg.norm(G) * np.linalg.norm(R))
    assert cos >= 0.999 and np.linalg.norm(G - R) / np.linalg.norm(R) <= 0.05


def test_adam_parity():
    rng = np.random.default_rng(1)
    p = {"w": rng.standard_normal(10007)}
    m = {"w": rng.standard_normal(10007) * 0.1}
    v = {"w": rng.uniform(0, 0.1, 10007)}
    gr = {"w": rng.standard_normal(10007)}
    # the kernel takes its hyper-parameters as FP32: give the oracle the same values
    f = lambda a: float(np.float32(a))  # noqa: E731
    P1, M1, V1 = ognn.adam(p, gr, m, v, step=7, lr=f(3e-3), beta1=f(0.9), beta2=f(0.999), eps=f(1e-8))
    pt, mt, vt = (cuda_f32(d["w"]) for d in (p, m, v))
    lpcg.adam_step(pt, cuda_f32(gr["w"]), mt, vt, 3e-3, 7)
    # FP32 vs FP64: a few ulps of the larger of the two terms of each update
    u = 2.0 ** -24
    tm = 8 * u * (0.9 * np.abs(m["w"]) + 0.1 * np.abs(gr["w"]))
    tv = 8 * u * (0.999 * v["w"] + 0.001 * gr["w"] ** 2)
    assert np.all(np.abs(host(mt) - M1["w"]) <= tm + 1e-5 * np.abs(M1["w"]))
    assert np.all(np.abs(host(vt) - V1["w"]) <= tv + 1e-5 * np.abs(V1["w"]))
    np.testing.assert_allclose(host(pt), P1["w"], rtol=1e-5, atol=1e-6)


def test_autograd_chain_matches_manual():
    A, b = g.heat_system_3d(8, 1e-3, 1, 2)
    x = np.linalg.solve(A.to_dense(), b)
    h, n_mp = 32, 2
    S = gpu_system(A)
    params = lpcg.pack_params(g.init_gnn_params(h, n_mp, seed=3), h, n_mp).cuda().requires_grad_(True)
    ws = lpcg.gnn_workspace(S, h, n_mp, train=True)
    bd, xd = cuda_f64(b), cuda_f64(x)
    L = lpcg.GnnL.apply(params, S, h, n_mp, bd, ws)
    loss = lpcg.LltLoss.apply(L, S, xd, bd)
    loss.backward()
    _, dl = lpcg.llt_loss(S, L.detach(), xd, bd)
    manual = lpcg.gnn_backward(S, params.detach(), h, n_mp, ws, dl)
    assert torch.equal(params.grad, manual)


def test_training_reduces_loss_on_one_batch():
    """Overfitting one small batch with Adam reduces the data loss by >= 10x."""
    mats, xs, bs = [], [], []
    for s in range(4):
        A, b = g.heat_system_3d(8, 1e-3, 10 + s, 20 + s)
        mats.append(A)
        bs.append(b)
        xs.append(np.linalg.solve(A.to_dense(), b))
    B, srp = g.block_diag_csr(mats)
    S = gpu_system(B, srp)
    h, n_mp = 32, 2
    params = lpcg.pack_params(g.init_gnn_params(h, n_mp, seed=0, gain=0.5), h, n_mp).cuda()
    m, v = torch.zeros_like(params), torch.zeros_like(params)
    ws = lpcg.gnn_workspace(S, h, n_mp, train=True)
    bd, xd = cuda_f64(np.concatenate(bs)), cuda_f64(np.concatenate(xs))
    losses = []
    for step in range(1, 301):
        L = lpcg.gnn_forward_train(S, params, h, n_mp, bd, ws)
        loss, dl = lpcg.llt_loss(S, L, xd, bd)
        losses.append(float(loss.sum()))
        grad = lpcg.gnn_backward(S, params, h, n_mp, ws, dl)
        lpcg.adam_step(params, grad, m, v, 3e-3, step)
    print(f"loss {losses[0]:.4g} -> {min(losses):.4g}")
    assert min(losses) <= 0.1 * losses[0]
