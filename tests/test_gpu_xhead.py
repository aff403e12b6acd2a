"""GPU parity of the initial-guess head (appendix comparing with a predicted
starting guess x^0): the node decoder's forward, its loss and its place in
the hand-written reverse mode, against the FP64 oracle.

Tolerances: the head is an MLP of the same shape as the edge decoder on
BF16-rounded latents, so its output takes the forward's bars
(tests/parity_bars.py): relative norm <= 2e-2 over all nodes and, node by
node, within 3e-2 of (|ref| + rms).  The loss runs in FP64 on the FP32 head
output and matches the oracle's formula on that same output to 1e-10
relative.  The reverse mode takes the network backward's bars: whole
gradient cosine >= 0.999 and relative norm <= 0.05, and per tensor the
relative error and 1 - cosine within 6 times those of a BF16 emulation on
the same inputs (tests/bf16_emul.py).  Its target is the solution A^-1 b, as in training:
with an independent random target the head's node gradients have random
signs, so the bias and first-layer gradients (sums over all nodes) cancel
down to their BF16 rounding noise, which measures nothing about the code.
"""
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


def _x0(S, P, h, n_mp, b, diag_mode=1):
    params = lpcg.pack_params(P, h, n_mp).cuda()
    ws = lpcg.gnn_workspace(S, h, n_mp)
    l_val, _, x0 = lpcg.gnn_predict_x0(S, params, h, n_mp, cuda_f64(b), ws, diag_mode=diag_mode)
    torch.cuda.synchronize()
    return host(l_val), host(x0)


@pytest.mark.parametrize("h,n_mp", [(32, 3), (64, 2)])
@pytest.mark.parametrize("name", ["poisson2d_32", "heat3d_13", "fem_40", "random_777", "tridiag_1000", "one"])
def test_x0_forward_parity(name, h, n_mp):
    print(f"[x0 fwd] {name} h={h} n_mp={n_mp}", flush=True)
    A = matrices_small()[name]
    b = np.random.default_rng(3).standard_normal(A.n)
    P = g.init_gnn_params(h, n_mp, seed=7, x_head=True)
    S = gpu_system(A)
    lg, x0 = _x0(S, P, h, n_mp, b)
    _, cache = ognn.forward(A, b, P, h, n_mp, diag_mode=1, x_head=True)
    print("bars:", PB.check_vector(x0, cache["x0"]), flush=True)
    # L from the same launch equals the plain predictor's, bit for bit
    P_nohead = {k: v for k, v in P.items() if not k.startswith("xdec.")}
    params = lpcg.pack_params(P_nohead, h, n_mp).cuda()
    lv, _ = lpcg.gnn_predict_L(S, params, h, n_mp, cuda_f64(b), lpcg.gnn_workspace(S, h, n_mp), diag_mode=1)
    np.testing.assert_array_equal(host(lv), lg)


def test_x0_zero_weights_closed_form():
    """All-zero weights but the head's output bias c: x0 = c rms(b) / s."""
    A, b = g.heat_system_3d(9, 1e-3, 1, 2)
    P = g.init_gnn_params(32, 2, seed=0, zero=True, x_head=True)
    P["xdec.b1"][:] = 0.75
    _, x0 = _x0(gpu_system(A), P, 32, 2, b)
    s = np.mean(O.diag(A))
    rms = np.sqrt(np.mean(b ** 2))
    np.testing.assert_allclose(x0, 0.75 * rms / s, rtol=1e-6)


def test_x0_colour_order_is_original_numbering():
    """The network is equivariant under renumbering: the colour-ordered
    system returns x0 in the caller's numbering, equal to the natural one up
    to the forward's BF16 error."""
    A, b = g.heat_system_3d(13, 1e-3, 5, 6)
    P = g.init_gnn_params(32, 3, seed=2, x_head=True)
    _, xn = _x0(gpu_system(A), P, 32, 3, b)
    _, xc = _x0(gpu_system(A, ordering=lpcg.ORDER_COLOR), P, 32, 3, b)
    _, cache = ognn.forward(A, b, P, 32, 3, diag_mode=1, x_head=True)
    for x in (xn, xc):
        PB.check_vector(x, cache["x0"])


def test_x0_batch_per_system_scaling():
    mats = [g.poisson_grid(12, 2), g.heat_system_3d(6, 1e-3, 1, 2)[0], g.fem_p1_delaunay(15, 0, 1)[0]]
    B, srp = g.block_diag_csr(mats)
    rng = np.random.default_rng(5)
    b = np.concatenate([rng.standard_normal(m.n) * 10.0 ** k for k, m in enumerate(mats)])
    P = g.init_gnn_params(32, 2, seed=8, x_head=True)
    _, x0 = _x0(gpu_system(B, srp), P, 32, 2, b)
    for s, m in enumerate(mats):
        r0, r1 = srp[s], srp[s + 1]
        _, cache = ognn.forward(m, b[r0:r1], P, 32, 2, diag_mode=1, x_head=True)
        PB.check_vector(x0[r0:r1], cache["x0"], f"x0 of system {s}")


def test_x0_loss_parity_and_errors():
    mats = [g.poisson_grid(10, 2), g.heat_system_3d(5, 1e-3, 3, 4)[0]]
    B, srp = g.block_diag_csr(mats)
    rng = np.random.default_rng(9)
    b = rng.standard_normal(B.n)
    x = rng.standard_normal(B.n)
    P = g.init_gnn_params(32, 2, seed=10, x_head=True)
    S = gpu_system(B, srp, ordering=lpcg.ORDER_COLOR)
    params = lpcg.pack_params(P, 32, 2).cuda()
    ws = lpcg.gnn_workspace(S, 32, 2)
    _, _, x0 = lpcg.gnn_predict_x0(S, params, 32, 2, cuda_f64(b), ws, diag_mode=1)
    loss = host(lpcg.x0_loss(S, params, 32, 2, ws, cuda_f64(x), weight=0.0, diag_mode=1))
    x0 = host(x0)
    for s, m in enumerate(mats):
        r0, r1 = srp[s], srp[s + 1]
        sc = np.mean(O.diag(m)) / np.sqrt(np.mean(b[r0:r1] ** 2))
        ref, _ = ognn.x0_loss(m, b[r0:r1], x[r0:r1], x0[r0:r1] * sc)
        assert abs(loss[s] - ref) <= 1e-10 * ref, (s, loss[s], ref)
    # a network without the head is rejected by both entry points
    P0 = {k: v for k, v in P.items() if not k.startswith("xdec.")}
    p0 = lpcg.pack_params(P0, 32, 2).cuda()
    with pytest.raises(lpcg.LpcgError):
        lpcg.gnn_predict_x0(S, p0, 32, 2, cuda_f64(b), ws, diag_mode=1)
    with pytest.raises(lpcg.LpcgError):
        lpcg.x0_loss(S, p0, 32, 2, ws, cuda_f64(x), diag_mode=1)


@pytest.mark.parametrize("with_l", [True, False])
@pytest.mark.parametrize("h,n_mp", [(32, 3), (64, 2)])
@pytest.mark.parametrize("name", ["poisson2d_32", "heat3d_13", "fem_40"])
def test_x0_backward_parity(name, h, n_mp, with_l):
    """Reverse mode with the head's loss against the solution x = A^-1 b (its
    training target), with (with_l) and without a gradient on L; the second
    case isolates the head -> node-latent chain."""
    print(f"[x0 bwd] {name} h={h} n_mp={n_mp} with_l={with_l}", flush=True)
    A = matrices_small()[name]
    rng = np.random.default_rng(11)
    b = rng.standard_normal(A.n)
    x = np.linalg.solve(A.to_dense(), b)
    P = g.init_gnn_params(h, n_mp, seed=12, x_head=True)
    pat = O.Pattern(A)
    S = gpu_system(A)
    params = lpcg.pack_params(P, h, n_mp).cuda()
    ws = lpcg.gnn_workspace(S, h, n_mp, train=True)
    gl = rng.standard_normal(pat.nnz_l).astype(np.float32) * (1.0 if with_l else 0.0)
    w = 0.3
    lpcg.gnn_forward_train(S, params, h, n_mp, cuda_f64(b), ws, diag_mode=1)
    lpcg.x0_loss(S, params, h, n_mp, ws, cuda_f64(x), weight=w, diag_mode=1)
    G = lpcg.unpack_params(lpcg.gnn_backward(S, params, h, n_mp, ws, cuda_f32(gl), diag_mode=1), h, n_mp)
    _, cache = ognn.forward(A, b, P, h, n_mp, rev=pat.rev, keep=True, diag_mode=1, x_head=True)
    _, gx = ognn.x0_loss(A, b, x, cache["xhat"])
    R = ognn.backward(P, cache, gl.astype(np.float64), w * gx)
    names = [k for k, _ in lpcg.param_layout(h, n_mp, True)]
    _, ce = EMU.forward(A, b, P, h, n_mp, pat.rev, diag_mode=1, keep=True, x_head=True)
    Em = EMU.backward(P, ce, gl.astype(np.float64), w * gx)
    print("bars", PB.check_grads({k: np.asarray(G[k], np.float64) for k in names}, R, Em, names),
          flush=True)


def test_backward_without_head_loss_matches_headless_network():
    """Without an x0 loss after the training forward the head's gradient is
    zero and every other gradient equals the headless network's bit for bit."""
    A, b = g.heat_system_3d(9, 1e-3, 7, 8)
    h, n_mp = 32, 3
    P = g.init_gnn_params(h, n_mp, seed=13, x_head=True)
    P0 = {k: v for k, v in P.items() if not k.startswith("xdec.")}
    S = gpu_system(A)
    gl = cuda_f32(np.random.default_rng(14).standard_normal(S.info["nnz_l"]))
    out = []
    for Q in (P, P0):
        params = lpcg.pack_params(Q, h, n_mp).cuda()
        ws = lpcg.gnn_workspace(S, h, n_mp, train=True)
        ws.fill_(0xFF)  # stale contents must not leak into the gradient
        lpcg.gnn_forward_train(S, params, h, n_mp, cuda_f64(b), ws, diag_mode=1)
        out.append(host(lpcg.gnn_backward(S, params, h, n_mp, ws, gl, diag_mode=1)))
    nh = out[1].shape[0]
    np.testing.assert_array_equal(out[0][:nh], out[1])
    assert np.all(out[0][nh:] == 0)
