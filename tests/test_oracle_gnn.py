"""Pins for the FP64 GNN oracle (forward and hand-written reverse mode).

Forward: a hand-computed 2-node example (tests/golden/gnn_two_node.json),
the all-zero-weight closed form, permutation equivariance of the symmetric
assembly, and n_mp-hop locality.  Backward: central finite differences and an
independent torch float64 autograd model written with different primitives.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle as O
import pdegen as g
from oracle import gnn

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_two_node_hand_example():
    fx = json.load(open(os.path.join(GOLD, "gnn_two_node.json")))
    A = g.csr_from_dense(np.array(fx["A"]))
    P = {k: np.array(v, dtype=float) for k, v in fx["params"].items()}
    for k, v in P.items():
        if k.endswith(("b0", "b1")):
            P[k] = v.reshape(-1)
    lval, _ = gnn.forward(A, np.array(fx["b"]), P, fx["h"], fx["n_mp"])
    np.testing.assert_allclose(lval, fx["expected_lval"], rtol=1e-15)


def test_zero_weights_closed_form():
    """All weights zero: every MLP returns its last bias, so d = dec.b1 on
    every edge; L_ij = sqrt(s) dec.b1 (i>j), L_ii = sqrt(s) max(softplus(dec.b1), 1e-6)."""
    A, b = g.heat_system_3d(5, 1e-3, k_seed=3, u0_seed=4)
    P = g.init_gnn_params(8, 3, seed=1, zero=True)
    c = float(P["dec.b1"][0])
    lval, _ = gnn.forward(A, b, P, 8, 3)
    pat = O.Pattern(A)
    s = np.mean(O.diag(A))
    row = np.repeat(np.arange(A.n), np.diff(pat.lrowptr))
    diag = pat.lcol == row
    np.testing.assert_allclose(lval[~diag], np.sqrt(s) * c, rtol=1e-15)
    np.testing.assert_allclose(lval[diag], np.sqrt(s) * np.log1p(np.exp(c)), rtol=1e-15)


def _sym_dense(A, lval):
    pat = O.Pattern(A)
    row = np.repeat(np.arange(A.n), np.diff(pat.lrowptr))
    S = np.zeros((A.n, A.n))
    S[row, pat.lcol] = lval
    S[pat.lcol, row] = lval
    return S


def test_permutation_equivariance():
    A = g.fem_p1_delaunay(10, 2, 3)[0]
    b = np.random.default_rng(0).standard_normal(A.n)
    P = g.init_gnn_params(6, 3, seed=2)
    lval, _ = gnn.forward(A, b, P, 6, 3)
    perm = np.random.default_rng(1).permutation(A.n)
    Ap = g.permute_csr(A, perm)
    lp, _ = gnn.forward(Ap, b[perm], P, 6, 3)
    S = _sym_dense(A, lval)
    Sp = _sym_dense(Ap, lp)
    np.testing.assert_allclose(Sp, S[np.ix_(perm, perm)], rtol=1e-12, atol=1e-12)


def test_locality_n_mp_hops():
    """L_ij depends on b only within n_mp hops of {i, j}: flipping the sign of a
    far b_k (rms(b) unchanged) leaves those entries bit-identical."""
    m, n_mp = 12, 3
    A = g.poisson_grid(m, 2)
    b = np.random.default_rng(3).standard_normal(A.n)
    P = g.init_gnn_params(8, n_mp, seed=4)
    l0, _ = gnn.forward(A, b, P, 8, n_mp)
    b2 = b.copy()
    b2[0] = -b2[0]  # corner node (0, 0)
    l1, _ = gnn.forward(A, b2, P, 8, n_mp)
    pat = O.Pattern(A)
    row = np.repeat(np.arange(A.n), np.diff(pat.lrowptr))
    col = pat.lcol

    def dist(i):
        return i % m + i // m  # graph distance to the corner on the grid
    far = np.minimum(dist(row), dist(col)) > n_mp
    assert far.sum() > 0 and (~far).sum() > 0
    assert np.array_equal(l0[far], l1[far])
    assert np.any(l0[~far] != l1[~far])


def _masks(A, b, P, h, n_mp):
    _, c = gnn.forward(A, b, P, h, n_mp, keep=True)
    return [c["mlp"][k][1] > 0 for k in sorted(c["mlp"])]


def _fd_check(A, b, P, h, n_mp, seed):
    """Central differences in a region where every ReLU keeps its side (the
    map is smooth there); eps is halved until the activation pattern at
    theta +- eps v equals the one at theta."""
    rng = np.random.default_rng(seed)
    lval, cache = gnn.forward(A, b, P, h, n_mp, keep=True)
    gl = rng.standard_normal(lval.shape[0])
    G = gnn.backward(P, cache, gl)
    m0 = _masks(A, b, P, h, n_mp)
    for _ in range(3):
        V = {k: rng.standard_normal(v.shape) for k, v in P.items()}
        eps = 1e-6
        while True:
            Pp = {k: P[k] + eps * V[k] for k in P}
            Pm = {k: P[k] - eps * V[k] for k in P}
            same = all(np.array_equal(a, c) for a, c in zip(m0, _masks(A, b, Pp, h, n_mp))) and \
                all(np.array_equal(a, c) for a, c in zip(m0, _masks(A, b, Pm, h, n_mp)))
            if same or eps < 1e-10:
                break
            eps /= 4
        fp = gl @ gnn.forward(A, b, Pp, h, n_mp)[0]
        fm = gl @ gnn.forward(A, b, Pm, h, n_mp)[0]
        fd = (fp - fm) / (2 * eps)
        an = sum(np.sum(G[k] * V[k]) for k in P)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (fd, an, eps)


def test_backward_finite_differences():
    A = g.poisson_grid(5, 2)
    b = np.random.default_rng(5).standard_normal(A.n)
    _fd_check(A, b, g.init_gnn_params(4, 2, seed=6), 4, 2, 7)
    F = g.fem_p1_delaunay(7, 1, 2)[0]
    bf = np.random.default_rng(8).standard_normal(F.n)
    _fd_check(F, bf, g.init_gnn_params(3, 3, seed=9), 3, 3, 10)


def _torch_model(A, b, P, h, n_mp, diag_mode=0, x_head=False):
    """Independent float64 model with torch primitives (index_add_, cat,
    softplus); modes 1/2 build L = L' D^(1/2) as a dense matrix product."""
    row = torch.as_tensor(A.row_of_entry(), dtype=torch.long)
    col = torch.as_tensor(A.colind, dtype=torch.long)
    val = torch.as_tensor(A.val)
    bt = torch.as_tensor(b)
    s = val[row == col].mean()
    rms = torch.sqrt((bt * bt).mean())
    T = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in P.items()}

    def mlp(name, x):
        return torch.relu(x @ T[name + ".W0"] + T[name + ".b0"]) @ T[name + ".W1"] + T[name + ".b1"]
    V = mlp("node_enc", (bt / rms)[:, None])
    E = mlp("edge_enc", (val / s)[:, None])
    for t in range(n_mp):
        m = torch.zeros(A.n, h, dtype=torch.float64).index_add_(0, row, E * V[col])
        V = mlp(f"mp{t}.node", torch.cat([V, m], 1))
        E = mlp(f"mp{t}.edge", torch.cat([E, V[row], V[col]], 1))
    d = mlp("dec", E)[:, 0]
    if x_head:
        T["__xhat"] = mlp("xdec", V)[:, 0]
    # pair average via a dense symmetric scatter
    Dm = torch.zeros(A.n, A.n, dtype=torch.float64).index_put((row, col), d)
    Sym = 0.5 * (Dm + Dm.T)
    lower = col <= row
    if diag_mode == 0:
        diag = torch.clamp(torch.nn.functional.softplus(torch.diagonal(Dm)), min=1e-6)
        Lfull = torch.tril(Sym, -1) + torch.diag(diag)
        return torch.sqrt(s) * Lfull[row[lower], col[lower]], T
    if diag_mode == 3:  # strictly lower as mode 1, diagonal completed
        Ad = torch.as_tensor(A.to_dense()).diagonal()
        Ls = torch.tril(Sym, -1) * torch.sqrt(Ad)[None, :]
        rad = Ad - (Ls * Ls).sum(1)
        ldg = torch.sqrt(torch.where(rad > 1e-3 * Ad, rad, 1e-3 * Ad))
        Lfull = Ls + torch.diag(ldg)
        return Lfull[row[lower], col[lower]], T
    if diag_mode == 1:
        dprime = torch.ones(A.n, dtype=torch.float64)
    else:
        dprime = torch.clamp(torch.nn.functional.softplus(torch.diagonal(Dm) + np.log(np.e - 1)), min=1e-6)
    Lp = torch.tril(Sym, -1) + torch.diag(dprime)
    Ad = torch.as_tensor(A.to_dense()).diagonal()
    Lfull = Lp @ torch.diag(torch.sqrt(Ad))
    return Lfull[row[lower], col[lower]], T


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_backward_matches_torch_autograd(mode):
    A = g.fem_p1_delaunay(8, 3, 4)[0]
    b = np.random.default_rng(11).standard_normal(A.n)
    h, n_mp = 5, 3
    P = g.init_gnn_params(h, n_mp, seed=12, gain=1.5)
    lval, cache = gnn.forward(A, b, P, h, n_mp, keep=True, diag_mode=mode)
    lt, T = _torch_model(A, b, P, h, n_mp, diag_mode=mode)
    np.testing.assert_allclose(lval, lt.detach().numpy(), rtol=1e-12, atol=1e-13)
    gl = np.random.default_rng(13).standard_normal(lval.shape[0])
    (lt * torch.as_tensor(gl)).sum().backward()
    G = gnn.backward(P, cache, gl)
    for k in P:
        np.testing.assert_allclose(G[k], T[k].grad.numpy(), rtol=1e-10, atol=1e-11, err_msg=k)


def test_training_loss_normalisation():
    """Per-system loss = ||L L^T x - b||^2 / rms(b)^2 (scale-free in b)."""
    A = g.poisson_grid(6, 2)
    pat = O.Pattern(A)
    b = np.random.default_rng(1).standard_normal(A.n)
    x = np.linalg.solve(A.to_dense(), b)
    lval = O.ic0(pat, A)[0]
    l1, g1 = gnn.training_loss(A, b, x, lval, pat.lrowptr, pat.lcol,
                               lambda lv, xx, bb: O.llt_loss(pat, lv, xx, bb))
    l2, g2 = gnn.training_loss(A, 10 * b, 10 * x, lval, pat.lrowptr, pat.lcol,
                               lambda lv, xx, bb: O.llt_loss(pat, lv, xx, bb))
    assert np.isclose(l1, l2, rtol=1e-12)
    np.testing.assert_allclose(g1, g2, rtol=1e-10, atol=1e-12 * np.max(np.abs(g1)))


def test_adam_first_step_is_signed_lr_and_minimises_quadratic():
    """First step from zero moments: m_hat = g, v_hat = g^2, so the update is
    lr * g / (|g| + eps) = lr * sign(g) up to eps.  On f(p) = sum(c p^2 / 2)
    the iterates approach the minimiser 0."""
    rng = np.random.default_rng(0)
    p0 = {"w": rng.standard_normal(50)}
    g = {"w": rng.standard_normal(50)}
    z = {"w": np.zeros(50)}
    p1, _, _ = gnn.adam(p0, g, z, z, step=1, lr=1e-2)
    np.testing.assert_allclose(p0["w"] - p1["w"], 1e-2 * g["w"] / (np.abs(g["w"]) + 1e-8), rtol=1e-12)
    assert np.all(np.sign(p0["w"] - p1["w"]) == np.sign(g["w"]))
    c = rng.uniform(0.5, 2.0, 50)
    p, m, v = {"w": rng.standard_normal(50)}, dict(z), dict(z)
    start = np.abs(p["w"]).max()
    for t in range(1, 3001):
        p, m, v = gnn.adam(p, {"w": c * p["w"]}, m, v, step=t, lr=1e-2)
    assert np.abs(p["w"]).max() < 0.05 * start


@pytest.mark.parametrize("mode", [1, 2])
def test_diag_mode1_zero_weights_closed_form_and_jacobi_start(mode):
    """diag_mode 1/2 (L' D L'^T with D = diag(A)) and all-zero weights except a
    zero decoder bias: L' = I, so P = diag(A) exactly (Jacobi); with decoder
    bias c: L_ij = sqrt(A_jj) c below the diagonal, L_ii = sqrt(A_ii) (mode 1)
    or sqrt(A_ii) log(1 + (e - 1) e^c) (mode 2: softplus(c + ln(e - 1)))."""
    A, b = g.heat_system_3d(5, 1e-3, k_seed=3, u0_seed=4)
    pat = O.Pattern(A)
    row = np.repeat(np.arange(A.n), np.diff(pat.lrowptr))
    diag = pat.lcol == row
    P = g.init_gnn_params(8, 2, seed=1, zero=True)
    c = float(P["dec.b1"][0])
    lval, _ = gnn.forward(A, b, P, 8, 2, diag_mode=mode)
    ad = O.diag(A)
    dscale = 1.0 if mode == 1 else np.log1p((np.e - 1.0) * np.exp(c))
    np.testing.assert_allclose(lval[diag], np.sqrt(ad) * dscale, rtol=1e-14)
    np.testing.assert_allclose(lval[~diag], np.sqrt(ad[pat.lcol[~diag]]) * c, rtol=1e-15)
    P["dec.b1"][:] = 0.0
    lval, _ = gnn.forward(A, b, P, 8, 2, diag_mode=mode)
    np.testing.assert_allclose(lval[diag], np.sqrt(ad), rtol=1e-15)
    x = np.random.default_rng(0).standard_normal(A.n)
    r1 = O.pcg(A, x, O.PC_LLT, pat, lval, tol=1e-10, maxit=5)
    r2 = O.pcg(A, x, O.PC_JACOBI, tol=1e-10, maxit=5)
    np.testing.assert_allclose(r1["x"], r2["x"], rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_diag_mode1_backward_finite_differences_and_torch(mode):
    A = g.fem_p1_delaunay(8, 3, 4)[0]
    b = np.random.default_rng(11).standard_normal(A.n)
    h, n_mp = 4, 2
    P = g.init_gnn_params(h, n_mp, seed=12, gain=1.5)
    lval, cache = gnn.forward(A, b, P, h, n_mp, keep=True, diag_mode=mode)
    rng = np.random.default_rng(3)
    gl = rng.standard_normal(lval.shape[0])
    G = gnn.backward(P, cache, gl)
    V = {k: rng.standard_normal(v.shape) for k, v in P.items()}
    eps = 1e-7
    fp = gl @ gnn.forward(A, b, {k: P[k] + eps * V[k] for k in P}, h, n_mp, diag_mode=mode)[0]
    fm = gl @ gnn.forward(A, b, {k: P[k] - eps * V[k] for k in P}, h, n_mp, diag_mode=mode)[0]
    fd = (fp - fm) / (2 * eps)
    an = sum(np.sum(G[k] * V[k]) for k in P)
    assert abs(fd - an) <= 1e-5 * max(1.0, abs(fd)), (fd, an)


def test_x_head_zero_weights_closed_form():
    """All-zero weights: the node decoder outputs its bias, so x0 = b1 rms(b)/s
    at every node (appendix "Comparison with Starting Guess")."""
    A, b = g.heat_system_3d(5, 1e-3, k_seed=3, u0_seed=4)
    P = g.init_gnn_params(8, 2, seed=1, zero=True, x_head=True)
    _, cache = gnn.forward(A, b, P, 8, 2, x_head=True)
    s = np.mean(O.diag(A))
    rms = np.sqrt(np.mean(b ** 2))
    np.testing.assert_allclose(cache["x0"], P["xdec.b1"][0] * rms / s, rtol=1e-15)


def test_x_head_backward_torch_and_finite_differences():
    A = g.fem_p1_delaunay(8, 3, 4)[0]
    b = np.random.default_rng(11).standard_normal(A.n)
    h, n_mp = 5, 2
    P = g.init_gnn_params(h, n_mp, seed=12, gain=1.5, x_head=True)
    lval, cache = gnn.forward(A, b, P, h, n_mp, keep=True, diag_mode=1, x_head=True)
    rng = np.random.default_rng(13)
    gl = rng.standard_normal(lval.shape[0])
    gx = rng.standard_normal(A.n)
    G = gnn.backward(P, cache, gl, gx)
    # independent float64 torch model with autograd
    lt, T = _torch_model(A, b, P, h, n_mp, diag_mode=1, x_head=True)
    np.testing.assert_allclose(cache["xhat"], T["__xhat"].detach().numpy(), rtol=1e-12, atol=1e-13)
    ((lt * torch.as_tensor(gl)).sum() + (T["__xhat"] * torch.as_tensor(gx)).sum()).backward()
    for k in P:
        np.testing.assert_allclose(G[k], T[k].grad.numpy(), rtol=1e-10, atol=1e-11, err_msg=k)
    # central differences along a random direction
    V = {k: rng.standard_normal(v.shape) for k, v in P.items()}
    eps = 1e-7

    def f(Q):
        lv, c = gnn.forward(A, b, Q, h, n_mp, diag_mode=1, x_head=True)
        return gl @ lv + gx @ c["xhat"]
    fd = (f({k: P[k] + eps * V[k] for k in P}) - f({k: P[k] - eps * V[k] for k in P})) / (2 * eps)
    an = sum(np.sum(G[k] * V[k]) for k in P)
    assert abs(fd - an) <= 1e-5 * max(1.0, abs(fd)), (fd, an)


def test_x0_loss_zero_at_solution_and_gradient():
    A, b = g.heat_system_3d(4, 1e-3, 1, 2)
    x = np.linalg.solve(A.to_dense(), b)
    s = np.mean(O.diag(A))
    rms = np.sqrt(np.mean(b ** 2))
    loss, gr = gnn.x0_loss(A, b, x, x * s / rms)
    assert loss == 0.0 and np.all(gr == 0.0)
    xh = np.random.default_rng(0).standard_normal(A.n)
    loss, gr = gnn.x0_loss(A, b, x, xh)
    v = np.random.default_rng(1).standard_normal(A.n)
    eps = 1e-6
    fd = (gnn.x0_loss(A, b, x, xh + eps * v)[0] - gnn.x0_loss(A, b, x, xh - eps * v)[0]) / (2 * eps)
    assert abs(fd - gr @ v) <= 1e-7 * max(1.0, abs(fd))


def test_diag_mode3_completed_diagonal():
    """Mode 3: every row with its radicand above the floor has
    (L L^T)_ii = A_ii (dense product, FP64); all-zero weights with decoder
    bias c give L_ij = sqrt(A_jj) c and L_ii = sqrt(max(A_ii - c^2 sum_j A_jj,
    1e-3 A_ii)), computed here from the dense matrix."""
    A, b = g.heat_system_3d(5, 1e-3, k_seed=3, u0_seed=4)
    pat = O.Pattern(A)
    Ad = A.to_dense()
    ad = np.diag(Ad)
    row = np.repeat(np.arange(A.n), np.diff(pat.lrowptr))
    P = g.init_gnn_params(8, 2, seed=21, gain=1.5)
    lval, _ = gnn.forward(A, b, P, 8, 2, diag_mode=3)
    Ld = np.zeros((A.n, A.n))
    Ld[row, pat.lcol] = lval
    strict = np.tril(Ld, -1)
    rad = ad - (strict ** 2).sum(1)
    act = rad > 1e-3 * ad
    assert act.sum() > 0
    np.testing.assert_allclose(np.diag(Ld @ Ld.T)[act], ad[act], rtol=1e-13)
    np.testing.assert_allclose(np.diag(Ld)[~act], np.sqrt(1e-3 * ad[~act]), rtol=1e-14)
    Z = g.init_gnn_params(8, 2, seed=1, zero=True)
    c = float(Z["dec.b1"][0])
    lz, _ = gnn.forward(A, b, Z, 8, 2, diag_mode=3)
    offp = np.where(Ad != 0, 1.0, 0.0) * (np.arange(A.n)[:, None] > np.arange(A.n)[None, :])
    Lz = offp * np.sqrt(ad)[None, :] * c
    dz = np.sqrt(np.maximum(ad - (Lz ** 2).sum(1), 1e-3 * ad))
    Lz += np.diag(dz)
    np.testing.assert_allclose(lz, Lz[row, pat.lcol], rtol=1e-14, atol=1e-300)
