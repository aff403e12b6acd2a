"""FP64 NumPy oracle of the preconditioner GNN -- TEST INFRASTRUCTURE ONLY.

Follows the paper's architecture (Method, "Architecture"; technical-details
appendix):
  * graph/matrix duality: every stored A_ij (diagonal included, as a self-loop)
    is a directed edge i->j with scalar feature A_ij; the right-hand side b is
    the scalar node feature;
  * encoders: node and edge MLPs lift the scalars to h-dimensional latents;
  * n_mp message-passing layers:
        v_{i,t+1}  = f_v(v_{i,t}, sum_j e_{ij,t} * v_{j,t})     (* elementwise)
        e_{ij,t+1} = f_e(e_{ij,t}, v_{i,t+1}, v_{j,t+1})        for every
    directed edge, i.e. both (i,j) and (j,i) are updated;
  * decoder: d_ij = f_dec(e_ij), a scalar per directed edge;
  * lower-triangular assembly: L_ij = (d_ij + d_ji)/2 for i > j.

Readings where the paper is silent (each listed in the design notes):
  * every MLP is Lin-ReLU-Lin ("l layers" = 2 Linear layers), width h;
  * the sum over j runs over every stored entry of row i (self-loop included),
    without degree normalisation;
  * normalisation: s = mean(diag A), edge input A_ij/s, node input b_i/rms(b);
    the network's factor is scaled back by sqrt(s): L = sqrt(s) * L_hat;
  * diag_mode 0: the diagonal, where the pair average is d_ii itself, is made
    positive with L_ii = max(softplus(d_ii), 1e-6) so that L L^T is SPD by
    construction, and L = sqrt(s) * L_hat;
  * diag_mode 1 (the appendix's L D L^T form with D = diag(A), reading L'
    as unit lower-triangular): P = L' D L'^T = L L^T with L = L' D^(1/2),
    i.e. L_ii = sqrt(A_ii), L_ij = sqrt(A_jj) (d_ij + d_ji)/2;
  * diag_mode 2 (the same form, reading L' as a general lower-triangular
    factor, which is what makes the appendix's equivalence with L L^T hold):
    L'_ii = max(softplus(d_ii + ln(e - 1)), 1e-6) > 0 (equal to 1 at
    d_ii = 0), so L_ii = sqrt(A_ii) L'_ii and L_ij = sqrt(A_jj) (d_ij + d_ji)/2.
    Zero decoder output gives L' = I, i.e. P = diag(A), in modes 1 and 2.
  * diag_mode 3 (a reading of the same L' D L'^T form in which the diagonal
    is not predicted but completed): the strictly-lower entries as in mode 1,
    L_ij = sqrt(A_jj) (d_ij + d_ji)/2, and
    L_ii = sqrt(max(A_ii - sum_{j<i} L_ij^2, 1e-3 A_ii)), so that
    diag(L L^T) = diag(A) wherever the floor is not reached.  On a red-black
    ordering, decoded values d_ij = A_ij / A_jj reproduce IC(0) exactly.

frobenius_loss: the loss_A ablation of the loss-function section, pinned by
a dense computation, finite differences, zero at an exact Cholesky factor
and a closed form for a diagonal L (tests/test_oracle_frobenius.py).

Pins (tests/test_oracle_gnn.py): all-zero weights give a closed form; a
2-node graph computed by hand; permutation equivariance; 5-hop locality;
the reverse-mode derivative against central finite differences, the
dot-product (adjoint) test and an independent torch-autograd float64 model.
"""
from __future__ import annotations

import numpy as np

SOFTPLUS_FLOOR = 1e-6
DIAG_SHIFT = float(np.log(np.e - 1.0))  # softplus(DIAG_SHIFT) = 1
COMPLETE_FLOOR = 1e-3  # mode 3: L_ii^2 >= 1e-3 A_ii


def _relu(x):
    return np.maximum(x, 0.0)


def _softplus(x):
    return np.where(x > 20.0, x, np.log1p(np.exp(np.minimum(x, 20.0))))


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _mlp_fwd(P, name, x):
    pre = x @ P[f"{name}.W0"] + P[f"{name}.b0"]
    hid = _relu(pre)
    out = hid @ P[f"{name}.W1"] + P[f"{name}.b1"]
    return out, (x, pre, hid)


def _mlp_bwd(P, name, cache, gout, G):
    x, pre, hid = cache
    G[f"{name}.W1"] += hid.T @ gout
    G[f"{name}.b1"] += gout.sum(axis=0)
    ghid = gout @ P[f"{name}.W1"].T
    gpre = ghid * (pre > 0.0)
    G[f"{name}.W0"] += x.T @ gpre
    G[f"{name}.b0"] += gpre.sum(axis=0)
    return gpre @ P[f"{name}.W0"].T


def normalisation(A, b):
    """(s, rms): s = mean of diag(A), rms = sqrt(mean(b^2)) (1 if b = 0)."""
    row = A.row_of_entry()
    s = float(np.mean(A.val[A.colind == row]))
    rms = float(np.sqrt(np.mean(np.asarray(b, np.float64) ** 2)))
    return s, (rms if rms > 0.0 else 1.0)


def reverse_map(A):
    """rev[k] = position of (j,i) for entry k = (i,j): search for key j*n+i in
    the row-major sorted key list of the CSR entries."""
    row = A.row_of_entry().astype(np.int64)
    col = A.colind.astype(np.int64)
    key = row * A.n + col
    q = np.searchsorted(key, col * A.n + row)
    assert np.all(q < A.nnz) and np.all(key[np.minimum(q, A.nnz - 1)] == col * A.n + row), \
        "pattern is not structurally symmetric"
    return q


def forward(A, b, P, h, n_mp, rev=None, keep=False, diag_mode=0, x_head=False):
    """L values on the lower pattern (i >= j) in CSR order, float64.

    Returns (lval, cache) where cache (if keep) holds what backward needs.
    With x_head the node decoder regresses the normalised solution from the
    final node latents (appendix "Comparison with Starting Guess"): the cache
    is always returned and holds xhat (normalised units, x s / rms(b)) and x0
    (the starting guess in the system's units).
    """
    row = A.row_of_entry().astype(np.int64)
    col = A.colind.astype(np.int64)
    n = A.n
    if rev is None:
        rev = reverse_map(A)
    s, rms = normalisation(A, b)
    ahat = (A.val / s)[:, None]
    bhat = (np.asarray(b, np.float64) / rms)[:, None]
    caches = {}
    V, caches["node_enc"] = _mlp_fwd(P, "node_enc", bhat)
    E, caches["edge_enc"] = _mlp_fwd(P, "edge_enc", ahat)
    Vs, Es = [V], [E]
    for t in range(n_mp):
        m = np.zeros((n, h))
        np.add.at(m, row, E * V[col])
        V, caches[f"mp{t}.node"] = _mlp_fwd(P, f"mp{t}.node", np.concatenate([V, m], axis=1))
        E, caches[f"mp{t}.edge"] = _mlp_fwd(P, f"mp{t}.edge",
                                            np.concatenate([E, V[row], V[col]], axis=1))
        Vs.append(V)
        Es.append(E)
    d, caches["dec"] = _mlp_fwd(P, "dec", E)
    d = d[:, 0]
    xhat = None
    if x_head:
        xo, caches["xdec"] = _mlp_fwd(P, "xdec", V)
        xhat = xo[:, 0]
        keep = True
    lower = col <= row
    diag = col == row
    if diag_mode == 0:
        lhat = np.where(diag, np.maximum(_softplus(d), SOFTPLUS_FLOOR), 0.5 * (d + d[rev]))
        lval = np.sqrt(s) * lhat[lower]
        colscale = None
    else:
        adiag = A.val[diag]                       # A_jj, j = 0..n-1
        colscale = np.sqrt(adiag[np.minimum(row, col)])  # sqrt(A_cc), cc = column of the lower entry
        if diag_mode in (1, 3):
            ldiag = np.sqrt(adiag[row])
        else:
            ldiag = colscale * np.maximum(_softplus(d + DIAG_SHIFT), SOFTPLUS_FLOOR)
        lfull = np.where(diag, ldiag, colscale * 0.5 * (d + d[rev]))
        if diag_mode == 3:  # complete the diagonal: diag(L L^T) = diag(A)
            strict = lower & ~diag
            ssq = np.zeros(n)
            np.add.at(ssq, row[strict], lfull[strict] ** 2)
            rad = adiag - ssq
            active = rad > COMPLETE_FLOOR * adiag       # the floor not reached
            ldg = np.sqrt(np.where(active, rad, COMPLETE_FLOOR * adiag))
            lfull = np.where(diag, ldg[row], lfull)
        lval = lfull[lower]
    cache = None
    if keep:
        cache = dict(row=row, col=col, rev=rev, s=s, rms=rms, d=d, lower=lower, diag=diag,
                     Vs=Vs, Es=Es, mlp=caches, n=n, h=h, n_mp=n_mp, diag_mode=diag_mode,
                     colscale=colscale, xhat=xhat, x0=None if xhat is None else xhat * rms / s,
                     lfull=lfull if diag_mode != 0 else None,
                     active=active if diag_mode == 3 else None)
    return lval, cache


def backward(P, cache, glval, gxhat=None):
    """Gradients of sum(glval * lval) (+ sum(gxhat * xhat) with the x_hat
    head) w.r.t. every parameter (float64 dict)."""
    G = {k: np.zeros_like(v) for k, v in P.items()}
    row, col, rev = cache["row"], cache["col"], cache["rev"]
    n, h, n_mp = cache["n"], cache["h"], cache["n_mp"]
    d, lower, diag = cache["d"], cache["lower"], cache["diag"]
    nnz = d.shape[0]
    gd = np.zeros(nnz)
    off = lower & ~diag
    if cache.get("diag_mode", 0) == 0:
        glhat = np.zeros(nnz)
        glhat[np.nonzero(lower)[0]] = np.sqrt(cache["s"]) * np.asarray(glval, np.float64)
        # diagonal: max(softplus(d), floor)
        sp = _softplus(d)
        gd += np.where(diag & (sp > SOFTPLUS_FLOOR), glhat * _sigmoid(d), 0.0)
    else:
        # strictly lower scaled by sqrt(A_jj); diagonal fixed to sqrt(A_ii)
        # (mode 1) or sqrt(A_ii) max(softplus(d_ii + shift), floor) (mode 2)
        glhat = np.zeros(nnz)
        glhat[np.nonzero(lower)[0]] = np.asarray(glval, np.float64)
        if cache["diag_mode"] == 3:
            # L_ii = sqrt(A_ii - sum_j L_ij^2): dL_ii / dL_ij = -L_ij / L_ii
            # for the strictly-lower entries of row i (0 at the floor)
            lf = cache["lfull"]
            gdiag = np.zeros(n)
            gdiag[row[diag]] = glhat[diag]
            strict = lower & ~diag
            ldiag = np.zeros(n)
            ldiag[row[diag]] = lf[diag]
            act = cache["active"][row]
            glhat = glhat + np.where(strict & act, -gdiag[row] * lf / ldiag[row], 0.0)
        if cache["diag_mode"] == 2:
            ds = d + DIAG_SHIFT
            gd += np.where(diag & (_softplus(ds) > SOFTPLUS_FLOOR),
                           glhat * cache["colscale"] * _sigmoid(ds), 0.0)
        glhat = glhat * np.where(diag, 0.0, cache["colscale"])
    # strictly lower: (d_k + d_rev(k)) / 2
    gd += np.where(off, 0.5 * glhat, 0.0)
    np.add.at(gd, rev[off], 0.5 * glhat[off])
    gE = _mlp_bwd(P, "dec", cache["mlp"]["dec"], gd[:, None], G)
    Vs, Es = cache["Vs"], cache["Es"]
    gV = np.zeros((n, h))
    if gxhat is not None:  # the x_hat head reads the final node latents
        gV = _mlp_bwd(P, "xdec", cache["mlp"]["xdec"], np.asarray(gxhat, np.float64)[:, None], G)
    for t in range(n_mp - 1, -1, -1):
        gX = _mlp_bwd(P, f"mp{t}.edge", cache["mlp"][f"mp{t}.edge"], gE, G)
        gE = gX[:, :h].copy()
        gV = gV.copy()
        np.add.at(gV, row, gX[:, h:2 * h])
        np.add.at(gV, col, gX[:, 2 * h:])
        gY = _mlp_bwd(P, f"mp{t}.node", cache["mlp"][f"mp{t}.node"], gV, G)
        gVt = gY[:, :h].copy()
        gm = gY[:, h:]
        Vt, Et = Vs[t], Es[t]
        # m_i = sum_{k in row i} E_k * V_{col k}
        gE += gm[row] * Vt[col]
        np.add.at(gVt, col, gm[row] * Et)
        gV = gVt
    _mlp_bwd(P, "node_enc", cache["mlp"]["node_enc"], gV, G)
    _mlp_bwd(P, "edge_enc", cache["mlp"]["edge_enc"], gE, G)
    return G


def training_loss(A, b, x, lval, pat_lrowptr, pat_lcol, llt_loss):
    """Per-system normalised data loss ||L L^T x - b||^2 / rms(b)^2 and its
    gradient w.r.t. L (llt_loss: the C oracle's raw loss/gradient routine)."""
    _, rms = normalisation(A, b)
    loss, g = llt_loss(lval, x, b)
    return loss / rms ** 2, g / rms ** 2


def x0_loss(A, b, x, xhat):
    """Regression loss of the x_hat head for one system: ||xhat - x s/rms(b)||^2
    in the network's normalised units, and its gradient w.r.t. xhat."""
    s, rms = normalisation(A, b)
    d = np.asarray(xhat, np.float64) - np.asarray(x, np.float64) * s / rms
    return float(d @ d), 2.0 * d


def frobenius_loss(A, lval, lrowptr, lcol):
    """The Frobenius loss of equation loss_A for one system,
    ||L L^T - A||_F^2 over every entry (the fill of L L^T included), divided
    by s^2 with s = mean(diag A) (scale-free reading), and its gradient with
    respect to the stored entries of L: d/dL_ij = 4 ((L L^T - A) L)_ij.
    Sparse products (scipy) on the explicit matrices."""
    import scipy.sparse as sp
    n = A.n
    L = sp.csr_matrix((np.asarray(lval, np.float64), np.asarray(lcol), np.asarray(lrowptr)), shape=(n, n))
    E = (L @ L.T - A.to_scipy()).tocsr()
    s, _ = normalisation(A, np.ones(n))
    loss = float(np.sum(E.data ** 2))
    G = (E @ L).tocsr()
    rows = np.repeat(np.arange(n), np.diff(lrowptr))
    g = 4.0 * np.asarray(G[rows, np.asarray(lcol)]).ravel()
    return loss / s ** 2, g / s ** 2


def adam(params, grads, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015, Algorithm 1) on dicts of float64
    arrays; returns (params, m, v) as new dicts."""
    P, M, Vv = {}, {}, {}
    for k in params:
        M[k] = beta1 * m[k] + (1 - beta1) * grads[k]
        Vv[k] = beta2 * v[k] + (1 - beta2) * grads[k] ** 2
        mhat = M[k] / (1 - beta1 ** step)
        vhat = Vv[k] / (1 - beta2 ** step)
        P[k] = params[k] - lr * mhat / (np.sqrt(vhat) + eps)
    return P, M, Vv
