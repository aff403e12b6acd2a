"""BF16 error model of the preconditioner GNN -- test-side only.

The GPU runs every Linear layer of the network on BF16 matrix-core
operands with FP32 accumulation and keeps node and edge latents in BF16.
This module replays the oracle's architecture (oracle/gnn.py) in NumPy
float64, rounding to BF16 (round to nearest even) exactly where the GPU
keeps a BF16 copy:

  * every GEMM operand: the layer input, the weights, the hidden layer
    after the ReLU, and in reverse mode the incoming gradient;
  * the stored latents V_t, E_t and the per-node projections of the first
    edge layer (factored as e W_e + (V W_a)[i] + (V W_b)[j]);
  * the aggregated message m_i before the node MLP.

Its outputs are used only to calibrate the parity bars of the GPU tests
(tests/parity_bars.py): the distance between this emulation and the FP64
oracle is the size of error that BF16 arithmetic alone produces, so a bar
set a few times above it passes a correct kernel and fails a kernel with a
localised or scale error.  It is not a reference for any test."""
from __future__ import annotations

import contextlib

import numpy as np

from oracle import gnn as ognn

_dither = None


@contextlib.contextmanager
def dithered(seed):
    """Inside the block every rounding first scales its operand by
    (1 + 2^-12 xi), xi ~ N(0, 1): a second, independent realisation of BF16
    rounding errors of the same size (a stand-in for another correct kernel
    with a different rounding order)."""
    global _dither
    old, _dither = _dither, np.random.default_rng(seed)
    try:
        yield
    finally:
        _dither = old


def bf16(x):
    """Round float64 values to BF16 (8-bit significand, RNE), through FP32."""
    x = np.asarray(x, np.float64)
    if _dither is not None:
        x = x * (1.0 + 2.0 ** -12 * _dither.standard_normal(x.shape))
    f = x.astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _mlp(P, name, x, store=True):
    W0, b0 = bf16(P[f"{name}.W0"]), P[f"{name}.b0"]
    W1, b1 = bf16(P[f"{name}.W1"]), P[f"{name}.b1"]
    xb = bf16(x)
    pre = xb @ W0 + b0
    hid = bf16(np.maximum(pre, 0.0))
    out = hid @ W1 + b1
    return (bf16(out) if store else out), (xb, pre, hid)


def _mlp_bwd(P, name, cache, gout, G):
    xb, pre, hid = cache
    g = bf16(gout)
    G[f"{name}.W1"] += hid.T @ g
    G[f"{name}.b1"] += g.sum(axis=0)
    gpre = bf16((g @ bf16(P[f"{name}.W1"]).T) * (pre > 0.0))
    G[f"{name}.W0"] += xb.T @ gpre
    G[f"{name}.b0"] += gpre.sum(axis=0)
    return gpre @ bf16(P[f"{name}.W0"]).T


def forward(A, b, P, h, n_mp, rev, diag_mode=0, keep=False, x_head=False):
    """L values in lower CSR order (as oracle.gnn.forward) with BF16 rounding;
    with x_head the cache also holds the head's x0 (system units)."""
    row = A.row_of_entry().astype(np.int64)
    col = A.colind.astype(np.int64)
    n = A.n
    s, rms = ognn.normalisation(A, b)
    V, cn = _mlp(P, "node_enc", (np.asarray(b, np.float64) / rms)[:, None])
    E, ce = _mlp(P, "edge_enc", (A.val / s)[:, None])
    caches = {"node_enc": cn, "edge_enc": ce}
    Vs, Es = [V], [E]
    for t in range(n_mp):
        m = np.zeros((n, h))
        np.add.at(m, row, E * V[col])
        V, caches[f"mp{t}.node"] = _mlp(P, f"mp{t}.node", np.concatenate([V, bf16(m)], axis=1))
        # factored first layer: E W_e + bf16(V W_a)[i] + bf16(V W_b)[j]
        W0 = bf16(P[f"mp{t}.edge.W0"])
        pa = bf16(V @ W0[h:2 * h])
        pb = bf16(V @ W0[2 * h:])
        pre = E @ W0[:h] + pa[row] + pb[col] + P[f"mp{t}.edge.b0"]
        hid = bf16(np.maximum(pre, 0.0))
        E = bf16(hid @ bf16(P[f"mp{t}.edge.W1"]) + P[f"mp{t}.edge.b1"])
        caches[f"mp{t}.edge"] = (np.concatenate([Es[-1], V[row], V[col]], axis=1), pre, hid)
        Vs.append(V)
        Es.append(E)
    d, caches["dec"] = _mlp(P, "dec", E, store=False)
    d = d[:, 0]
    x0 = None
    if x_head:
        xo, caches["xdec"] = _mlp(P, "xdec", V, store=False)
        x0 = xo[:, 0] * rms / s
        keep = True
    lower = col <= row
    diag = col == row
    if diag_mode == 0:
        lhat = np.where(diag, np.maximum(ognn._softplus(d), ognn.SOFTPLUS_FLOOR), 0.5 * (d + d[rev]))
        lval = np.sqrt(s) * lhat[lower]
        colscale = lfull = active = None
    else:
        adiag = A.val[diag]
        colscale = np.sqrt(adiag[np.minimum(row, col)])
        if diag_mode in (1, 3):
            ldiag = np.sqrt(adiag[row])
        else:
            ldiag = colscale * np.maximum(ognn._softplus(d + ognn.DIAG_SHIFT), ognn.SOFTPLUS_FLOOR)
        lfull = np.where(diag, ldiag, colscale * 0.5 * (d + d[rev]))
        active = None
        if diag_mode == 3:  # completed diagonal from the FP32-rounded strictly lower values
            strict = lower & ~diag
            l32 = lfull.astype(np.float32).astype(np.float64)
            ssq = np.zeros(n)
            np.add.at(ssq, row[strict], l32[strict] ** 2)
            rad = adiag - ssq
            active = rad > ognn.COMPLETE_FLOOR * adiag
            ldg = np.sqrt(np.where(active, rad, ognn.COMPLETE_FLOOR * adiag))
            lfull = np.where(diag, ldg[row], lfull)
        lval = lfull[lower]
    lval = lval.astype(np.float32).astype(np.float64)
    cache = None
    if keep:
        cache = dict(row=row, col=col, rev=rev, s=s, d=d, lower=lower, diag=diag, Vs=Vs, Es=Es,
                     mlp=caches, n=n, h=h, n_mp=n_mp, diag_mode=diag_mode, colscale=colscale, x0=x0,
                     lfull=lfull, active=active)
    return lval, cache


def backward(P, cache, glval, gxhat=None):
    """Parameter gradients of sum(glval * lval) (+ sum(gxhat * xhat) through
    the x^0 head) with BF16 operands."""
    G = {k: np.zeros_like(v, dtype=np.float64) for k, v in P.items()}
    row, col, rev = cache["row"], cache["col"], cache["rev"]
    n, h, n_mp = cache["n"], cache["h"], cache["n_mp"]
    d, lower, diag = cache["d"], cache["lower"], cache["diag"]
    gd = np.zeros(d.shape[0])
    off = lower & ~diag
    glhat = np.zeros(d.shape[0])
    glhat[np.nonzero(lower)[0]] = np.asarray(glval, np.float64)
    if cache["diag_mode"] == 0:
        glhat *= np.sqrt(cache["s"])
        gd += np.where(diag & (ognn._softplus(d) > ognn.SOFTPLUS_FLOOR), glhat * ognn._sigmoid(d), 0.0)
    else:
        if cache["diag_mode"] == 3:  # dL_ii / dL_ij = -L_ij / L_ii off the floor
            lf = cache["lfull"]
            gdiag, ldiag = np.zeros(n), np.zeros(n)
            gdiag[row[diag]] = glhat[diag]
            ldiag[row[diag]] = lf[diag]
            glhat = glhat + np.where(off & cache["active"][row], -gdiag[row] * lf / ldiag[row], 0.0)
        if cache["diag_mode"] == 2:
            ds = d + ognn.DIAG_SHIFT
            gd += np.where(diag & (ognn._softplus(ds) > ognn.SOFTPLUS_FLOOR),
                           glhat * cache["colscale"] * ognn._sigmoid(ds), 0.0)
        glhat = glhat * np.where(diag, 0.0, cache["colscale"])
    gd += np.where(off, 0.5 * glhat, 0.0)
    np.add.at(gd, rev[off], 0.5 * glhat[off])
    gE = _mlp_bwd(P, "dec", cache["mlp"]["dec"], gd[:, None], G)
    Vs, Es = cache["Vs"], cache["Es"]
    gV = np.zeros((n, h))
    if gxhat is not None:
        gV = _mlp_bwd(P, "xdec", cache["mlp"]["xdec"], np.asarray(gxhat, np.float64)[:, None], G)
    for t in range(n_mp - 1, -1, -1):
        gX = _mlp_bwd(P, f"mp{t}.edge", cache["mlp"][f"mp{t}.edge"], gE, G)
        gE = gX[:, :h].copy()
        gV = gV.copy()
        np.add.at(gV, row, gX[:, h:2 * h])
        np.add.at(gV, col, gX[:, 2 * h:])
        gY = _mlp_bwd(P, f"mp{t}.node", cache["mlp"][f"mp{t}.node"], gV, G)
        gVt = gY[:, :h].copy()
        gm = bf16(gY[:, h:])
        gE += gm[row] * Vs[t][col]
        np.add.at(gVt, col, gm[row] * Es[t])
        gV = gVt
    _mlp_bwd(P, "node_enc", cache["mlp"]["node_enc"], gV, G)
    _mlp_bwd(P, "edge_enc", cache["mlp"]["edge_enc"], gE, G)
    return G
