"""Training triples (A, b, x) for the preconditioner network, written by the
FP64 oracle -- TEST INFRASTRUCTURE (data generation only).

The Method section trains the network on tuples (A, x, b) of systems from the
PDE family the preconditioner is meant for, with x the solution of A x = b
(equation loss_Ab).  Here x comes from the oracle's own PCG (Appendix
algorithm "PCG", serial C, FP64) with its IC(0) factor, run to a relative
residual of 1e-12; where IC(0) meets a non-positive pivot the oracle's
Jacobi PCG is used instead.  Every x is checked afterwards with the oracle's
FP64 true residual.  The product never imports this module: the training
script reads the file it writes (plain arrays, no pickles).

Families (inputs from pdegen, seeded):
  heat3d  the 3D implicit heat step on an m^3 grid (k seeds 0.., u0 seeds
          10000 + seed); one shared pattern, per-system values
  fem2d   P1 FEM on a Delaunay triangulation of a side x side jittered grid
          (k seeds 0.., f seeds 20000 + seed); one pattern per system

    python -m oracle.triples --family fem2d --side 128 --nsys 1000 --out /tmp/fem2d_triples.npz
    python -m oracle.triples --family heat3d --m 32 --nsys 1000 --out /tmp/heat3d_triples.npz
"""
from __future__ import annotations

import argparse
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

TOL = 1e-12


def solve_oracle(A, b):
    """x with ||b - A x|| <= 1e-12 ||b|| from the oracle's PCG (IC(0), else
    Jacobi), restarted from the FP64 true residual (x += PCG(A, b - A x)) at
    most 3 times when the recurrence residual drifted from the true one;
    returns (x, iterations, true relative residual, preconditioner)."""
    import oracle as O
    pat = O.Pattern(A)
    lval, st = O.ic0(pat, A)
    kind = "ic0" if st == 0 else "jacobi"

    def pcg(rhs, tol):
        if kind == "ic0":
            r = O.pcg(A, rhs, O.PC_LLT, pat, lval, tol=tol, maxit=20 * A.n)
            if r["status"] == 0:
                return r
        return O.pcg(A, rhs, O.PC_JACOBI, tol=tol, maxit=20 * A.n)

    res = pcg(b, TOL)
    x, its = res["x"], res["iters"]
    nb = np.linalg.norm(b)
    for _ in range(3):
        rel = O.true_relres(A, b, x)
        if rel <= TOL:
            break
        r = b - O.spmv(A, x)
        d = pcg(r, TOL * nb / np.linalg.norm(r))
        x, its = x + d["x"], its + d["iters"]
    return x, its, O.true_relres(A, b, x), kind


def _one(args):
    family, size, seed = args
    import pdegen as g
    if family == "heat3d":
        A, b = g.heat_system_3d(size, 1e-3, k_seed=seed, u0_seed=10000 + seed)
    else:
        A, b, _ = g.fem_p1_delaunay(size, k_seed=seed, f_seed=20000 + seed)
    x, its, rel, kind = solve_oracle(A, b)
    return seed, A, b, x, its, rel, kind


def generate(family, size, seeds, workers):
    out = []
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        for i, o in enumerate(pool.imap(_one, [(family, size, s) for s in seeds], chunksize=4)):
            out.append(o)
            if (i + 1) % 100 == 0:
                print(f"[triples] {i + 1}/{len(seeds)} systems", flush=True)
    return out


def write(path, family, size, rows):
    seeds = np.array([r[0] for r in rows], np.int32)
    ns = np.array([r[1].n for r in rows], np.int64)
    nnzs = np.array([r[1].nnz for r in rows], np.int64)
    sys_rowptr = np.concatenate([[0], np.cumsum(ns)])
    sys_nnzptr = np.concatenate([[0], np.cumsum(nnzs)])
    rel = np.array([r[5] for r in rows])
    # every system's own row pointers (n_s + 1 entries each, starting at 0),
    # concatenated; system s's are rowptr[s + sys_rowptr[s] : s + 1 + sys_rowptr[s + 1]]
    arrays = dict(family=family, size=size, seeds=seeds, tol=TOL,
                  sys_rowptr=sys_rowptr, sys_nnzptr=sys_nnzptr,
                  rowptr=np.concatenate([r[1].rowptr for r in rows]).astype(np.int32),
                  colind=np.concatenate([r[1].colind for r in rows]).astype(np.int32),
                  val=np.concatenate([r[1].val for r in rows]),
                  b=np.concatenate([r[2] for r in rows]), x=np.concatenate([r[3] for r in rows]),
                  iters=np.array([r[4] for r in rows], np.int32), relres_true=rel,
                  precond=np.array([r[6] for r in rows]))
    np.savez(path, **arrays)
    return rel


def load(path):
    """The systems of a triples file as a list of (CSR, b, x) -- a reader for
    tests; the training script has its own."""
    from pdegen.csr import CSR
    z = np.load(path, allow_pickle=False)
    srp, snp = z["sys_rowptr"], z["sys_nnzptr"]
    rpa, ci, va, bb, xx = z["rowptr"], z["colind"], z["val"], z["b"], z["x"]  # each read once
    out = []
    for s in range(len(srp) - 1):
        n = int(srp[s + 1] - srp[s])
        rp = rpa[s + srp[s]:s + 1 + srp[s + 1]]
        a, c = int(snp[s]), int(snp[s + 1])
        out.append((CSR(n, rp, ci[a:c], va[a:c]), bb[srp[s]:srp[s + 1]], xx[srp[s]:srp[s + 1]]))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--family", choices=["heat3d", "fem2d"], required=True)
    ap.add_argument("--m", type=int, default=32, help="heat3d grid side")
    ap.add_argument("--side", type=int, default=128, help="fem2d point-grid side")
    ap.add_argument("--nsys", type=int, default=1000)
    ap.add_argument("--seed0", type=int, default=0)
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    size = args.m if args.family == "heat3d" else args.side
    t0 = time.time()
    rows = generate(args.family, size, list(range(args.seed0, args.seed0 + args.nsys)), args.workers)
    rel = write(args.out, args.family, size, rows)
    its = [r[4] for r in rows]
    kinds = {k: sum(r[6] == k for r in rows) for k in ("ic0", "jacobi")}
    print(f"[triples] {args.nsys} {args.family} systems -> {args.out} in {time.time() - t0:.1f}s; "
          f"oracle PCG iterations {min(its)}..{max(its)}, preconditioner {kinds}, "
          f"max true relative residual {rel.max():.2e}", flush=True)
    if not np.all(rel <= TOL * 1.0001):
        sys.exit(f"[triples] a solution misses {TOL:g}")


if __name__ == "__main__":
    main()
