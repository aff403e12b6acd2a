"""Train the preconditioner GNN on the GPU with the library's own forward,
hand-written backward, data loss and Adam kernels (paper: loss_Ab, Adam at
lr 1e-3; training-setup appendix).

Data: (A, b, x) triples read from a file written by the FP64 oracle's
triple generator (x from the oracle's PCG to a 1e-12 relative residual, the
third member of the paper's (A, x, b) training tuples):
  heat3d  implicit-Euler heat steps on an m^3 grid (7-point, k = exp(GRF
          sigma=1, ell=0.1), dt = 1e-3, b = u0 a smooth GRF), k seeds
          0..nsys-1; every system shares one pattern, so a batch of B
          systems is one block-diagonal pattern analysed once and each step
          swaps in the batch's values.
  fem2d   P1 FEM systems on jittered Delaunay meshes (one pattern per
          system): the systems are split once into fixed batches of B
          (seeded shuffle), each batch's block-diagonal pattern is analysed
          once, and each step trains on one batch.
--ordering color trains for the multicolour row ordering (the factor then
lives on tril(P A P^T)).  Held-out check: PCG iterations to 1e-6 with the
predicted L on unseen systems of the family (heat3d: eval_m^3, k seeds
5000+i, u0 seeds 6000+i; fem2d: the training mesh size, k seeds 5000+i, f
seeds 6000+i), every eval_every steps; the weights with the fewest held-out
iterations are kept (early stop on held-out; --head-only keeps the last
weights, since L does not change).

--x-head adds the initial-guess head (appendix comparing with a predicted
starting guess x^0): a node decoder regressing x s / rms(b), trained with
the weighted loss sum_i (x^_i - x_i s / rms(b))^2 next to the data loss (or
alone with --head-only, which updates only the head so L stays that of the
--init network); the held-out PCG then starts from the predicted x0.

    python -m oracle.triples --family heat3d --m 32 --nsys 1000 --out /tmp/heat3d_32.npz
    python -m paper_2305_16432_amd.train --triples /tmp/heat3d_32.npz \
        --out paper_2305_16432_amd/weights/heat3d_h32_mp3.npz

Fine-tuning on the 64^3 size the network is evaluated at (400 systems, k
seeds 0..399; held-out selection as above) gives the benchmark's network:

    python -m oracle.triples --family heat3d --m 64 --nsys 400 --out /tmp/heat3d_64.npz
    python -m paper_2305_16432_amd.train --triples /tmp/heat3d_64.npz --batch 4 --lr 1e-4 --steps 3000 \
        --init paper_2305_16432_amd/weights/heat3d_h32_mp3.npz \
        --out paper_2305_16432_amd/weights/heat3d_h32_mp3_ft64.npz

The red-black network (one message-passing layer, completed diagonal; a
single 32^3 batch of 8 systems is the most the colour analysis takes):

    python -m paper_2305_16432_amd.train --triples /tmp/heat3d_32.npz --batch 8 --h 32 --n-mp 1 \
        --diag-mode 3 --ordering color --steps 10000 --eval-systems 4 \
        --out paper_2305_16432_amd/weights/heat3d_h32_mp1_color3.npz

The 2D FEM network (h = 64, five message-passing layers, softplus diagonal;
1000 systems of a 128 x 128 jittered point grid, batch 32, Adam lr 1e-3):

    python -m oracle.triples --family fem2d --side 128 --nsys 1000 --out /tmp/fem2d_128.npz
    python -m paper_2305_16432_amd.train --triples /tmp/fem2d_128.npz --batch 32 --h 64 --n-mp 5 \
        --diag-mode 0 --out paper_2305_16432_amd/weights/fem2d_h64_mp5.npz
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def load_triples(path):
    """The systems of a triples file: list of (rowptr, colind, val, b, x)
    (NumPy), the family and its size parameter."""
    z = np.load(path, allow_pickle=False)
    # every array is read from the file once (each z[key] reads it afresh)
    srp, snp = z["sys_rowptr"], z["sys_nnzptr"]
    rp, ci, va, bb, xx = z["rowptr"], z["colind"], z["val"], z["b"], z["x"]
    rows = []
    for s in range(len(srp) - 1):
        lo, hi, a, c = int(srp[s]), int(srp[s + 1]), int(snp[s]), int(snp[s + 1])
        rows.append((rp[s + lo:s + 1 + hi], ci[a:c], va[a:c], bb[lo:hi], xx[lo:hi]))
    return rows, str(z["family"]), int(z["size"])


def shared_pattern(rows):
    r0 = rows[0]
    return all(r[0].shape == r0[0].shape and r[1].shape == r0[1].shape and np.array_equal(r[0], r0[0])
               and np.array_equal(r[1], r0[1]) for r in rows)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--triples", required=True,
                    help="(A, b, x) training file written by python -m oracle.triples")
    ap.add_argument("--nsys", type=int, default=0, help="use the first nsys systems of the file (0: all)")
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--h", type=int, default=32)
    ap.add_argument("--n-mp", type=int, default=3)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--diag-mode", type=int, default=1)
    ap.add_argument("--ordering", choices=["natural", "color"], default="natural")
    ap.add_argument("--loss", choices=["data", "frobenius"], default="data",
                    help="data: ||L L^T x - b||^2 (equation loss_Ab); frobenius: ||L L^T - A||_F^2 (loss_A ablation)")
    ap.add_argument("--x-head", action="store_true",
                    help="add the initial-guess head (node decoder regressing x); held-out PCG starts from its x0")
    ap.add_argument("--x-weight", type=float, default=1.0, help="weight of the head's loss")
    ap.add_argument("--head-only", action="store_true",
                    help="update only the head's weights (L stays that of the initial network)")
    ap.add_argument("--init", default=None, help="start from a saved network (.npz); its h, n_mp, "
                                                 "diag mode and ordering override the options")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--eval-every", type=int, default=100)
    ap.add_argument("--eval-m", type=int, default=64, help="heat3d: held-out grid side")
    ap.add_argument("--eval-maxit", type=int, default=2000)
    ap.add_argument("--eval-systems", type=int, default=1,
                    help="held-out systems (k seeds 5000+i, u0 seeds 6000+i); selection uses their mean iterations")
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    init = None
    if args.init:
        z = np.load(args.init, allow_pickle=False)
        init = z["params"]
        args.h, args.n_mp, args.diag_mode = int(z["h"]), int(z["n_mp"]), int(z["diag_mode"])
        args.ordering = "color" if int(z["ordering"]) == 1 else "natural"
    if args.head_only and not args.x_head:
        ap.error("--head-only needs --x-head")
    t0 = time.time()
    rows, family, size = load_triples(args.triples)
    if args.nsys:
        rows = rows[:args.nsys]
    args.nsys = len(rows)
    shared = shared_pattern(rows)
    print(f"[train] {args.nsys} {family} triples (size {size}, "
          f"{'one shared pattern' if shared else 'one pattern per system'}) in {time.time() - t0:.1f}s", flush=True)

    import torch

    import pdegen as g
    from paper_2305_16432_amd import lpcg
    print("[train] torch imported", flush=True)
    order = lpcg.ORDER_COLOR if args.ordering == "color" else lpcg.ORDER_NATURAL

    def batch_system(members):
        mats = [g.CSR(len(rows[i][0]) - 1, rows[i][0], rows[i][1], rows[i][2]) for i in members]
        B, srp = g.block_diag_csr(mats)
        return lpcg.analyze(torch.as_tensor(B.rowptr).cuda(), torch.as_tensor(B.colind).cuda(),
                            torch.as_tensor(B.val).cuda(), srp, order)

    rng = np.random.default_rng(args.seed)
    if shared:
        # one analysed pattern; each step gathers the batch's values
        S = batch_system(list(range(args.batch)))
        systems = [S]
        dv = torch.as_tensor(np.stack([r[2] for r in rows])).cuda()
        db = torch.as_tensor(np.stack([r[3] for r in rows])).cuda()
        dx = torch.as_tensor(np.stack([r[4] for r in rows])).cuda()
    else:
        # fixed batches (seeded shuffle), each analysed once
        perm = rng.permutation(args.nsys)
        groups = [perm[k:k + args.batch] for k in range(0, args.nsys - args.batch + 1, args.batch)]
        systems, bvec, xvec = [], [], []
        for gi, members in enumerate(groups):
            systems.append(batch_system(members))
            bvec.append(torch.as_tensor(np.concatenate([rows[i][3] for i in members])).cuda())
            xvec.append(torch.as_tensor(np.concatenate([rows[i][4] for i in members])).cuda())
        print(f"[train] {len(groups)} batches of {args.batch} systems analysed", flush=True)
        S = max(systems, key=lambda q: q.info["nnz"])
    h, n_mp = args.h, args.n_mp
    dm = args.diag_mode
    xh = args.x_head
    P0 = g.init_gnn_params(h, n_mp, seed=args.seed, gain=1.0, x_head=xh)
    # decoder output layer zero: training starts from a diagonal factor (modes
    # 1 and 2: L' = I, i.e. Jacobi; mode 0: L = sqrt(s) ln(2) I, plain CG)
    P0["dec.W1"][:] = 0.0
    P0["dec.b1"][:] = 0.0
    if xh:  # head output zero: the first evaluation starts PCG from x0 = 0
        P0["xdec.W1"][:] = 0.0
        P0["xdec.b1"][:] = 0.0
    if init is not None:
        P0.update({k: v for k, v in lpcg.unpack_params(init, h, n_mp).items() if xh or not k.startswith("xdec.")})
    params = lpcg.pack_params(P0, h, n_mp).cuda()
    grad_mask = None
    if args.head_only:
        grad_mask = torch.zeros_like(params)
        grad_mask[lpcg.param_count(h, n_mp, False):] = 1.0
    m1, v1 = torch.zeros_like(params), torch.zeros_like(params)
    ws = lpcg.gnn_workspace(S, h, n_mp, train=True)  # sized for the largest batch

    # held-out evaluation systems (unseen seeds, full size)
    held = []
    ric_its, rj_its = [], []
    for i in range(max(1, args.eval_systems)):
        if family == "heat3d":
            Ae, be = g.heat_system_3d(args.eval_m, 1e-3, k_seed=5000 + i, u0_seed=6000 + i)
        else:
            Ae, be, _ = g.fem_p1_delaunay(size, k_seed=5000 + i, f_seed=6000 + i)
        Se = lpcg.analyze(torch.as_tensor(Ae.rowptr).cuda(), torch.as_tensor(Ae.colind).cuda(),
                          torch.as_tensor(Ae.val).cuda(), None, order)
        bed = torch.as_tensor(be).cuda()
        lic, uic, _ = lpcg.ic0(Se)
        _, ric = lpcg.pcg_solve(Se, lpcg.PC_LLT, bed, l_val=lic, ut_val=uic, tol=1e-6, maxit=args.eval_maxit)
        _, rj = lpcg.pcg_solve(Se, lpcg.PC_JACOBI, bed, tol=1e-6, maxit=args.eval_maxit)
        ric_its.append(ric["iters"])
        rj_its.append(rj["iters"])
        held.append((Se, bed))
    Se = held[0][0]
    wse = lpcg.gnn_workspace(Se, h, n_mp)
    nl = Se.info["nnz_l"]
    le = torch.empty(nl, dtype=torch.float32, device="cuda")
    ue = torch.empty(nl, dtype=torch.float32, device="cuda")
    ric = {"iters": float(np.mean(ric_its))}
    rj = {"iters": float(np.mean(rj_its))}
    print(f"[train] held-out {len(held)} x n={Se.n} ({args.ordering} order, {Se.info['nlev_fwd']} levels): "
          f"IC(0) {ric_its} its, Jacobi {rj_its} its", flush=True)

    def evaluate(with_x0=xh, report=None):
        """Mean PCG iterations to 1e-6 over the held-out systems (10^6 if one fails)."""
        its = []
        for k, (Sk, bk) in enumerate(held):
            x0 = None
            if xh:
                _, _, x0 = lpcg.gnn_predict_x0(Sk, params, h, n_mp, bk, wse, le, ue, diag_mode=dm)
            else:
                lpcg.gnn_predict_L(Sk, params, h, n_mp, bk, wse, le, ue, diag_mode=dm)
            _, r, hist = lpcg.pcg_solve(Sk, lpcg.PC_LLT, bk, x=x0 if with_x0 else None, l_val=le, ut_val=ue,
                                        tol=1e-6, maxit=args.eval_maxit, hist=True)
            if report is not None and k == 0:  # first system: starting relative residual, then per tolerance
                hh = hist.cpu().numpy()
                report["start_relres"] = float(hh[0])
                report["iters_to"] = {f"1e-{e}": int(np.argmax(hh <= 10.0 ** -e)) if np.any(hh <= 10.0 ** -e)
                                      else None for e in range(1, 7)}
            its.append(r["iters"] if r["status"] == 0 else 10 ** 6)
        return float(np.mean(its)) if len(its) > 1 else its[0]

    log = {"loss": [], "eval": [], "ic0_iters": ric["iters"], "jacobi_iters": rj["iters"]}
    best = (evaluate(), 0, params.clone())
    log["eval"].append((0, best[0]))
    print(f"[train] step 0 held-out iters {best[0]}", flush=True)
    t0 = time.time()
    for step in range(1, args.steps + 1):
        if shared:
            idx = torch.as_tensor(rng.choice(args.nsys, args.batch, replace=False)).cuda()
            lpcg.update_values(S, dv[idx].reshape(-1).contiguous())
            bb = db[idx].reshape(-1).contiguous()
            xb = dx[idx].reshape(-1).contiguous()
        else:
            k = int(rng.integers(len(systems)))
            S, bb, xb = systems[k], bvec[k], xvec[k]
        L = lpcg.gnn_forward_train(S, params, h, n_mp, bb, ws, diag_mode=dm)
        if args.loss == "data":
            loss, dl = lpcg.llt_loss(S, L, xb, bb)
        else:
            loss, dl = lpcg.frob_loss(S, L)
        if xh:
            lx = lpcg.x0_loss(S, params, h, n_mp, ws, xb, weight=args.x_weight, diag_mode=dm)
            if args.head_only:
                loss, dl = lx, torch.zeros_like(dl)
            else:
                loss = loss + args.x_weight * lx
        grad = lpcg.gnn_backward(S, params, h, n_mp, ws, dl, diag_mode=dm)
        if grad_mask is not None:
            grad.mul_(grad_mask)
        lpcg.adam_step(params, grad, m1, v1, args.lr, step)
        if step % 10 == 0:
            log["loss"].append((step, float(loss.sum()) / args.batch))
        if step % args.eval_every == 0 or step == args.steps:
            it = evaluate()
            log["eval"].append((step, it))
            if it < best[0] or (args.head_only and step == args.steps):  # head-only keeps the last weights
                best = (it, step, params.clone())
            print(f"[train] step {step} loss/system {log['loss'][-1][1]:.4g} held-out iters {it} "
                  f"(best {best[0]} @ {best[1]}) {time.time() - t0:.1f}s", flush=True)
    if xh:
        params.copy_(best[2])
        log["from_x0"], log["from_zero"] = {}, {}
        evaluate(True, log["from_x0"])
        evaluate(False, log["from_zero"])
        print(f"[train] best network from its x0: {log['from_x0']}", flush=True)
        print(f"[train] best network from x = 0: {log['from_zero']}", flush=True)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.savez(args.out, params=best[2].cpu().numpy(), h=h, n_mp=n_mp, diag_mode=dm, ordering=order,
             best_step=best[1],
             best_iters=best[0], log=json.dumps(log), config=json.dumps(vars(args)))
    print(f"[train] saved {args.out}: best held-out iters {best[0]} at step {best[1]} "
          f"(IC(0) {ric['iters']}, Jacobi {rj['iters']})", flush=True)


if __name__ == "__main__":
    main()
