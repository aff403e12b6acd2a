"""Benchmark: time to relative residual 1e-6 and PCG iterations, learned-L vs
IC(0) (and Jacobi), on the 3D implicit-Euler heat step, 64^3 grid, 7-point
stencil, n = 262,144 (log-normal GRF conductivity, sigma = 1, dt = 1e-3).

A step is one pass of the hot path over one system: precompute the
preconditioner (GNN prediction of L, or the IC(0) factorisation, or the
Jacobi diagonal) and run PCG until ||r|| <= 1e-6 ||b|| with the FP64 true
residual checked.  The system, its pattern analysis and the network weights
are resident in HBM before the timed region.

Both row orderings of the library are measured: the natural one (the factor
on tril(A), as in the paper) and the multicolour one (red-black on this
grid; the factor on tril(P A P^T)), each with its own trained network.  The
headline value is learned-L in the natural ordering (the paper's setting),
compared with IC(0) in the same ordering; every method/ordering pair is in
"methods".

Prints one JSON line (see the end of main()).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# natural order: the network trained on 32^3 heat steps and fine-tuned on 64^3 ones
FEM_WEIGHTS = os.path.join(ROOT, "paper_2305_16432_amd", "weights", "fem2d_h64_mp5.npz")
WEIGHTS = {"natural": os.path.join(ROOT, "paper_2305_16432_amd", "weights", "heat3d_h32_mp3_ft64.npz"),
           "color": os.path.join(ROOT, "paper_2305_16432_amd", "weights", "heat3d_h32_mp1_color3.npz")}
PEAK_HBM = 8000.0  # GB/s, MI355X HBM3E
# HBM bytes of the roofline kernel measured with rocprofv3 --pmc FETCH_SIZE /
# WRITE_SIZE (scaled by the same counters on a copy of known size); valid
# only while the kernel source is the one that was profiled.
TRAFFIC = os.path.join(ROOT, "profiles", "pcg_parts_heat3d_64_traffic.json")


def measured_traffic(kernel):
    """HBM bytes per launch from the committed counter summary, or None when
    absent, for a kernel it does not list, or taken on different kernel
    sources (SHA-256 over the files it names)."""
    import hashlib
    if not os.path.exists(TRAFFIC):
        return None
    with open(TRAFFIC) as f:
        t = json.load(f)
    h = hashlib.sha256()
    for p in t.get("sources", []):
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    if t.get("source_sha256") != h.hexdigest() or kernel not in t.get("kernels", {}):
        return None
    return t["kernels"][kernel]["bytes_per_launch"]


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def hbm_bytes_sptrsv(info):
    """Algorithmic bytes of one substitution launch with FP32 values, int32
    indices: values + column indices (8 nnz_L), row pointers (4 (n+1)), the
    right-hand side and the result (8 n), the level-order row list (4 n)."""
    n, nl = info["n"], info["nnz_l"]
    return 8 * nl + 4 * (n + 1) + 8 * n + 4 * n


def hbm_bytes_pcg_parts(info, two_level, fused_xr=False):
    """Algorithmic bytes of the PCG iteration's three parts (FP32 vectors and
    values, int32 indices, FP64 x): the application z = (L L^T)^-1 r (two
    fused launches on a two-level system: L's values and indices in each
    half, r read twice, z written and read once; else the two substitutions),
    the SpMV w = A p with p = z + beta p_prev (A, z and p_prev read, p and w
    written), and the x, r update (x read and written in FP64, r read and
    written, p and w read).  fused_xr: the two-level pair performs the update
    (its bytes move to the application; no separate part)."""
    n, nnz, nl = info["n"], info["nnz"], info["nnz_l"]
    apply = 2 * (8 * nl + 4 * (n + 1)) + 16 * n if two_level else 2 * hbm_bytes_sptrsv(info)
    if fused_xr:
        return {"apply": apply + 32 * n, "spmv_p": 8 * nnz + 4 * (n + 1) + 16 * n}
    return {"apply": apply, "spmv_p": 8 * nnz + 4 * (n + 1) + 16 * n, "xr": 32 * n}


def hbm_bytes_spmv(info):
    """FP32 values + int32 columns (8 nnz), row pointers, x and y (8 n)."""
    n, nnz = info["n"], info["nnz"]
    return 8 * nnz + 4 * (n + 1) + 8 * n


def host_cpu_model():
    """The host CPU's model name (as lscpu prints it), from /proc/cpuinfo."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(A, b, tol, weights, budget_s=30.0):
    """The FP64 oracle on one host core, on the same 64^3 system in the
    natural ordering: learned L (NumPy FP64 network forward of the shipped
    natural-order weights, then the serial C PCG), IC(0) (serial C
    factorisation + PCG) and Jacobi (serial C PCG).  The learned leg runs
    once (its forward is the bulk of the sample); IC(0) and Jacobi up to 3
    times within the remaining budget.  value = the learned leg's time to
    tol (the metric's method), ms."""
    from threadpoolctl import threadpool_limits

    import oracle as O
    from oracle import gnn as ognn
    from pdegen.weights import gnn_param_shapes
    pat = O.Pattern(A)
    out = {}
    t_start = time.perf_counter()
    with threadpool_limits(1):
        if os.path.exists(weights):
            W = np.load(weights)
            h, n_mp, dm = int(W["h"]), int(W["n_mp"]), int(W["diag_mode"])
            flat, P, off = W["params"].astype(np.float64), {}, 0
            for name, shp in gnn_param_shapes(h, n_mp):
                k = int(np.prod(shp))
                P[name] = flat[off:off + k].reshape(shp)
                off += k
            t0 = time.perf_counter()
            lval, _ = ognn.forward(A, b, P, h, n_mp, rev=pat.rev, diag_mode=dm)
            t1 = time.perf_counter()
            res = O.pcg(A, b, O.PC_LLT, pat, lval, tol=tol)
            t2 = time.perf_counter()
            out["learned"] = dict(ms=(t2 - t0) * 1e3, precompute_ms=(t1 - t0) * 1e3, iters=res["iters"], runs=1)
        for name in ("ic0", "jacobi"):
            times, iters = [], None
            while len(times) < 3 and (not times or time.perf_counter() - t_start < budget_s):
                t0 = time.perf_counter()
                if name == "ic0":
                    lval, st = O.ic0(pat, A)
                    res = O.pcg(A, b, O.PC_LLT, pat, lval, tol=tol)
                else:
                    res = O.pcg(A, b, O.PC_JACOBI, tol=tol)
                times.append((time.perf_counter() - t0) * 1e3)
                iters = res["iters"]
            out[name] = dict(ms=float(np.mean(times)), iters=iters, runs=len(times))
    head = "learned" if "learned" in out else "ic0"
    return {"value": out[head]["ms"], "unit": "ms", "cores": 1, "kind": "oracle",
            "sample": f"{head} on the full 64^3 system to {tol:g}, natural order, FP64 on one core "
                      f"(NumPy network forward, serial C factorisation and PCG); IC(0) and Jacobi beside it "
                      f"in 'methods'",
            "methods": out, "host": host_cpu_model(), "host_cpus": os.cpu_count()}


PEAK_BF16_TFLOPS = 2500.0  # MI355X dense BF16 MFMA


def gnn_model(n, nnz, nnz_l, h, n_mp):
    """Algorithmic flops and HBM bytes of one network forward (factored first
    edge layer; BF16 latents, FP32 decoder output and factor; weights and
    index reads of the CSR row pointers neglected)."""
    hh = 2 * h * h
    flops = n * (2 * h + hh) + nnz * (2 * h + hh)                       # encoders
    flops += n_mp * (nnz * 2 * h + n * (2 * hh + hh) + n * 2 * hh + nnz * 2 * hh)  # aggregation, node MLP,
    flops += nnz * (hh + 2 * h)                                           # projections, edge MLP; decoder
    lat = 2 * h                                                           # bytes per BF16 latent row
    byts = n * (8 + lat) + nnz * (8 + 4 + lat)                            # encoders: b, A values, rows
    for t in range(n_mp):
        byts += n * lat + nnz * (lat + 4) + 3 * n * lat                   # node kernel: V, E, col; V', Pa, Pb
        byts += nnz * (lat + 8) + 2 * n * lat + (4 * nnz if t == n_mp - 1 else nnz * lat)  # edge kernel
    byts += nnz * 4 + nnz_l * 8                                           # assembly: d, L and U values
    return float(flops), float(byts)


def methods_learned(ordering, code, S):
    """(params, h, n_mp, diag_mode, workspace) of the shipped network for an
    ordering, or None."""
    import torch
    from paper_2305_16432_amd import lpcg
    if not os.path.exists(WEIGHTS[ordering]):
        return None
    W = np.load(WEIGHTS[ordering])
    if int(W["ordering"]) != code:
        return None
    h, n_mp, dmode = int(W["h"]), int(W["n_mp"]), int(W["diag_mode"])
    params = torch.as_tensor(W["params"].astype(np.float32)).cuda()
    return params, h, n_mp, dmode, lpcg.gnn_workspace(S, h, n_mp, train=False)


def run_seeds(args, S, lval, utval, x, coef, solve_kw, net):
    """Every test seed (same pattern, new values): precompute + PCG time
    (fastest of 3) and iterations of learned L, IC(0), symmetric
    Gauss-Seidel and Jacobi, with their means (outside the timed steps)."""
    import torch
    import pdegen as g
    from paper_2305_16432_amd import lpcg
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    dinv = torch.empty(S.n, dtype=torch.float32, device="cuda")
    rows = []
    for i in range(args.seeds):
        ks, us = args.k_seed + i, args.u_seed + i
        Ai, bi = g.heat_system_3d(args.m, 1e-3, ks, us)
        lpcg.update_values(S, torch.as_tensor(Ai.val).cuda())
        bdi = torch.as_tensor(bi).cuda()
        row = {"k_seed": ks, "u0_seed": us}
        pres = {"ic0": (lambda: lpcg.ic0(S, 0.0, 8, lval, utval), lpcg.PC_LLT),
                "sgs": (lambda: lpcg.sgs(S, lval, utval), lpcg.PC_LLT),
                "jacobi": (lambda: lpcg.jacobi(S, dinv), lpcg.PC_JACOBI)}
        if net is not None:
            params, h, n_mp, dmode, ws = net
            pres["learned"] = (lambda: lpcg.gnn_predict_L(S, params, h, n_mp, bdi, ws, lval, utval,
                                                          diag_mode=dmode), lpcg.PC_LLT)
        for name, (pre, kind) in pres.items():
            for _ in range(3):
                e0.record()
                pre()
                e1.record()
                x.zero_()
                _, res = lpcg.pcg_solve(S, kind, bdi, x=x, l_val=lval, ut_val=utval, dinv=dinv, coef=coef,
                                        **solve_kw)
                e2.record()
                torch.cuda.synchronize()
                if name not in row or e0.elapsed_time(e2) < row[name]["ms"]:
                    row[name] = dict(ms=e0.elapsed_time(e2), precompute_ms=e0.elapsed_time(e1),
                                     iters=res["iters"], relres_true=res["relres_true"], status=res["status"])
        rows.append(row)
        _log(f"seed {ks}/{us}: " + ", ".join(f"{k} {v['iters']} it {v['ms']:.2f} ms" for k, v in row.items()
                                               if isinstance(v, dict)))
    summary = {"per_seed": rows}
    for name in ("learned", "ic0", "sgs", "jacobi"):
        if all(name in r for r in rows):
            summary[name] = dict(ms_mean=float(np.mean([r[name]["ms"] for r in rows])),
                                 iters_mean=float(np.mean([r[name]["iters"] for r in rows])),
                                 iters_max=int(np.max([r[name]["iters"] for r in rows])),
                                 all_converged=all(r[name]["status"] == 0 for r in rows))
    if "learned" in summary:
        summary["learned_faster_than_ic0"] = sum(r["learned"]["ms"] < r["ic0"]["ms"] for r in rows)
        summary["learned_faster_than_jacobi"] = sum(r["learned"]["ms"] < r["jacobi"]["ms"] for r in rows)
    return summary


def run_c1(args, weights):
    """The 2D FEM workload: P1 FEM on a Delaunay triangulation of a 128 x 128
    jittered point grid (k = exp(GRF sigma=1, ell=0.1) per triangle, lumped
    load of f ~ N(0,1); k seed 1000, f seed 2000, n = 15,876 after the
    boundary), PCG to 1e-6 with the FP64 check: learned L from the 2D network
    (h = 64, five message-passing layers, softplus diagonal), IC(0) and
    Jacobi in the natural order, IC(0) in the colour order; the paper's
    protocol (12 runs, mean of the fastest 5)."""
    import torch

    import pdegen as g
    from paper_2305_16432_amd import lpcg
    A, b, _ = g.fem_p1_delaunay(128, k_seed=1000, f_seed=2000)
    bd = torch.as_tensor(b).cuda()
    x = torch.zeros_like(bd)
    out = {"workload": f"2D P1 FEM on a jittered 128x128 Delaunay grid, n={A.n}, nnz={A.nnz}, "
                       f"k=exp(GRF sigma=1, ell=0.1), k seed 1000, f seed 2000, tol=1e-06"}
    for ordering, code in (("natural", lpcg.ORDER_NATURAL), ("color", lpcg.ORDER_COLOR)):
        S = lpcg.analyze(torch.as_tensor(A.rowptr).cuda(), torch.as_tensor(A.colind).cuda(),
                         torch.as_tensor(A.val).cuda(), None, code)
        nl = S.info["nnz_l"]
        lval = torch.empty(nl, dtype=torch.float32, device="cuda")
        utval = torch.empty(nl, dtype=torch.float32, device="cuda")
        dinv = torch.empty(A.n, dtype=torch.float32, device="cuda")
        lpcg.ic0(S, 0.0, 8, lval, utval)
        lpcg.autotune(S, lval, utval, reps=3)
        meth = {"ic0": (lambda: lpcg.ic0(S, 0.0, 8, lval, utval), lpcg.PC_LLT)}
        if ordering == "natural":
            meth["jacobi"] = (lambda: lpcg.jacobi(S, dinv), lpcg.PC_JACOBI)
            if os.path.exists(weights):
                W = np.load(weights)
                h, n_mp, dmode = int(W["h"]), int(W["n_mp"]), int(W["diag_mode"])
                params = torch.as_tensor(W["params"].astype(np.float32)).cuda()
                ws = lpcg.gnn_workspace(S, h, n_mp, train=False)
                meth["learned"] = (lambda: lpcg.gnn_predict_L(S, params, h, n_mp, bd, ws, lval, utval,
                                                              diag_mode=dmode), lpcg.PC_LLT)
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        for name, (pre, kind) in meth.items():
            tot, prem, its = [], [], []
            for k in range(args.warmup + args.steps):
                e0.record()
                pre()
                e1.record()
                x.zero_()
                _, res = lpcg.pcg_solve(S, kind, bd, x=x, l_val=lval, ut_val=utval, dinv=dinv, tol=1e-6,
                                        check_every=0, max_restarts=2, use_graph=False)
                e2.record()
                torch.cuda.synchronize()
                if k >= args.warmup:
                    tot.append(e0.elapsed_time(e2))
                    prem.append(e0.elapsed_time(e1))
                    its.append(res["iters"])
            fast = np.argsort(tot)[:min(5, len(tot))]
            key = name if ordering == "natural" else f"{name}_{ordering}"
            out[key] = dict(ms=float(np.mean(np.array(tot)[fast])),
                            precompute_ms=float(np.mean(np.array(prem)[fast])), iters=int(np.max(its)),
                            relres_true=res["relres_true"], status=res["status"], levels=S.info["nlev_fwd"])
            _log(f"c1 {key}: {out[key]}")
        del S
    return out


def run_c4(args, weights):
    """The batched workload: 256 independent systems with sizes log-uniform in
    [2k, 200k] (half 2D P1 FEM, half 3D heat steps; seed 9), one block-diagonal
    analysis (natural order), FP64 iterative refinement over the batched FP32
    PCG (inner tolerance 1e-4) until every system reaches ||b - A x|| <=
    1e-10 ||b||.  A run = precompute (IC(0) of the whole batch, or the network
    on the whole batch) + the refinement solve, timed with events; one warm-up,
    then 3 runs (mean of the fastest 2).  Algorithmic bytes: per inner
    iteration of system i, 8 nnz_i + 12 n_i (SpMV) + 2 (8 nnz_L,i + 12 n_i)
    (substitutions) + 56 n_i (vector passes); per refinement step, the FP64
    residual 12 nnz_i + 24 n_i."""
    import torch

    import pdegen as g
    from paper_2305_16432_amd import lpcg
    t0 = time.perf_counter()
    sysl = g.mixed_batch_parallel(256, 2000, 200000, 9, workers=16)
    mats = [A for A, _ in sysl]
    B, srp = g.block_diag_csr(mats)
    b = np.concatenate([bb for _, bb in sysl])
    _log(f"c4: {len(mats)} systems, n={B.n}, nnz={B.nnz} generated in {time.perf_counter() - t0:.1f}s")
    S = lpcg.analyze(torch.as_tensor(B.rowptr).cuda(), torch.as_tensor(B.colind).cuda(),
                     torch.as_tensor(B.val).cuda(), srp, lpcg.ORDER_NATURAL)
    nl = S.info["nnz_l"]
    lval = torch.empty(nl, dtype=torch.float32, device="cuda")
    utval = torch.empty(nl, dtype=torch.float32, device="cuda")
    lpcg.ic0(S, 0.0, 8, lval, utval)
    lpcg.autotune(S, lval, utval, reps=2)
    bd = torch.as_tensor(b).cuda()
    x = torch.zeros_like(bd)
    ns = np.diff(srp)
    nnzs = np.array([A.nnz for A in mats])
    nnzl = (nnzs - ns) // 2 + ns
    per_it = 8 * nnzs + 12 * ns + 2 * (8 * nnzl + 12 * ns) + 56 * ns
    pres = {"ic0": lambda: lpcg.ic0(S, 0.0, 8, lval, utval)}
    if os.path.exists(weights):
        W = np.load(weights)
        h, n_mp, dmode = int(W["h"]), int(W["n_mp"]), int(W["diag_mode"])
        params = torch.as_tensor(W["params"].astype(np.float32)).cuda()
        ws = lpcg.gnn_workspace(S, h, n_mp, train=False)
        pres["learned"] = lambda: lpcg.gnn_predict_L(S, params, h, n_mp, bd, ws, lval, utval, diag_mode=dmode)
    out = {"workload": f"256 systems, sizes log-uniform in [2000, 200000] (half 2D P1 FEM, half 3D heat "
                       f"steps, seed 9), n={B.n}, nnz={B.nnz}; FP64 refinement to 1e-10 over FP32 PCG "
                       f"(inner tol 1e-4), natural order",
           "trsv_cfg": [lpcg.get_trsv_cfg(S, d) for d in (0, 1)], "spmv_cfg": lpcg.get_trsv_cfg(S, 2)}
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    for name, pre in pres.items():
        runs = []
        for k in range(4):
            e0.record()
            pre()
            e1.record()
            x.zero_()
            _, res = lpcg.pcg_solve_ir(S, lpcg.PC_LLT, bd, x=x, l_val=lval, ut_val=utval, tol=1e-10,
                                       tol_inner=1e-4, max_outer=20, maxit=5000, use_graph=True)
            e2.record()
            torch.cuda.synchronize()
            if k > 0:
                runs.append((e0.elapsed_time(e2), e0.elapsed_time(e1), res))
        runs.sort(key=lambda r: r[0])
        ms = float(np.mean([r[0] for r in runs[:2]]))
        res = runs[0][2]
        its = np.array([r["iters"] for r in res])
        steps = np.array([r["restarts"] for r in res])
        ok = all(r["status"] == 0 for r in res)
        byts = float(np.sum(its * per_it) + np.sum((steps + 1) * (12 * nnzs + 24 * ns)))
        out[name] = dict(ms=ms, precompute_ms=float(np.mean([r[1] for r in runs[:2]])), all_converged=ok,
                         inner_iters=dict(min=int(its.min()), median=float(np.median(its)), max=int(its.max()),
                                          sum=int(its.sum())),
                         refinement_steps_max=int(steps.max()), algorithmic_gb=byts / 1e9,
                         gbs=byts / (ms * 1e-3) / 1e9)
        _log(f"c4 {name}: {out[name]}")
    del S
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=12)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--m", type=int, default=64)
    ap.add_argument("--k-seed", type=int, default=1000)
    ap.add_argument("--u-seed", type=int, default=2000)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-c4", action="store_true", help="skip the batched 256-system workload")
    ap.add_argument("--no-c1", action="store_true", help="skip the 2D FEM workload")
    ap.add_argument("--orderings", default="natural,color")
    ap.add_argument("--methods", default="learned,ic0,sgs,jacobi")
    ap.add_argument("--seeds", type=int, default=10,
                    help="test seeds (k seed, u0 seed) + 0..seeds-1 run once per method after the timed steps")
    ap.add_argument("--no-tolerances", action="store_true",
                    help="skip the time-to-tolerance sweep (1e-2 .. 1e-10) per method and ordering")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="MiB of a plain device copy to run first (counter calibration under rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU; --gpus {args.gpus} is not supported "
              "(the solver does not shard a system across GPUs)", file=sys.stderr)
        sys.exit(2)

    import torch

    import pdegen as g
    from paper_2305_16432_amd import lpcg

    torch.cuda.set_device(0)
    if args.calibrate_copy > 0:  # a copy of known size: reads and writes calibrate_copy MiB each
        src = torch.ones(args.calibrate_copy * 2 ** 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        _log(f"calibration copy of {args.calibrate_copy} MiB done")
        del src, dst
    A, b = g.heat_system_3d(args.m, 1e-3, args.k_seed, args.u_seed)
    _log(f"system n={A.n} nnz={A.nnz}")
    bd = torch.as_tensor(b).cuda()
    x = torch.zeros_like(bd)
    # eager chunks of 8 iterations: on MI355X these measured faster than
    # replaying the same chunk as a captured graph (red-black IC(0) at 64^3:
    # 2.29 against 2.40 ms; Jacobi 2.72 against 2.79 ms); the graph path is
    # kept in the library (use_graph) and tested
    solve_kw = dict(tol=args.tol, check_every=0, max_restarts=2, use_graph=False)
    results, kernels, per_seed = {}, {}, {}
    gnn_dims = None
    for ordering in args.orderings.split(","):
        code = lpcg.ORDER_COLOR if ordering == "color" else lpcg.ORDER_NATURAL
        S = lpcg.analyze(torch.as_tensor(A.rowptr).cuda(), torch.as_tensor(A.colind).cuda(),
                         torch.as_tensor(A.val).cuda(), None, code)
        info = S.info
        _log(f"{ordering}: {info['nlev_fwd']} forward levels, {info['ncolors']} colours")
        nl = info["nnz_l"]
        lval = torch.empty(nl, dtype=torch.float32, device="cuda")
        utval = torch.empty(nl, dtype=torch.float32, device="cuda")
        dinv = torch.empty(A.n, dtype=torch.float32, device="cuda")

        def run_ic0():
            lpcg.ic0(S, 0.0, 8, lval, utval)

        maxit = A.n
        coef = torch.zeros(2 * (maxit + 1), dtype=torch.float64, device="cuda")

        def solve_llt():
            x.zero_()
            return lpcg.pcg_solve(S, lpcg.PC_LLT, bd, x=x, l_val=lval, ut_val=utval, coef=coef, **solve_kw)[1]

        def run_jacobi():
            lpcg.jacobi(S, dinv)

        def run_sgs():
            lpcg.sgs(S, lval, utval)

        def solve_jacobi():
            x.zero_()
            return lpcg.pcg_solve(S, lpcg.PC_JACOBI, bd, x=x, dinv=dinv, coef=coef, **solve_kw)[1]

        # per-pattern tuning of the substitution kernels (like the analysis,
        # done once per sparsity pattern, outside the timed region)
        lpcg.ic0(S, 0.0, 8, lval, utval)
        tune = lpcg.autotune(S, lval, utval, reps=3)
        cfg = [lpcg.get_trsv_cfg(S, d) for d in (0, 1)]
        _log(f"{ordering}: substitution configuration {cfg} ({len(tune)} candidates timed)")

        methods = {"ic0": (run_ic0, solve_llt)}
        if ordering == "natural":
            methods["jacobi"] = (run_jacobi, solve_jacobi)  # the same preconditioner in any order
        methods["sgs"] = (run_sgs, solve_llt)  # on this ordering's pattern
        if os.path.exists(WEIGHTS[ordering]):
            W = np.load(WEIGHTS[ordering])
            assert int(W["ordering"]) == code, "network trained for another ordering"
            h, n_mp, dmode = int(W["h"]), int(W["n_mp"]), int(W["diag_mode"])
            params = torch.as_tensor(W["params"].astype(np.float32)).cuda()
            ws = lpcg.gnn_workspace(S, h, n_mp, train=False)

            if ordering == "natural":
                gnn_dims = (A.n, A.nnz, info["nnz_l"], h, n_mp)

            def run_learned(params=params, h=h, n_mp=n_mp, dmode=dmode, ws=ws):
                lpcg.gnn_predict_L(S, params, h, n_mp, bd, ws, lval, utval, diag_mode=dmode)
            methods["learned"] = (run_learned, solve_llt)
        for name in [m for m in ("learned", "ic0", "sgs", "jacobi") if m in methods and m in args.methods]:
            pre, solve = methods[name]
            for _ in range(args.warmup):
                pre()
                solve()
            torch.cuda.synchronize()
            t_pre, t_solve, iters, relres = [], [], [], []
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            wall0 = time.perf_counter()
            for _ in range(args.steps):
                e0.record()
                pre()
                e1.record()
                res = solve()
                e2.record()
                torch.cuda.synchronize()
                t_pre.append(e0.elapsed_time(e1))
                t_solve.append(e1.elapsed_time(e2))
                iters.append(res["iters"])
                relres.append(res["relres_true"])
            torch.cuda.synchronize()
            wall = (time.perf_counter() - wall0) * 1e3 / args.steps
            key = name if ordering == "natural" else f"{name}_{ordering}"
            # condition number of the preconditioned operator (Lanczos, from the
            # coefficients of one more solve without restarts; outside the
            # timed region)
            solve_kw["max_restarts"] = 0
            r0 = solve()
            solve_kw["max_restarts"] = 2
            lmin, lmax = lpcg.lanczos_extremes(coef, r0["iters"]) if r0["iters"] > 0 else (None, None)
            # the paper's protocol (training-setup appendix): of the timed runs
            # (12 by default), the mean of the fastest 5
            tot = np.array(t_pre) + np.array(t_solve)
            fast = np.argsort(tot)[:min(5, len(tot))]
            results[key] = dict(ms=float(np.mean(tot[fast])), mean_all_ms=float(np.mean(tot)),
                                precompute_ms=float(np.mean(np.array(t_pre)[fast])),
                                solve_ms=float(np.mean(np.array(t_solve)[fast])),
                                wall_ms=wall, iters=int(np.max(iters)), relres_true=float(np.max(relres)),
                                status=res["status"], ordering=ordering,
                                kappa_lanczos=(lmax / lmin) if lmin else None,
                                us_per_iter=float(np.mean(np.array(t_solve)[fast])) * 1e3 / max(1, int(np.max(iters))))
            _log(f"{key}: {results[key]}")
            # the layout of the paper's PCG table: precompute + PCG to each
            # tolerance (FP64 true residual; FP64 restarts past the FP32
            # iteration's own accuracy), fastest of 3, outside the timed steps
            if not args.no_tolerances:
                sweep = {}
                for tol in (1e-2, 1e-4, 1e-6, 1e-8, 1e-10):
                    solve_kw["tol"], solve_kw["max_restarts"] = tol, 4
                    best_t = None
                    for _ in range(3):
                        e0.record()
                        pre()
                        r = solve()
                        e1.record()
                        torch.cuda.synchronize()
                        if best_t is None or e0.elapsed_time(e1) < best_t:
                            best_t = e0.elapsed_time(e1)
                            sweep[f"{tol:g}"] = dict(ms=best_t, iters=r["iters"], restarts=r["restarts"],
                                                     relres_true=r["relres_true"],
                                                     converged=r["status"] == 0)
                solve_kw["tol"], solve_kw["max_restarts"] = args.tol, 2
                results[key]["tolerances"] = sweep
                _log(f"{key} tolerances: " + ", ".join(f"{t}: {v['ms']:.2f} ms ({v['iters']})"
                                                       for t, v in sweep.items()))
        # kernel timings in this ordering (HIP events around each launch on its stream)
        lpcg.ic0(S, 0.0, 8, lval, utval)
        rhs = torch.as_tensor(b.astype(np.float32)).cuda()
        ms_f = lpcg.time_sptrsv(S, False, lval, utval, rhs, reps=50)
        ms_b = lpcg.time_sptrsv(S, True, lval, utval, rhs, reps=50)
        ms_spmv = lpcg.time_spmv(S, rhs, reps=100)
        bt, bs = hbm_bytes_sptrsv(info), hbm_bytes_spmv(info)
        # the PCG iteration's own kernels, timed live (HIP events between
        # its three parts, launched on this stream)
        parts_us = lpcg.time_pcg_kernels(S, lpcg.PC_LLT, bd, l_val=lval, ut_val=utval, reps=50)
        two_level = info["nlev_fwd"] == 2 and cfg[0]["mode"] == 1 and cfg[1]["mode"] == 1
        fused_xr = two_level and parts_us[2] == 0.0  # the pair's ELL form takes the x, r update
        pb = hbm_bytes_pcg_parts(info, two_level, fused_xr)
        parts = {k: dict(us=u, bytes=pb[k], gbs=pb[k] / (u * 1e-6) / 1e9)
                 for k, u in zip(("apply", "spmv_p", "xr"), parts_us) if k in pb}
        kernels[ordering] = dict(
            levels=info["nlev_fwd"], trsv_cfg=cfg, spmv_cfg=lpcg.get_trsv_cfg(S, 2), pcg_parts=parts,
            apply_form=("two-level pair with the x, r update" if fused_xr else "two-level pair") if two_level
            else "two substitutions",
            sptrsv_fwd=dict(us=ms_f * 1e3, bytes=bt, gbs=bt / (ms_f * 1e-3) / 1e9),
            sptrsv_bwd=dict(us=ms_b * 1e3, bytes=bt, gbs=bt / (ms_b * 1e-3) / 1e9),
            spmv=dict(us=ms_spmv * 1e3, bytes=bs, gbs=bs / (ms_spmv * 1e-3) / 1e9))
        _log(f"{ordering} kernels: {kernels[ordering]}")
        if args.seeds > 0:
            per_seed[ordering] = run_seeds(args, S, lval, utval, x, coef, solve_kw,
                                           methods_learned(ordering, code, S))
        del S

    # the network forward (the learned method's precompute) against the
    # BF16 MFMA and HBM peaks, from the flop and byte model above
    gnn_info = None
    if "learned" in results and gnn_dims is not None:
        gf, gb = gnn_model(*gnn_dims)
        t = results["learned"]["precompute_ms"] * 1e-3
        gnn_info = dict(ms=t * 1e3, gflop=gf / 1e9, tflops=gf / t / 1e12, mfma_frac=gf / t / 1e12 / PEAK_BF16_TFLOPS,
                        hbm_mb=gb / 1e6, gbs=gb / t / 1e9, hbm_frac=gb / t / 1e9 / PEAK_HBM,
                        h=gnn_dims[3], n_mp=gnn_dims[4])
    c1 = None if args.no_c1 else run_c1(args, FEM_WEIGHTS)
    c4 = None if args.no_c4 else run_c4(args, WEIGHTS["natural"])
    cpu = None
    if not args.no_cpu:
        os.environ.setdefault("OMP_NUM_THREADS", "1")
        cpu = cpu_baseline(A, b, args.tol, WEIGHTS["natural"])

    # headline: the fastest learned-L configuration over the orderings
    # measured (else the fastest IC(0)); beside it the fastest IC(0) and the
    # Jacobi result of the same run
    def best(prefix):
        keys = [k for k in results if k == prefix or k.startswith(prefix + "_")]
        return min(keys, key=lambda k: results[k]["ms"]) if keys else None

    def brief(k):
        if k is None:
            return None
        r = results[k]
        return dict(key=k, ms=r["ms"], precompute_ms=r["precompute_ms"], solve_ms=r["solve_ms"],
                    iters=r["iters"], ordering=r["ordering"])
    head = best("learned") or best("ic0")
    head_order = results[head]["ordering"]
    # roofline: the iteration part that takes the most time per iteration in
    # the value's ordering (measured live above)
    parts = kernels[head_order]["pcg_parts"]
    dom = max(parts, key=lambda k: parts[k]["us"])
    kf = parts[dom]
    dom_name = {"apply": f"L L^T application ({kernels[head_order]['apply_form']}, {head_order} order)",
                "spmv_p": f"k_spmv_pw: p = z + beta p_prev, w = A p, p.w ({head_order} order)",
                "xr": f"k_xr: x += alpha p, r -= alpha w, ||r||^2 ({head_order} order)"}[dom]
    ic0_same = "ic0" if head_order == "natural" else f"ic0_{head_order}"
    out = {
        "metric": "time-to-1e-6 rel. residual (ms) + PCG iters: learned-L vs IC(0), 3D 64³",
        "value": results[head]["ms"],
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": results[head]["ms"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (apply) / f64 (dots, true residual)",
        "data": "synthetic",
        "config": {"workload": f"3D implicit-Euler heat step, {args.m}^3 grid, 7-point, n={A.n}, "
                               f"k=exp(GRF sigma=1, ell=0.1), dt=1e-3, b=u0 GRF, tol={args.tol:g}",
                   "method_of_value": head, "ordering_of_value": head_order,
                   "iters_of_value": results[head]["iters"],
                   "ic0_same_ordering_ms": results.get(ic0_same, {}).get("ms"),
                   "ic0_same_ordering_iters": results.get(ic0_same, {}).get("iters"),
                   "best_learned": brief(best("learned")), "best_ic0": brief(best("ic0")),
                   "best_jacobi": brief(best("jacobi")), "best_sgs": brief(best("sgs")),
                   "timing": "12 timed runs per method after warm-up; value = mean of the fastest 5 "
                             "(the paper's protocol); mean_all_ms per method beside it",
                   "k_seed": args.k_seed, "u0_seed": args.u_seed},
        "methods": results,
        "roofline": {"bound": "hbm", "kernel": dom_name,
                     "achieved": kf["gbs"], "peak": PEAK_HBM, "unit": "GB/s", "frac": kf["gbs"] / PEAK_HBM,
                     "traffic": measured_traffic(dom_name), "bytes_per_launch": kf["bytes"], "us_per_launch": kf["us"],
                     "levels": kernels[head_order]["levels"], "kernels": kernels},
        "cpu_baseline": cpu,
        "seeds": per_seed if args.seeds > 0 else None,
        "gnn": gnn_info,
        "c1": c1,
        "c4": c4,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
