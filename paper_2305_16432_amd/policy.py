"""Host policy around the learned factor: learned L, then IC(0), then Jacobi.

The method's preconditioner P = L L^T is SPD only when every diagonal entry
of the predicted L is a positive finite number (Method: L Lᵀ is SPD by
construction when L is non-singular), and a network applied outside its
training distribution may give a poor or broken factor.  The solve
therefore falls back, in order:

  1. learned L (gnn_predict_L), accepted only if lpcg_check_factor passes,
     then PCG with it;
  2. IC(0) (the incomplete-Cholesky baseline of the Experiments section),
     whose pivot breakdown is retried inside the library on
     A + shift * diag(A) with a doubling shift;
  3. Jacobi (the diagonal baseline), which cannot break down on an SPD A.

A stage is abandoned when its factor is rejected, when PCG breaks down
(p^T A p <= 0 or non-finite) or when it reaches maxit without converging;
every stage starts again from x0.  The report names the stage that produced
x and why each earlier stage was left.

Every numerical step runs in the HIP library; this module only chooses
which entry points to call.  The backend is an argument so the policy can
be exercised with scripted outcomes; the default is the library itself."""
from __future__ import annotations

from dataclasses import dataclass, field

STAGES = ("learned", "ic0", "jacobi")


@dataclass
class SolveReport:
    stage: str = ""                 # stage whose x is returned ("" if none converged)
    status: int = -1                # library status of that stage's solve
    iters: int = 0
    relres_true: float = float("nan")
    shift: float = 0.0              # IC(0) diagonal shift used (ic0 stage)
    tried: list = field(default_factory=list)   # (stage, outcome) in order


class LibraryBackend:
    """The default backend: the HIP library through the ctypes binding."""

    def __init__(self):
        from . import lpcg
        self.L = lpcg

    def predict(self, S, net, b):
        import torch
        L = self.L
        ws = L.gnn_workspace(S, net["h"], net["n_mp"])
        nl = S.info["nnz_l"]
        l_val = torch.empty(nl, dtype=torch.float32, device="cuda")
        ut_val = torch.empty(nl, dtype=torch.float32, device="cuda")
        return L.gnn_predict_L(S, net["params"], net["h"], net["n_mp"], b, ws, l_val, ut_val,
                               diag_mode=net.get("diag_mode", 0))

    def check(self, S, l_val):
        return self.L.check_factor(S, l_val)

    def ic0(self, S, max_retries):
        try:
            l_val, ut_val, shift = self.L.ic0(S, max_retries=max_retries)
        except self.L.LpcgError as e:
            if e.code == self.L.EBREAKDOWN:
                return None
            raise
        return l_val, ut_val, shift

    def pcg(self, S, kind, b, l_val, ut_val, tol, maxit, max_restarts):
        L = self.L
        k = {"llt": L.PC_LLT, "jacobi": L.PC_JACOBI}[kind]
        return L.pcg_solve(S, k, b, l_val=l_val, ut_val=ut_val, tol=tol, maxit=maxit,
                           max_restarts=max_restarts)  # eager chunks: measured faster than graph replay


OK, ENOTCONV, EBREAKDOWN = 0, 3, 4


def solve(S, b, net=None, tol=1e-6, maxit=0, max_restarts=2, ic0_retries=8, backend=None):
    """PCG on the analysed system S for right-hand side b (device FP64) with
    the first preconditioner of learned L -> IC(0) -> Jacobi that works.
    net: None (skip the learned stage) or a dict with params (device FP32),
    h, n_mp and diag_mode.  Returns (x, SolveReport); x is the last stage's
    iterate if no stage converged (report.stage is then "")."""
    be = backend if backend is not None else LibraryBackend()
    rep = SolveReport()
    x = None

    def attempt(stage, kind, l_val, ut_val):
        nonlocal x
        xs, res = be.pcg(S, kind, b, l_val, ut_val, tol, maxit, max_restarts)
        x = xs
        st = res["status"]
        if st == OK:
            rep.stage, rep.status, rep.iters = stage, st, res["iters"]
            rep.relres_true = res["relres_true"]
            rep.tried.append((stage, "converged"))
            return True
        rep.status, rep.iters, rep.relres_true = st, res["iters"], res["relres_true"]
        rep.tried.append((stage, "breakdown" if st == EBREAKDOWN else "not converged"))
        return False

    if net is not None:
        l_val, ut_val = be.predict(S, net, b)
        ok, bad_row = be.check(S, l_val)
        if not ok:
            rep.tried.append(("learned", f"factor rejected at row {bad_row}"))
        elif attempt("learned", "llt", l_val, ut_val):
            return x, rep
    f = be.ic0(S, ic0_retries)
    if f is None:
        rep.tried.append(("ic0", "pivot breakdown after every shift"))
    else:
        l_val, ut_val, rep.shift = f
        if attempt("ic0", "llt", l_val, ut_val):
            return x, rep
    attempt("jacobi", "jacobi", None, None)
    return x, rep
