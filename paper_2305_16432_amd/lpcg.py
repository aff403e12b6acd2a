"""Thin Python binding of liblpcg.so (argument marshalling only).

Every function maps one-to-one onto the C entry point of the same name with
the `lpcg_` prefix (include/lpcg.h).  Tensors are torch CUDA tensors; the
library receives their device pointers and torch's current HIP stream.  No
computation of the method happens here, and there is no fallback: if the
shared library is missing or a call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblpcg.so")

OK, EINVAL, EHIP, ENOTCONV, EBREAKDOWN, ENONFINITE, ENOMEM = range(7)
PC_NONE, PC_JACOBI, PC_LLT = 0, 1, 2
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "EHIP", 3: "ENOTCONV", 4: "EBREAKDOWN",
                5: "ENONFINITE", 6: "ENOMEM"}


class LpcgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class _CSR(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int32), ("rowptr", C.c_void_p),
                ("colind", C.c_void_p), ("val", C.c_void_p)]


class _Info(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int32), ("nnz_l", C.c_int32),
                ("nlev_fwd", C.c_int32), ("nlev_bwd", C.c_int32),
                ("max_width_fwd", C.c_int32), ("max_width_bwd", C.c_int32),
                ("nsys", C.c_int32), ("ordering", C.c_int32), ("ncolors", C.c_int32)]


class _Precond(C.Structure):
    _fields_ = [("kind", C.c_int32), ("l_val", C.c_void_p), ("ut_val", C.c_void_p),
                ("dinv", C.c_void_p)]


class _Opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int32), ("check_every", C.c_int32),
                ("max_restarts", C.c_int32), ("use_graph", C.c_int32)]


class _Result(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("restarts", C.c_int32),
                ("reserved", C.c_int32), ("relres_rec", C.c_double), ("relres_true", C.c_double)]


class _TrsvCfg(C.Structure):
    _fields_ = [("direction", C.c_int32), ("mode", C.c_int32), ("waves", C.c_int32),
                ("backoff", C.c_int32), ("block_stride", C.c_int32), ("block_rows", C.c_int32),
                ("us", C.c_double), ("block_runs", C.c_int32)]


class _BlkSchedule(C.Structure):
    _fields_ = [("deps", C.c_int32), ("nblocks", C.c_int32), ("nchunks", C.c_int32), ("max_chunks", C.c_int32),
                ("brow", C.c_void_p), ("bch", C.c_void_p), ("chunks", C.c_void_p), ("rec", C.c_void_p),
                ("vsrc", C.c_void_p), ("run_shift", C.c_int32), ("run_stride", C.c_int32)]


class _Gnn(C.Structure):
    _fields_ = [("h", C.c_int32), ("n_mp", C.c_int32), ("params", C.c_void_p), ("diag_mode", C.c_int32),
                ("x_head", C.c_int32)]


_lib = None


def lib():
    """The loaded shared library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        L.lpcg_last_error.restype = C.c_char_p
        L.lpcg_version.restype = C.c_char_p
        if hasattr(L, "lpcg_gnn_param_count"):
            L.lpcg_gnn_param_count.restype = C.c_int64
            L.lpcg_gnn_param_count.argtypes = [C.c_int32, C.c_int32, C.c_int32]
            L.lpcg_gnn_workspace_bytes.restype = C.c_int64
            L.lpcg_gnn_workspace_bytes.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32]
        L.lpcg_destroy.restype = None
        _lib = L
    return _lib


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return C.c_void_p(t.data_ptr())


def _check(rc, what):
    if rc != OK:
        raise LpcgError(rc, f"{what}: {lib().lpcg_last_error().decode()}")


def _dev(t, dtype):
    t = torch.as_tensor(t)
    if t.dtype != dtype:
        raise TypeError(f"{dtype} expected, got {t.dtype}")
    return t if t.is_cuda else t.cuda()


class System:
    """Owns an lpcg_system handle (pattern analysis + values + work vectors)."""

    def __init__(self, handle, n, nnz):
        self._h = handle
        self.n, self.nnz = n, nnz
        self.info = get_info(self)

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("system destroyed")
        return self._h

    def close(self):
        if self._h is not None:
            torch.cuda.synchronize()
            lib().lpcg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ analysis
ORDER_NATURAL, ORDER_COLOR = 0, 1
COLOR_MAX_ROWS = 262144  # rows (whole batch) the colour ordering accepts


def analyze(rowptr, colind, val, sys_rowptr=None, ordering: int = ORDER_NATURAL) -> System:
    rowptr = _dev(rowptr, torch.int32).contiguous()
    colind = _dev(colind, torch.int32).contiguous()
    val = _dev(val, torch.float64).contiguous()
    n = rowptr.numel() - 1
    A = _CSR(n, colind.numel(), _ptr(rowptr), _ptr(colind), _ptr(val))
    out = C.c_void_p()
    if sys_rowptr is not None:
        import numpy as np
        sr = np.ascontiguousarray(sys_rowptr, dtype=np.int32)
        nsys = sr.shape[0] - 1
        srp = sr.ctypes.data_as(C.c_void_p)
    else:
        nsys, srp = 1, None
    rc = lib().lpcg_analyze(C.byref(A), srp, C.c_int32(nsys), C.c_int32(ordering), C.byref(out), _stream())
    _check(rc, "lpcg_analyze")
    return System(out, n, colind.numel())


def update_values(sys: System, val):
    val = _dev(val, torch.float64).contiguous()
    _check(lib().lpcg_update_values(sys.handle, _ptr(val), _stream()), "lpcg_update_values")


def get_info(sys: System) -> dict:
    info = _Info()
    _check(lib().lpcg_get_info(sys.handle, C.byref(info)), "lpcg_get_info")
    return {f: getattr(info, f) for f, _ in _Info._fields_}


def export_pattern(sys: System) -> dict:
    i = sys.info
    n, nnz, nl = i["n"], i["nnz"], i["nnz_l"]

    def e(k):
        return torch.empty(k, dtype=torch.int32, device="cuda")
    out = dict(lrowptr=e(n + 1), lcol=e(nl), lsrc=e(nl), urowptr=e(n + 1), ucol=e(nl), u2l=e(nl),
               rev=e(nnz), flevel=e(n), flev_ptr=e(i["nlev_fwd"] + 1), flev_rows=e(n),
               blevel=e(n), blev_ptr=e(i["nlev_bwd"] + 1), blev_rows=e(n))
    rc = lib().lpcg_export_pattern(sys.handle, *[_ptr(out[k]) for k in (
        "lrowptr", "lcol", "lsrc", "urowptr", "ucol", "u2l", "rev", "flevel", "flev_ptr",
        "flev_rows", "blevel", "blev_ptr", "blev_rows")], _stream())
    _check(rc, "lpcg_export_pattern")
    return out


def export_perm(sys: System):
    """perm[internal row] = original row (identity for the natural ordering)."""
    out = torch.empty(sys.info["n"], dtype=torch.int32, device="cuda")
    _check(lib().lpcg_export_perm(sys.handle, _ptr(out), _stream()), "lpcg_export_perm")
    return out


# ------------------------------------------------------------------ tuning
def autotune(sys: System, l_val, ut_val, reps: int = 5) -> list:
    """Time every substitution configuration, keep the fastest per
    direction; returns the measured table as a list of dicts."""
    cap = 256
    table = (_TrsvCfg * cap)()
    n = C.c_int32(0)
    rc = lib().lpcg_autotune(sys.handle, _ptr(l_val), _ptr(ut_val), C.c_int32(reps), table, C.c_int32(cap),
                             C.byref(n), _stream())
    _check(rc, "lpcg_autotune")
    return [{f: getattr(table[i], f) for f, _ in _TrsvCfg._fields_} for i in range(min(n.value, cap))]


def get_trsv_cfg(sys: System, direction: int) -> dict:
    c = _TrsvCfg()
    _check(lib().lpcg_get_trsv_cfg(sys.handle, C.c_int32(direction), C.byref(c)), "lpcg_get_trsv_cfg")
    return {f: getattr(c, f) for f, _ in _TrsvCfg._fields_ if f != "us"}


def set_trsv_cfg(sys: System, direction: int, mode: int, waves: int = 0, backoff: int = 1,
                 block_stride: int = 1, block_rows: int = 0, block_runs: int = 1):
    c = _TrsvCfg(direction, mode, waves, backoff, block_stride, block_rows, 0.0, block_runs)
    _check(lib().lpcg_set_trsv_cfg(sys.handle, C.byref(c)), "lpcg_set_trsv_cfg")


def blocked_schedule(rowptr, col, upper: bool, block_rows: int, block_runs: int = 1) -> dict:
    """Host schedule of the blocked substitution for a triangular CSR pattern
    (lower: diagonal last; upper: diagonal first), as NumPy arrays; position x
    of block b is row brow[b, 0] + (x >> run_shift) * run_stride + (x & (2^run_shift - 1))."""
    import numpy as np
    rp = np.ascontiguousarray(rowptr, dtype=np.int32)
    ci = np.ascontiguousarray(col, dtype=np.int32)
    n = rp.shape[0] - 1
    L = lib()
    out = _BlkSchedule()
    f = L.lpcg_blocked_schedule
    args = (C.c_int32(n), rp.ctypes.data_as(C.c_void_p), ci.ctypes.data_as(C.c_void_p), C.c_int32(int(upper)),
            C.c_int32(block_rows), C.c_int32(block_runs))
    _check(f(*args, C.byref(out)), "lpcg_blocked_schedule")
    w = out.deps
    arrs = dict(brow=np.zeros(2 * out.nblocks, np.int32), bch=np.zeros(out.nblocks + 1, np.int32),
                chunks=np.zeros(2 * out.nchunks, np.int32), rec=np.zeros(n * (2 * w + 2), np.int32),
                vsrc=np.zeros(n * (w + 1), np.int32))
    for k, a in arrs.items():
        setattr(out, k, a.ctypes.data_as(C.c_void_p))
    _check(f(*args, C.byref(out)), "lpcg_blocked_schedule")
    arrs.update(deps=w, nblocks=out.nblocks, nchunks=out.nchunks, max_chunks=out.max_chunks,
                run_shift=out.run_shift, run_stride=out.run_stride)
    arrs["brow"] = arrs["brow"].reshape(-1, 2)
    arrs["chunks"] = arrs["chunks"].reshape(-1, 2)
    arrs["rec"] = arrs["rec"].reshape(n, 2 * w + 2)
    arrs["vsrc"] = arrs["vsrc"].reshape(n, w + 1)
    return arrs


# ---------------------------------------------------------- building blocks
def spmv(sys: System, x, out=None):
    prec = 64 if x.dtype == torch.float64 else 32
    if prec == 32 and x.dtype != torch.float32:
        raise TypeError("float32 or float64 expected")
    if out is None:
        out = torch.empty_like(x)
    _check(lib().lpcg_spmv(sys.handle, C.c_int32(prec), _ptr(x), _ptr(out), _stream()), "lpcg_spmv")
    return out


def sptrsv(sys: System, transpose: bool, l_val, ut_val, rhs, out=None):
    if out is None:
        out = torch.empty_like(rhs)
    rc = lib().lpcg_sptrsv(sys.handle, C.c_int32(1 if transpose else 0), _ptr(l_val), _ptr(ut_val),
                           _ptr(rhs), _ptr(out), _stream())
    _check(rc, "lpcg_sptrsv")
    return out


def l_to_ut(sys: System, l_val, out=None):
    if out is None:
        out = torch.empty_like(l_val)
    _check(lib().lpcg_l_to_ut(sys.handle, _ptr(l_val), _ptr(out), _stream()), "lpcg_l_to_ut")
    return out


def check_factor(sys: System, l_val):
    """(ok, first bad row in the internal numbering or -1)."""
    bad = C.c_int32(0)
    rc = lib().lpcg_check_factor(sys.handle, _ptr(l_val), C.byref(bad), _stream())
    if rc not in (OK, ENONFINITE):
        _check(rc, "lpcg_check_factor")
    return rc == OK, bad.value


def sgs(sys: System, l_val=None, ut_val=None):
    """Symmetric Gauss-Seidel factor L = (D + A_<) D^-1/2 (and U = L^T)."""
    nl = sys.info["nnz_l"]
    if l_val is None:
        l_val = torch.empty(nl, dtype=torch.float32, device="cuda")
    if ut_val is None:
        ut_val = torch.empty(nl, dtype=torch.float32, device="cuda")
    _check(lib().lpcg_sgs(sys.handle, _ptr(l_val), _ptr(ut_val), _stream()), "lpcg_sgs")
    return l_val, ut_val


def ic0(sys: System, shift0=0.0, max_retries=8, l_val=None, ut_val=None):
    nl = sys.info["nnz_l"]
    if l_val is None:
        l_val = torch.empty(nl, dtype=torch.float32, device="cuda")
    if ut_val is None:
        ut_val = torch.empty(nl, dtype=torch.float32, device="cuda")
    used = C.c_double(0)
    rc = lib().lpcg_ic0(sys.handle, C.c_double(shift0), C.c_int32(max_retries), _ptr(l_val),
                        _ptr(ut_val), C.byref(used), _stream())
    _check(rc, "lpcg_ic0")
    return l_val, ut_val, used.value


def ic0_noalloc(sys: System, shift0=0.0, max_retries=8, l_val=None, ut_val=None):
    """lpcg_ic0_noalloc: IC(0) with the library's static FP64 scratch (no
    device allocation inside the call; nnz_l <= IC0_NOALLOC_MAX_NNZ_L)."""
    nl = sys.info["nnz_l"]
    if l_val is None:
        l_val = torch.empty(nl, dtype=torch.float32, device="cuda")
    if ut_val is None:
        ut_val = torch.empty(nl, dtype=torch.float32, device="cuda")
    used = C.c_double(0)
    rc = lib().lpcg_ic0_noalloc(sys.handle, C.c_double(shift0), C.c_int32(max_retries), _ptr(l_val),
                                _ptr(ut_val), C.byref(used), _stream())
    _check(rc, "lpcg_ic0_noalloc")
    return l_val, ut_val, used.value


IC0_NOALLOC_MAX_NNZ_L = 2097152


def jacobi(sys: System, out=None):
    if out is None:
        out = torch.empty(sys.n, dtype=torch.float32, device="cuda")
    _check(lib().lpcg_jacobi(sys.handle, _ptr(out), _stream()), "lpcg_jacobi")
    return out


# ---------------------------------------------------------------------- PCG
def pcg_solve(sys: System, kind: int, b, x=None, l_val=None, ut_val=None, dinv=None,
              tol=1e-6, maxit=0, check_every=0, max_restarts=0, use_graph=False,
              hist=False, raise_on_status=False, coef=None):
    """Returns (x, result dict[, hist tensor]).  coef: optional device FP64
    tensor of 2 (maxit + 1) entries that receives alpha_k / beta_k."""
    b = _dev(b, torch.float64).contiguous()
    if x is None:
        x = torch.zeros_like(b)
    P = _Precond(kind, _ptr(l_val), _ptr(ut_val), _ptr(dinv))
    mi = maxit if maxit > 0 else sys.n
    opts = _Opts(float(tol), int(mi), int(check_every), int(max_restarts), int(bool(use_graph)))
    res = _Result()
    h = torch.full((mi + 1,), float("nan"), dtype=torch.float64, device="cuda") if hist else None
    if coef is not None and coef.numel() < 2 * (mi + 1):
        raise ValueError("coef needs 2 (maxit + 1) entries")
    rc = lib().lpcg_pcg_solve(sys.handle, C.byref(P), _ptr(b), _ptr(x), C.byref(opts),
                              C.byref(res), _ptr(h), _ptr(coef), _stream())
    if rc not in (OK, ENOTCONV, EBREAKDOWN) or (raise_on_status and rc != OK):
        _check(rc, "lpcg_pcg_solve")
    out = {f: getattr(res, f) for f, _ in _Result._fields_ if f != "reserved"}
    if hist:
        return x, out, h[: res.iters + 1] if res.restarts == 0 else h
    return x, out


def pcg_solve_batched(sys: System, kind: int, b, x=None, l_val=None, ut_val=None, dinv=None,
                      tol=1e-6, maxit=0, check_every=8, max_restarts=0, use_graph=False,
                      raise_on_status=False):
    """One PCG per system of a batch; returns (x, list of per-system result dicts)."""
    b = _dev(b, torch.float64).contiguous()
    if x is None:
        x = torch.zeros_like(b)
    nsys = sys.info["nsys"]
    P = _Precond(kind, _ptr(l_val), _ptr(ut_val), _ptr(dinv))
    mi = maxit if maxit > 0 else sys.n
    opts = _Opts(float(tol), int(mi), int(check_every), int(max_restarts), int(bool(use_graph)))
    res = (_Result * nsys)()
    rc = lib().lpcg_pcg_solve_batched(sys.handle, C.byref(P), _ptr(b), _ptr(x), C.byref(opts), res, _stream())
    if rc not in (OK, ENOTCONV, EBREAKDOWN) or (raise_on_status and rc != OK):
        _check(rc, "lpcg_pcg_solve_batched")
    return x, [{f: getattr(r, f) for f, _ in _Result._fields_ if f != "reserved"} for r in res]


def pcg_solve_ir(sys: System, kind: int, b, x=None, l_val=None, ut_val=None, dinv=None,
                 tol=1e-10, tol_inner=1e-4, max_outer=20, maxit=0, check_every=8, use_graph=False,
                 raise_on_status=False):
    """FP64 iterative refinement over the FP32 batched PCG; returns (x, per-system results)."""
    b = _dev(b, torch.float64).contiguous()
    if x is None:
        x = torch.zeros_like(b)
    nsys = sys.info["nsys"]
    P = _Precond(kind, _ptr(l_val), _ptr(ut_val), _ptr(dinv))
    mi = maxit if maxit > 0 else sys.n
    opts = _Opts(float(tol_inner), int(mi), int(check_every), 0, int(bool(use_graph)))
    res = (_Result * nsys)()
    rc = lib().lpcg_pcg_solve_ir(sys.handle, C.byref(P), _ptr(b), _ptr(x), C.c_double(tol), C.c_double(tol_inner),
                                 C.c_int32(max_outer), C.byref(opts), res, _stream())
    if rc not in (OK, ENOTCONV, EBREAKDOWN) or (raise_on_status and rc != OK):
        _check(rc, "lpcg_pcg_solve_ir")
    return x, [{f: getattr(r, f) for f, _ in _Result._fields_ if f != "reserved"} for r in res]


def time_pcg_kernels(sys: System, kind: int, b, l_val=None, ut_val=None, dinv=None, reps: int = 20):
    """Mean microseconds of one PCG iteration's parts, launched eagerly with
    events between them: (application of L L^T, SpMV with p and p.w, x/r
    update)."""
    b = _dev(b, torch.float64).contiguous()
    P = _Precond(kind, _ptr(l_val), _ptr(ut_val), _ptr(dinv))
    out = (C.c_double * 3)()
    _check(lib().lpcg_time_pcg_kernels(sys.handle, C.byref(P), _ptr(b), C.c_int32(reps), out, _stream()),
           "lpcg_time_pcg_kernels")
    return tuple(out[i] for i in range(3))


def next_chunk(it: int, res: float, prev_it: int, prev_res: float, tol: float, maxit: int):
    """(iterations, predicted_final): the solver's rule for its next chunk
    of iterations (host computation in the library, no GPU)."""
    fin = C.c_int32(0)
    fn = lib().lpcg_next_chunk
    fn.restype = C.c_int32
    fn.argtypes = [C.c_int32, C.c_float, C.c_int32, C.c_float, C.c_double, C.c_int32, C.POINTER(C.c_int32)]
    n = fn(int(it), float(res), int(prev_it), float(prev_res), float(tol), int(maxit), C.byref(fin))
    return int(n), bool(fin.value)


def lanczos_extremes(coef, iters: int):
    """(lambda_min, lambda_max) of the preconditioned operator estimated from
    the PCG coefficients (host computation in the library)."""
    import numpy as np
    c = np.ascontiguousarray(coef.detach().cpu().numpy() if torch.is_tensor(coef) else coef, dtype=np.float64)
    lo, hi = C.c_double(0), C.c_double(0)
    _check(lib().lpcg_lanczos_extremes(c.ctypes.data_as(C.c_void_p), C.c_int32(iters), C.byref(lo), C.byref(hi)),
           "lpcg_lanczos_extremes")
    return lo.value, hi.value


# ------------------------------------------------------------------ timing
def time_sptrsv(sys: System, transpose: bool, l_val, ut_val, rhs, reps=20):
    """Mean duration (ms) of one substitution kernel launch (HIP events)."""
    out = torch.empty_like(rhs)
    ms = C.c_double(0)
    rc = lib().lpcg_time_sptrsv(sys.handle, C.c_int32(1 if transpose else 0), _ptr(l_val),
                                _ptr(ut_val), _ptr(rhs), _ptr(out), C.c_int32(reps), C.byref(ms),
                                _stream())
    _check(rc, "lpcg_time_sptrsv")
    return ms.value


def time_spmv(sys: System, x, reps=50):
    """Mean duration (ms) of one FP32 SpMV launch (HIP events)."""
    out = torch.empty_like(x)
    ms = C.c_double(0)
    rc = lib().lpcg_time_spmv(sys.handle, _ptr(x), _ptr(out), C.c_int32(reps), C.byref(ms), _stream())
    _check(rc, "lpcg_time_spmv")
    return ms.value


# ---------------------------------------------------------------------- GNN
def param_layout(h: int, n_mp: int, x_head: bool = False):
    """(name, shape) of every tensor of the flat FP32 parameter vector, in the
    order of include/lpcg.h (node_enc, edge_enc, mp{t}.node, mp{t}.edge, dec,
    and xdec with the initial-guess head; each MLP: W0, b0, W1, b1 with W
    stored [fan_in][fan_out])."""
    out = []

    def mlp(prefix, fin, fout):
        out.extend([(f"{prefix}.W0", (fin, h)), (f"{prefix}.b0", (h,)),
                    (f"{prefix}.W1", (h, fout)), (f"{prefix}.b1", (fout,))])
    mlp("node_enc", 1, h)
    mlp("edge_enc", 1, h)
    for t in range(n_mp):
        mlp(f"mp{t}.node", 2 * h, h)
        mlp(f"mp{t}.edge", 3 * h, h)
    mlp("dec", h, 1)
    if x_head:
        mlp("xdec", h, 1)
    return out


def param_count(h: int, n_mp: int, x_head: bool = False) -> int:
    return int(lib().lpcg_gnn_param_count(h, n_mp, 1 if x_head else 0))


def has_x_head(nparams: int, h: int, n_mp: int) -> bool:
    """Whether a flat parameter vector of nparams entries carries the head."""
    if nparams == param_count(h, n_mp, False):
        return False
    if nparams == param_count(h, n_mp, True):
        return True
    raise ValueError(f"{nparams} parameters match neither layout of h={h}, n_mp={n_mp}")


def pack_params(P: dict, h: int, n_mp: int) -> torch.Tensor:
    """Flatten a dict of named arrays into the library's FP32 layout (host);
    the head is packed when P holds xdec.*."""
    import numpy as np
    parts = []
    x_head = "xdec.W0" in P
    for name, shape in param_layout(h, n_mp, x_head):
        a = np.asarray(P[name], dtype=np.float32)
        if a.shape != shape:
            raise ValueError(f"{name}: shape {a.shape}, expected {shape}")
        parts.append(a.reshape(-1))
    flat = np.concatenate(parts)
    assert flat.shape[0] == param_count(h, n_mp, x_head)
    return torch.as_tensor(flat)


def unpack_params(flat, h: int, n_mp: int) -> dict:
    import numpy as np
    flat = np.asarray(flat.detach().cpu() if torch.is_tensor(flat) else flat)
    out, p = {}, 0
    for name, shape in param_layout(h, n_mp, has_x_head(flat.shape[0], h, n_mp)):
        k = int(np.prod(shape))
        out[name] = flat[p:p + k].reshape(shape)
        p += k
    return out


def gnn_workspace(sys: System, h: int, n_mp: int, train: bool = False) -> torch.Tensor:
    nbytes = int(lib().lpcg_gnn_workspace_bytes(sys.handle, h, n_mp, 1 if train else 0))
    if nbytes < 0:
        raise ValueError("invalid GNN dimensions")
    return torch.empty(nbytes, dtype=torch.uint8, device="cuda")


def _net(params, h, n_mp, diag_mode=0):
    if params.dtype != torch.float32:
        raise TypeError("params must be float32")
    # the head is present when the vector has the head's layout; the library
    # validates the dimensions themselves
    x_head = 1 if h > 0 and 1 <= n_mp and params.numel() == param_count(h, n_mp, True) else 0
    return _Gnn(h, n_mp, _ptr(params), diag_mode, x_head)


def gnn_predict_L(sys: System, params, h: int, n_mp: int, b, ws, l_val=None, ut_val=None, diag_mode=0):
    nl = sys.info["nnz_l"]
    if l_val is None:
        l_val = torch.empty(nl, dtype=torch.float32, device="cuda")
    net = _net(params, h, n_mp, diag_mode)
    rc = lib().lpcg_gnn_predict_L(sys.handle, C.byref(net), _ptr(b), _ptr(ws), C.c_int64(ws.numel()),
                                  _ptr(l_val), _ptr(ut_val), _stream())
    _check(rc, "lpcg_gnn_predict_L")
    return l_val, ut_val


def gnn_forward_train(sys: System, params, h: int, n_mp: int, b, ws, l_val=None, diag_mode=0):
    nl = sys.info["nnz_l"]
    if l_val is None:
        l_val = torch.empty(nl, dtype=torch.float32, device="cuda")
    net = _net(params, h, n_mp, diag_mode)
    rc = lib().lpcg_gnn_forward_train(sys.handle, C.byref(net), _ptr(b), _ptr(ws), C.c_int64(ws.numel()),
                                      _ptr(l_val), _stream())
    _check(rc, "lpcg_gnn_forward_train")
    return l_val


def gnn_predict_x0(sys: System, params, h: int, n_mp: int, b, ws, l_val=None, ut_val=None, x0=None,
                   diag_mode=0):
    """L (and U = L^T when ut_val is given) plus the head's starting guess x0
    (FP64 [n], original numbering); params must carry the head."""
    if l_val is None:
        l_val = torch.empty(sys.info["nnz_l"], dtype=torch.float32, device="cuda")
    if x0 is None:
        x0 = torch.empty(sys.n, dtype=torch.float64, device="cuda")
    net = _net(params, h, n_mp, diag_mode)
    rc = lib().lpcg_gnn_predict_x0(sys.handle, C.byref(net), _ptr(b), _ptr(ws), C.c_int64(ws.numel()),
                                   _ptr(l_val), _ptr(ut_val), _ptr(x0), _stream())
    _check(rc, "lpcg_gnn_predict_x0")
    return l_val, ut_val, x0


def x0_loss(sys: System, params, h: int, n_mp: int, ws, x, weight=1.0, diag_mode=0):
    """Per-system loss of the head against the solution x (device FP64
    [nsys]); with weight != 0 its scaled gradient is left in ws for
    gnn_backward."""
    loss = torch.empty(sys.info["nsys"], dtype=torch.float64, device="cuda")
    net = _net(params, h, n_mp, diag_mode)
    rc = lib().lpcg_x0_loss(sys.handle, C.byref(net), _ptr(ws), C.c_int64(ws.numel()), _ptr(x),
                            C.c_double(weight), _ptr(loss), _stream())
    _check(rc, "lpcg_x0_loss")
    return loss


def gnn_backward(sys: System, params, h: int, n_mp: int, ws, dl_val, dparams=None, diag_mode=0):
    if dparams is None:
        dparams = torch.empty_like(params)
    net = _net(params, h, n_mp, diag_mode)
    rc = lib().lpcg_gnn_backward(sys.handle, C.byref(net), _ptr(ws), C.c_int64(ws.numel()),
                                 _ptr(dl_val.contiguous()), _ptr(dparams), _stream())
    _check(rc, "lpcg_gnn_backward")
    return dparams


def llt_loss(sys: System, l_val, x, b, grad=True):
    """(loss per system [nsys] FP64, d sum(loss) / d L FP32 or None)."""
    loss = torch.empty(sys.info["nsys"], dtype=torch.float64, device="cuda")
    dl = torch.empty_like(l_val) if grad else None
    rc = lib().lpcg_llt_loss(sys.handle, _ptr(l_val), _ptr(x), _ptr(b), _ptr(loss), _ptr(dl), _stream())
    _check(rc, "lpcg_llt_loss")
    return loss, dl


def frob_loss(sys: System, l_val, grad=True):
    """Per-system ||L L^T - A||_F^2 / s^2 (device FP64 [nsys]) and its gradient."""
    loss = torch.empty(sys.info["nsys"], dtype=torch.float64, device="cuda")
    dl = torch.empty_like(l_val) if grad else None
    _check(lib().lpcg_frob_loss(sys.handle, _ptr(l_val), _ptr(loss), _ptr(dl), _stream()), "lpcg_frob_loss")
    return loss, dl


def adam_step(params, grads, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
    rc = lib().lpcg_adam_step(_ptr(params), _ptr(grads), _ptr(m), _ptr(v), C.c_int64(params.numel()),
                              C.c_float(lr), C.c_float(beta1), C.c_float(beta2), C.c_float(eps),
                              C.c_int32(step), _stream())
    _check(rc, "lpcg_adam_step")


class GnnL(torch.autograd.Function):
    """L = GNN(A, b; params) with the library's forward and hand-written
    backward (argument marshalling only)."""

    @staticmethod
    def forward(ctx, params, sys, h, n_mp, b, ws, diag_mode=0):
        l_val = gnn_forward_train(sys, params, h, n_mp, b, ws, diag_mode=diag_mode)
        ctx.sys, ctx.h, ctx.n_mp, ctx.ws, ctx.diag_mode = sys, h, n_mp, ws, diag_mode
        ctx.save_for_backward(params)
        return l_val

    @staticmethod
    def backward(ctx, g_l):
        (params,) = ctx.saved_tensors
        dparams = gnn_backward(ctx.sys, params, ctx.h, ctx.n_mp, ctx.ws, g_l.float().contiguous(),
                               diag_mode=ctx.diag_mode)
        return dparams, None, None, None, None, None, None


class LltLoss(torch.autograd.Function):
    """sum over systems of ||L L^T x - b||^2 / rms(b)^2 with the library's
    closed-form gradient."""

    @staticmethod
    def forward(ctx, l_val, sys, x, b):
        loss, dl = llt_loss(sys, l_val, x, b, grad=True)
        ctx.save_for_backward(dl)
        return loss.sum()

    @staticmethod
    def backward(ctx, g):
        (dl,) = ctx.saved_tensors
        return (dl * g.to(dl.dtype)), None, None, None
