"""Every substitution mode (dependency driven with several wave counts and
back-offs; level synchronous; single workgroup; blocked with several block
sizes) in both row orderings, against the oracle, and the autotuner that
chooses between them.

Bars: componentwise backward error |rhs - T y| <= 4 k u32 |T| |y| for the
solves (Higham's substitution bound in FP32, c = 4 covering FMA and the
division); PCG iterations within max(2, 10%) of the FP64 oracle's and the
FP64 true residual <= tol."""
import numpy as np
import pytest
import torch

import oracle as O
import pdegen as g
from paper_2305_16432_amd import lpcg
from tests.gpu_util import U32, cuda_f32, cuda_f64, gpu_system, host, matrices_small

pytestmark = pytest.mark.gpu

# (mode, waves, backoff, block stride, block rows)
CFGS = [(0, 256, 4, 1, 0), (0, 4096, 1, 1, 0), (0, 1024, 16, 1, 0), (0, 128, 16, 8, 0), (1, 0, 1, 1, 0),
        (2, 0, 1, 1, 0), (3, 0, 0, 1, 64), (3, 0, 1, 1, 256), (3, 0, 0, 1, 1024), (3, 0, 0, 8, 128)]


def _blocked_fits(pat):
    """The blocked mode takes rows with at most 7 dependencies."""
    return max(np.diff(pat.lrowptr).max(), np.diff(pat.urowptr).max()) - 1 <= 7


def _set_all(S, pat, cfg):
    """Set cfg in both directions; False when the blocked mode (correctly)
    refuses the pattern."""
    mode, waves, backoff, stride, brows = cfg
    if mode == 3 and not _blocked_fits(pat):
        with pytest.raises(lpcg.LpcgError) as e:
            lpcg.set_trsv_cfg(S, 0, mode, waves, backoff, stride, brows)
        assert e.value.code == lpcg.EINVAL
        return False
    for d in (0, 1):
        lpcg.set_trsv_cfg(S, d, mode, waves, backoff, stride, brows)
        got = lpcg.get_trsv_cfg(S, d)
        assert got["mode"] == mode and got["block_stride"] == stride
        assert got["block_rows"] == (brows if mode == 3 else 0)
    return True


def _lower(pat, seed):
    rng = np.random.default_rng(seed)
    lv = rng.uniform(-0.3, 0.3, pat.nnz_l)
    row = np.repeat(np.arange(len(pat.lrowptr) - 1), np.diff(pat.lrowptr))
    d = pat.lcol == row
    lv[d] = rng.uniform(1.0, 2.0, d.sum())
    return lv.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("cfg", CFGS)
@pytest.mark.parametrize("ordering", [0, 1])
@pytest.mark.parametrize("name", ["tridiag_1000", "heat3d_13", "fem_40", "random_777", "one"])
def test_sptrsv_modes(name, ordering, cfg):
    print(f"[trsv] {name} ordering {ordering} cfg {cfg}", flush=True)
    A = matrices_small()[name]
    if ordering:
        perm, _, _ = O.color_order(A)
        Ai = O.permute_sym(A, perm)
    else:
        perm, Ai = np.arange(A.n), A
    pat = O.Pattern(Ai)
    S = gpu_system(A, None, ordering)
    if not _set_all(S, pat, cfg):
        return
    lval = _lower(pat, 3)
    utv = lval[pat.usrc]
    rhs = np.random.default_rng(4).standard_normal(A.n).astype(np.float32).astype(np.float64)
    L = g.CSR(A.n, pat.lrowptr, pat.lcol, lval).to_scipy()
    k = max(1, np.diff(pat.lrowptr).max())
    # vectors in the caller's numbering; the factor acts on the internal order
    y = host(lpcg.sptrsv(S, False, cuda_f32(lval), cuda_f32(utv), cuda_f32(rhs))).astype(np.float64)[perm]
    z = host(lpcg.sptrsv(S, True, cuda_f32(lval), cuda_f32(utv), cuda_f32(rhs))).astype(np.float64)[perm]
    r = rhs[perm]
    assert np.all(np.abs(r - L @ y) <= 4 * k * U32 * (abs(L) @ np.abs(y)) + 1e-30)
    assert np.all(np.abs(r - L.T @ z) <= 4 * k * U32 * (abs(L.T) @ np.abs(z)) + 1e-30)
    np.testing.assert_allclose(y, O.trsv_lower(pat, lval, r), rtol=1e-3, atol=1e-5 * np.abs(y).max())
    np.testing.assert_allclose(z, O.trsv_upper(pat, lval, r), rtol=1e-3, atol=1e-5 * np.abs(z).max())


@pytest.mark.parametrize("cfg", CFGS)
@pytest.mark.parametrize("ordering", [0, 1])
@pytest.mark.parametrize("name", ["heat3d_13", "fem_40"])
def test_pcg_ic0_modes(name, ordering, cfg):
    A = matrices_small()[name]
    b = np.random.default_rng(2).standard_normal(A.n)
    if ordering:
        perm, _, _ = O.color_order(A)
        Ai = O.permute_sym(A, perm)
    else:
        perm, Ai = np.arange(A.n), A
    pat = O.Pattern(Ai)
    S = gpu_system(A, None, ordering)
    if not _set_all(S, pat, cfg):
        return
    l, ut, _ = lpcg.ic0(S)
    for use_graph in (False, True):
        x, res = lpcg.pcg_solve(S, lpcg.PC_LLT, cuda_f64(b), l_val=l, ut_val=ut, tol=1e-6, max_restarts=2,
                                use_graph=use_graph)
        lref, _ = O.ic0(pat, Ai)
        ro = O.pcg(Ai, b[perm], O.PC_LLT, pat, lref, tol=1e-6)
        assert res["status"] == 0 and O.true_relres(A, b, host(x)) <= 1e-6
        assert abs(res["iters"] - ro["iters"]) <= max(2, 0.1 * ro["iters"]), (res["iters"], ro["iters"])


@pytest.mark.parametrize("ordering", [0, 1])
def test_autotune_c3_full_size(ordering):
    print(f"[autotune] heat3d_64 ordering {ordering}", flush=True)
    A, b = g.heat_system_3d(64, 1e-3, 1000, 2000)
    S = gpu_system(A, None, ordering)
    l, ut, _ = lpcg.ic0(S)
    table = lpcg.autotune(S, l, ut, reps=3)
    assert len(table) >= 2
    for d in (0, 1):
        rows = [t for t in table if t["direction"] == d]
        best = min(rows, key=lambda t: t["us"])
        if ordering == 1:  # red-black: two levels, the fused pair needs the level mode both ways
            best = next(t for t in rows if t["mode"] == 1)
        got = lpcg.get_trsv_cfg(S, d)
        assert got["mode"] == best["mode"] and got["backoff"] == best["backoff"]
        assert got["block_stride"] == best["block_stride"] and got["block_rows"] == best["block_rows"]
        if best["mode"] == 0:
            assert got["waves"] == best["waves"]
        for t in sorted(rows, key=lambda t: t["us"])[:6]:
            print(f"  dir {d} mode {t['mode']} waves {t['waves']} backoff {t['backoff']} "
                  f"stride {t['block_stride']} rows {t['block_rows']}: {t['us']:.1f} us")
    # the SpMV: every lanes-per-row choice timed, the fastest kept
    sp = [t for t in table if t["direction"] == 2]
    assert {t["mode"] for t in sp} == {1, 4, 8, 16, 32, 64}  # 1: the ELL form (7-entry rows)
    best = min(sp, key=lambda t: t["us"])
    ell = next(t for t in sp if t["mode"] == 1)
    if ell["us"] <= 1.1 * best["us"]:  # the ELL form stays unless another is 10% faster
        best = ell
    got = lpcg.get_trsv_cfg(S, 2)
    assert got["mode"] == best["mode"] and got["waves"] == best["waves"]
    assert got["block_rows"] == best["block_rows"]
    assert {t["block_rows"] for t in sp} >= {0, 256, 512, 1024}  # the LDS-staged form timed too
    for t in sorted(sp, key=lambda t: t["us"])[:6]:
        print(f"  spmv: G {t['mode']} blocks {t['waves']} rows/block {t['block_rows']}: {t['us']:.1f} us")
    x, res = lpcg.pcg_solve(S, lpcg.PC_LLT, cuda_f64(b), l_val=l, ut_val=ut, tol=1e-6, max_restarts=2)
    assert res["status"] == 0 and O.true_relres(A, b, host(x)) <= 1e-6


@pytest.mark.parametrize("G", [4, 16, 64])
def test_spmv_lanes_per_row_within_bound(G):
    """Every SpMV lanes-per-row choice gives an FP32 product within the
    per-row bound of the FP64 oracle, and the PCG reaches the tolerance."""
    A = matrices_small()["fem_40"]
    S = gpu_system(A)
    x = np.random.default_rng(1).standard_normal(A.n).astype(np.float32)
    lpcg.set_trsv_cfg(S, 2, G, waves=37)
    assert lpcg.get_trsv_cfg(S, 2)["mode"] == G
    y = host(lpcg.spmv(S, torch.as_tensor(x).cuda()))
    ref = O.spmv(A, x.astype(np.float64))
    bound = O.spmv(g.CSR(A.n, A.rowptr, A.colind, np.abs(A.val)), np.abs(x.astype(np.float64)))
    k = np.diff(A.rowptr)
    assert np.all(np.abs(y - ref) <= 2 * k * U32 * bound + 1e-30)
    b = np.random.default_rng(2).standard_normal(A.n)
    xs, res = lpcg.pcg_solve(S, lpcg.PC_JACOBI, cuda_f64(b), tol=1e-6, max_restarts=2)
    assert res["status"] == 0 and O.true_relres(A, b, host(xs)) <= 1e-6


def _spmv_cases():
    m = matrices_small()
    return [(m["heat3d_13"], 0), (m["heat3d_13"], 1), (m["fem_40"], 0), (m["fem_40"], 1),
            (m["poisson2d_32"], 1), (m["tridiag_1000"], 0)]


@pytest.mark.parametrize("case", range(6))
def test_spmv_staged_matches_gather_bit_for_bit(case):
    """The LDS-staged SpMV (block of R rows, inputs staged over the block's
    column window) sums every row exactly as the gather form with the same
    lanes per row: equal bit for bit, ragged last blocks included; the PCG
    with the staged product ends as the gather form's does (the 1D Laplacian,
    kappa ~ 1e6, does not reach 1e-6 with FP32 Jacobi-PCG in n iterations in
    either form) and, where that converges, in the same iterations."""
    A, ordering = _spmv_cases()[case]
    print(f"[spmv staged] case {case} n={A.n} ordering {ordering}", flush=True)
    S = gpu_system(A, None, ordering)
    x = torch.as_tensor(np.random.default_rng(3).standard_normal(A.n).astype(np.float32)).cuda()
    b = np.random.default_rng(4).standard_normal(A.n)
    for G in (4, 8):
        lpcg.set_trsv_cfg(S, 2, G, waves=64)
        y0 = host(lpcg.spmv(S, x))
        _, r0 = lpcg.pcg_solve(S, lpcg.PC_JACOBI, cuda_f64(b), tol=1e-6, max_restarts=2)
        for R in (256, 512, 1024):
            lpcg.set_trsv_cfg(S, 2, G, block_rows=R)
            got = lpcg.get_trsv_cfg(S, 2)
            assert got["mode"] == G and got["block_rows"] == R and got["waves"] == -(-A.n // R)
            y1 = host(lpcg.spmv(S, x))
            assert np.array_equal(y0.view(np.uint32), y1.view(np.uint32)), (G, R)
            xs, r1 = lpcg.pcg_solve(S, lpcg.PC_JACOBI, cuda_f64(b), tol=1e-6, max_restarts=2)
            assert r1["status"] == r0["status"], (G, R, r0, r1)
            if r0["status"] == 0:
                assert O.true_relres(A, b, host(xs)) <= 1e-6
                assert abs(r1["iters"] - r0["iters"]) <= 1, (G, R, r0["iters"], r1["iters"])


@pytest.mark.parametrize("case", range(7))
def test_spmv_ell_within_bound(case):
    """The ELL SpMV (one row per lane, slots column-major, padding of value
    0): within the per-row FP32 bound of the FP64 oracle; Jacobi-PCG with it
    reaches the tolerance as the gather form does (iterations within
    max(2, 5%) when neither restarts); the FP64 product keeps the gather
    form.  A pattern with a
    row of more than 8 entries refuses it and keeps its configuration."""
    cases = _spmv_cases() + [(matrices_small()["bipartite_24"], 1)]
    A, ordering = cases[case]
    print(f"[spmv ell] case {case} n={A.n} ordering {ordering}", flush=True)
    S = gpu_system(A, None, ordering)
    xh = np.random.default_rng(8).standard_normal(A.n).astype(np.float32)
    x = torch.as_tensor(xh).cuda()
    b = np.random.default_rng(9).standard_normal(A.n)
    lpcg.set_trsv_cfg(S, 2, 4, waves=64)
    # an iteration budget of 4 n leaves the FP64 restarts room on the 1D
    # Laplacian (kappa ~ 4e5), whose FP32 iteration needs about n products
    _, r0 = lpcg.pcg_solve(S, lpcg.PC_JACOBI, cuda_f64(b), tol=1e-6, maxit=4 * A.n, max_restarts=4)
    k = np.diff(A.rowptr)
    if k.max() > 8:
        with pytest.raises(lpcg.LpcgError) as e:
            lpcg.set_trsv_cfg(S, 2, 1)
        assert e.value.code == lpcg.EINVAL
        assert lpcg.get_trsv_cfg(S, 2)["mode"] == 4
        return
    lpcg.set_trsv_cfg(S, 2, 1)
    got = lpcg.get_trsv_cfg(S, 2)
    assert got["mode"] == 1 and got["block_rows"] == 0 and got["waves"] == min(2048, -(-A.n // 256))
    y = host(lpcg.spmv(S, x))
    ref = O.spmv(A, xh.astype(np.float64))
    bound = O.spmv(g.CSR(A.n, A.rowptr, A.colind, np.abs(A.val)), np.abs(xh.astype(np.float64)))
    assert np.all(np.abs(y - ref) <= 2 * k * U32 * bound + 1e-30)
    x64 = np.random.default_rng(10).standard_normal(A.n)
    y64 = host(lpcg.spmv(S, cuda_f64(x64)))
    b64 = O.spmv(g.CSR(A.n, A.rowptr, A.colind, np.abs(A.val)), np.abs(x64))
    assert np.all(np.abs(y64 - O.spmv(A, x64)) <= 2 * k * 2.0 ** -53 * b64 + 1e-300)
    xs, r1 = lpcg.pcg_solve(S, lpcg.PC_JACOBI, cuda_f64(b), tol=1e-6, maxit=4 * A.n, max_restarts=4)
    assert r0["status"] == 0 and r1["status"] == 0, (r0, r1)
    assert O.true_relres(A, b, host(xs)) <= 1e-6
    if r0["restarts"] == 0 and r1["restarts"] == 0:
        # rounding differs from the gather form's (one lane sums a row), so
        # the iteration counts of an ill-conditioned system may part by a few
        # percent
        assert abs(r1["iters"] - r0["iters"]) <= max(2, 0.05 * r0["iters"]), (r0["iters"], r1["iters"])


def test_spmv_ell_c3_full_size():
    """64^3 in both orderings with the ELL product in force: IC(0)-PCG (the
    red-black order also through the pair's ELL form) reaches the tolerance
    with the gather form's iterations (within one)."""
    A, b = g.heat_system_3d(64, 1e-3, 1000, 2000)
    for ordering in (0, 1):
        print(f"[spmv ell] heat3d_64 ordering {ordering}", flush=True)
        S = gpu_system(A, None, ordering)
        l, ut, _ = lpcg.ic0(S)
        lpcg.set_trsv_cfg(S, 2, 4, waves=1024)
        _, r0 = lpcg.pcg_solve(S, lpcg.PC_LLT, cuda_f64(b), l_val=l, ut_val=ut, tol=1e-6, max_restarts=2)
        lpcg.set_trsv_cfg(S, 2, 1)
        xs, r1 = lpcg.pcg_solve(S, lpcg.PC_LLT, cuda_f64(b), l_val=l, ut_val=ut, tol=1e-6, max_restarts=2)
        assert r1["status"] == 0 and O.true_relres(A, b, host(xs)) <= 1e-6
        assert abs(r1["iters"] - r0["iters"]) <= 1, (r0["iters"], r1["iters"])


def test_spmv_staged_c3_full_size():
    """64^3 in both orderings: staged and gather products equal bit for bit;
    IC(0)-PCG with the staged product matches the gather form's iterations."""
    A, b = g.heat_system_3d(64, 1e-3, 1000, 2000)
    x = torch.as_tensor(np.random.default_rng(5).standard_normal(A.n).astype(np.float32)).cuda()
    for ordering in (0, 1):
        print(f"[spmv staged] heat3d_64 ordering {ordering}", flush=True)
        S = gpu_system(A, None, ordering)
        l, ut, _ = lpcg.ic0(S)
        lpcg.set_trsv_cfg(S, 2, 4, waves=1024)
        y0 = host(lpcg.spmv(S, x))
        _, r0 = lpcg.pcg_solve(S, lpcg.PC_LLT, cuda_f64(b), l_val=l, ut_val=ut, tol=1e-6, max_restarts=2)
        for R in (256, 1024):
            lpcg.set_trsv_cfg(S, 2, 4, block_rows=R)
            assert np.array_equal(y0.view(np.uint32), host(lpcg.spmv(S, x)).view(np.uint32)), R
            xs, r1 = lpcg.pcg_solve(S, lpcg.PC_LLT, cuda_f64(b), l_val=l, ut_val=ut, tol=1e-6, max_restarts=2)
            assert r1["status"] == 0 and O.true_relres(A, b, host(xs)) <= 1e-6
            assert abs(r1["iters"] - r0["iters"]) <= 1, (R, r0["iters"], r1["iters"])


def test_spmv_fp64_while_staged():
    """The FP64 product has no staged form: with the LDS-staged FP32 form in
    force it runs the gather form on the configured grid, within the FP64
    per-row bound of the oracle (before and after an autotune)."""
    A = matrices_small()["fem_40"]
    S = gpu_system(A)
    x = np.random.default_rng(7).standard_normal(A.n)
    ref = O.spmv(A, x)
    bound = O.spmv(g.CSR(A.n, A.rowptr, A.colind, np.abs(A.val)), np.abs(x))
    k = np.diff(A.rowptr)
    lpcg.set_trsv_cfg(S, 2, 4, block_rows=256)
    y = host(lpcg.spmv(S, cuda_f64(x)))
    assert np.all(np.abs(y - ref) <= 2 * k * 2.0 ** -53 * bound + 1e-300)
    l, ut, _ = lpcg.ic0(S)
    lpcg.autotune(S, l, ut, reps=1)
    assert lpcg.get_trsv_cfg(S, 2)["waves"] >= 1
    y = host(lpcg.spmv(S, cuda_f64(x)))
    assert np.all(np.abs(y - ref) <= 2 * k * 2.0 ** -53 * bound + 1e-300)


def test_spmv_staged_rejects_bad_rows():
    """Rows per block below 64, or more blocks than the partial slots
    (64^3 at 64 rows per block), are refused and the configuration in force
    stays (with its windows)."""
    A, _ = g.heat_system_3d(64, 1e-3, 1, 2)
    S = gpu_system(A)
    x = torch.as_tensor(np.random.default_rng(6).standard_normal(A.n).astype(np.float32)).cuda()
    lpcg.set_trsv_cfg(S, 2, 8, block_rows=512)
    y0 = host(lpcg.spmv(S, x))
    for bad in (32, 64, -1):
        with pytest.raises(lpcg.LpcgError) as e:
            lpcg.set_trsv_cfg(S, 2, 8, block_rows=bad)
        assert e.value.code == lpcg.EINVAL
        assert lpcg.get_trsv_cfg(S, 2)["block_rows"] == 512
    assert np.array_equal(y0.view(np.uint32), host(lpcg.spmv(S, x)).view(np.uint32))


def test_trsv_cfg_rejects_bad_values():
    S = gpu_system(g.poisson_grid(5, 2))
    for bad in [(3, 0, 0, 1), (0, 4, 0, 1), (0, 0, 0, 65), (0, 0, 0, 1, 3), (0, 3, 0, 1, 1, 32),
                (0, 3, 0, 1, 1, 1 << 17), (2, 12, 8), (2, 8, 0), (2, 8, 4096)]:
        with pytest.raises(lpcg.LpcgError) as e:
            lpcg.set_trsv_cfg(S, *bad)
        assert e.value.code == lpcg.EINVAL
    # single-workgroup mode: at most 3 x 1024 rows per level (red-black 80x80: 3200)
    W = gpu_system(g.poisson_grid(80, 2), None, 1)
    assert W.info["max_width_fwd"] > 3072
    with pytest.raises(lpcg.LpcgError) as e:
        lpcg.set_trsv_cfg(W, 0, 2)
    assert e.value.code == lpcg.EINVAL


@pytest.mark.parametrize("transpose", [False, True])
def test_single_workgroup_c3_full_size(transpose):
    """Mode 2 at 64^3 natural order (190 levels, widest 3072 rows): backward
    error against the GPU IC(0) factor."""
    A, b = g.heat_system_3d(64, 1e-3, 1000, 2000)
    pat = O.Pattern(A)
    S = gpu_system(A)
    for d in (0, 1):
        lpcg.set_trsv_cfg(S, d, 2)
    l, ut, _ = lpcg.ic0(S)
    lval = host(l).astype(np.float64)
    rhs = b.astype(np.float32).astype(np.float64)
    y = host(lpcg.sptrsv(S, transpose, l, ut, cuda_f32(rhs))).astype(np.float64)
    L = g.CSR(A.n, pat.lrowptr, pat.lcol, lval).to_scipy()
    T = L.T if transpose else L
    assert np.all(np.abs(rhs - T @ y) <= 4 * 4 * U32 * (abs(T) @ np.abs(y)))


@pytest.mark.parametrize("brows", [1024, 2048])
@pytest.mark.parametrize("transpose", [False, True])
def test_blocked_c3_full_size(transpose, brows):
    """Mode 3 at 64^3 natural order: backward error against the GPU IC(0)
    factor, and the same arithmetic as the dependency-driven mode (the row's
    entries in CSR order), reported."""
    print(f"[blocked] heat3d_64 transpose {transpose} rows {brows}", flush=True)
    A, b = g.heat_system_3d(64, 1e-3, 1000, 2000)
    pat = O.Pattern(A)
    S = gpu_system(A)
    l, ut, _ = lpcg.ic0(S)
    rhs = b.astype(np.float32).astype(np.float64)
    outs = {}
    for mode, br in ((0, 0), (3, brows)):
        for d in (0, 1):
            lpcg.set_trsv_cfg(S, d, mode, 0, 1 if mode == 0 else 0, 1, br)
        outs[mode] = host(lpcg.sptrsv(S, transpose, l, ut, cuda_f32(rhs))).astype(np.float64)
    y = outs[3]
    L = g.CSR(A.n, pat.lrowptr, pat.lcol, host(l).astype(np.float64)).to_scipy()
    T = L.T if transpose else L
    assert np.all(np.abs(rhs - T @ y) <= 4 * 4 * U32 * (abs(T) @ np.abs(y)))
    print("bit-identical to the dependency-driven mode:", np.array_equal(outs[0], y),
          "max rel diff", np.max(np.abs(outs[0] - y) / (np.abs(y) + 1e-30)))


def test_blocked_pcg_c3_full_size():
    """PCG at 64^3 with blocked substitutions in both directions (graph
    captured), also in the XCD-local variant: FP64 true residual and
    iterations equal to the dependency-driven run."""
    A, b = g.heat_system_3d(64, 1e-3, 1000, 2000)
    S = gpu_system(A)
    l, ut, _ = lpcg.ic0(S)
    its = {}
    for mode, br, stride in ((0, 0, 1), (3, 1024, 1), (3, 2048, 8)):
        for d in (0, 1):
            lpcg.set_trsv_cfg(S, d, mode, 0, 1 if mode == 0 else 0, stride, br)
        x, res = lpcg.pcg_solve(S, lpcg.PC_LLT, cuda_f64(b), l_val=l, ut_val=ut, tol=1e-6, max_restarts=2,
                                use_graph=True)
        assert res["status"] == 0 and O.true_relres(A, b, host(x)) <= 1e-6
        its[(mode, stride)] = res["iters"]
    assert abs(its[(3, 1)] - its[(0, 1)]) <= 1 and abs(its[(3, 8)] - its[(0, 1)]) <= 1, its


@pytest.mark.gpu
@pytest.mark.parametrize("transpose", [0, 1])
@pytest.mark.parametrize("brows,runs", [(2048, 2), (2048, 4), (2048, 8), (1024, 4)])
def test_banded_c3_full_size(transpose, brows, runs):
    """Banded blocks (runs of rows one 64^2-row plane apart) at 64^3 natural
    order: bit-identical to the dependency-driven mode (both accumulate a
    row's entries in CSR order) and to consecutive-row blocks."""
    print(f"[banded] heat3d_64 transpose {transpose} rows {brows} runs {runs}", flush=True)
    A, b = g.heat_system_3d(64, 1e-3, 1000, 2000)
    S = gpu_system(A)
    l, ut, _ = lpcg.ic0(S)
    rhs = cuda_f32(b.astype(np.float32).astype(np.float64))
    outs = {}
    for key, (mode, br, k) in {"dep": (0, 0, 1), "blk": (3, brows, 1), "band": (3, brows, runs)}.items():
        for d in (0, 1):
            lpcg.set_trsv_cfg(S, d, mode, 0, 1 if mode == 0 else 0, 1, br, k)
            got = lpcg.get_trsv_cfg(S, d)
            assert got["block_runs"] == (k if mode == 3 else 0)
        outs[key] = host(lpcg.sptrsv(S, transpose, l, ut, rhs))
    assert np.array_equal(outs["band"].view(np.uint32), outs["dep"].view(np.uint32))
    assert np.array_equal(outs["band"].view(np.uint32), outs["blk"].view(np.uint32))


@pytest.mark.gpu
def test_banded_pcg_c3_full_size():
    """PCG at 64^3 with banded blocks in both directions (graph captured,
    fused r.z in the backward solve): FP64 true residual, and iterations
    within one of the dependency-driven and consecutive-block runs (the r.z
    partials are summed per block, so the rounding of beta differs)."""
    A, b = g.heat_system_3d(64, 1e-3, 1000, 2000)
    S = gpu_system(A)
    l, ut, _ = lpcg.ic0(S)
    its = {}
    for key, (mode, br, k) in {"dep": (0, 0, 1), "blk": (3, 2048, 1), "band": (3, 2048, 4)}.items():
        for d in (0, 1):
            lpcg.set_trsv_cfg(S, d, mode, 0, 1 if mode == 0 else 0, 1, br, k)
        x, res = lpcg.pcg_solve(S, lpcg.PC_LLT, cuda_f64(b), l_val=l, ut_val=ut, tol=1e-6, max_restarts=2,
                                use_graph=True)
        assert res["status"] == 0 and O.true_relres(A, b, host(x)) <= 1e-6
        its[key] = res["iters"]
    assert abs(its["band"] - its["dep"]) <= 1 and abs(its["band"] - its["blk"]) <= 1, its


@pytest.mark.gpu
def test_banded_rejected_where_rows_do_not_tile():
    """A 13^3 grid (plane of 169 rows) cannot be cut into banded blocks: the
    configuration is refused and the previous one stays in force."""
    A = matrices_small()["heat3d_13"]
    S = gpu_system(A)
    lpcg.set_trsv_cfg(S, 0, 3, 0, 0, 1, 256, 1)
    with pytest.raises(lpcg.LpcgError) as e:
        lpcg.set_trsv_cfg(S, 0, 3, 0, 0, 1, 256, 4)
    assert e.value.code == lpcg.EINVAL
    got = lpcg.get_trsv_cfg(S, 0)
    assert got["mode"] == 3 and got["block_runs"] == 1
