"""The blocked substitution's schedule (host logic of the library, no GPU).

A solve emulated in FP64 from the schedule alone -- blocks in order, chunks in
order, each row from its record (dependency codes, the factor's values
through vsrc, the diagonal) -- must reproduce the oracle's substitution bit
for bit: both accumulate a row's entries in CSR order.  Structural checks:
every row appears exactly once, chunks hold at most 64 rows of one block,
an in-block dependency is produced in an earlier chunk of the same block, a
global one in an earlier block.  Banded blocks (several runs of rows one
stride apart) are checked the same way, through the schedule's position map."""
import numpy as np
import pytest

import oracle as O
import pdegen as g
from paper_2305_16432_amd import lpcg
from tests.gpu_util import matrices_small


def _emulate(S, n, vals, rhs):
    w = S["deps"]
    lsh, D = S["run_shift"], S["run_stride"]
    y = np.full(n, np.nan)
    block_of = np.full(n, -1)
    chunk_of = np.full(n, -1)
    seen = np.zeros(n, np.int64)
    for b in range(S["nblocks"]):
        r0, nr = S["brow"][b]

        def at(x):  # row of position x of this block
            return r0 + (x >> lsh) * D + (x & ((1 << lsh) - 1))
        rows = [at(x) for x in range(nr)]
        assert all(block_of[r] == -1 for r in rows) and rows == sorted(rows)
        block_of[rows] = b
        for c in range(S["bch"][b], S["bch"][b + 1]):
            p0, cnt = S["chunks"][c]
            assert 1 <= cnt <= 64 and 0 <= p0 and p0 + cnt <= nr
            for p in range(p0, p0 + cnt):
                rec = S["rec"][at(p)]
                vs = S["vsrc"][at(p)]
                assert 0 <= rec[w] < nr
                row = at(rec[w])
                seen[row] += 1
                acc = rhs[row]
                for t in range(w):
                    code = rec[t]
                    if code == -1:
                        assert vs[t] == -1
                        continue
                    dep = code if code >= 0 else at(-2 - code)
                    if code >= 0:
                        assert block_of[dep] != -1 and block_of[dep] < b, "global dependency not in an earlier block"
                    else:
                        assert chunk_of[dep] != -1 and chunk_of[dep] < c, "in-block dependency not in an earlier chunk"
                    acc -= vals[vs[t]] * y[dep]
                y[row] = acc / vals[vs[w]]
                chunk_of[row] = c
    assert np.all(seen == 1)
    return y


@pytest.mark.parametrize("brows", [64, 256, 1024])
@pytest.mark.parametrize("name", ["one", "tridiag_1000", "poisson2d_32", "poisson3d_9", "heat3d_13", "fem_40"])
def test_schedule_reproduces_substitution(name, brows):
    A = matrices_small()[name]
    pat = O.Pattern(A)
    rng = np.random.default_rng(7)
    lval = rng.uniform(-0.3, 0.3, pat.nnz_l)
    row = np.repeat(np.arange(A.n), np.diff(pat.lrowptr))
    lval[pat.lcol == row] = rng.uniform(1.0, 2.0, (pat.lcol == row).sum())
    rhs = rng.standard_normal(A.n)
    for upper in (False, True):
        rp, ci = (pat.urowptr, pat.ucol) if upper else (pat.lrowptr, pat.lcol)
        vals = pat.upper_values(lval) if upper else lval
        S = lpcg.blocked_schedule(rp, ci, upper, brows)
        assert S["deps"] == (3 if np.diff(rp).max() - 1 <= 3 else 7)
        assert S["nblocks"] == -(-A.n // brows)
        y = _emulate(S, A.n, vals, rhs)
        ref = O.trsv_upper(pat, lval, rhs) if upper else O.trsv_lower(pat, lval, rhs)
        np.testing.assert_array_equal(y, ref)


def test_schedule_levels_of_a_plane_block():
    """64^3-like structure at 16^3: a block of one plane (256 rows) has
    16 + 16 - 1 in-block levels, one chunk each (at most 16 rows per level)."""
    A = g.poisson_grid(16, 3)
    pat = O.Pattern(A)
    S = lpcg.blocked_schedule(pat.lrowptr, pat.lcol, False, 256)
    assert S["nblocks"] == 16
    assert all(S["bch"][b + 1] - S["bch"][b] == 31 for b in range(16))


def test_schedule_rejects():
    A = matrices_small()["random_777"]  # rows with more than 7 dependencies
    pat = O.Pattern(A)
    with pytest.raises(lpcg.LpcgError) as e:
        lpcg.blocked_schedule(pat.lrowptr, pat.lcol, False, 256)
    assert e.value.code == lpcg.EINVAL
    B = matrices_small()["heat3d_13"]
    pb = O.Pattern(B)
    for bad in (32, 1 << 17):
        with pytest.raises(lpcg.LpcgError):
            lpcg.blocked_schedule(pb.lrowptr, pb.lcol, False, bad)


def _factor(A, seed=7):
    pat = O.Pattern(A)
    rng = np.random.default_rng(seed)
    lval = rng.uniform(-0.3, 0.3, pat.nnz_l)
    row = np.repeat(np.arange(A.n), np.diff(pat.lrowptr))
    lval[pat.lcol == row] = rng.uniform(1.0, 2.0, (pat.lcol == row).sum())
    return pat, lval, rng.standard_normal(A.n)


@pytest.mark.parametrize("m,brows,runs", [(8, 64, 2), (8, 128, 2), (8, 128, 4), (8, 256, 4),
                                          (16, 256, 4), (16, 512, 4), (16, 512, 8), (16, 1024, 4)])
def test_banded_schedule_reproduces_substitution(m, brows, runs):
    """Banded blocks on an m^3 grid (runs one plane, m^2 rows, apart): both
    directions reproduce the oracle bit for bit, and every block is a band of
    `runs` consecutive planes."""
    A = g.poisson_grid(m, 3)
    pat, lval, rhs = _factor(A)
    for upper in (False, True):
        rp, ci = (pat.urowptr, pat.ucol) if upper else (pat.lrowptr, pat.lcol)
        vals = pat.upper_values(lval) if upper else lval
        S = lpcg.blocked_schedule(rp, ci, upper, brows, runs)
        assert S["run_stride"] == m * m and (1 << S["run_shift"]) == brows // runs
        assert S["nblocks"] == A.n // brows
        y = _emulate(S, A.n, vals, rhs)
        ref = O.trsv_upper(pat, lval, rhs) if upper else O.trsv_lower(pat, lval, rhs)
        np.testing.assert_array_equal(y, ref)


def test_banded_schedule_level_count():
    """A block of 4 planes x 4 y-rows x 16 x-rows of the 16^3 grid: its
    in-block levels are x + y + z, 15 + 3 + 3 + 1 = 22, each one chunk."""
    A = g.poisson_grid(16, 3)
    pat = O.Pattern(A)
    S = lpcg.blocked_schedule(pat.lrowptr, pat.lcol, False, 256, 4)
    assert S["nblocks"] == 16
    assert all(S["bch"][b + 1] - S["bch"][b] == 22 for b in range(16))


def test_banded_schedule_rejects():
    """Banded blocks that cannot tile the rows, or whose order would make a
    block wait on a later one, are refused (EINVAL)."""
    B = matrices_small()["heat3d_13"]  # plane of 169 rows: no power-of-two run divides it
    pb = O.Pattern(B)
    with pytest.raises(lpcg.LpcgError) as e:
        lpcg.blocked_schedule(pb.lrowptr, pb.lcol, False, 256, 4)
    assert e.value.code == lpcg.EINVAL
    # n = 256, every row depends on rows r - 1 and r - 64 (stride 64, runs of
    # 32): the first row of a run depends on the last row of the run before,
    # which lies in that run's last band, a later block than band 0
    rows, cols = [], []
    for r in range(256):
        for c in [c for c in (r - 64, r - 1) if c >= 0] + [r]:
            rows.append(r)
            cols.append(c)
    rp = np.zeros(257, np.int32)
    np.add.at(rp, np.asarray(rows) + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    with pytest.raises(lpcg.LpcgError) as e:
        lpcg.blocked_schedule(rp, np.asarray(cols, np.int32), False, 64, 2)
    assert e.value.code == lpcg.EINVAL


@pytest.mark.parametrize("brows,runs", [(128, 2), (256, 4), (512, 8)])
def test_banded_schedule_on_a_batch(brows, runs):
    """Banded blocks over a block-diagonal batch of four 8^3 heat steps (the
    stride is one 64-row plane; bands never need to cross a system): both
    directions reproduce the oracle bit for bit."""
    mats = [g.heat_system_3d(8, 1e-3, 50 + i, 60 + i)[0] for i in range(4)]
    B, _ = g.block_diag_csr(mats)
    pat, lval, rhs = _factor(B, seed=11)
    for upper in (False, True):
        rp, ci = (pat.urowptr, pat.ucol) if upper else (pat.lrowptr, pat.lcol)
        vals = pat.upper_values(lval) if upper else lval
        S = lpcg.blocked_schedule(rp, ci, upper, brows, runs)
        assert S["run_stride"] == 64 and S["nblocks"] == B.n // brows
        y = _emulate(S, B.n, vals, rhs)
        ref = O.trsv_upper(pat, lval, rhs) if upper else O.trsv_lower(pat, lval, rhs)
        np.testing.assert_array_equal(y, ref)


def _tri_solve(rp, ci, vals, rhs, upper):
    """Row-by-row substitution in CSR order (the definition), FP64."""
    n = len(rp) - 1
    y = np.zeros(n)
    for r in (range(n - 1, -1, -1) if upper else range(n)):
        acc, dg = rhs[r], None
        for k in range(rp[r], rp[r + 1]):
            if ci[k] == r:
                dg = vals[k]
            else:
                acc -= vals[k] * y[ci[k]]
        y[r] = acc / dg
    return y


def test_banded_schedules_of_random_patterns():
    """Random lower patterns on 512 rows (each row depends on a random subset
    of up to three offsets from a grid-like menu, the longest being 64) and
    their transposes, with random block sizes and run counts: every schedule
    the builder accepts keeps each cross-block dependency on an earlier
    block (checked by the emulation) and reproduces the substitution bit for
    bit; the ones it refuses are refused with EINVAL.  Both outcomes occur."""
    rng = np.random.default_rng(2024)
    n, menu = 512, [1, 2, 7, 8, 9, 56, 63, 64]
    accepted = refused = 0
    for case in range(24):
        offs = rng.choice(menu, size=rng.integers(1, 4), replace=False)
        offs = np.append(offs[offs != 64], 64)[-3:]  # the longest offset is 64
        rows, cols = [], []
        for r in range(n):
            deps = sorted({r - int(o) for o in offs if r - int(o) >= 0 and rng.random() < 0.9})
            rows += [r] * (len(deps) + 1)
            cols += deps + [r]
        rp = np.zeros(n + 1, np.int64)
        np.add.at(rp, np.asarray(rows) + 1, 1)
        rp = np.cumsum(rp)
        ci = np.asarray(cols, np.int64)
        vals = rng.uniform(-0.3, 0.3, len(ci))
        vals[ci == np.asarray(rows)] = rng.uniform(1.0, 2.0, n)
        rhs = rng.standard_normal(n)
        import scipy.sparse as sp
        L = sp.csr_matrix((vals, ci, rp), shape=(n, n))
        U = L.T.tocsr()
        U.sort_indices()
        brows = int(rng.choice([64, 128, 256]))
        runs = int(rng.choice([2, 4, 8]))
        for upper, M in ((False, L), (True, U)):
            try:
                S = lpcg.blocked_schedule(M.indptr.astype(np.int32), M.indices.astype(np.int32), upper, brows, runs)
            except lpcg.LpcgError as e:
                assert e.code == lpcg.EINVAL
                refused += 1
                continue
            accepted += 1
            y = _emulate(S, n, M.data, rhs)
            np.testing.assert_array_equal(y, _tri_solve(M.indptr, M.indices, M.data, rhs, upper))
    assert accepted > 0 and refused > 0, (accepted, refused)
