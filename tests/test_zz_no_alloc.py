"""lpcg_ic0_noalloc (IC(0) with the library's static device scratch, for
callers that cannot allocate) against lpcg_ic0 on the same systems: two
calls in a row, the second on a smaller system, each bit-identical to the
allocating entry point (same kernels, same FP64 order) and within the IC(0)
bar of the oracle; a system above the scratch limit is refused with EINVAL."""
import numpy as np
import pytest
import torch

import oracle as O
import pdegen as g
from paper_2305_16432_amd import lpcg
from tests.gpu_util import U32, gpu_system, host

pytestmark = pytest.mark.gpu


def _case(A):
    S = gpu_system(A)
    l_ref, ut_ref, sh_ref = lpcg.ic0(S)
    l_na, ut_na, sh_na = lpcg.ic0_noalloc(S)
    torch.cuda.synchronize()
    assert sh_na == sh_ref
    assert torch.equal(l_na, l_ref) and torch.equal(ut_na, ut_ref)
    pat = O.Pattern(A)
    lo, _ = O.ic0(pat, A)
    lg = host(l_na).astype(np.float64)
    assert np.all(np.abs(lg - lo) <= 1.0001 * U32 * np.abs(lo))
    return S


def test_ic0_noalloc_matches_ic0_twice_then_smaller():
    print("[no-alloc] heat3d 40^3 then 2D FEM 30", flush=True)
    A1, _ = g.heat_system_3d(40, 1e-3, 11, 12)
    _case(A1)
    A2 = g.fem_p1_delaunay(30, 3, 4)[0]
    _case(A2)
    # and once more on the larger system after the smaller one
    _case(A1)


def test_ic0_noalloc_shift_retry_matches():
    # an indefinite-ish SPD pattern where IC(0) needs a shift: same retries
    A = g.random_spd(600, 0.05, 9, dominance=0.05)
    S = gpu_system(A)
    try:
        l_ref, _, sh_ref = lpcg.ic0(S)
    except lpcg.LpcgError as e:
        with pytest.raises(lpcg.LpcgError) as ei:
            lpcg.ic0_noalloc(S)
        assert ei.value.code == e.code
        return
    l_na, _, sh_na = lpcg.ic0_noalloc(S)
    assert sh_na == sh_ref and torch.equal(l_na, l_ref)


def test_ic0_noalloc_refuses_above_limit():
    A = g.poisson_grid(90, 3)  # nnz_l = 2,916,000 > 2,097,152
    S = gpu_system(A)
    assert S.info["nnz_l"] > lpcg.IC0_NOALLOC_MAX_NNZ_L
    with pytest.raises(lpcg.LpcgError) as ei:
        lpcg.ic0_noalloc(S)
    assert ei.value.code == lpcg.EINVAL
    assert "scratch limit" in str(ei.value)
