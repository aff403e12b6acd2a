"""lpcg_check_factor: a factor passes when every diagonal entry is a positive
finite number and every entry is finite; otherwise the first offending row
(internal numbering) is reported with ENONFINITE.  Bit-exact (integer
result)."""
import numpy as np
import pytest
import torch

import pdegen as g
from paper_2305_16432_amd import lpcg
from tests.gpu_util import cuda_f32, gpu_system, host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("ordering", [0, 1])
def test_check_factor(ordering):
    A = g.heat_system_3d(9, 1e-3, 1, 2)[0]
    S = gpu_system(A, None, ordering)
    l, ut, _ = lpcg.ic0(S)
    assert lpcg.check_factor(S, l) == (True, -1)
    pat_rp = host(lpcg.export_pattern(S)["lrowptr"])  # rows in the internal numbering
    lh = host(l).copy()
    rng = np.random.default_rng(0)
    for kind in ("nan_offdiag", "neg_diag", "inf_diag", "zero_diag"):
        rows = sorted(rng.choice(np.arange(1, A.n), 3, replace=False))
        bad = lh.copy()
        for r in rows:
            d = pat_rp[r + 1] - 1
            if kind == "nan_offdiag":
                bad[pat_rp[r]] = np.nan
            elif kind == "neg_diag":
                bad[d] = -1.0
            elif kind == "inf_diag":
                bad[d] = np.inf
            else:
                bad[d] = 0.0
        ok, row = lpcg.check_factor(S, cuda_f32(bad))
        assert not ok and row == rows[0], (kind, row, rows)
