"""Shared helpers for the GPU parity tests (test-side only)."""
import numpy as np
import torch

import oracle as O
import pdegen as g
from paper_2305_16432_amd import lpcg

U32 = 2.0 ** -24
U64 = 2.0 ** -53


def cuda_i32(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def cuda_f64(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def cuda_f32(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def gpu_system(A, sys_rowptr=None, ordering=0):
    return lpcg.analyze(cuda_i32(A.rowptr), cuda_i32(A.colind), cuda_f64(A.val), sys_rowptr, ordering)


def matrices_small():
    """Named small systems spanning several waves, ragged tails and the
    degenerate shapes (1x1, tridiagonal chain, dense-ish rows)."""
    out = {
        "one": g.csr_from_dense(np.array([[3.0]])),
        "tridiag_1000": g.tridiag_1d(1000),
        "poisson2d_32": g.poisson_grid(32, 2),
        "poisson3d_9": g.poisson_grid(9, 3),
        "heat3d_13": g.heat_system_3d(13, 1e-3, 5, 6)[0],
        "fem_40": g.fem_p1_delaunay(40, 1, 2)[0],
        "random_777": g.random_spd(777, 0.01, 3),
        "dag_60": g.random_lower_dag(60, 0.2, 4),
        "bipartite_24": g.bipartite_grid(24),
    }
    return out
