"""Seeded synthetic PDE systems and random inputs.

This module produces the *inputs* of the learned-preconditioner PCG method:
sparse SPD stiffness matrices from discretised second-order PDEs (the
problem class of the paper's Preliminaries: Galerkin/finite-difference
discretisations of elliptic and parabolic equations with Dirichlet
boundaries), right-hand sides, random coefficient fields, random DAGs and
random network weights.  It holds none of the method's arithmetic (no PCG,
no triangular solve, no factorisation, no network evaluation): both the HIP
path and the CPU oracle consume what it returns, so both see identical data.

All matrices are returned in canonical CSR: int32 row pointers and column
indices, columns sorted ascending within each row, duplicates summed, the
diagonal always stored, float64 values.
"""
from .csr import CSR, canonical_csr, csr_from_dense, block_diag_csr, permute_csr
from .grf import grf
from .systems import (tridiag_1d, poisson_grid, bipartite_grid, heat_step_3d, heat_system_3d, fem_p1_delaunay,
                      random_spd, random_lower_dag, mixed_batch, mixed_batch_member, mixed_batch_sizes,
                      mixed_batch_parallel)
from .weights import gnn_param_shapes, init_gnn_params

__all__ = [
    "CSR", "canonical_csr", "csr_from_dense", "block_diag_csr", "permute_csr",
    "grf", "tridiag_1d", "poisson_grid", "bipartite_grid", "heat_step_3d", "heat_system_3d", "fem_p1_delaunay",
    "random_spd", "random_lower_dag", "mixed_batch", "mixed_batch_member", "mixed_batch_sizes",
    "mixed_batch_parallel", "gnn_param_shapes", "init_gnn_params",
]
