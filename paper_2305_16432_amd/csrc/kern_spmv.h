// CSR SpMV y = A x (Appendix PCG: w = A p; Method: one round of message
// passing).  G lanes of a wave share one row (G = 4..64 chosen from the mean
// row length), so a wave reads 64/G rows' entries as contiguous runs of the
// value and index arrays; partial row sums are combined with cross-lane
// shuffles.  Bytes per row: 8 per stored entry (FP32 value + int32 index) +
// 4 for the gathered x entry + 4 (row pointer) + 4 (y).
#pragma once

#include "device_util.h"

namespace lpcg {

template <int G, typename AT, typename VT, typename XT>
__device__ __forceinline__ AT row_dot(int a, int b, int sub, const int *__restrict__ ci,
                                      const VT *__restrict__ v, const XT *__restrict__ x) {
    AT acc = 0;
    for (int k = a + sub; k < b; k += G) acc += (AT)v[k] * (AT)x[ci[k]];
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
    return acc;
}

template <int G, typename VT, typename XT>
__global__ void __launch_bounds__(256) k_spmv(int n, const int *__restrict__ rp,
                                              const int *__restrict__ ci, const VT *__restrict__ v,
                                              const XT *__restrict__ x, XT *__restrict__ y) {
    const int sub = threadIdx.x % G;
    const int rows_per_pass = gridDim.x * (blockDim.x / G);
    for (int row = blockIdx.x * (blockDim.x / G) + threadIdx.x / G; row < n; row += rows_per_pass) {
        XT s = row_dot<G, XT>(rp[row], rp[row + 1], sub, ci, v, x);
        if (sub == 0) y[row] = s;
    }
}

}  // namespace lpcg
