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

// ELL form (slot t of row i at t * n + i, W slots, padding adds 0 * x_i):
// one row per lane, entries summed in the row's CSR order; W is a template
// argument so that every slot load is unconditional.
template <int W>
__global__ void __launch_bounds__(256) k_spmv_e(int n, const int *__restrict__ col,
                                                const float *__restrict__ val, const float *__restrict__ x,
                                                float *__restrict__ y) {
    for (int row = blockIdx.x * 256 + threadIdx.x; row < n; row += gridDim.x * 256) {
        // every slot's loads, then every gather, then the sum: two memory
        // round trips per row
        int c[W];
        float v[W], g[W];
#pragma unroll
        for (int t = 0; t < W; ++t) {
            c[t] = col[(size_t)t * n + row];
            v[t] = val[(size_t)t * n + row];
        }
#pragma unroll
        for (int t = 0; t < W; ++t) g[t] = x[c[t]];
        float acc = 0.f;
#pragma unroll
        for (int t = 0; t < W; ++t) acc += v[t] * g[t];
        y[row] = acc;
    }
}

// ---------------------------------------------------------------------------
// LDS-staged input.  Block b owns rows [b R, (b + 1) R) and first copies the
// input over its window of off-diagonal columns, win[2b] .. win[2b + 1]
// (lo > hi: none), into LDS with coalesced loads; the rows then read their
// off-diagonal inputs from LDS and the diagonal's from memory (a row's own
// input lies outside the window in multicolour orders, where a block's rows
// and their neighbours sit in different colours).  Per row the entries are
// summed as in k_spmv (same lanes, order and reduction), so the result is
// the same bit for bit.  Bytes per row: as k_spmv, with the gathered inputs
// replaced by the window (its length over R per row).  The windows are
// computed once per pattern and R (k_spmv_window, factor.hip).

// Copy len (>= 0) inputs g[0 .. len) into LDS, eight loads per thread in
// flight before their stores (loads clamped to the window, stores guarded).
template <typename F>
__device__ __forceinline__ void stage_window(float *sx, int len, F &&load) {
    for (int base = 0; base < len; base += 8 * 256) {
        float t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = load(min(base + u * 256 + (int)threadIdx.x, len - 1));
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = base + u * 256 + (int)threadIdx.x;
            if (i < len) sx[i] = t[u];
        }
    }
}

template <int G>
__global__ void __launch_bounds__(256) k_spmv_st(int n, int R, const int *__restrict__ rp,
                                                 const int *__restrict__ ci, const float *__restrict__ v,
                                                 const float *__restrict__ x, float *__restrict__ y,
                                                 const int *__restrict__ win) {
    extern __shared__ float sx[];
    const int r0 = blockIdx.x * R, r1 = min(n, r0 + R);
    const int lo = win[2 * blockIdx.x], len = win[2 * blockIdx.x + 1] - lo + 1;
    stage_window(sx, len, [&](int i) { return x[lo + i]; });
    __syncthreads();
    const int sub = threadIdx.x % G;
    for (int row = r0 + (int)threadIdx.x / G; row < r1; row += 256 / G) {
        float acc = 0;
        for (int k = rp[row] + sub; k < rp[row + 1]; k += G) {
            const int c = ci[k];
            acc += v[k] * (c == row ? x[row] : sx[c - lo]);
        }
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
        if (sub == 0) y[row] = acc;
    }
}

}  // namespace lpcg
