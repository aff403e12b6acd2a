// Sparse triangular substitution with the factor of P = L L^T (Appendix PCG,
// "Solve P z = r": forward L y = r, then backward L^T z = y).
//
// One launch per solve, dependency driven (no level barriers):
//  * rows are visited in level order (level sets of the analysis), handed
//    out 64 at a time to waves through a ticket counter, so a wave only ever
//    waits on rows that were handed out earlier, to waves already running;
//  * the output vector is preset to the kUnset bit pattern; a row's result,
//    stored with one agent-scope store, is its own ready flag;
//  * a lane issues the loads of all its dependencies at once, consumes the
//    ready prefix, and retries only what is missing (non-blocking inside the
//    wave, so dependencies between lanes of one wave cannot deadlock).
// Bytes per row: 8 per stored entry + 4 (rhs) + 4 (out) + 8 (row pointers)
// + 4 (level-order row id) + 4 per dependency value read.
#pragma once

#include "device_util.h"

namespace lpcg {

constexpr int kTrsvBatch = 8;
constexpr int kTrsvRegDeps = 8;  // rows with at most this many dependencies keep them in registers

// Solves one chunk of 64 rows of the level order starting at `base`.
// UPPER = 0: L in lower CSR, diagonal last; UPPER = 1: U = L^T in upper CSR,
// diagonal first.  Returns (per lane) the row solved (-1 if none) and its value.
//
// A row with at most kTrsvRegDeps dependencies loads its column indices and
// values into registers once, then each round re-reads all its dependency
// values with independent loads (one memory round trip per round) and, once
// none is unset, accumulates them in column order (fixed order: results are
// bit-reproducible).  Longer rows consume the ready prefix of their entries in
// batches of kTrsvBatch.
template <bool UPPER>
__device__ __forceinline__ int trsv_chunk(int n, int base, const int *__restrict__ order,
                                          const int *__restrict__ rp, const int *__restrict__ ci,
                                          const float *__restrict__ v, const float *__restrict__ rhs,
                                          uint32_t *ybits, float &yout, int backoff) {
    const int pos = base + lane_id();
    int row = -1, k = 0, kend = 0;
    float acc = 0.f, dg = 1.f;
    if (pos < n) {
        row = order[pos];
        const int a = rp[row], b = rp[row + 1];
        if (UPPER) {
            dg = v[a];
            k = a + 1;
            kend = b;
        } else {
            dg = v[b - 1];
            k = a;
            kend = b - 1;
        }
        acc = rhs[row];
    }
    const int nd = kend - k;
    const bool in_regs = nd <= kTrsvRegDeps;
    int cj[kTrsvRegDeps];
    float vj[kTrsvRegDeps];
#pragma unroll
    for (int t = 0; t < kTrsvRegDeps; ++t) {
        cj[t] = 0;
        vj[t] = 0.f;
        if (in_regs && t < nd) {
            cj[t] = ci[k + t];
            vj[t] = v[k + t];
        }
    }
    bool pending = row >= 0;
    while (__ballot(pending) != 0) {
        if (pending) {
            if (in_regs) {
                uint32_t got[kTrsvRegDeps];
#pragma unroll
                for (int t = 0; t < kTrsvRegDeps; ++t) got[t] = t < nd ? ld_agent(&ybits[cj[t]]) : 0u;
                bool ready = true;
#pragma unroll
                for (int t = 0; t < kTrsvRegDeps; ++t) ready = ready && (got[t] != kUnset);
                if (ready) {
#pragma unroll
                    for (int t = 0; t < kTrsvRegDeps; ++t)
                        if (t < nd) acc -= vj[t] * __uint_as_float(got[t]);
                    k = kend;
                }
            } else {
                while (k < kend) {
                    uint32_t got[kTrsvBatch];
                    const int m = min(kTrsvBatch, kend - k);
#pragma unroll
                    for (int t = 0; t < kTrsvBatch; ++t)
                        if (t < m) got[t] = ld_agent(&ybits[ci[k + t]]);
                    int used = 0;
#pragma unroll
                    for (int t = 0; t < kTrsvBatch; ++t) {
                        if (t < m && used == t && got[t] != kUnset) {
                            acc -= v[k + t] * __uint_as_float(got[t]);
                            ++used;
                        }
                    }
                    k += used;
                    if (used < m) break;
                }
            }
            if (k == kend) {
                const float yv = acc / dg;
                st_agent(&ybits[row], publishable(yv));
                yout = yv;
                pending = false;
            }
        }
        // back off between polling rounds (fewer polls in flight shorten
        // the latency of the stores being waited for)
        if (pending)
            for (int t = 0; t < backoff; ++t) __builtin_amdgcn_s_sleep(1);
    }
    return row;
}

template <bool UPPER>
__global__ void __launch_bounds__(256) k_sptrsv(int n, const int *__restrict__ order,
                                                const int *__restrict__ rp, const int *__restrict__ ci,
                                                const float *__restrict__ v,
                                                const float *__restrict__ rhs, uint32_t *ybits,
                                                int *ticket, int backoff, int stride) {
    if (blockIdx.x % stride != 0) return;  // placement: only every stride-th block works
    for (;;) {
        const int chunk = wave_ticket(ticket);
        if ((long)chunk * kWave >= n) break;
        float yv;
        trsv_chunk<UPPER>(n, chunk * kWave, order, rp, ci, v, rhs, ybits, yv, backoff);
    }
}

// ---------------------------------------------------------------------------
// Level-synchronous substitution: one launch per level (launch order is the
// only synchronisation, so loads and stores are plain).  G lanes share a row;
// the rows of a level are order[0 .. rows).  Returns the row's solution in
// lane sub == 0 of its group.  Accumulation: G strided partial sums combined
// by a shuffle tree (fixed order, bit-reproducible for a given G).
template <bool UPPER, int G>
__device__ __forceinline__ float trsv_level_row(int row, int sub, const int *__restrict__ rp,
                                                const int *__restrict__ ci, const float *__restrict__ v,
                                                const float *__restrict__ rhs, const float *__restrict__ y) {
    const int a = rp[row], b = rp[row + 1];
    const int k0 = UPPER ? a + 1 : a, k1 = UPPER ? b : b - 1;
    float acc = 0.f;
    for (int k = k0 + sub; k < k1; k += G) acc += v[k] * y[ci[k]];
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
    return (rhs[row] - acc) / v[UPPER ? a : b - 1];
}

template <bool UPPER, int G>
__global__ void __launch_bounds__(256) k_trsv_level(int rows, const int *__restrict__ order,
                                                    const int *__restrict__ rp, const int *__restrict__ ci,
                                                    const float *__restrict__ v, const float *__restrict__ rhs,
                                                    float *__restrict__ y) {
    const int sub = threadIdx.x % G;
    constexpr int per = 256 / G;
    for (int idx = blockIdx.x * per + threadIdx.x / G; idx < rows; idx += gridDim.x * per) {
        const int row = order[idx];
        const float yv = trsv_level_row<UPPER, G>(row, sub, rp, ci, v, rhs, y);
        if (sub == 0) y[row] = yv;
    }
}

// Blocks of one level launch: enough for the level's rows, at most one per
// 64 rows (so the per-block partial sums of a whole solve number at most
// chunks + levels).
inline int level_blocks(int rows, int G) {
    const int per = 256 / G;
    const int want = (rows + per - 1) / per;
    const int cap = (rows + 63) / 64;
    return want < cap ? want : cap;
}

static __global__ void k_fill_u32(int n, uint32_t *p, uint32_t v) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Number of waves for a dependency-driven launch: the requested count (0:
// 4096), never more than there are chunks.
inline int trsv_waves(int n, int want = 0) {
    const int chunks = (n + kWave - 1) / kWave;
    const int w = want > 0 ? want : 4096;
    return chunks < w ? chunks : w;
}

}  // namespace lpcg

// ---------------------------------------------------------------------------
// Single-workgroup substitution (mode 2): one block of kWgThreads threads
// walks every level, with a block barrier between levels, on the level-
// ordered packed pattern (lo_ptr/lo_col/lo_val/lo_diag of lpcg_system;
// level position q holds row rows[q]).  Communication stays inside one CU, so
// a level costs a block barrier and the y gathers instead of a cross-CU
// signal.  Loads that do not depend on y are software-pipelined: entry ranges,
// rows and diagonals two levels ahead, columns, values and right-hand sides
// one level ahead.  A thread handles at most kWgRows rows of a level (so the
// widest level may have kWgRows * kWgThreads rows); entries beyond kWgEnt per
// row are loaded inline.  Accumulation in entry (column) order.
constexpr int kWgThreads = 1024;
constexpr int kWgRows = 3;
constexpr int kWgEnt = 4;

struct WgA {  // stage A: per row of a level
    int row[kWgRows], e0[kWgRows], ne[kWgRows];
    float diag[kWgRows];
};
struct WgB {  // stage B: entries and right-hand side
    int col[kWgRows][kWgEnt];
    float val[kWgRows][kWgEnt];
    float rhs[kWgRows];
};

__device__ __forceinline__ void wg_load_a(WgA &A, int q0, int q1, const int *__restrict__ rows,
                                          const int *__restrict__ ptr, const float *__restrict__ diag) {
#pragma unroll
    for (int r = 0; r < kWgRows; ++r) {
        const int q = q0 + (int)threadIdx.x + r * kWgThreads;
        if (q < q1) {
            A.row[r] = rows[q];
            A.e0[r] = ptr[q];
            A.ne[r] = ptr[q + 1] - A.e0[r];
            A.diag[r] = diag[q];
        } else {
            A.row[r] = -1;
            A.e0[r] = 0;
            A.ne[r] = 0;
            A.diag[r] = 1.f;
        }
    }
}

__device__ __forceinline__ void wg_load_b(WgB &B, const WgA &A, const int *__restrict__ col,
                                          const float *__restrict__ val, const float *__restrict__ rhs) {
#pragma unroll
    for (int r = 0; r < kWgRows; ++r) {
#pragma unroll
        for (int j = 0; j < kWgEnt; ++j) {
            const bool ok = j < A.ne[r];
            B.col[r][j] = ok ? col[A.e0[r] + j] : 0;
            B.val[r][j] = ok ? val[A.e0[r] + j] : 0.f;
        }
        B.rhs[r] = A.row[r] >= 0 ? rhs[A.row[r]] : 0.f;
    }
}

// Solve the rows of one level; returns sum over this thread's rows of
// w[row] * y[row] when w is given (the r.z partial of the backward solve).
__device__ __forceinline__ double wg_solve(const WgA &A, const WgB &B, const int *__restrict__ col,
                                           const float *__restrict__ val, float *y, const float *w) {
    double dot = 0.0;
#pragma unroll
    for (int r = 0; r < kWgRows; ++r) {
        if (A.row[r] < 0) continue;
        float acc = 0.f;
#pragma unroll
        for (int j = 0; j < kWgEnt; ++j)
            if (j < A.ne[r]) acc += B.val[r][j] * y[B.col[r][j]];
        for (int j = kWgEnt; j < A.ne[r]; ++j) acc += val[A.e0[r] + j] * y[col[A.e0[r] + j]];
        const float yv = (B.rhs[r] - acc) / A.diag[r];
        y[A.row[r]] = yv;
        if (w) dot += (double)w[A.row[r]] * (double)yv;
    }
    return dot;
}

// Whole substitution in the calling block (all threads call; contains block
// barriers).  lev_ptr is the device level pointer array (nlev + 1 entries).
__device__ __forceinline__ double wg_substitute(int nlev, const int *__restrict__ lev_ptr,
                                                const int *__restrict__ rows, const int *__restrict__ ptr,
                                                const int *__restrict__ col, const float *__restrict__ val,
                                                const float *__restrict__ diag, const float *__restrict__ rhs,
                                                float *y, const float *w) {
    WgA A0, A1, A2;
    WgB B0, B1;
    wg_load_a(A0, lev_ptr[0], lev_ptr[1], rows, ptr, diag);
    wg_load_b(B0, A0, col, val, rhs);
    if (nlev > 1) wg_load_a(A1, lev_ptr[1], lev_ptr[2], rows, ptr, diag);
    double dot = 0.0;
    for (int l = 0; l < nlev; ++l) {
        if (l + 1 < nlev) wg_load_b(B1, A1, col, val, rhs);
        if (l + 2 < nlev) wg_load_a(A2, lev_ptr[l + 2], lev_ptr[l + 3], rows, ptr, diag);
        dot += wg_solve(A0, B0, col, val, y, w);
        __syncthreads();
        A0 = A1;
        A1 = A2;
        B0 = B1;
    }
    return dot;
}

static __global__ void __launch_bounds__(kWgThreads) k_trsv_wg(int nlev, const int *__restrict__ lev_ptr,
                                                        const int *__restrict__ rows, const int *__restrict__ ptr,
                                                        const int *__restrict__ col, const float *__restrict__ val,
                                                        const float *__restrict__ diag,
                                                        const float *__restrict__ rhs, float *y) {
    wg_substitute(nlev, lev_ptr, rows, ptr, col, val, diag, rhs, y, nullptr);
}

// Values of one factor in level-ordered packed form: val_lo[e] = v[src[e]],
// diag_lo[q] = v[dsrc[q]].
static __global__ void k_lo_prep(int noff, int n, const int *__restrict__ src, const int *__restrict__ dsrc,
                          const float *__restrict__ v, float *__restrict__ val_lo, float *__restrict__ diag_lo) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < noff) val_lo[i] = v[src[i]];
    if (i < n) diag_lo[i] = v[dsrc[i]];
}
