// Sparse triangular substitution with the factor of P = L L^T (Appendix PCG,
// "Solve P z = r": forward L y = r, then backward L^T z = y).  Four modes,
// chosen per direction by the autotuner: dependency driven (below), level
// synchronous, single workgroup, and blocked (sections further down).  Every
// mode accumulates a row's entries in CSR order.
//
// Dependency-driven mode, one launch per solve (no level barriers):
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

namespace lpcg {

// ---------------------------------------------------------------------------
// Blocked substitution (mode 3).  The rows are cut into blocks of B rows, taken
// in solve order (ascending for L, descending for L^T); one wave owns a block,
// blocks are handed out through a ticket in that order.  A block is either B
// consecutive rows or, banded, K runs of B/K consecutive rows that lie a fixed
// stride apart (the pattern's longest dependency, one grid plane on a
// natural-order grid), so that several planes of a band share a wave and their
// plane-to-plane dependencies stay in its LDS.  A host-built schedule lists a
// block's rows by their level inside the block (longest path over in-block
// dependencies), in chunks of at most 64 rows of one level.  The wave copies
// its block's records and right-hand side into LDS once, then walks the
// chunks: in-block dependencies are read from LDS; dependencies on rows of
// earlier blocks are polled from global memory (the value is its own ready
// flag, as in the dependency-driven mode), their loads issued kBlkDist chunks
// ahead in a register ring.  Every load of the ring is unconditional (slots
// without such a dependency read entry 0 and ignore it) so that the waits for
// one chunk leave the later chunks' loads in flight.  Accumulation follows the
// row's CSR order, as in the other modes.
//
// Record of a row (2W + 2 words, W = 3 or 7 dependencies at most): words
// [0, W) dependency codes (>= 0: global row; -1: none; <= -2: in-block row
// of slot -2 - code), word W the row's slot in the block, words W+1 .. 2W
// the values, word 2W + 1 the diagonal.  A slot x of block b is the row
// blk_row(x): its rows ascending.  Record p of block b (schedule order) is
// stored at global position blk_row(p), so the blocks' records tile [0, n).
// The values are packed per factor by k_blk_pack.
constexpr int kBlkDist = 2;

// Schedule of one direction (device arrays).
struct BlkSched {
    const int *brow;  // [2 nb]: first (smallest) row and row count of block b
    const int *bch;   // [nb + 1]: chunk range of block b
    const int2 *ch;   // chunk table: first record (relative to the block) and rows
    const int *rec;   // [n * (2W + 2)] records, block b's at its rows' positions
    int nb, bmax, chmax;
    int lsh, dstride;  // runs of 2^lsh rows, dstride apart (one run: lsh >= log2 B)
};

// Row of slot (or stored record) x of the block whose first row is r0.
__device__ __forceinline__ int blk_row(const BlkSched &S, int r0, int x) {
    return r0 + (x >> S.lsh) * S.dstride + (x & ((1 << S.lsh) - 1));
}

template <int W>
struct BlkSlot {
    int code[W];
    int row;
    float val[W];
    float dg, rhs, rr;
    uint32_t gv[W];
    bool act;
};

// Record of chunk c for this lane; cc = the chunk's table entry (read one
// step earlier, so the record read does not wait on it).
template <int W>
__device__ __forceinline__ void blk_read(BlkSlot<W> &q, const int *rec, int2 cc, int c, int nch) {
    constexpr int RW = 2 * W + 2;
    const int l = lane_id();
    q.act = c < nch && l < cc.y;
    const int p = cc.x + min(l, cc.y - 1);
    const int4 *r4 = reinterpret_cast<const int4 *>(rec + p * RW);
    int w[RW];
#pragma unroll
    for (int i = 0; i < RW / 4; ++i) {
        const int4 t = r4[i];
        w[4 * i] = t.x;
        w[4 * i + 1] = t.y;
        w[4 * i + 2] = t.z;
        w[4 * i + 3] = t.w;
    }
#pragma unroll
    for (int t = 0; t < W; ++t) {
        q.code[t] = w[t];
        q.val[t] = __int_as_float(w[W + 1 + t]);
    }
    q.row = w[W];
    q.dg = __int_as_float(w[2 * W + 1]);
}

template <int W, bool RZ>
__device__ __forceinline__ void blk_issue(BlkSlot<W> &q, const float *rsh, const uint32_t *ybits,
                                          const float *rrsh) {
    q.rhs = rsh[q.row];
    if constexpr (RZ) q.rr = rrsh[q.row];
#pragma unroll
    for (int t = 0; t < W; ++t) q.gv[t] = ld_agent(&ybits[max(q.code[t], 0)]);
}

// Solve one chunk; returns the lane's solution value (0 for idle lanes).
// Values the prefetch found unset are re-read one by one until published.
// Idle lanes hold the record of the chunk's last row (blk_read clamps them
// to it), so they wait for the same values, compute the same result and
// store the same bits to the same places.  The stores therefore need no
// branch, and the compiler can count them among the memory operations in
// flight, so its waits keep the prefetched chunks in flight.
template <int W>
__device__ __forceinline__ float blk_process(BlkSlot<W> &q, float *ysh, const BlkSched &S, int r0,
                                             uint32_t *ybits, int backoff) {
    bool ready = true;
#pragma unroll
    for (int t = 0; t < W; ++t) ready = ready && (q.code[t] < 0 || q.gv[t] != kUnset);
    while (__ballot(!ready) != 0) {
        for (int s = 0; s < backoff; ++s) __builtin_amdgcn_s_sleep(1);
        if (!ready) {
            ready = true;
#pragma unroll
            for (int t = 0; t < W; ++t)
                if (q.code[t] >= 0 && q.gv[t] == kUnset) {
                    q.gv[t] = ld_agent(&ybits[q.code[t]]);
                    ready = ready && q.gv[t] != kUnset;
                }
        }
    }
    float yl[W];
#pragma unroll
    for (int t = 0; t < W; ++t) yl[t] = ysh[q.code[t] <= -2 ? -2 - q.code[t] : 0];
    float acc = q.rhs;
#pragma unroll
    for (int t = 0; t < W; ++t) {
        const float dep = q.code[t] >= 0 ? __uint_as_float(q.gv[t]) : yl[t];
        if (q.code[t] != -1) acc -= q.val[t] * dep;
    }
    const float y = acc / q.dg;
    ysh[q.row] = y;
    st_agent(&ybits[blk_row(S, r0, q.row)], publishable(y));
    // LDS ordering between the lanes of the wave (no global wait)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return q.act ? y : 0.f;
}

// Dynamic LDS of the blocked kernels: records, right-hand side, solution,
// chunk table and (fused PCG backward solve) the rr entries of one block.
template <int W>
inline size_t blk_lds_bytes(int bmax, int chmax) {
    return (size_t)bmax * (2 * W + 2 + 3) * 4 + (size_t)chmax * 8;
}

// Block b of a solve: stage, then walk the chunks.  RZ: the lane's sum of
// rr[row] * solution[row] is returned (fixed order: the lane's chunks in
// schedule order); otherwise rr is not read and 0 is returned.
template <int W, bool RZ>
__device__ double blk_solve(const BlkSched &S, int b, const float *rhs, uint32_t *ybits, const float *rr,
                            int backoff) {
    constexpr int RW = 2 * W + 2;
    extern __shared__ int blk_dyn[];
    int *rec = blk_dyn;
    float *rsh = reinterpret_cast<float *>(rec + S.bmax * RW);
    float *ysh = rsh + S.bmax;
    int2 *ch = reinterpret_cast<int2 *>(ysh + S.bmax);
    float *rrsh = reinterpret_cast<float *>(ch + S.chmax);
    const int l = lane_id();
    const int r0 = S.brow[2 * b], nr = S.brow[2 * b + 1];
    const int c0 = S.bch[b], nch = S.bch[b + 1] - c0;
    {  // staging: every load of a batch is issued before its stores.  Lanes
       // past the end load the last element and store it back to the same
       // place, so no branch guards a store (a guarded store would let the
       // compiler sink its load into the branch and serialise the batch).
        constexpr int Q4 = RW / 4;  // 16-byte pieces per record
        const int4 *src = reinterpret_cast<const int4 *>(S.rec);
        int4 *dst = reinterpret_cast<int4 *>(rec);
        const int n4 = nr * Q4;
        for (int i = l; i < n4; i += kWave * 8) {
            int4 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int x = min(i + u * kWave, n4 - 1);
                v[u] = src[(size_t)blk_row(S, r0, x / Q4) * Q4 + x % Q4];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) dst[min(i + u * kWave, n4 - 1)] = v[u];
        }
        for (int i = l; i < nr; i += kWave * 8) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = rhs[blk_row(S, r0, min(i + u * kWave, nr - 1))];
#pragma unroll
            for (int u = 0; u < 8; ++u) rsh[min(i + u * kWave, nr - 1)] = v[u];
        }
        if constexpr (RZ)
            for (int i = l; i < nr; i += kWave * 8) {
                float v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = rr[blk_row(S, r0, min(i + u * kWave, nr - 1))];
#pragma unroll
                for (int u = 0; u < 8; ++u) rrsh[min(i + u * kWave, nr - 1)] = v[u];
            }
        for (int i = l; i < nch; i += kWave) ch[i] = S.ch[c0 + i];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    constexpr int R = kBlkDist + 2;
    BlkSlot<W> q[R];
#pragma unroll
    for (int j = 0; j <= kBlkDist; ++j) blk_read<W>(q[j], rec, ch[min(j, nch - 1)], j, nch);
#pragma unroll
    for (int j = 0; j < kBlkDist; ++j) blk_issue<W, RZ>(q[j], rsh, ybits, rrsh);
    int2 ccn = ch[min(kBlkDist + 1, nch - 1)];  // table entry of the next record to read
    double rz = 0.0;
    for (int c = 0; c < nch; c += R) {
#pragma unroll
        for (int j = 0; j < R; ++j) {
            if (c + j < nch) {
                blk_read<W>(q[(j + kBlkDist + 1) % R], rec, ccn, c + j + kBlkDist + 1, nch);
                ccn = ch[min(c + j + kBlkDist + 2, nch - 1)];
                blk_issue<W, RZ>(q[(j + kBlkDist) % R], rsh, ybits, rrsh);
                const float y = blk_process<W>(q[j], ysh, S, r0, ybits, backoff);
                if constexpr (RZ) rz += (double)q[j].rr * (double)y;
            }
        }
    }
    return rz;
}

// XCD-local variant: only the waves running on XCD 0 (hardware register
// XCC_ID) take tickets, so every exchange between blocks stays in that XCD's
// L2; the grid is launched 8 times larger.  Waves elsewhere hold no ticket, so
// the ticket argument (a wave only waits on blocks held by running waves)
// is unchanged.
__device__ __forceinline__ bool blk_off_xcd(int local) {
    return local && (__builtin_amdgcn_s_getreg((20) | (0 << 6) | (3 << 11)) & 7) != 0;
}

template <int W>
static __global__ void __launch_bounds__(kWave) k_sptrsv_blk(BlkSched S, const float *__restrict__ rhs,
                                                            uint32_t *ybits, int *ticket, int backoff,
                                                            int local) {
    if (blk_off_xcd(local)) return;
    for (;;) {
        const int b = wave_ticket(ticket);
        if (b >= S.nb) break;
        blk_solve<W, false>(S, b, rhs, ybits, nullptr, backoff);
    }
}

// Pack one factor's values into the records: vsrc[q * (W + 1) + t] is the
// position of value t of record q in the factor's value array (-1: none),
// entry W the diagonal's.
template <int W>
static __global__ void k_blk_pack(int n, const int *__restrict__ vsrc, const float *__restrict__ v,
                                  int *__restrict__ rec) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    constexpr int RW = 2 * W + 2;
#pragma unroll
    for (int t = 0; t <= W; ++t) {
        const int k = vsrc[(size_t)q * (W + 1) + t];
        rec[(size_t)q * RW + W + 1 + t] = k >= 0 ? __float_as_int(v[k]) : 0;
    }
}

}  // namespace lpcg
