// Standalone building blocks: SpMV, triangular solves, IC(0), Jacobi.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <type_traits>

#include "device_util.h"
#include "kern_spmv.h"
#include "kern_sptrsv.h"
#include "lpcg_internal.h"

namespace lpcg {
namespace {

int nblk(long n, int t) { return (int)((n + t - 1) / t); }

__global__ void k_zero_i32(int *p, int count) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
}

// CSR SpMV with G = group lanes per row (64 / G rows per wavefront) on
// `blocks` blocks (0: the system's tuned grid), or (FP32, rows > 0, windows
// prepared for that R) the LDS-staged form with `rows` rows per block, or
// (group 1, or group 0 when the tuned form is ELL; A's FP32 values) the ELL
// form.
template <typename VT, typename XT>
int launch_spmv(const lpcg_system *s, const VT *v, const XT *x, XT *y, hipStream_t st, int group = 0,
                int blocks = 0, int rows = -1) {
    const int threads = 256;
    if constexpr (std::is_same<VT, float>::value && std::is_same<XT, float>::value) {
        if (group == 0 && s->spmv_ell && v == s->val32) group = 1;
    }
    if (group == 0) group = s->spmv_group;
    if (blocks == 0) blocks = s->spmv_blocks;
    if (rows < 0) rows = s->spmv_rows;
    if constexpr (std::is_same<VT, float>::value && std::is_same<XT, float>::value) {
        if (group == 1) {  // ELL form (A's FP32 values only)
            if (s->ea_w == 0 || v != s->val32) {
                set_error("SpMV: the ELL form serves A's FP32 values of a pattern with rows of at most %d entries",
                          kEllMaxW);
                return LPCG_EINVAL;
            }
            const int eb = std::max(1, std::min(kMaxSpmvBlocks, nblk(s->n, threads)));
            switch (s->ea_w) {
                case 1: k_spmv_e<1><<<eb, threads, 0, st>>>(s->n, s->ea_col, s->ea_val, x, y); break;
                case 2: k_spmv_e<2><<<eb, threads, 0, st>>>(s->n, s->ea_col, s->ea_val, x, y); break;
                case 3: k_spmv_e<3><<<eb, threads, 0, st>>>(s->n, s->ea_col, s->ea_val, x, y); break;
                case 4: k_spmv_e<4><<<eb, threads, 0, st>>>(s->n, s->ea_col, s->ea_val, x, y); break;
                case 5: k_spmv_e<5><<<eb, threads, 0, st>>>(s->n, s->ea_col, s->ea_val, x, y); break;
                case 6: k_spmv_e<6><<<eb, threads, 0, st>>>(s->n, s->ea_col, s->ea_val, x, y); break;
                case 7: k_spmv_e<7><<<eb, threads, 0, st>>>(s->n, s->ea_col, s->ea_val, x, y); break;
                default: k_spmv_e<8><<<eb, threads, 0, st>>>(s->n, s->ea_col, s->ea_val, x, y); break;
            }
            LPCG_LAUNCH_CHECK();
            return LPCG_OK;
        }
        if (rows > 0) {
            if (rows != s->spmv_win_rows) {
                set_error("SpMV: windows not prepared for %d rows per block", rows);
                return LPCG_EINVAL;
            }
            const int nb = nblk(s->n, rows);
            const size_t lds = sizeof(float) * (size_t)std::max(1, s->spmv_wmax);
            switch (group) {
                case 4: k_spmv_st<4><<<nb, threads, lds, st>>>(s->n, rows, s->rowptr, s->colind, v, x, y, s->spmv_win); break;
                case 8: k_spmv_st<8><<<nb, threads, lds, st>>>(s->n, rows, s->rowptr, s->colind, v, x, y, s->spmv_win); break;
                case 16: k_spmv_st<16><<<nb, threads, lds, st>>>(s->n, rows, s->rowptr, s->colind, v, x, y, s->spmv_win); break;
                case 32: k_spmv_st<32><<<nb, threads, lds, st>>>(s->n, rows, s->rowptr, s->colind, v, x, y, s->spmv_win); break;
                default: k_spmv_st<64><<<nb, threads, lds, st>>>(s->n, rows, s->rowptr, s->colind, v, x, y, s->spmv_win); break;
            }
            LPCG_LAUNCH_CHECK();
            return LPCG_OK;
        }
    }
    switch (group) {
        case 4: k_spmv<4><<<blocks, threads, 0, st>>>(s->n, s->rowptr, s->colind, v, x, y); break;
        case 8: k_spmv<8><<<blocks, threads, 0, st>>>(s->n, s->rowptr, s->colind, v, x, y); break;
        case 16: k_spmv<16><<<blocks, threads, 0, st>>>(s->n, s->rowptr, s->colind, v, x, y); break;
        case 32: k_spmv<32><<<blocks, threads, 0, st>>>(s->n, s->rowptr, s->colind, v, x, y); break;
        default: k_spmv<64><<<blocks, threads, 0, st>>>(s->n, s->rowptr, s->colind, v, x, y); break;
    }
    LPCG_LAUNCH_CHECK();
    return LPCG_OK;
}

// ------------------------------------------------------------------ IC(0)
// Incomplete Cholesky with zero fill on tril(A) (the paper's IC baseline):
//   L_ij = (A_ij - sum_{k<j, k in S_i and S_j} L_ik L_jk) / L_jj   (j < i)
//   L_ii = sqrt(A_ii (1 + shift) - sum_{k<i} L_ik^2)
// Row i depends on the rows j of its strictly-lower entries, the same DAG as
// the forward substitution: rows are handed out in forward level order
// through a ticket.  FP64; every stored value is preset to kUnset64 and is its
// own ready flag (agent-scope stores and loads), so no fence orders a row's
// values against a separate flag.  A lane restarts the entry it is working on
// when some value it needs is not yet published (non-blocking in the wave).
constexpr uint64_t kUnset64 = 0x7fffffffffffffffull;
constexpr int kIcRegDeps = 8;

__device__ __forceinline__ uint64_t ld64(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st64(uint64_t *p, double v) {
    uint64_t b = __double_as_longlong(v);
    __hip_atomic_store(p, (v != v) ? kCanonNan64 : b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void __launch_bounds__(256) k_ic0(int n, const int *__restrict__ order,
                                             const int *__restrict__ lrp, const int *__restrict__ lci,
                                             const int *__restrict__ lsrc,
                                             const double *__restrict__ aval, double shift,
                                             uint64_t *l64, int *ticket, int *bad_row, int backoff) {
    for (;;) {
        const int chunk = wave_ticket(ticket);
        if ((long)chunk * kWave >= n) break;
        const int pos = chunk * kWave + lane_id();
        int row = -1, a = 0, b = 0, p = 0;
        if (pos < n) {
            row = order[pos];
            a = lrp[row];
            b = lrp[row + 1];
            p = a;
        }
        // Diagonal positions of the rows this row depends on (<= 8 of them
        // are polled together, one memory round trip per round, before the
        // entries are computed in order).
        const int nd = b - a - 1;
        const bool poll_first = nd > 0 && nd <= kIcRegDeps;
        int jdiag[kIcRegDeps];
#pragma unroll
        for (int t = 0; t < kIcRegDeps; ++t) jdiag[t] = (poll_first && t < nd) ? lrp[lci[a + t] + 1] - 1 : 0;
        bool diags_ready = !poll_first;
        bool pending = row >= 0;
        while (__ballot(pending) != 0) {
            if (pending && !diags_ready) {
                uint64_t got[kIcRegDeps];
#pragma unroll
                for (int t = 0; t < kIcRegDeps; ++t) got[t] = t < nd ? ld64(&l64[jdiag[t]]) : 0ull;
                bool ready = true;
#pragma unroll
                for (int t = 0; t < kIcRegDeps; ++t) ready = ready && (got[t] != kUnset64);
                diags_ready = ready;
            }
            bool progress = pending && diags_ready;
            while (progress) {
                if (p < b - 1) {
                    const int j = lci[p];
                    const int jd = lrp[j + 1] - 1;
                    const uint64_t djb = ld64(&l64[jd]);
                    if (djb == kUnset64) { progress = false; break; }
                    double sacc = aval[lsrc[p]];
                    int ia = a, ib = lrp[j];
                    bool ok = true;
                    while (ia < p && ib < jd) {
                        const int ka = lci[ia], kb = lci[ib];
                        if (ka == kb) {
                            const uint64_t ljk = ld64(&l64[ib]);
                            if (ljk == kUnset64) { ok = false; break; }
                            const double lik = __longlong_as_double(ld64(&l64[ia]));
                            sacc -= lik * __longlong_as_double(ljk);
                            ++ia;
                            ++ib;
                        } else if (ka < kb) {
                            ++ia;
                        } else {
                            ++ib;
                        }
                    }
                    if (!ok) { progress = false; break; }
                    st64(&l64[p], sacc / __longlong_as_double(djb));
                    ++p;
                } else {
                    double d = aval[lsrc[p]] * (1.0 + shift);
                    for (int q = a; q < p; ++q) {
                        const double l = __longlong_as_double(ld64(&l64[q]));
                        d -= l * l;
                    }
                    if (!(d > 0.0) || !isfinite(d)) {
                        atomicMin(bad_row, row);
                        d = 1.0;  // keep dependants going; the result is rejected
                    }
                    st64(&l64[p], sqrt(d));
                    pending = false;
                    progress = false;
                }
            }
            if (pending)
                for (int t = 0; t < backoff; ++t) __builtin_amdgcn_s_sleep(1);
        }
    }
}

__global__ void k_fill_u64(int count, uint64_t *p, uint64_t v) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

__global__ void k_l64_to_f32(int nnz_l, const double *__restrict__ l64, const int *__restrict__ u2l,
                             float *__restrict__ lval, float *__restrict__ utval) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nnz_l) return;
    if (lval) lval[k] = (float)l64[k];
    if (utval) utval[k] = (float)l64[u2l[k]];
}

// Symmetric Gauss-Seidel factor on tril(A): L_ij = A_ij / sqrt(A_jj) (the
// diagonal becomes sqrt(A_ii)), in FP64 and stored FP32.
__global__ void k_sgs(int nnz_l, const int *__restrict__ lsrc, const int *__restrict__ lcol,
                      const double *__restrict__ val64, const double *__restrict__ diag64,
                      const int *__restrict__ u2l, float *__restrict__ lval, float *__restrict__ utval) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnz_l) return;
    if (lval) lval[p] = (float)(val64[lsrc[p]] / sqrt(diag64[lcol[p]]));
    if (utval) {
        const int q = u2l[p];
        utval[p] = (float)(val64[lsrc[q]] / sqrt(diag64[lcol[q]]));
    }
}

__global__ void k_l_to_ut(int nnz_l, const float *__restrict__ lval, const int *__restrict__ u2l,
                          float *__restrict__ utval) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nnz_l) utval[k] = lval[u2l[k]];
}

__global__ void k_jacobi(int n, const double *__restrict__ diag, float *__restrict__ dinv) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dinv[i] = (float)(1.0 / diag[i]);
}

__global__ void k_set_i32(int *p, int v) { *p = v; }

// Window of block b: the smallest and largest off-diagonal column of its rows
// (columns are sorted, so each row contributes its first and last
// off-diagonal entry); *wmax receives the longest window.
__global__ void __launch_bounds__(256) k_spmv_window(int n, int R, const int *__restrict__ rp,
                                                     const int *__restrict__ ci, int *__restrict__ win,
                                                     int *__restrict__ wmax) {
    __shared__ int slo[256 / kWave], shi[256 / kWave];
    const int r0 = blockIdx.x * R, r1 = min(n, r0 + R);
    int lo = 0x7fffffff, hi = -1;
    for (int row = r0 + (int)threadIdx.x; row < r1; row += blockDim.x) {
        const int a = rp[row], e = rp[row + 1];
        const int f = a < e && ci[a] == row ? a + 1 : a;
        const int l = a < e && ci[e - 1] == row ? e - 2 : e - 1;
        if (f < e && ci[f] != row) lo = min(lo, ci[f]);
        if (l >= a && ci[l] != row) hi = max(hi, ci[l]);
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        lo = min(lo, __shfl_xor(lo, off, kWave));
        hi = max(hi, __shfl_xor(hi, off, kWave));
    }
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) {
        slo[w] = lo;
        shi[w] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < (int)blockDim.x / kWave; ++i) {
            lo = min(lo, slo[i]);
            hi = max(hi, shi[i]);
        }
        if (hi < lo) lo = hi + 1;  // empty window
        win[2 * blockIdx.x] = lo;
        win[2 * blockIdx.x + 1] = hi;
        if (hi >= lo) atomicMax(wmax, hi - lo + 1);
    }
}


}  // namespace

int spmv32(const lpcg_system *s, const float *x, float *y, hipStream_t st) {
    return launch_spmv<float, float>(s, s->val32, x, y, st);
}

// Column windows of the LDS-staged SpMV for R rows per block (synchronous).
// EINVAL when the blocks exceed the published-partial slots or the longest
// window the LDS budget (kSpmvMaxWindow inputs).
int spmv_prepare_window(lpcg_system *s, int R, hipStream_t st) {
    if (R < 64 || nblk(s->n, R) > kMaxSpmvBlocks) {
        set_error("SpMV: %d rows per block give %d blocks (1 .. %d)", R, nblk(s->n, std::max(R, 1)), kMaxSpmvBlocks);
        return LPCG_EINVAL;
    }
    if (s->spmv_win_rows == R) return s->spmv_wmax <= kSpmvMaxWindow ? LPCG_OK : LPCG_EINVAL;
    if (!s->spmv_win) {
        void *q = nullptr;
        LPCG_HIP(hipMalloc(&q, sizeof(int) * (2 * (size_t)kMaxSpmvBlocks + 1)));
        s->allocs.push_back(q);
        s->spmv_win = (int *)q;
    }
    int *wmax = s->spmv_win + 2 * kMaxSpmvBlocks;
    k_set_i32<<<1, 1, 0, st>>>(wmax, 0);
    k_spmv_window<<<nblk(s->n, R), 256, 0, st>>>(s->n, R, s->rowptr, s->colind, s->spmv_win, wmax);
    LPCG_LAUNCH_CHECK();
    int h = 0;
    LPCG_HIP(hipMemcpyAsync(&h, wmax, sizeof(int), hipMemcpyDeviceToHost, st));
    LPCG_HIP(hipStreamSynchronize(st));
    s->spmv_win_rows = R;
    s->spmv_wmax = h;
    if (h > kSpmvMaxWindow) {
        set_error("SpMV: a window of %d inputs exceeds the LDS budget (%d) at %d rows per block", h,
                  kSpmvMaxWindow, R);
        return LPCG_EINVAL;
    }
    return LPCG_OK;
}
int spmv64(const lpcg_system *s, const double *x, double *y, hipStream_t st) {
    return launch_spmv<double, double>(s, s->val64, x, y, st);
}

// Whether the single-workgroup mode can take a direction: every level must
// fit in kWgRows rows per thread.
bool wg_mode_fits(const lpcg_system *s, int transpose) {
    return (transpose ? s->max_w_b : s->max_w_f) <= kWgRows * kWgThreads;
}

// ---------------------------------------------------------------- mode 3
constexpr size_t kBlkLdsMax = 144 * 1024;  // dynamic LDS of a blocked wave (160 KB per CU)

// Cached PCG graphs hold the kernel arguments of their capture, blocked
// schedules included: every change of a schedule or configuration drops them.
void drop_graphs(lpcg_system *s) {
    if (s->graph_exec) {
        (void)hipGraphExecDestroy(s->graph_exec);
        s->graph_exec = nullptr;
    }
    s->graph_key.clear();
    if (s->bgraph_exec) {
        (void)hipGraphExecDestroy(s->bgraph_exec);
        s->bgraph_exec = nullptr;
    }
    s->bgraph_key.clear();
}

void blk_free(lpcg_system *s, int d) {
    drop_graphs(s);
    for (int **p : {&s->blk_brow[d], &s->blk_bch[d], &s->blk_ch[d], &s->blk_rec[d], &s->blk_vsrc[d]}) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
    s->blk_B[d] = 0;
    s->blk_K[d] = 1;
    s->blk_lsh[d] = 30;
    s->blk_D[d] = 0;
}

template <typename T>
static int upload(T **dst, const std::vector<T> &h) {
    LPCG_HIP(hipMalloc((void **)dst, sizeof(T) * std::max<size_t>(1, h.size())));
    LPCG_HIP(hipMemcpy(*dst, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice));
    return LPCG_OK;
}

// Schedule of direction d (0: L rows ascending, 1: U = L^T rows descending)
// for blocks of B rows: per block, the rows ordered by their level inside the
// block, cut into chunks of at most 64 rows of one level, and one record per
// row (dependency codes in CSR order, row, and the positions of the values).
// Pure host code: rp/ci is the direction's CSR pattern (diagonal stored).
struct BlkHost {
    int W = 0, nb = 0, chmax = 0, lsh = 30, D = 0;
    std::vector<int> brow, bch, ch, rec, vsrc;
};

// Longest dependency offset of a triangular pattern (L: rows ascending,
// diagonal last; U: diagonal first): the stride between the runs of a banded
// block (one grid plane for a natural-order grid).
static int blk_dep_offset(int n, const int *rp, const int *ci, int d) {
    int D = 0;
    for (int r = 0; r < n; ++r)
        if (rp[r + 1] - rp[r] > 1) D = std::max(D, d ? ci[rp[r + 1] - 1] - r : r - ci[rp[r]]);
    return D;
}

static int blk_build(int n, const int *rp, const int *ci, int d, int B, int K, BlkHost &o) {
    if (n <= 0 || B < 64 || B > (1 << 16)) {
        set_error("blocked substitution: block size %d outside [64, 65536] (n = %d)", B, n);
        return LPCG_EINVAL;
    }
    int maxdep = 0;
    for (int r = 0; r < n; ++r) maxdep = std::max(maxdep, rp[r + 1] - rp[r] - 1);
    const int W = maxdep <= 3 ? 3 : maxdep <= 7 ? 7 : 0;
    if (!W) {
        set_error("blocked substitution: a row has %d dependencies (at most 7)", maxdep);
        return LPCG_EINVAL;
    }
    // Banded blocks (K > 1): K runs of len = B / K consecutive rows, D rows
    // apart (D = the longest dependency offset).  Group g holds the rows
    // [g K D, (g + 1) K D), cut into D / len bands; block (g, q) is band q of
    // every run of the group.  Blocks are numbered g-major in row order and
    // ticketed in solve order (descending for U).
    int len = B, D = 0, lsh = 30, Q = 1;
    if (K > 1) {
        D = blk_dep_offset(n, rp, ci, d);
        len = B / K;
        lsh = 0;
        while ((1 << lsh) < len) ++lsh;
        if (B % K || (1 << lsh) != len || D < len || D % len || (long)n % ((long)K * D)) {
            set_error("blocked substitution: %d runs of %d rows do not tile %d rows with stride %d", K, len, n, D);
            return LPCG_EINVAL;
        }
        Q = D / len;
    } else if (K != 1) {
        set_error("blocked substitution: %d runs per block", K);
        return LPCG_EINVAL;
    }
    const long G = (long)K * D;
    const int RW = 2 * W + 2, nb = K > 1 ? (int)(n / G) * Q : (n + B - 1) / B;
    o = BlkHost{};
    o.W = W;
    o.nb = nb;
    o.lsh = lsh;
    o.D = D;
    o.brow.assign(2 * (size_t)nb, 0);
    o.bch.assign(1, 0);
    o.rec.assign((size_t)n * RW, 0);
    o.vsrc.assign((size_t)n * (W + 1), -1);
    std::vector<int> lev(n, 0), cnt, order;
    for (int b = 0; b < nb; ++b) {
        int r0, nr, idx = 0;
        if (K > 1) {
            idx = d ? nb - 1 - b : b;
            r0 = (int)((idx / Q) * G + (long)(idx % Q) * len);
            nr = B;
        } else {
            r0 = d ? std::max(0, n - (b + 1) * B) : b * B;
            nr = (d ? n - b * B : std::min(n, (b + 1) * B)) - r0;
        }
        o.brow[2 * b] = r0;
        o.brow[2 * b + 1] = nr;
        auto row_of = [&](int x) { return r0 + (x >> lsh) * D + (x & ((1 << lsh) - 1)); };
        // slot of row c in this block, or -1
        auto slot_of = [&](int c) -> int {
            if (K == 1) return c >= r0 && c < r0 + nr ? c - r0 : -1;
            const long off = c - (long)(idx / Q) * G;
            if (off < 0 || off >= G || (off % D) / len != idx % Q) return -1;
            return (int)((off / D) * len + off % D - (long)(idx % Q) * len);
        };
        int maxl = 0;
        for (int i = 0; i < nr; ++i) {  // solve order inside the block
            const int x = d ? nr - 1 - i : i, r = row_of(x);
            int l = 0;
            for (int k = rp[r]; k < rp[r + 1]; ++k) {
                const int c = ci[k];
                if (c == r) continue;
                if (slot_of(c) >= 0) {
                    l = std::max(l, lev[c] + 1);
                } else if (K > 1) {  // another block: it must hold an earlier ticket
                    const long oc = c % G;
                    const int idc = (int)((c / G) * Q + (oc % D) / len);
                    if (d ? idc <= idx : idc >= idx) {
                        set_error("blocked substitution: banded blocks of %d runs are not in dependency order", K);
                        return LPCG_EINVAL;
                    }
                }
            }
            lev[r] = l;
            maxl = std::max(maxl, l);
        }
        cnt.assign(maxl + 2, 0);
        for (int x = 0; x < nr; ++x) ++cnt[lev[row_of(x)] + 1];
        for (int l = 0; l <= maxl; ++l) cnt[l + 1] += cnt[l];
        order.assign(nr, 0);
        std::vector<int> fill(cnt.begin(), cnt.end() - 1);
        for (int i = 0; i < nr; ++i) {
            const int r = row_of(d ? nr - 1 - i : i);
            order[fill[lev[r]]++] = r;
        }
        const int cbase = (int)o.ch.size() / 2;
        for (int l = 0; l <= maxl; ++l)
            for (int p = cnt[l]; p < cnt[l + 1]; p += kWave) {
                o.ch.push_back(p);
                o.ch.push_back(std::min(kWave, cnt[l + 1] - p));
            }
        o.bch.push_back((int)o.ch.size() / 2);
        o.chmax = std::max(o.chmax, (int)o.ch.size() / 2 - cbase);
        for (int p = 0; p < nr; ++p) {  // record p at the block's p-th row position
            const int r = order[p], at = row_of(p);
            int *w = &o.rec[(size_t)at * RW];
            int *vs = &o.vsrc[(size_t)at * (W + 1)];
            for (int t = 0; t < W; ++t) w[t] = -1;
            w[W] = slot_of(r);
            int t = 0;
            for (int k = rp[r]; k < rp[r + 1]; ++k) {
                const int c = ci[k];
                if (c == r) {
                    vs[W] = k;
                    continue;
                }
                const int sc = slot_of(c);
                w[t] = sc >= 0 ? -2 - sc : c;
                vs[t] = k;
                ++t;
            }
        }
    }
    const size_t lds = W == 3 ? blk_lds_bytes<3>(B, o.chmax) : blk_lds_bytes<7>(B, o.chmax);
    if (lds > kBlkLdsMax) {
        set_error("blocked substitution: %zu bytes of LDS for block size %d (at most %zu)", lds, B, kBlkLdsMax);
        return LPCG_EINVAL;
    }
    return LPCG_OK;
}

int blk_prepare(lpcg_system *s, int d, int B, int K) {
    if (s->blk_B[d] == B && s->blk_K[d] == K && s->blk_rec[d]) return LPCG_OK;
    const int n = s->n, nl = s->nnz_l;
    std::vector<int> rp(n + 1), ci(nl);
    LPCG_HIP(hipDeviceSynchronize());
    LPCG_HIP(hipMemcpy(rp.data(), d ? s->urowptr : s->lrowptr, sizeof(int) * (n + 1), hipMemcpyDeviceToHost));
    LPCG_HIP(hipMemcpy(ci.data(), d ? s->ucol : s->lcol, sizeof(int) * nl, hipMemcpyDeviceToHost));
    BlkHost o;
    int rc = blk_build(n, rp.data(), ci.data(), d, B, K, o);
    if (rc) return rc;
    blk_free(s, d);
    if ((rc = upload(&s->blk_brow[d], o.brow)) || (rc = upload(&s->blk_bch[d], o.bch)) ||
        (rc = upload(&s->blk_ch[d], o.ch)) || (rc = upload(&s->blk_rec[d], o.rec)) ||
        (rc = upload(&s->blk_vsrc[d], o.vsrc))) {
        blk_free(s, d);
        return rc;
    }
    s->blk_B[d] = B;
    s->blk_K[d] = K;
    s->blk_lsh[d] = o.lsh;
    s->blk_D[d] = o.D;
    s->blk_W[d] = o.W;
    s->blk_nb[d] = o.nb;
    s->blk_chmax[d] = o.chmax;
    // allow the blocked kernels' dynamic LDS (set here, before any launch or
    // graph capture that uses the schedule)
    LPCG_HIP(hipFuncSetAttribute((const void *)k_sptrsv_blk<3>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)kBlkLdsMax));
    LPCG_HIP(hipFuncSetAttribute((const void *)k_sptrsv_blk<7>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)kBlkLdsMax));
    return LPCG_OK;
}

int blk_pack(const lpcg_system *s, int d, const float *lval, const float *utval, hipStream_t st) {
    const float *v = d ? utval : lval;
    if (s->blk_W[d] == 3) k_blk_pack<3><<<nblk(s->n, 256), 256, 0, st>>>(s->n, s->blk_vsrc[d], v, s->blk_rec[d]);
    else k_blk_pack<7><<<nblk(s->n, 256), 256, 0, st>>>(s->n, s->blk_vsrc[d], v, s->blk_rec[d]);
    LPCG_LAUNCH_CHECK();
    return LPCG_OK;
}

static BlkSched blk_sched(const lpcg_system *s, int d) {
    return BlkSched{s->blk_brow[d], s->blk_bch[d], reinterpret_cast<const int2 *>(s->blk_ch[d]), s->blk_rec[d],
                    s->blk_nb[d], s->blk_B[d], s->blk_chmax[d], s->blk_lsh[d], s->blk_D[d]};
}

// Enqueue the kernels of one substitution with configuration c: the
// dependency-driven kernel expects y preset to kUnset and the ticket zeroed,
// the single-workgroup kernel the factor's values in level-ordered form
// (trsv_presets does both); the level-synchronous launches need nothing.
int trsv_kernels(const lpcg_system *s, int transpose, const TrsvCfg &c, const float *lval,
                 const float *utval, const float *rhs, float *y, int *ticket, hipStream_t st) {
    const int n = s->n;
    const bool up = transpose != 0;
    const int *order = up ? s->blev_rows : s->flev_rows;
    const int *rp = up ? s->urowptr : s->lrowptr;
    const int *ci = up ? s->ucol : s->lcol;
    const float *v = up ? utval : lval;
    if (c.mode == 0) {
        const int blocks = nblk(trsv_waves(n, c.waves), 4) * c.stride;
        if (up)
            k_sptrsv<true><<<blocks, 256, 0, st>>>(n, order, rp, ci, v, rhs, (uint32_t *)y, ticket, c.backoff,
                                                   c.stride);
        else
            k_sptrsv<false><<<blocks, 256, 0, st>>>(n, order, rp, ci, v, rhs, (uint32_t *)y, ticket, c.backoff,
                                                    c.stride);
        LPCG_LAUNCH_CHECK();
        return LPCG_OK;
    }
    if (c.mode == 3) {
        const int d = up ? 1 : 0;
        if (s->blk_B[d] != c.blk || s->blk_K[d] != c.runs || !s->blk_rec[d]) {
            set_error("blocked substitution: no schedule for block size %d in %d runs", c.blk, c.runs);
            return LPCG_EINVAL;
        }
        const BlkSched S = blk_sched(s, d);
        const int local = c.stride == 8, grid = S.nb * (local ? 8 : 1);
        if (s->blk_W[d] == 3)
            k_sptrsv_blk<3><<<grid, kWave, blk_lds_bytes<3>(S.bmax, S.chmax), st>>>(S, rhs, (uint32_t *)y, ticket,
                                                                                 c.backoff, local);
        else
            k_sptrsv_blk<7><<<grid, kWave, blk_lds_bytes<7>(S.bmax, S.chmax), st>>>(S, rhs, (uint32_t *)y, ticket,
                                                                                 c.backoff, local);
        LPCG_LAUNCH_CHECK();
        return LPCG_OK;
    }
    if (c.mode == 2) {
        const int d = up ? 1 : 0;
        k_trsv_wg<<<1, kWgThreads, 0, st>>>(up ? s->nlev_b : s->nlev_f, up ? s->blev_ptr : s->flev_ptr, order,
                                            s->lo_ptr[d], s->lo_col[d], s->lo_val[d], s->lo_diag[d], rhs, y);
        LPCG_LAUNCH_CHECK();
        return LPCG_OK;
    }
    const std::vector<int> &lp = up ? s->h_blev_ptr : s->h_flev_ptr;
    for (size_t l = 0; l + 1 < lp.size(); ++l) {
        const int rows = lp[l + 1] - lp[l];
        const int nb = level_blocks(rows, s->trsv_g);
        const int *ord = order + lp[l];
#define LPCG_LVL(UP, G) k_trsv_level<UP, G><<<nb, 256, 0, st>>>(rows, ord, rp, ci, v, rhs, y)
        if (up) {
            if (s->trsv_g == 4) LPCG_LVL(true, 4);
            else if (s->trsv_g == 8) LPCG_LVL(true, 8);
            else LPCG_LVL(true, 16);
        } else {
            if (s->trsv_g == 4) LPCG_LVL(false, 4);
            else if (s->trsv_g == 8) LPCG_LVL(false, 8);
            else LPCG_LVL(false, 16);
        }
#undef LPCG_LVL
    }
    LPCG_LAUNCH_CHECK();
    return LPCG_OK;
}

// Level-ordered values of one direction's factor (single-workgroup mode).
int lo_prepare(const lpcg_system *s, int transpose, const float *lval, const float *utval, hipStream_t st) {
    const int d = transpose ? 1 : 0;
    const int noff = s->nnz_l - s->n;
    k_lo_prep<<<nblk(std::max(noff, s->n), 256), 256, 0, st>>>(noff, s->n, s->lo_src[d], s->lo_dsrc[d],
                                                                 transpose ? utval : lval, s->lo_val[d],
                                                                 s->lo_diag[d]);
    LPCG_LAUNCH_CHECK();
    return LPCG_OK;
}

int trsv_presets(const lpcg_system *s, int transpose, const TrsvCfg &c, const float *lval, const float *utval,
                 float *y, int *ticket, hipStream_t st) {
    if (c.mode == 2) return lo_prepare(s, transpose, lval, utval, st);
    if (c.mode == 3) {
        int rc = blk_prepare(const_cast<lpcg_system *>(s), transpose ? 1 : 0, c.blk, c.runs);
        if (rc || (rc = blk_pack(s, transpose ? 1 : 0, lval, utval, st))) return rc;
    } else if (c.mode != 0) {
        return LPCG_OK;
    }
    k_fill_u32<<<nblk(s->n, 256), 256, 0, st>>>(s->n, (uint32_t *)y, kUnset);
    k_zero_i32<<<1, 64, 0, st>>>(ticket, 1);
    LPCG_LAUNCH_CHECK();
    return LPCG_OK;
}

int sptrsv32(const lpcg_system *s, int transpose, const float *lval, const float *utval,
             const float *rhs, float *y, int *ticket, hipStream_t st) {
    const TrsvCfg &c = s->trsv[transpose ? 1 : 0];
    int rc = trsv_presets(s, transpose, c, lval, utval, y, ticket, st);
    if (rc) return rc;
    return trsv_kernels(s, transpose, c, lval, utval, rhs, y, ticket, st);
}

}  // namespace lpcg

using namespace lpcg;

extern "C" int lpcg_spmv(const lpcg_system *s, int32_t prec, const void *x, void *y,
                         hipStream_t st) {
    if (!s || !x || !y || (prec != 32 && prec != 64)) {
        set_error("lpcg_spmv: invalid arguments");
        return LPCG_EINVAL;
    }
    if (!s->perm) {
        if (prec == 32) return spmv32(s, (const float *)x, (float *)y, st);
        return spmv64(s, (const double *)x, (double *)y, st);
    }
    // reordered system: x and y are in the caller's numbering
    int rc;
    if (prec == 32) {
        float *xi = (float *)s->t64a, *yi = (float *)s->t64b;
        if ((rc = to_internal_f32(s, (const float *)x, xi, st)) || (rc = spmv32(s, xi, yi, st))) return rc;
        return from_internal_f32(s, yi, (float *)y, st);
    }
    if ((rc = to_internal_f64(s, (const double *)x, s->t64a, st)) || (rc = spmv64(s, s->t64a, s->t64b, st)))
        return rc;
    return from_internal_f64(s, s->t64b, (double *)y, st);
}

extern "C" int lpcg_sptrsv(const lpcg_system *s, int32_t transpose, const float *l_val,
                           const float *ut_val, const float *rhs, float *y, hipStream_t st) {
    if (!s || !rhs || !y || rhs == y || (transpose ? !ut_val : !l_val)) {
        set_error("lpcg_sptrsv: invalid arguments");
        return LPCG_EINVAL;
    }
    if (!s->perm) return sptrsv32(s, transpose, l_val, ut_val, rhs, y, s->ctrl + C_TICKET_X, st);
    float *ri = (float *)s->t64a, *yi = (float *)s->t64b;
    int rc;
    if ((rc = to_internal_f32(s, rhs, ri, st)) ||
        (rc = sptrsv32(s, transpose, l_val, ut_val, ri, yi, s->ctrl + C_TICKET_X, st)))
        return rc;
    return from_internal_f32(s, yi, y, st);
}

extern "C" int lpcg_l_to_ut(const lpcg_system *s, const float *l_val, float *ut_val,
                            hipStream_t st) {
    if (!s || !l_val || !ut_val) {
        set_error("lpcg_l_to_ut: invalid arguments");
        return LPCG_EINVAL;
    }
    k_l_to_ut<<<nblk(s->nnz_l, 256), 256, 0, st>>>(s->nnz_l, l_val, s->u2l, ut_val);
    LPCG_LAUNCH_CHECK();
    return LPCG_OK;
}

extern "C" int lpcg_jacobi(const lpcg_system *s, float *dinv, hipStream_t st) {
    if (!s || !dinv) {
        set_error("lpcg_jacobi: invalid arguments");
        return LPCG_EINVAL;
    }
    k_jacobi<<<nblk(s->n, 256), 256, 0, st>>>(s->n, s->diag64, dinv);
    LPCG_LAUNCH_CHECK();
    return LPCG_OK;
}

namespace lpcg {
namespace {

// IC(0) with the FP64 factor in l64 (nnz_l doubles, preset here): the body
// shared by the allocating and the no-allocation entry points.
int ic0_run(const lpcg_system *s, double shift0, int32_t max_retries, float *l_val, float *ut_val,
            double *shift_used, double *l64, hipStream_t st) {
    int *flags = s->ctrl + C_TICKET_X;  // ticket
    int *bad = s->ctrl + C_STATUS;      // reused as the bad-row slot
    double shift = shift0;
    for (int attempt = 0; attempt <= std::max(0, (int)max_retries); ++attempt) {
        k_fill_u64<<<nblk(s->nnz_l, 256), 256, 0, st>>>(s->nnz_l, (uint64_t *)l64, kUnset64);
        k_set_i32<<<1, 1, 0, st>>>(flags, 0);
        k_set_i32<<<1, 1, 0, st>>>(bad, 0x7fffffff);
        // same DAG as the forward substitution: reuse the wave count and
        // back-off of its fastest dependency-driven configuration (tuned), or
        // of the forward direction when that runs dependency driven
        const TrsvCfg &fc = s->ic0_tuned ? s->ic0_cfg : s->trsv[0];
        const int blocks = nblk(trsv_waves(s->n, fc.mode == 0 ? fc.waves : 0), 4);
        k_ic0<<<blocks, 256, 0, st>>>(s->n, s->flev_rows, s->lrowptr, s->lcol, s->lsrc, s->val64, shift,
                                      (uint64_t *)l64, flags, bad, fc.mode == 0 ? fc.backoff : 1);
        LPCG_LAUNCH_CHECK();
        int hbad = 0;
        LPCG_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
        LPCG_HIP(hipStreamSynchronize(st));
        if (hbad == 0x7fffffff) {
            k_l64_to_f32<<<nblk(s->nnz_l, 256), 256, 0, st>>>(s->nnz_l, l64, s->u2l, l_val, ut_val);
            LPCG_LAUNCH_CHECK();
            LPCG_HIP(hipStreamSynchronize(st));
            if (shift_used) *shift_used = shift;
            return LPCG_OK;
        }
        set_error("lpcg_ic0: non-positive pivot at row %d (shift %g)", hbad, shift);
        shift = shift == 0.0 ? 1e-3 : 2.0 * shift;
    }
    return LPCG_EBREAKDOWN;
}

// Scratch of lpcg_ic0_noalloc: the FP64 factor of one call.  Each device
// holds its own copy for the life of the process; host code never passes
// the symbol itself to a kernel, only the device address looked up below.
constexpr size_t kIc0ScratchDoubles = (size_t)LPCG_IC0_NOALLOC_MAX_NNZ_L;
__device__ __align__(256) double scratch[kIc0ScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
int ic0_scratch(double **out) {
    int dev = -1;
    LPCG_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("lpcg_ic0_noalloc: device ordinal %d out of range", dev);
        return LPCG_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("lpcg_ic0_noalloc: hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                      hipGetErrorString(e));
            return LPCG_EHIP;
        }
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return LPCG_OK;
}

}  // namespace
}  // namespace lpcg

using namespace lpcg;

extern "C" int lpcg_ic0(const lpcg_system *s, double shift0, int32_t max_retries, float *l_val,
                        float *ut_val, double *shift_used, hipStream_t st) {
    if (!s || (!l_val && !ut_val) || shift0 < 0) {
        set_error("lpcg_ic0: invalid arguments");
        return LPCG_EINVAL;
    }
    double *l64 = nullptr;
    LPCG_HIP(hipMallocAsync((void **)&l64, sizeof(double) * (size_t)s->nnz_l, st));
    const int rc = ic0_run(s, shift0, max_retries, l_val, ut_val, shift_used, l64, st);
    LPCG_HIP(hipFreeAsync(l64, st));
    LPCG_HIP(hipStreamSynchronize(st));
    return rc;
}

extern "C" int lpcg_ic0_noalloc(const lpcg_system *s, double shift0, int32_t max_retries, float *l_val,
                                float *ut_val, double *shift_used, hipStream_t st) {
    if (!s || (!l_val && !ut_val) || shift0 < 0) {
        set_error("lpcg_ic0_noalloc: invalid arguments");
        return LPCG_EINVAL;
    }
    if ((size_t)s->nnz_l > kIc0ScratchDoubles) {
        set_error("lpcg_ic0_noalloc: nnz_l = %d exceeds the scratch limit of %zu entries "
                  "(LPCG_IC0_NOALLOC_MAX_NNZ_L); use lpcg_ic0", s->nnz_l, kIc0ScratchDoubles);
        return LPCG_EINVAL;
    }
    double *l64 = nullptr;
    int rc = ic0_scratch(&l64);
    if (rc) return rc;
    return ic0_run(s, shift0, max_retries, l_val, ut_val, shift_used, l64, st);
}

// Factor validation: the first row whose diagonal is not a positive finite
// number or that holds a non-finite entry (L rows store the diagonal last).
__global__ void k_check_factor(int n, const int *__restrict__ lrowptr, const float *__restrict__ lval,
                               int *__restrict__ bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int a = lrowptr[i], b = lrowptr[i + 1];
    bool ok = lval[b - 1] > 0.f && isfinite(lval[b - 1]);
    for (int k = a; k < b - 1; ++k) ok = ok && isfinite(lval[k]);
    if (!ok) atomicMin(bad, i);
}

extern "C" int lpcg_check_factor(const lpcg_system *s, const float *l_val, int32_t *bad_row, hipStream_t st) {
    if (!s || !l_val) {
        set_error("lpcg_check_factor: invalid arguments");
        return LPCG_EINVAL;
    }
    int *bad = s->ctrl + C_STATUS;  // scratch word (the solvers set it afresh)
    k_set_i32<<<1, 1, 0, st>>>(bad, 0x7fffffff);
    k_check_factor<<<nblk(s->n, 256), 256, 0, st>>>(s->n, s->lrowptr, l_val, bad);
    LPCG_LAUNCH_CHECK();
    int h = 0;
    LPCG_HIP(hipMemcpyAsync(&h, bad, sizeof(int), hipMemcpyDeviceToHost, st));
    LPCG_HIP(hipStreamSynchronize(st));
    if (bad_row) *bad_row = h == 0x7fffffff ? -1 : h;
    if (h != 0x7fffffff) {
        set_error("lpcg_check_factor: row %d (internal numbering) has a non-positive or non-finite diagonal or a "
                  "non-finite entry", h);
        return LPCG_ENONFINITE;
    }
    return LPCG_OK;
}

extern "C" int lpcg_sgs(const lpcg_system *s, float *l_val, float *ut_val, hipStream_t st) {
    if (!s || (!l_val && !ut_val)) {
        set_error("lpcg_sgs: invalid arguments");
        return LPCG_EINVAL;
    }
    k_sgs<<<nblk(s->nnz_l, 256), 256, 0, st>>>(s->nnz_l, s->lsrc, s->lcol, s->val64, s->diag64, s->u2l, l_val,
                                                ut_val);
    LPCG_LAUNCH_CHECK();
    return LPCG_OK;
}

namespace {
struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair() {
        if (a) hipEventDestroy(a);
        if (b) hipEventDestroy(b);
    }
};
}  // namespace

extern "C" int lpcg_time_sptrsv(const lpcg_system *s, int32_t transpose, const float *l_val,
                                const float *ut_val, const float *rhs, float *y, int32_t reps,
                                double *ms_out, hipStream_t st) {
    if (!s || !rhs || !y || rhs == y || reps <= 0 || !ms_out || (transpose ? !ut_val : !l_val)) {
        set_error("lpcg_time_sptrsv: invalid arguments");
        return LPCG_EINVAL;
    }
    EventPair ev;
    LPCG_HIP(hipEventCreate(&ev.a));
    LPCG_HIP(hipEventCreate(&ev.b));
    int *ticket = s->ctrl + C_TICKET_X;
    const TrsvCfg &c = s->trsv[transpose ? 1 : 0];
    double total = 0;
    for (int r = 0; r < reps; ++r) {
        int rc = trsv_presets(s, transpose, c, l_val, ut_val, y, ticket, st);
        if (rc) return rc;
        LPCG_HIP(hipEventRecord(ev.a, st));
        rc = trsv_kernels(s, transpose, c, l_val, ut_val, rhs, y, ticket, st);
        if (rc) return rc;
        LPCG_HIP(hipEventRecord(ev.b, st));
        LPCG_HIP(hipEventSynchronize(ev.b));
        float ms = 0;
        LPCG_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
        total += ms;
    }
    *ms_out = total / reps;
    return LPCG_OK;
}

extern "C" int lpcg_time_spmv(const lpcg_system *s, const float *x, float *y, int32_t reps,
                              double *ms_out, hipStream_t st) {
    if (!s || !x || !y || reps <= 0 || !ms_out) {
        set_error("lpcg_time_spmv: invalid arguments");
        return LPCG_EINVAL;
    }
    EventPair ev;
    LPCG_HIP(hipEventCreate(&ev.a));
    LPCG_HIP(hipEventCreate(&ev.b));
    LPCG_HIP(hipEventRecord(ev.a, st));
    for (int r = 0; r < reps; ++r) {
        int rc = spmv32(s, x, y, st);
        if (rc) return rc;
    }
    LPCG_HIP(hipEventRecord(ev.b, st));
    LPCG_HIP(hipEventSynchronize(ev.b));
    float ms = 0;
    LPCG_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
    *ms_out = (double)ms / reps;
    return LPCG_OK;
}

extern "C" int lpcg_blocked_schedule(int32_t n, const int32_t *rowptr, const int32_t *col, int32_t upper,
                                     int32_t block_rows, int32_t block_runs, lpcg_blk_schedule *out) {
    if (!out || !rowptr || !col || (upper != 0 && upper != 1)) {
        set_error("lpcg_blocked_schedule: invalid arguments");
        return LPCG_EINVAL;
    }
    BlkHost o;
    const int rc = blk_build(n, rowptr, col, upper, block_rows, block_runs > 0 ? block_runs : 1, o);
    if (rc) return rc;
    const int nch = (int)o.ch.size() / 2;
    const bool fill = out->brow && out->bch && out->chunks && out->rec && out->vsrc;
    if (fill && (out->nblocks != o.nb || out->nchunks != nch || out->deps != o.W)) {
        set_error("lpcg_blocked_schedule: output sized for another schedule");
        return LPCG_EINVAL;
    }
    out->deps = o.W;
    out->nblocks = o.nb;
    out->nchunks = nch;
    out->max_chunks = o.chmax;
    out->run_shift = o.lsh;
    out->run_stride = o.D;
    if (fill) {
        std::copy(o.brow.begin(), o.brow.end(), out->brow);
        std::copy(o.bch.begin(), o.bch.end(), out->bch);
        std::copy(o.ch.begin(), o.ch.end(), out->chunks);
        std::copy(o.rec.begin(), o.rec.end(), out->rec);
        std::copy(o.vsrc.begin(), o.vsrc.end(), out->vsrc);
    }
    return LPCG_OK;
}

extern "C" int lpcg_get_trsv_cfg(const lpcg_system *s, int32_t direction, lpcg_trsv_cfg *out) {
    if (!s || !out || direction < 0 || direction > 2) {
        set_error("lpcg_get_trsv_cfg: invalid arguments");
        return LPCG_EINVAL;
    }
    if (direction == 2) {  // the SpMV: lanes per row and grid
        std::memset(out, 0, sizeof(*out));
        out->direction = 2;
        out->mode = s->spmv_ell ? 1 : s->spmv_group;
        out->waves = s->spmv_ell ? std::max(1, std::min(kMaxSpmvBlocks, nblk(s->n, kVecThreads)))
                     : s->spmv_rows > 0 ? nblk(s->n, s->spmv_rows)
                                        : s->spmv_blocks;
        out->block_rows = s->spmv_ell ? 0 : s->spmv_rows;
        return LPCG_OK;
    }
    const TrsvCfg &c = s->trsv[direction];
    out->direction = direction;
    out->mode = c.mode;
    out->waves = c.mode == 0 ? trsv_waves(s->n, c.waves) : 0;
    out->backoff = c.backoff;
    out->block_stride = c.stride;
    out->block_rows = c.mode == 3 ? c.blk : 0;
    out->us = 0;
    out->block_runs = c.mode == 3 ? c.runs : 0;
    return LPCG_OK;
}

extern "C" int lpcg_set_trsv_cfg(lpcg_system *s, const lpcg_trsv_cfg *cfg) {
    if (s && cfg && cfg->direction == 2) {  // the SpMV: G lanes per row on `waves` blocks, or staged, or ELL
        const int G = cfg->mode, R = cfg->block_rows;
        if (G == 1) {  // the ELL form: rows of at most kEllMaxW entries (the gather form's settings stay)
            if (s->ea_w == 0 || s->nsys != 1) {
                set_error("lpcg_set_trsv_cfg: no ELL form (a row has more than %d entries, or a batched system)",
                          kEllMaxW);
                return LPCG_EINVAL;
            }
            s->spmv_ell = true;
            s->spmv_rows = 0;
            drop_graphs(s);
            return LPCG_OK;
        }
        if ((G != 4 && G != 8 && G != 16 && G != 32 && G != 64) || R < 0 ||
            (R == 0 && (cfg->waves < 1 || cfg->waves > kMaxSpmvBlocks))) {
            set_error("lpcg_set_trsv_cfg: SpMV lanes per row must be 4, 8, 16, 32 or 64 and blocks 1..%d",
                      kMaxSpmvBlocks);
            return LPCG_EINVAL;
        }
        if (R > 0) {  // LDS-staged: R rows per block
            int rc = spmv_prepare_window(s, R, 0);
            if (rc) {
                // the previous configuration stays in force, with its windows
                if (s->spmv_rows > 0) (void)spmv_prepare_window(s, s->spmv_rows, 0);
                return rc;
            }
        }
        s->spmv_group = G;
        if (R == 0) s->spmv_blocks = cfg->waves;
        s->spmv_rows = R;
        s->spmv_ell = false;
        drop_graphs(s);
        return LPCG_OK;
    }
    if (!s || !cfg || cfg->direction < 0 || cfg->direction > 1 || cfg->mode < 0 || cfg->mode > 3 ||
        cfg->waves < 0 || cfg->backoff < 0 || cfg->backoff > 64 ||
        (cfg->block_stride != 0 && cfg->block_stride != 1 && cfg->block_stride != 2 &&
         cfg->block_stride != 4 && cfg->block_stride != 8)) {
        set_error("lpcg_set_trsv_cfg: invalid configuration");
        return LPCG_EINVAL;
    }
    if (cfg->mode == 2 && !wg_mode_fits(s, cfg->direction)) {
        set_error("lpcg_set_trsv_cfg: a level has more than %d rows, too wide for the single-workgroup mode",
                  kWgRows * kWgThreads);
        return LPCG_EINVAL;
    }
    if (cfg->mode == 3) {  // builds the schedule (synchronous)
        const int rc = blk_prepare(s, cfg->direction, cfg->block_rows > 0 ? cfg->block_rows : 1024,
                                   cfg->block_runs > 0 ? cfg->block_runs : 1);
        if (rc) return rc;
    }
    TrsvCfg &c = s->trsv[cfg->direction];
    c.mode = cfg->mode;
    c.waves = cfg->waves;
    c.backoff = cfg->backoff;
    c.stride = cfg->block_stride > 0 ? cfg->block_stride : 1;
    c.blk = cfg->mode == 3 ? (cfg->block_rows > 0 ? cfg->block_rows : 1024) : 0;
    c.runs = cfg->mode == 3 && cfg->block_runs > 0 ? cfg->block_runs : 1;
    drop_graphs(s);  // the cached PCG graphs launch the old kernels
    return LPCG_OK;
}

extern "C" int lpcg_autotune(lpcg_system *s, const float *l_val, const float *ut_val, int32_t reps,
                             lpcg_trsv_cfg *table, int32_t table_len, int32_t *n_table, hipStream_t st) {
    if (!s || !l_val || !ut_val || reps <= 0 || (table_len > 0 && !table)) {
        set_error("lpcg_autotune: invalid arguments");
        return LPCG_EINVAL;
    }
    EventPair ev;
    LPCG_HIP(hipEventCreate(&ev.a));
    LPCG_HIP(hipEventCreate(&ev.b));
    // right-hand side of ones in p, result in w (PCG work vectors)
    k_fill_u32<<<nblk(s->n, 256), 256, 0, st>>>(s->n, (uint32_t *)s->p, 0x3f800000u);
    LPCG_LAUNCH_CHECK();
    int *ticket = s->ctrl + C_TICKET_X;
    int count = 0;
    for (int dir = 0; dir < 2; ++dir) {
        const int nlev = dir ? s->nlev_b : s->nlev_f;
        std::vector<TrsvCfg> cands;
        if (nlev <= kLevelModeTuneLevels) cands.push_back(TrsvCfg{1, 0, 1, 1});
        if (wg_mode_fits(s, dir)) cands.push_back(TrsvCfg{2, 0, 1, 1});
        for (int B : {512, 1024, 2048})  // blocked mode, where the rows and the LDS allow it
            if (B < s->n && blk_prepare(s, dir, B) == LPCG_OK)
                for (int bo : {0, 1})
                    for (int xl : {1, 8}) cands.push_back(TrsvCfg{3, 0, bo, xl, B, 1});  // 8: on XCD 0 only
        for (int B : {1024, 2048})  // banded blocks, where the pattern tiles into them
            for (int K : {2, 4, 8})
                if (B < s->n && blk_prepare(s, dir, B, K) == LPCG_OK)
                    for (int bo : {0, 1}) cands.push_back(TrsvCfg{3, 0, bo, 1, B, K});
        for (int w : {64, 128, 256, 512, 1024, 2048, 4096})
            for (int bo : {1, 4, 16, 64}) {
                if (w > trsv_waves(s->n, 1 << 30) && w != 64) continue;  // more waves than chunks
                cands.push_back(TrsvCfg{0, w, bo, 1});
                if (w <= 512) cands.push_back(TrsvCfg{0, w, bo, 8});  // all waves on one XCD
            }
        double best = 1e30, best0 = 1e30;
        TrsvCfg best_c = s->trsv[dir];
        for (const TrsvCfg &c : cands) {
            double tot = 0;
            for (int r = 0; r <= reps; ++r) {  // first run warms up
                int rc = trsv_presets(s, dir, c, l_val, ut_val, s->w, ticket, st);
                if (rc) return rc;
                LPCG_HIP(hipEventRecord(ev.a, st));
                rc = trsv_kernels(s, dir, c, l_val, ut_val, s->p, s->w, ticket, st);
                if (rc) return rc;
                LPCG_HIP(hipEventRecord(ev.b, st));
                LPCG_HIP(hipEventSynchronize(ev.b));
                float ms = 0;
                LPCG_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
                if (r > 0) tot += ms;
            }
            const double us = 1e3 * tot / reps;
            if (count < table_len) {
                lpcg_trsv_cfg &e = table[count];
                e.direction = dir;
                e.mode = c.mode;
                e.waves = c.mode == 0 ? trsv_waves(s->n, c.waves) : 0;
                e.backoff = c.backoff;
                e.block_stride = c.stride;
                e.block_rows = c.mode == 3 ? c.blk : 0;
                e.us = us;
                e.block_runs = c.mode == 3 ? c.runs : 0;
            }
            ++count;
            if (us < best) {
                best = us;
                best_c = c;
            }
            if (dir == 0 && c.mode == 0 && c.stride == 1 && us < best0) {  // IC(0) walks the same DAG
                best0 = us;
                s->ic0_cfg = c;
                s->ic0_tuned = true;
            }
        }
        // a two-level system applies L L^T in the PCG with the fused pair
        // (two launches for both directions), which needs the level mode in
        // both directions: it beats any pair of standalone substitutions
        if (s->two_level_p > 0) best_c = TrsvCfg{1, 0, 1, 1};
        if (best_c.mode == 3) {  // leave the winner's schedule in place
            const int rc = blk_prepare(s, dir, best_c.blk, best_c.runs);
            if (rc) return rc;
        }
        s->trsv[dir] = best_c;
    }
    // SpMV: lanes per row G (64 / G rows per wavefront) and grid size, then
    // the LDS-staged form with R rows per block where the windows fit.  Each
    // candidate is timed as the PCG's product kernel (p = z + beta p_prev,
    // w = A p and p.w; batches of reps back-to-back launches), which is where the choice
    // counts: the plain product ranks G = 4 and 8 within a few percent, the
    // PCG's form (two gathered vectors per entry) does not
    {
        double best = 1e30, best_gather = 1e30;
        int best_g = s->spmv_group, best_b = s->spmv_blocks, best_r = 0, gather_b = s->spmv_blocks;
        int gather_g = s->spmv_group;
        auto time_one = [&](int G, int blocks, int R, double &us) -> int {
            const int rc = time_pcg_product(s, G, blocks, R, reps, us, st);
            if (rc) return rc;
            if (count < table_len) {
                lpcg_trsv_cfg &e = table[count];
                std::memset(&e, 0, sizeof(e));
                e.direction = 2;
                e.mode = G;
                e.waves = R > 0 ? nblk(s->n, R) : blocks;
                e.block_rows = R;
                e.us = us;
            }
            ++count;
            if (us < best) {
                best = us;
                best_g = G;
                best_b = blocks;
                best_r = R;
            }
            if (G > 1 && R == 0 && us < best_gather) {
                best_gather = us;
                gather_g = G;
                gather_b = blocks;
            }
            return LPCG_OK;
        };
        for (int G : {4, 8, 16, 32, 64})
            for (int cap : {512, 1024, 2048}) {
                const int blocks = std::max(1, std::min(cap, nblk(s->n, kVecThreads / G)));
                if (cap > 512 && blocks < cap / 2) continue;  // the same grid as a smaller cap
                double us;
                int rc = time_one(G, blocks, 0, us);
                if (rc) return rc;
            }
        for (int R : {256, 512, 1024}) {
            if (nblk(s->n, R) > kMaxSpmvBlocks || spmv_prepare_window(s, R, st) != LPCG_OK) continue;
            for (int G : {4, 8}) {
                double us;
                int rc = time_one(G, 0, R, us);
                if (rc) return rc;
            }
        }
        if (s->ea_w > 0) {  // the ELL form (one row per lane)
            double us;
            const int eb = std::max(1, std::min(kMaxSpmvBlocks, nblk(s->n, kVecThreads)));
            int rc = time_one(1, eb, 0, us);
            if (rc) return rc;
            // it stays unless another form is at least 10% faster: it moves
            // the fewest bytes and needs no lanes-per-row choice, and timings
            // taken under a profiler (whose per-launch cost narrows every
            // gap) then still pick it
            if (us <= 1.1 * best) {
                best = us;
                best_g = 1;
                best_b = eb;
                best_r = 0;
            }
        }
        // the gather form's lanes and grid stay valid ones (the FP64 product
        // and any later gather-form launch use them) when the staged or the
        // ELL form wins
        s->spmv_ell = best_g == 1;
        s->spmv_group = best_g == 1 ? gather_g : best_g;
        s->spmv_blocks = best_r > 0 || best_g == 1 ? gather_b : best_b;
        s->spmv_rows = best_r;
        if (best_r > 0) {
            int rc = spmv_prepare_window(s, best_r, st);
            if (rc) return rc;
        }
    }
    if (n_table) *n_table = count;
    drop_graphs(s);
    return LPCG_OK;
}
