// Pattern analysis: the graph view of A (Method, "Learning Preconditioners":
// every stored A_ij is a directed edge i -> j) and the dependency structure of
// the triangular solves with L on tril(A) and with L^T.
//
// Integer work, done once per sparsity pattern, on the GPU:
//   1. per-row validation (ascending unique columns, diagonal present), row of
//      every entry, position of the diagonal, count of lower entries;
//   2. reverse-edge map rev[k] (binary search of (j,i) in row j);
//   3. lower CSR of L (diagonal last) and upper CSR of U = L^T (diagonal
//      first) with the U -> L position map (through rev);
//   4. forward / backward levels, level(i) = 1 + max level of the rows i
//      depends on (0 if none), computed by a dependency-driven kernel;
//   5. level sets: rows sorted by (level, row) with a stable radix sort.
// Optional multicolour ordering (LPCG_ORDER_COLOR): first-fit colours in row
// order on the lower-triangle graph (a dependency-driven kernel over the
// forward levels of the natural ordering), rows stably sorted by (system,
// colour), and the analysis above repeated on P A P^T.  Rows of one colour
// are mutually independent, so the triangular solves of the reordered system
// have at most as many levels as there are colours (2 on a grid graph:
// red-black).  This reordering is a solver-side choice, not part of the
// method; the preconditioner it gives differs from the natural-order one.
#include <hipcub/hipcub.hpp>

#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "device_util.h"
#include "lpcg_internal.h"

namespace lpcg {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int hip_fail(hipError_t e, const char *what, const char *file, int line) {
    set_error("HIP error %d (%s) in %s at %s:%d", (int)e, hipGetErrorString(e), what, file, line);
    return LPCG_EHIP;
}

namespace {

enum AnalyzeErr : int {
    E_COL_RANGE = 1,
    E_UNSORTED = 2,
    E_NO_DIAG = 4,
    E_UNSYM = 8,
    E_CROSS_SYS = 16,
};

__global__ void k_rows(int n, const int *__restrict__ rowptr, const int *__restrict__ col,
                       const int *__restrict__ row_sys, const int *__restrict__ sys_rowptr,
                       int *__restrict__ erow, int *__restrict__ dpos, int *__restrict__ nl,
                       int *__restrict__ nu, int *err) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int a = rowptr[i], b = rowptr[i + 1];
    int lo = sys_rowptr[row_sys[i]], hi = sys_rowptr[row_sys[i] + 1];
    int e = 0, d = -1, cl = 0, prev = -1;
    for (int k = a; k < b; ++k) {
        int j = col[k];
        erow[k] = i;
        if (j < 0 || j >= n) { e |= E_COL_RANGE; continue; }
        if (j <= prev) e |= E_UNSORTED;
        if (j < lo || j >= hi) e |= E_CROSS_SYS;
        prev = j;
        if (j == i) d = k;
        if (j <= i) ++cl;
    }
    if (d < 0) e |= E_NO_DIAG;
    dpos[i] = d;
    nl[i] = cl;
    nu[i] = (b - a) - cl + 1;
    if (e) atomicOr(err, e);
}

__global__ void k_rev(int nnz, const int *__restrict__ rowptr, const int *__restrict__ col,
                      const int *__restrict__ erow, int *__restrict__ rev, int *err) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nnz) return;
    int i = erow[k], j = col[k];
    int lo = rowptr[j], hi = rowptr[j + 1] - 1, found = -1;
    while (lo <= hi) {
        int mid = (lo + hi) >> 1;
        int c = col[mid];
        if (c == i) { found = mid; break; }
        if (c < i) lo = mid + 1; else hi = mid - 1;
    }
    rev[k] = found;
    if (found < 0) atomicOr(err, (int)E_UNSYM);
}

__global__ void k_fill_lu(int n, const int *__restrict__ rowptr, const int *__restrict__ col,
                          const int *__restrict__ dpos, const int *__restrict__ rev,
                          const int *__restrict__ lrowptr, const int *__restrict__ urowptr,
                          int *__restrict__ lcol, int *__restrict__ lsrc, int *__restrict__ ucol,
                          int *__restrict__ u2l) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int a = rowptr[i], d = dpos[i], b = rowptr[i + 1];
    int lo = lrowptr[i];
    for (int k = a; k <= d; ++k) {
        lcol[lo + (k - a)] = col[k];
        lsrc[lo + (k - a)] = k;
    }
    int uo = urowptr[i];
    for (int k = d; k < b; ++k) {
        int q = uo + (k - d);
        int j = col[k];
        ucol[q] = j;
        // entry (j, i) of A is a lower entry of row j: its L position
        int kr = rev[k];
        u2l[q] = lrowptr[j] + (kr - rowptr[j]);
    }
}

// Longest-path level of every row of a triangular dependency DAG.  UPPER = 0:
// rows ascending, row i waits for the strictly-lower columns of its L row;
// UPPER = 1: rows descending, waits for the strictly-upper columns of its U
// row.  level[] is preset to -1; a published level (>= 0) is its own ready
// flag.  Rows are handed out in a topological order through a ticket, so
// every row a wave waits on belongs to a wave that is already running; lanes
// never block inside the wave (each retry re-reads only what is missing).
template <bool UPPER>
__global__ void k_levels(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                         int *level, int *ticket) {
    const int lane = lane_id();
    for (;;) {
        const int chunk = wave_ticket(ticket);
        if ((long)chunk * kWave >= n) break;
        int pos = chunk * kWave + lane;
        int row = -1, k = 0, kend = 0, lv = 0;
        if (pos < n) {
            row = UPPER ? n - 1 - pos : pos;
            k = UPPER ? rp[row] + 1 : rp[row];
            kend = UPPER ? rp[row + 1] : rp[row + 1] - 1;
        }
        bool pending = row >= 0;
        while (__ballot(pending) != 0) {
            if (pending) {
                while (k < kend) {
                    int v = ld_agent_i(&level[ci[k]]);
                    if (v < 0) break;
                    lv = max(lv, v + 1);
                    ++k;
                }
                if (k == kend) {
                    st_agent_i(&level[row], lv);
                    pending = false;
                }
            }
            if (pending) __builtin_amdgcn_s_sleep(1);
        }
    }
}

// First-fit colour of every row (rows handed out in forward level order,
// so a row only waits on rows handed out earlier): colour(i) = smallest
// c >= 0 that no strictly-lower neighbour j of row i has.  color[] is preset
// to -1; a published colour is its own ready flag.
__global__ void k_colors(int n, const int *__restrict__ order, const int *__restrict__ lrp,
                         const int *__restrict__ lci, int *color, int *ticket) {
    const int lane = lane_id();
    for (;;) {
        const int chunk = wave_ticket(ticket);
        if ((long)chunk * kWave >= n) break;
        const int pos = chunk * kWave + lane;
        int row = -1, k0 = 0, k = 0, kend = 0;
        if (pos < n) {
            row = order[pos];
            k0 = k = lrp[row];
            kend = lrp[row + 1] - 1;  // diagonal last
        }
        bool pending = row >= 0;
        while (__ballot(pending) != 0) {
            if (pending) {
                while (k < kend && ld_agent_i(&color[lci[k]]) >= 0) ++k;
                if (k == kend) {
                    // every neighbour's colour is final: take the smallest free one
                    uint64_t taken = 0;
                    bool big = false;
                    for (int q = k0; q < kend; ++q) {
                        const int c = ld_agent_i(&color[lci[q]]);
                        if (c < 64) taken |= 1ull << c;
                        else big = true;
                    }
                    int c = taken == ~0ull ? 64 : __builtin_ctzll(~taken);
                    if (big || c == 64) {  // rare: colours beyond 63 among the neighbours
                        for (bool hit = true; hit;) {
                            hit = false;
                            for (int q = k0; q < kend && !hit; ++q) hit = ld_agent_i(&color[lci[q]]) == c;
                            if (hit) ++c;
                        }
                    }
                    st_agent_i(&color[row], c);
                    pending = false;
                }
            }
            if (pending) __builtin_amdgcn_s_sleep(1);
        }
    }
}

__global__ void k_color_keys(int n, const int *__restrict__ row_sys, const int *__restrict__ color,
                             int ncolors, int *__restrict__ keys, int *__restrict__ iota) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    keys[i] = row_sys[i] * ncolors + color[i];
    iota[i] = i;
}

__global__ void k_perm_rows(int n, const int *__restrict__ perm, const int *__restrict__ rowptr,
                            int *__restrict__ iperm, int *__restrict__ len) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int o = perm[r];
    iperm[o] = r;
    len[r] = rowptr[o + 1] - rowptr[o];
}

// Row r of P A P^T: the entries of original row perm[r], columns renumbered
// through iperm and sorted ascending (insertion sort; rows are short).
// psrc[k'] = original position of internal entry k'.
__global__ void k_perm_fill(int n, const int *__restrict__ perm, const int *__restrict__ iperm,
                            const int *__restrict__ rowptr, const int *__restrict__ col,
                            const int *__restrict__ nrp, int *__restrict__ ncol, int *__restrict__ psrc) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int o = perm[r], a = rowptr[o], len = rowptr[o + 1] - a, base = nrp[r];
    for (int t = 0; t < len; ++t) {
        const int c = iperm[col[a + t]], src = a + t;
        int q = t;
        while (q > 0 && ncol[base + q - 1] > c) {
            ncol[base + q] = ncol[base + q - 1];
            psrc[base + q] = psrc[base + q - 1];
            --q;
        }
        ncol[base + q] = c;
        psrc[base + q] = src;
    }
}

__global__ void k_gather_vals(int nnz, const int *__restrict__ psrc, const double *__restrict__ v,
                              double *__restrict__ out) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nnz) out[k] = v[psrc[k]];
}

template <typename T>
__global__ void k_vec_gather(int n, const int *__restrict__ perm, const T *__restrict__ src, T *__restrict__ dst) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) dst[r] = src[perm[r]];
}

// Two vectors into the internal order in one launch (a solve's b and x).
__global__ void k_vec_gather2(int n, const int *__restrict__ perm, const double *__restrict__ s0,
                              double *__restrict__ d0, const double *__restrict__ s1, double *__restrict__ d1) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) {
        const int q = perm[r];
        const double v0 = s0[q], v1 = s1[q];
        d0[r] = v0;
        d1[r] = v1;
    }
}

template <typename T>
__global__ void k_vec_scatter(int n, const int *__restrict__ perm, const T *__restrict__ src, T *__restrict__ dst) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) dst[perm[r]] = src[r];
}

// Level-ordered packed pattern of one triangular factor (UPPER = 0: L rows,
// diagonal last; UPPER = 1: U rows, diagonal first), rows in `order`.
template <bool UPPER>
__global__ void k_lo_count(int n, const int *__restrict__ order, const int *__restrict__ rp, int *__restrict__ cnt) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int row = order[q];
    cnt[q] = rp[row + 1] - rp[row] - 1;
}

template <bool UPPER>
__global__ void k_lo_fill(int n, const int *__restrict__ order, const int *__restrict__ rp,
                          const int *__restrict__ ci, const int *__restrict__ ptr, int *__restrict__ col,
                          int *__restrict__ src, int *__restrict__ dsrc) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int row = order[q], a = rp[row], b = rp[row + 1];
    const int k0 = UPPER ? a + 1 : a, k1 = UPPER ? b : b - 1;
    int e = ptr[q];
    for (int k = k0; k < k1; ++k, ++e) {
        col[e] = ci[k];
        src[e] = k;
    }
    dsrc[q] = UPPER ? a : b - 1;
}

__global__ void k_iota_fill(int n, int *iota, int *lev_f, int *lev_b) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        iota[i] = i;
        if (lev_f) lev_f[i] = -1;
        if (lev_b) lev_b[i] = -1;
    }
}

// lev_ptr from keys sorted ascending: levels are contiguous 0..nlev-1 (every
// level of a longest-path layering is nonempty).
__global__ void k_lev_ptr(int n, const int *__restrict__ skey, int *__restrict__ lev_ptr) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (i == 0 || skey[i] != skey[i - 1]) lev_ptr[skey[i]] = i;
    if (i == n - 1) lev_ptr[skey[i] + 1] = n;
}

__global__ void k_row_sys(int nsys, const int *__restrict__ sys_rowptr, int *__restrict__ row_sys) {
    int s = blockIdx.x;
    if (s >= nsys) return;
    for (int i = sys_rowptr[s] + threadIdx.x; i < sys_rowptr[s + 1]; i += blockDim.x) row_sys[i] = s;
}

// Values in internal order (psrc: gather from the caller's entry order, or
// null for the natural ordering); diagonal copy for Jacobi and the GNN.
__global__ void k_values(int nnz, int n, const double *__restrict__ v64, const int *__restrict__ psrc,
                         const int *__restrict__ dpos, double *__restrict__ val64,
                         float *__restrict__ val32, double *__restrict__ diag64) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nnz) {
        double v = v64[psrc ? psrc[k] : k];
        val64[k] = v;
        val32[k] = (float)v;
    }
    if (k < n) diag64[k] = v64[psrc ? psrc[dpos[k]] : dpos[k]];
}

int nblk(long n, int t) { return (int)((n + t - 1) / t); }

// dst[i] = src[pos[i]] (pos < 0: padding, 0)
__global__ void k_ell_pack(long count, const int *__restrict__ pos, const float *__restrict__ src,
                           float *__restrict__ dst) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) {
        const int k = pos[i];
        dst[i] = k >= 0 ? src[k] : 0.f;
    }
}

__global__ void k_fill_part(long n, uint64_t *p) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = kPartUnset;
}

template <typename T>
int dalloc(lpcg_system *s, T **p, size_t count) {
    void *q = nullptr;
    size_t bytes = count * sizeof(T);
    if (bytes == 0) bytes = sizeof(T);
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) {
        set_error("hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
        return LPCG_ENOMEM;
    }
    s->allocs.push_back(q);
    *p = (T *)q;
    return LPCG_OK;
}

// Levels of one direction + level sets.
int build_levels(lpcg_system *s, bool upper, int *level, int *lev_ptr_tmp_out_unused, hipStream_t st,
                 int **lev_ptr, int **lev_rows, std::vector<int> &h_ptr, int &nlev, int &maxw,
                 int *iota, int *keys_out, int *ticket) {
    (void)lev_ptr_tmp_out_unused;
    const int n = s->n;
    LPCG_HIP(hipMemsetAsync(ticket, 0, sizeof(int), st));
    const int waves = std::min(nblk(n, kWave), 8192);
    if (upper)
        k_levels<true><<<nblk(waves, 4), 256, 0, st>>>(n, s->urowptr, s->ucol, level, ticket);
    else
        k_levels<false><<<nblk(waves, 4), 256, 0, st>>>(n, s->lrowptr, s->lcol, level, ticket);
    LPCG_LAUNCH_CHECK();
    // max level -> number of levels
    int *d_max = nullptr;
    int rc;
    if ((rc = dalloc(s, &d_max, 1))) return rc;
    size_t tmp_bytes = 0;
    LPCG_HIP(hipcub::DeviceReduce::Max(nullptr, tmp_bytes, level, d_max, n, st));
    void *tmp = nullptr;
    LPCG_HIP(hipMallocAsync(&tmp, tmp_bytes, st));
    LPCG_HIP(hipcub::DeviceReduce::Max(tmp, tmp_bytes, level, d_max, n, st));
    int hmax = 0;
    LPCG_HIP(hipMemcpyAsync(&hmax, d_max, sizeof(int), hipMemcpyDeviceToHost, st));
    LPCG_HIP(hipStreamSynchronize(st));
    LPCG_HIP(hipFreeAsync(tmp, st));
    nlev = hmax + 1;
    int bits = 1;
    while ((1 << bits) <= hmax) ++bits;
    int rc2;
    if ((rc2 = dalloc(s, lev_rows, n))) return rc2;
    if ((rc2 = dalloc(s, lev_ptr, nlev + 1))) return rc2;
    tmp_bytes = 0;
    LPCG_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, level, keys_out, iota, *lev_rows,
                                                n, 0, bits, st));
    LPCG_HIP(hipMallocAsync(&tmp, tmp_bytes, st));
    LPCG_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, level, keys_out, iota, *lev_rows, n,
                                                0, bits, st));
    k_lev_ptr<<<nblk(n, 256), 256, 0, st>>>(n, keys_out, *lev_ptr);
    LPCG_LAUNCH_CHECK();
    h_ptr.resize(nlev + 1);
    LPCG_HIP(hipMemcpyAsync(h_ptr.data(), *lev_ptr, sizeof(int) * (nlev + 1), hipMemcpyDeviceToHost, st));
    LPCG_HIP(hipStreamSynchronize(st));
    LPCG_HIP(hipFreeAsync(tmp, st));
    maxw = 0;
    for (int i = 0; i < nlev; ++i) maxw = std::max(maxw, h_ptr[i + 1] - h_ptr[i]);
    return LPCG_OK;
}

int analyze_impl(const lpcg_csr *A, const int32_t *h_sys, int32_t nsys, lpcg_system *s,
                 hipStream_t st) {
    const int n = A->n, nnz = A->nnz;
    s->n = n;
    s->nnz = nnz;
    s->nsys = nsys;
    int rc;
#define ALLOC(p, c) if ((rc = dalloc(s, &(p), (size_t)(c)))) return rc
    ALLOC(s->rowptr, n + 1);
    ALLOC(s->colind, nnz);
    ALLOC(s->erow, nnz);
    ALLOC(s->dpos, n);
    ALLOC(s->rev, nnz);
    ALLOC(s->lrowptr, n + 1);
    ALLOC(s->urowptr, n + 1);
    ALLOC(s->sys_rowptr, nsys + 1);
    ALLOC(s->row_sys, n);
    LPCG_HIP(hipMemcpyAsync(s->rowptr, A->rowptr, sizeof(int) * (n + 1), hipMemcpyDeviceToDevice, st));
    LPCG_HIP(hipMemcpyAsync(s->colind, A->colind, sizeof(int) * (size_t)nnz, hipMemcpyDeviceToDevice, st));
    s->h_sys_rowptr.assign(h_sys, h_sys + nsys + 1);
    LPCG_HIP(hipMemcpyAsync(s->sys_rowptr, s->h_sys_rowptr.data(), sizeof(int) * (nsys + 1),
                            hipMemcpyHostToDevice, st));
    k_row_sys<<<nsys, 256, 0, st>>>(nsys, s->sys_rowptr, s->row_sys);
    LPCG_LAUNCH_CHECK();
    int *nl = nullptr, *nu = nullptr, *err = nullptr;
    ALLOC(nl, n + 1);
    ALLOC(nu, n + 1);
    ALLOC(err, 1);
    LPCG_HIP(hipMemsetAsync(err, 0, sizeof(int), st));
    LPCG_HIP(hipMemsetAsync(nl + n, 0, sizeof(int), st));
    LPCG_HIP(hipMemsetAsync(nu + n, 0, sizeof(int), st));
    // rowptr sanity is checked on the host copy of its endpoints
    int ends[2];
    LPCG_HIP(hipMemcpyAsync(&ends[0], A->rowptr, sizeof(int), hipMemcpyDeviceToHost, st));
    LPCG_HIP(hipMemcpyAsync(&ends[1], A->rowptr + n, sizeof(int), hipMemcpyDeviceToHost, st));
    LPCG_HIP(hipStreamSynchronize(st));
    if (ends[0] != 0 || ends[1] != nnz) {
        set_error("rowptr[0] = %d, rowptr[n] = %d, expected 0 and nnz = %d", ends[0], ends[1], nnz);
        return LPCG_EINVAL;
    }
    k_rows<<<nblk(n, 256), 256, 0, st>>>(n, s->rowptr, s->colind, s->row_sys, s->sys_rowptr, s->erow,
                                          s->dpos, nl, nu, err);
    LPCG_LAUNCH_CHECK();
    int herr = 0;
    LPCG_HIP(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
    LPCG_HIP(hipStreamSynchronize(st));
    if (herr) {
        set_error("invalid CSR pattern (flags %d: 1 column out of range, 2 unsorted/duplicate, "
                  "4 missing diagonal, 16 row crosses a system boundary)", herr);
        return LPCG_EINVAL;
    }
    k_rev<<<nblk(nnz, 256), 256, 0, st>>>(nnz, s->rowptr, s->colind, s->erow, s->rev, err);
    LPCG_LAUNCH_CHECK();
    LPCG_HIP(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
    LPCG_HIP(hipStreamSynchronize(st));
    if (herr) {
        set_error("pattern is not structurally symmetric");
        return LPCG_EINVAL;
    }
    // exclusive scans -> lrowptr, urowptr
    size_t tb = 0;
    LPCG_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, nl, s->lrowptr, n + 1, st));
    void *tmp = nullptr;
    LPCG_HIP(hipMallocAsync(&tmp, tb, st));
    LPCG_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tb, nl, s->lrowptr, n + 1, st));
    LPCG_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tb, nu, s->urowptr, n + 1, st));
    int nnzl = 0, nnzu = 0;
    LPCG_HIP(hipMemcpyAsync(&nnzl, s->lrowptr + n, sizeof(int), hipMemcpyDeviceToHost, st));
    LPCG_HIP(hipMemcpyAsync(&nnzu, s->urowptr + n, sizeof(int), hipMemcpyDeviceToHost, st));
    LPCG_HIP(hipStreamSynchronize(st));
    LPCG_HIP(hipFreeAsync(tmp, st));
    if (nnzl != nnzu) {
        set_error("lower/upper counts differ (%d vs %d)", nnzl, nnzu);
        return LPCG_EINVAL;
    }
    s->nnz_l = nnzl;
    ALLOC(s->lcol, nnzl);
    ALLOC(s->lsrc, nnzl);
    ALLOC(s->ucol, nnzl);
    ALLOC(s->u2l, nnzl);
    k_fill_lu<<<nblk(n, 256), 256, 0, st>>>(n, s->rowptr, s->colind, s->dpos, s->rev, s->lrowptr,
                                             s->urowptr, s->lcol, s->lsrc, s->ucol, s->u2l);
    LPCG_LAUNCH_CHECK();
    // levels
    int *iota = nullptr, *keys = nullptr, *ticket = nullptr;
    ALLOC(s->flevel, n);
    ALLOC(s->blevel, n);
    ALLOC(iota, n);
    ALLOC(keys, n);
    ALLOC(ticket, 1);
    k_iota_fill<<<nblk(n, 256), 256, 0, st>>>(n, iota, s->flevel, s->blevel);
    LPCG_LAUNCH_CHECK();
    if ((rc = build_levels(s, false, s->flevel, nullptr, st, &s->flev_ptr, &s->flev_rows, s->h_flev_ptr,
                           s->nlev_f, s->max_w_f, iota, keys, ticket)))
        return rc;
    if ((rc = build_levels(s, true, s->blevel, nullptr, st, &s->blev_ptr, &s->blev_rows, s->h_blev_ptr,
                           s->nlev_b, s->max_w_b, iota, keys, ticket)))
        return rc;
    // level-ordered packed patterns for the single-workgroup substitution
    for (int d = 0; d < 2; ++d) {
        const int *order = d ? s->blev_rows : s->flev_rows;
        const int *rp = d ? s->urowptr : s->lrowptr;
        const int *ci = d ? s->ucol : s->lcol;
        const int noff = s->nnz_l - n;
        ALLOC(s->lo_ptr[d], n + 1);
        ALLOC(s->lo_col[d], std::max(noff, 1));
        ALLOC(s->lo_src[d], std::max(noff, 1));
        ALLOC(s->lo_dsrc[d], n);
        ALLOC(s->lo_val[d], std::max(noff, 1));
        ALLOC(s->lo_diag[d], n);
        int *cnt = nl;  // n + 1 ints of scratch (the lower counts are no longer needed)
        if (d) k_lo_count<true><<<nblk(n, 256), 256, 0, st>>>(n, order, rp, cnt);
        else k_lo_count<false><<<nblk(n, 256), 256, 0, st>>>(n, order, rp, cnt);
        LPCG_HIP(hipMemsetAsync(cnt + n, 0, sizeof(int), st));
        size_t tb2 = 0;
        LPCG_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb2, cnt, s->lo_ptr[d], n + 1, st));
        void *tmp2 = nullptr;
        LPCG_HIP(hipMallocAsync(&tmp2, tb2, st));
        LPCG_HIP(hipcub::DeviceScan::ExclusiveSum(tmp2, tb2, cnt, s->lo_ptr[d], n + 1, st));
        LPCG_HIP(hipFreeAsync(tmp2, st));
        if (d)
            k_lo_fill<true><<<nblk(n, 256), 256, 0, st>>>(n, order, rp, ci, s->lo_ptr[d], s->lo_col[d],
                                                            s->lo_src[d], s->lo_dsrc[d]);
        else
            k_lo_fill<false><<<nblk(n, 256), 256, 0, st>>>(n, order, rp, ci, s->lo_ptr[d], s->lo_col[d],
                                                             s->lo_src[d], s->lo_dsrc[d]);
        LPCG_LAUNCH_CHECK();
    }
    // values and solver work space
    ALLOC(s->val64, nnz);
    ALLOC(s->val32, nnz);
    ALLOC(s->diag64, n);
    ALLOC(s->r, n);
    ALLOC(s->p, n);
    ALLOC(s->p2, n);
    ALLOC(s->w, n);
    ALLOC(s->z, n);
    ALLOC(s->y, n);
    ALLOC(s->dinv, n);
    ALLOC(s->t64a, n);
    ALLOC(s->t64b, n);
    ALLOC(s->t64c, n);
    ALLOC(s->sys_tmp, 2 * (size_t)nsys);
    s->vec_blocks = std::max(1, std::min(kMaxVecBlocks, nblk(n, kVecThreads)));
    const int chunks = nblk(n, kWave);
    // per-block partials: vector kernels, SpMV, one per 64-row chunk of the
    // dependency-driven substitution, or one per block of the level launches
    s->npart = std::max(std::max(kMaxVecBlocks, kMaxSpmvBlocks), chunks + std::max(s->nlev_f, s->nlev_b));
    // batched-solve segments (host-built from the system boundaries)
    {
        std::vector<int> ss, r0, r1, sp(nsys + 1, 0);
        for (int sy = 0; sy < nsys; ++sy) {
            sp[sy] = (int)ss.size();
            for (int a0 = s->h_sys_rowptr[sy]; a0 < s->h_sys_rowptr[sy + 1]; a0 += kSegRows) {
                ss.push_back(sy);
                r0.push_back(a0);
                r1.push_back(std::min(a0 + kSegRows, s->h_sys_rowptr[sy + 1]));
            }
        }
        sp[nsys] = (int)ss.size();
        s->nseg = (int)ss.size();
        ALLOC(s->seg_sys, s->nseg);
        ALLOC(s->seg_row0, s->nseg);
        ALLOC(s->seg_row1, s->nseg);
        ALLOC(s->sys_seg_ptr, nsys + 1);
        LPCG_HIP(hipMemcpyAsync(s->seg_sys, ss.data(), sizeof(int) * s->nseg, hipMemcpyHostToDevice, st));
        LPCG_HIP(hipMemcpyAsync(s->seg_row0, r0.data(), sizeof(int) * s->nseg, hipMemcpyHostToDevice, st));
        LPCG_HIP(hipMemcpyAsync(s->seg_row1, r1.data(), sizeof(int) * s->nseg, hipMemcpyHostToDevice, st));
        LPCG_HIP(hipMemcpyAsync(s->sys_seg_ptr, sp.data(), sizeof(int) * (nsys + 1), hipMemcpyHostToDevice, st));
        LPCG_HIP(hipStreamSynchronize(st));  // the host vectors go out of scope
        ALLOC(s->bscal, 8 * (size_t)nsys);
        ALLOC(s->bctrl, 8 * (size_t)nsys);
        ALLOC(s->ir_rel, nsys);
        ALLOC(s->ir_flag, nsys);
        s->npart = std::max(s->npart, s->nseg);
    }
    ALLOC(s->part, 4 * (size_t)s->npart);
    ALLOC(s->sync_part, 4 * (size_t)s->npart);
    k_fill_part<<<nblk(4L * s->npart, 256), 256, 0, st>>>(4L * s->npart, (uint64_t *)s->sync_part);
    ALLOC(s->scal, S_NSCAL);
    ALLOC(s->ctrl, C_NCTRL);
    LPCG_HIP(hipHostMalloc((void **)&s->h_ctrl, sizeof(int) * C_NCTRL, hipHostMallocDefault));
    LPCG_HIP(hipHostMalloc((void **)&s->h_scal, sizeof(double) * S_NSCAL, hipHostMallocDefault));
    // substitution defaults: level-synchronous launches when there are few
    // levels (multicolour orderings), dependency driven otherwise
    const double lmean = (double)s->nnz_l / n;
    s->trsv_g = lmean <= 4 ? 4 : lmean <= 8 ? 8 : 16;
    s->trsv[0].mode = s->nlev_f <= kLevelModeMaxLevels ? 1 : 0;
    s->trsv[1].mode = s->nlev_b <= kLevelModeMaxLevels ? 1 : 0;
    {  // row-aligned tiles of at most 32 entries for the network's fused pass
        std::vector<int> hrp(n + 1), tiles(1, 0);
        LPCG_HIP(hipMemcpyAsync(hrp.data(), s->rowptr, sizeof(int) * (n + 1), hipMemcpyDeviceToHost, st));
        LPCG_HIP(hipStreamSynchronize(st));
        bool ok = true;
        for (int r = 0; r < n && ok;) {
            int r1 = r;
            while (r1 < n && hrp[r1 + 1] - hrp[r] <= 32) ++r1;
            ok = r1 > r;
            tiles.push_back(r1);
            r = r1;
        }
        s->gtiles = 0;
        if (ok) {
            std::vector<int> te(tiles.size());
            for (size_t j = 0; j < tiles.size(); ++j) te[j] = hrp[tiles[j]];
            ALLOC(s->gtile_row, tiles.size());
            ALLOC(s->gtile_e, tiles.size());
            LPCG_HIP(hipMemcpyAsync(s->gtile_row, tiles.data(), sizeof(int) * tiles.size(), hipMemcpyHostToDevice,
                                    st));
            LPCG_HIP(hipMemcpyAsync(s->gtile_e, te.data(), sizeof(int) * te.size(), hipMemcpyHostToDevice, st));
            LPCG_HIP(hipStreamSynchronize(st));
            s->gtiles = (int)tiles.size() - 1;
        }
    }
    s->two_level_p = 0;
    if (s->nlev_f == 2 && s->h_flev_ptr.size() == 3 && s->h_flev_ptr[1] > 0) {
        // level 0 lists its rows ascending: it is the prefix [0, p) exactly
        // when its last row is p - 1
        const int p = s->h_flev_ptr[1];
        int last = -1;
        LPCG_HIP(hipMemcpyAsync(&last, s->flev_rows + (p - 1), sizeof(int), hipMemcpyDeviceToHost, st));
        LPCG_HIP(hipStreamSynchronize(st));
        if (last == p - 1) s->two_level_p = p;
    }
    // ELL forms of single systems (the batched solver does not use them): A,
    // and the two-level pair's suffix rows of L and prefix rows of U = L^T
    if (nsys == 1) {
        std::vector<int> hrp(n + 1), hci(nnz);
        LPCG_HIP(hipMemcpyAsync(hrp.data(), s->rowptr, sizeof(int) * (n + 1), hipMemcpyDeviceToHost, st));
        LPCG_HIP(hipMemcpyAsync(hci.data(), s->colind, sizeof(int) * (size_t)nnz, hipMemcpyDeviceToHost, st));
        LPCG_HIP(hipStreamSynchronize(st));
        int wa = 0;
        for (int i = 0; i < n; ++i) wa = std::max(wa, hrp[i + 1] - hrp[i]);
        if (wa >= 1 && wa <= kEllMaxW) {
            const size_t m = (size_t)wa * n;
            std::vector<int> col(m), pos(m);
            for (int t = 0; t < wa; ++t)
                for (int i = 0; i < n; ++i) {
                    const int k = hrp[i] + t;
                    const bool real = k < hrp[i + 1];
                    col[(size_t)t * n + i] = real ? hci[k] : i;
                    pos[(size_t)t * n + i] = real ? k : -1;
                }
            ALLOC(s->ea_col, m);
            ALLOC(s->ea_pos, m);
            ALLOC(s->ea_val, m);
            LPCG_HIP(hipMemcpyAsync(s->ea_col, col.data(), sizeof(int) * m, hipMemcpyHostToDevice, st));
            LPCG_HIP(hipMemcpyAsync(s->ea_pos, pos.data(), sizeof(int) * m, hipMemcpyHostToDevice, st));
            LPCG_HIP(hipStreamSynchronize(st));
            s->ea_w = wa;
        }
        const int p = s->two_level_p;
        if (p > 0 && p < n) {
            const int nb = n - p;
            std::vector<int> lrp(n + 1), lc(nnzl), urp(n + 1), uc(nnzl);
            LPCG_HIP(hipMemcpyAsync(lrp.data(), s->lrowptr, sizeof(int) * (n + 1), hipMemcpyDeviceToHost, st));
            LPCG_HIP(hipMemcpyAsync(lc.data(), s->lcol, sizeof(int) * (size_t)nnzl, hipMemcpyDeviceToHost, st));
            LPCG_HIP(hipMemcpyAsync(urp.data(), s->urowptr, sizeof(int) * (n + 1), hipMemcpyDeviceToHost, st));
            LPCG_HIP(hipMemcpyAsync(uc.data(), s->ucol, sizeof(int) * (size_t)nnzl, hipMemcpyDeviceToHost, st));
            LPCG_HIP(hipStreamSynchronize(st));
            int ws = 0, wp = 0;
            for (int i = p; i < n; ++i) ws = std::max(ws, lrp[i + 1] - lrp[i] - 1);  // L rows: diagonal last
            for (int j = 0; j < p; ++j) wp = std::max(wp, urp[j + 1] - urp[j] - 1);  // U rows: diagonal first
            if (ws >= 1 && ws <= kEllMaxW && wp <= kEllMaxW) {
                std::vector<int> scol((size_t)ws * nb), spos((size_t)ws * nb), sdpos(nb);
                std::vector<int> pcol((size_t)std::max(wp, 1) * p), ppos((size_t)std::max(wp, 1) * p), pdpos(p);
                for (int i = 0; i < nb; ++i) {
                    const int k0 = lrp[p + i], k1 = lrp[p + i + 1] - 1;
                    sdpos[i] = k1;
                    for (int t = 0; t < ws; ++t) {
                        const bool real = k0 + t < k1;
                        scol[(size_t)t * nb + i] = real ? lc[k0 + t] : 0;
                        spos[(size_t)t * nb + i] = real ? k0 + t : -1;
                    }
                }
                for (int j = 0; j < p; ++j) {
                    const int k0 = urp[j] + 1, k1 = urp[j + 1];
                    pdpos[j] = urp[j];
                    for (int t = 0; t < wp; ++t) {
                        const bool real = k0 + t < k1;
                        pcol[(size_t)t * p + j] = real ? uc[k0 + t] : p;
                        ppos[(size_t)t * p + j] = real ? k0 + t : -1;
                    }
                }
                const size_t ms = (size_t)ws * nb, mp = (size_t)std::max(wp, 1) * p;
                ALLOC(s->e2_scol, ms);
                ALLOC(s->e2_spos, ms);
                ALLOC(s->e2_sdpos, nb);
                ALLOC(s->e2_pcol, mp);
                ALLOC(s->e2_ppos, mp);
                ALLOC(s->e2_pdpos, p);
                ALLOC(s->e2_sval, ms);
                ALLOC(s->e2_sdiag, nb);
                ALLOC(s->e2_pval, mp);
                ALLOC(s->e2_pdiag, p);
                LPCG_HIP(hipMemcpyAsync(s->e2_scol, scol.data(), sizeof(int) * ms, hipMemcpyHostToDevice, st));
                LPCG_HIP(hipMemcpyAsync(s->e2_spos, spos.data(), sizeof(int) * ms, hipMemcpyHostToDevice, st));
                LPCG_HIP(hipMemcpyAsync(s->e2_sdpos, sdpos.data(), sizeof(int) * nb, hipMemcpyHostToDevice, st));
                LPCG_HIP(hipMemcpyAsync(s->e2_pcol, pcol.data(), sizeof(int) * mp, hipMemcpyHostToDevice, st));
                LPCG_HIP(hipMemcpyAsync(s->e2_ppos, ppos.data(), sizeof(int) * mp, hipMemcpyHostToDevice, st));
                LPCG_HIP(hipMemcpyAsync(s->e2_pdpos, pdpos.data(), sizeof(int) * p, hipMemcpyHostToDevice, st));
                LPCG_HIP(hipStreamSynchronize(st));
                s->e2_ws = ws;
                s->e2_wp = wp;
            }
        }
    }
    // SpMV lanes per row from the mean row length
    const double mean = (double)nnz / n;
    s->spmv_group = mean <= 4 ? 4 : mean <= 8 ? 8 : mean <= 16 ? 16 : mean <= 32 ? 32 : 64;
    s->spmv_blocks = std::max(1, std::min(kMaxSpmvBlocks, nblk(n, kVecThreads / s->spmv_group)));
    k_values<<<nblk(std::max(n, nnz), 256), 256, 0, st>>>(nnz, n, A->val, nullptr, s->dpos, s->val64,
                                                           s->val32, s->diag64);
    LPCG_LAUNCH_CHECK();
    if ((rc = ell_pack_a(s, st))) return rc;
    LPCG_HIP(hipStreamSynchronize(st));
#undef ALLOC
    return LPCG_OK;
}

// Multicolour analysis: natural analysis of A (validation, lower pattern,
// forward levels) in a scratch system, colours, the permutation, P A P^T,
// then the full analysis of P A P^T into s.
int analyze_color(const lpcg_csr *A, const int32_t *h_sys, int32_t nsys, lpcg_system *s, hipStream_t st) {
    const int n = A->n, nnz = A->nnz;
    lpcg_system *s0 = new (std::nothrow) lpcg_system();
    if (!s0) return LPCG_ENOMEM;
    std::vector<void *> tmp;
    auto cleanup = [&](int rc) {
        hipStreamSynchronize(st);
        for (void *p : tmp) hipFree(p);
        lpcg_destroy(s0);
        return rc;
    };
    auto talloc = [&](void **p, size_t bytes) -> int {
        hipError_t e = hipMalloc(p, bytes ? bytes : 4);
        if (e != hipSuccess) {
            set_error("hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
            return LPCG_ENOMEM;
        }
        tmp.push_back(*p);
        return LPCG_OK;
    };
    int rc = analyze_impl(A, h_sys, nsys, s0, st);
    if (rc) return cleanup(rc);
    int *color = nullptr, *ticket = nullptr, *keys = nullptr, *skeys = nullptr, *iota = nullptr, *d_max = nullptr;
    int *perm = nullptr, *iperm = nullptr, *len = nullptr, *nrp = nullptr, *ncol = nullptr, *psrc = nullptr;
    double *nval = nullptr;
    if ((rc = talloc((void **)&color, sizeof(int) * n)) || (rc = talloc((void **)&ticket, sizeof(int))) ||
        (rc = talloc((void **)&keys, sizeof(int) * n)) || (rc = talloc((void **)&skeys, sizeof(int) * n)) ||
        (rc = talloc((void **)&iota, sizeof(int) * n)) || (rc = talloc((void **)&d_max, sizeof(int))) ||
        (rc = talloc((void **)&len, sizeof(int) * (n + 1))) || (rc = talloc((void **)&nrp, sizeof(int) * (n + 1))) ||
        (rc = talloc((void **)&ncol, sizeof(int) * (size_t)nnz)) ||
        (rc = talloc((void **)&nval, sizeof(double) * (size_t)nnz)))
        return cleanup(rc);
    if (hipMemsetAsync(color, 0xff, sizeof(int) * n, st) != hipSuccess ||
        hipMemsetAsync(ticket, 0, sizeof(int), st) != hipSuccess)
        return cleanup(hip_fail(hipGetLastError(), "hipMemsetAsync", __FILE__, __LINE__));
    const int waves = std::min(nblk(n, kWave), 8192);
    k_colors<<<nblk(waves, 4), 256, 0, st>>>(n, s0->flev_rows, s0->lrowptr, s0->lcol, color, ticket);
    if (hipGetLastError() != hipSuccess) return cleanup(hip_fail(hipErrorLaunchFailure, "k_colors", __FILE__, __LINE__));
    size_t tb = 0;
    void *cub = nullptr;
    hipcub::DeviceReduce::Max(nullptr, tb, color, d_max, n, st);
    if ((rc = talloc(&cub, tb))) return cleanup(rc);
    hipcub::DeviceReduce::Max(cub, tb, color, d_max, n, st);
    int hmax = 0;
    hipMemcpyAsync(&hmax, d_max, sizeof(int), hipMemcpyDeviceToHost, st);
    if (hipStreamSynchronize(st) != hipSuccess)
        return cleanup(hip_fail(hipGetLastError(), "colouring", __FILE__, __LINE__));
    const int ncolors = hmax + 1;
    if ((long)nsys * ncolors >= (1L << 30)) {
        set_error("lpcg_analyze: %d systems x %d colours overflow the sort key", nsys, ncolors);
        return cleanup(LPCG_EINVAL);
    }
    int bits = 1;
    while ((1L << bits) < (long)nsys * ncolors) ++bits;
    k_color_keys<<<nblk(n, 256), 256, 0, st>>>(n, s0->row_sys, color, ncolors, keys, iota);
    // perm: rows sorted by (system, colour), stable (ascending rows within a key)
    if ((rc = dalloc(s, &s->perm, n)) || (rc = dalloc(s, &s->iperm, n))) return cleanup(rc);
    perm = s->perm;
    iperm = s->iperm;
    tb = 0;
    hipcub::DeviceRadixSort::SortPairs(nullptr, tb, keys, skeys, iota, perm, n, 0, bits, st);
    void *cub2 = nullptr;
    if ((rc = talloc(&cub2, tb))) return cleanup(rc);
    hipcub::DeviceRadixSort::SortPairs(cub2, tb, keys, skeys, iota, perm, n, 0, bits, st);
    hipMemsetAsync(len + n, 0, sizeof(int), st);
    k_perm_rows<<<nblk(n, 256), 256, 0, st>>>(n, perm, s0->rowptr, iperm, len);
    tb = 0;
    hipcub::DeviceScan::ExclusiveSum(nullptr, tb, len, nrp, n + 1, st);
    void *cub3 = nullptr;
    if ((rc = talloc(&cub3, tb))) return cleanup(rc);
    hipcub::DeviceScan::ExclusiveSum(cub3, tb, len, nrp, n + 1, st);
    if ((rc = dalloc(s, &s->psrc, nnz))) return cleanup(rc);
    psrc = s->psrc;
    k_perm_fill<<<nblk(n, 256), 256, 0, st>>>(n, perm, iperm, s0->rowptr, s0->colind, nrp, ncol, psrc);
    k_gather_vals<<<nblk(nnz, 256), 256, 0, st>>>(nnz, psrc, A->val, nval);
    if (hipGetLastError() != hipSuccess) return cleanup(hip_fail(hipErrorLaunchFailure, "permute", __FILE__, __LINE__));
    lpcg_csr B{n, nnz, nrp, ncol, nval};
    if ((rc = analyze_impl(&B, h_sys, nsys, s, st))) return cleanup(rc);
    if ((rc = dalloc(s, &s->bperm, n)) || (rc = dalloc(s, &s->xperm, n))) return cleanup(rc);
    s->ordering = LPCG_ORDER_COLOR;
    s->ncolors = ncolors;
    return cleanup(LPCG_OK);
}

}  // namespace
}  // namespace lpcg

using namespace lpcg;

extern "C" const char *lpcg_last_error(void) { return g_err; }
extern "C" const char *lpcg_version(void) { return "lpcg 0.1 (gfx950)"; }

namespace lpcg {
template <typename T>
static int permute_vec(const lpcg_system *s, const T *src, T *dst, bool to_int, hipStream_t st) {
    if (!s->perm) {
        if (src != dst) LPCG_HIP(hipMemcpyAsync(dst, src, sizeof(T) * s->n, hipMemcpyDeviceToDevice, st));
        return LPCG_OK;
    }
    if (to_int) k_vec_gather<T><<<nblk(s->n, 256), 256, 0, st>>>(s->n, s->perm, src, dst);
    else k_vec_scatter<T><<<nblk(s->n, 256), 256, 0, st>>>(s->n, s->perm, src, dst);
    LPCG_LAUNCH_CHECK();
    return LPCG_OK;
}
int to_internal_f64(const lpcg_system *s, const double *src, double *dst, hipStream_t st) {
    return permute_vec(s, src, dst, true, st);
}
int to_internal_f64_2(const lpcg_system *s, const double *s0, double *d0, const double *s1, double *d1,
                      hipStream_t st) {
    if (!s->perm) {
        int rc = permute_vec(s, s0, d0, true, st);
        return rc ? rc : permute_vec(s, s1, d1, true, st);
    }
    k_vec_gather2<<<nblk(s->n, 256), 256, 0, st>>>(s->n, s->perm, s0, d0, s1, d1);
    LPCG_LAUNCH_CHECK();
    return LPCG_OK;
}
int from_internal_f64(const lpcg_system *s, const double *src, double *dst, hipStream_t st) {
    return permute_vec(s, src, dst, false, st);
}
int to_internal_f32(const lpcg_system *s, const float *src, float *dst, hipStream_t st) {
    return permute_vec(s, src, dst, true, st);
}
int from_internal_f32(const lpcg_system *s, const float *src, float *dst, hipStream_t st) {
    return permute_vec(s, src, dst, false, st);
}

int ell_pack_a(const lpcg_system *s, hipStream_t st) {
    if (s->ea_w == 0) return LPCG_OK;
    const long m = (long)s->ea_w * s->n;
    k_ell_pack<<<nblk(m, 256), 256, 0, st>>>(m, s->ea_pos, s->val32, s->ea_val);
    LPCG_LAUNCH_CHECK();
    return LPCG_OK;
}
}  // namespace lpcg

extern "C" int lpcg_analyze(const lpcg_csr *A, const int32_t *sys_rowptr, int32_t nsys, int32_t ordering,
                            lpcg_system **out, hipStream_t stream) {
    set_error("");
    if (!A || !out || A->n <= 0 || A->nnz < A->n || !A->rowptr || !A->colind || !A->val) {
        set_error("lpcg_analyze: invalid arguments");
        return LPCG_EINVAL;
    }
    std::vector<int> one = {0, A->n};
    const int32_t *h_sys = one.data();
    if (sys_rowptr && nsys > 1) {
        h_sys = sys_rowptr;
        if (sys_rowptr[0] != 0 || sys_rowptr[nsys] != A->n) {
            set_error("lpcg_analyze: sys_rowptr must start at 0 and end at n");
            return LPCG_EINVAL;
        }
        for (int i = 0; i < nsys; ++i)
            if (sys_rowptr[i + 1] <= sys_rowptr[i]) {
                set_error("lpcg_analyze: empty or decreasing system %d", i);
                return LPCG_EINVAL;
            }
    } else {
        nsys = 1;
    }
    if (ordering != LPCG_ORDER_NATURAL && ordering != LPCG_ORDER_COLOR) {
        set_error("lpcg_analyze: unknown ordering %d", ordering);
        return LPCG_EINVAL;
    }
    if (ordering == LPCG_ORDER_COLOR && A->n > LPCG_COLOR_MAX_ROWS) {
        set_error("lpcg_analyze: the colour ordering takes at most %d rows (got %d)", LPCG_COLOR_MAX_ROWS, A->n);
        return LPCG_EINVAL;
    }
    lpcg_system *s = new (std::nothrow) lpcg_system();
    if (!s) return LPCG_ENOMEM;
    int rc = ordering == LPCG_ORDER_COLOR ? analyze_color(A, h_sys, nsys, s, stream)
                                          : analyze_impl(A, h_sys, nsys, s, stream);
    if (rc != LPCG_OK) {
        hipStreamSynchronize(stream);
        lpcg_destroy(s);
        return rc;
    }
    *out = s;
    return LPCG_OK;
}

extern "C" int lpcg_update_values(lpcg_system *s, const double *val, hipStream_t stream) {
    if (!s || !val) {
        set_error("lpcg_update_values: invalid arguments");
        return LPCG_EINVAL;
    }
    k_values<<<nblk(std::max(s->n, s->nnz), 256), 256, 0, stream>>>(s->nnz, s->n, val, s->psrc, s->dpos,
                                                                       s->val64, s->val32, s->diag64);
    LPCG_LAUNCH_CHECK();
    return ell_pack_a(s, stream);
}

extern "C" int lpcg_get_info(const lpcg_system *s, lpcg_info *info) {
    if (!s || !info) {
        set_error("lpcg_get_info: invalid arguments");
        return LPCG_EINVAL;
    }
    info->n = s->n;
    info->nnz = s->nnz;
    info->nnz_l = s->nnz_l;
    info->nlev_fwd = s->nlev_f;
    info->nlev_bwd = s->nlev_b;
    info->max_width_fwd = s->max_w_f;
    info->max_width_bwd = s->max_w_b;
    info->nsys = s->nsys;
    info->ordering = s->ordering;
    info->ncolors = s->ncolors;
    return LPCG_OK;
}

extern "C" int lpcg_export_pattern(const lpcg_system *s, int32_t *lrowptr, int32_t *lcol,
                                   int32_t *lsrc, int32_t *urowptr, int32_t *ucol, int32_t *u2l,
                                   int32_t *rev, int32_t *flevel, int32_t *flev_ptr,
                                   int32_t *flev_rows, int32_t *blevel, int32_t *blev_ptr,
                                   int32_t *blev_rows, hipStream_t st) {
    if (!s) {
        set_error("lpcg_export_pattern: null system");
        return LPCG_EINVAL;
    }
    auto cp = [&](int32_t *dst, const int *src, size_t count) -> int {
        if (dst) LPCG_HIP(hipMemcpyAsync(dst, src, count * sizeof(int), hipMemcpyDeviceToDevice, st));
        return LPCG_OK;
    };
    int rc = 0;
    rc |= cp(lrowptr, s->lrowptr, s->n + 1);
    rc |= cp(lcol, s->lcol, s->nnz_l);
    rc |= cp(lsrc, s->lsrc, s->nnz_l);
    rc |= cp(urowptr, s->urowptr, s->n + 1);
    rc |= cp(ucol, s->ucol, s->nnz_l);
    rc |= cp(u2l, s->u2l, s->nnz_l);
    rc |= cp(rev, s->rev, s->nnz);
    rc |= cp(flevel, s->flevel, s->n);
    rc |= cp(flev_ptr, s->flev_ptr, s->nlev_f + 1);
    rc |= cp(flev_rows, s->flev_rows, s->n);
    rc |= cp(blevel, s->blevel, s->n);
    rc |= cp(blev_ptr, s->blev_ptr, s->nlev_b + 1);
    rc |= cp(blev_rows, s->blev_rows, s->n);
    return rc ? LPCG_EHIP : LPCG_OK;
}

extern "C" int lpcg_export_perm(const lpcg_system *s, int32_t *perm, hipStream_t st) {
    if (!s || !perm) {
        set_error("lpcg_export_perm: invalid arguments");
        return LPCG_EINVAL;
    }
    if (s->perm) {
        LPCG_HIP(hipMemcpyAsync(perm, s->perm, sizeof(int) * s->n, hipMemcpyDeviceToDevice, st));
    } else {
        k_iota_fill<<<nblk(s->n, 256), 256, 0, st>>>(s->n, perm, nullptr, nullptr);
        LPCG_LAUNCH_CHECK();
    }
    return LPCG_OK;
}

extern "C" void lpcg_destroy(lpcg_system *s) {
    if (!s) return;
    drop_graphs(s);
    if (s->cap_stream) hipStreamDestroy(s->cap_stream);
    for (int d = 0; d < 2; ++d) blk_free(s, d);
    for (void *p : s->allocs) hipFree(p);
    if (s->h_ctrl) hipHostFree(s->h_ctrl);
    if (s->h_scal) hipHostFree(s->h_scal);
    delete s;
}
