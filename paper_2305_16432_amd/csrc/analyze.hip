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

__global__ void k_iota_fill(int n, int *iota, int *lev_f, int *lev_b) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) { iota[i] = i; lev_f[i] = -1; lev_b[i] = -1; }
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

__global__ void k_values(int nnz, int n, const double *__restrict__ v64, const int *__restrict__ dpos,
                         double *__restrict__ val64, float *__restrict__ val32,
                         double *__restrict__ diag64) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nnz) {
        double v = v64[k];
        val64[k] = v;
        val32[k] = (float)v;
    }
    if (k < n) diag64[k] = v64[dpos[k]];
}

int nblk(long n, int t) { return (int)((n + t - 1) / t); }

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
    // values and solver work space
    ALLOC(s->val64, nnz);
    ALLOC(s->val32, nnz);
    ALLOC(s->diag64, n);
    ALLOC(s->r, n);
    ALLOC(s->p, n);
    ALLOC(s->w, n);
    ALLOC(s->z, n);
    ALLOC(s->y, n);
    ALLOC(s->dinv, n);
    ALLOC(s->t64a, n);
    ALLOC(s->t64b, n);
    ALLOC(s->t64c, n);
    ALLOC(s->sys_tmp, 2 * (size_t)nsys);
    s->vec_blocks = std::max(1, std::min(kMaxVecBlocks, nblk(n, kVecThreads * 4)));
    const int chunks = nblk(n, kWave);
    s->npart = std::max(std::max(kMaxVecBlocks, kMaxSpmvBlocks), chunks);
    ALLOC(s->part, 4 * (size_t)s->npart);
    ALLOC(s->scal, S_NSCAL);
    ALLOC(s->ctrl, C_NCTRL);
    LPCG_HIP(hipHostMalloc((void **)&s->h_ctrl, sizeof(int) * C_NCTRL, hipHostMallocDefault));
    LPCG_HIP(hipHostMalloc((void **)&s->h_scal, sizeof(double) * S_NSCAL, hipHostMallocDefault));
    // SpMV lanes per row from the mean row length
    const double mean = (double)nnz / n;
    s->spmv_group = mean <= 4 ? 4 : mean <= 8 ? 8 : mean <= 16 ? 16 : mean <= 32 ? 32 : 64;
    s->spmv_blocks = std::max(1, std::min(kMaxSpmvBlocks, nblk(n, kVecThreads / s->spmv_group)));
    k_values<<<nblk(std::max(n, nnz), 256), 256, 0, st>>>(nnz, n, A->val, s->dpos, s->val64, s->val32,
                                                           s->diag64);
    LPCG_LAUNCH_CHECK();
    LPCG_HIP(hipStreamSynchronize(st));
#undef ALLOC
    return LPCG_OK;
}

}  // namespace
}  // namespace lpcg

using namespace lpcg;

extern "C" const char *lpcg_last_error(void) { return g_err; }
extern "C" const char *lpcg_version(void) { return "lpcg 0.1 (gfx950)"; }

extern "C" int lpcg_analyze(const lpcg_csr *A, const int32_t *sys_rowptr, int32_t nsys,
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
    lpcg_system *s = new (std::nothrow) lpcg_system();
    if (!s) return LPCG_ENOMEM;
    int rc = analyze_impl(A, h_sys, nsys, s, stream);
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
    k_values<<<nblk(std::max(s->n, s->nnz), 256), 256, 0, stream>>>(s->nnz, s->n, val, s->dpos,
                                                                       s->val64, s->val32, s->diag64);
    LPCG_LAUNCH_CHECK();
    return LPCG_OK;
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

extern "C" void lpcg_destroy(lpcg_system *s) {
    if (!s) return;
    if (s->graph_exec) hipGraphExecDestroy(s->graph_exec);
    if (s->cap_stream) hipStreamDestroy(s->cap_stream);
    for (void *p : s->allocs) hipFree(p);
    if (s->h_ctrl) hipHostFree(s->h_ctrl);
    if (s->h_scal) hipHostFree(s->h_scal);
    delete s;
}
