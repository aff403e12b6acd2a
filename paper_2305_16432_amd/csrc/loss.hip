// Data loss of the Method section (equation loss_Ab) and Adam.
//
//   loss_s = || L L^T x - b ||^2 / rms(b)^2   over the rows of system s
//   d loss / d L_ij = 2 (r_i u_j + x_i w_j) / rms(b)^2,
//   u = L^T x, r = L u - b, w = L^T r.
// Two triangular MAT-VECS (not solves) per product, FP64 accumulation, row-wise
// gathers (L^T through the U = L^T pattern and the U -> L map), so every sum
// has a fixed order.
//
// Frobenius loss of equation loss_A (the ablation of the loss-function
// section): loss_s = ||L L^T - A||_F^2 / s^2 over every entry, s = mean(diag A)
// of system s, gradient 4 (L L^T - A) L / s^2 on L's entries.  E = L L^T - A is
// formed explicitly on the pattern pattern(A) u pattern(L L^T), built once
// per system by a row-wise symbolic product (row a of L L^T: the rows of U =
// L^T reached through the columns of L's row a).
#include <algorithm>
#include <vector>

#include "device_util.h"
#include "lpcg_internal.h"

namespace lpcg {
namespace {

int nblk(long n, int t) { return (int)((n + t - 1) / t); }

// y_j = sum_{i >= j} L_ij x_i  (row j of U = L^T)
__global__ void k_ltmul(int n, const int *__restrict__ urp, const int *__restrict__ ucol,
                        const int *__restrict__ u2l, const float *__restrict__ lval,
                        const double *__restrict__ x, double *__restrict__ y) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double s = 0;
    for (int q = urp[j]; q < urp[j + 1]; ++q) s += (double)lval[u2l[q]] * x[ucol[q]];
    y[j] = s;
}

// r_i = sum_j L_ij u_j - b_i
__global__ void k_lmul_res(int n, const int *__restrict__ lrp, const int *__restrict__ lcol,
                           const float *__restrict__ lval, const double *__restrict__ u,
                           const double *__restrict__ b, double *__restrict__ r) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0;
    for (int p = lrp[i]; p < lrp[i + 1]; ++p) s += (double)lval[p] * u[lcol[p]];
    r[i] = s - b[i];
}

// per system: rms(b)^2 and loss = sum r^2 / rms^2 (one block per system)
__global__ void k_sys_loss(int nsys, const int *__restrict__ sys_rowptr, const double *__restrict__ b,
                           const double *__restrict__ r, double *__restrict__ rms2,
                           double *__restrict__ loss) {
    __shared__ double lds[256 / kWave];
    const int sy = blockIdx.x;
    const int r0 = sys_rowptr[sy], r1 = sys_rowptr[sy + 1];
    double sb = 0, sr = 0;
    for (int i = r0 + threadIdx.x; i < r1; i += 256) {
        sb += b[i] * b[i];
        sr += r[i] * r[i];
    }
    sb = block_sum<256>(sb, lds);
    sr = block_sum<256>(sr, lds);
    if (threadIdx.x == 0) {
        double m = sb / (double)(r1 - r0);
        if (!(m > 0)) m = 1.0;
        rms2[sy] = m;
        loss[sy] = sr / m;
    }
}

__global__ void k_llt_grad(int nnz_l, const int *__restrict__ lsrc, const int *__restrict__ erow,
                           const int *__restrict__ lcol, const int *__restrict__ row_sys,
                           const double *__restrict__ rms2, const double *__restrict__ r,
                           const double *__restrict__ u, const double *__restrict__ x,
                           const double *__restrict__ w, float *__restrict__ dl) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnz_l) return;
    const int i = erow[lsrc[p]], j = lcol[p];
    dl[p] = (float)(2.0 * (r[i] * u[j] + x[i] * w[j]) / rms2[row_sys[i]]);
}

__global__ void k_adam(long count, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

constexpr int kFrobRow = 256;  // most entries a row of E may have

// Candidate columns of row a of E (A's row, and U rows c for c in L's row a),
// sorted and unique, into out[] (at most kFrobRow); returns the count, or -1
// if the row has more entries than fit.
__device__ int e_row_cols(int a, const int *__restrict__ rp, const int *__restrict__ ci,
                          const int *__restrict__ lrp, const int *__restrict__ lcol,
                          const int *__restrict__ urp, const int *__restrict__ ucol, int *out) {
    int m = 0;
    auto add = [&](int c) -> bool {
        int q = m;
        while (q > 0 && out[q - 1] > c) --q;
        if (q > 0 && out[q - 1] == c) return true;
        if (m == kFrobRow) return false;
        for (int t = m; t > q; --t) out[t] = out[t - 1];
        out[q] = c;
        ++m;
        return true;
    };
    for (int k = rp[a]; k < rp[a + 1]; ++k)
        if (!add(ci[k])) return -1;
    for (int p = lrp[a]; p < lrp[a + 1]; ++p) {
        const int c = lcol[p];
        for (int q = urp[c]; q < urp[c + 1]; ++q)
            if (!add(ucol[q])) return -1;
    }
    return m;
}

__global__ void k_e_count(int n, const int *__restrict__ rp, const int *__restrict__ ci, const int *__restrict__ lrp,
                          const int *__restrict__ lcol, const int *__restrict__ urp, const int *__restrict__ ucol,
                          int *__restrict__ cnt, int *__restrict__ err) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    int buf[kFrobRow];
    const int m = e_row_cols(a, rp, ci, lrp, lcol, urp, ucol, buf);
    if (m < 0) atomicOr(err, 1);
    cnt[a] = m < 0 ? 0 : m;
}

__global__ void k_e_fill(int n, const int *__restrict__ rp, const int *__restrict__ ci, const int *__restrict__ lrp,
                         const int *__restrict__ lcol, const int *__restrict__ urp, const int *__restrict__ ucol,
                         const int *__restrict__ erp, int *__restrict__ ecol) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    int buf[kFrobRow];
    const int m = e_row_cols(a, rp, ci, lrp, lcol, urp, ucol, buf);
    for (int t = 0; t < m; ++t) ecol[erp[a] + t] = buf[t];
}

__device__ __forceinline__ int find_col(const int *__restrict__ cols, int lo, int hi, int c) {
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cols[mid] < c) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Row a of E = L L^T - A (FP64): -A_ab, then + L_ac L_bc for c in L's row a
// (ascending) and b in U's row c (ascending); erowsq[a] = sum_b E_ab^2.
__global__ void k_e_vals(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                         const double *__restrict__ aval, const int *__restrict__ lrp,
                         const int *__restrict__ lcol, const int *__restrict__ urp, const int *__restrict__ ucol,
                         const int *__restrict__ u2l, const float *__restrict__ lval,
                         const int *__restrict__ erp, const int *__restrict__ ecol, double *__restrict__ ev,
                         double *__restrict__ erowsq) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    const int e0 = erp[a], e1 = erp[a + 1];
    for (int e = e0; e < e1; ++e) ev[e] = 0.0;
    for (int k = rp[a]; k < rp[a + 1]; ++k) ev[find_col(ecol, e0, e1, ci[k])] -= aval[k];
    for (int p = lrp[a]; p < lrp[a + 1]; ++p) {
        const int c = lcol[p];
        const double lac = lval[p];
        for (int q = urp[c]; q < urp[c + 1]; ++q)
            ev[find_col(ecol, e0, e1, ucol[q])] += lac * (double)lval[u2l[q]];
    }
    double sq = 0;
    for (int e = e0; e < e1; ++e) sq += ev[e] * ev[e];
    erowsq[a] = sq;
}

// per system: s^2 = mean(diag A)^2 and loss = sum of row sums of E^2 / s^2
__global__ void k_frob_sys(int nsys, const int *__restrict__ sys_rowptr, const double *__restrict__ diag,
                           const double *__restrict__ erowsq, double *__restrict__ s2, double *__restrict__ loss) {
    __shared__ double lds[256 / kWave];
    const int sy = blockIdx.x;
    const int r0 = sys_rowptr[sy], r1 = sys_rowptr[sy + 1];
    double sd = 0, se = 0;
    for (int i = r0 + threadIdx.x; i < r1; i += 256) {
        sd += diag[i];
        se += erowsq[i];
    }
    sd = block_sum<256>(sd, lds);
    se = block_sum<256>(se, lds);
    if (threadIdx.x == 0) {
        const double sm = sd / (double)(r1 - r0);
        const double q = sm * sm > 0 ? sm * sm : 1.0;
        s2[sy] = q;
        loss[sy] = se / q;
    }
}

// d loss / d L_ij = 4 sum_b E_ib L_bj / s^2 over row i of E (L_bj: column j
// in L's row b, b >= j)
__global__ void k_frob_grad(int nnz_l, const int *__restrict__ lsrc, const int *__restrict__ erow,
                            const int *__restrict__ lrp, const int *__restrict__ lcol,
                            const float *__restrict__ lval, const int *__restrict__ erp,
                            const int *__restrict__ ecol, const double *__restrict__ ev,
                            const int *__restrict__ row_sys, const double *__restrict__ s2,
                            float *__restrict__ g) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnz_l) return;
    const int i = erow[lsrc[p]], j = lcol[p];
    double acc = 0;
    for (int e = erp[i]; e < erp[i + 1]; ++e) {
        const int b = ecol[e];
        if (b < j) continue;
        const int q = find_col(lcol, lrp[b], lrp[b + 1], j);
        if (q < lrp[b + 1] && lcol[q] == j) acc += ev[e] * (double)lval[q];
    }
    g[p] = (float)(4.0 * acc / s2[row_sys[i]]);
}

}  // namespace
}  // namespace lpcg

using namespace lpcg;

extern "C" int lpcg_llt_loss(const lpcg_system *s, const float *l_val, const double *x, const double *b,
                             double *loss, float *dl_val, hipStream_t st) {
    if (!s || !l_val || !x || !b || !loss) {
        set_error("lpcg_llt_loss: invalid arguments");
        return LPCG_EINVAL;
    }
    const int n = s->n;
    double *u = s->t64a, *r = s->t64b, *w = s->t64c, *rms2 = s->sys_tmp;
    if (s->perm) {  // x and b arrive in the caller's numbering
        int rc;
        if ((rc = to_internal_f64(s, x, s->xperm, st)) || (rc = to_internal_f64(s, b, s->bperm, st))) return rc;
        x = s->xperm;
        b = s->bperm;
    }
    k_ltmul<<<nblk(n, 256), 256, 0, st>>>(n, s->urowptr, s->ucol, s->u2l, l_val, x, u);
    k_lmul_res<<<nblk(n, 256), 256, 0, st>>>(n, s->lrowptr, s->lcol, l_val, u, b, r);
    k_sys_loss<<<s->nsys, 256, 0, st>>>(s->nsys, s->sys_rowptr, b, r, rms2, loss);
    if (dl_val) {
        k_ltmul<<<nblk(n, 256), 256, 0, st>>>(n, s->urowptr, s->ucol, s->u2l, l_val, r, w);
        k_llt_grad<<<nblk(s->nnz_l, 256), 256, 0, st>>>(s->nnz_l, s->lsrc, s->erow, s->lcol, s->row_sys, rms2,
                                                         r, u, x, w, dl_val);
    }
    LPCG_LAUNCH_CHECK();
    return LPCG_OK;
}

extern "C" int lpcg_adam_step(float *params, const float *grads, float *m, float *v, int64_t count, float lr,
                              float beta1, float beta2, float eps, int32_t step, hipStream_t st) {
    if (!params || !grads || !m || !v || count <= 0 || step < 1) {
        set_error("lpcg_adam_step: invalid arguments");
        return LPCG_EINVAL;
    }
    const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
    k_adam<<<(int)((count + 255) / 256), 256, 0, st>>>((long)count, params, grads, m, v, lr, beta1, beta2, eps,
                                                        c1, c2);
    LPCG_LAUNCH_CHECK();
    return LPCG_OK;
}

extern "C" int lpcg_frob_loss(lpcg_system *s, const float *l_val, double *loss, float *dl_val, hipStream_t st) {
    if (!s || !l_val || !loss) {
        set_error("lpcg_frob_loss: invalid arguments");
        return LPCG_EINVAL;
    }
    const int n = s->n;
    if (!s->erp) {  // symbolic product, once per system
        int *cnt = nullptr, *err = nullptr;
        LPCG_HIP(hipMalloc(&cnt, sizeof(int) * (n + 1)));
        LPCG_HIP(hipMalloc(&err, sizeof(int)));
        std::vector<void *> tmp = {cnt, err};
        auto fail = [&](int rc) {
            hipStreamSynchronize(st);
            for (void *p : tmp) hipFree(p);
            return rc;
        };
        if (hipMemsetAsync(err, 0, sizeof(int), st) != hipSuccess || hipMemsetAsync(cnt + n, 0, sizeof(int), st) != hipSuccess)
            return fail(hip_fail(hipGetLastError(), "hipMemsetAsync", __FILE__, __LINE__));
        k_e_count<<<nblk(n, 128), 128, 0, st>>>(n, s->rowptr, s->colind, s->lrowptr, s->lcol, s->urowptr, s->ucol, cnt,
                                                 err);
        int herr = 0;
        std::vector<int> hcnt(n + 1);
        if (hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(hcnt.data(), cnt, sizeof(int) * (n + 1), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return fail(hip_fail(hipGetLastError(), "frobenius pattern", __FILE__, __LINE__));
        if (herr) {
            set_error("lpcg_frob_loss: a row of L L^T has more than %d entries", kFrobRow);
            return fail(LPCG_EINVAL);
        }
        std::vector<int> hrp(n + 1, 0);
        for (int i = 0; i < n; ++i) hrp[i + 1] = hrp[i] + hcnt[i];
        s->nnz_e = hrp[n];
        void *p1 = nullptr, *p2 = nullptr, *p3 = nullptr, *p4 = nullptr;
        if (hipMalloc(&p1, sizeof(int) * (n + 1)) != hipSuccess || hipMalloc(&p2, sizeof(int) * (size_t)s->nnz_e) != hipSuccess ||
            hipMalloc(&p3, sizeof(double) * (size_t)s->nnz_e) != hipSuccess || hipMalloc(&p4, sizeof(double) * n) != hipSuccess) {
            for (void *p : {p1, p2, p3, p4})
                if (p) hipFree(p);
            set_error("lpcg_frob_loss: allocation of the L L^T pattern failed");
            return fail(LPCG_ENOMEM);
        }
        s->allocs.push_back(p1);
        s->allocs.push_back(p2);
        s->allocs.push_back(p3);
        s->allocs.push_back(p4);
        s->erp = (int *)p1;
        s->ecol = (int *)p2;
        s->eval = (double *)p3;
        s->erowsq = (double *)p4;
        if (hipMemcpyAsync(s->erp, hrp.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice, st) != hipSuccess)
            return fail(hip_fail(hipGetLastError(), "hipMemcpyAsync", __FILE__, __LINE__));
        k_e_fill<<<nblk(n, 128), 128, 0, st>>>(n, s->rowptr, s->colind, s->lrowptr, s->lcol, s->urowptr, s->ucol,
                                                s->erp, s->ecol);
        if (hipStreamSynchronize(st) != hipSuccess)
            return fail(hip_fail(hipGetLastError(), "frobenius pattern", __FILE__, __LINE__));
        fail(LPCG_OK);
    }
    k_e_vals<<<nblk(n, 128), 128, 0, st>>>(n, s->rowptr, s->colind, s->val64, s->lrowptr, s->lcol, s->urowptr,
                                            s->ucol, s->u2l, l_val, s->erp, s->ecol, s->eval, s->erowsq);
    k_frob_sys<<<s->nsys, 256, 0, st>>>(s->nsys, s->sys_rowptr, s->diag64, s->erowsq, s->sys_tmp, loss);
    if (dl_val)
        k_frob_grad<<<nblk(s->nnz_l, 256), 256, 0, st>>>(s->nnz_l, s->lsrc, s->erow, s->lrowptr, s->lcol, l_val,
                                                          s->erp, s->ecol, s->eval, s->row_sys, s->sys_tmp, dl_val);
    LPCG_LAUNCH_CHECK();
    return LPCG_OK;
}
