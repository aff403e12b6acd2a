// Data loss of the Method section (equation loss_Ab) and Adam.
//
//   loss_s = || L L^T x - b ||^2 / rms(b)^2   over the rows of system s
//   d loss / d L_ij = 2 (r_i u_j + x_i w_j) / rms(b)^2,
//   u = L^T x, r = L u - b, w = L^T r.
// Two triangular MAT-VECS (not solves) per product, FP64 accumulation, row-wise
// gathers (L^T through the U = L^T pattern and the U -> L map), so every sum
// has a fixed order.
#include <algorithm>

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
