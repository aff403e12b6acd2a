// PCG (Appendix algorithm "PCG") on the GPU.
//
//   r0 = b - A x0;  z0 = P^-1 r0;  then for k = 1, 2, ...:
//   p_k = z_{k-1} + beta p_{k-1} (p_1 = z_0);  w = A p_k;  alpha = r.z / p.w;
//   x += alpha p;  r -= alpha w;  stop if ||r|| <= tol ||b||;  z = P^-1 r;
//   beta = r.z(new) / r.z(old).
//
// Precision: A's values, r, p, w, z in FP32; x, b and every dot product /
// norm in FP64; the final true residual ||b - A x|| in FP64 (FP64 values).
//
// Control: the iteration state lives on the device (ctrl words, FP64
// scalars).  Each kernel returns at once when the done flag is set, so the
// host enqueues chunks of iterations (optionally as a captured hipGraph) and
// reads the flag only between chunks.  Every dot product is reduced in a
// fixed order: every block publishes its partial (an agent-scope atomic store
// into a slot preset to a sentinel, so the value is its own ready flag), and
// the block of highest index waits for the slots, sums them in index order and
// computes the scalar the next kernel needs: runs are bit-reproducible, no
// launch is spent on a reduction, and neither an arrival counter (device-scope
// atomics on one address serialise) nor a cache-flushing fence is needed.
// The product's p.w partials are plain stores instead, summed in the same
// order by every block of the next launch (which needs alpha first), so the
// product ends without a reducer.
//
// Kernels of one iteration (it = products A p so far):
//   LLT:    fwd   y = L^-1 r                       (kern_sptrsv.h, either mode)
//           bwd   z = L^-T y, r.z partials; reducer block: beta
//   all:    spmv  p = z + beta p_prev (p double-buffered by the parity of
//                 it), w = A p computed from z and p_prev on the fly, p.w
//                 partials
//           xr    alpha and the breakdown test from the p.w partials (every
//                 block), x += alpha p, r -= alpha w, ||r||^2 (Jacobi/none:
//                 r.z) partials, Jacobi's z = dinv r, presets of the
//                 dependency-driven substitution; reducer block: it += 1,
//                 convergence test (Jacobi/none: beta)
// Jacobi writes z = dinv r where it updates r and no preconditioning reads r
// as z, so an iteration is two launches; LLT adds the substitutions (two
// launches in all for the two-level orderings, see k_llt2_*; the ELL form of
// that pair also performs the update: three launches, see k_llt2e_*).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "device_util.h"
#include "kern_spmv.h"
#include "kern_sptrsv.h"
#include "lpcg_internal.h"

namespace lpcg {

int spmv32(const lpcg_system *s, const float *x, float *y, hipStream_t st);
int lo_prepare(const lpcg_system *s, int transpose, const float *lval, const float *utval, hipStream_t st);

namespace {

constexpr int VT = kVecThreads;

struct Args {
    int n, np_vec, np_rz, maxit, kind;
    // the product kernel stores its p.w partials to part_pw (plain stores,
    // np_pw slots); the next launch (k_xr, or the red-black pair) reduces
    // them in every block and takes alpha
    int np_pw;
    int backoff_f, backoff_b, stride_f, stride_b, reset_y, reset_z;
    const int *rp, *ci;
    const float *v32;
    const double *v64;
    const int *lrp, *lci, *urp, *uci, *forder, *border;
    int nlev_f, nlev_b;
    const int *flp, *blp;                             // device level pointers
    const int *lo_ptr_f, *lo_col_f, *lo_ptr_b, *lo_col_b;  // level-ordered packed patterns
    const float *lo_val_f, *lo_diag_f, *lo_val_b, *lo_diag_b;
    BlkSched blk_f, blk_b;                            // blocked-mode schedules
    const float *lval, *utval, *dinv;
    const double *b;
    double *x;
    float *r, *p0, *p1, *w;
    uint32_t *y, *z;
    double *part_rr, *part_rz, *part_pw, *part_bb;  // plain partials (setup, true residual)
    double *sp_rz, *sp_pw, *sp_rr, *sp_rz2;          // published partials (reducer-block sums)
    double *scal, *hist, *coef;
    int *ctrl;
    double tol2;
};

// The done flag is only raised by an earlier launch or by the reducer block
// after every other block of the launch has published (and so has read the
// flag), so every block of a launch sees the same value; one thread
// reads it so that the block branches uniformly around its barriers.
__device__ __forceinline__ bool is_done(const Args &a) {
    __shared__ int flag;
    if (threadIdx.x == 0) flag = a.ctrl[C_DONE];
    __syncthreads();
    return flag != 0;
}

// The same flag read by every wave, with no block barrier, so that a kernel
// can issue it together with its first data loads (which are in bounds and
// harmless when the flag is set).  Every wave of a launch reads the same
// value: the flag is raised only by an earlier launch or by a reducer block
// after every other block has published its partial (each block reads the
// flag before it publishes) and after the reducer's own block barriers.
// readfirstlane keeps the branch on it scalar.
__device__ __forceinline__ bool done_now(int flag) { return __builtin_amdgcn_readfirstlane(flag) != 0; }

// Control words and FP64 scalars read at a kernel's start through the vector
// memory path: a scalar load would share its wait counter with the kernel's
// argument loads, so the first data loads (which need the arguments) would
// wait for it too.
__device__ __forceinline__ int ld_ctrl(const int *p) { return ld_agent_i(p); }

// Marks a loaded word as a per-lane value.  The compiler otherwise reads a
// load from a uniform address into a scalar register at once, which waits for
// that load before the kernel's other loads are issued; called after those.
__device__ __forceinline__ int lane_value(int v) {
    asm volatile("" : "+v"(v));
    return v;
}
__device__ __forceinline__ double ld_scal(const double *p) {
    return __longlong_as_double((long long)ld_agent_u64(reinterpret_cast<const uint64_t *>(p)));
}

// The block of highest index reduces: after publishing its own partial it
// sums every published slot (reduce_published waits for each to become
// visible).  Only that block waits, and it waits on blocks that never wait on
// it, so the wait always ends; no counter or fence is needed.
__device__ __forceinline__ bool is_reducer() { return blockIdx.x == gridDim.x - 1; }

// Convergence bookkeeping after ||r||^2 (thread 0 of the deciding block).
__device__ __forceinline__ void record_residual(const Args &a, double rr, int it) {
    const double bb = a.scal[S_BB];
    const bool conv = !(rr > a.tol2 * bb);
    const bool cap = !conv && it >= a.maxit;
    const bool bad = !isfinite(rr);
    if (a.hist && it <= a.maxit) a.hist[it] = sqrt(rr / bb);
    a.scal[S_RR] = rr;
    a.ctrl[C_RES] = __float_as_int((float)(rr / bb));
    a.ctrl[C_RES_IT] = it;
    if (conv || cap || bad) {
        a.ctrl[C_DONE] = 1;
        a.ctrl[C_STATUS] = conv ? LPCG_OK : bad ? LPCG_EBREAKDOWN : LPCG_ENOTCONV;
        a.ctrl[C_ITERS] = it;
    }
}

// (A x)_i in FP64 from the FP64 values, summed in entry order.  The row's
// entries are loaded eight at a time (indices clamped into the row) and their
// inputs gathered together, so a row of up to eight entries costs three
// dependent round trips instead of two per entry.
__device__ __forceinline__ double row_ax64(const Args &a, int i) {
    const int beg = a.rp[i], end = a.rp[i + 1];
    double s = 0;
    for (int k0 = beg; k0 < end; k0 += 8) {
        int c[8];
        double v[8], xv[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int k = min(k0 + t, end - 1);
            c[t] = a.ci[k];
            v[t] = a.v64[k];
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) xv[t] = a.x[c[t]];
#pragma unroll
        for (int t = 0; t < 8; ++t)
            if (k0 + t < end) s += v[t] * xv[t];
    }
    return s;
}

// r = b - A x (FP64 product, FP32 r), ||b||^2, ||r||^2 and (Jacobi/none) r.z
// partials; presets y, z for dependency-driven substitutions.
template <int KIND>
__global__ void __launch_bounds__(VT) k_setup(Args a) {
    __shared__ double lds[VT / kWave];
    double bb = 0, rr = 0, rz = 0;
    for (int i = blockIdx.x * VT + threadIdx.x; i < a.n; i += gridDim.x * VT) {
        const double s = row_ax64(a, i);
        const double bi = a.b[i];
        const float ri = (float)(bi - s);
        a.r[i] = ri;
        bb += bi * bi;
        rr += (double)ri * ri;
        if (KIND == LPCG_PC_JACOBI) {
            rz += (double)ri * ri * a.dinv[i];
            a.z[i] = __float_as_uint(a.dinv[i] * ri);
        }
        if (KIND == LPCG_PC_NONE) rz += (double)ri * ri;
        if (KIND == LPCG_PC_LLT) {
            a.y[i] = kUnset;
            a.z[i] = kUnset;
        }
    }
    bb = block_sum<VT>(bb, lds);
    rr = block_sum<VT>(rr, lds);
    rz = block_sum<VT>(rz, lds);
    if (threadIdx.x == 0) {
        a.part_bb[blockIdx.x] = bb;
        a.part_rr[blockIdx.x] = rr;
        if (KIND != LPCG_PC_LLT) a.part_rz[blockIdx.x] = rz;
    }
}

// Single block: control words, ||b||^2, first convergence test; for
// Jacobi/none the first r.z and beta = 0.
template <int KIND>
__global__ void __launch_bounds__(VT) k_setup_scal(Args a) {
    __shared__ double lds[VT / kWave];
    const double bb0 = reduce_partials<VT>(a.part_bb, a.np_vec, lds);
    const double rr = reduce_partials<VT>(a.part_rr, a.np_vec, lds);
    const double rz = KIND != LPCG_PC_LLT ? reduce_partials<VT>(a.part_rz, a.np_vec, lds) : 0.0;
    if (threadIdx.x == 0) {
        const double bb = bb0 > 0 ? bb0 : 1.0;
        a.scal[S_BB] = bb;
        a.scal[S_RZ0] = rz;
        a.scal[S_BETA] = 0;
        a.scal[S_RR] = rr;
        a.ctrl[C_IT] = 0;
        a.ctrl[C_PHASE] = 0;
        a.ctrl[C_ITERS] = 0;
        a.ctrl[C_TICKET_F] = 0;
        a.ctrl[C_TICKET_B] = 0;
        a.ctrl[C_STATUS] = LPCG_OK;
        a.ctrl[C_RES0] = __float_as_int((float)(rr / bb));
        a.ctrl[C_RES] = a.ctrl[C_RES0];
        a.ctrl[C_RES_IT] = 0;
        const bool conv = !(rr > a.tol2 * bb);
        a.ctrl[C_DONE] = conv ? 1 : 0;
        if (a.hist) a.hist[0] = sqrt(rr / bb);
    }
}

// beta from the r.z partials (reducer block of the backward substitution;
// BS threads).
__device__ __forceinline__ void set_beta(const Args &a, double rz, int it) {
    const double old = a.scal[S_RZ0];
    a.scal[S_BETA] = it == 0 ? 0.0 : rz / old;
    a.scal[S_RZ0] = rz;
    if (a.coef && it >= 1 && it <= a.maxit) a.coef[2 * it + 1] = rz / old;
}

template <int BS = VT>
__device__ __forceinline__ void finish_rz(const Args &a, double *lds) {
    const double rz = reduce_published<BS>(a.sp_rz, a.np_rz, lds);
    if (threadIdx.x == 0) set_beta(a, rz, a.ctrl[C_IT]);
}

__global__ void __launch_bounds__(256) k_llt_fwd(Args a) {
    if (blockIdx.x % a.stride_f != 0) return;  // placement: only every stride-th block works
    if (is_done(a)) return;
    int *ticket = a.ctrl + C_TICKET_F;
    for (;;) {
        const int chunk = wave_ticket(ticket);
        if ((long)chunk * kWave >= a.n) break;
        float yv;
        trsv_chunk<false>(a.n, chunk * kWave, a.forder, a.lrp, a.lci, a.lval, a.r, a.y, yv, a.backoff_f);
    }
}

__global__ void __launch_bounds__(256) k_llt_bwd(Args a) {
    __shared__ double lds[VT / kWave];
    if (blockIdx.x % a.stride_b != 0) return;  // placement: only every stride-th block works
    if (is_done(a)) return;
    int *ticket = a.ctrl + C_TICKET_B;
    for (;;) {
        const int chunk = wave_ticket(ticket);
        if ((long)chunk * kWave >= a.n) break;
        float zv = 0.f;
        const int row = trsv_chunk<true>(a.n, chunk * kWave, a.border, a.urp, a.uci, a.utval,
                                         (const float *)a.y, a.z, zv, a.backoff_b);
        double rz = row >= 0 ? (double)a.r[row] * (double)zv : 0.0;
        rz = wave_sum(rz);
        if (lane_id() == 0) publish_partial(a.sp_rz, chunk, rz);
    }
    // reducer: the working block of highest index
    if ((int)blockIdx.x == ((int)gridDim.x - 1) / a.stride_b * a.stride_b) finish_rz(a, lds);
}

// Blocked forms (mode 3): one wave per block of rows (block stride 8: the
// XCD-local variant); the backward one publishes one r.z partial per block
// (in the block's fixed order) and the wave that solved the last block
// reduces them to beta (it waits only on blocks of lower tickets, held by
// running waves).
template <int W>
__global__ void __launch_bounds__(kWave) k_llt_fwd_blk(Args a) {
    if (blk_off_xcd(a.stride_f == 8)) return;
    if (is_done(a)) return;
    int *ticket = a.ctrl + C_TICKET_F;
    for (;;) {
        const int b = wave_ticket(ticket);
        if (b >= a.blk_f.nb) break;
        blk_solve<W, false>(a.blk_f, b, a.r, a.y, nullptr, a.backoff_f);
    }
}

template <int W>
__global__ void __launch_bounds__(kWave) k_llt_bwd_blk(Args a) {
    __shared__ double lds[1];
    if (blk_off_xcd(a.stride_b == 8)) return;
    if (is_done(a)) return;
    int *ticket = a.ctrl + C_TICKET_B;
    bool last = false;
    for (;;) {
        const int b = wave_ticket(ticket);
        if (b >= a.blk_b.nb) break;
        double rz = blk_solve<W, true>(a.blk_b, b, (const float *)a.y, a.z, a.r, a.backoff_b);
        rz = wave_sum(rz);
        if (lane_id() == 0) publish_partial(a.sp_rz, b, rz);
        last = last || b == a.blk_b.nb - 1;
    }
    if (last) finish_rz<kWave>(a, lds);
}

// Level-synchronous forms of the two substitutions: one launch per level
// (rows a.forder/a.border[lev0 .. lev0 + rows)).  Every backward launch
// writes one r.z partial per block at part_rz[part0 + block]; the last
// backward launch (last = 1) also finishes beta.
template <int G>
__global__ void __launch_bounds__(256) k_llt_fwd_level(Args a, int lev0, int rows) {
    if (is_done(a)) return;
    const int sub = threadIdx.x % G;
    constexpr int per = 256 / G;
    float *y = (float *)a.y;
    for (int idx = blockIdx.x * per + threadIdx.x / G; idx < rows; idx += gridDim.x * per) {
        const int row = a.forder[lev0 + idx];
        const float yv = trsv_level_row<false, G>(row, sub, a.lrp, a.lci, a.lval, a.r, y);
        if (sub == 0) y[row] = yv;
    }
}

template <int G>
__global__ void __launch_bounds__(256) k_llt_bwd_level(Args a, int lev0, int rows, int part0, int last) {
    __shared__ double lds[VT / kWave];
    if (is_done(a)) return;
    const int sub = threadIdx.x % G;
    constexpr int per = 256 / G;
    const float *y = (const float *)a.y;
    float *z = (float *)a.z;
    double rz = 0;
    for (int idx = blockIdx.x * per + threadIdx.x / G; idx < rows; idx += gridDim.x * per) {
        const int row = a.border[lev0 + idx];
        const float zv = trsv_level_row<true, G>(row, sub, a.urp, a.uci, a.utval, y, z);
        if (sub == 0) {
            z[row] = zv;
            rz += (double)a.r[row] * (double)zv;
        }
    }
    rz = block_sum<VT>(rz, lds);
    if (threadIdx.x == 0) publish_partial(a.sp_rz, part0 + blockIdx.x, rz);
    if (last && is_reducer()) finish_rz(a, lds);
}

// Two-level form of z = L^-T L^-1 r for systems whose forward level 0 is the
// row prefix [0, p) (rows without strictly-lower entries; p = two_level_p)
// and whose other rows all lie on level 1, as multicolour orderings of
// red-black grids give.  Then no edge joins two rows of the prefix or two rows
// of the suffix, so
//   prefix rows have L_jj as their only entry, at position j of l_val:
//     y_j = r_j / L_jj                                  (elementwise)
//   suffix rows:  y_i = (r_i - sum_{j<i} L_ij y_j) / L_ii,  z_i = y_i / L_ii
//     (their column of L holds only the diagonal)
//   prefix rows:  z_j = (y_j - sum_{i>j} L_ij z_i) / L_jj
// Two launches instead of one per level and direction: the suffix kernel
// forms y of its prefix neighbours on the fly; the prefix kernel recomputes
// y_j.  Each publishes one r.z partial per block; the prefix kernel's
// reducer block takes beta from all of them.
template <int G>
__global__ void __launch_bounds__(256) k_llt2_suffix(Args a, int p) {
    __shared__ double lds[VT / kWave];
    const int n = a.n;
    const int sub = threadIdx.x % G;
    constexpr int per = 256 / G;
    const int *__restrict__ lrp = a.lrp;
    const int *__restrict__ lci = a.lci;
    const float *__restrict__ lv = a.lval;
    const float *__restrict__ rv = a.r;
    float *__restrict__ z = (float *)a.z;
    // memory round trips per row: the done flag with the row's bounds and
    // r_i; its entries and L_ii; the gathers (two entries per lane at once)
    int row = p + blockIdx.x * per + threadIdx.x / G;
    int k0 = 0, k1 = 0;
    float ri = 0.f;
    const int flag = ld_ctrl(a.ctrl + C_DONE);
    if (row < n) {
        k0 = lrp[row];
        k1 = lrp[row + 1] - 1;
        ri = rv[row];
    }
    if (done_now(flag)) return;
    double rz = 0;
    while (row < n) {
        const float d = lv[k1];
        float acc = 0.f;
        for (int k = k0 + sub; k < k1; k += 2 * G) {
            const bool h2 = k + G < k1;
            const int j1 = lci[k];
            const float l1 = lv[k];
            int j2 = 0;
            float l2 = 0.f;
            if (h2) {
                j2 = lci[k + G];
                l2 = lv[k + G];
            }
            const float g1 = rv[j1] / lv[j1];
            float g2 = 0.f;
            if (h2) g2 = rv[j2] / lv[j2];
            acc += l1 * g1;
            if (h2) acc += l2 * g2;
        }
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
        if (sub == 0) {
            const float zv = ((ri - acc) / d) / d;
            z[row] = zv;
            rz += (double)ri * (double)zv;
        }
        row += gridDim.x * per;
        if (row < n) {
            k0 = lrp[row];
            k1 = lrp[row + 1] - 1;
            ri = rv[row];
        }
    }
    rz = block_sum<VT>(rz, lds);
    if (threadIdx.x == 0) publish_partial(a.sp_rz, blockIdx.x, rz);
}

template <int G>
__global__ void __launch_bounds__(256) k_llt2_prefix(Args a, int p, int part0) {
    __shared__ double lds[VT / kWave];
    const int sub = threadIdx.x % G;
    constexpr int per = 256 / G;
    const int *__restrict__ urp = a.urp;
    const int *__restrict__ uci = a.uci;
    const float *__restrict__ uv = a.utval;
    const float *__restrict__ rv = a.r;
    float *z = (float *)a.z;
    // round trips as in k_llt2_suffix (the z gathered here is the suffix
    // rows', which this kernel does not write)
    int row = blockIdx.x * per + threadIdx.x / G;
    int k0 = 0, k1 = 0;
    float ri = 0.f;
    const int flag = ld_ctrl(a.ctrl + C_DONE);
    if (row < p) {
        k0 = urp[row];
        k1 = urp[row + 1];
        ri = rv[row];
    }
    if (done_now(flag)) return;
    double rz = 0;
    while (row < p) {
        const float d = uv[k0];
        float acc = 0.f;
        for (int k = k0 + 1 + sub; k < k1; k += 2 * G) {
            const bool h2 = k + G < k1;
            const int j1 = uci[k];
            const float u1 = uv[k];
            int j2 = 0;
            float u2 = 0.f;
            if (h2) {
                j2 = uci[k + G];
                u2 = uv[k + G];
            }
            const float g1 = z[j1];
            float g2 = 0.f;
            if (h2) g2 = z[j2];
            acc += u1 * g1;
            if (h2) acc += u2 * g2;
        }
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
        if (sub == 0) {
            const float zv = (ri / d - acc) / d;
            z[row] = zv;
            rz += (double)ri * (double)zv;
        }
        row += gridDim.x * per;
        if (row < p) {
            k0 = urp[row];
            k1 = urp[row + 1];
            ri = rv[row];
        }
    }
    rz = block_sum<VT>(rz, lds);
    if (threadIdx.x == 0) publish_partial(a.sp_rz, part0 + blockIdx.x, rz);
    if (is_reducer()) finish_rz(a, lds);
}

// ELL form of the two-level pair (slots built with the pattern, this
// factor's values packed per solve by k_e2_pack): one row per lane, so a
// row's loads take two memory round trips (its slots, diagonal and r with
// the done flag; then the gathers) instead of three (bounds, entries,
// gathers).  A row's entries are summed in its CSR order.  W: the slot
// count (1..kEllMaxW), a template argument so that every slot load is
// unconditional and all are issued before the first wait.
struct E2 {
    int p, ws, wp;
    const int *scol, *pcol;
    const float *sval, *sdiag, *pval, *pdiag;
};

// The iteration's x, r update rides along (three launches per iteration
// instead of four).  The product before the application k >= 1 published
// its p.w partials without reducing them (defer); every block of both
// kernels sums them in the same fixed order, so all take the same
// alpha_k = r.z_(k-1) / p.w (a breakdown is seen by all alike and the
// prefix kernel's reducer records it).  Each kernel then forms
// r_i - alpha w_i for its own rows and writes it with x_i + alpha p_i; the
// suffix kernel forms its prefix neighbours' new r on the fly (the same
// fused multiply-add, so the same value the prefix kernel writes).  Both
// publish ||r||^2 partials; the prefix kernel's reducer counts the product,
// takes the convergence test and beta from one wait on both sets of
// partials.  The solve's first application (C_PHASE = 0) updates nothing.

// The deferred p.w partials: this thread's slots tid, tid + VT, ... (at most
// kMaxSpmvBlocks in all), loaded with the kernel's first data and summed
// only after its done test (a sum placed among the loads makes the compiler
// wait for them there), in the order reduce_published takes.
constexpr int kPwShare = kMaxSpmvBlocks / VT;

// (The partial arrays hold kMaxSpmvBlocks slots, so every load is in
// bounds; the slots past np_pw are read and left out of the sum.)
__device__ __forceinline__ void pw_load(const Args &a, double (&v)[kPwShare]) {
#pragma unroll
    for (int u = 0; u < kPwShare; ++u) v[u] = a.part_pw[(int)threadIdx.x + u * VT];
}

// alpha of the pending update (every block alike); false on a breakdown
// (p.w <= 0 or not finite, or r.z not finite).
__device__ __forceinline__ bool deferred_alpha(const Args &a, const double (&v)[kPwShare], double rz_old,
                                               double *lds, double &alpha) {
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < kPwShare; ++u)
        if ((int)threadIdx.x + u * VT < a.np_pw) s += v[u];
    const double pwt = block_sum<VT>(s, lds);
    alpha = rz_old / pwt;
    return pwt > 0.0 && isfinite(pwt) && isfinite(rz_old);
}

template <int W>
__global__ void __launch_bounds__(VT) k_llt2e_suffix(Args a, E2 e) {
    __shared__ double lds[VT / kWave];
    const int p = e.p, nb = a.n - p;
    const int i = blockIdx.x * VT + threadIdx.x;  // suffix row p + i
    const float *__restrict__ rv = a.r;
    const float *__restrict__ lv = a.lval;
    const float *__restrict__ wv = a.w;
    int col[W];
    float val[W];
    float d = 1.f, ri = 0.f, wi = 0.f, pa = 0.f, pb = 0.f;
    double xi = 0.0;
    const int flag = ld_ctrl(a.ctrl + C_DONE);
    int it = ld_ctrl(a.ctrl + C_IT);
    int phase = ld_ctrl(a.ctrl + C_PHASE);
    const double rz_old = ld_scal(a.scal + S_RZ0);
    double share[kPwShare];
    pw_load(a, share);
    if (i < nb) {
#pragma unroll
        for (int t = 0; t < W; ++t)
            {
                col[t] = e.scol[(size_t)t * nb + i];
                val[t] = e.sval[(size_t)t * nb + i];
            }
        d = e.sdiag[i];
        ri = rv[p + i];
        wi = wv[p + i];
        xi = a.x[p + i];
        pa = a.p0[p + i];
        pb = a.p1[p + i];
    }
    if (done_now(flag)) return;
    it = lane_value(it);
    const bool upd = done_now(phase);  // wave-uniform read of the phase word
    double alpha = 0.0;
    if (upd && !deferred_alpha(a, share, rz_old, lds, alpha)) return;  // breakdown: the prefix kernel records it
    const float af = (float)alpha;
    double rz = 0, rr = 0;
    if (i < nb) {
        float g[W];
#pragma unroll
        for (int t = 0; t < W; ++t)
            {
                float rj = rv[col[t]];
                if (upd) rj = __fmaf_rn(-af, wv[col[t]], rj);
                g[t] = rj / lv[col[t]];  // y_j = r_j / L_jj of prefix row j
            }
        if (upd) {  // p_k was written to the buffer of parity k - 1 = it
            ri = __fmaf_rn(-af, wi, ri);
            a.r[p + i] = ri;
            a.x[p + i] = __fma_rn(alpha, (double)((it & 1) ? pb : pa), xi);
            rr = (double)ri * ri;
        }
        float acc = 0.f;
#pragma unroll
        for (int t = 0; t < W; ++t)
            acc += val[t] * g[t];
        const float zv = ((ri - acc) / d) / d;
        ((float *)a.z)[p + i] = zv;
        rz = (double)ri * (double)zv;
    }
    rz = block_sum<VT>(rz, lds);
    if (upd) rr = block_sum<VT>(rr, lds);
    if (threadIdx.x == 0) {
        publish_partial(a.sp_rz, blockIdx.x, rz);
        if (upd) publish_partial(a.sp_rr, blockIdx.x, rr);
    }
}

template <int W>
__global__ void __launch_bounds__(VT) k_llt2e_prefix(Args a, E2 e, int part0) {
    __shared__ double lds[VT / kWave];
    const int p = e.p;
    const int j = blockIdx.x * VT + threadIdx.x;  // prefix row j
    float *z = (float *)a.z;  // reads the suffix rows' z, writes the prefix rows'
    int col[W > 0 ? W : 1];
    float val[W > 0 ? W : 1];
    float d = 1.f, rj = 0.f, wj = 0.f, pa = 0.f, pb = 0.f;
    double xj = 0.0;
    const int flag = ld_ctrl(a.ctrl + C_DONE);
    int it = ld_ctrl(a.ctrl + C_IT);
    int phase = ld_ctrl(a.ctrl + C_PHASE);
    const double rz_old = ld_scal(a.scal + S_RZ0);
    double share[kPwShare];
    pw_load(a, share);
    if (j < p) {
#pragma unroll
        for (int t = 0; t < W; ++t)
            {
                col[t] = e.pcol[(size_t)t * p + j];
                val[t] = e.pval[(size_t)t * p + j];
            }
        d = e.pdiag[j];
        rj = a.r[j];
        wj = a.w[j];
        xj = a.x[j];
        pa = a.p0[j];
        pb = a.p1[j];
    }
    if (done_now(flag)) return;
    it = lane_value(it);
    const bool upd = done_now(phase);
    double alpha = 0.0;
    if (upd && !deferred_alpha(a, share, rz_old, lds, alpha)) {
        if (is_reducer() && threadIdx.x == 0) {  // the breakdown of product it + 1
            a.ctrl[C_DONE] = 1;
            a.ctrl[C_STATUS] = LPCG_EBREAKDOWN;
            a.ctrl[C_ITERS] = it + 1;
            a.ctrl[C_IT] = it + 1;
        }
        return;
    }
    double rz = 0, rr = 0;
    if (j < p) {
        float g[W > 0 ? W : 1];
#pragma unroll
        for (int t = 0; t < W; ++t)
            g[t] = z[col[t]];
        if (upd) {
            rj = __fmaf_rn(-(float)alpha, wj, rj);
            a.r[j] = rj;
            a.x[j] = __fma_rn(alpha, (double)((it & 1) ? pb : pa), xj);
            rr = (double)rj * rj;
        }
        float acc = 0.f;
#pragma unroll
        for (int t = 0; t < W; ++t)
            acc += val[t] * g[t];
        const float zv = (rj / d - acc) / d;
        z[j] = zv;
        rz = (double)rj * (double)zv;
    }
    rz = block_sum<VT>(rz, lds);
    if (upd) rr = block_sum<VT>(rr, lds);
    if (threadIdx.x == 0) {
        publish_partial(a.sp_rz, part0 + blockIdx.x, rz);
        if (upd) publish_partial(a.sp_rr, part0 + blockIdx.x, rr);
    }
    if (!is_reducer()) return;
    if (upd) {  // product k = it + 1 done: alpha_k, the test of r_k, beta_k
        double rzt, rrt;
        reduce_published2<VT>(a.sp_rz, a.sp_rr, a.np_rz, lds, rzt, rrt);
        if (threadIdx.x == 0) {
            const int k = it + 1;
            a.ctrl[C_IT] = k;
            a.scal[S_ALPHA] = alpha;
            if (a.coef && k <= a.maxit) a.coef[2 * k] = alpha;
            record_residual(a, rrt, k);
            set_beta(a, rzt, k);
        }
    } else {  // the first application: r.z of r_0
        const double rzt = reduce_published<VT>(a.sp_rz, a.np_rz, lds);
        if (threadIdx.x == 0) {
            set_beta(a, rzt, 0);
            a.ctrl[C_PHASE] = 1;
        }
    }
}

// One factor's values into the pair's ELL slots (padding: 0) and diagonals.
// Slot indices past the row's width are clamped to its last slot and padding
// positions to entry 0, so that every load is unconditional and a thread's
// loads take two round trips (positions, then values); only the stores and
// the padding's zero depend on them.
__global__ void k_e2_pack(int n, int p, int ws, int wp, const int *__restrict__ spos,
                          const int *__restrict__ sdpos, const int *__restrict__ ppos,
                          const int *__restrict__ pdpos, const float *__restrict__ lval,
                          const float *__restrict__ utval, float *__restrict__ sval, float *__restrict__ sdiag,
                          float *__restrict__ pval, float *__restrict__ pdiag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int nb = n - p;
    const bool fs = i < nb && ws > 0, fp = i < p && wp > 0;
    const int is = fs ? i : 0, ip = fp ? i : 0;
    int ks[kEllMaxW], kp[kEllMaxW];
#pragma unroll
    for (int t = 0; t < kEllMaxW; ++t) {
        ks[t] = fs ? spos[(size_t)min(t, ws - 1) * nb + is] : -1;
        kp[t] = fp ? ppos[(size_t)min(t, wp - 1) * p + ip] : -1;
    }
    const int ds = i < nb ? sdpos[i] : 0, dp = i < p ? pdpos[i] : 0;
    float vs[kEllMaxW], vp[kEllMaxW];
#pragma unroll
    for (int t = 0; t < kEllMaxW; ++t) {
        vs[t] = lval[max(ks[t], 0)];
        vp[t] = utval[max(kp[t], 0)];
    }
    const float dvs = lval[ds], dvp = utval[dp];
#pragma unroll
    for (int t = 0; t < kEllMaxW; ++t) {
        if (fs && t < ws) sval[(size_t)t * nb + i] = ks[t] >= 0 ? vs[t] : 0.f;
        if (fp && t < wp) pval[(size_t)t * p + i] = kp[t] >= 0 ? vp[t] : 0.f;
    }
    if (i < nb) sdiag[i] = dvs;
    if (i < p) pdiag[i] = dvp;
}

// Single-workgroup substitutions (one block walking all levels): forward,
// backward, or both in one launch; the backward part also forms r.z with a
// block reduction and beta, so no partials are published.
__global__ void __launch_bounds__(kWgThreads) k_llt_wg(Args a, int do_fwd, int do_bwd) {
    __shared__ double lds[kWgThreads / kWave];
    if (is_done(a)) return;
    if (do_fwd)
        wg_substitute(a.nlev_f, a.flp, a.forder, a.lo_ptr_f, a.lo_col_f, a.lo_val_f, a.lo_diag_f, a.r,
                      (float *)a.y, nullptr);
    if (do_bwd) {
        const double rz = wg_substitute(a.nlev_b, a.blp, a.border, a.lo_ptr_b, a.lo_col_b, a.lo_val_b,
                                        a.lo_diag_b, (const float *)a.y, (float *)a.z, a.r);
        const double t = block_sum<kWgThreads>(rz, lds);
        if (threadIdx.x == 0) {
            const int it = a.ctrl[C_IT];
            const double old = a.scal[S_RZ0];
            a.scal[S_BETA] = it == 0 ? 0.0 : t / old;
            a.scal[S_RZ0] = t;
            if (a.coef && it >= 1 && it <= a.maxit) a.coef[2 * it + 1] = t / old;
        }
    }
}

// p = z + beta p_prev, w = A p and p.w partials (reduced by the next launch,
// which takes alpha and the breakdown test).
// Each thread takes two rows at a time (row and row + one grid's rows) and
// up to two entries of each per lane at once, so that its loads take three
// memory round trips per pair: the done flag, the iteration state, both
// rows' bounds and diagonal z; their entries and diagonal p_prev; the
// gathers.  Per lane the entries are summed in the order k0 + sub,
// k0 + sub + G, ..., as in k_spmv_pw_st.
template <int G, int KIND>
__global__ void __launch_bounds__(VT) k_spmv_pw(Args a) {
    __shared__ double lds[VT / kWave];
    const int n = a.n;
    const int sub = threadIdx.x % G;
    const int rpp = gridDim.x * (VT / G);  // rows per grid pass
    // the arrays this kernel reads never alias the ones it writes (p_new, w):
    // restrict-qualified copies let the compiler keep the gathers in flight
    // across the stores
    const int *__restrict__ rp = a.rp;
    const int *__restrict__ ci = a.ci;
    const float *__restrict__ v = a.v32;
    const float *__restrict__ zs = KIND == LPCG_PC_NONE ? a.r : (const float *)a.z;
    float *__restrict__ w = a.w;
    int ra = blockIdx.x * (VT / G) + threadIdx.x / G;
    int a0 = 0, a1 = 0, b0 = 0, b1 = 0;
    float za = 0.f, zb = 0.f;
    const int flag = ld_ctrl(a.ctrl + C_DONE);
    int it = ld_ctrl(a.ctrl + C_IT);
    const float beta = (float)ld_scal(a.scal + S_BETA);
    if (ra < n) {
        a0 = rp[ra];
        a1 = rp[ra + 1];
        za = zs[ra];
    }
    if (ra + rpp < n) {
        b0 = rp[ra + rpp];
        b1 = rp[ra + rpp + 1];
        zb = zs[ra + rpp];
    }
    if (done_now(flag)) return;
    it = lane_value(it);
    const bool first = it == 0;
    const float *__restrict__ pq = (it & 1) ? a.p0 : a.p1;
    float *__restrict__ pnw = (it & 1) ? a.p1 : a.p0;
    double pw = 0;
    while (ra < n) {
        const int rb = ra + rpp;
        const bool hb = rb < n;
        const float pa = first ? za : __fmaf_rn(beta, pq[ra], za);
        const float pb = !hb ? 0.f : first ? zb : __fmaf_rn(beta, pq[rb], zb);
        const int la = a1 - a0, lb = b1 - b0;  // lb = 0 without a second row
        float acca = 0.f, accb = 0.f;
        for (int t = sub; t < max(la, lb); t += 2 * G) {
            const bool ia1 = t < la, ia2 = t + G < la, ib1 = t < lb, ib2 = t + G < lb;
            int ja1 = 0, ja2 = 0, jb1 = 0, jb2 = 0;
            float va1 = 0.f, va2 = 0.f, vb1 = 0.f, vb2 = 0.f;
            if (ia1) { ja1 = ci[a0 + t]; va1 = v[a0 + t]; }
            if (ia2) { ja2 = ci[a0 + t + G]; va2 = v[a0 + t + G]; }
            if (ib1) { jb1 = ci[b0 + t]; vb1 = v[b0 + t]; }
            if (ib2) { jb2 = ci[b0 + t + G]; vb2 = v[b0 + t + G]; }
            float ga1 = 0.f, ga2 = 0.f, gb1 = 0.f, gb2 = 0.f;
            if (ia1) ga1 = first ? zs[ja1] : __fmaf_rn(beta, pq[ja1], zs[ja1]);
            if (ia2) ga2 = first ? zs[ja2] : __fmaf_rn(beta, pq[ja2], zs[ja2]);
            if (ib1) gb1 = first ? zs[jb1] : __fmaf_rn(beta, pq[jb1], zs[jb1]);
            if (ib2) gb2 = first ? zs[jb2] : __fmaf_rn(beta, pq[jb2], zs[jb2]);
            if (ia1) acca += va1 * ga1;
            if (ia2) acca += va2 * ga2;
            if (ib1) accb += vb1 * gb1;
            if (ib2) accb += vb2 * gb2;
        }
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) {
            acca += __shfl_xor(acca, off, G);
            accb += __shfl_xor(accb, off, G);
        }
        if (sub == 0) {
            pnw[ra] = pa;
            w[ra] = acca;
            pw += (double)pa * (double)acca;
            if (hb) {
                pnw[rb] = pb;
                w[rb] = accb;
                pw += (double)pb * (double)accb;
            }
        }
        ra += 2 * rpp;
        if (ra < n) {
            a0 = rp[ra];
            a1 = rp[ra + 1];
            za = zs[ra];
        }
        if (ra + rpp < n) {
            b0 = rp[ra + rpp];
            b1 = rp[ra + rpp + 1];
            zb = zs[ra + rpp];
        }
    }
    pw = block_sum<VT>(pw, lds);
    if (threadIdx.x == 0) a.part_pw[blockIdx.x] = pw;  // reduced by the next launch (k_xr or the pair)
}

// ELL form of k_spmv_pw (A's slots and FP32 values, analysis-built): one
// row per lane; the first row's loads take two memory round trips (its slots
// and z with the done flag and the iteration state; then the gathers and its
// p_prev).  A row's entries are summed in its CSR order (padding slots add
// 0 * p_i).
struct EA {
    int w;
    const int *col;
    const float *val;
};

template <int W, int KIND>
__global__ void __launch_bounds__(VT) k_spmv_pw_e(Args a, EA e) {
    __shared__ double lds[VT / kWave];
    const int n = a.n;
    const float *__restrict__ zs = KIND == LPCG_PC_NONE ? a.r : (const float *)a.z;
    const int *__restrict__ ec = e.col;
    const float *__restrict__ ev = e.val;
    float *__restrict__ wv = a.w;
    int row = blockIdx.x * VT + threadIdx.x;
    int col[W];
    float val[W];
    float zr = 0.f;
    const int flag = ld_ctrl(a.ctrl + C_DONE);
    int it = ld_ctrl(a.ctrl + C_IT);
    const float beta = (float)ld_scal(a.scal + S_BETA);
    if (row < n) {
#pragma unroll
        for (int t = 0; t < W; ++t)
            {
                col[t] = ec[(size_t)t * n + row];
                val[t] = ev[(size_t)t * n + row];
            }
        zr = zs[row];
    }
    if (done_now(flag)) return;
    it = lane_value(it);
    const bool first = it == 0;
    const float *__restrict__ pq = (it & 1) ? a.p0 : a.p1;
    float *__restrict__ pnw = (it & 1) ? a.p1 : a.p0;
    double pw = 0;
    while (row < n) {
        float g[W];
#pragma unroll
        for (int t = 0; t < W; ++t)
            g[t] = first ? zs[col[t]] : __fmaf_rn(beta, pq[col[t]], zs[col[t]]);
        const float pr = first ? zr : __fmaf_rn(beta, pq[row], zr);
        float acc = 0.f;
#pragma unroll
        for (int t = 0; t < W; ++t)
            acc += val[t] * g[t];
        pnw[row] = pr;
        wv[row] = acc;
        pw += (double)pr * (double)acc;
        row += gridDim.x * VT;
        if (row < n) {
#pragma unroll
            for (int t = 0; t < W; ++t)
                {
                    col[t] = ec[(size_t)t * n + row];
                    val[t] = ev[(size_t)t * n + row];
                }
            zr = zs[row];
        }
    }
    pw = block_sum<VT>(pw, lds);
    if (threadIdx.x == 0) a.part_pw[blockIdx.x] = pw;  // reduced by the next launch (k_xr or the pair)
}

// LDS-staged form of k_spmv_pw (kern_spmv.h): block b forms the new search
// direction p_j = z_j + beta p_prev_j over its column window into LDS (each
// input read once per block, in order), writes p and w = A p for its own rows
// (the diagonal's p from its own inputs) and stores its p.w partial.  The
// arithmetic per entry and the reduction are those of k_spmv_pw: p, w and
// p.w agree bit for bit.
template <int G, int KIND>
__global__ void __launch_bounds__(VT) k_spmv_pw_st(Args a, int R, const int *__restrict__ win) {
    extern __shared__ float sp[];
    __shared__ double lds[VT / kWave];
    if (is_done(a)) return;
    const int it = a.ctrl[C_IT];
    const bool first = it == 0;
    const float beta = (float)a.scal[S_BETA];
    const int *__restrict__ rp = a.rp;
    const int *__restrict__ ci = a.ci;
    const float *__restrict__ v = a.v32;
    const float *__restrict__ zs = KIND == LPCG_PC_NONE ? a.r : (const float *)a.z;
    const float *__restrict__ pq = (it & 1) ? a.p0 : a.p1;
    float *__restrict__ pnw = (it & 1) ? a.p1 : a.p0;
    float *__restrict__ w = a.w;
    const int r0 = blockIdx.x * R, r1 = min(a.n, r0 + R);
    const int lo = win[2 * blockIdx.x], len = win[2 * blockIdx.x + 1] - lo + 1;
    stage_window(sp, len, [&](int i) {
        const float zj = zs[lo + i];
        return first ? zj : __fmaf_rn(beta, pq[lo + i], zj);
    });
    __syncthreads();
    const int sub = threadIdx.x % G;
    double pw = 0;
    for (int row = r0 + (int)threadIdx.x / G; row < r1; row += VT / G) {
        const float zi = zs[row];
        const float pi = first ? zi : __fmaf_rn(beta, pq[row], zi);
        float acc = 0.f;
        for (int k = rp[row] + sub; k < rp[row + 1]; k += G) {
            const int c = ci[k];
            acc += v[k] * (c == row ? pi : sp[c - lo]);
        }
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
        if (sub == 0) {
            pnw[row] = pi;
            w[row] = acc;
            pw += (double)pi * (double)acc;
        }
    }
    pw = block_sum<VT>(pw, lds);
    if (threadIdx.x == 0) a.part_pw[blockIdx.x] = pw;  // reduced by the next launch (k_xr or the pair)
}

// x += alpha p, r -= alpha w, ||r||^2 (Jacobi/none: r.z) partials, presets
// for the dependency-driven substitutions; the reducer block takes the
// convergence test (Jacobi/none: and beta) and rearms the tickets.
template <int KIND>
__global__ void __launch_bounds__(VT) k_xr(Args a) {
    __shared__ double lds[VT / kWave];
    const int n = a.n;
    // element-wise: each index is read and written by one thread only
    const float *__restrict__ wr = a.w;
    const float *__restrict__ dv = a.dinv;
    double *__restrict__ xr = a.x;
    float *__restrict__ rv = a.r;
    uint32_t *__restrict__ zb = a.z;
    // the first element's w, r, x (and 1/diag) are loaded with the done flag,
    // the iteration state and the product's p.w partials, and so is p from
    // both buffers (which one holds the current direction depends on the
    // iteration): one memory round trip
    int i = blockIdx.x * VT + threadIdx.x;
    float wi = 0.f, ri0 = 0.f, di = 0.f, pa = 0.f, pb = 0.f;
    double xi = 0.0;
    const int flag = ld_ctrl(a.ctrl + C_DONE);
    int it = ld_ctrl(a.ctrl + C_IT);
    const double rz_old = ld_scal(a.scal + S_RZ0);
    double share[kPwShare];
    pw_load(a, share);
    const float *__restrict__ p0 = a.p0;
    const float *__restrict__ p1 = a.p1;
    if (i < n) {
        wi = wr[i];
        ri0 = rv[i];
        xi = xr[i];
        pa = p0[i];
        pb = p1[i];
        if (KIND == LPCG_PC_JACOBI) di = dv[i];
    }
    if (done_now(flag)) return;
    it = lane_value(it);
    const int k = it + 1;  // the product this update completes
    double alpha;
    if (!deferred_alpha(a, share, rz_old, lds, alpha)) {
        if (is_reducer() && threadIdx.x == 0) {
            a.ctrl[C_DONE] = 1;
            a.ctrl[C_STATUS] = LPCG_EBREAKDOWN;
            a.ctrl[C_ITERS] = k;
            a.ctrl[C_IT] = k;
        }
        return;
    }
    const float af = (float)alpha;
    const bool odd = (it & 1) != 0;  // p_k is in the buffer of parity k - 1
    const float *__restrict__ pr = odd ? p1 : p0;
    float pi = odd ? pb : pa;
    double rr = 0, rzn = 0;
    while (i < n) {
        xr[i] = __fma_rn(alpha, (double)pi, xi);
        const float ri = __fmaf_rn(-af, wi, ri0);
        rv[i] = ri;
        rr += (double)ri * ri;
        if (KIND == LPCG_PC_JACOBI) {
            rzn += (double)ri * ri * di;
            zb[i] = __float_as_uint(di * ri);
        }
        if (KIND == LPCG_PC_NONE) rzn += (double)ri * ri;
        if (KIND == LPCG_PC_LLT) {
            if (a.reset_y) a.y[i] = kUnset;
            if (a.reset_z) zb[i] = kUnset;
        }
        i += gridDim.x * VT;
        if (i < n) {
            wi = wr[i];
            ri0 = rv[i];
            xi = xr[i];
            pi = pr[i];
            if (KIND == LPCG_PC_JACOBI) di = dv[i];
        }
    }
    rr = block_sum<VT>(rr, lds);
    if (KIND != LPCG_PC_LLT) rzn = block_sum<VT>(rzn, lds);
    if (threadIdx.x == 0) {
        publish_partial(a.sp_rr, blockIdx.x, rr);
        if (KIND != LPCG_PC_LLT) publish_partial(a.sp_rz2, blockIdx.x, rzn);
    }
    if (!is_reducer()) return;
    double rrt, rzt = 0.0;
    if (KIND != LPCG_PC_LLT) reduce_published2<VT>(a.sp_rr, a.sp_rz2, gridDim.x, lds, rrt, rzt);
    else rrt = reduce_published<VT>(a.sp_rr, gridDim.x, lds);
    if (threadIdx.x == 0) {
        a.ctrl[C_IT] = k;
        a.scal[S_ALPHA] = alpha;
        if (a.coef && k <= a.maxit) a.coef[2 * k] = alpha;
        record_residual(a, rrt, k);
        if (KIND != LPCG_PC_LLT) {
            set_beta(a, rzt, k);
        } else {
            a.ctrl[C_TICKET_F] = 0;
            a.ctrl[C_TICKET_B] = 0;
        }
    }
}

// FP64 true residual partials ||b - A x||^2 (FP64 values), in the setup's
// ||b||^2 slots, which nothing reads during the iteration: the host may append
// these two kernels to a chunk that is still running.
__global__ void __launch_bounds__(VT) k_true_res(Args a) {
    __shared__ double lds[VT / kWave];
    double rr = 0;
    for (int i = blockIdx.x * VT + threadIdx.x; i < a.n; i += gridDim.x * VT) {
        const double s = row_ax64(a, i);
        const double ri = a.b[i] - s;
        rr += ri * ri;
    }
    rr = block_sum<VT>(rr, lds);
    if (threadIdx.x == 0) a.part_bb[blockIdx.x] = rr;
}

__global__ void __launch_bounds__(VT) k_true_fin(Args a) {
    __shared__ double lds[VT / kWave];
    const double rr = reduce_partials<VT>(a.part_bb, a.np_vec, lds);
    if (threadIdx.x == 0) a.scal[S_TRUE] = rr;
}

// Dynamic LDS above the default limit for the blocked kernels of direction d
// (set before any launch or capture).
int blk_set_lds(const lpcg_system *s, int d) {
    const int b = (int)(s->blk_W[d] == 3 ? blk_lds_bytes<3>(s->blk_B[d], s->blk_chmax[d])
                                         : blk_lds_bytes<7>(s->blk_B[d], s->blk_chmax[d]));
    const void *k = s->blk_W[d] == 3 ? (d ? (const void *)k_llt_bwd_blk<3> : (const void *)k_llt_fwd_blk<3>)
                                     : (d ? (const void *)k_llt_bwd_blk<7> : (const void *)k_llt_fwd_blk<7>);
    LPCG_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, b));
    return LPCG_OK;
}

// The PCG iteration applies L L^T through the two-level pair when the system
// has the two-level structure and both substitutions run level-synchronous
// (the tuner's choice for so few levels).
bool two_level_path(const lpcg_system *s) {
    return s->two_level_p > 0 && s->two_level_p < s->n && s->trsv[0].mode == 1 && s->trsv[1].mode == 1;
}

// The pair runs in its ELL form whenever the analysis built it (rows of at
// most kEllMaxW entries).
bool e2_path(const lpcg_system *s) { return two_level_path(s) && s->e2_ws > 0; }

E2 e2_args(const lpcg_system *s) {
    return E2{s->two_level_p, s->e2_ws, s->e2_wp, s->e2_scol, s->e2_pcol,
              s->e2_sval, s->e2_sdiag, s->e2_pval, s->e2_pdiag};
}

EA ea_args(const lpcg_system *s) { return EA{s->ea_w, s->ea_col, s->ea_val}; }

int ell_blocks(const lpcg_system *s) { return std::max(1, std::min(kMaxSpmvBlocks, (s->n + VT - 1) / VT)); }

// ELL launches with the slot count as a template argument (1..kEllMaxW).
template <int KIND>
void launch_spmv_pw_e(const lpcg_system *s, const Args &a, hipStream_t st) {
    const int eb = ell_blocks(s);
    const EA e = ea_args(s);
    switch (s->ea_w) {
        case 1: k_spmv_pw_e<1, KIND><<<eb, VT, 0, st>>>(a, e); break;
        case 2: k_spmv_pw_e<2, KIND><<<eb, VT, 0, st>>>(a, e); break;
        case 3: k_spmv_pw_e<3, KIND><<<eb, VT, 0, st>>>(a, e); break;
        case 4: k_spmv_pw_e<4, KIND><<<eb, VT, 0, st>>>(a, e); break;
        case 5: k_spmv_pw_e<5, KIND><<<eb, VT, 0, st>>>(a, e); break;
        case 6: k_spmv_pw_e<6, KIND><<<eb, VT, 0, st>>>(a, e); break;
        case 7: k_spmv_pw_e<7, KIND><<<eb, VT, 0, st>>>(a, e); break;
        default: k_spmv_pw_e<8, KIND><<<eb, VT, 0, st>>>(a, e); break;
    }
}

void launch_pair_e(const lpcg_system *s, const Args &a, hipStream_t st) {
    const int p = s->two_level_p;
    const int nbs = (s->n - p + VT - 1) / VT, nbp = (p + VT - 1) / VT;
    const E2 e = e2_args(s);
    switch (s->e2_ws) {
        case 1: k_llt2e_suffix<1><<<nbs, VT, 0, st>>>(a, e); break;
        case 2: k_llt2e_suffix<2><<<nbs, VT, 0, st>>>(a, e); break;
        case 3: k_llt2e_suffix<3><<<nbs, VT, 0, st>>>(a, e); break;
        case 4: k_llt2e_suffix<4><<<nbs, VT, 0, st>>>(a, e); break;
        case 5: k_llt2e_suffix<5><<<nbs, VT, 0, st>>>(a, e); break;
        case 6: k_llt2e_suffix<6><<<nbs, VT, 0, st>>>(a, e); break;
        case 7: k_llt2e_suffix<7><<<nbs, VT, 0, st>>>(a, e); break;
        default: k_llt2e_suffix<8><<<nbs, VT, 0, st>>>(a, e); break;
    }
    switch (s->e2_wp) {
        case 0: k_llt2e_prefix<0><<<nbp, VT, 0, st>>>(a, e, nbs); break;
        case 1: k_llt2e_prefix<1><<<nbp, VT, 0, st>>>(a, e, nbs); break;
        case 2: k_llt2e_prefix<2><<<nbp, VT, 0, st>>>(a, e, nbs); break;
        case 3: k_llt2e_prefix<3><<<nbp, VT, 0, st>>>(a, e, nbs); break;
        case 4: k_llt2e_prefix<4><<<nbp, VT, 0, st>>>(a, e, nbs); break;
        case 5: k_llt2e_prefix<5><<<nbp, VT, 0, st>>>(a, e, nbs); break;
        case 6: k_llt2e_prefix<6><<<nbp, VT, 0, st>>>(a, e, nbs); break;
        case 7: k_llt2e_prefix<7><<<nbp, VT, 0, st>>>(a, e, nbs); break;
        default: k_llt2e_prefix<8><<<nbp, VT, 0, st>>>(a, e, nbs); break;
    }
}

// Blocks of the PCG's product kernel in the form in force (enqueue_spmv).
int product_grid(const lpcg_system *s) {
    if (s->spmv_ell && s->ea_w > 0) return ell_blocks(s);
    if (s->spmv_rows > 0) return (s->n + s->spmv_rows - 1) / s->spmv_rows;
    return s->spmv_blocks;
}

// One iteration = the application z = P^-1 r (LLT only), the SpMV with the
// new search direction and p.w, and the x, r update; enqueued in parts so
// that the timing aid can bracket each.
template <int KIND>
int enqueue_apply(const lpcg_system *s, const Args &a, hipStream_t st) {
    if (KIND == LPCG_PC_LLT && e2_path(s)) {  // the x, r update rides along (k_xr is not launched)
        launch_pair_e(s, a, st);
    } else if (KIND == LPCG_PC_LLT && two_level_path(s)) {
        const int G = s->trsv_g, p = s->two_level_p;
        const int nbs = level_blocks(s->n - p, G), nbp = level_blocks(p, G);
        if (G == 4) {
            k_llt2_suffix<4><<<nbs, 256, 0, st>>>(a, p);
            k_llt2_prefix<4><<<nbp, 256, 0, st>>>(a, p, nbs);
        } else if (G == 8) {
            k_llt2_suffix<8><<<nbs, 256, 0, st>>>(a, p);
            k_llt2_prefix<8><<<nbp, 256, 0, st>>>(a, p, nbs);
        } else {
            k_llt2_suffix<16><<<nbs, 256, 0, st>>>(a, p);
            k_llt2_prefix<16><<<nbp, 256, 0, st>>>(a, p, nbs);
        }
    } else if (KIND == LPCG_PC_LLT) {
        const int G = s->trsv_g;
        const bool wf = s->trsv[0].mode == 2, wb = s->trsv[1].mode == 2;
        if (wf) {
            k_llt_wg<<<1, kWgThreads, 0, st>>>(a, 1, wb ? 1 : 0);
        } else if (s->trsv[0].mode == 3) {
            const int grid = a.blk_f.nb * (a.stride_f == 8 ? 8 : 1);
            if (s->blk_W[0] == 3)
                k_llt_fwd_blk<3><<<grid, kWave, blk_lds_bytes<3>(a.blk_f.bmax, a.blk_f.chmax), st>>>(a);
            else
                k_llt_fwd_blk<7><<<grid, kWave, blk_lds_bytes<7>(a.blk_f.bmax, a.blk_f.chmax), st>>>(a);
        } else if (s->trsv[0].mode == 0) {
            k_llt_fwd<<<(trsv_waves(s->n, s->trsv[0].waves) + 3) / 4 * s->trsv[0].stride, 256, 0, st>>>(a);
        } else {
            const std::vector<int> &lp = s->h_flev_ptr;
            for (size_t l = 0; l + 1 < lp.size(); ++l) {
                const int rows = lp[l + 1] - lp[l], nb = level_blocks(rows, G);
                if (G == 4) k_llt_fwd_level<4><<<nb, 256, 0, st>>>(a, lp[l], rows);
                else if (G == 8) k_llt_fwd_level<8><<<nb, 256, 0, st>>>(a, lp[l], rows);
                else k_llt_fwd_level<16><<<nb, 256, 0, st>>>(a, lp[l], rows);
            }
        }
        if (wb) {
            if (!wf) k_llt_wg<<<1, kWgThreads, 0, st>>>(a, 0, 1);
        } else if (s->trsv[1].mode == 3) {
            const int grid = a.blk_b.nb * (a.stride_b == 8 ? 8 : 1);
            if (s->blk_W[1] == 3)
                k_llt_bwd_blk<3><<<grid, kWave, blk_lds_bytes<3>(a.blk_b.bmax, a.blk_b.chmax), st>>>(a);
            else
                k_llt_bwd_blk<7><<<grid, kWave, blk_lds_bytes<7>(a.blk_b.bmax, a.blk_b.chmax), st>>>(a);
        } else if (s->trsv[1].mode == 0) {
            k_llt_bwd<<<(trsv_waves(s->n, s->trsv[1].waves) + 3) / 4 * s->trsv[1].stride, 256, 0, st>>>(a);
        } else {
            const std::vector<int> &lp = s->h_blev_ptr;
            int part0 = 0;
            for (size_t l = 0; l + 1 < lp.size(); ++l) {
                const int rows = lp[l + 1] - lp[l], nb = level_blocks(rows, G);
                const int last = l + 2 == lp.size();
                if (G == 4) k_llt_bwd_level<4><<<nb, 256, 0, st>>>(a, lp[l], rows, part0, last);
                else if (G == 8) k_llt_bwd_level<8><<<nb, 256, 0, st>>>(a, lp[l], rows, part0, last);
                else k_llt_bwd_level<16><<<nb, 256, 0, st>>>(a, lp[l], rows, part0, last);
                part0 += nb;
            }
        }
    }
    LPCG_LAUNCH_CHECK();
    return LPCG_OK;
}

template <int KIND>
int enqueue_spmv(const lpcg_system *s, const Args &a, hipStream_t st) {
    if (s->spmv_ell && s->ea_w > 0) {
        launch_spmv_pw_e<KIND>(s, a, st);
        LPCG_LAUNCH_CHECK();
        return LPCG_OK;
    }
    if (s->spmv_rows > 0) {  // LDS-staged (windows prepared when the configuration was set)
        const int R = s->spmv_rows, nb = (s->n + R - 1) / R;
        const size_t lds = sizeof(float) * (size_t)std::max(1, s->spmv_wmax);
        switch (s->spmv_group) {
            case 4: k_spmv_pw_st<4, KIND><<<nb, VT, lds, st>>>(a, R, s->spmv_win); break;
            case 8: k_spmv_pw_st<8, KIND><<<nb, VT, lds, st>>>(a, R, s->spmv_win); break;
            case 16: k_spmv_pw_st<16, KIND><<<nb, VT, lds, st>>>(a, R, s->spmv_win); break;
            case 32: k_spmv_pw_st<32, KIND><<<nb, VT, lds, st>>>(a, R, s->spmv_win); break;
            default: k_spmv_pw_st<64, KIND><<<nb, VT, lds, st>>>(a, R, s->spmv_win); break;
        }
        LPCG_LAUNCH_CHECK();
        return LPCG_OK;
    }
    const int sb = s->spmv_blocks;
    switch (s->spmv_group) {
        case 4: k_spmv_pw<4, KIND><<<sb, VT, 0, st>>>(a); break;
        case 8: k_spmv_pw<8, KIND><<<sb, VT, 0, st>>>(a); break;
        case 16: k_spmv_pw<16, KIND><<<sb, VT, 0, st>>>(a); break;
        case 32: k_spmv_pw<32, KIND><<<sb, VT, 0, st>>>(a); break;
        default: k_spmv_pw<64, KIND><<<sb, VT, 0, st>>>(a); break;
    }
    LPCG_LAUNCH_CHECK();
    return LPCG_OK;
}

template <int KIND>
int enqueue_xr(const lpcg_system *s, const Args &a, hipStream_t st) {
    if (KIND == LPCG_PC_LLT && e2_path(s)) return LPCG_OK;  // done by the next application
    k_xr<KIND><<<s->vec_blocks, VT, 0, st>>>(a);
    LPCG_LAUNCH_CHECK();
    return LPCG_OK;
}

template <int KIND>
int enqueue_iteration(const lpcg_system *s, const Args &a, hipStream_t st) {
    int rc;
    if ((rc = enqueue_apply<KIND>(s, a, st)) || (rc = enqueue_spmv<KIND>(s, a, st))) return rc;
    return enqueue_xr<KIND>(s, a, st);
}

// Iterations to launch before the next look at the done flag, when the
// caller fixed no interval.  The recorded relative residual (squared) decays
// about geometrically in PCG, so its decay rate over the iterations since the
// previous look is extrapolated to the tolerance.  The extrapolation spans at
// most four times the iterations it was measured over and stops past the
// iteration cap; without a decay to measure it is kChunk0.  Every look costs
// a host round trip and every iteration launched after convergence the
// launches of an iteration, so both errors cost about the same.  The decay
// quickens late in a solve (CG's superlinear phase), which a rate measured
// earlier misses, so the extrapolation is shortened by kLate: on recorded
// histories of red-black IC(0) and Jacobi solves at 64^3 (tolerances 1e-2,
// 1e-6, 1e-10) 0.85 gave 3-4 looks and at most 6 iterations past convergence,
// 1.0 up to 18.
constexpr int kChunk0 = 8;
constexpr double kLate = 0.85;

struct ChunkPlan {
    int prev_it = 0;
    float prev_res = -1.0f;  // read from C_RES0 at the first look
    double rate = 0;         // last measured d log(res) / d iteration (< 0: decaying)
};

// it, res: the last recorded iteration and its ||r||^2 / ||b||^2.
int next_chunk(int it, float res, double tol2, int maxit, ChunkPlan &c, bool &fin) {
    fin = false;
    const int span = it - c.prev_it;
    const float res_prev = c.prev_res;
    c.prev_it = it;
    c.prev_res = res;
    if (span <= 0 || !(res > 0.0f) || !(res_prev > 0.0f) || !std::isfinite(res)) return kChunk0;
    const double rate = (std::log((double)res) - std::log((double)res_prev)) / span;
    if (!(rate < -1e-6)) return kChunk0;
    c.rate = rate;
    const double cap = std::min(4.0 * span, (double)std::max(1, maxit - it + 1));
    const double need = tol2 > 0 ? std::ceil(kLate * (std::log(tol2) - std::log((double)res)) / rate) : cap;
    fin = tol2 > 0 && need <= cap;
    return (int)std::max(1.0, std::min(need, cap));
}

int next_chunk(const int *ctrl, double tol2, int maxit, ChunkPlan &c, bool &fin) {
    if (c.prev_res < 0.0f) memcpy(&c.prev_res, &ctrl[C_RES0], sizeof(float));
    float res;
    memcpy(&res, &ctrl[C_RES], sizeof(float));
    return next_chunk(ctrl[C_RES_IT], res, tol2, maxit, c, fin);
}

// First chunk of a restart from the FP64 true residual (relative, squared:
// res0): the previous attempt's decay rate extrapolated from res0, at most
// kChunk0; 0 without a rate to extrapolate.
int restart_chunk(double res0, double tol2, double rate) {
    if (!(rate < 0) || !(res0 > 0) || !(tol2 > 0) || !std::isfinite(res0)) return 0;
    const double need = std::ceil((std::log(tol2) - std::log(res0)) / rate);
    return need <= kChunk0 ? (int)std::max(1.0, need) : 0;
}

template <int KIND>
// first_chunk: iterations of the first chunk (0: kChunk0), predicted to reach
// the tolerance when nonzero.  A chunk predicted to reach it is followed by
// the FP64 true residual, which then comes back with the done flag
// (true_ready) instead of after one more round trip.
int run_solve(lpcg_system *s, const Args &a, const lpcg_solve_opts &o, int first_chunk, int &iters_total,
              int &status, double &rate, bool &true_ready, hipStream_t st) {
    const int vb = s->vec_blocks;
    k_setup<KIND><<<vb, VT, 0, st>>>(a);
    k_setup_scal<KIND><<<1, VT, 0, st>>>(a);
    LPCG_LAUNCH_CHECK();
    const bool adaptive = o.check_every <= 0 && !o.use_graph;
    // the fused red-black path records iteration k in the launches of k + 1
    const int lag = KIND == LPCG_PC_LLT && e2_path(s) ? 1 : 0;
    bool fin = adaptive && first_chunk > 0;
    int chunk = o.check_every > 0 ? o.check_every : fin ? first_chunk + lag : kChunk0;
    true_ready = false;
    hipGraphExec_t exec = nullptr;
    if (o.use_graph) {
        // key: kernel arguments + preconditioner kind + chunk length
        std::vector<unsigned char> key(sizeof(Args) + 15 * sizeof(int) + 2 * sizeof(void *));
        memcpy(key.data(), &a, sizeof(Args));
        const int extra[15] = {KIND, chunk, s->trsv[0].mode, s->trsv[0].waves, s->trsv[0].backoff,
                               s->trsv[1].mode, s->trsv[1].waves, s->trsv[1].backoff, s->trsv_g,
                               s->trsv[0].blk, s->trsv[1].blk, s->trsv[0].runs, s->trsv[1].runs,
                               s->blk_nb[0], s->blk_nb[1]};
        // (the block strides travel in Args and are part of the key through it)
        memcpy(key.data() + sizeof(Args), extra, sizeof(extra));
        const void *sched[2] = {s->blk_rec[0], s->blk_rec[1]};  // blocked schedules in the graph
        memcpy(key.data() + sizeof(Args) + sizeof(extra), sched, sizeof(sched));
        if (s->graph_exec && s->graph_key == key) {
            exec = s->graph_exec;
        } else {
            if (s->graph_exec) {
                (void)hipGraphExecDestroy(s->graph_exec);
                s->graph_exec = nullptr;
            }
            if (!s->cap_stream) LPCG_HIP(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
            hipGraph_t graph = nullptr;
            LPCG_HIP(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
            int rc = LPCG_OK;
            for (int c = 0; c < chunk && rc == LPCG_OK; ++c) rc = enqueue_iteration<KIND>(s, a, s->cap_stream);
            hipError_t e = hipStreamEndCapture(s->cap_stream, &graph);
            if (rc != LPCG_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return rc;
            }
            LPCG_HIP(e);
            hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            LPCG_HIP(ie);
            s->graph_exec = exec;
            s->graph_key = key;
        }
    }
    int rc = LPCG_OK;
    long launched = 0;
    ChunkPlan plan;
    for (;;) {
        if (exec) {
            hipError_t e = hipGraphLaunch(exec, st);
            if (e != hipSuccess) { rc = hip_fail(e, "hipGraphLaunch", __FILE__, __LINE__); break; }
        } else {
            for (int c = 0; c < chunk && rc == LPCG_OK; ++c) rc = enqueue_iteration<KIND>(s, a, st);
            if (rc != LPCG_OK) break;
        }
        launched += chunk;
        if (fin) {
            k_true_res<<<vb, VT, 0, st>>>(a);
            k_true_fin<<<1, VT, 0, st>>>(a);
            LPCG_LAUNCH_CHECK();
        }
        hipError_t e = hipMemcpyAsync(s->h_ctrl, s->ctrl, sizeof(int) * C_NCTRL, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess && fin)
            e = hipMemcpyAsync(s->h_scal, s->scal, sizeof(double) * S_NSCAL, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) { rc = hip_fail(e, "pcg control readback", __FILE__, __LINE__); break; }
        if (s->h_ctrl[C_DONE]) {
            true_ready = fin;
            break;
        }
        // the device stops at maxit (plus the one-iteration lag of the fused
        // red-black update), so this only trips on a kernel that never set the flag
        if (launched > (long)a.maxit + 4L * std::max(chunk, kChunk0) + 8) {
            set_error("pcg: done flag never set");
            rc = LPCG_EHIP;
            break;
        }
        if (adaptive) chunk = next_chunk(s->h_ctrl, a.tol2, a.maxit, plan, fin);
    }
    if (rc != LPCG_OK) return rc;
    if (plan.rate < 0) rate = plan.rate;
    iters_total += s->h_ctrl[C_ITERS];
    status = s->h_ctrl[C_STATUS];
    return LPCG_OK;
}

// Kernel arguments of a solve on system s with preconditioner P from x (both
// in the caller's numbering; a reordered system works on internal copies),
// with the factor's values packed for the configured substitution modes.
int build_args(lpcg_system *s, const lpcg_precond *P, const double *b, double *x, double tol, int maxit,
               double *hist, double *coef, Args &a, hipStream_t st) {
    a = Args{};
    a.n = s->n;
    a.np_vec = s->vec_blocks;
    a.maxit = maxit > 0 ? maxit : s->n;
    a.kind = P->kind;
    a.np_pw = product_grid(s);
    a.backoff_f = s->trsv[0].backoff;
    a.backoff_b = s->trsv[1].backoff;
    a.stride_f = s->trsv[0].stride;
    a.stride_b = s->trsv[1].stride;
    a.reset_y = s->trsv[0].mode == 0 || s->trsv[0].mode == 3;
    a.reset_z = s->trsv[1].mode == 0 || s->trsv[1].mode == 3;
    if (e2_path(s)) {
        a.np_rz = (s->n - s->two_level_p + VT - 1) / VT + (s->two_level_p + VT - 1) / VT;
    } else if (two_level_path(s)) {
        a.np_rz = level_blocks(s->n - s->two_level_p, s->trsv_g) + level_blocks(s->two_level_p, s->trsv_g);
    } else if (s->trsv[1].mode == 0) {
        a.np_rz = (s->n + kWave - 1) / kWave;
    } else if (s->trsv[1].mode == 3) {
        a.np_rz = s->blk_nb[1];
    } else {
        a.np_rz = 0;
        for (size_t l = 0; l + 1 < s->h_blev_ptr.size(); ++l)
            a.np_rz += level_blocks(s->h_blev_ptr[l + 1] - s->h_blev_ptr[l], s->trsv_g);
    }
    a.rp = s->rowptr;
    a.ci = s->colind;
    a.v32 = s->val32;
    a.v64 = s->val64;
    a.lrp = s->lrowptr;
    a.lci = s->lcol;
    a.urp = s->urowptr;
    a.uci = s->ucol;
    a.forder = s->flev_rows;
    a.border = s->blev_rows;
    a.nlev_f = s->nlev_f;
    a.nlev_b = s->nlev_b;
    a.flp = s->flev_ptr;
    a.blp = s->blev_ptr;
    a.lo_ptr_f = s->lo_ptr[0];
    a.lo_col_f = s->lo_col[0];
    a.lo_val_f = s->lo_val[0];
    a.lo_diag_f = s->lo_diag[0];
    a.lo_ptr_b = s->lo_ptr[1];
    a.lo_col_b = s->lo_col[1];
    a.lo_val_b = s->lo_val[1];
    a.lo_diag_b = s->lo_diag[1];
    a.lval = P->l_val;
    a.utval = P->ut_val;
    a.dinv = P->dinv ? P->dinv : s->dinv;
    // a reordered system solves (P A P^T)(P x) = P b in its internal order
    if (s->perm) {
        int rc;
        if ((rc = to_internal_f64_2(s, b, s->bperm, x, s->xperm, st))) return rc;
    }
    a.b = s->perm ? s->bperm : b;
    a.x = s->perm ? s->xperm : x;
    a.r = s->r;
    a.p0 = s->p;
    a.p1 = s->p2;
    a.w = s->w;
    a.y = (uint32_t *)s->y;
    a.z = (uint32_t *)s->z;
    a.part_rr = s->part;
    a.part_rz = s->part + s->npart;
    a.part_pw = s->part + 2 * (size_t)s->npart;
    a.part_bb = s->part + 3 * (size_t)s->npart;
    a.sp_rz = s->sync_part;
    a.sp_pw = s->sync_part + s->npart;
    a.sp_rr = s->sync_part + 2 * (size_t)s->npart;
    a.sp_rz2 = s->sync_part + 3 * (size_t)s->npart;
    a.scal = s->scal;
    a.hist = hist;
    a.coef = coef;
    a.ctrl = s->ctrl;
    a.tol2 = tol * tol;
    if (P->kind == LPCG_PC_LLT && e2_path(s)) {  // the factor's values in the pair's ELL slots
        const int nmax = std::max(s->n - s->two_level_p, s->two_level_p);
        k_e2_pack<<<(nmax + 255) / 256, 256, 0, st>>>(s->n, s->two_level_p, s->e2_ws, s->e2_wp, s->e2_spos,
                                                      s->e2_sdpos, s->e2_ppos, s->e2_pdpos, P->l_val, P->ut_val,
                                                      s->e2_sval, s->e2_sdiag, s->e2_pval, s->e2_pdiag);
        LPCG_LAUNCH_CHECK();
    }
    if (P->kind == LPCG_PC_LLT) {  // the factor's values in the layouts of the single-workgroup and blocked modes
        for (int d = 0; d < 2; ++d) {
            int rc = LPCG_OK;
            if (s->trsv[d].mode == 2) rc = lo_prepare(s, d, P->l_val, P->ut_val, st);
            if (s->trsv[d].mode == 3) {
                if ((rc = blk_prepare(s, d, s->trsv[d].blk, s->trsv[d].runs)) ||
                    (rc = blk_pack(s, d, P->l_val, P->ut_val, st)))
                    return rc;
                rc = blk_set_lds(s, d);
            }
            if (rc) return rc;
        }
        a.blk_f = BlkSched{s->blk_brow[0], s->blk_bch[0], reinterpret_cast<const int2 *>(s->blk_ch[0]),
                           s->blk_rec[0], s->blk_nb[0], s->blk_B[0], s->blk_chmax[0], s->blk_lsh[0], s->blk_D[0]};
        a.blk_b = BlkSched{s->blk_brow[1], s->blk_bch[1], reinterpret_cast<const int2 *>(s->blk_ch[1]),
                           s->blk_rec[1], s->blk_nb[1], s->blk_B[1], s->blk_chmax[1], s->blk_lsh[1], s->blk_D[1]};
    }
    if (P->kind == LPCG_PC_JACOBI && !P->dinv) {
        int rc = lpcg_jacobi(s, s->dinv, st);
        if (rc) return rc;
    }
    return LPCG_OK;
}

// State of the timed product launches: not done, iteration 1 (so the kernel
// takes p = z + beta p_prev with the gathers of both), beta = 1/2.
__global__ void k_product_state(Args a) {
    if (threadIdx.x == 0) {
        a.ctrl[C_DONE] = 0;
        a.ctrl[C_IT] = 1;
        a.scal[S_BETA] = 0.5;
        a.scal[S_RZ0] = 1.0;
    }
}

}  // namespace

// Duration of the PCG's product kernel (p = z + beta p_prev, w = A p and the
// p.w partials) with G lanes per row on `blocks` blocks, or LDS-staged with
// R > 0 rows per block (windows prepared for R), or in the ELL form for
// G = 1 (built with the pattern): the median over three batches of reps
// back-to-back launches, after a warm-up batch.  Runs on the system's work
// vectors with z = p_prev = 1 and A's FP32 values; overwrites z, both search
// directions, w and the control words.  The autotuner ranks its SpMV
// candidates with it.
int time_pcg_product(lpcg_system *s, int G, int blocks, int R, int reps, double &us, hipStream_t st) {
    if (G == 1 && s->ea_w == 0) {
        set_error("SpMV: no ELL form for this pattern");
        return LPCG_EINVAL;
    }
    Args a{};
    a.n = s->n;
    a.maxit = 1 << 30;
    a.kind = LPCG_PC_LLT;
    a.rp = s->rowptr;
    a.ci = s->colind;
    a.v32 = s->val32;
    a.z = (uint32_t *)s->z;
    a.p0 = s->p;
    a.p1 = s->p2;
    a.w = s->w;
    a.part_pw = s->part + 2 * (size_t)s->npart;  // the kernel stores its p.w partials there
    a.np_pw = product_grid(s);
    a.scal = s->scal;
    a.ctrl = s->ctrl;
    const int fb = (s->n + 255) / 256;
    k_fill_u32<<<fb, 256, 0, st>>>(s->n, a.z, 0x3f800000u);
    k_fill_u32<<<fb, 256, 0, st>>>(s->n, (uint32_t *)s->p, 0x3f800000u);
    k_fill_u32<<<fb, 256, 0, st>>>(s->n, (uint32_t *)s->p2, 0x3f800000u);
    LPCG_LAUNCH_CHECK();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    LPCG_HIP(hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        LPCG_HIP(he);
    }
    const size_t lds = sizeof(float) * (size_t)std::max(1, s->spmv_wmax);
    const int nb = R > 0 ? (s->n + R - 1) / R : blocks;
    // The product no longer changes its own control state (its p.w partials
    // are reduced by the next launch), so after one state preset the
    // candidate is launched back to back: `reps` launches between two events
    // per batch, and the median over three batches after a warm-up one.  A
    // profiler's per-launch cost then adds alike to every candidate instead
    // of swamping one launch's time.
    k_product_state<<<1, 64, 0, st>>>(a);
    auto launch = [&]() {
        if (G == 1) {
            launch_spmv_pw_e<LPCG_PC_LLT>(s, a, st);
        } else if (R > 0) {
            switch (G) {
                case 4: k_spmv_pw_st<4, LPCG_PC_LLT><<<nb, VT, lds, st>>>(a, R, s->spmv_win); break;
                case 8: k_spmv_pw_st<8, LPCG_PC_LLT><<<nb, VT, lds, st>>>(a, R, s->spmv_win); break;
                case 16: k_spmv_pw_st<16, LPCG_PC_LLT><<<nb, VT, lds, st>>>(a, R, s->spmv_win); break;
                case 32: k_spmv_pw_st<32, LPCG_PC_LLT><<<nb, VT, lds, st>>>(a, R, s->spmv_win); break;
                default: k_spmv_pw_st<64, LPCG_PC_LLT><<<nb, VT, lds, st>>>(a, R, s->spmv_win); break;
            }
        } else {
            switch (G) {
                case 4: k_spmv_pw<4, LPCG_PC_LLT><<<nb, VT, 0, st>>>(a); break;
                case 8: k_spmv_pw<8, LPCG_PC_LLT><<<nb, VT, 0, st>>>(a); break;
                case 16: k_spmv_pw<16, LPCG_PC_LLT><<<nb, VT, 0, st>>>(a); break;
                case 32: k_spmv_pw<32, LPCG_PC_LLT><<<nb, VT, 0, st>>>(a); break;
                default: k_spmv_pw<64, LPCG_PC_LLT><<<nb, VT, 0, st>>>(a); break;
            }
        }
    };
    std::vector<float> t;
    hipError_t e = hipGetLastError();
    for (int batch = 0; batch <= 3 && e == hipSuccess; ++batch) {
        if ((e = hipEventRecord(e0, st)) != hipSuccess) break;
        for (int r = 0; r < reps; ++r) launch();
        if ((e = hipGetLastError()) != hipSuccess) break;
        if ((e = hipEventRecord(e1, st)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess) break;
        float ms = 0;
        if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
        if (batch > 0) t.push_back(ms / reps);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    LPCG_HIP(e);
    std::sort(t.begin(), t.end());
    us = 1e3 * (double)t[t.size() / 2];
    return LPCG_OK;
}

}  // namespace lpcg

using namespace lpcg;

extern "C" int lpcg_pcg_solve(lpcg_system *s, const lpcg_precond *P, const double *b, double *x,
                              const lpcg_solve_opts *opts, lpcg_result *res, double *hist, double *coef,
                              hipStream_t st) {
    if (!s || !P || !b || !x || !opts || !res || !(opts->tol >= 0)) {
        set_error("lpcg_pcg_solve: invalid arguments");
        return LPCG_EINVAL;
    }
    if (P->kind == LPCG_PC_LLT && (!P->l_val || !P->ut_val)) {
        set_error("lpcg_pcg_solve: LLT preconditioner needs l_val and ut_val");
        return LPCG_EINVAL;
    }
    if (P->kind != LPCG_PC_LLT && P->kind != LPCG_PC_JACOBI && P->kind != LPCG_PC_NONE) {
        set_error("lpcg_pcg_solve: unknown preconditioner kind %d", P->kind);
        return LPCG_EINVAL;
    }
    Args a{};
    {
        const int rc = build_args(s, P, b, x, opts->tol, opts->maxit, hist, coef, a, st);
        if (rc) return rc;
    }

    res->iters = 0;
    res->restarts = 0;
    res->status = LPCG_OK;
    int iters = 0, status = LPCG_OK;
    const int maxit0 = a.maxit;
    int first = 0;
    double rate = 0;
    bool true_ready = false;
    for (int attempt = 0;; ++attempt) {
        int rc;
        if (P->kind == LPCG_PC_LLT)
            rc = run_solve<LPCG_PC_LLT>(s, a, *opts, first, iters, status, rate, true_ready, st);
        else if (P->kind == LPCG_PC_JACOBI)
            rc = run_solve<LPCG_PC_JACOBI>(s, a, *opts, first, iters, status, rate, true_ready, st);
        else rc = run_solve<LPCG_PC_NONE>(s, a, *opts, first, iters, status, rate, true_ready, st);
        if (rc != LPCG_OK) return rc;
        if (!true_ready) {  // FP64 true residual; the same readback brings the recursive ||r||^2
            k_true_res<<<s->vec_blocks, VT, 0, st>>>(a);
            k_true_fin<<<1, VT, 0, st>>>(a);
            LPCG_LAUNCH_CHECK();
            LPCG_HIP(hipMemcpyAsync(s->h_scal, s->scal, sizeof(double) * S_NSCAL, hipMemcpyDeviceToHost, st));
            LPCG_HIP(hipStreamSynchronize(st));
        }
        const double truerel = sqrt(s->h_scal[S_TRUE] / s->h_scal[S_BB]);
        res->relres_rec = sqrt(s->h_scal[S_RR] / s->h_scal[S_BB]);
        res->relres_true = truerel;
        if (status == LPCG_OK && truerel > opts->tol && attempt < opts->max_restarts &&
            iters < maxit0) {
            res->restarts = attempt + 1;
            a.maxit = std::max(1, maxit0 - iters);
            first = restart_chunk(truerel * truerel, a.tol2, rate);
            continue;
        }
        break;
    }
    res->iters = iters;
    res->status = status;
    if (s->perm) {
        int rc = from_internal_f64(s, s->xperm, x, st);
        if (rc) return rc;
        LPCG_HIP(hipStreamSynchronize(st));
    }
    if (status == LPCG_ENOTCONV) set_error("pcg: no convergence within maxit");
    if (status == LPCG_EBREAKDOWN) set_error("pcg: breakdown (p.Ap <= 0 or non-finite)");
    return status;
}

extern "C" int32_t lpcg_next_chunk(int32_t it, float res, int32_t prev_it, float prev_res, double tol,
                                   int32_t maxit, int32_t *predicted_final) {
    ChunkPlan c;
    c.prev_it = prev_it;
    c.prev_res = prev_res;
    bool fin = false;
    const int n = next_chunk(it, res, tol * tol, maxit, c, fin);
    if (predicted_final) *predicted_final = fin ? 1 : 0;
    return n;
}

// Extreme eigenvalues of the CG-Lanczos tridiagonal T_k of the preconditioned
// operator (appendix "Condition Number Comparison"): T_ii = 1/alpha_i +
// beta_{i-1}/alpha_{i-1}, T_i,i+1 = sqrt(beta_i)/alpha_i.  Each extreme is
// found by bisection on the Sturm count (number of eigenvalues below x) inside
// the Gershgorin interval.
namespace lpcg {
namespace {

struct EvPair {
    hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
    ~EvPair() {
        for (hipEvent_t &x : e)
            if (x) (void)hipEventDestroy(x);
    }
};

template <int KIND>
int time_parts(lpcg_system *s, const Args &a, int reps, double *out_us, hipStream_t st) {
    EvPair ev;
    for (hipEvent_t &x : ev.e) LPCG_HIP(hipEventCreate(&x));
    k_setup<KIND><<<s->vec_blocks, VT, 0, st>>>(a);
    k_setup_scal<KIND><<<1, VT, 0, st>>>(a);
    LPCG_LAUNCH_CHECK();
    double tot[3] = {0, 0, 0};
    for (int r = 0; r <= reps; ++r) {  // the first round warms up
        int rc;
        LPCG_HIP(hipEventRecord(ev.e[0], st));
        if ((rc = enqueue_apply<KIND>(s, a, st))) return rc;
        LPCG_HIP(hipEventRecord(ev.e[1], st));
        if ((rc = enqueue_spmv<KIND>(s, a, st))) return rc;
        LPCG_HIP(hipEventRecord(ev.e[2], st));
        if ((rc = enqueue_xr<KIND>(s, a, st))) return rc;
        LPCG_HIP(hipEventRecord(ev.e[3], st));
        LPCG_HIP(hipEventSynchronize(ev.e[3]));
        if (r == 0) continue;
        for (int k = 0; k < 3; ++k) {
            float ms = 0;
            LPCG_HIP(hipEventElapsedTime(&ms, ev.e[k], ev.e[k + 1]));
            tot[k] += ms;
        }
    }
    for (int k = 0; k < 3; ++k) out_us[k] = 1e3 * tot[k] / reps;
    if (KIND != LPCG_PC_LLT) out_us[0] = 0.0;  // no application kernel
    if (KIND == LPCG_PC_LLT && e2_path(s)) out_us[2] = 0.0;  // the update runs in the application
    return LPCG_OK;
}

}  // namespace
}  // namespace lpcg

extern "C" int lpcg_time_pcg_kernels(lpcg_system *s, const lpcg_precond *P, const double *b, int32_t reps,
                                     double *out_us, hipStream_t st) {
    if (!s || !P || !b || reps <= 0 || !out_us || (P->kind == LPCG_PC_LLT && (!P->l_val || !P->ut_val)) ||
        (P->kind != LPCG_PC_LLT && P->kind != LPCG_PC_JACOBI && P->kind != LPCG_PC_NONE)) {
        set_error("lpcg_time_pcg_kernels: invalid arguments");
        return LPCG_EINVAL;
    }
    // x = 0 in a work vector; tolerance 0 so that the iterations never stop
    double *x0 = s->t64c;
    LPCG_HIP(hipMemsetAsync(x0, 0, sizeof(double) * (size_t)s->n, st));
    Args a{};
    int rc = build_args(s, P, b, x0, 0.0, 1 << 30, nullptr, nullptr, a, st);
    if (rc) return rc;
    if (P->kind == LPCG_PC_LLT) rc = time_parts<LPCG_PC_LLT>(s, a, reps, out_us, st);
    else if (P->kind == LPCG_PC_JACOBI) rc = time_parts<LPCG_PC_JACOBI>(s, a, reps, out_us, st);
    else rc = time_parts<LPCG_PC_NONE>(s, a, reps, out_us, st);
    if (rc) return rc;
    LPCG_HIP(hipStreamSynchronize(st));
    return LPCG_OK;
}

extern "C" int lpcg_lanczos_extremes(const double *coef, int32_t k, double *lmin, double *lmax) {
    if (!coef || k < 1 || !lmin || !lmax) {
        set_error("lpcg_lanczos_extremes: invalid arguments");
        return LPCG_EINVAL;
    }
    std::vector<double> d(k), e2(k, 0.0), e(k, 0.0);
    for (int i = 0; i < k; ++i) {
        const double al = coef[2 * (i + 1)];
        if (!(al > 0) || !std::isfinite(al)) {
            set_error("lpcg_lanczos_extremes: alpha_%d = %g is not positive", i + 1, al);
            return LPCG_EINVAL;
        }
        d[i] = 1.0 / al;
        if (i > 0) d[i] += coef[2 * i + 1] / coef[2 * i];
        if (i + 1 < k) {
            const double be = coef[2 * (i + 1) + 1];
            e[i] = std::sqrt(std::max(be, 0.0)) / al;
            e2[i] = e[i] * e[i];
        }
    }
    double lo = d[0], hi = d[0];
    for (int i = 0; i < k; ++i) {
        const double r = (i > 0 ? e[i - 1] : 0.0) + (i + 1 < k ? e[i] : 0.0);
        lo = std::min(lo, d[i] - r);
        hi = std::max(hi, d[i] + r);
    }
    auto below = [&](double x) {  // eigenvalues of T smaller than x
        int c = 0;
        double q = 1.0;
        for (int i = 0; i < k; ++i) {
            q = d[i] - x - (i > 0 ? e2[i - 1] / q : 0.0);
            if (q == 0.0) q = -1e-300;
            if (q < 0) ++c;
        }
        return c;
    };
    auto kth = [&](int idx) {  // idx-th smallest eigenvalue (0-based)
        double a = lo, b = hi;
        for (int it = 0; it < 200 && b - a > 1e-15 * std::max(std::fabs(a), std::fabs(b)); ++it) {
            const double m = 0.5 * (a + b);
            if (below(m) > idx) b = m;
            else a = m;
        }
        return 0.5 * (a + b);
    };
    *lmin = kth(0);
    *lmax = kth(k - 1);
    return LPCG_OK;
}
