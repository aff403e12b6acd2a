// Batched PCG and FP64 iterative refinement.
//
// A batch is a block-diagonal system of independent SPD systems analysed
// once (lpcg_analyze with sys_rowptr).  lpcg_pcg_solve_batched runs one PCG
// (Appendix algorithm "PCG") per system: every system has its own alpha,
// beta, r.z, residual test, iteration count and status, and all systems
// advance in the same launches until every one has converged, hit maxit or
// broken down.  A system that has finished stops updating.
//
// Vector kernels run one block per segment (at most kSegRows rows, never
// crossing a system), so every block works for exactly one system.  Dot
// products are fixed order: each block publishes its partial into a slot
// preset to a sentinel (the value is its own ready flag) and the last segment
// block of a system sums that system's slots in index order and updates the
// system's scalars.  The substitutions with L and L^T run over the whole batch
// with the configured kernels (rows of finished systems recompute the same
// values, since their r no longer changes).
//
// lpcg_pcg_solve_ir wraps the batched solver in an FP64 refinement loop:
// r = b - A x in FP64, an inner FP32 PCG on A d = r to tol_inner, x += d,
// until every system has ||b - A x|| <= tol ||b|| (systems already there get a
// zero right-hand side, so the inner solver leaves them alone).
#include <algorithm>
#include <cstring>

#include "device_util.h"
#include "kern_spmv.h"
#include "kern_sptrsv.h"
#include "lpcg_internal.h"

namespace lpcg {
namespace {

constexpr int BT = 256;                   // threads per segment block
constexpr int kRowsPerThread = kSegRows / BT;

// per-system FP64 scalars and control words (8 of each per system)
enum BScal : int { B_BB = 0, B_RZ = 1, B_RR = 2, B_ALPHA = 3, B_BETA = 4, B_TRUE = 5 };
enum BCtrl : int { B_DONE = 0, B_STATUS = 1, B_IT = 2, B_ITERS = 3 };

struct BArgs {
    int n, nseg, maxit, reset_y, reset_z;
    const int *seg_sys, *seg_row0, *seg_row1, *sys_seg_ptr;
    const int *rp, *ci;
    const float *v32;
    const double *v64;
    const float *dinv;
    const double *b;
    double *x;
    float *r, *p0, *p1, *w;
    uint32_t *y, *z;
    double *sp0, *sp1, *sp2;  // published partial slots, one per segment
    double *bs;
    int *bc;
    int *ndone, *tickets;     // tickets[0], tickets[1]: forward, backward
    double tol2;
};

struct Seg {
    int sys, r0, r1;
    bool reducer;
};

// Segment of this block; `active` (uniform) is false when the system has
// finished.  The done flag of a system is raised only by its reducer after
// every segment of the system has published in that launch, so all blocks of
// a system in one launch read the same value.
__device__ __forceinline__ Seg segment(const BArgs &a, bool &active, bool check_done) {
    __shared__ int act;
    Seg g;
    g.sys = a.seg_sys[blockIdx.x];
    g.r0 = a.seg_row0[blockIdx.x];
    g.r1 = a.seg_row1[blockIdx.x];
    g.reducer = (int)blockIdx.x == a.sys_seg_ptr[g.sys + 1] - 1;
    if (threadIdx.x == 0) act = check_done ? (a.bc[8 * g.sys + B_DONE] == 0) : 1;
    __syncthreads();
    active = act != 0;
    return g;
}

// Sum of the system's published slots (reducer block only).
__device__ __forceinline__ double sys_sum(const BArgs &a, double *slots, const Seg &g, double *lds) {
    const int s0 = a.sys_seg_ptr[g.sys], s1 = a.sys_seg_ptr[g.sys + 1];
    return reduce_published<BT>(slots + s0, s1 - s0, lds);
}

__device__ __forceinline__ void finish_system(const BArgs &a, int sy, int status, int iters) {
    a.bc[8 * sy + B_DONE] = 1;
    a.bc[8 * sy + B_STATUS] = status;
    a.bc[8 * sy + B_ITERS] = iters;
    atomicAdd(a.ndone, 1);
}

// r = b - A x (FP64 product), ||b||^2, ||r||^2 and (Jacobi/none) r.z per
// system; presets of the dependency-driven substitutions; first test.
template <int KIND>
__global__ void __launch_bounds__(BT) kb_setup(BArgs a) {
    __shared__ double lds[BT / kWave];
    bool active;
    const Seg g = segment(a, active, false);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.tickets[0] = 0;
        a.tickets[1] = 0;
    }
    double bb = 0, rr = 0, rz = 0;
    for (int i = g.r0 + threadIdx.x; i < g.r1; i += BT) {
        double s = 0;
        for (int k = a.rp[i]; k < a.rp[i + 1]; ++k) s += a.v64[k] * a.x[a.ci[k]];
        const double bi = a.b[i];
        const float ri = (float)(bi - s);
        a.r[i] = ri;
        bb += bi * bi;
        rr += (double)ri * ri;
        if (KIND == LPCG_PC_JACOBI) rz += (double)ri * ri * a.dinv[i];
        if (KIND == LPCG_PC_NONE) rz += (double)ri * ri;
        if (KIND == LPCG_PC_LLT) {
            a.y[i] = kUnset;
            a.z[i] = kUnset;
        }
    }
    bb = block_sum<BT>(bb, lds);
    rr = block_sum<BT>(rr, lds);
    rz = block_sum<BT>(rz, lds);
    if (threadIdx.x == 0) {
        publish_partial(a.sp0, blockIdx.x, bb);
        publish_partial(a.sp1, blockIdx.x, rr);
        publish_partial(a.sp2, blockIdx.x, rz);
    }
    if (!g.reducer) return;
    const double bbt = sys_sum(a, a.sp0, g, lds);
    const double rrt = sys_sum(a, a.sp1, g, lds);
    const double rzt = sys_sum(a, a.sp2, g, lds);
    if (threadIdx.x == 0) {
        double *bs = a.bs + 8 * g.sys;
        int *bc = a.bc + 8 * g.sys;
        const double bbs = bbt > 0 ? bbt : 1.0;
        bs[B_BB] = bbs;
        bs[B_RR] = rrt;
        bs[B_RZ] = KIND == LPCG_PC_LLT ? 0.0 : rzt;
        bs[B_BETA] = 0.0;
        bc[B_IT] = 0;
        bc[B_ITERS] = 0;
        bc[B_STATUS] = LPCG_OK;
        bc[B_DONE] = 0;
        if (!(rrt > a.tol2 * bbs)) finish_system(a, g.sys, LPCG_OK, 0);
    }
}

// LLT: r.z per system after the substitutions, beta; rearms the tickets of
// the dependency-driven substitutions for the next iteration.
__global__ void __launch_bounds__(BT) kb_rz(BArgs a) {
    __shared__ double lds[BT / kWave];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.tickets[0] = 0;
        a.tickets[1] = 0;
    }
    bool active;
    const Seg g = segment(a, active, true);
    if (!active) return;
    double rz = 0;
    for (int i = g.r0 + threadIdx.x; i < g.r1; i += BT) rz += (double)a.r[i] * (double)__uint_as_float(a.z[i]);
    rz = block_sum<BT>(rz, lds);
    if (threadIdx.x == 0) publish_partial(a.sp2, blockIdx.x, rz);
    if (!g.reducer) return;
    const double t = sys_sum(a, a.sp2, g, lds);
    if (threadIdx.x == 0) {
        double *bs = a.bs + 8 * g.sys;
        const int it = a.bc[8 * g.sys + B_IT];
        bs[B_BETA] = it == 0 ? 0.0 : t / bs[B_RZ];
        bs[B_RZ] = t;
    }
}

template <int KIND>
__device__ __forceinline__ float bdir(const BArgs &a, int j, bool first, float beta, const float *__restrict__ pp) {
    float zj;
    if (KIND == LPCG_PC_LLT) zj = __uint_as_float(a.z[j]);
    else if (KIND == LPCG_PC_JACOBI) zj = a.dinv[j] * a.r[j];
    else zj = a.r[j];
    return first ? zj : __fmaf_rn(beta, pp[j], zj);
}

// p = z + beta p_prev, w = A p, p.w per system; alpha, breakdown, it += 1.
template <int G, int KIND>
__global__ void __launch_bounds__(BT) kb_spmv_pw(BArgs a) {
    __shared__ double lds[BT / kWave];
    bool active;
    const Seg g = segment(a, active, true);
    if (!active) return;
    const int it = a.bc[8 * g.sys + B_IT];
    const bool first = it == 0;
    const float beta = (float)a.bs[8 * g.sys + B_BETA];
    float *pn = (it & 1) ? a.p1 : a.p0;
    const float *pp = (it & 1) ? a.p0 : a.p1;
    const int sub = threadIdx.x % G;
    double pw = 0;
    for (int row = g.r0 + threadIdx.x / G; row < g.r1; row += BT / G) {
        float acc = 0.f;
        for (int k = a.rp[row] + sub; k < a.rp[row + 1]; k += G)
            acc += a.v32[k] * bdir<KIND>(a, a.ci[k], first, beta, pp);
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
        if (sub == 0) {
            const float pi = bdir<KIND>(a, row, first, beta, pp);
            pn[row] = pi;
            a.w[row] = acc;
            pw += (double)pi * (double)acc;
        }
    }
    pw = block_sum<BT>(pw, lds);
    if (threadIdx.x == 0) publish_partial(a.sp0, blockIdx.x, pw);
    if (!g.reducer) return;
    const double pwt = sys_sum(a, a.sp0, g, lds);
    if (threadIdx.x == 0) {
        double *bs = a.bs + 8 * g.sys;
        a.bc[8 * g.sys + B_IT] = it + 1;
        if (!(pwt > 0.0) || !isfinite(pwt) || !isfinite(bs[B_RZ])) finish_system(a, g.sys, LPCG_EBREAKDOWN, it + 1);
        else bs[B_ALPHA] = bs[B_RZ] / pwt;
    }
}

// x += alpha p, r -= alpha w, ||r||^2 (Jacobi/none: r.z) per system, presets
// of the dependency-driven substitutions; convergence test (and beta).
template <int KIND>
__global__ void __launch_bounds__(BT) kb_xr(BArgs a) {
    __shared__ double lds[BT / kWave];
    bool active;
    const Seg g = segment(a, active, true);
    if (!active) return;
    const int it = a.bc[8 * g.sys + B_IT];
    const float *p = ((it - 1) & 1) ? a.p1 : a.p0;
    const double alpha = a.bs[8 * g.sys + B_ALPHA];
    const float af = (float)alpha;
    double rr = 0, rz = 0;
    for (int i = g.r0 + threadIdx.x; i < g.r1; i += BT) {
        a.x[i] += alpha * (double)p[i];
        const float ri = a.r[i] - af * a.w[i];
        a.r[i] = ri;
        rr += (double)ri * ri;
        if (KIND == LPCG_PC_JACOBI) rz += (double)ri * ri * a.dinv[i];
        if (KIND == LPCG_PC_NONE) rz += (double)ri * ri;
        if (KIND == LPCG_PC_LLT) {
            if (a.reset_y) a.y[i] = kUnset;
            if (a.reset_z) a.z[i] = kUnset;
        }
    }
    rr = block_sum<BT>(rr, lds);
    if (KIND != LPCG_PC_LLT) rz = block_sum<BT>(rz, lds);
    if (threadIdx.x == 0) {
        publish_partial(a.sp1, blockIdx.x, rr);
        if (KIND != LPCG_PC_LLT) publish_partial(a.sp2, blockIdx.x, rz);
    }
    if (!g.reducer) return;
    const double rrt = sys_sum(a, a.sp1, g, lds);
    const double rzt = KIND != LPCG_PC_LLT ? sys_sum(a, a.sp2, g, lds) : 0.0;
    if (threadIdx.x == 0) {
        double *bs = a.bs + 8 * g.sys;
        bs[B_RR] = rrt;
        const bool conv = !(rrt > a.tol2 * bs[B_BB]);
        const bool bad = !isfinite(rrt);
        if (conv || bad || it >= a.maxit)
            finish_system(a, g.sys, conv ? LPCG_OK : bad ? LPCG_EBREAKDOWN : LPCG_ENOTCONV, it);
        if (KIND != LPCG_PC_LLT) {
            bs[B_BETA] = rzt / bs[B_RZ];
            bs[B_RZ] = rzt;
        }
    }
}

// ||b - A x||^2 per system (FP64 values), into bs[B_TRUE]; with `out` given
// also stores r = b - A x (FP64) for the refinement loop, and with `rel` the
// relative residual and the converged flag (rel <= tol).
__global__ void __launch_bounds__(BT) kb_true(BArgs a, double *out, double *rel, int *flag, double tol) {
    __shared__ double lds[BT / kWave];
    bool active;
    const Seg g = segment(a, active, false);
    double rr = 0, bb = 0;
    for (int i = g.r0 + threadIdx.x; i < g.r1; i += BT) {
        double s = 0;
        for (int k = a.rp[i]; k < a.rp[i + 1]; ++k) s += a.v64[k] * a.x[a.ci[k]];
        const double ri = a.b[i] - s;
        if (out) out[i] = ri;
        rr += ri * ri;
        bb += a.b[i] * a.b[i];
    }
    rr = block_sum<BT>(rr, lds);
    bb = block_sum<BT>(bb, lds);
    if (threadIdx.x == 0) {
        publish_partial(a.sp0, blockIdx.x, rr);
        publish_partial(a.sp1, blockIdx.x, bb);
    }
    if (!g.reducer) return;
    const double rrt = sys_sum(a, a.sp0, g, lds);
    const double bbt = sys_sum(a, a.sp1, g, lds);
    if (threadIdx.x == 0) {
        a.bs[8 * g.sys + B_TRUE] = rrt;
        if (rel) {
            const double rl = sqrt(rrt / (bbt > 0 ? bbt : 1.0));
            rel[g.sys] = rl;
            flag[g.sys] = rl <= tol ? 1 : 0;
        }
    }
}

// Refinement helpers: zero the right-hand side of converged systems; x += d.
__global__ void __launch_bounds__(BT) kb_mask_rhs(BArgs a, double *r, const int *flag) {
    const int sy = a.seg_sys[blockIdx.x];
    if (!flag[sy]) return;
    for (int i = a.seg_row0[blockIdx.x] + threadIdx.x; i < a.seg_row1[blockIdx.x]; i += BT) r[i] = 0.0;
}

__global__ void __launch_bounds__(BT) kb_axpy(int n, double *x, const double *d) {
    const int i = blockIdx.x * BT + threadIdx.x;
    if (i < n) x[i] += d[i];
}

__global__ void kb_zero_i32(int *p) { *p = 0; }

template <int KIND>
int enqueue_batch_iteration(const lpcg_system *s, const BArgs &a, const lpcg_precond *P, hipStream_t st) {
    const int nseg = s->nseg;
    if (KIND == LPCG_PC_LLT) {
        int rc = trsv_kernels(s, 0, s->trsv[0], P->l_val, P->ut_val, a.r, (float *)a.y, a.tickets, st);
        if (rc) return rc;
        rc = trsv_kernels(s, 1, s->trsv[1], P->l_val, P->ut_val, (const float *)a.y, (float *)a.z, a.tickets + 1,
                          st);
        if (rc) return rc;
        kb_rz<<<nseg, BT, 0, st>>>(a);
    }
    switch (s->spmv_group) {
        case 4: kb_spmv_pw<4, KIND><<<nseg, BT, 0, st>>>(a); break;
        case 8: kb_spmv_pw<8, KIND><<<nseg, BT, 0, st>>>(a); break;
        case 16: kb_spmv_pw<16, KIND><<<nseg, BT, 0, st>>>(a); break;
        case 32: kb_spmv_pw<32, KIND><<<nseg, BT, 0, st>>>(a); break;
        default: kb_spmv_pw<64, KIND><<<nseg, BT, 0, st>>>(a); break;
    }
    kb_xr<KIND><<<nseg, BT, 0, st>>>(a);
    LPCG_LAUNCH_CHECK();
    return LPCG_OK;
}

// One batched solve (internal numbering) of A x = b from the current x;
// adds the iterations of every system to iters[] and leaves status/relres in
// the per-system arrays.
template <int KIND>
int run_batch(lpcg_system *s, const BArgs &a, const lpcg_precond *P, const lpcg_solve_opts &o, hipStream_t st) {
    const int nseg = s->nseg;
    kb_zero_i32<<<1, 1, 0, st>>>(a.ndone);
    kb_setup<KIND><<<nseg, BT, 0, st>>>(a);
    LPCG_LAUNCH_CHECK();
    const int chunk = o.check_every > 0 ? o.check_every : 8;
    hipGraphExec_t exec = nullptr;
    if (o.use_graph) {
        // key: kernel arguments, configuration, factor and blocked-schedule
        // arrays (the graph holds the pointers it was captured with)
        std::vector<unsigned char> key(sizeof(BArgs) + 16 * sizeof(int) + 4 * sizeof(void *));
        memcpy(key.data(), &a, sizeof(BArgs));
        const int extra[16] = {KIND, chunk, s->trsv[0].mode, s->trsv[0].waves, s->trsv[0].backoff, s->trsv[0].stride,
                               s->trsv[1].mode, s->trsv[1].waves, s->trsv[1].backoff, s->trsv[1].stride,
                               s->trsv[0].blk, s->trsv[1].blk, s->trsv[0].runs, s->trsv[1].runs,
                               s->blk_nb[0], s->blk_nb[1]};
        memcpy(key.data() + sizeof(BArgs), extra, sizeof(extra));
        const void *vals[4] = {P->l_val, P->ut_val, s->blk_rec[0], s->blk_rec[1]};
        memcpy(key.data() + sizeof(BArgs) + sizeof(extra), vals, sizeof(vals));
        if (s->bgraph_exec && s->bgraph_key == key) {
            exec = s->bgraph_exec;
        } else {
            if (s->bgraph_exec) {
                hipGraphExecDestroy(s->bgraph_exec);
                s->bgraph_exec = nullptr;
            }
            if (!s->cap_stream) LPCG_HIP(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
            hipGraph_t graph = nullptr;
            LPCG_HIP(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
            int rc = LPCG_OK;
            for (int c = 0; c < chunk && rc == LPCG_OK; ++c) rc = enqueue_batch_iteration<KIND>(s, a, P, s->cap_stream);
            hipError_t e = hipStreamEndCapture(s->cap_stream, &graph);
            if (rc != LPCG_OK) {
                if (graph) hipGraphDestroy(graph);
                return rc;
            }
            LPCG_HIP(e);
            hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            hipGraphDestroy(graph);
            LPCG_HIP(ie);
            s->bgraph_exec = exec;
            s->bgraph_key = key;
        }
    }
    for (int guard = 0;; ++guard) {
        // all done already (e.g. zero right-hand sides)?
        LPCG_HIP(hipMemcpyAsync(s->h_ctrl, s->ctrl, sizeof(int) * C_NCTRL, hipMemcpyDeviceToHost, st));
        LPCG_HIP(hipStreamSynchronize(st));
        if (s->h_ctrl[C_NDONE] >= s->nsys) break;
        if (guard > a.maxit / std::max(1, chunk) + 4) {
            set_error("batched pcg: systems still running after maxit");
            return LPCG_EHIP;
        }
        if (exec) {
            LPCG_HIP(hipGraphLaunch(exec, st));
        } else {
            for (int c = 0; c < chunk; ++c) {
                int rc = enqueue_batch_iteration<KIND>(s, a, P, st);
                if (rc) return rc;
            }
        }
    }
    return LPCG_OK;
}

int batch_solve_internal(lpcg_system *s, const lpcg_precond *P, const double *b, double *x,
                         const lpcg_solve_opts &o, double tol, std::vector<lpcg_result> &res, hipStream_t st) {
    BArgs a{};
    a.n = s->n;
    a.nseg = s->nseg;
    a.maxit = o.maxit > 0 ? o.maxit : s->n;
    a.reset_y = s->trsv[0].mode == 0 || s->trsv[0].mode == 3;
    a.reset_z = s->trsv[1].mode == 0 || s->trsv[1].mode == 3;
    a.seg_sys = s->seg_sys;
    a.seg_row0 = s->seg_row0;
    a.seg_row1 = s->seg_row1;
    a.sys_seg_ptr = s->sys_seg_ptr;
    a.rp = s->rowptr;
    a.ci = s->colind;
    a.v32 = s->val32;
    a.v64 = s->val64;
    a.dinv = P->dinv ? P->dinv : s->dinv;
    a.b = b;
    a.x = x;
    a.r = s->r;
    a.p0 = s->p;
    a.p1 = s->p2;
    a.w = s->w;
    a.y = (uint32_t *)s->y;
    a.z = (uint32_t *)s->z;
    a.sp0 = s->sync_part;
    a.sp1 = s->sync_part + s->npart;
    a.sp2 = s->sync_part + 2 * (size_t)s->npart;
    a.bs = s->bscal;
    a.bc = s->bctrl;
    a.ndone = s->ctrl + C_NDONE;
    a.tickets = s->ctrl + C_TICKET_F;  // C_TICKET_B follows
    a.tol2 = tol * tol;
    const int nsys = s->nsys;
    std::vector<double> hb(8 * (size_t)nsys);
    std::vector<int> hc(8 * (size_t)nsys);
    res.assign(nsys, lpcg_result{});
    const int maxit0 = a.maxit;
    for (int attempt = 0;; ++attempt) {
        int rc;
        if (P->kind == LPCG_PC_LLT) rc = run_batch<LPCG_PC_LLT>(s, a, P, o, st);
        else if (P->kind == LPCG_PC_JACOBI) rc = run_batch<LPCG_PC_JACOBI>(s, a, P, o, st);
        else rc = run_batch<LPCG_PC_NONE>(s, a, P, o, st);
        if (rc) return rc;
        kb_true<<<s->nseg, BT, 0, st>>>(a, nullptr, nullptr, nullptr, 0.0);
        LPCG_LAUNCH_CHECK();
        LPCG_HIP(hipMemcpyAsync(hb.data(), s->bscal, sizeof(double) * hb.size(), hipMemcpyDeviceToHost, st));
        LPCG_HIP(hipMemcpyAsync(hc.data(), s->bctrl, sizeof(int) * hc.size(), hipMemcpyDeviceToHost, st));
        LPCG_HIP(hipStreamSynchronize(st));
        bool again = false;
        int used = 0;
        for (int sy = 0; sy < nsys; ++sy) {
            lpcg_result &r = res[sy];
            r.iters += hc[8 * sy + B_ITERS];
            used = std::max(used, r.iters);
            r.status = hc[8 * sy + B_STATUS];
            r.relres_rec = sqrt(hb[8 * sy + B_RR] / hb[8 * sy + B_BB]);
            r.relres_true = sqrt(hb[8 * sy + B_TRUE] / hb[8 * sy + B_BB]);
            if (r.status == LPCG_OK && r.relres_true > tol) again = true;
        }
        if (!again || attempt >= o.max_restarts || used >= maxit0) break;
        for (int sy = 0; sy < nsys; ++sy)
            if (res[sy].status == LPCG_OK && res[sy].relres_true > tol) res[sy].restarts = attempt + 1;
        a.maxit = std::max(1, maxit0 - used);
    }
    return LPCG_OK;
}

int check_precond(const lpcg_precond *P, const char *who) {
    if (P->kind == LPCG_PC_LLT && (!P->l_val || !P->ut_val)) {
        set_error("%s: LLT preconditioner needs l_val and ut_val", who);
        return LPCG_EINVAL;
    }
    if (P->kind != LPCG_PC_LLT && P->kind != LPCG_PC_JACOBI && P->kind != LPCG_PC_NONE) {
        set_error("%s: unknown preconditioner kind %d", who, P->kind);
        return LPCG_EINVAL;
    }
    return LPCG_OK;
}

int prepare_precond(lpcg_system *s, const lpcg_precond *P, hipStream_t st) {
    if (P->kind == LPCG_PC_LLT)
        for (int d = 0; d < 2; ++d) {
            int rc = LPCG_OK;
            if (s->trsv[d].mode == 2) rc = lo_prepare(s, d, P->l_val, P->ut_val, st);
            if (s->trsv[d].mode == 3 && !(rc = blk_prepare(s, d, s->trsv[d].blk, s->trsv[d].runs)))
                rc = blk_pack(s, d, P->l_val, P->ut_val, st);
            if (rc) return rc;
        }
    if (P->kind == LPCG_PC_JACOBI && !P->dinv) return lpcg_jacobi(s, s->dinv, st);
    return LPCG_OK;
}

int worst_status(const std::vector<lpcg_result> &r) {
    for (const lpcg_result &x : r)
        if (x.status != LPCG_OK) return x.status;
    return LPCG_OK;
}

}  // namespace
}  // namespace lpcg

using namespace lpcg;

extern "C" int lpcg_pcg_solve_batched(lpcg_system *s, const lpcg_precond *P, const double *b, double *x,
                                      const lpcg_solve_opts *opts, lpcg_result *res, hipStream_t st) {
    if (!s || !P || !b || !x || !opts || !res || !(opts->tol >= 0)) {
        set_error("lpcg_pcg_solve_batched: invalid arguments");
        return LPCG_EINVAL;
    }
    int rc = check_precond(P, "lpcg_pcg_solve_batched");
    if (rc || (rc = prepare_precond(s, P, st))) return rc;
    if (s->perm) {
        if ((rc = to_internal_f64(s, b, s->bperm, st)) || (rc = to_internal_f64(s, x, s->xperm, st))) return rc;
    }
    std::vector<lpcg_result> r;
    rc = batch_solve_internal(s, P, s->perm ? s->bperm : b, s->perm ? s->xperm : x, *opts, opts->tol, r, st);
    if (rc) return rc;
    if (s->perm) {
        if ((rc = from_internal_f64(s, s->xperm, x, st))) return rc;
        LPCG_HIP(hipStreamSynchronize(st));
    }
    std::copy(r.begin(), r.end(), res);
    const int status = worst_status(r);
    if (status == LPCG_ENOTCONV) set_error("batched pcg: a system did not converge within maxit");
    if (status == LPCG_EBREAKDOWN) set_error("batched pcg: breakdown in a system (p.Ap <= 0 or non-finite)");
    return status;
}

extern "C" int lpcg_pcg_solve_ir(lpcg_system *s, const lpcg_precond *P, const double *b, double *x, double tol,
                                 double tol_inner, int32_t max_outer, const lpcg_solve_opts *inner,
                                 lpcg_result *res, hipStream_t st) {
    if (!s || !P || !b || !x || !inner || !res || !(tol > 0) || !(tol_inner > 0) || max_outer < 1) {
        set_error("lpcg_pcg_solve_ir: invalid arguments");
        return LPCG_EINVAL;
    }
    int rc = check_precond(P, "lpcg_pcg_solve_ir");
    if (rc || (rc = prepare_precond(s, P, st))) return rc;
    const double *bi = b;
    double *xi = x;
    if (s->perm) {
        if ((rc = to_internal_f64(s, b, s->bperm, st)) || (rc = to_internal_f64(s, x, s->xperm, st))) return rc;
        bi = s->bperm;
        xi = s->xperm;
    }
    const int nsys = s->nsys;
    std::vector<lpcg_result> total(nsys, lpcg_result{});
    std::vector<double> rel(nsys);
    std::vector<int> flag(nsys);
    BArgs a{};
    a.n = s->n;
    a.nseg = s->nseg;
    a.seg_sys = s->seg_sys;
    a.seg_row0 = s->seg_row0;
    a.seg_row1 = s->seg_row1;
    a.sys_seg_ptr = s->sys_seg_ptr;
    a.rp = s->rowptr;
    a.ci = s->colind;
    a.v64 = s->val64;
    a.b = bi;
    a.x = xi;
    a.sp0 = s->sync_part;
    a.sp1 = s->sync_part + s->npart;
    a.bs = s->bscal;
    a.bc = s->bctrl;
    double *r64 = s->t64a, *d64 = s->t64b;
    lpcg_solve_opts io = *inner;
    io.tol = tol_inner;
    io.max_restarts = 0;
    for (int outer = 0;; ++outer) {
        kb_true<<<s->nseg, BT, 0, st>>>(a, r64, s->ir_rel, s->ir_flag, tol);
        LPCG_LAUNCH_CHECK();
        LPCG_HIP(hipMemcpyAsync(rel.data(), s->ir_rel, sizeof(double) * nsys, hipMemcpyDeviceToHost, st));
        LPCG_HIP(hipMemcpyAsync(flag.data(), s->ir_flag, sizeof(int) * nsys, hipMemcpyDeviceToHost, st));
        LPCG_HIP(hipStreamSynchronize(st));
        bool all = true;
        for (int sy = 0; sy < nsys; ++sy) {
            total[sy].relres_true = rel[sy];
            all = all && flag[sy];
        }
        if (all || outer >= max_outer) break;
        // inner FP32 PCG on A d = r (converged systems: r = 0, d = 0)
        kb_mask_rhs<<<s->nseg, BT, 0, st>>>(a, r64, s->ir_flag);
        LPCG_HIP(hipMemsetAsync(d64, 0, sizeof(double) * s->n, st));
        std::vector<lpcg_result> part;
        if ((rc = batch_solve_internal(s, P, r64, d64, io, tol_inner, part, st))) return rc;
        kb_axpy<<<(s->n + BT - 1) / BT, BT, 0, st>>>(s->n, xi, d64);
        LPCG_LAUNCH_CHECK();
        for (int sy = 0; sy < nsys; ++sy) {
            total[sy].iters += part[sy].iters;
            if (!flag[sy]) total[sy].restarts += 1;  // outer refinement steps
            if (part[sy].status == LPCG_EBREAKDOWN) total[sy].status = LPCG_EBREAKDOWN;
            total[sy].relres_rec = part[sy].relres_rec;
        }
    }
    for (int sy = 0; sy < nsys; ++sy)
        if (total[sy].status == LPCG_OK && !flag[sy]) total[sy].status = LPCG_ENOTCONV;
    if (s->perm) {
        if ((rc = from_internal_f64(s, s->xperm, x, st))) return rc;
    }
    LPCG_HIP(hipStreamSynchronize(st));
    std::copy(total.begin(), total.end(), res);
    const int status = worst_status(total);
    if (status == LPCG_ENOTCONV) set_error("refinement: a system missed tol after max_outer steps");
    if (status == LPCG_EBREAKDOWN) set_error("refinement: breakdown in an inner solve");
    return status;
}
