// Internal declarations of liblpcg (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "lpcg.h"

namespace lpcg {

// thread-local error message
void set_error(const char *fmt, ...);
int hip_fail(hipError_t e, const char *what, const char *file, int line);

// Blocks of the fixed-grid vector kernels.  Partial sums are written one per
// block, so the grid must stay fixed for the reduction order to be fixed.
constexpr int kVecThreads = 256;
constexpr int kMaxVecBlocks = 1024;
constexpr int kMaxSpmvBlocks = 2048;
constexpr int kEllMaxW = 8;  // longest row (stored entries) of the ELL forms
constexpr int kSpmvMaxWindow = 16384;  // inputs one block of the LDS-staged SpMV may stage (64 KB)
// Default substitution mode: level-synchronous up to this many levels.
constexpr int kLevelModeMaxLevels = 16;
// The autotuner tries level-synchronous launches up to this many levels.
constexpr int kLevelModeTuneLevels = 1024;
// Rows per segment (one block) of the batched solver's vector kernels.
constexpr int kSegRows = 1024;

// Layout of the small control words and FP64 scalars of a PCG solve.
enum Ctrl : int {
    C_DONE = 0,      // nonzero: every later kernel of the solve returns at once
    C_STATUS = 1,    // LPCG_OK / ENOTCONV / EBREAKDOWN
    C_IT = 2,        // products A p done so far (k of the algorithm)
    C_ITERS = 3,     // iteration count at exit
    C_TICKET_F = 4,  // work counter of the forward substitution
    C_TICKET_B = 5,  // work counter of the backward substitution
    C_TICKET_X = 6,  // spare work counter (standalone solves)
    C_MAXIT = 7,
    C_NDONE = 8,     // batched solve: systems finished
    C_PHASE = 9,     // fused red-black path: 0 before the solve's first application, 1 after
    C_RES = 10,      // ||r||^2 / ||b||^2 of the last recorded iteration (FP32 bits), for the host
    C_RES_IT = 11,   // the iteration C_RES belongs to
    C_RES0 = 12,     // ||r0||^2 / ||b||^2 (FP32 bits)
    C_NCTRL = 16
};
enum Scal : int {
    S_BB = 0,        // ||b||^2
    S_RZ0 = 1,       // r.z, parity 0
    S_RZ1 = 2,       // r.z, parity 1
    S_RR = 3,        // ||r||^2 at exit (recursive)
    S_TOL2 = 4,      // tol^2
    S_BETA = 5,
    S_TRUE = 6,      // ||b - A x||^2 (FP64 true residual)
    S_ALPHA = 7,     // alpha of the current iteration
    S_NSCAL = 16
};

// Configuration of one substitution direction: mode 0 = dependency driven
// (one launch; `waves` waves in blocks whose index is a multiple of `stride`,
// `backoff` sleep rounds between polls), mode 1 =
// level synchronous (one launch per level, `g` lanes per row), mode 2 = one
// workgroup walking all levels with block barriers, mode 3 = blocked (one
// wave per block of `blk` consecutive rows, in-block dependencies through
// LDS, `backoff` sleep rounds between polls of the others).
struct TrsvCfg {
    int mode = 0, waves = 0, backoff = 1, stride = 1, blk = 0, runs = 1;
};

}  // namespace lpcg

struct lpcg_system {
    int n = 0, nnz = 0, nnz_l = 0;
    int nlev_f = 0, nlev_b = 0, max_w_f = 0, max_w_b = 0;
    int nsys = 1;
    // pattern (device)
    int *rowptr = nullptr, *colind = nullptr, *erow = nullptr, *dpos = nullptr, *rev = nullptr;
    int *lrowptr = nullptr, *lcol = nullptr, *lsrc = nullptr;
    int *urowptr = nullptr, *ucol = nullptr, *u2l = nullptr;
    int *flevel = nullptr, *flev_ptr = nullptr, *flev_rows = nullptr;
    int *blevel = nullptr, *blev_ptr = nullptr, *blev_rows = nullptr;
    int *sys_rowptr = nullptr, *row_sys = nullptr;
    // row ordering (LPCG_ORDER_*): the system holds P A P^T with
    // perm[new] = original row, iperm[original] = new row and psrc[k'] = the
    // position in the caller's CSR of internal entry k'.  All three are null
    // for the natural ordering.
    int ordering = 0, ncolors = 0;
    int *perm = nullptr, *iperm = nullptr, *psrc = nullptr;
    double *bperm = nullptr, *xperm = nullptr;  // caller vectors in internal order
    std::vector<int> h_flev_ptr, h_blev_ptr, h_sys_rowptr;
    // level-ordered packed factor patterns (index 0: L rows in forward level
    // order, 1: U = L^T rows in backward level order): for level position q,
    // off-diagonal entries lo_ptr[q] .. lo_ptr[q+1] with columns lo_col and
    // positions lo_src in the CSR value array; lo_dsrc[q] = the diagonal's
    // position.  lo_val / lo_diag hold one factor's values in that order
    // (prepared per solve) for the single-workgroup substitution.
    int *lo_ptr[2] = {nullptr, nullptr}, *lo_col[2] = {nullptr, nullptr};
    int *lo_src[2] = {nullptr, nullptr}, *lo_dsrc[2] = {nullptr, nullptr};
    float *lo_val[2] = {nullptr, nullptr}, *lo_diag[2] = {nullptr, nullptr};
    // blocked substitution (mode 3), per direction: the schedule built for
    // block size blk_B[d] (0: none) with records of blk_W[d] dependencies
    // (kern_sptrsv.h describes the arrays); blk_vsrc maps record values to
    // positions in the factor's value array
    int blk_B[2] = {0, 0}, blk_W[2] = {0, 0}, blk_nb[2] = {0, 0}, blk_chmax[2] = {0, 0};
    // banded blocks: blk_K[d] runs of 2^blk_lsh[d] rows, blk_D[d] apart (K = 1: consecutive rows)
    int blk_K[2] = {1, 1}, blk_lsh[2] = {30, 30}, blk_D[2] = {0, 0};
    int *blk_brow[2] = {nullptr, nullptr}, *blk_bch[2] = {nullptr, nullptr}, *blk_ch[2] = {nullptr, nullptr};
    int *blk_rec[2] = {nullptr, nullptr}, *blk_vsrc[2] = {nullptr, nullptr};
    // values (device)
    double *val64 = nullptr;
    float *val32 = nullptr;
    double *diag64 = nullptr;
    // solver work vectors (device)
    float *r = nullptr, *p = nullptr, *w = nullptr, *z = nullptr, *y = nullptr, *dinv = nullptr;
    float *p2 = nullptr;  // second search-direction buffer (p alternates by iteration parity)
    double *t64a = nullptr, *t64b = nullptr, *t64c = nullptr;  // FP64 work vectors (loss)
    double *sys_tmp = nullptr;                                  // [2 * nsys] per-system scalars
    double *part = nullptr;      // partial sums (3 x max(kMaxVecBlocks, chunks))
    int npart = 0;               // stride between the partial arrays
    double *sync_part = nullptr; // 4 x npart published partials (slots preset to kPartUnset):
                                 // backward r.z, SpMV p.w, update ||r||^2 and r.z
    double *scal = nullptr;      // FP64 scalars (Scal)
    int *ctrl = nullptr;         // control words (Ctrl)
    int *h_ctrl = nullptr;       // pinned host mirror of ctrl
    double *h_scal = nullptr;    // pinned host mirror of scal
    int vec_blocks = 1;          // grid of the fixed-grid vector kernels
    int spmv_blocks = 1;         // grid of the fused SpMV + p.w kernel
    int spmv_group = 8;          // lanes per row in SpMV
    // LDS-staged SpMV (kern_spmv.h): spmv_rows = R > 0 rows per block, each
    // block staging its input over the window spmv_win[2b], spmv_win[2b + 1]
    // (device; computed for spmv_win_rows); 0 = the gather form
    int spmv_rows = 0;
    int spmv_win_rows = 0;
    int spmv_wmax = 0;           // longest window (elements) for spmv_win_rows
    int *spmv_win = nullptr;     // [2 * kMaxSpmvBlocks]
    lpcg::TrsvCfg trsv[2];       // forward (L) and backward (L^T) substitution
    lpcg::TrsvCfg ic0_cfg;       // IC(0): the fastest dependency-driven forward configuration
    bool ic0_tuned = false;
    int trsv_g = 8;              // lanes per row of the level-synchronous kernel
    // Two-level structure: the forward level 0 is exactly rows [0, two_level_p)
    // (no strictly-lower entries) and every other row is level 1 (0: not so).
    // Multicolour orderings of bipartite graphs (red-black grids) have it.
    int two_level_p = 0;
    // ELL forms (one row per lane; slot t of row i at t * rows + i, so a
    // wave's loads of one slot are contiguous; padding: value 0 at a valid
    // column) for patterns whose rows have at most kEllMaxW entries.  The
    // two-level pair: suffix rows [p, n) of L without the diagonal (e2_ws
    // slots, columns in the prefix) and prefix rows [0, p) of U = L^T without
    // the diagonal (e2_wp slots, columns in the suffix); *_pos = source
    // position in l_val / ut_val (-1: padding), *_dpos = the diagonal's.  The
    // values of one factor are packed per solve.  e2_ws = 0: not built.
    int e2_ws = 0, e2_wp = 0;
    int *e2_scol = nullptr, *e2_spos = nullptr, *e2_sdpos = nullptr;
    int *e2_pcol = nullptr, *e2_ppos = nullptr, *e2_pdpos = nullptr;
    float *e2_sval = nullptr, *e2_sdiag = nullptr, *e2_pval = nullptr, *e2_pdiag = nullptr;
    // A in ELL form (ea_w slots per row, the diagonal included; padding
    // column = the row itself), FP32 values packed with every value update.
    // ea_w = 0: not built.  spmv_ell: the PCG's product and the FP32 SpMV use
    // it (an autotuner candidate beside the gather and staged forms).
    int ea_w = 0;
    int *ea_col = nullptr, *ea_pos = nullptr;
    float *ea_val = nullptr;
    bool spmv_ell = false;
    // Row-aligned edge tiles of the network's fused inference pass: tile j
    // holds the whole rows gtile_row[j] .. gtile_row[j+1]-1, at most 32 stored
    // entries in all (0 tiles: some row has more than 32 entries).
    int *gtile_row = nullptr;
    int *gtile_e = nullptr;  // first stored entry of each tile's rows: rowptr[gtile_row[j]]
    int gtiles = 0;
    // batched solves: row segments of at most kSegRows rows that never cross
    // a system (one block each), the segment range of every system, and the
    // per-system FP64 scalars / control words
    int nseg = 0;
    int *seg_sys = nullptr, *seg_row0 = nullptr, *seg_row1 = nullptr, *sys_seg_ptr = nullptr;
    double *bscal = nullptr;  // [nsys * 8]
    int *bctrl = nullptr;     // [nsys * 8]
    double *ir_rel = nullptr; // [nsys] refinement: relative residual per system
    int *ir_flag = nullptr;   // [nsys] refinement: 1 = converged
    // Frobenius loss: CSR pattern of E = L L^T - A (built at the first call)
    int nnz_e = 0;
    int *erp = nullptr, *ecol = nullptr;
    double *eval = nullptr, *erowsq = nullptr;
    hipGraphExec_t bgraph_exec = nullptr;
    std::vector<unsigned char> bgraph_key;
    // cached iteration-chunk graph of the last PCG solve (captured on a
    // private stream, launched on the caller's)
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<unsigned char> graph_key;
    std::vector<void *> allocs;
};

#define LPCG_HIP(call)                                                               \
    do {                                                                             \
        hipError_t _e = (call);                                                      \
        if (_e != hipSuccess) return ::lpcg::hip_fail(_e, #call, __FILE__, __LINE__); \
    } while (0)

#define LPCG_LAUNCH_CHECK() LPCG_HIP(hipGetLastError())

namespace lpcg {
// Permutation of caller vectors (original numbering) to and from the
// system's internal order: to_internal: dst[r] = src[perm[r]];
// from_internal: dst[perm[r]] = src[r].  No-ops (plain copies are not made)
// when the system has the natural ordering; callers test s->perm first.
int to_internal_f64(const lpcg_system *s, const double *src, double *dst, hipStream_t st);
int to_internal_f64_2(const lpcg_system *s, const double *s0, double *d0, const double *s1, double *d1,
                      hipStream_t st);
int from_internal_f64(const lpcg_system *s, const double *src, double *dst, hipStream_t st);
int to_internal_f32(const lpcg_system *s, const float *src, float *dst, hipStream_t st);
int from_internal_f32(const lpcg_system *s, const float *src, float *dst, hipStream_t st);
// Substitution launches shared by the single and batched solvers (factor.hip).
struct TrsvCfg;
int trsv_kernels(const lpcg_system *s, int transpose, const TrsvCfg &c, const float *lval, const float *utval,
                 const float *rhs, float *y, int *ticket, hipStream_t st);
int lo_prepare(const lpcg_system *s, int transpose, const float *lval, const float *utval, hipStream_t st);
// Blocked mode: build (host, synchronous) the schedule of direction d for
// block size B in K runs (K = 1: consecutive rows); pack one factor's values
// into its records; free it.
int blk_prepare(lpcg_system *s, int d, int B, int K = 1);
int blk_pack(const lpcg_system *s, int d, const float *lval, const float *utval, hipStream_t st);
void blk_free(lpcg_system *s, int d);
void drop_graphs(lpcg_system *s);
// Pack A's FP32 values into the ELL form (no-op when not built).
int ell_pack_a(const lpcg_system *s, hipStream_t st);
// Duration (us, median of batches of back-to-back launches) of the PCG's
// product kernel for an SpMV candidate
// (pcg.hip; overwrites the solver's work vectors and control words).
int time_pcg_product(lpcg_system *s, int G, int blocks, int R, int reps, double &us, hipStream_t st);
}  // namespace lpcg
