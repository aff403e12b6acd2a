/*
 * lpcg_oracle.c -- plain, slow, serial FP64 reference for learned-preconditioner
 * PCG.  TEST INFRASTRUCTURE ONLY: nothing in the product library links or calls
 * this file; only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark load it.
 *
 * Every routine is the textbook definition written out, in the order of the
 * paper's notation, with no blocking, fusion or reordering:
 *   - graph/matrix duality (Method, "Learning Preconditioners"): the nonzeros of
 *     A are the directed edges; the lower triangle (i >= j) carries L.
 *   - PCG (Appendix, Algorithm "PCG"), preconditioner P = L L^T applied by a
 *     forward and a backward triangular substitution ("Solve P z = r").
 *   - IC(0) (the incomplete Cholesky baseline of the Experiments section):
 *     L on the pattern of tril(A) with (L L^T)_ij = A_ij on that pattern.
 *   - the data loss sum ||L L^T x - b||^2 (Method, equation loss_Ab) and its
 *     gradient with respect to the entries of L.
 *
 * The PCG optionally records its coefficients (coef[2k] = alpha_k,
 * coef[2k+1] = beta_k), from which the Lanczos tridiagonal of the
 * preconditioned operator follows (the condition-number estimate of the
 * appendix "Condition Number Comparison").
 *
 * All arrays are host arrays.  Indices are int32, CSR rows sorted ascending.
 * Build: gcc -O2 -ffp-contract=off -shared -fPIC (no FMA contraction, so every
 * product and sum is rounded exactly as written).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Patterns                                                                  */
/* ------------------------------------------------------------------------ */

/* Lower triangle of the pattern (entries with col <= row), in CSR order.
 * src[k] = position in A of the k-th L entry.  Returns nnz_L. */
int orc_lower_pattern(int n, const int *rowptr, const int *col,
                      int *lrowptr, int *lcol, int *src)
{
    int k = 0;
    lrowptr[0] = 0;
    for (int i = 0; i < n; ++i) {
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            if (col[p] <= i) {
                lcol[k] = col[p];
                src[k] = p;
                ++k;
            }
        }
        lrowptr[i + 1] = k;
    }
    return k;
}

/* Transpose of a CSR pattern with values (the explicit transpose: entry (i,j)
 * of the input becomes entry (j,i) of the output, rows sorted ascending).
 * tsrc[q] = position in the input of the q-th output entry. */
void orc_transpose(int n, const int *rowptr, const int *col,
                   int *trowptr, int *tcol, int *tsrc)
{
    int nnz = rowptr[n];
    int *cnt = (int *)calloc((size_t)n + 1, sizeof(int));
    for (int p = 0; p < nnz; ++p) cnt[col[p] + 1]++;
    for (int i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    memcpy(trowptr, cnt, sizeof(int) * ((size_t)n + 1));
    /* rows visited in ascending order, so each output row is filled with
     * ascending column indices */
    for (int i = 0; i < n; ++i) {
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int j = col[p];
            int q = cnt[j]++;
            tcol[q] = i;
            tsrc[q] = p;
        }
    }
    free(cnt);
}

/* rev[k] = position of entry (j,i) for entry k = (i,j); -1 if absent.
 * Returns the number of entries without a mirror (0 for a symmetric pattern). */
int orc_rev(int n, const int *rowptr, const int *col, int *rev)
{
    int missing = 0;
    for (int i = 0; i < n; ++i) {
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int j = col[p];
            rev[p] = -1;
            for (int q = rowptr[j]; q < rowptr[j + 1]; ++q) {
                if (col[q] == i) { rev[p] = q; break; }
            }
            if (rev[p] < 0) ++missing;
        }
    }
    return missing;
}

/* Forward levels of the lower-triangular DAG: level(i) = 0 if row i has no
 * strictly-lower entry, else 1 + max over strictly-lower columns j of level(j).
 * (Longest-path depth; rows in ascending order are a topological order.)
 * Returns the number of levels. */
int orc_levels_lower(int n, const int *lrowptr, const int *lcol, int *level)
{
    int nlev = 0;
    for (int i = 0; i < n; ++i) {
        int lv = 0;
        for (int p = lrowptr[i]; p < lrowptr[i + 1]; ++p) {
            int j = lcol[p];
            if (j < i && level[j] + 1 > lv) lv = level[j] + 1;
        }
        level[i] = lv;
        if (lv + 1 > nlev) nlev = lv + 1;
    }
    return nlev;
}

/* Backward levels for the solve with L^T, given the CSR of U = L^T (row i holds
 * columns j >= i): level(i) = 0 if no j > i, else 1 + max level(j). Rows are
 * visited in descending order (a topological order of that DAG). */
int orc_levels_upper(int n, const int *urowptr, const int *ucol, int *level)
{
    int nlev = 0;
    for (int i = n - 1; i >= 0; --i) {
        int lv = 0;
        for (int p = urowptr[i]; p < urowptr[i + 1]; ++p) {
            int j = ucol[p];
            if (j > i && level[j] + 1 > lv) lv = level[j] + 1;
        }
        level[i] = lv;
        if (lv + 1 > nlev) nlev = lv + 1;
    }
    return nlev;
}

/* Greedy (first-fit) colouring visiting rows in ascending order: colour(i)
 * is the smallest non-negative integer that no neighbour j < i (a strictly
 * lower entry of row i) already has.  Adjacent rows get different colours, so
 * in an ordering by colour the rows of one colour depend only on rows of
 * smaller colours.  Returns the number of colours. */
int orc_greedy_colors(int n, const int *lrowptr, const int *lcol, int *color)
{
    int ncol = 0;
    char *taken = (char *)calloc((size_t)n + 1, 1);
    for (int i = 0; i < n; ++i) {
        for (int p = lrowptr[i]; p < lrowptr[i + 1]; ++p)
            if (lcol[p] < i) taken[color[lcol[p]]] = 1;
        int c = 0;
        while (taken[c]) ++c;
        color[i] = c;
        if (c + 1 > ncol) ncol = c + 1;
        for (int p = lrowptr[i]; p < lrowptr[i + 1]; ++p)
            if (lcol[p] < i) taken[color[lcol[p]]] = 0;
    }
    free(taken);
    return ncol;
}

/* Level sets: rows grouped by level, levels ascending, rows ascending inside a
 * level.  lev_ptr[nlev+1], lev_rows[n]. */
void orc_level_sets(int n, const int *level, int nlev, int *lev_ptr, int *lev_rows)
{
    for (int s = 0; s <= nlev; ++s) lev_ptr[s] = 0;
    for (int i = 0; i < n; ++i) lev_ptr[level[i] + 1]++;
    for (int s = 0; s < nlev; ++s) lev_ptr[s + 1] += lev_ptr[s];
    int *fill = (int *)malloc(sizeof(int) * (size_t)(nlev + 1));
    memcpy(fill, lev_ptr, sizeof(int) * (size_t)(nlev + 1));
    for (int i = 0; i < n; ++i) lev_rows[fill[level[i]]++] = i;
    free(fill);
}

/* ------------------------------------------------------------------------ */
/* Products and substitutions                                                */
/* ------------------------------------------------------------------------ */

/* y = A x : y_i = sum_k val[k] * x[col[k]] over row i, in CSR order. */
void orc_spmv(int n, const int *rowptr, const int *col, const double *val,
              const double *x, double *y)
{
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) s += val[p] * x[col[p]];
        y[i] = s;
    }
}

/* Forward substitution L y = r, L lower CSR with the diagonal stored:
 * y_i = (r_i - sum_{j<i} L_ij y_j) / L_ii, rows in ascending order. */
void orc_trsv_lower(int n, const int *lrowptr, const int *lcol, const double *lval,
                    const double *r, double *y)
{
    for (int i = 0; i < n; ++i) {
        double s = r[i];
        double d = 0.0;
        for (int p = lrowptr[i]; p < lrowptr[i + 1]; ++p) {
            int j = lcol[p];
            if (j < i) s -= lval[p] * y[j];
            else d = lval[p];
        }
        y[i] = s / d;
    }
}

/* Backward substitution U z = y with U upper CSR (diagonal stored):
 * z_i = (y_i - sum_{j>i} U_ij z_j) / U_ii, rows in descending order.  Called
 * with U = L^T built by orc_transpose. */
void orc_trsv_upper(int n, const int *urowptr, const int *ucol, const double *uval,
                    const double *y, double *z)
{
    for (int i = n - 1; i >= 0; --i) {
        double s = y[i];
        double d = 0.0;
        for (int p = urowptr[i]; p < urowptr[i + 1]; ++p) {
            int j = ucol[p];
            if (j > i) s -= uval[p] * z[j];
            else d = uval[p];
        }
        z[i] = s / d;
    }
}

/* ------------------------------------------------------------------------ */
/* IC(0)                                                                     */
/* ------------------------------------------------------------------------ */

/* Incomplete Cholesky with zero fill on the pattern of tril(A):
 *   L_ij = (A_ij - sum_{k<j, k in S_i and S_j} L_ik L_jk) / L_jj   (j < i)
 *   L_ii = sqrt(A_ii - sum_{k<i} L_ik^2)
 * rows in ascending order.  aval: A's values on the lower pattern (same
 * positions as lcol).  shift: factor A + shift*diag(A) instead.
 * Returns 0, or (i+1) for the first row whose pivot is <= 0 or not finite. */
int orc_ic0(int n, const int *lrowptr, const int *lcol, const double *aval,
            double shift, double *lval)
{
    for (int i = 0; i < n; ++i) {
        int r0 = lrowptr[i], r1 = lrowptr[i + 1];
        for (int p = r0; p < r1; ++p) {
            int j = lcol[p];
            if (j < i) {
                /* sum over k in S_i intersect S_j with k < j (merge of the two
                 * ascending column lists) */
                double s = aval[p];
                int a = r0, b = lrowptr[j];
                while (a < r1 && b < lrowptr[j + 1]) {
                    int ka = lcol[a], kb = lcol[b];
                    if (ka >= j || kb >= j) break;
                    if (ka == kb) { s -= lval[a] * lval[b]; ++a; ++b; }
                    else if (ka < kb) ++a;
                    else ++b;
                }
                lval[p] = s / lval[lrowptr[j + 1] - 1];
            } else {
                double d = aval[p] * (1.0 + shift);
                for (int q = r0; q < p; ++q) d -= lval[q] * lval[q];
                if (!(d > 0.0) || !isfinite(d)) return i + 1;
                lval[p] = sqrt(d);
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* PCG (Appendix algorithm "PCG")                                            */
/* ------------------------------------------------------------------------ */

enum { ORC_PC_NONE = 0, ORC_PC_JACOBI = 1, ORC_PC_LLT = 2 };

typedef struct {
    int kind;
    /* ORC_PC_JACOBI */
    const double *diag;
    /* ORC_PC_LLT: L lower CSR and U = L^T upper CSR */
    const int *lrowptr, *lcol; const double *lval;
    const int *urowptr, *ucol; const double *uval;
} orc_precond;

static void apply_prec(int n, const orc_precond *P, const double *r, double *z, double *tmp)
{
    if (P->kind == ORC_PC_NONE) {
        for (int i = 0; i < n; ++i) z[i] = r[i];
    } else if (P->kind == ORC_PC_JACOBI) {
        for (int i = 0; i < n; ++i) z[i] = r[i] / P->diag[i];
    } else {
        orc_trsv_lower(n, P->lrowptr, P->lcol, P->lval, r, tmp);
        orc_trsv_upper(n, P->urowptr, P->ucol, P->uval, tmp, z);
    }
}

static double dot(int n, const double *a, const double *b)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Status codes shared in meaning (not in code) with the product library. */
enum { ORC_OK = 0, ORC_NOTCONV = 1, ORC_BREAKDOWN = 2 };

/* Solve A x = b.  x holds x0 on entry and the last iterate on exit.
 * Stops when ||r_k||_2 <= tol * ||b||_2 (relative reading of the algorithm's
 * epsilon).  *iters = number of products A p (k of the algorithm).
 * hist (optional, length maxit+1): ||r_k||_2 / ||b||_2 for k = 0..iters.
 * pvec (optional, n * (maxit+1)): the search directions p_1..p_k, for tests. */
int orc_pcg(int n, const int *rowptr, const int *col, const double *val,
            const double *b, double *x, const orc_precond *P, double tol, int maxit,
            int *iters, double *relres, double *hist, double *pvec, double *coef)
{
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *z = (double *)malloc(sizeof(double) * (size_t)n);
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    double *t = (double *)malloc(sizeof(double) * (size_t)n);
    int status = ORC_OK;
    int k = 0;
    double bnorm = sqrt(dot(n, b, b));
    if (bnorm == 0.0) bnorm = 1.0;

    /* r0 = b - A x0 */
    orc_spmv(n, rowptr, col, val, x, w);
    for (int i = 0; i < n; ++i) r[i] = b[i] - w[i];
    double rn = sqrt(dot(n, r, r));
    if (hist) hist[0] = rn / bnorm;
    if (!(rn > tol * bnorm)) {           /* already converged: no iteration */
        *iters = 0; *relres = rn / bnorm;
        free(r); free(z); free(p); free(w); free(t);
        return ORC_OK;
    }
    /* Solve P z0 = r0;  p1 = z0;  w = A p1;  alpha1 = r0.z0 / p1.w */
    apply_prec(n, P, r, z, t);
    for (int i = 0; i < n; ++i) p[i] = z[i];
    double rz = dot(n, r, z);
    while (1) {
        orc_spmv(n, rowptr, col, val, p, w);
        ++k;
        if (pvec) memcpy(pvec + (size_t)(k - 1) * n, p, sizeof(double) * (size_t)n);
        double pw = dot(n, p, w);
        if (!(pw > 0.0) || !isfinite(pw) || !isfinite(rz)) { status = ORC_BREAKDOWN; break; }
        double alpha = rz / pw;
        if (coef) coef[2 * k] = alpha;                  /* alpha_k */
        for (int i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
        for (int i = 0; i < n; ++i) r[i] = r[i] - alpha * w[i];
        rn = sqrt(dot(n, r, r));
        if (hist) hist[k] = rn / bnorm;
        if (!(rn > tol * bnorm)) break;                 /* while ||r_k|| > eps */
        if (k >= maxit) { status = ORC_NOTCONV; break; }
        apply_prec(n, P, r, z, t);                      /* Solve P z_k = r_k */
        double rz_new = dot(n, r, z);
        double beta = rz_new / rz;                      /* beta_k */
        if (coef) coef[2 * k + 1] = beta;
        for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        rz = rz_new;
    }
    *iters = k;
    *relres = rn / bnorm;
    free(r); free(z); free(p); free(w); free(t);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Data loss (Method, equation loss_Ab) and its gradient w.r.t. L            */
/* ------------------------------------------------------------------------ */

/* Lower-triangular product y = L x (L lower CSR incl. diagonal). */
static void lmul(int n, const int *lrowptr, const int *lcol, const double *lval,
                 const double *x, double *y)
{
    orc_spmv(n, lrowptr, lcol, lval, x, y);
}

/* y = L^T x computed from L's rows: y_j = sum_i L_ij x_i. */
static void ltmul(int n, const int *lrowptr, const int *lcol, const double *lval,
                  const double *x, double *y)
{
    for (int j = 0; j < n; ++j) y[j] = 0.0;
    for (int i = 0; i < n; ++i)
        for (int p = lrowptr[i]; p < lrowptr[i + 1]; ++p) y[lcol[p]] += lval[p] * x[i];
}

/* loss = || L L^T x - b ||^2.  If grad != NULL, grad[k] = d loss / d L_k for
 * every stored entry k = (i,j) of L:  2 (r_i u_j + x_i w_j) with u = L^T x,
 * r = L u - b, w = L^T r  (derivative of the quadratic form, entry by entry). */
double orc_llt_loss(int n, const int *lrowptr, const int *lcol, const double *lval,
                    const double *x, const double *b, double *grad)
{
    double *u = (double *)malloc(sizeof(double) * (size_t)n);
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    ltmul(n, lrowptr, lcol, lval, x, u);
    lmul(n, lrowptr, lcol, lval, u, q);
    double loss = 0.0;
    for (int i = 0; i < n; ++i) { q[i] = q[i] - b[i]; loss += q[i] * q[i]; }
    if (grad) {
        ltmul(n, lrowptr, lcol, lval, q, w);
        for (int i = 0; i < n; ++i)
            for (int p = lrowptr[i]; p < lrowptr[i + 1]; ++p) {
                int j = lcol[p];
                grad[p] = 2.0 * (q[i] * u[j] + x[i] * w[j]);
            }
    }
    free(u); free(q); free(w);
    return loss;
}
