/*
 * cr_oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.
 *
 * A plain, slow, obviously correct FP64 CPU implementation of block cyclic
 * reduction for Hermitian positive definite (HPD) block-tridiagonal systems,
 * written from the paper "Review of Cyclic Reduction for Parallel Solution of
 * Hermitian Positive Definite Block-Tridiagonal Linear Systems"
 * (M. Neuenhofen, arXiv 1807.00370).  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP implementation.
 *
 * Problem (Section 1, Eq. (Axb), Eq. (Data)): diagonal blocks A_1..A_N,
 * sub-diagonal blocks B_1..B_{N-1} (B_j sits at block row j+1, column j; its
 * conjugate transpose at row j, column j+1), right-hand sides y_1..y_N, all
 * complex; the matrix is Hermitian positive definite; unknowns x_1..x_N.
 *
 * Storage: C99 double complex, row-major blocks, 0-based arrays:
 *   A + (j-1)*m*m  is A_j   (only the lower triangle and Re(diagonal) are read)
 *   B + (j-1)*m*m  is B_j   (N-1 blocks)
 *   y + (j-1)*m*k  is y_j   (m x k, row-major), likewise x.
 *
 * Three solvers that reach the same x = A^{-1} y (and a hybrid of the first
 * two, cro_solve_hybrid: the one-sided reduction down to a level of at most
 * a given number of blocks, then Algorithm 1 on that level's system):
 *   cro_solve_cr      one-sided cyclic reduction: at each level the odd-index
 *                     blocks are eliminated through the even system of
 *                     Eq. (even) (formulas for V_j, F_j, v_j in Eq. (Formulas)),
 *                     the even system is solved recursively, and the odd
 *                     unknowns come back from the first block row of the
 *                     reordered system of Section 2.
 *   cro_solve_pcr     Algorithm 1 as printed: both the odd system Eq. (odd) and
 *                     the even system Eq. (even) are formed and solved
 *                     recursively, then the solution is reassembled.
 *   cro_solve_thomas  block Cholesky of the block-tridiagonal matrix, a
 *                     sequential method used as an independent cross-check.
 *
 * Every Schur term G^H M^{-1} G is formed as the paper's Section 4 prescribes:
 * L = chol(M), Gt = L \ G, Z = Gt^H Gt (the printed "Gt^H Gt^H" is read as
 * Gt^H Gt).  Cross terms G1^H M^{-1} G2 use the same L: (L\G1)^H (L\G2).
 * Hermitian results are computed on the lower triangle and mirrored, and their
 * diagonal is made real, so that reduced diagonal blocks are exactly Hermitian
 * (Section 4).
 *
 * Positive definiteness (Section 2, "Determination of Positive Definiteness";
 * Section 4): a Cholesky pivot d that is not > 0 (NaN included) is a
 * breakdown.  The level in which a breakdown happens is finished, the
 * lexicographically smallest (level, block) is reported, x is filled with NaN
 * and the recursion stops.  "block" is the 1-based index of the block row in
 * the original numbering.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

typedef struct {
    int32_t status; /* 0: HPD, solved; 1: not HPD (Cholesky breakdown) */
    int32_t level;  /* level of the first breakdown, -1 if none        */
    int64_t block;  /* original 1-based block index, -1 if none        */
} cro_info;

static void info_clear(cro_info *f) { f->status = 0; f->level = -1; f->block = -1; }

static void info_fail(cro_info *f, int level, int64_t block)
{
    if (!f->status || level < f->level || (level == f->level && block < f->block)) {
        f->status = 1;
        f->level = level;
        f->block = block;
    }
}

static cplx *cmalloc(size_t n) { return (cplx *)calloc(n ? n : 1, sizeof(cplx)); }

/* ---------------------------------------------------------------- dense kernels */

/* L = chol(A): A = L L^H, L lower triangular with real positive diagonal.
 * Reads only the lower triangle and the real part of the diagonal of A.
 * Returns 1 on breakdown (pivot not > 0). */
static int chol(int m, const cplx *A, cplx *L)
{
    memset(L, 0, (size_t)m * m * sizeof(cplx));
    for (int c = 0; c < m; ++c) {
        double d = creal(A[c * m + c]);
        for (int t = 0; t < c; ++t) {
            cplx l = L[c * m + t];
            d -= creal(l) * creal(l) + cimag(l) * cimag(l);
        }
        if (!(d > 0.0))
            return 1;
        double s = sqrt(d);
        L[c * m + c] = s;
        for (int r = c + 1; r < m; ++r) {
            cplx v = A[r * m + c];
            for (int t = 0; t < c; ++t)
                v -= L[r * m + t] * conj(L[c * m + t]);
            L[r * m + c] = v / s;
        }
    }
    return 0;
}

/* X = L^{-1} G by forward substitution; G and X are m x nc row-major. */
static void fwd_sub(int m, int nc, const cplx *L, const cplx *G, cplx *X)
{
    for (int r = 0; r < m; ++r)
        for (int c = 0; c < nc; ++c) {
            cplx v = G[r * nc + c];
            for (int t = 0; t < r; ++t)
                v -= L[r * m + t] * X[t * nc + c];
            X[r * nc + c] = v / creal(L[r * m + r]);
        }
}

/* X = L^{-H} G by backward substitution. */
static void bwd_sub(int m, int nc, const cplx *L, const cplx *G, cplx *X)
{
    for (int r = m - 1; r >= 0; --r)
        for (int c = 0; c < nc; ++c) {
            cplx v = G[r * nc + c];
            for (int t = r + 1; t < m; ++t)
                v -= conj(L[t * m + r]) * X[t * nc + c];
            X[r * nc + c] = v / creal(L[r * m + r]);
        }
}

/* BH = B^H for an m x m block. */
static void herm_t(int m, const cplx *B, cplx *BH)
{
    for (int r = 0; r < m; ++r)
        for (int c = 0; c < m; ++c)
            BH[r * m + c] = conj(B[c * m + r]);
}

/* Z -= X1^H X2 with X1 m x n1, X2 m x n2, Z n1 x n2 (all entries). */
static void sub_gram(int m, int n1, int n2, const cplx *X1, const cplx *X2, cplx *Z)
{
    for (int a = 0; a < n1; ++a)
        for (int b = 0; b < n2; ++b) {
            cplx s = 0;
            for (int t = 0; t < m; ++t)
                s += conj(X1[t * n1 + a]) * X2[t * n2 + b];
            Z[a * n2 + b] -= s;
        }
}

/* Z -= X^H X on the lower triangle only (X m x n, Z n x n). */
static void sub_gram_lower(int m, int n, const cplx *X, cplx *Z)
{
    for (int a = 0; a < n; ++a)
        for (int b = 0; b <= a; ++b) {
            cplx s = 0;
            for (int t = 0; t < m; ++t)
                s += conj(X[t * n + a]) * X[t * n + b];
            Z[a * n + b] -= s;
        }
}

/* Make an m x m block exactly Hermitian from its lower triangle. */
static void mirror_lower(int m, cplx *Z)
{
    for (int a = 0; a < m; ++a) {
        Z[a * m + a] = creal(Z[a * m + a]);
        for (int b = 0; b < a; ++b)
            Z[b * m + a] = conj(Z[a * m + b]);
    }
}

/* Y -= M X with M m x m (full), X m x k. */
static void sub_mul(int m, int k, const cplx *M, const cplx *X, cplx *Y)
{
    for (int r = 0; r < m; ++r)
        for (int c = 0; c < k; ++c) {
            cplx s = 0;
            for (int t = 0; t < m; ++t)
                s += M[r * m + t] * X[t * k + c];
            Y[r * k + c] -= s;
        }
}

/* Y -= M^H X. */
static void sub_mul_h(int m, int k, const cplx *M, const cplx *X, cplx *Y)
{
    for (int r = 0; r < m; ++r)
        for (int c = 0; c < k; ++c) {
            cplx s = 0;
            for (int t = 0; t < m; ++t)
                s += conj(M[t * m + r]) * X[t * k + c];
            Y[r * k + c] -= s;
        }
}

/* Y -= Herm(A) X where Herm(A) is the Hermitian matrix with A's lower
 * triangle and the real part of A's diagonal. */
static void sub_herm_mul(int m, int k, const cplx *A, const cplx *X, cplx *Y)
{
    for (int r = 0; r < m; ++r)
        for (int c = 0; c < k; ++c) {
            cplx s = 0;
            for (int t = 0; t < m; ++t) {
                cplx a;
                if (t < r)
                    a = A[r * m + t];
                else if (t == r)
                    a = creal(A[r * m + r]);
                else
                    a = conj(A[t * m + r]);
                s += a * X[t * k + c];
            }
            Y[r * k + c] -= s;
        }
}

static void fill_nan(size_t n, cplx *x)
{
    for (size_t i = 0; i < n; ++i)
        x[i] = NAN + NAN * I;
}

/* ------------------------------------------------ per-block elimination pieces */

/* Factor diagonal block A_i of the current level and form, by the Section 4
 * recipe, Pt = L\Bnext^H (Bnext couples i with the next block), Qt = L\Bprev
 * (Bprev couples i with the previous block) and gt = L\y_i.  A missing
 * neighbour coupling (NULL) gives a zero block, which is the boundary
 * convention B_0 = B_N = 0 of Section 2. */
typedef struct {
    cplx *L, *P, *Q, *g;
    int hasP, hasQ;
} elim;

static int elim_block(int m, int k, const cplx *A, const cplx *Bprev, const cplx *Bnext,
                      const cplx *y, elim *e, cplx *tmp)
{
    e->hasP = Bnext != NULL;
    e->hasQ = Bprev != NULL;
    if (chol(m, A, e->L))
        return 1;
    if (Bnext) {
        herm_t(m, Bnext, tmp);
        fwd_sub(m, m, e->L, tmp, e->P);
    }
    if (Bprev)
        fwd_sub(m, m, e->L, Bprev, e->Q);
    if (y)
        fwd_sub(m, k, e->L, y, e->g);
    return 0;
}

static void elim_alloc(elim *e, int m, int k)
{
    e->L = cmalloc((size_t)m * m);
    e->P = cmalloc((size_t)m * m);
    e->Q = cmalloc((size_t)m * m);
    e->g = cmalloc((size_t)m * k);
    e->hasP = e->hasQ = 0;
}

static void elim_free(elim *e) { free(e->L); free(e->P); free(e->Q); free(e->g); }

/* Diagonal block of a reduced system, Eq. (Formulas):
 *   Z = A_c - B_l A_l^{-1} B_l^H - B_r^H A_r^{-1} B_r
 * with left neighbour term Pt_l^H Pt_l and right neighbour term Qt_r^H Qt_r.
 * Right-hand side: z = y_c - Pt_l^H gt_l - Qt_r^H gt_r. */
static void reduce_diag(int m, int k, const cplx *Ac, const cplx *yc, const elim *l,
                        const elim *r, cplx *Z, cplx *z)
{
    for (int a = 0; a < m; ++a)
        for (int b = 0; b <= a; ++b)
            Z[a * m + b] = Ac[a * m + b];
    if (l && l->hasP)
        sub_gram_lower(m, m, l->P, Z);
    if (r && r->hasQ)
        sub_gram_lower(m, m, r->Q, Z);
    mirror_lower(m, Z);
    memcpy(z, yc, (size_t)m * k * sizeof(cplx));
    if (l && l->hasP)
        sub_gram(m, m, k, l->P, l->g, z);
    if (r && r->hasQ)
        sub_gram(m, m, k, r->Q, r->g, z);
}

/* Off-diagonal block of a reduced system, Eq. (Formulas):
 *   F = -B_{c+1} A_c^{-1} B_c = -Pt_c^H Qt_c  (eliminated block c in between). */
static void reduce_off(int m, const elim *c, cplx *F)
{
    memset(F, 0, (size_t)m * m * sizeof(cplx));
    sub_gram(m, m, m, c->P, c->Q, F);
}

/* ------------------------------------------------------- one-sided reduction */

static void pcr_solver(int n, int m, int k, const cplx *A, const cplx *B, const cplx *y,
                       const int64_t *orig, cplx *x, int depth, cro_info *info);

/* One level of the one-sided reduction.  hyb > 0: once a level holds at most
 * hyb blocks, the rest of the system is solved by Algorithm 1 (both half
 * systems at every level, pcr_solver) instead, with its levels numbered on
 * from this one and its blocks in the original numbering. */
static void cr_level(int n, int m, int k, const cplx *A, const cplx *B, const cplx *y,
                     cplx *x, int level, int64_t ostride, int hyb, cro_info *info)
{
    /* 0-based position p at this level is original block (p+1)*ostride. */
    const size_t mm = (size_t)m * m, mk = (size_t)m * k;
    if (hyb > 0 && n <= hyb) {
        int64_t *orig = (int64_t *)malloc((size_t)n * sizeof(int64_t));
        for (int p = 0; p < n; ++p)
            orig[p] = (int64_t)(p + 1) * ostride;
        pcr_solver(n, m, k, A, B, y, orig, x, level, info);
        free(orig);
        return;
    }
    const int ne = (n + 1) / 2; /* odd 1-based positions: eliminated   */
    const int nk = n / 2;       /* even 1-based positions: kept, Eq. (even) */
    elim *E = (elim *)calloc((size_t)ne, sizeof(elim));
    int *fail = (int *)calloc((size_t)ne, sizeof(int));
    for (int t = 0; t < ne; ++t)
        elim_alloc(&E[t], m, k);

#pragma omp parallel
    {
        cplx *tmp = cmalloc(mm);
#pragma omp for schedule(static)
        for (int t = 0; t < ne; ++t) {
            int p = 2 * t;
            fail[t] = elim_block(m, k, A + p * mm, p >= 1 ? B + (p - 1) * mm : NULL,
                                 p + 1 < n ? B + p * mm : NULL, y + p * mk, &E[t], tmp);
        }
        free(tmp);
    }
    int failed = 0;
    for (int t = 0; t < ne; ++t)
        if (fail[t]) {
            info_fail(info, level, (int64_t)(2 * t + 1) * ostride);
            failed = 1;
        }
    if (failed) {
        fill_nan((size_t)n * mk, x);
    } else {
        if (nk > 0) {
            /* Even system (V, F, v) of Eq. (even), block-tridiagonal of size nk. */
            cplx *V = cmalloc((size_t)nk * mm), *F = cmalloc((size_t)nk * mm);
            cplx *v = cmalloc((size_t)nk * mk), *xe = cmalloc((size_t)nk * mk);
#pragma omp parallel for schedule(static)
            for (int j = 0; j < nk; ++j) {
                int q = 2 * j + 1; /* kept position; neighbours q-1, q+1 eliminated */
                const elim *l = &E[j];
                const elim *r = (q + 1 < n) ? &E[j + 1] : NULL;
                reduce_diag(m, k, A + q * mm, y + q * mk, l, r, V + j * mm, v + j * mk);
                if (j + 1 < nk)
                    reduce_off(m, &E[j + 1], F + j * mm);
            }
            cr_level(nk, m, k, V, F, v, xe, level + 1, ostride * 2, hyb, info);
            for (int j = 0; j < nk; ++j)
                memcpy(x + (2 * j + 1) * mk, xe + j * mk, mk * sizeof(cplx));
            free(V); free(F); free(v); free(xe);
        }
        if (info->status) {
            fill_nan((size_t)n * mk, x);
        } else {
            /* Odd unknowns from the first block row of the reordered system:
             * D_1 x_o + C^H x_e = y_o, i.e.
             * x_i = A_i^{-1} (y_i - B_{i-1} x_{i-1} - B_i^H x_{i+1})
             *     = L^{-H} (gt - Qt x_{i-1} - Pt x_{i+1}). */
#pragma omp parallel
            {
                cplx *w = cmalloc(mk);
#pragma omp for schedule(static)
                for (int t = 0; t < ne; ++t) {
                    int p = 2 * t;
                    memcpy(w, E[t].g, mk * sizeof(cplx));
                    if (E[t].hasQ)
                        sub_mul(m, k, E[t].Q, x + (p - 1) * mk, w);
                    if (E[t].hasP)
                        sub_mul(m, k, E[t].P, x + (p + 1) * mk, w);
                    bwd_sub(m, k, E[t].L, w, x + p * mk);
                }
                free(w);
            }
        }
    }
    for (int t = 0; t < ne; ++t)
        elim_free(&E[t]);
    free(E);
    free(fail);
}

int cro_solve_cr(int N, int m, int k, const cplx *A, const cplx *B, const cplx *y, cplx *x,
                 cro_info *info)
{
    if (N < 1 || m < 1 || k < 1)
        return -1;
    info_clear(info);
    cr_level(N, m, k, A, B, y, x, 0, 1, 0, info);
    return 0;
}

/* The one-sided reduction until a level holds at most hyb blocks, then
 * Algorithm 1 on that level's system (hyb = 0: one-sided throughout). */
int cro_solve_hybrid(int N, int m, int k, int hyb, const cplx *A, const cplx *B, const cplx *y,
                     cplx *x, cro_info *info)
{
    if (N < 1 || m < 1 || k < 1 || hyb < 0)
        return -1;
    info_clear(info);
    cr_level(N, m, k, A, B, y, x, 0, 1, hyb, info);
    return 0;
}

/* --------------------------------------------------------------- Algorithm 1 */

static void pcr_solver(int n, int m, int k, const cplx *A, const cplx *B, const cplx *y,
                       const int64_t *orig, cplx *x, int depth, cro_info *info)
{
    const size_t mm = (size_t)m * m, mk = (size_t)m * k;
    if (n == 1) {
        /* Base case: Cholesky's method on the m x m system. */
        cplx *L = cmalloc(mm), *w = cmalloc(mk);
        if (chol(m, A, L)) {
            info_fail(info, depth, orig[0]);
            fill_nan(mk, x);
        } else {
            fwd_sub(m, k, L, y, w);
            bwd_sub(m, k, L, w, x);
        }
        free(L); free(w);
        return;
    }
    /* N even is assumed by the split; an odd system is extended by one
     * identity block (A = I, B = 0, y = 0), the boundary convention of
     * Section 2, which leaves x and positive definiteness unchanged. */
    int n2 = n + (n & 1);
    const cplx *Ap = A, *Bp = B, *yp = y;
    const int64_t *op = orig;
    cplx *Apad = NULL, *Bpad = NULL, *ypad = NULL;
    int64_t *opad = NULL;
    if (n2 != n) {
        Apad = cmalloc((size_t)n2 * mm);
        Bpad = cmalloc((size_t)(n2 - 1) * mm);
        ypad = cmalloc((size_t)n2 * mk);
        opad = (int64_t *)malloc((size_t)n2 * sizeof(int64_t));
        memcpy(Apad, A, (size_t)n * mm * sizeof(cplx));
        for (int a = 0; a < m; ++a)
            Apad[(size_t)n * mm + a * m + a] = 1.0;
        if (n > 1)
            memcpy(Bpad, B, (size_t)(n - 1) * mm * sizeof(cplx));
        memcpy(ypad, y, (size_t)n * mk * sizeof(cplx));
        memcpy(opad, orig, (size_t)n * sizeof(int64_t));
        opad[n] = -1;
        Ap = Apad; Bp = Bpad; yp = ypad; op = opad;
    }
    /* Every diagonal block is factored once; its pieces serve both systems. */
    elim *E = (elim *)calloc((size_t)n2, sizeof(elim));
    int *fail = (int *)calloc((size_t)n2, sizeof(int));
    for (int i = 0; i < n2; ++i)
        elim_alloc(&E[i], m, k);
#pragma omp parallel
    {
        cplx *tmp = cmalloc(mm);
#pragma omp for schedule(static)
        for (int i = 0; i < n2; ++i)
            fail[i] = elim_block(m, k, Ap + i * mm, i >= 1 ? Bp + (i - 1) * mm : NULL,
                                 i + 1 < n2 ? Bp + i * mm : NULL, yp + i * mk, &E[i], tmp);
        free(tmp);
    }
    int failed = 0;
    for (int i = 0; i < n2; ++i)
        if (fail[i]) {
            info_fail(info, depth, op[i]);
            failed = 1;
        }
    if (failed) {
        fill_nan((size_t)n * mk, x);
    } else {
        int h = n2 / 2;
        cplx *U = cmalloc((size_t)h * mm), *Eo = cmalloc((size_t)h * mm), *u = cmalloc((size_t)h * mk);
        cplx *V = cmalloc((size_t)h * mm), *F = cmalloc((size_t)h * mm), *v = cmalloc((size_t)h * mk);
        cplx *xo = cmalloc((size_t)h * mk), *xe = cmalloc((size_t)h * mk);
        int64_t *oo = (int64_t *)malloc((size_t)h * sizeof(int64_t));
        int64_t *oe = (int64_t *)malloc((size_t)h * sizeof(int64_t));
#pragma omp parallel for schedule(static)
        for (int j = 1; j <= h; ++j) {
            /* 1-based paper indices; block i sits at 0-based i-1.  Terms with
             * index 0 or n2+1 vanish (B_0 = B_N = 0). */
            int io = 2 * j - 1, ie = 2 * j;
            /* U_j = A_{2j-1} - B_{2j-2} A_{2j-2}^{-1} B_{2j-2}^H - B_{2j-1}^H A_{2j}^{-1} B_{2j-1} */
            reduce_diag(m, k, Ap + (io - 1) * mm, yp + (io - 1) * mk,
                        io - 1 >= 1 ? &E[io - 2] : NULL, &E[ie - 1],
                        U + (j - 1) * mm, u + (j - 1) * mk);
            /* E_j = -B_{2j} A_{2j}^{-1} B_{2j-1} */
            if (j < h)
                reduce_off(m, &E[ie - 1], Eo + (j - 1) * mm);
            /* V_j = A_{2j} - B_{2j-1} A_{2j-1}^{-1} B_{2j-1}^H - B_{2j}^H A_{2j+1}^{-1} B_{2j} */
            reduce_diag(m, k, Ap + (ie - 1) * mm, yp + (ie - 1) * mk, &E[io - 1],
                        ie + 1 <= n2 ? &E[ie] : NULL, V + (j - 1) * mm, v + (j - 1) * mk);
            /* F_j = -B_{2j+1} A_{2j+1}^{-1} B_{2j} */
            if (j < h)
                reduce_off(m, &E[ie], F + (j - 1) * mm);
            oo[j - 1] = op[io - 1];
            oe[j - 1] = op[ie - 1];
        }
        for (int i = 0; i < n2; ++i)
            elim_free(&E[i]);
        free(E);
        E = NULL;
        pcr_solver(h, m, k, U, Eo, u, oo, xo, depth + 1, info);
        pcr_solver(h, m, k, V, F, v, oe, xe, depth + 1, info);
        /* Reassemble x from x_o and x_e (the pad block, if any, is dropped). */
        for (int j = 1; j <= h; ++j) {
            if (2 * j - 1 <= n)
                memcpy(x + (2 * j - 2) * mk, xo + (j - 1) * mk, mk * sizeof(cplx));
            if (2 * j <= n)
                memcpy(x + (2 * j - 1) * mk, xe + (j - 1) * mk, mk * sizeof(cplx));
        }
        if (info->status)
            fill_nan((size_t)n * mk, x);
        free(U); free(Eo); free(u); free(V); free(F); free(v);
        free(xo); free(xe); free(oo); free(oe);
    }
    if (E) {
        for (int i = 0; i < n2; ++i)
            elim_free(&E[i]);
        free(E);
    }
    free(fail);
    free(Apad); free(Bpad); free(ypad); free(opad);
}

int cro_solve_pcr(int N, int m, int k, const cplx *A, const cplx *B, const cplx *y, cplx *x,
                  cro_info *info)
{
    if (N < 1 || m < 1 || k < 1)
        return -1;
    info_clear(info);
    int64_t *orig = (int64_t *)malloc((size_t)N * sizeof(int64_t));
    for (int i = 0; i < N; ++i)
        orig[i] = i + 1;
    pcr_solver(N, m, k, A, B, y, orig, x, 0, info);
    free(orig);
    return 0;
}

/* One split of Section 2 for an even-sized system: returns U, E, u (odd
 * system, Eq. (odd)) and V, F, v (even system, Eq. (even)) computed with the
 * formulas of Eq. (Formulas).  Exposed so that tests can hold the formulas
 * against dense Schur complements.  Returns 1 on breakdown, -1 on bad sizes. */
int cro_split(int N, int m, int k, const cplx *A, const cplx *B, const cplx *y, cplx *U,
              cplx *E, cplx *u, cplx *V, cplx *F, cplx *v)
{
    if (N < 2 || (N & 1) || m < 1 || k < 1)
        return -1;
    const size_t mm = (size_t)m * m, mk = (size_t)m * k;
    elim *El = (elim *)calloc((size_t)N, sizeof(elim));
    cplx *tmp = cmalloc(mm);
    int failed = 0;
    for (int i = 0; i < N; ++i) {
        elim_alloc(&El[i], m, k);
        failed |= elim_block(m, k, A + i * mm, i >= 1 ? B + (i - 1) * mm : NULL,
                             i + 1 < N ? B + i * mm : NULL, y + i * mk, &El[i], tmp);
    }
    if (!failed) {
        int h = N / 2;
        for (int j = 1; j <= h; ++j) {
            int io = 2 * j - 1, ie = 2 * j;
            reduce_diag(m, k, A + (io - 1) * mm, y + (io - 1) * mk,
                        io - 1 >= 1 ? &El[io - 2] : NULL, &El[ie - 1], U + (j - 1) * mm,
                        u + (j - 1) * mk);
            if (j < h)
                reduce_off(m, &El[ie - 1], E + (j - 1) * mm);
            reduce_diag(m, k, A + (ie - 1) * mm, y + (ie - 1) * mk, &El[io - 1],
                        ie + 1 <= N ? &El[ie] : NULL, V + (j - 1) * mm, v + (j - 1) * mk);
            if (j < h)
                reduce_off(m, &El[ie], F + (j - 1) * mm);
        }
    }
    for (int i = 0; i < N; ++i)
        elim_free(&El[i]);
    free(El);
    free(tmp);
    return failed;
}

/* ------------------------------------------------------ block Cholesky (Thomas) */

/* A = L L^H with L block lower bidiagonal: diagonal blocks Ld_j (lower
 * triangular) and sub-diagonal blocks C_j = B_j Ld_j^{-H}:
 *   Ld_j = chol(A_j - C_{j-1} C_{j-1}^H),  C_j^H = Ld_j^{-1} B_j^H,
 *   Ld_j w_j = y_j - C_{j-1} w_{j-1},      Ld_j^H x_j = w_j - C_j^H x_{j+1}. */
int cro_solve_thomas(int N, int m, int k, const cplx *A, const cplx *B, const cplx *y, cplx *x,
                     cro_info *info)
{
    if (N < 1 || m < 1 || k < 1)
        return -1;
    info_clear(info);
    const size_t mm = (size_t)m * m, mk = (size_t)m * k;
    cplx *Ld = cmalloc((size_t)N * mm), *CH = cmalloc((size_t)N * mm);
    cplx *w = cmalloc((size_t)N * mk), *S = cmalloc(mm), *t1 = cmalloc(mm), *r = cmalloc(mk);
    for (int j = 0; j < N; ++j) {
        memcpy(S, A + j * mm, mm * sizeof(cplx));
        memcpy(r, y + j * mk, mk * sizeof(cplx));
        if (j > 0) {
            /* S -= C_{j-1} C_{j-1}^H = (C^H)^H (C^H) on the lower triangle */
            sub_gram_lower(m, m, CH + (j - 1) * mm, S);
            /* r -= C_{j-1} w_{j-1} = (C^H)^H w */
            sub_mul_h(m, k, CH + (j - 1) * mm, w + (j - 1) * mk, r);
        }
        if (chol(m, S, Ld + j * mm)) {
            info_fail(info, 0, j + 1);
            break;
        }
        fwd_sub(m, k, Ld + j * mm, r, w + j * mk);
        if (j + 1 < N) {
            herm_t(m, B + j * mm, t1);
            fwd_sub(m, m, Ld + j * mm, t1, CH + j * mm);
        }
    }
    if (info->status) {
        fill_nan((size_t)N * mk, x);
    } else {
        for (int j = N - 1; j >= 0; --j) {
            memcpy(r, w + j * mk, mk * sizeof(cplx));
            if (j + 1 < N)
                sub_mul(m, k, CH + j * mm, x + (j + 1) * mk, r);
            bwd_sub(m, k, Ld + j * mm, r, x + j * mk);
        }
    }
    free(Ld); free(CH); free(w); free(S); free(t1); free(r);
    return 0;
}

/* ------------------------------------------------------------ residual, adjoint */

/* r = y - A x with the Hermitian reading of A_j (Eq. (Axb)):
 * r_j = y_j - B_{j-1} x_{j-1} - A_j x_j - B_j^H x_{j+1}. */
void cro_residual(int N, int m, int k, const cplx *A, const cplx *B, const cplx *x,
                  const cplx *y, cplx *r)
{
    const size_t mm = (size_t)m * m, mk = (size_t)m * k;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < N; ++j) {
        cplx *rj = r + j * mk;
        memcpy(rj, y + j * mk, mk * sizeof(cplx));
        if (j > 0)
            sub_mul(m, k, B + (j - 1) * mm, x + (j - 1) * mk, rj);
        sub_herm_mul(m, k, A + j * mm, x + j * mk, rj);
        if (j + 1 < N)
            sub_mul_h(m, k, B + j * mm, x + (j + 1) * mk, rj);
    }
}

/* Adjoint of x = A^{-1} y for a real loss with gradient gx = dL/dx (PyTorch's
 * conjugate-Wirtinger convention): lam = A^{-H} gx = A^{-1} gx (lam is given),
 * grad y = lam, grad A (dense) = -lam x^H, hence per block
 *   gA_j = -lam_j x_j^H,   gB_j = -(lam_{j+1} x_j^H + x_{j+1} lam_j^H). */
void cro_backward(int N, int m, int k, const cplx *x, const cplx *lam, cplx *gA, cplx *gB)
{
    const size_t mm = (size_t)m * m, mk = (size_t)m * k;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < N; ++j) {
        const cplx *lj = lam + j * mk, *xj = x + j * mk;
        for (int a = 0; a < m; ++a)
            for (int b = 0; b < m; ++b) {
                cplx s = 0;
                for (int c = 0; c < k; ++c)
                    s += lj[a * k + c] * conj(xj[b * k + c]);
                gA[j * mm + a * m + b] = -s;
            }
        if (j + 1 < N) {
            const cplx *l1 = lam + (j + 1) * mk, *x1 = x + (j + 1) * mk;
            for (int a = 0; a < m; ++a)
                for (int b = 0; b < m; ++b) {
                    cplx s = 0;
                    for (int c = 0; c < k; ++c)
                        s += l1[a * k + c] * conj(xj[b * k + c]) + x1[a * k + c] * conj(lj[b * k + c]);
                    gB[j * mm + a * m + b] = -s;
                }
        }
    }
}

int cro_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the later parallel regions (timing of the CPU baseline). */
void cro_set_num_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}
