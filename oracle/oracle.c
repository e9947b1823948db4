/*
 * CPU oracle for IDR(s)stab(l) and M(s)stab(l) in FP64.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this code.  It shares no source with
 * the HIP library: it is a plain, slow, sequential restatement of the paper
 * (Neuenhofen, "M(s)stab(l): A Generalization of IDR(s)stab(l) for Sequences
 * of Linear Systems", arXiv 1604.06043), written for checking by eye.
 *
 * Readings of the paper that this file commits to (listed again, with the
 * reasons, in the design notes of the repository):
 *   - The stopping test of Algorithm 1 is relative: ||r|| <= tol ||b||,
 *     compared on squares.  The loop runs on the recursive residual; on exit
 *     the true residual b - A x is formed (one counted check MV) and, while it
 *     still exceeds tol, it replaces r and the loop continues (at most
 *     max_repl times), as the ocean experiment of Section 5.1 replaces the
 *     residual after the solution update.  With replace_every = k > 0 the
 *     recursive residual is also replaced by b - A x at the end of every k-th
 *     cycle while it is above the tolerance (one counted check MV each): the
 *     ocean run of Section 5.1 does so after every cycle (k = 1), on the
 *     split-preconditioned system.  These periodic replacements are counted
 *     with the others but do not use up max_repl.
 *   - The solution update of Algorithm 1 sums over i = 1..l (the printed
 *     lower index is a typo).  x and u_q use the level vectors from before
 *     r and v_q are overwritten.
 *   - "Choose gamma / eta such that ... is orthogonal to P" is the s x s system
 *     (P^T B) c = P^T y, solved by LU with partial pivoting; the system is
 *     declared singular when a pivot is <= 1e-14 times the largest entry of
 *     its column.
 *   - tau = Z^+ r^(0) is solved through the normal equations (Cholesky, then
 *     LU if Cholesky fails); a singular Gram matrix is a breakdown.
 *   - For IDR(s)stab the input U, V are the Arnoldi basis of level s of the
 *     initial residual (Section 5, preliminaries): u_1 = r/||r||, v_q = A u_q,
 *     u_{q+1} = MGS-orthonormalized v_q; s MVs.
 *   - M(s)stab is Algorithm 1 called with the P, U, V fetched from a former
 *     solve (Section 4.2).  Fetching copies U, V at the end of a cycle
 *     (Section 5, preliminaries); the policy decides which cycle end.
 *   - Every product with A is counted: the initial residual, the Arnoldi MVs,
 *     l(s+1) per cycle (Table 1), and the true-residual checks separately.
 *   - A breakdown (singular small system) drops U, V and restarts from the
 *     true residual b - A x (one counted MV) with an Arnoldi basis, at most
 *     twice per solve; a third breakdown is returned as an error.
 *   - Optionally (not in the paper) the fetched U, V are orthonormalized by
 *     CholQR in FP64 (orc_cholqr), keeping V = A U.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no FMA contraction, so every
 * a*b+c below rounds twice, as written).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_NOT_CONVERGED 1
#define ORC_E_INVALID (-1)
#define ORC_E_NOMEM (-3)
#define ORC_E_BREAKDOWN (-4)
#define ORC_E_NONFINITE (-5)

#define ORC_MSTAB 0
#define ORC_IDRSTAB 1

#define ORC_FETCH_THRESHOLD 0
#define ORC_FETCH_AT_LEVEL 1
#define ORC_FETCH_AT_END 2
#define ORC_FETCH_ONCE 3
#define ORC_FETCH_NEVER 4
#define ORC_FETCH_ESTIMATE 5

#define ORC_MAX_RESTARTS 2

/* ------------------------------------------------------------------------ */
/* Matrix assembly: upwind finite differences for                            */
/*   A = I/dt - div(kappa grad .) + beta . grad                              */
/* on n^dim interior nodes of the unit square/cube, x fastest, Dirichlet.    */
/* ------------------------------------------------------------------------ */

int64_t orc_convdiff_nnz(int dim, int64_t n)
{
    int64_t cells = 1, faces = 1;
    for (int d = 0; d < dim; ++d) cells *= n;
    faces = (n - 1);
    for (int d = 1; d < dim; ++d) faces *= n;
    return cells + 2 * dim * faces;
}

static double face_kappa(const double *kappa, int64_t a, int64_t b, int interior)
{
    if (!kappa) return 1.0;
    if (!interior) return kappa[a];
    double ka = kappa[a], kb = kappa[b];
    return (2.0 * ka * kb) / (ka + kb);
}

/*
 * Row i, in column order: -z, -y, -x, diagonal, +x, +y, +z (those that exist).
 * Face coefficient kf (1, or the harmonic mean of the two node values; the
 * node's own value at a boundary face).  Convection uses the backward
 * difference for beta_d > 0 and the forward difference otherwise.
 *   diag  = inv_dt, then += kf*h^-2 for faces -x,+x,-y,+y,-z,+z in that order,
 *           then += |beta_d| h^-1 for d = x, y, z
 *   minus neighbour (-d):  -(kf h^-2) - max(beta_d, 0) h^-1
 *   plus  neighbour (+d):  -(kf h^-2) + min(beta_d, 0) h^-1
 */
void orc_assemble_convdiff(int dim, int64_t n, const double *beta, double inv_dt,
                           const double *kappa, int32_t *row_ptr, int32_t *col, double *val)
{
    double hinv = (double)(n + 1);
    double hinv2 = hinv * hinv;
    int64_t stride[3] = {1, n, n * n};
    int64_t N = 1;
    for (int d = 0; d < dim; ++d) N *= n;
    int64_t pos = 0;
    for (int64_t i = 0; i < N; ++i) {
        int64_t c[3] = {i % n, (i / n) % n, (dim == 3) ? i / (n * n) : 0};
        row_ptr[i] = (int32_t)pos;
        /* face coefficients in order -x,+x,-y,+y,-z,+z */
        double kf[3][2];
        for (int d = 0; d < dim; ++d) {
            kf[d][0] = face_kappa(kappa, i, i - stride[d], c[d] > 0);
            kf[d][1] = face_kappa(kappa, i, i + stride[d], c[d] < n - 1);
        }
        double diag = inv_dt;
        for (int d = 0; d < dim; ++d) {
            diag = diag + kf[d][0] * hinv2;
            diag = diag + kf[d][1] * hinv2;
        }
        for (int d = 0; d < dim; ++d) diag = diag + fabs(beta[d]) * hinv;
        /* lower neighbours, highest stride first */
        for (int d = dim - 1; d >= 0; --d) {
            if (c[d] > 0) {
                double bp = beta[d] > 0.0 ? beta[d] : 0.0;
                col[pos] = (int32_t)(i - stride[d]);
                val[pos] = -(kf[d][0] * hinv2) - bp * hinv;
                ++pos;
            }
        }
        col[pos] = (int32_t)i;
        val[pos] = diag;
        ++pos;
        for (int d = 0; d < dim; ++d) {
            if (c[d] < n - 1) {
                double bm = beta[d] < 0.0 ? beta[d] : 0.0;
                col[pos] = (int32_t)(i + stride[d]);
                val[pos] = -(kf[d][1] * hinv2) + bm * hinv;
                ++pos;
            }
        }
    }
    row_ptr[N] = (int32_t)pos;
}

/* ------------------------------------------------------------------------ */
/* Dense helpers                                                             */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t n;
    const int32_t *rp, *ci;
    const double *va;
    int64_t mv; /* products with A performed */
    /* optional ILU(0) split preconditioning (Section 5.1): the factors in A's
       pattern (lu) and one scratch vector; the operator is then
       L^{-1} A U^{-1} */
    const double *lu;
    double *tmp;
} Mat;

static void plain_product(const Mat *A, const double *x, double *y)
{
    for (int64_t i = 0; i < A->n; ++i) {
        double acc = 0.0;
        for (int64_t k = A->rp[i]; k < A->rp[i + 1]; ++k) acc += A->va[k] * x[A->ci[k]];
        y[i] = acc;
    }
}

/* y = L^{-1} w for the unit lower factor stored below the diagonal of lu
   (rows in order; y may alias w): y_i = w_i - sum_{k<i} l_ik y_k, the
   products subtracted in column order. */
void orc_ilu_lower(int64_t n, const int32_t *rp, const int32_t *ci, const double *lu,
                   const double *w, double *y)
{
    for (int64_t i = 0; i < n; ++i) {
        double acc = w[i];
        for (int64_t k = rp[i]; k < rp[i + 1] && ci[k] < i; ++k) acc -= lu[k] * y[ci[k]];
        y[i] = acc;
    }
}

/* x = U^{-1} z for the upper factor stored on and above the diagonal of lu
   (rows from the last; x may alias z): x_i = (z_i - sum_{j>i} u_ij x_j) / u_ii,
   the products subtracted in column order. */
void orc_ilu_upper(int64_t n, const int32_t *rp, const int32_t *ci, const double *lu,
                   const double *z, double *x)
{
    for (int64_t i = n - 1; i >= 0; --i) {
        double acc = z[i];
        int64_t dk = -1;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            if (ci[k] == i) dk = k;
            else if (ci[k] > i) acc -= lu[k] * x[ci[k]];
        }
        x[i] = acc / lu[dk];
    }
}

/* y = U x with the same upper factor: y_i = u_ii x_i + sum_{j>i} u_ij x_j in
   column order. */
void orc_ilu_upper_mul(int64_t n, const int32_t *rp, const int32_t *ci, const double *lu,
                       const double *x, double *y)
{
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
            if (ci[k] >= i) acc += lu[k] * x[ci[k]];
        y[i] = acc;
    }
}

static void matvec(Mat *A, const double *x, double *y)
{
    if (A->lu) {
        orc_ilu_upper(A->n, A->rp, A->ci, A->lu, x, A->tmp);
        plain_product(A, A->tmp, y);
        orc_ilu_lower(A->n, A->rp, A->ci, A->lu, y, y);
    } else {
        plain_product(A, x, y);
    }
    A->mv++;
}

/*
 * ILU(0) of a CSR matrix with sorted columns (Section 5.1 preconditions with
 * an incomplete LU factorization without fill-in): L unit lower and U upper
 * in A's pattern with (LU)_ij = a_ij on that pattern.  Rows in order; in row
 * i, for each k < i of its pattern in column order: l_ik = a_ik / u_kk, then
 * a_ij -= l_ik u_kj for every j > k of row i's pattern that row k also holds.
 * lu (nnz) receives L below the diagonal and U on and above it.  Returns 0,
 * or 1 if a row lacks its diagonal entry or a pivot u_ii is zero or not
 * finite.
 */
int orc_ilu0(int64_t n, const int32_t *rp, const int32_t *ci, const double *va, double *lu)
{
    memcpy(lu, va, sizeof(double) * (size_t)rp[n]);
    int64_t *dpos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!dpos) return ORC_E_NOMEM;
    for (int64_t i = 0; i < n; ++i) {
        dpos[i] = -1;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
            if (ci[k] == i) dpos[i] = k;
        if (dpos[i] < 0) { free(dpos); return 1; }
    }
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t kk = rp[i]; kk < rp[i + 1] && ci[kk] < i; ++kk) {
            const int64_t k = ci[kk];
            lu[kk] = lu[kk] / lu[dpos[k]];
            const double lik = lu[kk];
            /* row k's entries right of column k, merged with row i's right of kk */
            int64_t p = dpos[k] + 1;
            for (int64_t jj = kk + 1; jj < rp[i + 1]; ++jj) {
                while (p < rp[k + 1] && ci[p] < ci[jj]) ++p;
                if (p < rp[k + 1] && ci[p] == ci[jj]) lu[jj] -= lik * lu[p];
            }
        }
        const double d = lu[dpos[i]];
        if (!(d != 0.0) || !isfinite(d)) { free(dpos); return 1; }
    }
    free(dpos);
    return 0;
}

/*
 * A multicolour order of the symmetrized pattern (A + A^T, diagonal ignored):
 * nodes in index order each take the smallest colour that none of their
 * already coloured neighbours has.  perm[new] = old lists colour 0 first,
 * then colour 1, ..., index order within a colour; colour_ptr[c] is the first
 * new index of colour c (colour_ptr[ncolours] = n).  No two neighbours share
 * a colour, so in this order the rows of one colour have no entries in each
 * other's columns.  Returns the number of colours, or -1 on allocation
 * failure.  colour_ptr needs room for n + 1 entries.
 */
int orc_multicolour(int64_t n, const int32_t *rp, const int32_t *ci, int32_t *perm, int32_t *colour_ptr)
{
    const int64_t nnz = rp[n];
    int32_t *tp = calloc((size_t)n + 1, sizeof(int32_t));
    int32_t *tc = malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    int32_t *col = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t *mark = malloc(sizeof(int64_t) * (size_t)(n + 1));
    int32_t *fill = calloc((size_t)n + 1, sizeof(int32_t));
    if (!tp || !tc || !col || !mark || !fill) {
        free(tp); free(tc); free(col); free(mark); free(fill);
        return -1;
    }
    /* transposed pattern */
    for (int64_t k = 0; k < nnz; ++k) tp[ci[k] + 1]++;
    for (int64_t i = 0; i < n; ++i) tp[i + 1] += tp[i];
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) tc[tp[ci[k]] + fill[ci[k]]++] = (int32_t)i;
    int ncol = 0;
    for (int64_t c = 0; c <= n; ++c) mark[c] = -1;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
            if (ci[k] < i) mark[col[ci[k]]] = i;
        for (int64_t k = tp[i]; k < tp[i + 1]; ++k)
            if (tc[k] < i) mark[col[tc[k]]] = i;
        int c = 0;
        while (mark[c] == i) ++c;
        col[i] = c;
        if (c + 1 > ncol) ncol = c + 1;
    }
    for (int c = 0; c <= ncol; ++c) colour_ptr[c] = 0;
    for (int64_t i = 0; i < n; ++i) colour_ptr[col[i] + 1]++;
    for (int c = 0; c < ncol; ++c) colour_ptr[c + 1] += colour_ptr[c];
    for (int c = 0; c <= ncol; ++c) fill[c] = 0;
    for (int64_t i = 0; i < n; ++i) perm[colour_ptr[col[i]] + fill[col[i]]++] = (int32_t)i;
    free(tp); free(tc); free(col); free(mark); free(fill);
    return ncol;
}

void orc_spmv(int64_t n, const int32_t *rp, const int32_t *ci, const double *va,
              const double *x, double *y)
{
    Mat A = {n, rp, ci, va, 0, NULL, NULL};
    matvec(&A, x, y);
}

/* Inner products are plain sums in one of three orders: 0 from the first
 * index to the last (the default), 1 from the last to the first, 2 in blocks
 * of 256 consecutive terms, each summed from its first term, whose sums are
 * then added pairwise (a balanced tree over the blocks).  All three compute the
 * same definition; the tests compare them to measure how much the iteration
 * amplifies rounding alone. */
static _Thread_local int sum_order = 0;   /* per calling thread */

void orc_set_sum_order(int order) { sum_order = (order == 1 || order == 2) ? order : 0; }

#define ORC_SUM_BLOCK 256

static double tree_sum(const double *v, int64_t m)
{
    if (m == 1) return v[0];
    int64_t h = m / 2;
    return tree_sum(v, h) + tree_sum(v + h, m - h);
}

static double dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    if (sum_order == 1) {
        for (int64_t i = n - 1; i >= 0; --i) s += a[i] * b[i];
    } else if (sum_order == 2 && n > 0) {
        int64_t nb = (n + ORC_SUM_BLOCK - 1) / ORC_SUM_BLOCK;
        double *blk = (double *)malloc((size_t)nb * sizeof(double));
        if (!blk) abort();
        for (int64_t k = 0; k < nb; ++k) {
            double t = 0.0;
            int64_t e = (k + 1) * ORC_SUM_BLOCK < n ? (k + 1) * ORC_SUM_BLOCK : n;
            for (int64_t i = k * ORC_SUM_BLOCK; i < e; ++i) t += a[i] * b[i];
            blk[k] = t;
        }
        s = tree_sum(blk, nb);
        free(blk);
    } else {
        for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    }
    return s;
}

/* Solve the m x m system M c = g (M row-major, copied) by Gaussian elimination
 * with partial pivoting.  Returns 0, or 1 when a pivot is <= 1e-14 times the
 * largest magnitude in its column of M (a column-scale-invariant test: the
 * columns of P^T V can differ by many orders of magnitude when recycled data
 * meet a fresh residual). */
static int lu_solve(int m, const double *Min, const double *g, double *c)
{
    double M[64], y[8], cmax[8];
    for (int j = 0; j < m; ++j) cmax[j] = 0.0;
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
            M[i * m + j] = Min[i * m + j];
            if (fabs(M[i * m + j]) > cmax[j]) cmax[j] = fabs(M[i * m + j]);
        }
    for (int i = 0; i < m; ++i) y[i] = g[i];
    for (int k = 0; k < m; ++k) {
        int piv = k;
        for (int i = k + 1; i < m; ++i)
            if (fabs(M[i * m + k]) > fabs(M[piv * m + k])) piv = i;
        if (!(fabs(M[piv * m + k]) > 1e-14 * cmax[k])) return 1;
        if (piv != k) {
            for (int j = 0; j < m; ++j) {
                double t = M[k * m + j]; M[k * m + j] = M[piv * m + j]; M[piv * m + j] = t;
            }
            double t = y[k]; y[k] = y[piv]; y[piv] = t;
        }
        for (int i = k + 1; i < m; ++i) {
            double f = M[i * m + k] / M[k * m + k];
            for (int j = k + 1; j < m; ++j) M[i * m + j] -= f * M[k * m + j];
            y[i] -= f * y[k];
        }
    }
    for (int i = m - 1; i >= 0; --i) {
        double acc = y[i];
        for (int j = i + 1; j < m; ++j) acc -= M[i * m + j] * c[j];
        c[i] = acc / M[i * m + i];
    }
    return 0;
}

/* Least squares through the normal equations G t = c (G SPD, row-major). */
static int spd_solve(int m, const double *G, const double *c, double *t)
{
    double L[64], y[8];
    int ok = 1;
    memset(L, 0, sizeof(L));
    for (int j = 0; j < m && ok; ++j) {
        double d = G[j * m + j];
        for (int k = 0; k < j; ++k) d -= L[j * m + k] * L[j * m + k];
        if (!(d > 0.0)) { ok = 0; break; }
        L[j * m + j] = sqrt(d);
        for (int i = j + 1; i < m; ++i) {
            double e = G[i * m + j];
            for (int k = 0; k < j; ++k) e -= L[i * m + k] * L[j * m + k];
            L[i * m + j] = e / L[j * m + j];
        }
    }
    if (!ok) return lu_solve(m, G, c, t);
    for (int i = 0; i < m; ++i) {
        double acc = c[i];
        for (int k = 0; k < i; ++k) acc -= L[i * m + k] * y[k];
        y[i] = acc / L[i * m + i];
    }
    for (int i = m - 1; i >= 0; --i) {
        double acc = y[i];
        for (int k = i + 1; k < m; ++k) acc -= L[k * m + i] * t[k];
        t[i] = acc / L[i * m + i];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1 with the recycling protocol                                   */
/* ------------------------------------------------------------------------ */

typedef struct {
    Mat A;
    int s, ell;
    int64_t n;
    const double *P;   /* n x s, column-major */
    double *W;         /* levels -1..ell of the s auxiliary vectors */
    double *R;         /* levels 0..ell of the residual */
} Work;

#define WCOL(w, i, q) ((w)->W + ((int64_t)((i) + 1) * (w)->s + (q)) * (w)->n)
#define RCOL(w, i) ((w)->R + (int64_t)(i) * (w)->n)

/* out[a] = p_a . y */
static void project(const Work *w, const double *y, double *out)
{
    for (int a = 0; a < w->s; ++a) out[a] = dot(w->n, w->P + (int64_t)a * w->n, y);
}

/* Arnoldi basis of level s for the residual r: U orthonormal, V = A U. */
static int arnoldi(Work *w, const double *r)
{
    int64_t n = w->n;
    int s = w->s;
    double nr = sqrt(dot(n, r, r));
    if (!(nr > 0.0)) return 1;
    double *u1 = WCOL(w, -1, 0);
    for (int64_t e = 0; e < n; ++e) u1[e] = r[e] / nr;
    for (int q = 0; q < s; ++q) {
        double *uq = WCOL(w, -1, q), *vq = WCOL(w, 0, q);
        matvec(&w->A, uq, vq);
        if (q + 1 < s) {
            double *un = WCOL(w, -1, q + 1);
            memcpy(un, vq, (size_t)n * sizeof(double));
            for (int j = 0; j <= q; ++j) {
                const double *uj = WCOL(w, -1, j);
                double h = dot(n, uj, un);
                for (int64_t e = 0; e < n; ++e) un[e] -= h * uj[e];
            }
            double nn = sqrt(dot(n, un, un));
            if (!(nn > 1e-14 * sqrt(dot(n, vq, vq)))) return 1;
            for (int64_t e = 0; e < n; ++e) un[e] /= nn;
        }
    }
    return 0;
}

/*
 * One cycle of Algorithm 1 (the while-loop body), in place.
 * On entry R[0] = r, x = x, W[-1] = U, W[0] = V.  On exit R[0] = new r,
 * W[-1] = new U, W[0] = new V, x updated.  Returns 0 or 1 (breakdown).
 * If dump != NULL the state after the level loop is copied there before the
 * degree-l minimization, followed by tau.
 */
/*
 * The gamma step of level k: gamma such that r^(k) - V^(k) gamma is orthogonal
 * to P, then r^(i) -= V^(i) gamma for i = 0..k and x += U gamma.  At k = 0 with
 * recycled U, V this is the projection of a new right-hand side onto the
 * recycled data (Section 4.2).  Returns 1 on a singular P^T V^(k).
 */
static int gamma_step(Work *w, int k, double *x)
{
    const int s = w->s;
    const int64_t n = w->n;
    double M[64], g[8], c[8], colp[8][8];
    for (int q = 0; q < s; ++q) project(w, WCOL(w, k, q), colp[q]);
    for (int a = 0; a < s; ++a)
        for (int q = 0; q < s; ++q) M[a * s + q] = colp[q][a];
    project(w, RCOL(w, k), g);
    if (lu_solve(s, M, g, c)) return 1;
    for (int i = 0; i <= k; ++i) {
        double *ri = RCOL(w, i);
        for (int q = 0; q < s; ++q) {
            const double *vq = WCOL(w, i, q);
            for (int64_t e = 0; e < n; ++e) ri[e] -= c[q] * vq[e];
        }
    }
    for (int q = 0; q < s; ++q) {
        const double *uq = WCOL(w, -1, q);
        for (int64_t e = 0; e < n; ++e) x[e] += c[q] * uq[e];
    }
    return 0;
}

static int cycle(Work *w, double *x, double *dump)
{
    const int s = w->s, ell = w->ell;
    const int64_t n = w->n;
    double M[64], g[8], c[8], colp[8][8];

    for (int k = 0; k < ell; ++k) {
        if (gamma_step(w, k, x)) return 1;
        matvec(&w->A, RCOL(w, k), RCOL(w, k + 1));

        for (int q = 0; q < s; ++q) {
            /* eta_q: r^(k+1) - [V^(k+1)_{1:q-1}, V^(k)_{q:s}] eta orthogonal to P */
            for (int p = 0; p < s; ++p) project(w, WCOL(w, p < q ? k + 1 : k, p), colp[p]);
            for (int a = 0; a < s; ++a)
                for (int p = 0; p < s; ++p) M[a * s + p] = colp[p][a];
            project(w, RCOL(w, k + 1), g);
            if (lu_solve(s, M, g, c)) return 1;
            /* v_q^(i) := r^(i+1) - [V^(i+1)_{1:q-1}, V^(i)_{q:s}] eta, i = -1..k */
            for (int i = -1; i <= k; ++i) {
                double *vq = WCOL(w, i, q);
                const double *rr = RCOL(w, i + 1);
                for (int64_t e = 0; e < n; ++e) {
                    double acc = rr[e];
                    for (int p = 0; p < s; ++p) {
                        const double *src = (p < q) ? WCOL(w, i + 1, p) : WCOL(w, i, p);
                        acc -= c[p] * src[e];
                    }
                    vq[e] = acc;
                }
            }
            matvec(&w->A, WCOL(w, k, q), WCOL(w, k + 1, q));
        }
    }

    /* degree-l residual minimization: tau = Z^+ r^(0), Z = [r^(1..l)] */
    double G[64], t[8], cc[8];
    for (int i = 0; i < ell; ++i) {
        for (int j = 0; j < ell; ++j) G[i * ell + j] = dot(n, RCOL(w, i + 1), RCOL(w, j + 1));
        cc[i] = dot(n, RCOL(w, i + 1), RCOL(w, 0));
    }
    if (spd_solve(ell, G, cc, t)) return 1;

    if (dump) {
        double *d = dump;
        memcpy(d, x, (size_t)n * sizeof(double)); d += n;
        memcpy(d, w->R, (size_t)n * (ell + 1) * sizeof(double)); d += n * (ell + 1);
        memcpy(d, w->W, (size_t)n * s * (ell + 2) * sizeof(double)); d += (int64_t)n * s * (ell + 2);
        for (int i = 0; i < ell; ++i) d[i] = t[i];
    }

    /* x := x^(0) + sum_i tau_i r^(i-1)        (before r^(0) changes) */
    for (int i = 1; i <= ell; ++i) {
        const double *ri = RCOL(w, i - 1);
        for (int64_t e = 0; e < n; ++e) x[e] += t[i - 1] * ri[e];
    }
    /* u_q := v_q^(-1) - sum_i tau_i v_q^(i-1) (before v_q^(0) changes) */
    for (int q = 0; q < s; ++q) {
        double *uq = WCOL(w, -1, q);
        for (int i = 1; i <= ell; ++i) {
            const double *vi = WCOL(w, i - 1, q);
            for (int64_t e = 0; e < n; ++e) uq[e] -= t[i - 1] * vi[e];
        }
    }
    /* v_q := v_q^(0) - sum_i tau_i v_q^(i) */
    for (int q = 0; q < s; ++q) {
        double *vq = WCOL(w, 0, q);
        for (int i = 1; i <= ell; ++i) {
            const double *vi = WCOL(w, i, q);
            for (int64_t e = 0; e < n; ++e) vq[e] -= t[i - 1] * vi[e];
        }
    }
    /* r := r^(0) - sum_i tau_i r^(i) */
    {
        double *r0 = RCOL(w, 0);
        for (int i = 1; i <= ell; ++i) {
            const double *ri = RCOL(w, i);
            for (int64_t e = 0; e < n; ++e) r0[e] -= t[i - 1] * ri[e];
        }
    }
    return 0;
}

/*
 * Orthonormalize recycled data (not in the paper: an option of this build,
 * applied where a solve fetches U, V).  CholQR in FP64: G = U^T U = R^T R
 * (Cholesky, R upper triangular), then U := U R^{-1} and V := V R^{-1},
 * column by column by forward substitution (u'_j = (u_j - sum_{i<j} R_ij u'_i)
 * / R_jj).  U^T U becomes I, V = A U is kept (V R^{-1} = A U R^{-1}), and the
 * ranges of U and V do not change, so the projection of the next right-hand
 * side onto the recycled data is the same in exact arithmetic.  V may be NULL
 * (U only).  Returns 1, leaving U and V untouched, when G is not numerically
 * positive definite (a pivot d <= 0 or d <= 1e-28 G_jj).
 */
int orc_cholqr(int64_t n, int s, double *U, double *V)
{
    if (n < 1 || s < 1 || s > 8 || !U) return -1;
    double G[64], L[64];
    for (int i = 0; i < s; ++i)
        for (int j = i; j < s; ++j) {
            G[i * s + j] = dot(n, U + (int64_t)i * n, U + (int64_t)j * n);
            G[j * s + i] = G[i * s + j];
        }
    /* G = L L^T, L lower; R = L^T */
    memset(L, 0, sizeof(L));
    for (int j = 0; j < s; ++j) {
        double d = G[j * s + j];
        for (int k = 0; k < j; ++k) d -= L[j * s + k] * L[j * s + k];
        if (!(d > 0.0) || !(d > 1e-28 * G[j * s + j])) return 1;
        L[j * s + j] = sqrt(d);
        for (int i = j + 1; i < s; ++i) {
            double e = G[i * s + j];
            for (int k = 0; k < j; ++k) e -= L[i * s + k] * L[j * s + k];
            L[i * s + j] = e / L[j * s + j];
        }
    }
    for (int m = 0; m < (V ? 2 : 1); ++m) {
        double *B = m == 0 ? U : V;
        for (int j = 0; j < s; ++j) {
            double *bj = B + (int64_t)j * n;
            for (int64_t e = 0; e < n; ++e) {
                double acc = bj[e];
                for (int i = 0; i < j; ++i) acc -= L[j * s + i] * B[(int64_t)i * n + e];
                bj[e] = acc / L[j * s + j];
            }
        }
    }
    return 0;
}

/*
 * The projection of a right-hand side onto recycled data (Section 4.2: the
 * first gamma step of a solve that starts from a former solve's U, V):
 * gamma with r - V gamma orthogonal to P, then r -= V gamma, x += U gamma, in
 * place.  P, U, V: n x s column-major.  Returns 1 on a singular P^T V.
 */
int orc_recycle_start(int64_t n, int s, const double *P, const double *U, const double *V,
                      double *r, double *x)
{
    if (n <= 0 || s < 1 || s > 8) return -1;
    Work w;
    w.A.n = n; w.A.rp = NULL; w.A.ci = NULL; w.A.va = NULL; w.A.mv = 0;
    w.A.lu = NULL; w.A.tmp = NULL;
    w.s = s; w.ell = 1; w.n = n; w.P = P;
    w.W = (double *)calloc((size_t)n * s * 3, sizeof(double));
    w.R = (double *)calloc((size_t)n * 2, sizeof(double));
    if (!w.W || !w.R) { free(w.W); free(w.R); return ORC_E_NOMEM; }
    memcpy(WCOL(&w, -1, 0), U, (size_t)n * s * sizeof(double));
    memcpy(WCOL(&w, 0, 0), V, (size_t)n * s * sizeof(double));
    memcpy(RCOL(&w, 0), r, (size_t)n * sizeof(double));
    int bd = gamma_step(&w, 0, x);
    if (!bd) memcpy(r, RCOL(&w, 0), (size_t)n * sizeof(double));
    free(w.W); free(w.R);
    return bd;
}

/*
 * The fetch point "shortly before the residual drops" (Section 5, how to
 * choose the fetching point), estimated from a finished solve's convergence:
 * the cycle k* with the largest one-cycle reduction of the recursive
 * residual, res[k-1] / res[k] over cycles k >= 1 of the history (the first
 * such cycle on ties), and the fetch at the end of the cycle before it,
 * max(1, k* - 1).  hist_res[0] is the initial residual, hist_res[k] the one
 * after cycle k.  Returns -1 when the solve ran no cycle.
 */
int64_t orc_estimate_fetch_cycle(const double *hist_res, int64_t len)
{
    int64_t best_k = -1;
    double best = -1.0;
    for (int64_t k = 1; k < len; ++k) {
        const double f = hist_res[k] > 0.0 ? hist_res[k - 1] / hist_res[k] : INFINITY;
        if (f > best) { best = f; best_k = k; }
    }
    if (best_k < 0) return -1;
    return best_k > 1 ? best_k - 1 : 1;
}

/*
 * Solve A x = b (x holds x0 on entry).
 *
 * Recycle state (U, V: n x s column-major, *rec_level, *rec_have) is read when
 * method == ORC_MSTAB and *rec_have, and written at the fetch point chosen by
 * `fetch` (left unchanged if the policy never fires).
 *
 * out_i64[0..8]: mv (initial + Arnoldi + cycles), mv_check, cycles, level of
 *                the final U,V, fetched level (-1 if none), converged,
 *                recycled (started from recycled data), restarts, replacements
 * out_f64[0..1]: final recursive and true relative residual
 * hist: (total MVs, recursive relative residual) after the initial residual
 *       and after every cycle.
 * est_cycle (FETCH_ESTIMATE; in/out): the fetch cycle estimated from the
 *       previous solve of the sequence (-1: none yet, so this solve fetches
 *       nothing and the next one starts like IDR(s)stab); this solve fetches
 *       at the end of that cycle (or of its last one, if it stops earlier),
 *       and on return holds the estimate from this solve's history.
 * dump: if dump_cycle >= 0, the state after the level loop of that cycle:
 *       x, R[0..l], W[-1..l] (n each) then tau (l values); after it, the
 *       state after the same cycle's update: x, r, U, V.
 */
int orc_solve(int64_t n, const int32_t *rp, const int32_t *ci, const double *va,
              int s, int ell, const double *P,
              double tol, int64_t max_mv, int method, int fetch, double fetch_rel,
              int64_t fetch_level, int max_repl, int replace_every, int orth,
              const double *b, double *x,
              double *U, double *V, int64_t *rec_level, int *rec_have,
              int64_t *out_i64, double *out_f64,
              int64_t *hist_mv, double *hist_res, int64_t hist_cap, int64_t *hist_len,
              int64_t dump_cycle, double *dump, int64_t *est_cycle, const double *ilu)
{
    if (n <= 0 || s < 1 || s > 8 || ell < 1 || ell > 8 || n <= s) return ORC_E_INVALID;
    Work w;
    w.A.n = n; w.A.rp = rp; w.A.ci = ci; w.A.va = va; w.A.mv = 0;
    w.A.lu = ilu; w.A.tmp = NULL;
    w.s = s; w.ell = ell; w.n = n; w.P = P;
    w.W = (double *)calloc((size_t)n * s * (ell + 2), sizeof(double));
    w.R = (double *)calloc((size_t)n * (ell + 1), sizeof(double));
    double *t = (double *)calloc((size_t)n, sizeof(double));
    if (ilu) w.A.tmp = (double *)calloc((size_t)n, sizeof(double));
    if (!w.W || !w.R || !t || (ilu && !w.A.tmp)) {
        free(w.W); free(w.R); free(t); free(w.A.tmp);
        return ORC_E_NOMEM;
    }

    const int64_t est_in = est_cycle ? *est_cycle : -1;
    int64_t mv_check = 0, cycles = 0, hl = 0, fetched = -1, level = 0;
    int converged = 0, recycled = 0, restarts = 0, repl = 0, repl_end = 0, status = ORC_OK;
    int64_t since_true = 0;   /* cycles since r was last the true residual */
    double rr = 0.0, relres_true = -1.0;
    const double tol2 = tol * tol;

#define HIST(res) do { if (hl < hist_cap) { hist_mv[hl] = w.A.mv + mv_check; hist_res[hl] = (res); } ++hl; } while (0)

    double nb2 = dot(n, b, b);
    if (!isfinite(nb2)) { status = ORC_E_NONFINITE; goto done; }
    if (nb2 == 0.0) {
        memset(x, 0, (size_t)n * sizeof(double));
        converged = 1; rr = 0.0; relres_true = 0.0;
        goto done;
    }

    double *r = RCOL(&w, 0);
    matvec(&w.A, x, r);
    for (int64_t e = 0; e < n; ++e) r[e] = b[e] - r[e];
    rr = dot(n, r, r);
    int r_is_true = 1;
    HIST(sqrt(rr / nb2));
    if (!isfinite(rr)) { status = ORC_E_NONFINITE; goto done; }

    int have_uv = 0;
    if (method == ORC_MSTAB && *rec_have) {
        memcpy(WCOL(&w, -1, 0), U, (size_t)n * s * sizeof(double));
        memcpy(WCOL(&w, 0, 0), V, (size_t)n * s * sizeof(double));
        level = *rec_level;
        have_uv = 1;
        recycled = 1;
    }

    for (;;) {
        while (rr > tol2 * nb2 && w.A.mv < max_mv) {
            if (!have_uv) {
                if (arnoldi(&w, r)) { status = ORC_E_BREAKDOWN; goto done; }
                have_uv = 1;
                level = 0;
                continue; /* re-check the MV budget */
            }
            int bd = cycle(&w, x, (cycles == dump_cycle) ? dump : NULL);
            if (bd) {
                if (restarts < ORC_MAX_RESTARTS) {
                    /* drop U, V (recycled or not) and restart from the true
                     * residual of the current x with a fresh Arnoldi basis */
                    ++restarts;
                    have_uv = 0;
                    matvec(&w.A, x, r);
                    for (int64_t e = 0; e < n; ++e) r[e] = b[e] - r[e];
                    r_is_true = 1;
                    since_true = 0;
                    rr = dot(n, r, r);
                    if (!isfinite(rr)) { status = ORC_E_NONFINITE; goto done; }
                    continue;
                }
                status = ORC_E_BREAKDOWN;
                goto done;
            }
            ++cycles;
            level += ell;
            r_is_true = 0;
            rr = dot(n, r, r);
            if (!isfinite(rr)) { status = ORC_E_NONFINITE; goto done; }
            if (cycles - 1 == dump_cycle && dump) {
                double *d = dump + (int64_t)n * (2 + ell + s * (ell + 2)) + ell;
                memcpy(d, x, (size_t)n * sizeof(double)); d += n;
                memcpy(d, r, (size_t)n * sizeof(double)); d += n;
                memcpy(d, WCOL(&w, -1, 0), (size_t)n * 2 * s * sizeof(double));
            }
            ++since_true;
            if (replace_every > 0 && since_true >= replace_every && rr > tol2 * nb2 &&
                w.A.mv < max_mv) {
                /* periodic replacement after the solution update */
                Mat Ap = w.A;
                matvec(&Ap, x, r);
                ++mv_check;
                for (int64_t e = 0; e < n; ++e) r[e] = b[e] - r[e];
                rr = dot(n, r, r);
                if (!isfinite(rr)) { status = ORC_E_NONFINITE; goto done; }
                r_is_true = 1;
                since_true = 0;
                ++repl;
            }
            HIST(sqrt(rr / nb2));
            double rel = sqrt(rr / nb2);
            int fire = 0;
            switch (fetch) {
            case ORC_FETCH_THRESHOLD: fire = (fetched < 0 && rel <= fetch_rel); break;
            case ORC_FETCH_AT_LEVEL: fire = (level == fetch_level); break;
            case ORC_FETCH_ONCE: fire = (!*rec_have && fetched < 0 && rel <= fetch_rel); break;
            case ORC_FETCH_ESTIMATE: fire = (est_in > 0 && fetched < 0 && cycles == est_in); break;
            default: break;
            }
            if (fire) {
                memcpy(U, WCOL(&w, -1, 0), (size_t)n * s * sizeof(double));
                memcpy(V, WCOL(&w, 0, 0), (size_t)n * s * sizeof(double));
                if (orth) orc_cholqr(n, s, U, V);
                fetched = level;
            }
        }
        /* finish: the true residual decides */
        if (r_is_true) {
            relres_true = sqrt(rr / nb2);
            converged = rr <= tol2 * nb2;
            break;
        }
        Mat Ac = w.A;
        matvec(&Ac, x, t);
        ++mv_check;
        for (int64_t e = 0; e < n; ++e) t[e] = b[e] - t[e];
        double tt = dot(n, t, t);
        relres_true = sqrt(tt / nb2);
        if (!isfinite(tt)) { status = ORC_E_NONFINITE; goto done; }
        if (tt <= tol2 * nb2) { converged = 1; break; }
        if (rr <= tol2 * nb2 && repl_end < max_repl && w.A.mv < max_mv) {
            memcpy(r, t, (size_t)n * sizeof(double));
            rr = tt;
            r_is_true = 1;
            since_true = 0;
            ++repl;
            ++repl_end;
            continue;
        }
        break;
    }
    if (!converged && status == ORC_OK) status = ORC_NOT_CONVERGED;
    if (cycles > 0 && fetched < 0 && (fetch == ORC_FETCH_AT_END ||
                                      (fetch == ORC_FETCH_THRESHOLD) ||
                                      (fetch == ORC_FETCH_ONCE && !*rec_have) ||
                                      (fetch == ORC_FETCH_ESTIMATE && est_in > 0))) {
        memcpy(U, WCOL(&w, -1, 0), (size_t)n * s * sizeof(double));
        memcpy(V, WCOL(&w, 0, 0), (size_t)n * s * sizeof(double));
        if (orth) orc_cholqr(n, s, U, V);
        fetched = level;
    }
    if (fetched >= 0) { *rec_level = fetched; *rec_have = 1; }
    if (fetch == ORC_FETCH_ESTIMATE && est_cycle)
        *est_cycle = orc_estimate_fetch_cycle(hist_res, hl < hist_cap ? hl : hist_cap);

done:
    out_i64[0] = w.A.mv;
    out_i64[1] = mv_check;
    out_i64[2] = cycles;
    out_i64[3] = level;
    out_i64[4] = fetched;
    out_i64[5] = converged;
    out_i64[6] = recycled;
    out_i64[7] = restarts;
    out_i64[8] = repl;
    out_f64[0] = nb2 > 0.0 ? sqrt(rr / nb2) : 0.0;
    out_f64[1] = relres_true;
    *hist_len = hl;
    free(w.W); free(w.R); free(t); free(w.A.tmp);
    return status;
#undef HIST
}

/* ------------------------------------------------------------------------ */
/* Textbook BiCGStab (van der Vorst 1992) with shadow vector rhat, `iters`    */
/* iterations, no stopping test: the s = l = 1 special case pins the cycle.  */
/* ------------------------------------------------------------------------ */
int orc_bicgstab(int64_t n, const int32_t *rp, const int32_t *ci, const double *va,
                 const double *b, double *x, const double *rhat, int iters)
{
    Mat A = {n, rp, ci, va, 0, NULL, NULL};
    double *r = calloc((size_t)n, sizeof(double)), *p = calloc((size_t)n, sizeof(double));
    double *v = calloc((size_t)n, sizeof(double)), *sv = calloc((size_t)n, sizeof(double));
    double *tv = calloc((size_t)n, sizeof(double));
    if (!r || !p || !v || !sv || !tv) { free(r); free(p); free(v); free(sv); free(tv); return ORC_E_NOMEM; }
    matvec(&A, x, r);
    for (int64_t e = 0; e < n; ++e) r[e] = b[e] - r[e];
    double rho_old = 1.0, alpha = 1.0, omega = 1.0;
    for (int it = 0; it < iters; ++it) {
        double rho = dot(n, rhat, r);
        double beta = (rho / rho_old) * (alpha / omega);
        for (int64_t e = 0; e < n; ++e) p[e] = r[e] + beta * (p[e] - omega * v[e]);
        matvec(&A, p, v);
        alpha = rho / dot(n, rhat, v);
        for (int64_t e = 0; e < n; ++e) sv[e] = r[e] - alpha * v[e];
        matvec(&A, sv, tv);
        omega = dot(n, tv, sv) / dot(n, tv, tv);
        for (int64_t e = 0; e < n; ++e) x[e] += alpha * p[e] + omega * sv[e];
        for (int64_t e = 0; e < n; ++e) r[e] = sv[e] - omega * tv[e];
        rho_old = rho;
    }
    free(r); free(p); free(v); free(sv); free(tv);
    return ORC_OK;
}

/*
 * Restarted GMRES(m) (Saad and Schultz), one of the comparison methods of
 * Section 5.1, for A x = b from x (in/out).
 *
 * Each restart cycle starts from the true residual r = b - A x, beta = ||r||,
 * v_1 = r (1 / beta), g = beta e_1.  Arnoldi step j: w = A v_j, orthogonalized
 * against v_1..v_j by classical Gram-Schmidt applied twice (c = V^T w, then
 * w -= V c element by element in basis order; the Hessenberg column is the
 * sum of the two passes' c), h_{j+1,j} = ||w||.  The column is rotated by
 * the cycle's earlier Givens rotations, a new rotation (c, s) = (h_jj, h_{j+1,j})
 * / hypot(h_jj, h_{j+1,j}) zeroes h_{j+1,j}, and |g_{j+1}| after it is the
 * residual norm of the least-squares solution over the Krylov space.  The
 * cycle ends after m steps, when that estimate is <= tol ||b||, when
 * h_{j+1,j} = 0 (the Krylov space is invariant: the least-squares solution is
 * exact) or when the product budget is spent; then y solves the rotated
 * triangular system by back substitution and x += V y.  The next cycle's
 * true residual decides convergence (||r|| <= tol ||b||).  A zero rotation
 * denominator (h_jj = h_{j+1,j} = 0) ends the cycle before that column; a
 * cycle that keeps no column is a breakdown.  Every product with A counts,
 * the true residuals included.  A zero b gives x = 0 with no product.
 * ilu: optional split ILU(0) operator L^{-1} A U^{-1} (as orc_solve).
 *
 * out_i64[0..3]: mv, Arnoldi steps, restart cycles, converged
 * out_f64[0..1]: last estimate and true relative residual
 * hist: (MVs, relative residual) after the initial residual and after every
 *       Arnoldi step (the estimate).
 */
int orc_gmres(int64_t n, const int32_t *rp, const int32_t *ci, const double *va, int m,
              double tol, int64_t max_mv, const double *b, double *x,
              int64_t *out_i64, double *out_f64,
              int64_t *hist_mv, double *hist_res, int64_t hist_cap, int64_t *hist_len,
              const double *ilu)
{
    if (n <= 0 || m < 1) return ORC_E_INVALID;
    Mat A = {n, rp, ci, va, 0, ilu, NULL};
    double *V = calloc((size_t)n * (size_t)(m + 1), sizeof(double));
    double *w = calloc((size_t)n, sizeof(double));
    double *H = calloc((size_t)(m + 1) * (size_t)m, sizeof(double));   /* H[i * m + j] */
    double *cs = calloc((size_t)m, sizeof(double)), *sn = calloc((size_t)m, sizeof(double));
    double *g = calloc((size_t)(m + 1), sizeof(double)), *y = calloc((size_t)m, sizeof(double));
    double *c = calloc((size_t)(m + 1), sizeof(double));
    if (ilu) A.tmp = calloc((size_t)n, sizeof(double));
    int status = ORC_OK;
    int64_t steps = 0, cycles = 0, hl = 0;
    int converged = 0;
    double est = -1.0, relres_true = -1.0, nb = 0.0;
    if (!V || !w || !H || !cs || !sn || !g || !y || !c || (ilu && !A.tmp)) { status = ORC_E_NOMEM; goto done; }

#define GHIST(res) do { if (hl < hist_cap) { hist_mv[hl] = A.mv; hist_res[hl] = (res); } ++hl; } while (0)

    nb = sqrt(dot(n, b, b));
    if (!isfinite(nb)) { status = ORC_E_NONFINITE; goto done; }
    if (nb == 0.0) {
        for (int64_t e = 0; e < n; ++e) x[e] = 0.0;
        converged = 1;
        relres_true = 0.0;
        est = 0.0;
        goto done;
    }
    const double thr = tol * nb;
    for (;;) {
        /* the true residual */
        matvec(&A, x, V);
        for (int64_t e = 0; e < n; ++e) V[e] = b[e] - V[e];
        const double beta = sqrt(dot(n, V, V));
        if (!isfinite(beta)) { status = ORC_E_NONFINITE; break; }
        if (cycles == 0) GHIST(beta / nb);
        relres_true = beta / nb;
        if (beta <= thr) { converged = 1; break; }
        if (A.mv >= max_mv) break;
        const double inv = 1.0 / beta;
        for (int64_t e = 0; e < n; ++e) V[e] = V[e] * inv;
        for (int i = 0; i <= m; ++i) g[i] = 0.0;
        g[0] = beta;
        for (int64_t i = 0; i < (int64_t)(m + 1) * m; ++i) H[i] = 0.0;
        int k = 0;
        for (int j = 0; j < m; ++j) {
            const double *vj = V + (size_t)j * n;
            matvec(&A, vj, w);
            ++steps;
            for (int pass = 0; pass < 2; ++pass) {
                for (int i = 0; i <= j; ++i) c[i] = dot(n, V + (size_t)i * n, w);
                for (int64_t e = 0; e < n; ++e) {
                    double a = w[e];
                    for (int i = 0; i <= j; ++i) a = fma(-c[i], V[(size_t)i * n + e], a);
                    w[e] = a;
                }
                for (int i = 0; i <= j; ++i) H[i * m + j] += c[i];
            }
            const double hn = sqrt(dot(n, w, w));
            if (!isfinite(hn)) { status = ORC_E_NONFINITE; goto done; }
            for (int i = 0; i < j; ++i) {
                const double t = cs[i] * H[i * m + j] + sn[i] * H[(i + 1) * m + j];
                H[(i + 1) * m + j] = -sn[i] * H[i * m + j] + cs[i] * H[(i + 1) * m + j];
                H[i * m + j] = t;
            }
            const double d = hypot(H[j * m + j], hn);
            if (!(d > 0.0)) break;   /* singular on the Krylov space: keep columns 0..j-1 */
            cs[j] = H[j * m + j] / d;
            sn[j] = hn / d;
            H[j * m + j] = d;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            k = j + 1;
            est = fabs(g[j + 1]);
            GHIST(est / nb);
            if (est <= thr || !(hn > 0.0) || A.mv >= max_mv) break;
            const double ih = 1.0 / hn;
            double *vn = V + (size_t)(j + 1) * n;
            for (int64_t e = 0; e < n; ++e) vn[e] = w[e] * ih;
        }
        if (k == 0) { status = ORC_E_BREAKDOWN; break; }
        for (int i = k - 1; i >= 0; --i) {
            double a = g[i];
            for (int l = i + 1; l < k; ++l) a -= H[i * m + l] * y[l];
            y[i] = a / H[i * m + i];
        }
        for (int64_t e = 0; e < n; ++e) {
            double a = x[e];
            for (int i = 0; i < k; ++i) a = fma(y[i], V[(size_t)i * n + e], a);
            x[e] = a;
        }
        ++cycles;
    }
#undef GHIST
    if (status == ORC_OK && !converged) status = ORC_NOT_CONVERGED;
done:
    if (out_i64) {
        out_i64[0] = A.mv;
        out_i64[1] = steps;
        out_i64[2] = cycles;
        out_i64[3] = converged;
    }
    if (out_f64) {
        out_f64[0] = est < 0 ? -1.0 : est / (nb > 0 ? nb : 1.0);
        out_f64[1] = relres_true;
    }
    if (hist_len) *hist_len = hl;
    free(V); free(w); free(H); free(cs); free(sn); free(g); free(y); free(c); free(A.tmp);
    return status;
}
