// ILU(0) split preconditioning in a multicolour order (the incomplete LU
// factorization without fill-in that Section 5.1 of arXiv 1604.06043 uses in
// the split form L^-1 A R^-1 y = L^-1 b, x = R^-1 y, here with R = U).
//
// The matrix A' = Pi A Pi^T is ordered colour by colour (a greedy colouring
// of A's symmetrized pattern, done on the host), so that the rows of one
// colour have no entries in each other's columns.  Then:
//   - the factorization of the rows of colour c reads only rows of earlier
//     colours (final by then): one launch per colour, one thread per row;
//   - a solve with L (unit lower) visits the colours in order and one with U
//     in reverse, one launch per colour;
// and the operator of the iteration, L^-1 A' U^-1, is one upper solve, one
// product with A' and one lower solve, followed by the projection epilogue of
// the product kernels.  Every row follows the same operations in the same
// order as a sequential row-by-row implementation, so the factors and the
// operator are bit-exact against one.
#pragma once

#include "kernels.hpp"

namespace mstab {

// Rows [r0, r1) (one colour): ILU(0), IKJ form, in place on lu (A' values on
// entry).  Row i: for each k < i of its pattern in column order,
// l_ik = a_ik / u_kk, then a_ij -= l_ik u_kj for each j > k of row i that row k
// also holds (both rows sorted: a merge).  dpos[i]: position of row i's
// diagonal.  *bad (zero beforehand) is set if a pivot is zero or not finite.
__global__ __launch_bounds__(BLOCK) void k_ilu0_rows(int64_t r0, int64_t r1, const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ ci, double *lu,
                                                     const int32_t *__restrict__ dpos, int *bad)
{
#pragma clang fp contract(off)
    for (int64_t i = r0 + (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < r1;
         i += (int64_t)gridDim.x * BLOCK) {
        const int32_t end = rp[i + 1];
        for (int32_t kk = rp[i]; kk < end && ci[kk] < i; ++kk) {
            const int32_t k = ci[kk];
            const double lik = lu[kk] / lu[dpos[k]];
            lu[kk] = lik;
            const int32_t kend = rp[k + 1];
            int32_t p = dpos[k] + 1;
            for (int32_t jj = kk + 1; jj < end; ++jj) {
                const int32_t cj = ci[jj];
                while (p < kend && ci[p] < cj) ++p;
                if (p < kend && ci[p] == cj) lu[jj] = lu[jj] - lik * lu[p];
            }
        }
        const double d = lu[dpos[i]];
        if (!(d != 0.0) || !isfinite(d))
            __hip_atomic_store(bad, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Rows [r0, r1) of y := L^-1 y in place: y_i -= l_ik y_k over k < i in
// column order (the k lie in earlier colours, final by then).
__global__ __launch_bounds__(BLOCK) void k_ilu_lower_rows(int64_t r0, int64_t r1, const int32_t *__restrict__ rp,
                                                          const int32_t *__restrict__ ci,
                                                          const double *__restrict__ lu,
                                                          const int32_t *__restrict__ dpos, double *y)
{
#pragma clang fp contract(off)
    for (int64_t i = r0 + (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < r1;
         i += (int64_t)gridDim.x * BLOCK) {
        double acc = y[i];
        const int32_t d = dpos[i];
        for (int32_t k = rp[i]; k < d; ++k) acc = acc - lu[k] * y[ci[k]];
        y[i] = acc;
    }
}

// Rows [r0, r1) of x := U^-1 z: x_i = (z_i - sum_{j>i} u_ij x_j) / u_ii in
// column order (the j lie in later colours, final by then).
__global__ __launch_bounds__(BLOCK) void k_ilu_upper_rows(int64_t r0, int64_t r1, const int32_t *__restrict__ rp,
                                                          const int32_t *__restrict__ ci,
                                                          const double *__restrict__ lu,
                                                          const int32_t *__restrict__ dpos,
                                                          const double *__restrict__ z, double *x)
{
#pragma clang fp contract(off)
    for (int64_t i = r0 + (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < r1;
         i += (int64_t)gridDim.x * BLOCK) {
        double acc = z[i];
        const int32_t d = dpos[i], end = rp[i + 1];
        for (int32_t k = d + 1; k < end; ++k) acc = acc - lu[k] * x[ci[k]];
        x[i] = acc / lu[d];
    }
}

// y = U x (all rows): y_i = u_ii x_i + sum_{j>i} u_ij x_j in column order.
__global__ __launch_bounds__(BLOCK) void k_ilu_upper_mul(int64_t n, const int32_t *__restrict__ rp,
                                                         const int32_t *__restrict__ ci,
                                                         const double *__restrict__ lu,
                                                         const int32_t *__restrict__ dpos,
                                                         const double *__restrict__ x, double *__restrict__ y)
{
#pragma clang fp contract(off)
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        double acc = 0.0;
        const int32_t end = rp[i + 1];
        for (int32_t k = dpos[i]; k < end; ++k) acc = acc + lu[k] * x[ci[k]];
        y[i] = acc;
    }
}

// The end of a preconditioned product: y = t (or b - t for the residual
// roles), then the projection epilogue and the role's small solve, exactly
// as at the end of a product kernel.
template <typename T, int S>
__global__ __launch_bounds__(SPMV_BLOCK) void k_vec_out(int64_t n, const T *__restrict__ t,
                                                        const T *__restrict__ b, T *__restrict__ y,
                                                        Ctl *ctl, double *part, int stride, SpmvArgs a)
{
    if (ctl->st.flags) return;
    const bool resid = (a.act == ACT_RESID || a.act == ACT_TRUE);
    double vals[S + 2];
#pragma unroll
    for (int v = 0; v < S + 2; ++v) vals[v] = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * SPMV_BLOCK + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * SPMV_BLOCK)
        spmv_row_out<T, S>(r, t[r], resid, b, y, a.pkey, vals);
    spmv_finalize<S>(vals, ctl, part, stride, a);
}

}  // namespace mstab

namespace mstab {

// The factors in the product's sliced layout, for the solves of every
// product: the strictly lower entries of each row (L) and the strictly upper
// ones (U) each in 64-row slices, entry j of row r at sp[r / 64] + 64 j + r % 64
// (row lengths from A''s row pointer and the diagonal positions), and U's
// diagonal per row.  The j-th entries of a wavefront's 64 rows are one
// contiguous load.
struct IluSell {
    int64_t *lsp = nullptr, *usp = nullptr;   // n_slices + 1
    int32_t *lcol = nullptr, *ucol = nullptr;
    double *lval = nullptr, *uval = nullptr;
    double *udiag = nullptr;                  // n
};

// Copies the factors of rows [0, n) from CSR (lu) into the sliced arrays.
__global__ __launch_bounds__(BLOCK) void k_ilu_to_sell(int64_t n, const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ ci,
                                                       const double *__restrict__ lu,
                                                       const int32_t *__restrict__ dpos, IluSell f)
{
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        const int32_t b = rp[i], d = dpos[i], e = rp[i + 1];
        const int64_t lb = f.lsp[i / SLICE] + (i % SLICE), ub = f.usp[i / SLICE] + (i % SLICE);
        for (int32_t k = b; k < d; ++k) {
            f.lcol[lb + (int64_t)(k - b) * SLICE] = ci[k];
            f.lval[lb + (int64_t)(k - b) * SLICE] = lu[k];
        }
        for (int32_t k = d + 1; k < e; ++k) {
            f.ucol[ub + (int64_t)(k - d - 1) * SLICE] = ci[k];
            f.uval[ub + (int64_t)(k - d - 1) * SLICE] = lu[k];
        }
        f.udiag[i] = lu[d];
    }
}

// Rows [r0, r1) of y := L^-1 y in place from the sliced factors: the same
// operations in the same order as k_ilu_lower_rows.
__global__ __launch_bounds__(BLOCK) void k_ilu_lower_sell(int64_t r0, int64_t r1, const int32_t *__restrict__ rp,
                                                          const int32_t *__restrict__ dpos, IluSell f, double *y)
{
#pragma clang fp contract(off)
    for (int64_t i = r0 + (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < r1;
         i += (int64_t)gridDim.x * BLOCK) {
        double acc = y[i];
        const int32_t len = dpos[i] - rp[i];
        const int64_t base = f.lsp[i / SLICE] + (i % SLICE);
        for (int32_t j = 0; j < len; ++j) {
            const int64_t k = base + (int64_t)j * SLICE;
            acc = acc - f.lval[k] * y[f.lcol[k]];
        }
        y[i] = acc;
    }
}

// Rows [r0, r1) of x := U^-1 z from the sliced factors: the same operations
// in the same order as k_ilu_upper_rows.
__global__ __launch_bounds__(BLOCK) void k_ilu_upper_sell(int64_t r0, int64_t r1, const int32_t *__restrict__ rp,
                                                          const int32_t *__restrict__ dpos, IluSell f,
                                                          const double *__restrict__ z, double *x)
{
#pragma clang fp contract(off)
    for (int64_t i = r0 + (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < r1;
         i += (int64_t)gridDim.x * BLOCK) {
        double acc = z[i];
        const int32_t len = rp[i + 1] - dpos[i] - 1;
        const int64_t base = f.usp[i / SLICE] + (i % SLICE);
        for (int32_t j = 0; j < len; ++j) {
            const int64_t k = base + (int64_t)j * SLICE;
            acc = acc - f.uval[k] * x[f.ucol[k]];
        }
        x[i] = acc / f.udiag[i];
    }
}

}  // namespace mstab

namespace mstab {

// Eisenstat's form of the split operator.  Where ILU(0) modifies no
// off-diagonal entry (no k < min(i, j) couples rows i and j through both
// (i, k) and (k, j): a pattern without triangles, such as the 5- and 7-point
// stencils), the factors are L = I + L_A D_U^-1 and U = D_U + U_A with L_A, U_A
// the strictly lower and upper parts of A' and D_U the pivots, and
//   L^-1 A' U^-1 x = L^-1 (x + (D_A - 2 D_U) t) + D_U t,   t = U^-1 x
// (A' t = L_A t + D_A t + U_A t with U_A t = x - D_U t, and
// L^-1 L_A D_U^-1 = I - L^-1): the two triangular solves and no product with A'.
// Equal to the three-step form in exact arithmetic; rounded differently.

// *bad (zero beforehand) is set if some factor entry is not the one the
// form assumes: a strictly upper entry different from A''s, or a strictly
// lower one different from a_ik / u_kk (the factorization's own division).
__global__ __launch_bounds__(BLOCK) void k_ilu_check_eis(int64_t n, const int32_t *__restrict__ rp,
                                                         const int32_t *__restrict__ ci,
                                                         const double *__restrict__ va,
                                                         const double *__restrict__ lu,
                                                         const int32_t *__restrict__ dpos, int *bad)
{
#pragma clang fp contract(off)
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        const int32_t d = dpos[i];
        bool ok = true;
        for (int32_t k = rp[i]; k < d; ++k) ok = ok && (lu[k] == va[k] / lu[dpos[ci[k]]]);
        for (int32_t k = d + 1; k < rp[i + 1]; ++k) ok = ok && (lu[k] == va[k]);
        if (!ok) __hip_atomic_store(bad, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// dd = D_A - 2 D_U, du = D_U
__global__ __launch_bounds__(BLOCK) void k_ilu_eis_diag(int64_t n, const double *__restrict__ va,
                                                        const double *__restrict__ lu,
                                                        const int32_t *__restrict__ dpos, double *dd, double *du)
{
#pragma clang fp contract(off)
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        const double u = lu[dpos[i]];
        dd[i] = va[dpos[i]] - 2.0 * u;
        du[i] = u;
    }
}

// w = x + dd t
__global__ __launch_bounds__(BLOCK) void k_ilu_eis_mid(int64_t n, const double *__restrict__ x,
                                                       const double *__restrict__ t,
                                                       const double *__restrict__ dd, double *__restrict__ w)
{
#pragma clang fp contract(off)
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        w[i] = x[i] + dd[i] * t[i];
}

// The end of an Eisenstat-form product: y = v + du t (or b minus that for
// the residual roles), then the projection epilogue and the role's small
// solve, as k_vec_out.
template <typename T, int S>
__global__ __launch_bounds__(SPMV_BLOCK) void k_vec_out_eis(int64_t n, const T *__restrict__ v,
                                                            const T *__restrict__ t, const T *__restrict__ du,
                                                            const T *__restrict__ b, T *__restrict__ y,
                                                            Ctl *ctl, double *part, int stride, SpmvArgs a)
{
#pragma clang fp contract(off)
    if (ctl->st.flags) return;
    const bool resid = (a.act == ACT_RESID || a.act == ACT_TRUE);
    double vals[S + 2];
#pragma unroll
    for (int q = 0; q < S + 2; ++q) vals[q] = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * SPMV_BLOCK + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * SPMV_BLOCK)
        spmv_row_out<T, S>(r, v[r] + du[r] * t[r], resid, b, y, a.pkey, vals);
    spmv_finalize<S>(vals, ctl, part, stride, a);
}

}  // namespace mstab
