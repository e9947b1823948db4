// CSR assembly of the upwind finite-difference convection-diffusion matrix
//   A = inv_dt I - div(kappa grad .) + beta . grad
// on n^dim interior nodes (x fastest), one thread per row.  Row offsets come
// from a closed form (rows before i minus the rows that lack each neighbour),
// so no scan is needed.  Floating-point contraction is off in this file: every
// value is formed with the rounding order stated in mstab.h, which makes the
// result reproducible bit for bit by any IEEE-754 implementation of the same
// order.
#include "mstab.h"

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#pragma clang fp contract(off)

namespace {

constexpr int ABLOCK = 256;

// Number of entries in rows 0..i-1.
__host__ __device__ inline int64_t entries_before(int64_t i, int dim, int64_t n)
{
    const int64_t plane = n * n;
    int64_t cnt = i;                                            // diagonals
    // x: rows with cx == 0 lack -x (ceil(i/n) of them), rows with cx == n-1 lack +x
    cnt += i - (i + n - 1) / n;
    cnt += i - i / n;
    // y: per plane of n*n rows the first n lack -y, the last n lack +y
    {
        const int64_t full = i / plane, rem = i % plane;
        const int64_t lo = full * n + (rem < n ? rem : n);
        const int64_t hi_rem = rem - n * (n - 1);
        const int64_t hi = full * n + (hi_rem > 0 ? hi_rem : 0);
        cnt += i - lo;
        cnt += i - hi;
    }
    if (dim == 3) {
        const int64_t lo = i < plane ? i : plane;
        const int64_t hi_rem = i - plane * (n - 1);
        const int64_t hi = hi_rem > 0 ? hi_rem : 0;
        cnt += i - lo;
        cnt += i - hi;
    }
    return cnt;
}

__device__ inline double face_kappa(const double *kappa, int64_t a, int64_t b, bool interior)
{
    if (!kappa) return 1.0;
    if (!interior) return kappa[a];
    const double ka = kappa[a], kb = kappa[b];
    return (2.0 * ka * kb) / (ka + kb);
}

__global__ __launch_bounds__(ABLOCK) void k_assemble(int dim, int64_t n, int64_t N, double b0,
                                                     double b1, double b2, double inv_dt,
                                                     const double *__restrict__ kappa,
                                                     int32_t *__restrict__ row_ptr,
                                                     int32_t *__restrict__ col,
                                                     double *__restrict__ val)
{
    const double beta[3] = {b0, b1, b2};
    const double hinv = (double)(n + 1);
    const double hinv2 = hinv * hinv;
    const int64_t stride[3] = {1, n, n * n};
    for (int64_t i = (int64_t)blockIdx.x * ABLOCK + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * ABLOCK) {
        const int64_t c[3] = {i % n, (i / n) % n, dim == 3 ? i / (n * n) : 0};
        int64_t pos = entries_before(i, dim, n);
        row_ptr[i] = (int32_t)pos;
        if (i == N - 1) row_ptr[N] = (int32_t)entries_before(N, dim, n);
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
        for (int d = dim - 1; d >= 0; --d) {
            if (c[d] > 0) {
                const double bp = beta[d] > 0.0 ? beta[d] : 0.0;
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
                const double bm = beta[d] < 0.0 ? beta[d] : 0.0;
                col[pos] = (int32_t)(i + stride[d]);
                val[pos] = -(kf[d][1] * hinv2) + bm * hinv;
                ++pos;
            }
        }
    }
}

}  // namespace

extern "C" {

int64_t mstab_convdiff_nnz(int32_t dim, int64_t n)
{
    if ((dim != 2 && dim != 3) || n < 1) return -1;
    int64_t N = dim == 2 ? n * n : n * n * n;
    return entries_before(N, dim, n);
}

mstab_status mstab_assemble_convdiff(int32_t dim, int64_t n, const double *beta, double inv_dt,
                                     const double *kappa, int32_t *row_ptr, int32_t *col_idx,
                                     double *val, void *hip_stream)
{
    if ((dim != 2 && dim != 3) || n < 2 || !beta || !row_ptr || !col_idx || !val)
        return MSTAB_E_INVALID;
    const int64_t N = dim == 2 ? n * n : n * n * n;
    if (entries_before(N, dim, n) >= ((int64_t)1 << 31)) return MSTAB_E_INVALID;
    hipStream_t st = (hipStream_t)hip_stream;
    int64_t grid = (N + ABLOCK - 1) / ABLOCK;
    if (grid > 65536) grid = 65536;
    hipLaunchKernelGGL(k_assemble, dim3((unsigned)grid), dim3(ABLOCK), 0, st, (int)dim, n, N,
                       beta[0], beta[1], dim == 3 ? beta[2] : 0.0, inv_dt, kappa, row_ptr,
                       col_idx, val);
    if (hipGetLastError() != hipSuccess) return MSTAB_E_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return MSTAB_E_HIP;
    return MSTAB_OK;
}

}  // extern "C"
