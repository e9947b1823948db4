// Restarted GMRES(m) (Saad and Schultz), the Krylov method the paper compares
// M(s)stab(l) with in Section 5.1: the kernels of one Arnoldi step and of the
// cycle's end.  The host loop (Engine::gmres) launches them, reads the
// residual estimate after every step and decides when a cycle ends.
//
// Arnoldi step j: w = A v_j (the product kernels, no projection state), then
// classical Gram-Schmidt applied twice: c = V^T w over the basis vectors in
// chunks of up to 32 (k_gm_dots), w -= V c element by element in basis order
// (k_gm_axpy), again, the second update also reducing ||w||^2; k_gm_column
// sums the two passes' coefficients into the Hessenberg column, rotates it by the cycle's earlier
// Givens rotations, forms the new rotation and updates g, whose entry j+1 is
// the residual norm of the least-squares solution.  At the cycle's end
// k_gm_solve back-substitutes the rotated triangular system and k_gm_axpy adds
// V y to x.
#pragma once

#include "kernels.hpp"

namespace mstab {

// Device state of a GMRES(m) cycle (doubles), laid out for m:
//   H[(m+1) m] row-major (H[i m + j]), cs[m], sn[m], g[m+1], y[m], c1[m+1],
//   c2[m+1], then GM_SCAL scalars.
enum : int { GM_HN = 0, GM_EST = 1, GM_SINGULAR = 2, GM_BETA = 3, GM_SCAL = 4 };
struct GmLayout {
    int m;
    __host__ __device__ int64_t H() const { return 0; }
    __host__ __device__ int64_t cs() const { return (int64_t)(m + 1) * m; }
    __host__ __device__ int64_t sn() const { return cs() + m; }
    __host__ __device__ int64_t g() const { return sn() + m; }
    __host__ __device__ int64_t y() const { return g() + m + 1; }
    __host__ __device__ int64_t c(int pass) const { return y() + m + (int64_t)pass * (m + 1); }
    __host__ __device__ int64_t scal() const { return c(2); }
    __host__ __device__ int64_t size() const { return scal() + GM_SCAL; }
};

// Basis vectors a launch of k_gm_dots or k_gm_axpy covers at most; the
// kernels come in widths CH = 8 and 32 (the narrow one for the first steps of
// a cycle and short restarts: fewer registers, more wavefronts per SIMD).
constexpr int GM_CHUNK = 32;

// out[j0 + i] = v_{j0+i} . w (i < nv <= CH) and ||w||^2 into ctl->st.aux.
// Workgroup partials, the last workgroup's fixed-order totals.
template <typename T, int CH>
__global__ __launch_bounds__(BLOCK) void k_gm_dots(int64_t ld, const T *__restrict__ V, int j0, int nv,
                                                   const T *__restrict__ w, double *out, Ctl *ctl,
                                                   double *part, int stride)
{
    if (ctl->st.flags) return;
    double acc[CH + 1];
#pragma unroll
    for (int v = 0; v <= CH; ++v) acc[v] = 0.0;
    const T *V0 = V + (int64_t)j0 * ld;
    for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < ld; e += (int64_t)gridDim.x * BLOCK) {
        const double wv = (double)w[e];
#pragma unroll
        for (int i = 0; i < CH; ++i)
            if (i < nv) acc[i] += (double)V0[(int64_t)i * ld + e] * wv;
        acc[CH] += wv * wv;
    }
    block_partials<CH + 1>(acc, CH + 1, part, stride);
    __shared__ double tot[CH + 1];
    if (!last_block_reduce(part, stride, CH + 1, &ctl->counter[3], ctl->gcount[3], tot)) return;
    if (threadIdx.x != 0) return;
    for (int i = 0; i < nv; ++i) out[j0 + i] = tot[i];
    ctl->st.aux = tot[CH];
    if (!isfinite(tot[CH])) ctl->st.flags |= FLAG_NONFINITE;
}

// w += sign * sum_{i<nv} coef[j0+i] v_{j0+i} (nv <= CH), one fused
// multiply-add per basis vector in basis order.  With norm, also ||w||^2 of
// the updated w into ctl->st.aux (the second Gram-Schmidt pass's last chunk:
// the norm that gives h_{j+1,j}), as k_gm_dots reduces it.
template <typename T, int CH>
__global__ __launch_bounds__(BLOCK) void k_gm_axpy(int64_t ld, const T *__restrict__ V, int j0, int nv,
                                                   const double *coef, double sign, T *w, Ctl *ctl, int norm,
                                                   double *part, int stride)
{
    if (ctl->st.flags) return;
    T c[CH];
#pragma unroll
    for (int i = 0; i < CH; ++i) c[i] = (i < nv) ? (T)(sign * coef[j0 + i]) : (T)0;
    const T *V0 = V + (int64_t)j0 * ld;
    double acc[1] = {0.0};
    for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < ld; e += (int64_t)gridDim.x * BLOCK) {
        T a = w[e];
#pragma unroll
        for (int i = 0; i < CH; ++i)
            if (i < nv) a = fmaT(c[i], V0[(int64_t)i * ld + e], a);
        w[e] = a;
        acc[0] += (double)a * (double)a;
    }
    if (!norm) return;
    block_partials<1>(acc, 1, part, stride);
    __shared__ double tot[1];
    if (!last_block_reduce(part, stride, 1, &ctl->counter[3], ctl->gcount[3], tot)) return;
    if (threadIdx.x != 0) return;
    ctl->st.aux = tot[0];
    if (!isfinite(tot[0])) ctl->st.flags |= FLAG_NONFINITE;
}

// Start of a cycle: beta = sqrt(||r||^2) (st.tt of the true-residual product),
// v_1 = r (1 / beta) in place, g = beta e_1, H = 0.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_gm_start(int64_t ld, T *v, double *state, int m, const Ctl *ctl)
{
    const GmLayout L{m};
    const double beta = sqrt(ctl->st.tt);
    const T inv = (T)(1.0 / beta);
    for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < ld; e += (int64_t)gridDim.x * BLOCK)
        v[e] = v[e] * inv;
    if (blockIdx.x == 0) {
        for (int64_t i = threadIdx.x; i < L.size(); i += BLOCK) state[i] = 0.0;
        __syncthreads();
        if (threadIdx.x == 0) {
            state[L.g()] = beta;
            state[L.scal() + GM_BETA] = beta;
        }
    }
}

// Column j of the Hessenberg matrix: h = c1 + c2 (the two Gram-Schmidt
// passes), h_{j+1,j} = sqrt(st.aux); the earlier rotations, then the new one
// ((c, s) = (h_jj, h_{j+1,j}) / hypot(h_jj, h_{j+1,j})), g_{j+1} = -s g_j,
// g_j = c g_j; GM_EST = |g_{j+1}|.  A zero denominator sets GM_SINGULAR and
// leaves g as it was.  One thread.
__global__ void k_gm_column(double *state, int m, int j, const Ctl *ctl)
{
#pragma clang fp contract(off)
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const GmLayout L{m};
    double *H = state + L.H(), *cs = state + L.cs(), *sn = state + L.sn(), *g = state + L.g();
    const double *c1 = state + L.c(0), *c2 = state + L.c(1);
    double *sc = state + L.scal();
    for (int i = 0; i <= j; ++i) H[i * m + j] = (0.0 + c1[i]) + c2[i];
    const double hn = sqrt(ctl->st.aux);
    sc[GM_HN] = hn;
    for (int i = 0; i < j; ++i) {
        const double t = cs[i] * H[i * m + j] + sn[i] * H[(i + 1) * m + j];
        H[(i + 1) * m + j] = -sn[i] * H[i * m + j] + cs[i] * H[(i + 1) * m + j];
        H[i * m + j] = t;
    }
    const double d = hypot(H[j * m + j], hn);
    if (!(d > 0.0)) {
        sc[GM_SINGULAR] = 1.0;
        return;
    }
    cs[j] = H[j * m + j] / d;
    sn[j] = hn / d;
    H[j * m + j] = d;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    sc[GM_EST] = fabs(g[j + 1]);
}

// v_{j+1} = w (1 / h_{j+1,j})
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_gm_scale(int64_t ld, const T *w, T *dst, const double *state, int m)
{
    const GmLayout L{m};
    const T ih = (T)(1.0 / state[L.scal() + GM_HN]);
    for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < ld; e += (int64_t)gridDim.x * BLOCK)
        dst[e] = w[e] * ih;
}

// y solves the rotated k x k upper triangular system R y = g (back
// substitution, the products subtracted in column order).  One thread.
__global__ void k_gm_solve(double *state, int m, int k)
{
#pragma clang fp contract(off)
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const GmLayout L{m};
    const double *H = state + L.H(), *g = state + L.g();
    double *y = state + L.y();
    for (int i = k - 1; i >= 0; --i) {
        double a = g[i];
        for (int l = i + 1; l < k; ++l) a -= H[i * m + l] * y[l];
        y[i] = a / H[i * m + i];
    }
}

}  // namespace mstab
