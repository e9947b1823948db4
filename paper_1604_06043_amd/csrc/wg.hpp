// One workgroup per system: the whole solve of Algorithm 1 (initial residual,
// the Arnoldi start of Section 5's preliminaries or the recycled start of
// Section 4.2, the cycles, the true-residual replacements of Section 5.1, the
// fetch of U, V and the stopping test) in one kernel, with workgroup barriers
// between its steps and the small solves in LDS.  A grid of B workgroups
// advances B independent systems at once, so that systems too small to fill
// the chip (a 64 x 64 grid: 4096 rows) fill it together.
//
// The element operations are those of the grid-wide kernels (k_gamma, k_eta,
// k_eta_low, k_poly, the product), in the same order per element; the sums
// run over the workgroup's threads in a fixed order (each thread's rows in
// row order, then the wavefront's butterfly, then the wavefronts in index
// order), so results are deterministic and independent of the other systems
// of the launch.  The control flow is that of the host loop of the grid
// engine, taken by every thread on values read from LDS after a barrier.
//
// The matrix is read from the handle's device copy (diagonal storage with
// streamed or constant values, or sliced ELLPACK, as for the grid engine);
// products are rounded, then added in column order (contraction off), so a
// product equals the sequential CSR product bit for bit.
#pragma once

#include "kernels.hpp"
#include "mstab.h"

namespace mstab {
namespace wg {

#ifndef MSTAB_WG_NT
#define MSTAB_WG_NT 256
#endif
#ifndef MSTAB_WG_U
#define MSTAB_WG_U 4
#endif
constexpr int NT = MSTAB_WG_NT;                         // threads per workgroup
constexpr int NW = NT / 64;
constexpr int HIST = 256;                               // history entries kept per solve
constexpr int NV = (MAXL + 1) * (MAXL + 2) / 2;         // largest reduction (the Gram pairs)
constexpr int64_t MAX_N = (int64_t)1 << 20;

// One system of a launch: inputs set by the host, results written by thread 0.
struct Job {
    Sell<double> A;                     // the handle's device copy of the matrix
    const double *b;
    double *x;                          // x0 in, x out (n entries)
    double *W, *R, *T;                  // s(l+2), l+1 and 1 vectors of ld entries
    double *recU, *recV, *rec_ptv;      // recycle store (s vectors each; MAXS x MAXS)
    int64_t *hist_mv;                   // HIST entries, hist_stride apart
    double *hist_res;
    int64_t hist_stride;
    int64_t n, ld, max_mv, fetch_level;
    double tol, fetch_rel;
    PBasis pkey;
    int32_t s, ell, method, fetch, max_repl, replace_every;
    // recycle state, in and out
    int32_t rec_have;
    int64_t rec_level, est_cycle;
    // results
    int32_t status, converged, recycled, restarts, replacements;
    int64_t mv, mv_check, cycles, level, fetched, hist_len;
    double relres_rec, relres_true;
};

struct Shared {
    double red[NW][NV];
    double tot[NV];
    double ptv[MAXL + 1][MAXS][MAXS];   // [i][q][a] = p_a . v_q^(i)
    double ptr[MAXL + 1][MAXS];         // [i][a] = p_a . r^(i)
    double ptt[MAXS];
    double gamma[MAXS];
    double eta_all[MAXS][MAXS];         // [q][p]: eta of step q of the current level
    double tau[MAXL];
    double h[MAXS + 1];
    double rr, bb, tt, aux, aux0, thr2;
    int64_t mv;
    int32_t flags, where;
};

// Sum of vals[0..nv) over the workgroup into sh.tot (all threads call it).
template <int K>
__device__ __forceinline__ void reduce(double (&vals)[K], int nv, Shared &sh)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < K; ++v) {
        if (v < nv) {
            const double w = wave_sum(vals[v]);
            if (lane == 0) sh.red[wave][v] = w;
        }
    }
    __syncthreads();
    for (int v = threadIdx.x; v < nv; v += NT) {
        double a = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) a += sh.red[w][v];
        sh.tot[v] = a;
    }
    __syncthreads();
}

__device__ __forceinline__ bool all_finite(const Shared &sh, int nv)
{
    bool f = true;
    for (int v = 0; v < nv; ++v) f = f && isfinite(sh.tot[v]);
    return f;
}

__device__ __forceinline__ void set_flags(Shared &sh, int32_t flags, int32_t where)
{
    if (threadIdx.x == 0 && flags) {
        sh.flags |= flags;
        if (where) sh.where = where;
    }
}

// A value every thread of the workgroup holds alike (read from LDS after a
// barrier), moved to scalar registers: the control flow built on it is then
// visibly uniform and the value takes no vector registers.
__device__ __forceinline__ int32_t rfl(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t rfl(int64_t v)
{
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double rfl(double v)
{
    return __builtin_bit_cast(double, rfl(__builtin_bit_cast(int64_t, v)));
}

// S: s; LC: a bound on l (l <= LC <= MAXL) that sizes the per-thread arrays
// PM: where P's entries come from (pval_m: 1 the caller's matrix, 0 the
// generator), fixed per instantiation so that the row loops do not test it.
template <int S, int LC, int PM>
struct Solver {
    // rows a thread loads before it uses any of them (rows NT apart)
    static constexpr int U = S <= 4 ? MSTAB_WG_U : (MSTAB_WG_U + 1) / 2;
    const Job &J;
    Shared &sh;
    int n, ell;
    int64_t ld;
    double *W, *R;
    PBasis pk;

    __device__ Solver(const Job &j, Shared &s) : J(j), sh(s)
    {
        pk = j.pkey;
        n = (int)j.n;
        ld = j.ld;
        ell = j.ell;
        W = j.W;
        R = j.R;
    }
    __device__ double *Wc(int lev, int q) const { return W + ((int64_t)(lev + 1) * S + q) * ld; }
    __device__ double *Rc(int i) const { return R + (int64_t)i * ld; }

    // The rows of a thread for a matrix in diagonal storage with at most 8
    // diagonals: the loads of UU rows (gathers, and the values unless they are
    // constant) are issued before any is used; present entries are added in
    // ascending column order.  out(e, sum, b_e) finishes row e.
    template <bool CST, int UU, typename Out>
    __device__ __forceinline__ void dia_block(const Sell<double> &A, int nd, const double *src, Out &out)
    {
#pragma clang fp contract(off)
        const bool resid = out.resid;
        for (int e0 = threadIdx.x; e0 < n; e0 += UU * NT) {
            double v[CST ? 1 : UU][8], xv[UU][8], bv[UU];
#pragma unroll
            for (int u = 0; u < UU; ++u) {
                const int e = e0 + u * NT;
                const int er = e < n ? e : e0;
#pragma unroll
                for (int d = 0; d < 8; ++d) {
                    if (d < nd) {
                        const int64_t c = er + A.doff.off[d];
                        if constexpr (!CST) v[u][d] = A.dval[dia_index(er, d, nd)];
                        xv[u][d] = (c >= 0 && c < n) ? src[c] : 0.0;
                    }
                }
                bv[u] = resid ? J.b[er] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < UU; ++u) {
                const int e = e0 + u * NT;
                if (e >= n) break;
                const uint32_t m = A.dmask[e];
                double sum = 0.0;
#pragma unroll
                for (int d = 0; d < 8; ++d) {
                    if (d < nd) {
                        const double val = CST ? A.cv.c[d] : v[CST ? 0 : u][d];
                        const double prod = val * xv[u][d];
                        const double nsum = sum + prod;
                        sum = ((m >> d) & 1u) ? nsum : sum;
                    }
                }
                out(e, sum, bv[u]);
            }
        }
    }

    // y = A x (or b - A x) with P^T y, ||y||^2 (and ||b||^2), then the
    // bookkeeping and small solve of the product's role (spmv_finalize's).
    __device__ __forceinline__ void product(const double *src, double *dst, int act, int k, int q)
    {
#pragma clang fp contract(off)
        if (rfl(sh.flags)) return;
        const bool resid = act == ACT_RESID || act == ACT_TRUE;
        double vals[S + 2];
#pragma unroll
        for (int v = 0; v < S + 2; ++v) vals[v] = 0.0;
        const Sell<double> &A = J.A;
        const int nd = A.nd;
        struct Out {
            bool resid;
            double *dst;
            PBasis pkey;
            double (&vals)[S + 2];
            __device__ __forceinline__ void operator()(int e, double sum, double bv)
            {
#pragma clang fp contract(off)
                double yv = sum;
                if (resid) {
                    yv = bv - sum;
                    vals[S + 1] += bv * bv;
                }
                dst[e] = yv;
                vals[S] += yv * yv;
#pragma unroll
                for (int a = 0; a < S; ++a) vals[a] += pval_m<PM>(pkey, (uint32_t)e, a) * yv;
            }
        } out{resid, dst, pk, vals};
        if (nd > 0 && nd <= 8) {
            if (A.dconst) dia_block<true, U>(A, nd, src, out);
            else dia_block<false, 2>(A, nd, src, out);
        } else {
            for (int e = threadIdx.x; e < n; e += NT) {
                double sum = 0.0;
                if (nd > 0) {
                    // diagonal storage: present entries in ascending column order
                    const uint32_t m = A.dmask[e];
                    for (int d = 0; d < nd; ++d) {
                        const int64_t c = e + A.doff.off[d];
                        const double v = A.dconst ? A.cv.c[d] : A.dval[dia_index(e, d, nd)];
                        const double xv = (c >= 0 && c < n) ? src[c] : 0.0;
                        const double prod = v * xv;
                        const double nsum = sum + prod;
                        sum = ((m >> d) & 1u) ? nsum : sum;
                    }
                } else {
                    // sliced ELLPACK: entry j of row e at slice_ptr[e / 64] + 64 j + e % 64
                    const int64_t k0 = A.slice_ptr[e >> 6] + (e & 63);
                    const int32_t len = A.rp[e + 1] - A.rp[e];
                    for (int32_t j = 0; j < len; ++j) {
                        const int64_t kk = k0 + (int64_t)j * SLICE;
                        const double prod = A.val[kk] * src[A.col[kk]];
                        sum = sum + prod;
                    }
                }
                out(e, sum, resid ? J.b[e] : 0.0);
            }
        }
        reduce<S + 2>(vals, S + 2, sh);
        if (threadIdx.x < 64) {
            const int lane = threadIdx.x, ri = lane >> 3, cj = lane & 7;
            const double *tot = sh.tot;
            int32_t flags = all_finite(sh, S + 2) ? 0 : FLAG_NONFINITE, where = WHERE_NONE;
            switch (act) {
            case ACT_RESID:
                if (lane < S) sh.ptr[0][lane] = tot[lane];
                if (lane == 0) {
                    sh.rr = tot[S];
                    sh.bb = tot[S + 1];
                    sh.mv += 1;
                }
                break;
            case ACT_TRUE:
                if (lane < S) sh.ptt[lane] = tot[lane];
                if (lane == 0) {
                    sh.tt = tot[S];
                    sh.bb = tot[S + 1];
                }
                break;
            case ACT_ARN:
                if (lane < S) sh.ptv[0][q][lane] = tot[lane];
                if (lane == 0) sh.mv += 1;
                break;
            case ACT_R: {
                // eta_1 of level k: (P^T V^(k)) eta = P^T r^(k+1)
                if (lane < S) sh.ptr[k + 1][lane] = tot[lane];
                if (lane == 0) sh.mv += 1;
                if (!flags) {
                    const double m = (ri < S && cj < S) ? sh.ptv[k][cj][ri] : 0.0;
                    const double yv = ri < S ? tot[ri] : 0.0;
                    double c;
                    const bool ok = wave_lu(S, m, yv, c);
                    wave_store(S, ok, c, sh.eta_all[0]);
                    if (!ok) { flags |= FLAG_BREAKDOWN; where = WHERE_ETA; }
                }
                break;
            }
            case ACT_V: {
                if (lane < S) sh.ptv[k + 1][q][lane] = tot[lane];
                if (lane == 0) sh.mv += 1;
                if (!flags && (q + 1 < S || k + 1 < ell)) {
                    const bool in = ri < S && cj < S;
                    double m = 0.0;
                    double *out;
                    int w;
                    if (q + 1 < S) {
                        // eta_{q+1} of level k: columns p <= q from level k+1, p > q from level k
                        if (in) m = (cj == q) ? tot[ri] : (cj < q ? sh.ptv[k + 1][cj][ri] : sh.ptv[k][cj][ri]);
                        out = sh.eta_all[q + 1];
                        w = WHERE_ETA;
                    } else {
                        // gamma of level k+1: (P^T V^(k+1)) gamma = P^T r^(k+1)
                        if (in) m = (cj == q) ? tot[ri] : sh.ptv[k + 1][cj][ri];
                        out = sh.gamma;
                        w = WHERE_GAMMA;
                    }
                    const double yv = ri < S ? sh.ptr[k + 1][ri] : 0.0;
                    double c;
                    const bool ok = wave_lu(S, m, yv, c);
                    wave_store(S, ok, c, out);
                    if (!ok) { flags |= FLAG_BREAKDOWN; where = w; }
                }
                break;
            }
            default:
                break;
            }
            set_flags(sh, flags, where);
        }
        __syncthreads();
    }

    // r^(i) -= V^(i) gamma (i = 0..k), x += U gamma: one pass per level
    // (each element's operations as k_gamma's)
    __device__ void gamma_step(int k)
    {
        if (rfl(sh.flags)) return;
        double g[S];
#pragma unroll
        for (int q = 0; q < S; ++q) g[q] = rfl(sh.gamma[q]);
        for (int i = -1; i <= k; ++i) {
            // i = -1: x += U gamma; else r^(i) -= V^(i) gamma
            double *y = i < 0 ? J.x : Rc(i);
            const double sg = i < 0 ? 1.0 : -1.0;
            for (int e0 = threadIdx.x; e0 < n; e0 += U * NT) {
                double acc[U], w[U][S];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int e = min(e0 + u * NT, n - 1);
                    acc[u] = y[e];
#pragma unroll
                    for (int q = 0; q < S; ++q) w[u][q] = Wc(i, q)[e];
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int e = e0 + u * NT;
                    if (e >= n) break;
#pragma unroll
                    for (int q = 0; q < S; ++q) acc[u] = fmaT(sg * g[q], w[u][q], acc[u]);
                    y[e] = acc[u];
                }
            }
        }
        __syncthreads();
    }

    // v_q^(k) := r^(k+1) - sum_{p<q} eta_p v_p^(k+1) - sum_{p>=q} eta_p v_p^(k)
    __device__ void eta_step(int k, int q)
    {
        if (rfl(sh.flags)) return;
        double h[S];
#pragma unroll
        for (int p = 0; p < S; ++p) h[p] = rfl(sh.eta_all[q][p]);
        for (int e0 = threadIdx.x; e0 < n; e0 += U * NT) {
            double acc[U], w[U][S];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = min(e0 + u * NT, n - 1);
                acc[u] = Rc(k + 1)[e];
#pragma unroll
                for (int p = 0; p < S; ++p) w[u][p] = ((p < q) ? Wc(k + 1, p) : Wc(k, p))[e];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = e0 + u * NT;
                if (e >= n) break;
#pragma unroll
                for (int p = 0; p < S; ++p) acc[u] = fmaT(-h[p], w[u][p], acc[u]);
                Wc(k, q)[e] = acc[u];
            }
        }
        __syncthreads();
    }

    // levels -1..k-1 of the s steps of level k, top down (k_eta_low's order);
    // the coefficients are read from LDS where they are used (held in
    // registers, s^2 of them would crowd out the workgroups sharing a CU)
    __device__ void eta_low(int k)
    {
        if (rfl(sh.flags)) return;
        const volatile double *eta = &sh.eta_all[0][0];
        for (int e0 = threadIdx.x; e0 < n; e0 += U * NT) {
            double up[U][S];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = min(e0 + u * NT, n - 1);
#pragma unroll
                for (int p = 0; p < S; ++p) up[u][p] = Wc(k, p)[e];
            }
            for (int i = k - 1; i >= -1; --i) {
                double old[U][S], r[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int e = min(e0 + u * NT, n - 1);
                    r[u] = Rc(i + 1)[e];
#pragma unroll
                    for (int p = 0; p < S; ++p) old[u][p] = Wc(i, p)[e];
                }
#pragma unroll
                for (int q = 0; q < S; ++q) {
                    double acc[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) acc[u] = r[u];
#pragma unroll
                    for (int p = 0; p < S; ++p) {
                        const double c = eta[q * MAXS + p];
#pragma unroll
                        for (int u = 0; u < U; ++u) acc[u] = fmaT(-c, (p < q) ? up[u][p] : old[u][p], acc[u]);
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int e = e0 + u * NT;
                        if (e < n) Wc(i, q)[e] = acc[u];
                        old[u][q] = acc[u];
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int p = 0; p < S; ++p) up[u][p] = old[u][p];
            }
        }
        __syncthreads();
    }

    // Gram matrix of [r^(0..l)] and tau = Z^+ r^(0) by the normal equations
    __device__ void gram()
    {
        if (rfl(sh.flags)) return;
        constexpr int NGL = (LC + 1) * (LC + 2) / 2;
        double acc[NGL];
#pragma unroll
        for (int v = 0; v < NGL; ++v) acc[v] = 0.0;
        for (int e0 = threadIdx.x; e0 < n; e0 += U * NT) {
            double z[U][LC + 1];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = e0 + u * NT;
#pragma unroll
                for (int i = 0; i <= LC; ++i) z[u][i] = (i <= ell && e < n) ? Rc(i)[e] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (e0 + u * NT >= n) break;
                int v = 0;
#pragma unroll
                for (int i = 0; i <= LC; ++i)
#pragma unroll
                    for (int j = i; j <= LC; ++j) {
                        if (j <= ell) acc[v] += z[u][i] * z[u][j];
                        ++v;
                    }
            }
        }
        // pair (i, j), i <= j <= LC, at i*(LC+1) - i*(i-1)/2 + (j - i)
        reduce<NGL>(acc, NGL, sh);
        if (threadIdx.x < 64) {
            const int lane = threadIdx.x, ri = lane >> 3, cj = lane & 7;
            auto at = [&](int i, int j) {
                if (i > j) { int t = i; i = j; j = t; }
                return sh.tot[i * (LC + 1) - i * (i - 1) / 2 + (j - i)];
            };
            bool finite = true;
            for (int i = 0; i <= ell; ++i)
                for (int j = i; j <= ell; ++j) finite = finite && isfinite(at(i, j));
            const double g = (ri < ell && cj < ell) ? at(ri + 1, cj + 1) : 0.0;
            const double yv = ri < ell ? at(0, ri + 1) : 0.0;
            double t;
            const bool ok = wave_spd(ell, g, yv, t);
            wave_store(ell, ok, t, sh.tau);
            set_flags(sh, (finite ? 0 : FLAG_NONFINITE) | (ok ? 0 : FLAG_BREAKDOWN), ok ? 0 : WHERE_TAU);
        }
        __syncthreads();
    }

    // x, r, u_q, v_q from the levels (k_poly's element operations), then P^T r,
    // P^T V, ||r||^2 and the next cycle's gamma.  One pass for x and r, then
    // one per column q (each with its own s sums: the totals are those of a
    // single pass, value by value, with far fewer registers).
    __device__ void poly()
    {
        if (rfl(sh.flags)) return;
        double tau[LC];
#pragma unroll
        for (int i = 0; i < LC; ++i) tau[i] = (i < ell) ? rfl(sh.tau[i]) : 0.0;
        bool finite = true;
        {
            double acc[S + 1];
#pragma unroll
            for (int v = 0; v <= S; ++v) acc[v] = 0.0;
            for (int e0 = threadIdx.x; e0 < n; e0 += U * NT) {
                double xa[U], z[U][LC + 1];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int e = min(e0 + u * NT, n - 1);
                    xa[u] = J.x[e];
#pragma unroll
                    for (int i = 0; i <= LC; ++i)
                        if (i <= ell) z[u][i] = Rc(i)[e];
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int e = e0 + u * NT;
                    if (e >= n) break;
                    double ra = z[u][0];
#pragma unroll
                    for (int i = 1; i <= LC; ++i) {
                        if (i > ell) break;
                        xa[u] = fmaT(tau[i - 1], z[u][i - 1], xa[u]);
                        ra = fmaT(-tau[i - 1], z[u][i], ra);
                    }
                    J.x[e] = xa[u];
                    Rc(0)[e] = ra;
#pragma unroll
                    for (int a = 0; a < S; ++a) acc[a] += pval_m<PM>(pk, (uint32_t)e, a) * ra;
                    acc[S] += ra * ra;
                }
            }
            reduce<S + 1>(acc, S + 1, sh);
            if (threadIdx.x < 64) {
                if (threadIdx.x < S) sh.ptr[0][threadIdx.x] = sh.tot[threadIdx.x];
                if (threadIdx.x == 0) sh.rr = sh.tot[S];
            }
            finite = all_finite(sh, S + 1);
        }
        for (int q = 0; q < S; ++q) {
            double acc[S];
#pragma unroll
            for (int v = 0; v < S; ++v) acc[v] = 0.0;
            for (int e0 = threadIdx.x; e0 < n; e0 += U * NT) {
                double z[U][LC + 2];   // v_q^(-1..l)
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int e = min(e0 + u * NT, n - 1);
#pragma unroll
                    for (int i = -1; i <= LC; ++i)
                        if (i <= ell) z[u][i + 1] = Wc(i, q)[e];
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int e = e0 + u * NT;
                    if (e >= n) break;
                    double ua = z[u][0], va = z[u][1];
#pragma unroll
                    for (int i = 1; i <= LC; ++i) {
                        if (i > ell) break;
                        ua = fmaT(-tau[i - 1], z[u][i], ua);
                        va = fmaT(-tau[i - 1], z[u][i + 1], va);
                    }
                    Wc(-1, q)[e] = ua;
                    Wc(0, q)[e] = va;
#pragma unroll
                    for (int a = 0; a < S; ++a) acc[a] += pval_m<PM>(pk, (uint32_t)e, a) * va;
                }
            }
            reduce<S>(acc, S, sh);
            if (threadIdx.x < S) sh.ptv[0][q][threadIdx.x] = sh.tot[threadIdx.x];
            finite = finite && all_finite(sh, S);
        }
        __syncthreads();
        if (threadIdx.x < 64) {
            const int lane = threadIdx.x, ri = lane >> 3, cj = lane & 7;
            const double rr = rfl(sh.rr);
            int32_t flags = finite ? 0 : FLAG_NONFINITE, where = WHERE_NONE;
            if (finite && rr > rfl(sh.thr2)) {
                const double m = (ri < S && cj < S) ? sh.ptv[0][cj][ri] : 0.0;
                const double yv = ri < S ? sh.ptr[0][ri] : 0.0;
                double c;
                const bool ok = wave_lu(S, m, yv, c);
                wave_store(S, ok, c, sh.gamma);
                if (!ok) { flags |= FLAG_BREAKDOWN; where = WHERE_GAMMA; }
            }
            set_flags(sh, flags, where);
        }
        __syncthreads();
    }

    // gamma of level 0 from P^T V, P^T r (replace: r is the true residual
    // just computed, whose P^T r and norm become the recursive ones)
    __device__ void small(bool replace)
    {
        __syncthreads();
        if (threadIdx.x < 64) {
            const int lane = threadIdx.x, ri = lane >> 3, cj = lane & 7;
            double rr = rfl(sh.rr);
            const double *rhs = sh.ptr[0];
            if (replace) {
                rr = rfl(sh.tt);
                rhs = sh.ptt;
                if (lane < S) sh.ptr[0][lane] = sh.ptt[lane];
            }
            if (!rfl(sh.flags) && rr > rfl(sh.thr2)) {
                const double m = (ri < S && cj < S) ? sh.ptv[0][cj][ri] : 0.0;
                const double yv = ri < S ? rhs[ri] : 0.0;
                double c;
                const bool ok = wave_lu(S, m, yv, c);
                wave_store(S, ok, c, sh.gamma);
                if (!ok) set_flags(sh, FLAG_BREAKDOWN, WHERE_GAMMA);
            }
            if (replace && lane == 0) sh.rr = rr;
        }
        __syncthreads();
    }

    // h_j = u_j . w (j < nu), ||w||^2 into aux (and aux0 if first)
    __device__ void dots(int nu, const double *w, bool first)
    {
        if (rfl(sh.flags)) return;
        double acc[MAXS + 1];
#pragma unroll
        for (int v = 0; v <= MAXS; ++v) acc[v] = 0.0;
        for (int e = threadIdx.x; e < n; e += NT) {
            const double wv = w[e];
#pragma unroll
            for (int j = 0; j < MAXS; ++j)
                if (j < nu) acc[j] += Wc(-1, j)[e] * wv;
            acc[MAXS] += wv * wv;
        }
        reduce<MAXS + 1>(acc, MAXS + 1, sh);
        if (threadIdx.x == 0) {
            for (int j = 0; j < nu; ++j) sh.h[j] = sh.tot[j];
            sh.aux = sh.tot[MAXS];
            if (first) sh.aux0 = sh.tot[MAXS];
            if (!isfinite(sh.tot[MAXS])) sh.flags |= FLAG_NONFINITE;
        }
        __syncthreads();
    }

    // out = w - sum_j h_j u_j
    __device__ void gs(int nu, const double *w, double *out)
    {
        if (rfl(sh.flags)) return;
        double h[MAXS];
#pragma unroll
        for (int j = 0; j < MAXS; ++j) h[j] = (j < nu) ? rfl(sh.h[j]) : 0.0;
        for (int e = threadIdx.x; e < n; e += NT) {
            double a = w[e];
#pragma unroll
            for (int j = 0; j < MAXS; ++j)
                if (j < nu) a = fmaT(-h[j], Wc(-1, j)[e], a);
            out[e] = a;
        }
        __syncthreads();
    }

    // dst = src / sqrt(norm2), norm2 = aux (mode 0) or rr (mode 1); a norm
    // below 1e-14 of the product's (mode 0) or zero is an Arnoldi breakdown
    __device__ void normalize(const double *src, double *dst, int mode)
    {
        if (rfl(sh.flags)) return;
        const double nrm2 = mode == 0 ? rfl(sh.aux) : rfl(sh.rr);
        const bool bad = (mode == 0 && !(nrm2 > 1e-28 * rfl(sh.aux0))) || !(nrm2 > 0.0);
        if (bad) {
            __syncthreads();
            set_flags(sh, FLAG_BREAKDOWN, WHERE_ARNOLDI);
            __syncthreads();
            return;
        }
        const double inv = 1.0 / sqrt(nrm2);
        for (int e = threadIdx.x; e < n; e += NT) dst[e] = src[e] * inv;
        __syncthreads();
    }

    // Arnoldi basis of level s of r^(0): U orthonormal, V = A U (classical
    // Gram-Schmidt applied twice), then gamma
    __device__ void arnoldi()
    {
        normalize(Rc(0), Wc(-1, 0), 1);
        for (int q = 0; q < S; ++q) {
            product(Wc(-1, q), Wc(0, q), ACT_ARN, 0, q);
            if (q + 1 < S) {
                double *w = Wc(-1, q + 1);
                dots(q + 1, Wc(0, q), true);
                gs(q + 1, Wc(0, q), w);
                dots(q + 1, w, false);
                gs(q + 1, w, w);
                dots(0, w, false);
                normalize(w, w, 0);
            }
        }
        small(false);
    }

    __device__ void cycle()
    {
        gamma_step(0);
        for (int k = 0; k < ell; ++k) {
            product(Rc(k), Rc(k + 1), ACT_R, k, 0);
            for (int q = 0; q < S; ++q) {
                eta_step(k, q);
                product(Wc(k, q), Wc(k + 1, q), ACT_V, k, q);
            }
            eta_low(k);
            if (k + 1 < ell) gamma_step(k + 1);
        }
        gram();
        poly();
    }

    __device__ void copy(double *dst, const double *src, int count)
    {
        for (int c = 0; c < count; ++c)
            for (int e = threadIdx.x; e < n; e += NT) dst[(int64_t)c * ld + e] = src[(int64_t)c * ld + e];
        __syncthreads();
    }

    __device__ void fetch()
    {
        copy(J.recU, Wc(-1, 0), S);
        copy(J.recV, Wc(0, 0), S);
        if (threadIdx.x < MAXS * MAXS) J.rec_ptv[threadIdx.x] = (&sh.ptv[0][0][0])[threadIdx.x];
        __syncthreads();
    }

    // (the leading barrier: every thread has read the control values before
    // thread 0 changes them)
    __device__ void clear_flags()
    {
        __syncthreads();
        if (threadIdx.x == 0) {
            sh.flags = 0;
            sh.where = WHERE_NONE;
        }
        __syncthreads();
    }

    __device__ void set_thr2(double v)
    {
        __syncthreads();
        if (threadIdx.x == 0) sh.thr2 = v;
        __syncthreads();
    }
};

#ifndef MSTAB_WG_WAVES
#define MSTAB_WG_WAVES 2
#endif
template <int S, int LC, int PM>
__device__ __forceinline__ void solve_job(Job &J, Shared &sh)
{
    Solver<S, LC, PM> E(J, sh);
    const int n = E.n;
    if (threadIdx.x == 0) {
        sh.flags = 0;
        sh.where = WHERE_NONE;
        sh.mv = 0;
        sh.thr2 = 0.0;
        sh.rr = sh.bb = sh.tt = sh.aux = sh.aux0 = 0.0;
    }
    __syncthreads();

    int status = MSTAB_OK;
    bool converged = false, recycled = false;
    int restarts = 0, replacements = 0, periodic_repl = 0;
    int64_t mv = 0, mv_check = 0, cycles = 0, level = 0, fetched = -1, hl = 0;
    double rr = 0.0, relres_rec = 0.0, relres_true = -1.0;
    int64_t est_out = J.est_cycle;
    int32_t rec_have = J.rec_have;
    int64_t rec_level = J.rec_level;
    // the estimate of the fetch cycle, kept up to date over the history
    double est_best = -1.0, est_prev = 0.0;
    int64_t est_k = -1;
    auto hist = [&](int64_t m, double res) {
        if (threadIdx.x == 0 && hl < HIST) {
            J.hist_mv[hl * J.hist_stride] = m;
            J.hist_res[hl * J.hist_stride] = res;
        }
        if (hl >= 1) {
            const double f = res > 0.0 ? est_prev / res : INFINITY;
            if (f > est_best) { est_best = f; est_k = hl; }
        }
        est_prev = res;
        ++hl;
    };

    const double tol2 = J.tol * J.tol;
    double bb, thr2, rr_true_mark;
    int64_t since_true = 0;
    bool r_is_true = true, have_uv = false, had_rec, fire;
    int64_t est_in;

    E.product(J.x, E.Rc(0), ACT_RESID, 0, 0);
    bb = rfl(sh.bb);
    if ((rfl(sh.flags) & FLAG_NONFINITE) || !isfinite(bb)) {
        status = MSTAB_E_NONFINITE;
        mv = 0;
        goto done;
    }
    if (bb == 0.0) {
        for (int e = threadIdx.x; e < n; e += NT) J.x[e] = 0.0;
        converged = true;
        relres_true = 0.0;
        mv = 0;
        goto done;
    }
    thr2 = tol2 * bb;
    E.set_thr2(thr2);
    rr = rfl(sh.rr);
    rr_true_mark = rr;
    mv = rfl(sh.mv);
    hist(mv, sqrt(rr / bb));

    if (J.method == MSTAB_METHOD_MSTAB && rec_have) {
        E.copy(E.Wc(-1, 0), J.recU, S);
        E.copy(E.Wc(0, 0), J.recV, S);
        if (threadIdx.x < MAXS * MAXS) (&sh.ptv[0][0][0])[threadIdx.x] = J.rec_ptv[threadIdx.x];
        __syncthreads();
        level = rec_level;
        have_uv = true;
        recycled = true;
        E.small(false);
    }
    had_rec = rec_have;
    est_in = J.est_cycle;

    for (;;) {
        while (rr > thr2 && mv < J.max_mv) {
            if (!have_uv) {
                E.arnoldi();
                have_uv = true;
                level = 0;
                mv = rfl(sh.mv);
                if (rfl(sh.flags) & FLAG_NONFINITE) { status = MSTAB_E_NONFINITE; goto out; }
                if ((rfl(sh.flags) & FLAG_BREAKDOWN) && rfl(sh.where) == WHERE_ARNOLDI) {
                    status = MSTAB_E_BREAKDOWN;
                    goto out;
                }
                continue;
            }
            E.cycle();
            mv = rfl(sh.mv);
            if (rfl(sh.flags) & FLAG_NONFINITE) { status = MSTAB_E_NONFINITE; goto out; }
            if (rfl(sh.flags) & FLAG_BREAKDOWN) {
                if (restarts < 2) {
                    ++restarts;
                    have_uv = false;
                    E.clear_flags();
                    E.set_thr2(0.0);   // no gamma solve until the basis is rebuilt
                    E.product(J.x, E.Rc(0), ACT_RESID, 0, 0);
                    E.set_thr2(thr2);
                    mv = rfl(sh.mv);
                    rr = rfl(sh.rr);
                    rr_true_mark = rr;
                    r_is_true = true;
                    since_true = 0;
                    if ((rfl(sh.flags) & FLAG_NONFINITE) || !isfinite(rr)) {
                        status = MSTAB_E_NONFINITE;
                        goto out;
                    }
                    continue;
                }
                status = MSTAB_E_BREAKDOWN;
                goto out;
            }
            ++cycles;
            level += E.ell;
            r_is_true = false;
            rr = rfl(sh.rr);
            ++since_true;
            if (J.replace_every > 0 && since_true >= J.replace_every && rr > thr2 && mv < J.max_mv) {
                ++periodic_repl;
                since_true = 0;
                E.product(J.x, J.T, ACT_TRUE, 0, 0);
                E.copy(E.Rc(0), J.T, 1);
                E.small(true);
                ++mv_check;
                ++replacements;
                if (rfl(sh.flags) & FLAG_NONFINITE) { status = MSTAB_E_NONFINITE; goto out; }
                if (rfl(sh.flags) & FLAG_BREAKDOWN) { status = MSTAB_E_BREAKDOWN; goto out; }
                rr = rfl(sh.rr);
                rr_true_mark = rr;
                r_is_true = true;
            }
            hist(mv + mv_check, sqrt(rr / bb));
            {
                const double rel = sqrt(rr / bb);
                fire = false;
                switch (J.fetch) {
                case MSTAB_FETCH_THRESHOLD: fire = (fetched < 0 && rel <= J.fetch_rel); break;
                case MSTAB_FETCH_AT_LEVEL: fire = (level == J.fetch_level); break;
                case MSTAB_FETCH_ONCE: fire = (!had_rec && fetched < 0 && rel <= J.fetch_rel); break;
                case MSTAB_FETCH_ESTIMATE: fire = (est_in > 0 && fetched < 0 && cycles == est_in); break;
                default: break;
                }
            }
            if (fire) {
                E.fetch();
                rec_level = level;
                rec_have = 1;
                fetched = level;
            }
        }
        // finish: the true residual decides
        if (r_is_true) {
            relres_true = sqrt(rr / bb);
            converged = rr <= thr2;
            break;
        }
        E.product(J.x, J.T, ACT_TRUE, 0, 0);
        ++mv_check;
        {
            const double tt = rfl(sh.tt);
            relres_true = sqrt(tt / bb);
            if (!isfinite(tt)) { status = MSTAB_E_NONFINITE; goto out; }
            if (tt <= thr2) { converged = true; break; }
            if (rr <= thr2 && replacements - periodic_repl < J.max_repl && mv < J.max_mv) {
                E.copy(E.Rc(0), J.T, 1);
                E.small(true);
                rr = tt;
                r_is_true = true;
                since_true = 0;
                ++replacements;
                continue;
            }
        }
        break;
    }
    (void)rr_true_mark;
    if (!converged) status = MSTAB_NOT_CONVERGED;
    if (cycles > 0 && fetched < 0 &&
        (J.fetch == MSTAB_FETCH_AT_END || J.fetch == MSTAB_FETCH_THRESHOLD ||
         (J.fetch == MSTAB_FETCH_ONCE && !had_rec) || (J.fetch == MSTAB_FETCH_ESTIMATE && est_in > 0))) {
        E.fetch();
        rec_level = level;
        rec_have = 1;
        fetched = level;
    }
    if (J.fetch == MSTAB_FETCH_ESTIMATE) est_out = est_k < 0 ? -1 : (est_k > 1 ? est_k - 1 : 1);
out:
    mv = rfl(sh.mv);
    relres_rec = sqrt(rr / bb);
done:
    __syncthreads();
    if (threadIdx.x == 0) {
        J.status = status;
        J.converged = converged;
        J.recycled = recycled;
        J.restarts = restarts;
        J.replacements = replacements;
        J.mv = mv;
        J.mv_check = mv_check;
        J.cycles = cycles;
        J.level = level;
        J.fetched = fetched;
        J.hist_len = hl;
        J.relres_rec = relres_rec;
        J.relres_true = relres_true;
        J.rec_have = rec_have;
        J.rec_level = rec_level;
        J.est_cycle = est_out;
    }
}

// PM: every job of the launch takes P's entries from the generator (0) or
// from its handle's matrix (1); the host groups the jobs accordingly.
template <int S, int LC, int PM>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(MSTAB_WG_WAVES))) void k_solve(Job *jobs)
{
    __shared__ Shared sh;
    solve_job<S, LC, PM>(jobs[blockIdx.x], sh);
}

// k_solve<s, lc, pm> over count jobs (device array) on st; lc is 2, 4 or 8
// (the bound on l the kernel is built for), pm whether the jobs' P is a
// matrix.  Defined in wg.hip, a translation unit of its own.
void launch(int s, int lc, bool pm, int count, Job *jobs, hipStream_t st);

}  // namespace wg
}  // namespace mstab
