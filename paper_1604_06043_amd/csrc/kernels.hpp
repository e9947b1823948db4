// Device kernels of the M(s)stab(l) iteration for gfx950 (CDNA4).
//
// Notation follows Algorithm 1 of arXiv 1604.06043: levels r^(i) (R[i],
// i = 0..l) of the residual and v_q^(i) (W[i][q], i = -1..l, q = 0..s-1) of the
// s auxiliary vectors, with U = V^(-1) and V = V^(0).  Every vector is a
// column of ld elements (ld a multiple of 256; entries n..ld-1 stay zero).
//
// Reductions are deterministic: each workgroup writes one partial per value
// (value-major, [value][block]); the last workgroup to finish (found with an
// agent-scope atomic counter) adds the partials in a fixed order, then one
// thread runs the small FP64 solve that the next kernel needs (gamma, eta_q or
// tau) and stores the coefficients in the control block.  No host round trip
// happens inside a cycle.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mstab {

constexpr int MAXS = 8;
constexpr int MAXL = 8;
constexpr int BLOCK = 256;
constexpr int NWAVE = BLOCK / 64;

enum : int32_t { FLAG_BREAKDOWN = 1, FLAG_NONFINITE = 2 };
enum : int32_t { WHERE_NONE = 0, WHERE_GAMMA = 1, WHERE_ETA = 2, WHERE_TAU = 3, WHERE_ARNOLDI = 4 };

// Copied to the host after every cycle.
struct Status {
    double rr;      // ||r||^2 of the recursive residual
    double bb;      // ||b||^2
    double tt;      // ||b - A x||^2 of the last true-residual kernel
    double aux;     // Gram-Schmidt norm of the vector being orthonormalized
    double aux0;    // norm^2 of the Arnoldi product before orthogonalization
    int32_t flags;
    int32_t where;
    int64_t mv;     // products with A performed by the iteration kernels
};

constexpr int GROUP_PAD = 32;   // unsigned ints per group arrival counter (a 128-byte line)

struct Ctl {
    Status st;
    double thr2;                        // tol^2 ||b||^2, set by the host
    double ptv[MAXL + 1][MAXS][MAXS];   // [i][q][a] = p_a . v_q^(i), i = 0..l
    double ptr[MAXL + 1][MAXS];         // [i][a] = p_a . r^(i)
    double ptt[MAXS];                   // P^T of the last true residual
    double gamma[MAXS];
    double eta[MAXS];
    double eta_all[MAXS][MAXS];         // [q][p]: eta of step q of the current level
    double tau[MAXL];
    double h[MAXS + 1];                 // Gram-Schmidt coefficients
    double prec[MAXS][MAXS];            // [q][a] = p_a . v_q of refreshed fetched data
    double chol[MAXS][MAXS];            // Cholesky factor L (lower) of U^T U of fetched data
    int32_t chol_ok;                    // U^T U was numerically positive definite
    unsigned int counter[4];            // last-workgroup counters (zero between launches)
    // per counter, the arrival counters of eight workgroup groups, one
    // 128-byte line each (zero between launches)
    alignas(128) unsigned int gcount[4][8 * GROUP_PAD];
};

// ---------------------------------------------------------------------------
// Cut-space basis P: entry (row, q) regenerated from a counter-based hash
// (MurmurHash3's 32-bit finalizer of key + (8 row + q) * 0x9E3779B9), top 24
// bits mapped to [-1, 1).  Exact in FP32 and FP64; nothing is stored.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

__device__ __forceinline__ double pval(uint32_t key, uint32_t row, int q)
{
    uint32_t ctr = (row * 8u + (uint32_t)q) * 0x9E3779B9u + key;
    int32_t t = (int32_t)(fmix32(ctr) >> 8) - (1 << 23);
    return (double)t * 0x1p-23;
}

// The cut-space basis as the kernels see it: entry (row, q) from the
// generator above with key, or, when m is set, from a caller's n x s matrix
// copied to the device (column q at m + q ld).  The choice is uniform across
// a launch.
struct PBasis {
    uint32_t key = 0;
    const double *m = nullptr;
    int64_t ld = 0;
    PBasis() = default;
    __host__ __device__ PBasis(uint32_t k, const double *mm = nullptr, int64_t l = 0) : key(k), m(mm), ld(l) {}
};

__device__ __forceinline__ double pval(const PBasis &p, uint32_t row, int q)
{
    return p.m ? p.m[(int64_t)q * p.ld + row] : pval(p.key, row, q);
}

// The same with the choice fixed at compile time where a kernel has hoisted
// it out of its row loop: PM = 1 the caller's matrix, 0 the generator, -1
// decided per call.
template <int PM>
__device__ __forceinline__ double pval_m(const PBasis &p, uint32_t row, int q)
{
    if constexpr (PM == 1)
        return p.m[(int64_t)q * p.ld + row];
    else if constexpr (PM == 0)
        return pval(p.key, row, q);
    else
        return pval(p, row, q);
}

__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// ---------------------------------------------------------------------------
// Small dense solves (FP64) in one wavefront.  Callers hand over an m x m
// system (m <= 8) with entry (i, j) in lane 8 i + j and y_i in the lanes of
// row i; the solve gathers row i into lane i (eight independent shuffles) and
// then works lane-per-row: the pivot row and every value a step needs from
// another row come from v_readlane into scalar registers, so the dependent
// chain of the elimination has no LDS round trips.  Every lane executes the
// same instruction stream, and the result does not depend on which wavefront
// runs it.  The pivot is the first largest magnitude in the column (lowest
// row on ties); a pivot <= 1e-14 times the largest magnitude of its column
// marks the system singular.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double shfl_d(double v, int src) { return __shfl(v, src); }

// v of lane `src` (wavefront-uniform src) in every lane
__device__ __forceinline__ double lane_d(double v, int src)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u & 0xFFFFFFFFu), src);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), src);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Solves A c = y with partial pivoting; returns ok (uniform).  On return the
// lanes of row i hold c_i in `c`.
__device__ bool wave_lu(int m, double a, double y, double &c)
{
    const int lane = threadIdx.x & 63, i = lane >> 3, j = lane & 7;
    const bool in = (i < m) && (j < m);
    // largest magnitude of column j (xor over the row bits keeps j); lane j
    // (row 0) holds it for column j
    double cm = in ? fabs(a) : 0.0;
    for (int o = 8; o < 64; o <<= 1) cm = fmax(cm, __shfl_xor(cm, o));
    // row (lane & 7) of the system into this lane
    double r[8];
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) r[jj] = shfl_d(a, (lane & 7) * 8 + jj);
    double yr = shfl_d(y, (lane & 7) * 8);
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (k >= m) break;
        // pivot: first largest magnitude among rows k..m-1 of column k
        double best = -1.0;
        int piv = k;
        for (int ii = k; ii < m; ++ii) {
            const double v = fabs(lane_d(r[k], ii));
            if (v > best) { best = v; piv = ii; }
        }
        ok = ok && (best > 1e-14 * lane_d(cm, k));
        // exchange rows k and piv
        double rk[8], rp[8];
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) {
            rk[jj] = lane_d(r[jj], k);
            rp[jj] = lane_d(r[jj], piv);
        }
        const double yk = lane_d(yr, k), yp = lane_d(yr, piv);
        if (lane == k) {
#pragma unroll
            for (int jj = 0; jj < 8; ++jj) r[jj] = rp[jj];
            yr = yp;
        } else if (lane == piv) {
#pragma unroll
            for (int jj = 0; jj < 8; ++jj) r[jj] = rk[jj];
            yr = yk;
        }
        // eliminate below the pivot (its row is now rp, yp)
        const double inv = 1.0 / rp[k];
        if (lane > k && lane < m) {
            const double f = r[k] * inv;
#pragma unroll
            for (int jj = k + 1; jj < 8; ++jj)
                if (jj < m) r[jj] = fma(-f, rp[jj], r[jj]);
            yr = fma(-f, yp, yr);
        }
    }
    // back substitution, column by column
    c = 0.0;
#pragma unroll
    for (int k = 7; k >= 0; --k) {
        if (k >= m) continue;
        const double ck = lane_d(yr, k) / lane_d(r[k], k);
        if (lane < k) yr = fma(-r[k], ck, yr);
        if (i == k) c = ck;
    }
    return ok;
}

// Normal equations G t = c (G SPD): right-looking Cholesky, then the two
// triangular solves; LU when G is not numerically SPD.  Same lane-per-row
// layout as wave_lu after the gather.
__device__ bool wave_spd(int m, double g, double y, double &t)
{
    const int lane = threadIdx.x & 63, i = lane >> 3;
    const double g0 = g, y0 = y;
    double r[8];
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) r[jj] = shfl_d(g, (lane & 7) * 8 + jj);
    double yr = shfl_d(y, (lane & 7) * 8);
    bool spd = true;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (k >= m) break;
        const double akk = lane_d(r[k], k);
        spd = spd && (akk > 0.0);
        const double lkk = sqrt(fmax(akk, 0.0));
        // L_ik of this lane's row
        const double lv = (lane == k) ? lkk : ((lane > k && lane < m) ? r[k] / lkk : 0.0);
#pragma unroll
        for (int jj = k + 1; jj < 8; ++jj) {
            if (jj >= m) break;
            const double ljk = lane_d(lv, jj);
            if (lane > k && lane < m) r[jj] = fma(-lv, ljk, r[jj]);
        }
        if (lane >= k) r[k] = lv;
    }
    if (!spd) return wave_lu(m, g0, y0, t);
    // forward: L z = y
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (k >= m) break;
        const double zk = lane_d(yr, k) / lane_d(r[k], k);
        if (lane > k && lane < m) yr = fma(-r[k], zk, yr);
        if (lane == k) yr = zk;
    }
    // backward: L^T t = z (row k of L^T is column k of L: entry L_jk sits in lane j)
    t = 0.0;
#pragma unroll
    for (int k = 7; k >= 0; --k) {
        if (k >= m) continue;
        const double tk = lane_d(yr, k) / lane_d(r[k], k);
        // L_ki for this lane's i < k is lane k's r[i]
        double lki = 0.0;
#pragma unroll
        for (int ii = 0; ii < 8; ++ii)
            if (ii < k) {
                const double v = lane_d(r[ii], k);
                if (lane == ii) lki = v;
            }
        if (lane < k) yr = fma(-lki, tk, yr);
        if (i == k) t = tk;
    }
    return true;
}

// Writes the solution of a projected system to out[0..m) (lane 8 i holds c_i),
// zeroes on breakdown.  Called by the whole wavefront 0.
__device__ __forceinline__ void wave_store(int m, bool ok, double c, double *out)
{
    const int lane = threadIdx.x & 63, i = lane >> 3, j = lane & 7;
    if (j == 0 && i < m) out[i] = ok ? c : 0.0;
}

// ---------------------------------------------------------------------------
// Last-workgroup reduction.
//
// The partials and the arrival counter are exchanged through agent-scope
// atomic loads and stores, which are coherent across the device's dies
// without the whole-cache write-back that an agent-scope fence costs here.
// A writer waits for its partial stores to complete before the workgroup
// barrier; thread 0 then arrives, in two stages (its group's counter, and
// the group's last workgroup the launch's counter: no single address takes
// every workgroup's atomic).  The workgroup that completes the last group
// reads every partial (atomically, agent scope) and adds them in a fixed
// order, so the totals do not depend on which workgroup finishes last.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void part_store(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double part_load(const double *p)
{
    return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// wait until this thread's outstanding memory operations have completed
__device__ __forceinline__ void wait_memory() { __builtin_amdgcn_s_waitcnt(0); }

// Up to 1024 workgroups: a lane's share of one value's partials is at most 16
// loads, all issued before the first is used.
constexpr int MAX_PARTIAL_BLOCKS = 1024;

template <int NT = BLOCK>
__device__ bool last_block_reduce(const double *part, int stride, int nv, unsigned int *counter,
                                  unsigned int *groups, double *tot)
{
    constexpr int NW = NT / 64;
    __shared__ int s_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        // arrival in two stages: workgroup b counts on the counter of group
        // b mod 8, and the last of each group on the launch's counter, so that
        // no counter takes more than an eighth of the grid's atomics
        const unsigned G = gridDim.x < 8u ? gridDim.x : 8u;
        const unsigned g = blockIdx.x % G;
        const unsigned gs = gridDim.x / G + (g < gridDim.x % G ? 1u : 0u);
        unsigned int *gc = groups + g * GROUP_PAD;
        const unsigned prev = __hip_atomic_fetch_add(gc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        bool last = false;
        if (prev == gs - 1) {
            __hip_atomic_store(gc, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned p2 = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            last = (p2 == G - 1);
        }
        s_last = last;
    }
    __syncthreads();
    if (!s_last) return false;
    // the partials were stored coherently and completed before their
    // workgroups arrived; agent-scope loads read them past this die's cache
    // (cheaper here than an acquire fence and plain loads)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nb = (int)gridDim.x;
    for (int v = wave; v < nv; v += NW) {
        const double *pv = part + (size_t)v * stride;
        double a[MAX_PARTIAL_BLOCKS / 64];
#pragma unroll
        for (int m = 0; m < MAX_PARTIAL_BLOCKS / 64; ++m) {
            const int b = lane + 64 * m;
            a[m] = (b < nb) ? part_load(pv + b) : 0.0;
        }
#pragma unroll
        for (int h = MAX_PARTIAL_BLOCKS / 128; h > 0; h >>= 1)
#pragma unroll
            for (int m = 0; m < h; ++m) a[m] += a[m + h];
        const double acc = wave_sum(a[0]);
        if (lane == 0) tot[v] = acc;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

// Block-level sum of up to NV per-thread values into part[.][blockIdx.x].
// vals[v] are per-thread contributions; the block result is written by
// threads t < nv.
template <int NV, int NT = BLOCK>
__device__ void block_partials(double (&vals)[NV], int nv, double *part, int stride)
{
    constexpr int NW = NT / 64;
    __shared__ double s_red[NW][NV];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        if (v < nv) {
            double w = wave_sum(vals[v]);
            if (lane == 0) s_red[wave][v] = w;
        }
    }
    __syncthreads();
    for (int v = threadIdx.x; v < nv; v += NT) {
        double a = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) a += s_red[w][v];
        part_store(part + (size_t)v * stride + blockIdx.x, a);
    }
    wait_memory();
}

// ---------------------------------------------------------------------------
// Sparse product with projection epilogue: y = A x (or y = b - A x), then the
// workgroup partials of P^T y (s values), ||y||^2 and ||b||^2.
//
// Storage: sliced ELLPACK with 64-row slices (built from the caller's CSR at
// create time).  Entry j of row r = 64 t + l sits at slice_ptr[t] + 64 j + l,
// so the j-th entries of a wavefront's 64 rows are one contiguous 64-element
// load, run to the slice's longest row; padded entries (column 0, value 0)
// are loaded with the rest but never added (row lengths come from the CSR row
// pointer).  One thread per row; indices and values are loaded eight at a
// time before their gathers from x.  Products are rounded, then added in CSR
// order (contraction off): the textbook order, so the result equals a
// sequential CSR product bit for bit.  At most 1024 workgroups keep the
// number of partials, and with it the final reduction, small.
// ---------------------------------------------------------------------------
enum : int32_t {
    ACT_NONE = 0,
    ACT_RESID = 1,   // y = b - A x is the residual r^(0): ptr[0], rr, bb
    ACT_TRUE = 2,    // y = b - A x is a true residual check: ptt, tt
    ACT_R = 3,       // y = r^(k+1): ptr[k+1]; solve eta_1 of level k
    ACT_V = 4,       // y = v_q^(k+1): ptv[k+1][q]; solve eta_{q+1} or gamma of level k+1
    ACT_ARN = 5,     // y = v_q = A u_q (Arnoldi): ptv[0][q]
    ACT_PROJ = 6,    // P^T y, ||y||^2 into ptt / tt (diagnostics)
    ACT_RECV = 7     // y = A u_q of fetched data: prec[q]
};

struct SpmvArgs {
    int32_t act, k, q, s, ell;
    PBasis pkey;
};

#ifndef MSTAB_SPMV_BLOCK
#define MSTAB_SPMV_BLOCK 512
#endif
constexpr int SPMV_BLOCK = MSTAB_SPMV_BLOCK;
constexpr int SLICE = 64;

constexpr int MAX_DIAG = 16;
struct DiaOffsets {
    int64_t off[MAX_DIAG];   // column - row of each stored diagonal, ascending
};
constexpr unsigned long long DIA_EMPTY = 0x8000000000000000ull;   // unused table slot

// A diagonal-storage matrix whose every diagonal holds one value wherever it
// is present (a constant-coefficient stencil) keeps only those values: c[d]
// is the value in the copy's precision, widened to double.
struct DiaConst {
    double c[MAX_DIAG];
};

// Diagonal storage is sliced like the rows: the nd values of 64 consecutive
// rows lie together, diagonal by diagonal, so a wavefront's loads of a slice
// are one contiguous block of nd * 64 entries.
__host__ __device__ __forceinline__ int64_t dia_index(int64_t r, int d, int nd)
{
    return (r / 64) * (int64_t)nd * 64 + (int64_t)d * 64 + (r % 64);
}

// Sliced ELLPACK copy of a CSR matrix (device arrays).
template <typename T>
struct Sell {
    int64_t n = 0, nnz = 0, padded = 0;
    const int32_t *rp = nullptr;     // the CSR row pointer (row lengths)
    int64_t *slice_ptr = nullptr;    // n_slices + 1
    int32_t *col = nullptr;          // padded
    T *val = nullptr;                // padded
    // Diagonal storage, used instead when every entry lies on one of nd <= 16
    // diagonals (stencil matrices): offsets ascending, values at
    // dval[dia_index(r, d, nd)] (zero where row r has no entry d), and a
    // presence mask per row (bit d).
    int nd = 0;
    DiaOffsets doff{};
    uint16_t *dmask = nullptr;
    T *dval = nullptr;
    // constant diagonals: dval is not kept, the values are cv.c[d]
    bool dconst = false;
    DiaConst cv{};
};

// Structure check of a caller's CSR matrix before any kernel reads it through
// its indices: every column index in [0, n) and strictly increasing within
// its row.  The row pointer has already been checked on the host (rp[0] = 0,
// non-decreasing, rp[n] = nnz), so every read stays inside col_idx[0, nnz).
// *bad (zero beforehand) is set to 1 on the first violation.
static __global__ __launch_bounds__(BLOCK) void k_csr_check(int64_t n, const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ ci, int *bad)
{
    for (int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * BLOCK) {
        int64_t prev = -1;
        for (int32_t j = rp[r]; j < rp[r + 1]; ++j) {
            const int64_t c = ci[j];
            if (c <= prev || c >= n) {
                __hip_atomic_store(bad, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            prev = c;
        }
    }
}

// Scatter CSR rows into the sliced layout (one thread per row).
template <typename TD, typename TS>
__global__ __launch_bounds__(BLOCK) void k_to_sell(int64_t n, const int32_t *__restrict__ rp,
                                                   const int32_t *__restrict__ ci,
                                                   const TS *__restrict__ va,
                                                   const int64_t *__restrict__ slice_ptr,
                                                   int32_t *__restrict__ scol,
                                                   TD *__restrict__ sval)
{
    for (int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * BLOCK) {
        const int64_t base = slice_ptr[r / SLICE] + (r % SLICE);
        const int32_t k0 = rp[r], len = rp[r + 1] - k0;
        for (int32_t j = 0; j < len; ++j) {
            if (scol) scol[base + (int64_t)j * SLICE] = ci[k0 + j];
            sval[base + (int64_t)j * SLICE] = (TD)va[k0 + j];
        }
    }
}

// The distinct diagonals (column - row) of a CSR matrix, collected into a
// table of MAX_DIAG slots.  Every thread probes the slots in the same order
// and claims an empty one by compare-and-swap, so a value enters once; a
// value that finds no slot sets *overflow.
static __global__ __launch_bounds__(BLOCK) void k_dia_offsets(int64_t n, const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ ci,
                                                       unsigned long long *table, int *overflow)
{
    // Each workgroup first collects the offsets of its rows in an LDS table,
    // then merges that table into the global one: the global table then sees
    // at most MAX_DIAG probes per workgroup instead of one per entry.  More
    // than MAX_DIAG distinct offsets in one workgroup means more in the matrix.
    __shared__ unsigned long long s_tab[MAX_DIAG];
    __shared__ int s_over;
    if (threadIdx.x < MAX_DIAG) s_tab[threadIdx.x] = DIA_EMPTY;
    if (threadIdx.x == 0) s_over = 0;
    __syncthreads();
    bool over = false;
    for (int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * BLOCK) {
        for (int32_t j = rp[r]; j < rp[r + 1]; ++j) {
            const unsigned long long off = (unsigned long long)((int64_t)ci[j] - r);
            bool placed = false;
            for (int t = 0; t < MAX_DIAG && !placed; ++t) {
                unsigned long long cur =
                    __hip_atomic_load(&s_tab[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (cur == DIA_EMPTY) cur = atomicCAS(&s_tab[t], DIA_EMPTY, off);
                placed = (cur == DIA_EMPTY || cur == off);
            }
            over |= !placed;
        }
    }
    if (over) s_over = 1;
    __syncthreads();
    if (threadIdx.x < MAX_DIAG) {
        const unsigned long long off = s_tab[threadIdx.x];
        bool placed = (off == DIA_EMPTY);
        for (int t = 0; t < MAX_DIAG && !placed; ++t) {
            unsigned long long cur =
                __hip_atomic_load(&table[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (cur == DIA_EMPTY) cur = atomicCAS(&table[t], DIA_EMPTY, off);
            placed = (cur == DIA_EMPTY || cur == off);
        }
        if (!placed || (threadIdx.x == 0 && s_over))
            __hip_atomic_store(overflow, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Scatter CSR rows into diagonal storage (dval zeroed beforehand).
template <typename TD, typename TS>
__global__ __launch_bounds__(BLOCK) void k_to_dia(int64_t n, const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ ci,
                                                  const TS *__restrict__ va, int nd,
                                                  DiaOffsets doff, uint16_t *__restrict__ mask,
                                                  TD *__restrict__ dval)
{
    for (int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * BLOCK) {
        uint32_t m = 0;
        for (int32_t j = rp[r]; j < rp[r + 1]; ++j) {
            const int64_t off = (int64_t)ci[j] - r;
            int d = 0;
            while (d < nd - 1 && doff.off[d] != off) ++d;
            dval[dia_index(r, d, nd)] = (TD)va[j];
            m |= 1u << d;
        }
        if (mask) mask[r] = (uint16_t)m;
    }
}

// Smallest and largest bit pattern of the present values of each diagonal
// (lohi[d] and lohi[MAX_DIAG + d], combined by atomic min/max; the caller
// starts them at all ones and zero).  Equal patterns mean a constant diagonal.
template <typename TD>
__global__ __launch_bounds__(BLOCK) void k_dia_range(int64_t n, int nd, const uint16_t *__restrict__ mask,
                                                     const TD *__restrict__ dval,
                                                     unsigned long long *lohi)
{
    __shared__ unsigned long long s_lo[MAX_DIAG], s_hi[MAX_DIAG];
    if (threadIdx.x < MAX_DIAG) {
        s_lo[threadIdx.x] = ~0ull;
        s_hi[threadIdx.x] = 0ull;
    }
    __syncthreads();
    for (int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * BLOCK) {
        const uint32_t m = mask[r];
        for (int d = 0; d < nd; ++d)
            if ((m >> d) & 1u) {
                const TD v = dval[dia_index(r, d, nd)];
                unsigned long long bits;
                if constexpr (sizeof(TD) == 8) bits = __builtin_bit_cast(unsigned long long, v);
                else bits = (unsigned long long)__builtin_bit_cast(uint32_t, v);
                atomicMin(&s_lo[d], bits);
                atomicMax(&s_hi[d], bits);
            }
    }
    __syncthreads();
    if (threadIdx.x < nd) {
        atomicMin(&lohi[threadIdx.x], s_lo[threadIdx.x]);
        atomicMax(&lohi[MAX_DIAG + threadIdx.x], s_hi[threadIdx.x]);
    }
}

// S = number of projection columns (a.s must equal S; 0 for a plain product).
// Each wavefront takes 64 consecutive rows = one slice, so the slice offset and
// width are wavefront-uniform (scalar registers) and the loop over the width
// has no divergence.  Padding entries hold column 0 and value 0 and every slice
// is allocated in full, so the index and value loads run to the slice width
// for all 64 lanes; the row lengths only select which products are added.
// Adding nothing for a padding entry keeps the CSR-order sum exact.
// y[r] (and the residual form b[r] - sum) plus the row's share of the partials.
template <typename T, int S, int PM = -1>
__device__ __forceinline__ void spmv_row_out(int64_t r, T sum, bool resid, const T *__restrict__ b,
                                             T *__restrict__ y, PBasis pkey,
                                             double (&vals)[S + 2])
{
#pragma clang fp contract(off)
    T yv = sum;
    if (resid) {
        const T bv = b[r];
        yv = bv - sum;
        vals[S + 1] += (double)bv * (double)bv;
    }
    y[r] = yv;
    const double yd = (double)yv;
    vals[S] += yd * yd;
#pragma unroll
    for (int j = 0; j < S; ++j) vals[j] += pval_m<PM>(pkey, (uint32_t)r, j) * yd;
}

// The end of every product kernel: workgroup partials of P^T y, ||y||^2 and
// ||b||^2, the last workgroup's fixed-order totals, and (wavefront 0) the
// bookkeeping and small solve that the product's role calls for.
template <int S>
__device__ void spmv_finalize(double (&vals)[S + 2], Ctl *ctl, double *part, int stride,
                              const SpmvArgs &a)
{
    const int lane = threadIdx.x & 63;
    const int nv = S + 2;
    const int ri = lane >> 3, cj = lane & 7;
    const int s = a.s;
    // the small solve's operands that earlier launches wrote (P^T V columns
    // other than this product's own, P^T r^(k+1)) are loaded before the
    // reduction, so that the last workgroup does not wait for them after it
    double pm = 0.0, py = 0.0;
    if (threadIdx.x < 64) {
        const bool in = ri < s && cj < s;
        if (a.act == ACT_R) {
            if (in) pm = ctl->ptv[a.k][cj][ri];
        } else if (a.act == ACT_V && (a.q + 1 < s || a.k + 1 < a.ell)) {
            if (in && cj != a.q)
                pm = (a.q + 1 < s && cj > a.q) ? ctl->ptv[a.k][cj][ri] : ctl->ptv[a.k + 1][cj][ri];
            if (ri < s) py = ctl->ptr[a.k + 1][ri];
        }
    }
    block_partials<S + 2, SPMV_BLOCK>(vals, nv, part, stride);
    __shared__ double tot[MAXS + 2];
    if (!last_block_reduce<SPMV_BLOCK>(part, stride, nv, &ctl->counter[0], ctl->gcount[0], tot)) return;
    if (threadIdx.x >= 64) return;   // wavefront 0 finalizes

    bool finite = true;
    for (int v = 0; v < nv; ++v) finite = finite && isfinite(tot[v]);
    int32_t flags = finite ? 0 : FLAG_NONFINITE, where = WHERE_NONE;
    switch (a.act) {
    case ACT_RESID:
        if (lane < s) ctl->ptr[0][lane] = tot[lane];
        if (lane == 0) {
            ctl->st.rr = tot[s];
            ctl->st.bb = tot[s + 1];
            ctl->st.mv += 1;
        }
        break;
    case ACT_TRUE:
        if (lane < s) ctl->ptt[lane] = tot[lane];
        if (lane == 0) {
            ctl->st.tt = tot[s];
            ctl->st.bb = tot[s + 1];
        }
        break;
    case ACT_PROJ:
        if (lane < s) ctl->ptt[lane] = tot[lane];
        if (lane == 0) ctl->st.tt = tot[s];
        break;
    case ACT_ARN:
        if (lane < s) ctl->ptv[0][a.q][lane] = tot[lane];
        if (lane == 0) ctl->st.mv += 1;
        break;
    case ACT_RECV:
        if (lane < s) ctl->prec[a.q][lane] = tot[lane];
        if (lane == 0) ctl->st.mv += 1;
        break;
    case ACT_R: {
        // y = r^(k+1); eta_1 of level k: (P^T V^(k)) eta = P^T r^(k+1)
        if (lane < s) ctl->ptr[a.k + 1][lane] = tot[lane];
        if (lane == 0) ctl->st.mv += 1;
        if (!flags) {
            const double m = pm;   // (P^T V^(k))[ri][cj], zero outside s x s
            const double yv = ri < s ? tot[ri] : 0.0;
            double c;
            const bool ok = wave_lu(s, m, yv, c);
            wave_store(s, ok, c, ctl->eta);
            if (!ok) { flags |= FLAG_BREAKDOWN; where = WHERE_ETA; }
        }
        break;
    }
    case ACT_V: {
        // y = v_q^(k+1)
        if (lane < s) ctl->ptv[a.k + 1][a.q][lane] = tot[lane];
        if (lane == 0) ctl->st.mv += 1;
        if (!flags && (a.q + 1 < s || a.k + 1 < a.ell)) {
            const bool in = ri < s && cj < s;
            double m = 0.0, yv = 0.0;
            double *out;
            int w;
            // eta_{q+1} at level k: columns p <= q from level k+1, p > q from
            // level k; gamma of level k+1: (P^T V^(k+1)) gamma = P^T r^(k+1).
            // Column q is this product's; the others were preloaded (pm).
            if (in) m = (cj == a.q) ? tot[ri] : pm;
            if (a.q + 1 < s) {
                out = ctl->eta;
                w = WHERE_ETA;
            } else {
                out = ctl->gamma;
                w = WHERE_GAMMA;
            }
            yv = py;
            double c;
            const bool ok = wave_lu(s, m, yv, c);
            wave_store(s, ok, c, out);
            if (!ok) { flags |= FLAG_BREAKDOWN; where = w; }
        }
        break;
    }
    default:
        break;
    }
    if (lane == 0 && flags) {
        ctl->st.flags |= flags;
        if (where) ctl->st.where = where;
    }
}

// TM: type of the stored matrix values (T, or float for FP64 vectors with an
// FP32 copy of the matrix); each value is converted to T before its product.
template <typename T, int S, typename TM, int PM>
__device__ __forceinline__ void sell_rows(int64_t n, const int32_t *__restrict__ rp,
                                          const int64_t *__restrict__ slice_ptr,
                                          const int32_t *__restrict__ scol, const TM *__restrict__ sval,
                                          const T *__restrict__ x, T *__restrict__ y,
                                          const T *__restrict__ b, bool resid, PBasis pkey,
                                          double (&vals)[S + 2])
{
#pragma clang fp contract(off)
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nslices = (n + SLICE - 1) / SLICE;
    for (int64_t t = (int64_t)blockIdx.x * (SPMV_BLOCK / SLICE) + wave; t < nslices;
         t += (int64_t)gridDim.x * (SPMV_BLOCK / SLICE)) {
        const int64_t sp0 = slice_ptr[t];
        const int32_t w = (int32_t)((slice_ptr[t + 1] - sp0) / SLICE);
        const int64_t r = t * SLICE + lane;
        const bool valid = r < n;
        const int32_t len = valid ? rp[r + 1] - rp[r] : 0;
        const TM *vp = sval + sp0 + lane;
        const int32_t *cp = scol + sp0 + lane;
        T sum = (T)0;
        for (int32_t j0 = 0; j0 < w; j0 += 8) {
            int32_t c[8];
            TM v[8];
            T xv[8];
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (j0 + j < w) {
                    // the matrix is streamed once per product: keep it out of the caches
                    c[j] = __builtin_nontemporal_load(cp + (int64_t)(j0 + j) * SLICE);
                    v[j] = __builtin_nontemporal_load(vp + (int64_t)(j0 + j) * SLICE);
                }
            // every index and value load in flight before the first is used: with
            // FP32 values the scheduler otherwise converts each value as it
            // arrives and waits on the loads one pair at a time
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (j0 + j < w) xv[j] = x[c[j]];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (j0 + j < w) {
                    const T prod = (T)v[j] * xv[j];
                    const T nsum = sum + prod;
                    sum = (j0 + j < len) ? nsum : sum;
                }
        }
        if (valid) spmv_row_out<T, S, PM>(r, sum, resid, b, y, pkey, vals);
    }
}

// PM (all product kernels): where P's entries come from (pval_m), chosen by
// the host per launch, so that each variant is register-allocated on its own.
template <typename T, int S, typename TM, int PM>
__global__ __launch_bounds__(SPMV_BLOCK) void k_spmv(int64_t n, const int32_t *__restrict__ rp,
                                                     const int64_t *__restrict__ slice_ptr,
                                                     const int32_t *__restrict__ scol,
                                                     const TM *__restrict__ sval,
                                                     const T *__restrict__ x,
                                                     T *__restrict__ y,
                                                     const T *__restrict__ b, Ctl *ctl,
                                                     double *part, int stride, SpmvArgs a)
{
    if (ctl->st.flags) return;
    const bool resid = (a.act == ACT_RESID || a.act == ACT_TRUE);
    double vals[S + 2];
#pragma unroll
    for (int v = 0; v < S + 2; ++v) vals[v] = 0.0;
    sell_rows<T, S, TM, PM>(n, rp, slice_ptr, scol, sval, x, y, b, resid, a.pkey, vals);
    spmv_finalize<S>(vals, ctl, part, stride, a);
}

// The rows of one thread for the diagonal-storage product.  CST: constant
// diagonals (values from cv), else values streamed from dval.  x is gathered
// wherever the column lies in [0, n) (the presence bits only select the sum),
// so the gathers do not wait for the mask.
template <bool CST, typename T, typename TM>
__device__ __forceinline__ void dia_load8(int64_t r, int64_t n, int nd, int d0, const DiaOffsets &doff,
                                          const DiaConst &cv, const TM *__restrict__ dval,
                                          const T *__restrict__ x, T (&v)[8], T (&xv)[8])
{
#pragma unroll
    for (int j = 0; j < 8; ++j)
        if (d0 + j < nd) {
            const int64_t c = r + doff.off[d0 + j];
            if constexpr (CST)
                v[j] = (T)cv.c[d0 + j];
            else   // the matrix is streamed once per product: keep it out of the caches
                v[j] = (T)__builtin_nontemporal_load(dval + dia_index(r, d0 + j, nd));
            xv[j] = (c >= 0 && c < n) ? x[c] : (T)0;
        }
}

template <typename T>
__device__ __forceinline__ void dia_add8(int nd, int d0, uint32_t m, const T (&v)[8], const T (&xv)[8], T &sum)
{
#pragma clang fp contract(off)
#pragma unroll
    for (int j = 0; j < 8; ++j)
        if (d0 + j < nd) {
            const T prod = v[j] * xv[j];
            const T nsum = sum + prod;
            sum = ((m >> (d0 + j)) & 1u) ? nsum : sum;
        }
}

template <bool CST, typename T, int S, typename TM, int PM>
__device__ __forceinline__ void dia_rows(int64_t n, int nd, const DiaOffsets &doff, const DiaConst &cv,
                                         const uint16_t *__restrict__ mask,
                                         const TM *__restrict__ dval, const T *__restrict__ x,
                                         T *__restrict__ y, const T *__restrict__ b, bool resid,
                                         PBasis pkey, double (&vals)[S + 2])
{
    for (int64_t r = (int64_t)blockIdx.x * SPMV_BLOCK + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * SPMV_BLOCK) {
        const uint32_t m = mask[r];
        T sum = (T)0;
        for (int d0 = 0; d0 < nd; d0 += 8) {
            T v[8], xv[8];
            dia_load8<CST, T, TM>(r, n, nd, d0, doff, cv, dval, x, v, xv);
            dia_add8(nd, d0, m, v, xv, sum);
        }
        spmv_row_out<T, S, PM>(r, sum, resid, b, y, pkey, vals);
    }
}

// The rows of one thread for a constant-diagonal matrix with a compile-time
// number of diagonals (ND = 7: the 3-D seven-point stencils, ND = 5: the 2-D
// five-point ones).  The offsets and values sit in scalar registers for the
// whole launch, indices are 32-bit, and each gather's column is clamped to
// the row itself when it falls outside [0, n) (the presence bit of such an
// entry is always clear), so the ND gathers issue back to back with no
// branch; products are rounded and added in ascending column order exactly
// as in dia_rows.
#ifndef MSTAB_DIA_RPI
#define MSTAB_DIA_RPI 1
#endif
template <typename T, int S, int ND, int PM, int RPI = MSTAB_DIA_RPI>
__device__ __forceinline__ void dia_rows_const(int64_t n, const DiaOffsets &doff, const DiaConst &cv,
                                               const uint16_t *__restrict__ mask, const T *__restrict__ x,
                                               T *__restrict__ y, const T *__restrict__ b, bool resid,
                                               PBasis pkey, double (&vals)[S + 2])
{
#pragma clang fp contract(off)
    const int32_t n32 = (int32_t)n;
    int32_t off[ND];
    T cst[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        off[d] = (int32_t)doff.off[d];
        cst[d] = (T)cv.c[d];
    }
    // RPI rows per pass (grid-stride apart, so each wavefront's loads stay
    // contiguous): all their gathers are issued before the first is summed
    const int32_t stride = (int32_t)(gridDim.x * SPMV_BLOCK);
    for (int32_t r0 = (int32_t)(blockIdx.x * SPMV_BLOCK + threadIdx.x); r0 < n32; r0 += RPI * stride) {
        T xv[RPI][ND];
#pragma unroll
        for (int u = 0; u < RPI; ++u) {
            const int32_t r = r0 + u * stride;
            const int32_t rr = r < n32 ? r : r0;
#pragma unroll
            for (int d = 0; d < ND; ++d) {
                const uint32_t c = (uint32_t)(rr + off[d]);
                xv[u][d] = x[c < (uint32_t)n32 ? c : (uint32_t)rr];
            }
        }
        // the presence mask is needed only by the sum: keep its load behind the
        // gathers, so that waiting for it does not hold their issue back
        asm volatile("" ::: "memory");
        uint32_t m[RPI];
#pragma unroll
        for (int u = 0; u < RPI; ++u) {
            const int32_t r = r0 + u * stride;
            m[u] = mask[r < n32 ? r : r0];
        }
        // every gather and mask load issued before the first sum: without this
        // the scheduler starts summing after four gathers and holds the rest back
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < RPI; ++u) {
            const int32_t r = r0 + u * stride;
            if (u > 0 && r >= n32) break;
            T sum = (T)0;
#pragma unroll
            for (int d = 0; d < ND; ++d) {
                const T prod = cst[d] * xv[u][d];
                const T nsum = sum + prod;
                sum = ((m[u] >> d) & 1u) ? nsum : sum;
            }
            spmv_row_out<T, S, PM>(r, sum, resid, b, y, pkey, vals);
        }
    }
}

// v of lane l - 1 (dpp_shr1) or lane l + 1 (dpp_shl1) across the wavefront
// (DPP wavefront shifts; the end lane receives 0)
__device__ __forceinline__ double dpp_shr1(double v)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u & 0xFFFFFFFFu), 0x138, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), 0x138, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double dpp_shl1(double v)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u & 0xFFFFFFFFu), 0x130, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), 0x130, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float dpp_shr1(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xF, 0xF, false));
}
__device__ __forceinline__ float dpp_shl1(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x130, 0xF, 0xF, false));
}

// two-element vectors of the compiler's own (usable with the nontemporal loads)
typedef double pair_d __attribute__((ext_vector_type(2)));
typedef float pair_f __attribute__((ext_vector_type(2)));
template <typename T> struct Vec2;
template <> struct Vec2<double> { using type = pair_d; };
template <> struct Vec2<float> { using type = pair_f; };

// One row's share of the partials, in spmv_row_out's order (no memory
// operations: the caller has loaded b and stores y).
template <typename T, int S, int PM>
__device__ __forceinline__ void row_acc(int64_t r, T yv, T bv, bool resid, PBasis pkey, double (&vals)[S + 2])
{
#pragma clang fp contract(off)
    if (resid) vals[S + 1] += (double)bv * (double)bv;
    const double yd = (double)yv;
    vals[S] += yd * yd;
#pragma unroll
    for (int j = 0; j < S; ++j) vals[j] += pval_m<PM>(pkey, (uint32_t)r, j) * yd;
}

// Diagonal storage with ND diagonals (7 or 5), two consecutive rows per
// thread: each even offset's two x values are one 8- or 16-byte load, and the
// offsets -1, 0, +1 of both rows come from the thread's own pair and one value
// of each neighbouring lane's (DPP shifts); with values
// streamed (CST false) each diagonal's two values are one load too: five
// 16-byte x loads per two rows where one row per thread takes fourteen 8-byte
// ones.  Needs n even, the offsets -1, 0,
// +1 in the middle and every other offset even (pairs_ok on the host).  Each
// row's products and sum are those of dia_rows and dia_rows_const, so y is
// the same bit for bit; the partials add row 2p before row 2p + 1.
template <bool CST, typename T, int S, typename TM, int ND, int PM>
__device__ __forceinline__ void dia_pairs(int64_t n, const DiaOffsets &doff, const DiaConst &cv,
                                          const uint16_t *__restrict__ mask, const TM *__restrict__ dval,
                                          const T *__restrict__ x, T *__restrict__ y,
                                          const T *__restrict__ b, bool resid, PBasis pkey,
                                          double (&vals)[S + 2])
{
#pragma clang fp contract(off)
    using V2 = typename Vec2<T>::type;
    using M2 = typename Vec2<TM>::type;
    constexpr int C = ND / 2;
    const int32_t n32 = (int32_t)n;
    const int32_t np = n32 / 2;
    int32_t off[ND];
    T cst[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        off[d] = (d == C - 1) ? -2 : (d == C + 1) ? 2 : (int32_t)doff.off[d];
        cst[d] = (T)cv.c[d];
    }
    const int32_t stride = (int32_t)(gridDim.x * SPMV_BLOCK);
    for (int32_t p = (int32_t)(blockIdx.x * SPMV_BLOCK + threadIdx.x); p < np; p += stride) {
        const int32_t r0 = 2 * p;
        V2 xo[ND];
        M2 mv[ND];
        // x[r0 - 1] and x[r0 + 2] are the neighbouring lanes' centre values:
        // only the wavefront's end lanes load them
        const int lane = threadIdx.x & 63;
        T xm1 = (T)0, xp2 = (T)0;
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            const uint32_t c = (uint32_t)(r0 + off[d]);
            if (d == C - 1) {
                if (lane == 0) xm1 = x[c < (uint32_t)n32 ? c + 1 : (uint32_t)r0];
            } else if (d == C + 1) {
                if (lane == 63) xp2 = x[c < (uint32_t)n32 ? c : (uint32_t)r0];
            } else {
                xo[d] = *reinterpret_cast<const V2 *>(x + (c < (uint32_t)n32 ? c : (uint32_t)r0));
            }
            if constexpr (!CST)   // the matrix is streamed once per product: keep it out of the caches
                mv[d] = __builtin_nontemporal_load(reinterpret_cast<const M2 *>(dval + dia_index(r0, d, ND)));
        }
        // the mask, b and the sums come after every load has been issued
        asm volatile("" ::: "memory");
        const uint32_t m2 = *reinterpret_cast<const uint32_t *>(mask + r0);
        V2 bv;
        if (resid) bv = *reinterpret_cast<const V2 *>(b + r0);
        __builtin_amdgcn_sched_barrier(0);
        {
            // x[r0 - 1] is the left lane's xo[C].y, x[r0 + 2] the right lane's xo[C].x
            // (lanes past the end of the rows hold values whose entries the masks drop)
            const T ly = dpp_shr1(xo[C].y), rx = dpp_shl1(xo[C].x);
            xo[C - 1].y = lane == 0 ? xm1 : ly;
            xo[C + 1].x = lane == 63 ? xp2 : rx;
        }
        T x0[ND], x1[ND];
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            if (d == C - 1) { x0[d] = xo[C - 1].y; x1[d] = xo[C].x; }
            else if (d == C) { x0[d] = xo[C].x; x1[d] = xo[C].y; }
            else if (d == C + 1) { x0[d] = xo[C].y; x1[d] = xo[C + 1].x; }
            else { x0[d] = xo[d].x; x1[d] = xo[d].y; }
        }
        const uint32_t m0 = m2 & 0xFFFFu, m1 = m2 >> 16;
        T s0 = (T)0, s1 = (T)0;
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            const T a0 = CST ? cst[d] : (T)mv[d].x, a1 = CST ? cst[d] : (T)mv[d].y;
            const T p0 = a0 * x0[d], p1 = a1 * x1[d];
            const T n0 = s0 + p0, n1 = s1 + p1;
            s0 = ((m0 >> d) & 1u) ? n0 : s0;
            s1 = ((m1 >> d) & 1u) ? n1 : s1;
        }
        V2 yv;
        yv.x = resid ? bv.x - s0 : s0;
        yv.y = resid ? bv.y - s1 : s1;
        *reinterpret_cast<V2 *>(y + r0) = yv;
        row_acc<T, S, PM>(r0, yv.x, resid ? bv.x : (T)0, resid, pkey, vals);
        row_acc<T, S, PM>(r0 + 1, yv.y, resid ? bv.y : (T)0, resid, pkey, vals);
    }
}

template <typename T, int S, typename TM, bool CST, int ND, int PM>
__global__ __launch_bounds__(SPMV_BLOCK)
__attribute__((amdgpu_waves_per_eu(sizeof(TM) == 4 ? 8 : 1))) void k_spmv_dia_pair(int64_t n, DiaOffsets doff,
                                                                                    DiaConst cv,
                                                                                    const uint16_t *__restrict__ mask,
                                                                                    const TM *__restrict__ dval,
                                                                                    const T *__restrict__ x,
                                                                                    T *__restrict__ y,
                                                                                    const T *__restrict__ b, Ctl *ctl,
                                                                                    double *part, int stride,
                                                                                    SpmvArgs a)
{
    if (ctl->st.flags) return;
    const bool resid = (a.act == ACT_RESID || a.act == ACT_TRUE);
    double vals[S + 2];
#pragma unroll
    for (int v = 0; v < S + 2; ++v) vals[v] = 0.0;
    dia_pairs<CST, T, S, TM, ND, PM>(n, doff, cv, mask, dval, x, y, b, resid, a.pkey, vals);
    spmv_finalize<S>(vals, ctl, part, stride, a);
}


// The same product for a matrix in diagonal storage (stencil matrices): one
// thread per row, the diagonals' values of 64 consecutive rows one 512-byte
// read each (or, for constant diagonals, no matrix reads at all beyond the
// presence mask), no column indices.  Present entries are multiplied, rounded
// and added in ascending column order (the CSR order), so the result equals the
// sliced product bit for bit.
// CST: constant diagonals (dval unused), else values streamed from dval.
// With FP32 values, 8 wavefronts per SIMD fit without spills; left alone the
// register allocator settles on 7 for some s, which cost a sequence on the
// FP32 copy of a 256^3 matrix 12% of its throughput.
template <typename T, int S, typename TM, bool CST, int PM>
__global__ __launch_bounds__(SPMV_BLOCK)
__attribute__((amdgpu_waves_per_eu(sizeof(TM) == 4 ? 8 : 1))) void k_spmv_dia(int64_t n, int nd, DiaOffsets doff,
                                                         DiaConst cv,
                                                         const uint16_t *__restrict__ mask,
                                                         const TM *__restrict__ dval,
                                                         const T *__restrict__ x,
                                                         T *__restrict__ y,
                                                         const T *__restrict__ b, Ctl *ctl,
                                                         double *part, int stride, SpmvArgs a)
{
    if (ctl->st.flags) return;
    const bool resid = (a.act == ACT_RESID || a.act == ACT_TRUE);
    double vals[S + 2];
#pragma unroll
    for (int v = 0; v < S + 2; ++v) vals[v] = 0.0;
    dia_rows<CST, T, S, TM, PM>(n, nd, doff, cv, mask, dval, x, y, b, resid, a.pkey, vals);
    spmv_finalize<S>(vals, ctl, part, stride, a);
}

// Constant diagonals, ND of them (5 or 7), one row per thread (where the
// paired form does not apply).
template <typename T, int S, int ND, int PM>
__global__ __launch_bounds__(SPMV_BLOCK)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 8 : 1))) void k_spmv_dia_const(int64_t n, DiaOffsets doff, DiaConst cv,
                                                               const uint16_t *__restrict__ mask,
                                                               const T *__restrict__ x,
                                                               T *__restrict__ y,
                                                               const T *__restrict__ b, Ctl *ctl,
                                                               double *part, int stride, SpmvArgs a)
{
    if (ctl->st.flags) return;
    const bool resid = (a.act == ACT_RESID || a.act == ACT_TRUE);
    double vals[S + 2];
#pragma unroll
    for (int v = 0; v < S + 2; ++v) vals[v] = 0.0;
    dia_rows_const<T, S, ND, PM>(n, doff, cv, mask, x, y, b, resid, a.pkey, vals);
    spmv_finalize<S>(vals, ctl, part, stride, a);
}

// 16-byte vectors of T (2 doubles or 4 floats) for the streaming kernels.
template <typename T> struct Vec16;
template <> struct Vec16<double> { using type = double2; static constexpr int W = 2; };
template <> struct Vec16<float> { using type = float4; static constexpr int W = 4; };

template <typename T>
__device__ __forceinline__ void ld16(const T *p, T (&v)[Vec16<T>::W])
{
    using VT = typename Vec16<T>::type;
    const VT t = *reinterpret_cast<const VT *>(p);
    __builtin_memcpy(v, &t, sizeof(VT));
}

template <typename T>
__device__ __forceinline__ void st16(T *p, const T (&v)[Vec16<T>::W])
{
    using VT = typename Vec16<T>::type;
    VT t;
    __builtin_memcpy(&t, v, sizeof(VT));
    *reinterpret_cast<VT *>(p) = t;
}

// ---------------------------------------------------------------------------
// gamma step of level k:  r^(i) -= V^(i) gamma (i = 0..k),  x += U gamma.
// Each thread handles one 16-byte vector of every column (ld is a multiple
// of 256, so every column start is 16-byte aligned).
// ---------------------------------------------------------------------------
template <typename T, int S>
__global__ __launch_bounds__(BLOCK) void k_gamma(int64_t ld, T *__restrict__ W, T *__restrict__ R,
                                                 T *__restrict__ X, int k, const Ctl *ctl)
{
    if (ctl->st.flags) return;
    constexpr int VW = Vec16<T>::W;
    T g[S];
#pragma unroll
    for (int q = 0; q < S; ++q) g[q] = (T)ctl->gamma[q];
    for (int64_t e = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) * VW; e < ld;
         e += (int64_t)gridDim.x * BLOCK * VW) {
        for (int i = 0; i <= k; ++i) {
            T acc[VW], w[VW];
            ld16(R + i * ld + e, acc);
            const T *Wi = W + (int64_t)(i + 1) * S * ld;
#pragma unroll
            for (int q = 0; q < S; ++q) {
                ld16(Wi + q * ld + e, w);
#pragma unroll
                for (int c = 0; c < VW; ++c) acc[c] = fmaT(-g[q], w[c], acc[c]);
            }
            st16(R + i * ld + e, acc);
        }
        T acc[VW], w[VW];
        ld16(X + e, acc);
#pragma unroll
        for (int q = 0; q < S; ++q) {
            ld16(W + q * ld + e, w);
#pragma unroll
            for (int c = 0; c < VW; ++c) acc[c] = fmaT(g[q], w[c], acc[c]);
        }
        st16(X + e, acc);
    }
}

// ---------------------------------------------------------------------------
// eta step (level k, column q):
//   v_q^(i) := r^(i+1) - sum_{p<q} eta_p v_p^(i+1) - sum_{p>=q} eta_p v_p^(i),
//   i = -1..k.  The old v_q^(i) is read before it is overwritten.
// ---------------------------------------------------------------------------
template <typename T, int S>
__global__ __launch_bounds__(BLOCK) void k_eta(int64_t ld, T *__restrict__ W,
                                               const T *__restrict__ R, int k, int q, Ctl *ctl)
{
    // step q of level k, top level only:
    //   v_q^(k) := r^(k+1) - sum_{p<q} eta_p v_p^(k+1) - sum_{p>=q} eta_p v_p^(k)
    // (the levels below k are not read again before the level ends; k_eta_low
    // updates them all at once).  eta is kept for k_eta_low.
    if (ctl->st.flags) return;
    constexpr int VW = Vec16<T>::W;
    T h[S];
#pragma unroll
    for (int p = 0; p < S; ++p) h[p] = (T)ctl->eta[p];
    if (blockIdx.x == 0 && threadIdx.x < S) ctl->eta_all[q][threadIdx.x] = ctl->eta[threadIdx.x];
    const T *Wi = W + (int64_t)(k + 1) * S * ld;   // level k
    const T *Wn = Wi + (int64_t)S * ld;            // level k + 1
    for (int64_t e = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) * VW; e < ld;
         e += (int64_t)gridDim.x * BLOCK * VW) {
        T acc[VW], w[S][VW];
        ld16(R + (int64_t)(k + 1) * ld + e, acc);
#pragma unroll
        for (int p = 0; p < S; ++p) ld16(((p < q) ? Wn : Wi) + p * ld + e, w[p]);
#pragma unroll
        for (int p = 0; p < S; ++p)
#pragma unroll
            for (int c = 0; c < VW; ++c) acc[c] = fmaT(-h[p], w[p][c], acc[c]);
        st16(W + (int64_t)((k + 1) * S + q) * ld + e, acc);
    }
}

// The levels -1..k-1 of all s steps of level k, top down in one pass:
//   v_q^(i) := r^(i+1) - sum_{p<q} eta_{q,p} v_p^(i+1) - sum_{p>=q} eta_{q,p} v_p^(i)
// with v^(i+1) already updated (level k by k_eta, lower ones earlier in this
// pass, carried in registers) and v_p^(i), p >= q, still the old values.
// Same operations in the same order as s per-step passes over all levels.
template <typename T, int S>
__global__ __launch_bounds__(BLOCK) void k_eta_low(int64_t ld, T *__restrict__ W,
                                                   const T *__restrict__ R, int k, const Ctl *ctl)
{
    if (ctl->st.flags) return;
    constexpr int VW = Vec16<T>::W;
    for (int64_t e = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) * VW; e < ld;
         e += (int64_t)gridDim.x * BLOCK * VW) {
        T up[S][VW];   // updated level i + 1
#pragma unroll
        for (int p = 0; p < S; ++p) ld16(W + (int64_t)((k + 1) * S + p) * ld + e, up[p]);
        for (int i = k - 1; i >= -1; --i) {
            T old[S][VW], r[VW];
            ld16(R + (int64_t)(i + 1) * ld + e, r);
#pragma unroll
            for (int p = 0; p < S; ++p) ld16(W + (int64_t)((i + 1) * S + p) * ld + e, old[p]);
#pragma unroll
            for (int q = 0; q < S; ++q) {
                T acc[VW];
#pragma unroll
                for (int c = 0; c < VW; ++c) acc[c] = r[c];
#pragma unroll
                for (int p = 0; p < S; ++p) {
                    const T hp = (T)ctl->eta_all[q][p];
#pragma unroll
                    for (int c = 0; c < VW; ++c)
                        acc[c] = fmaT(-hp, (p < q) ? up[p][c] : old[p][c], acc[c]);
                }
                st16(W + (int64_t)((i + 1) * S + q) * ld + e, acc);
#pragma unroll
                for (int c = 0; c < VW; ++c) old[q][c] = acc[c];   // old[q] is not read again
            }
#pragma unroll
            for (int p = 0; p < S; ++p)
#pragma unroll
                for (int c = 0; c < VW; ++c) up[p][c] = old[p][c];
        }
    }
}

// k_eta_low of level k fused with the gamma step of level k + 1 (which
// follows it in Algorithm 1: the level loop's next pass starts with gamma):
//   v_q^(i) := r^(i+1) - sum_{p<q} eta_{q,p} v_p^(i+1) - sum_{p>=q} eta_{q,p} v_p^(i),
//       i = k-1 .. -1 (as k_eta_low),
//   r^(i) := r^(i) - V^(i) gamma, i = 0..k+1, and x := x + U gamma (as k_gamma),
// where the gamma step reads the V levels this pass has just written (kept in
// registers) and the eta step reads each r^(i) before its gamma update, as the
// two kernels in sequence do.  Same operations in the same order per element.
template <typename T, int S>
__global__ __launch_bounds__(BLOCK) void k_eta_low_gamma(int64_t ld, T *__restrict__ W,
                                                         T *__restrict__ R, T *__restrict__ X,
                                                         int k, const Ctl *ctl)
{
    if (ctl->st.flags) return;
    constexpr int VW = Vec16<T>::W;
    T g[S];
#pragma unroll
    for (int q = 0; q < S; ++q) g[q] = (T)ctl->gamma[q];
    for (int64_t e = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) * VW; e < ld;
         e += (int64_t)gridDim.x * BLOCK * VW) {
        // r^(k+1) -= V^(k+1) gamma (level k+1 is final: the products of level k)
        {
            T acc[VW], w[VW];
            ld16(R + (int64_t)(k + 1) * ld + e, acc);
#pragma unroll
            for (int q = 0; q < S; ++q) {
                ld16(W + (int64_t)((k + 2) * S + q) * ld + e, w);
#pragma unroll
                for (int c = 0; c < VW; ++c) acc[c] = fmaT(-g[q], w[c], acc[c]);
            }
            st16(R + (int64_t)(k + 1) * ld + e, acc);
        }
        T up[S][VW];   // updated level i (starting with level k, written by k_eta)
#pragma unroll
        for (int p = 0; p < S; ++p) ld16(W + (int64_t)((k + 1) * S + p) * ld + e, up[p]);
        for (int i = k; i >= 0; --i) {
            // r^(i) before its gamma update feeds the eta step of level i - 1
            T r[VW], old[S][VW];
            ld16(R + (int64_t)i * ld + e, r);
#pragma unroll
            for (int p = 0; p < S; ++p) ld16(W + (int64_t)(i * S + p) * ld + e, old[p]);
            // gamma step on r^(i) with the new V^(i)
            {
                T acc[VW];
#pragma unroll
                for (int c = 0; c < VW; ++c) acc[c] = r[c];
#pragma unroll
                for (int q = 0; q < S; ++q)
#pragma unroll
                    for (int c = 0; c < VW; ++c) acc[c] = fmaT(-g[q], up[q][c], acc[c]);
                st16(R + (int64_t)i * ld + e, acc);
            }
            // eta steps of level i - 1
#pragma unroll
            for (int q = 0; q < S; ++q) {
                T acc[VW];
#pragma unroll
                for (int c = 0; c < VW; ++c) acc[c] = r[c];
#pragma unroll
                for (int p = 0; p < S; ++p) {
                    const T hp = (T)ctl->eta_all[q][p];
#pragma unroll
                    for (int c = 0; c < VW; ++c)
                        acc[c] = fmaT(-hp, (p < q) ? up[p][c] : old[p][c], acc[c]);
                }
                st16(W + (int64_t)(i * S + q) * ld + e, acc);
#pragma unroll
                for (int c = 0; c < VW; ++c) old[q][c] = acc[c];
            }
#pragma unroll
            for (int p = 0; p < S; ++p)
#pragma unroll
                for (int c = 0; c < VW; ++c) up[p][c] = old[p][c];
        }
        // x += U gamma with the new U = level -1
        T acc[VW];
        ld16(X + e, acc);
#pragma unroll
        for (int q = 0; q < S; ++q)
#pragma unroll
            for (int c = 0; c < VW; ++c) acc[c] = fmaT(g[q], up[q][c], acc[c]);
        st16(X + e, acc);
    }
}

// ---------------------------------------------------------------------------
// Gram matrix of [r^(0), ..., r^(l)] (upper triangle, row-major pairs) and the
// tau solve  (Z^T Z) tau = Z^T r^(0),  Z = [r^(1..l)].
// ---------------------------------------------------------------------------
template <int L>
__device__ void gram_finalize(double (&acc)[(L + 1) * (L + 2) / 2], Ctl *ctl, double *part, int stride);

template <typename T, int L>
__global__ __launch_bounds__(BLOCK) void k_gram(int64_t ld, const T *__restrict__ R, Ctl *ctl,
                                                double *part, int stride)
{
    if (ctl->st.flags) return;
    constexpr int NV = (L + 1) * (L + 2) / 2;
    constexpr int VW = Vec16<T>::W;
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    // four 16-byte groups per thread per pass, all loads issued before use
    constexpr int U = 4;
    const int64_t step = (int64_t)gridDim.x * BLOCK * VW;
    for (int64_t e0 = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) * VW; e0 < ld; e0 += step * U) {
        T z[U][L + 1][VW];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = e0 + u * step;
#pragma unroll
            for (int i = 0; i <= L; ++i) {
                if (e < ld) ld16(R + i * ld + e, z[u][i]);
                else
#pragma unroll
                    for (int c = 0; c < VW; ++c) z[u][i][c] = (T)0;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int c = 0; c < VW; ++c) {
                int v = 0;
#pragma unroll
                for (int i = 0; i <= L; ++i)
#pragma unroll
                    for (int j = i; j <= L; ++j) acc[v++] += (double)z[u][i][c] * (double)z[u][j][c];
            }
    }
    gram_finalize<L>(acc, ctl, part, stride);
}

// The end of k_gram and k_eta_low_gram: workgroup partials of the Gram pairs,
// the last workgroup's fixed-order totals and (wavefront 0) the tau solve.
template <int L>
__device__ void gram_finalize(double (&acc)[(L + 1) * (L + 2) / 2], Ctl *ctl, double *part, int stride)
{
    constexpr int NV = (L + 1) * (L + 2) / 2;
    block_partials<NV>(acc, NV, part, stride);
    __shared__ double tot[NV];
    if (!last_block_reduce(part, stride, NV, &ctl->counter[1], ctl->gcount[1], tot)) return;
    if (threadIdx.x >= 64) return;   // wavefront 0 finalizes
    const int lane = threadIdx.x, ri = lane >> 3, cj = lane & 7;
    // pair (i, j), i <= j, sits at index i*(L+1) - i*(i-1)/2 + (j - i)
    auto at = [&](int i, int j) {
        if (i > j) { int t = i; i = j; j = t; }
        return tot[i * (L + 1) - i * (i - 1) / 2 + (j - i)];
    };
    bool finite = true;
    for (int v = 0; v < NV; ++v) finite = finite && isfinite(tot[v]);
    const double g = (ri < L && cj < L) ? at(ri + 1, cj + 1) : 0.0;
    const double yv = ri < L ? at(0, ri + 1) : 0.0;
    double t;
    const bool ok = wave_spd(L, g, yv, t);
    wave_store(L, ok, t, ctl->tau);
    if (lane == 0) {
        if (!finite) ctl->st.flags |= FLAG_NONFINITE;
        if (!ok) {
            ctl->st.flags |= FLAG_BREAKDOWN;
            ctl->st.where = WHERE_TAU;
        }
    }
}

// k_eta_low of the last level (k = l - 1) fused with the Gram matrix of
// [r^(0), ..., r^(l)] and the tau solve that follow it in Algorithm 1: the
// eta steps read r^(0..l-1) anyway, and the residual levels are final after
// the last product of the level loop.  The eta updates are those of
// k_eta_low; the Gram pairs are summed per thread in element order and then
// as in k_gram.  Launch with at most MAX_PARTIAL_BLOCKS workgroups.
template <typename T, int S, int L>
__global__ __launch_bounds__(BLOCK) void k_eta_low_gram(int64_t ld, T *__restrict__ W,
                                                        const T *__restrict__ R, Ctl *ctl,
                                                        double *part, int stride)
{
    if (ctl->st.flags) return;
    constexpr int VW = Vec16<T>::W;
    constexpr int NV = (L + 1) * (L + 2) / 2;
    constexpr int K = L - 1;
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    for (int64_t e = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) * VW; e < ld;
         e += (int64_t)gridDim.x * BLOCK * VW) {
        T z[L + 1][VW];
        ld16(R + (int64_t)L * ld + e, z[L]);
        T up[S][VW];   // updated level i + 1
#pragma unroll
        for (int p = 0; p < S; ++p) ld16(W + (int64_t)((K + 1) * S + p) * ld + e, up[p]);
#pragma unroll
        for (int i = K - 1; i >= -1; --i) {
            T old[S][VW];
            ld16(R + (int64_t)(i + 1) * ld + e, z[i + 1]);
#pragma unroll
            for (int p = 0; p < S; ++p) ld16(W + (int64_t)((i + 1) * S + p) * ld + e, old[p]);
#pragma unroll
            for (int q = 0; q < S; ++q) {
                T a2[VW];
#pragma unroll
                for (int c = 0; c < VW; ++c) a2[c] = z[i + 1][c];
#pragma unroll
                for (int p = 0; p < S; ++p) {
                    const T hp = (T)ctl->eta_all[q][p];
#pragma unroll
                    for (int c = 0; c < VW; ++c)
                        a2[c] = fmaT(-hp, (p < q) ? up[p][c] : old[p][c], a2[c]);
                }
                st16(W + (int64_t)((i + 1) * S + q) * ld + e, a2);
#pragma unroll
                for (int c = 0; c < VW; ++c) old[q][c] = a2[c];
            }
#pragma unroll
            for (int p = 0; p < S; ++p)
#pragma unroll
                for (int c = 0; c < VW; ++c) up[p][c] = old[p][c];
        }
#pragma unroll
        for (int c = 0; c < VW; ++c) {
            int v = 0;
#pragma unroll
            for (int i = 0; i <= L; ++i)
#pragma unroll
                for (int j = i; j <= L; ++j) acc[v++] += (double)z[i][c] * (double)z[j][c];
        }
    }
    gram_finalize<L>(acc, ctl, part, stride);
}

// ---------------------------------------------------------------------------
// Degree-l update (x and u_q from the levels before r and v_q change):
//   x   := x + sum_i tau_i r^(i-1)        r   := r^(0) - sum_i tau_i r^(i)
//   u_q := v_q^(-1) - sum_i tau_i v_q^(i-1)   v_q := v_q^(0) - sum_i tau_i v_q^(i)
// with the epilogue P^T r, P^T v_q, ||r||^2, then gamma of level 0 of the next
// cycle (only when the residual is still above the threshold).
// ---------------------------------------------------------------------------
template <typename T, int S, int L, int PM>
__global__ __launch_bounds__(BLOCK) void k_poly(int64_t n, int64_t ld, int ell_rt,
                                                T *__restrict__ W, T *__restrict__ R,
                                                T *__restrict__ X, PBasis pkey, Ctl *ctl,
                                                double *part, int stride)
{
    if (ctl->st.flags) return;
    constexpr int NV = S + S * S + 1;
    const int ell = L > 0 ? L : ell_rt;     // compile-time degree lets every load issue up front
    T tau[MAXL];
#pragma unroll
    for (int i = 0; i < MAXL; ++i) tau[i] = (i < ell) ? (T)ctl->tau[i] : (T)0;
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < ld;
         e += (int64_t)gridDim.x * BLOCK) {
        double p[S];
#pragma unroll
        for (int a = 0; a < S; ++a) p[a] = (e < n) ? pval_m<PM>(pkey, (uint32_t)e, a) : 0.0;
        if (L > 0 && S <= 4) {
            // every level of every column of this element in registers first
            constexpr int LL = L > 0 ? L : 1;
            T rv[LL + 1], wv[S][LL + 2];
            const T xa0 = X[e];
#pragma unroll
            for (int i = 0; i <= LL; ++i) rv[i] = R[(int64_t)i * ld + e];
#pragma unroll
            for (int q = 0; q < S; ++q)
#pragma unroll
                for (int i = 0; i <= LL + 1; ++i) wv[q][i] = W[(int64_t)(i * S + q) * ld + e];
            T xa = xa0, ra = rv[0];
#pragma unroll
            for (int i = 1; i <= LL; ++i) {
                xa = fmaT(tau[i - 1], rv[i - 1], xa);
                ra = fmaT(-tau[i - 1], rv[i], ra);
            }
            X[e] = xa;
            R[e] = ra;
            const double rd = (double)ra;
#pragma unroll
            for (int a = 0; a < S; ++a) acc[a] += p[a] * rd;
            acc[S + S * S] += rd * rd;
#pragma unroll
            for (int q = 0; q < S; ++q) {
                T ua = wv[q][0], va = wv[q][1];          // v_q^(-1), v_q^(0)
#pragma unroll
                for (int i = 1; i <= LL; ++i) {
                    ua = fmaT(-tau[i - 1], wv[q][i], ua);
                    va = fmaT(-tau[i - 1], wv[q][i + 1], va);
                }
                W[(int64_t)q * ld + e] = ua;
                W[(int64_t)(S + q) * ld + e] = va;
                const double vd = (double)va;
#pragma unroll
                for (int a = 0; a < S; ++a) acc[S + q * S + a] += p[a] * vd;
            }
            continue;
        }
        // x and r
        {
            T xa = X[e];
            T ra = R[e];
            T prev = ra;
#pragma unroll
            for (int i = 1; i <= (L > 0 ? L : MAXL); ++i) {
                if (L == 0 && i > ell) break;
                const T ri = R[(int64_t)i * ld + e];
                xa = fmaT(tau[i - 1], prev, xa);
                ra = fmaT(-tau[i - 1], ri, ra);
                prev = ri;
            }
            X[e] = xa;
            R[e] = ra;
            const double rd = (double)ra;
#pragma unroll
            for (int a = 0; a < S; ++a) acc[a] += p[a] * rd;
            acc[S + S * S] += rd * rd;
        }
#pragma unroll
        for (int q = 0; q < S; ++q) {
            T ua = W[(int64_t)q * ld + e];              // v_q^(-1)
            T prev = W[(int64_t)(S + q) * ld + e];      // v_q^(0)
            T va = prev;
#pragma unroll
            for (int i = 1; i <= (L > 0 ? L : MAXL); ++i) {
                if (L == 0 && i > ell) break;
                const T vi = W[(int64_t)((i + 1) * S + q) * ld + e];
                ua = fmaT(-tau[i - 1], prev, ua);
                va = fmaT(-tau[i - 1], vi, va);
                prev = vi;
            }
            W[(int64_t)q * ld + e] = ua;
            W[(int64_t)(S + q) * ld + e] = va;
            const double vd = (double)va;
#pragma unroll
            for (int a = 0; a < S; ++a) acc[S + q * S + a] += p[a] * vd;
        }
    }
    block_partials<NV>(acc, NV, part, stride);
    __shared__ double tot[NV];
    if (!last_block_reduce(part, stride, NV, &ctl->counter[2], ctl->gcount[2], tot)) return;
    if (threadIdx.x >= 64) return;   // wavefront 0 finalizes
    const int lane = threadIdx.x, ri = lane >> 3, cj = lane & 7;
    bool finite = true;
    for (int v = 0; v < NV; ++v) finite = finite && isfinite(tot[v]);
    if (lane < S) ctl->ptr[0][lane] = tot[lane];
    for (int idx = lane; idx < S * S; idx += 64) ctl->ptv[0][idx / S][idx % S] = tot[S + idx];
    const double rr = tot[S + S * S];
    if (lane == 0) {
        ctl->st.rr = rr;
        if (!finite) ctl->st.flags |= FLAG_NONFINITE;
    }
    if (!finite || !(rr > ctl->thr2)) return;
    // gamma of level 0 of the next cycle: (P^T V) gamma = P^T r
    const bool in = ri < S && cj < S;
    const double m = in ? tot[S + cj * S + ri] : 0.0;
    const double yv = ri < S ? tot[ri] : 0.0;
    double c;
    const bool ok = wave_lu(S, m, yv, c);
    wave_store(S, ok, c, ctl->gamma);
    if (lane == 0 && !ok) {
        ctl->st.flags |= FLAG_BREAKDOWN;
        ctl->st.where = WHERE_GAMMA;
    }
}

// ---------------------------------------------------------------------------
// Single-thread control steps.
// ---------------------------------------------------------------------------
enum : int32_t {
    SMALL_GAMMA0 = 0,          // gamma of level 0 from ptv[0], ptr[0]
    SMALL_REPLACE = 1,         // r := true residual: ptr[0] = ptt, rr = tt, then gamma
    SMALL_CLEAR = 2            // clear flags
};

static __global__ void k_set_thr2(Ctl *ctl, double thr2)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) ctl->thr2 = thr2;
}

// One wavefront (launch with 64 threads).
static __global__ void k_small(Ctl *ctl, int s, int what)
{
    const int lane = threadIdx.x, ri = lane >> 3, cj = lane & 7;
    if (what == SMALL_CLEAR) {
        if (lane == 0) {
            ctl->st.flags = 0;
            ctl->st.where = WHERE_NONE;
        }
        return;
    }
    const double *rhs = ctl->ptr[0];
    double rr = ctl->st.rr;
    if (what == SMALL_REPLACE) {
        rhs = ctl->ptt;
        rr = ctl->st.tt;
        if (lane < s) ctl->ptr[0][lane] = ctl->ptt[lane];
        if (lane == 0) ctl->st.rr = rr;
    }
    if (ctl->st.flags) return;
    if (!(rr > ctl->thr2)) return;
    const bool in = ri < s && cj < s;
    const double m = in ? ctl->ptv[0][cj][ri] : 0.0;
    const double yv = ri < s ? rhs[ri] : 0.0;
    double c;
    const bool ok = wave_lu(s, m, yv, c);
    wave_store(s, ok, c, ctl->gamma);
    if (lane == 0 && !ok) {
        ctl->st.flags |= FLAG_BREAKDOWN;
        ctl->st.where = WHERE_GAMMA;
    }
}

// ---------------------------------------------------------------------------
// Arnoldi (classical Gram-Schmidt applied twice) helpers.
// ---------------------------------------------------------------------------

// h_j = u_j . w (j < nu) and ||w||^2 into ctl->h / ctl->st.aux; slot 0 keeps the
// norm in aux0 as well (first pass: norm of the fresh product).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_dots(int64_t ld, const T *__restrict__ U, int nu,
                                                const T *__restrict__ w, int first, Ctl *ctl,
                                                double *part, int stride)
{
    if (ctl->st.flags) return;
    double acc[MAXS + 1];
#pragma unroll
    for (int v = 0; v <= MAXS; ++v) acc[v] = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < ld;
         e += (int64_t)gridDim.x * BLOCK) {
        const double wv = (double)w[e];
#pragma unroll
        for (int j = 0; j < MAXS; ++j)
            if (j < nu) acc[j] += (double)U[(int64_t)j * ld + e] * wv;
        acc[MAXS] += wv * wv;
    }
    // pack [h_0..h_{nu-1}, norm]
    double vals[MAXS + 1];
#pragma unroll
    for (int v = 0; v <= MAXS; ++v) vals[v] = 0.0;
#pragma unroll
    for (int j = 0; j < MAXS; ++j)
        if (j < nu) vals[j] = acc[j];
    // norm goes to index nu
#pragma unroll
    for (int j = 0; j <= MAXS; ++j)
        if (j == nu) vals[j] = acc[MAXS];
    block_partials<MAXS + 1>(vals, nu + 1, part, stride);
    __shared__ double tot[MAXS + 1];
    if (!last_block_reduce(part, stride, nu + 1, &ctl->counter[3], ctl->gcount[3], tot)) return;
    if (threadIdx.x != 0) return;
    for (int j = 0; j < nu; ++j) ctl->h[j] = tot[j];
    ctl->st.aux = tot[nu];
    if (first) ctl->st.aux0 = tot[nu];
    if (!isfinite(tot[nu])) ctl->st.flags |= FLAG_NONFINITE;
}

// out = w - sum_j h_j u_j
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_gs(int64_t ld, const T *__restrict__ U, int nu,
                                              const T *w, T *out, const Ctl *ctl)
{
    if (ctl->st.flags) return;
    T h[MAXS];
#pragma unroll
    for (int j = 0; j < MAXS; ++j) h[j] = (j < nu) ? (T)ctl->h[j] : (T)0;
    for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < ld;
         e += (int64_t)gridDim.x * BLOCK) {
        T a = w[e];
#pragma unroll
        for (int j = 0; j < MAXS; ++j)
            if (j < nu) a = fmaT(-h[j], U[(int64_t)j * ld + e], a);
        out[e] = a;
    }
}

// dst = src / sqrt(norm2), norm2 = st.aux (mode 0) or st.rr (mode 1).  In mode 0
// a norm below 1e-14 of the product's norm is an Arnoldi breakdown.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_normalize(int64_t ld, const T *src, T *dst, int mode,
                                                     Ctl *ctl)
{
    if (ctl->st.flags) return;
    const double nrm2 = mode == 0 ? ctl->st.aux : ctl->st.rr;
    if (mode == 0 && !(nrm2 > 1e-28 * ctl->st.aux0)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            ctl->st.flags |= FLAG_BREAKDOWN;
            ctl->st.where = WHERE_ARNOLDI;
        }
        return;
    }
    if (!(nrm2 > 0.0)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            ctl->st.flags |= FLAG_BREAKDOWN;
            ctl->st.where = WHERE_ARNOLDI;
        }
        return;
    }
    const T inv = (T)(1.0 / sqrt(nrm2));
    for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < ld;
         e += (int64_t)gridDim.x * BLOCK)
        dst[e] = src[e] * inv;
}

// ---------------------------------------------------------------------------
// Elementwise helpers.
// ---------------------------------------------------------------------------
template <typename TD, typename TS>
__global__ __launch_bounds__(BLOCK) void k_copy_cast(int64_t n, const TS *__restrict__ src,
                                                     TD *__restrict__ dst)
{
    for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * BLOCK)
        dst[e] = (TD)src[e];
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_fill(int64_t n, T *dst, T v)
{
    for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * BLOCK)
        dst[e] = v;
}

// r32 = (float)(r64 * inv_sigma)
static __global__ __launch_bounds__(BLOCK) void k_scale_to_f32(int64_t n, const double *__restrict__ r,
                                                        double inv_sigma, float *__restrict__ out)
{
    for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * BLOCK)
        out[e] = (float)(r[e] * inv_sigma);
}

// x64 += sigma * (double)d32
static __global__ __launch_bounds__(BLOCK) void k_correct(int64_t n, const float *__restrict__ d,
                                                   double sigma, double *__restrict__ x)
{
    for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * BLOCK)
        x[e] = fma(sigma, (double)d[e], x[e]);
}

// P^T y and ||y||^2 of one vector.  dst 0: ptv[0][q] (recycled V); dst 1: ptt, tt;
// dst 2: prec[q] (fetched V).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_project(int64_t n, const T *__restrict__ y,
                                                   PBasis pkey, int s, int dst, int q, Ctl *ctl,
                                                   double *part, int stride)
{
    double acc[MAXS + 1];
#pragma unroll
    for (int v = 0; v <= MAXS; ++v) acc[v] = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * BLOCK) {
        const double yv = (double)y[e];
#pragma unroll
        for (int a = 0; a < MAXS; ++a)
            if (a < s) acc[a] += pval(pkey, (uint32_t)e, a) * yv;
        acc[MAXS] += yv * yv;
    }
    double vals[MAXS + 1];
#pragma unroll
    for (int v = 0; v <= MAXS; ++v) vals[v] = (v < s) ? acc[v] : ((v == s) ? acc[MAXS] : 0.0);
    block_partials<MAXS + 1>(vals, s + 1, part, stride);
    __shared__ double tot[MAXS + 1];
    if (!last_block_reduce(part, stride, s + 1, &ctl->counter[3], ctl->gcount[3], tot)) return;
    if (threadIdx.x != 0) return;
    if (dst == 0) {
        for (int a = 0; a < s; ++a) ctl->ptv[0][q][a] = tot[a];
    } else if (dst == 2) {
        for (int a = 0; a < s; ++a) ctl->prec[q][a] = tot[a];
    } else {
        for (int a = 0; a < s; ++a) ctl->ptt[a] = tot[a];
        ctl->st.tt = tot[s];
    }
}

// ---------------------------------------------------------------------------
// Orthonormalization of fetched recycle data (an option; the paper keeps U, V
// as a cycle leaves them): CholQR in FP64.  G = U^T U = L L^T, then
// U := U L^-T and V := V L^-T column by column, which keeps V = A U and the
// span of U (so the projection of the next right-hand side, Section 4.2, is
// unchanged in exact arithmetic).
// ---------------------------------------------------------------------------

// Upper triangle of U^T U (FP64 sums of products of the stored values), then
// in one thread the Cholesky factor: d_j = g_jj - sum_k l_jk^2,
// l_jj = sqrt(d_j), l_ij = (g_ij - sum_k l_ik l_jk) / l_jj, each product
// rounded before its subtraction.  d_j <= 1e-28 g_jj (or not positive) means
// G is not numerically positive definite: chol_ok = 0 and the data stay as
// fetched.
template <typename T, int S>
__global__ __launch_bounds__(BLOCK) void k_chol_gram(int64_t ld, const T *__restrict__ U, Ctl *ctl,
                                                     double *part, int stride)
{
#pragma clang fp contract(off)
    constexpr int NV = S * (S + 1) / 2;
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < ld;
         e += (int64_t)gridDim.x * BLOCK) {
        double u[S];
#pragma unroll
        for (int i = 0; i < S; ++i) u[i] = (double)U[(int64_t)i * ld + e];
        int v = 0;
#pragma unroll
        for (int i = 0; i < S; ++i)
#pragma unroll
            for (int j = i; j < S; ++j) acc[v++] += u[i] * u[j];
    }
    block_partials<NV>(acc, NV, part, stride);
    __shared__ double tot[NV];
    if (!last_block_reduce(part, stride, NV, &ctl->counter[3], ctl->gcount[3], tot)) return;
    if (threadIdx.x != 0) return;
    double G[S][S], L[S][S];
    int v = 0;
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
        for (int j = i; j < S; ++j) {
            G[i][j] = G[j][i] = tot[v++];
            L[i][j] = L[j][i] = 0.0;
        }
    bool ok = true;
#pragma unroll
    for (int j = 0; j < S; ++j) {
        double d = G[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
        ok = ok && (d > 0.0) && (d > 1e-28 * G[j][j]);
        L[j][j] = sqrt(d);
#pragma unroll
        for (int i = j + 1; i < S; ++i) {
            double t = G[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
            L[i][j] = t / L[j][j];
        }
    }
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
        for (int j = 0; j < S; ++j) ctl->chol[i][j] = L[i][j];
    ctl->chol_ok = ok ? 1 : 0;
}

// B := B L^-T for the s columns of U and (if not NULL) V, element by element:
// x_j = (b_j - sum_{i<j} l_ji x_i) / l_jj in FP64 with each product rounded,
// the result rounded to T.  Nothing is written unless chol_ok.
template <typename T, int S>
__global__ __launch_bounds__(BLOCK) void k_chol_apply(int64_t ld, T *__restrict__ U, T *__restrict__ V,
                                                      const Ctl *ctl)
{
#pragma clang fp contract(off)
    if (!ctl->chol_ok) return;
    double L[S][S];
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) L[i][j] = ctl->chol[i][j];
    for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < ld;
         e += (int64_t)gridDim.x * BLOCK) {
        for (int m = 0; m < (V ? 2 : 1); ++m) {
            T *B = m == 0 ? U : V;
            double x[S];
#pragma unroll
            for (int j = 0; j < S; ++j) {
                double a = (double)B[(int64_t)j * ld + e];
#pragma unroll
                for (int i = 0; i < j; ++i) a -= L[j][i] * x[i];
                x[j] = a / L[j][j];
            }
#pragma unroll
            for (int j = 0; j < S; ++j) B[(int64_t)j * ld + e] = (T)x[j];
        }
    }
}

// Implicit Euler right-hand side b = x inv_dt + f, multiply then add (no contraction).
static __global__ __launch_bounds__(BLOCK) void k_rhs_step(int64_t n, const double *__restrict__ x,
                                                    double inv_dt, const double *__restrict__ f,
                                                    double *__restrict__ b)
{
#pragma clang fp contract(off)
    for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * BLOCK) {
        const double t = x[e] * inv_dt;
        b[e] = t + f[e];
    }
}

// Split diagonal preconditioning (Section 5.1's split form, L = R = |D|^(1/2)):
// e_i = sqrt(|a_ii|) and d_i = 1 / e_i, both correctly rounded.  A row whose
// diagonal entry is not stored, zero or not finite sets *bad (and gets 1).
static __global__ __launch_bounds__(BLOCK) void k_jacobi_diag(int64_t n, const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ ci,
                                                       const double *__restrict__ va,
                                                       double *__restrict__ d,
                                                       double *__restrict__ e, int *bad)
{
    for (int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * BLOCK) {
        double a = 0.0;
        for (int32_t j = rp[r]; j < rp[r + 1]; ++j)
            if (ci[j] == r) a = va[j];
        double ev = 1.0;
        if (a != 0.0 && isfinite(a)) ev = sqrt(fabs(a));
        else __hip_atomic_store(bad, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        e[r] = ev;
        d[r] = 1.0 / ev;
    }
}

// Values of L^-1 A R^-1: out_k = (a_ij d_i) d_j, two roundings, no contraction.
static __global__ __launch_bounds__(BLOCK) void k_jacobi_scale(int64_t n, const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ ci,
                                                        const double *__restrict__ va,
                                                        const double *__restrict__ d,
                                                        double *__restrict__ out)
{
#pragma clang fp contract(off)
    for (int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * BLOCK) {
        const double di = d[r];
        for (int32_t j = rp[r]; j < rp[r + 1]; ++j) {
            const double t = va[j] * di;
            out[j] = t * d[ci[j]];
        }
    }
}

// y = x * w elementwise (y may alias x).
static __global__ __launch_bounds__(BLOCK) void k_mul(int64_t n, const double *x,
                                               const double *__restrict__ w, double *y)
{
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * BLOCK)
        y[i] = x[i] * w[i];
}

}  // namespace mstab
