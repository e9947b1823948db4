// Host side of the M(s)stab(l) / IDR(s)stab(l) solver and its C ABI.
//
// One Engine<T> runs Algorithm 1 of arXiv 1604.06043 in precision T with all
// state on the device; the host only enqueues kernels and reads a 56-byte
// status block once per cycle.  The FP64 mode runs Engine<double> on the
// system itself (with an FP32 copy of the matrix for the iteration's products
// in the F32_MATRIX mode); the F32_REFINE mode runs Engine<float> on the
// residual scaled by its FP64 norm, replacing the FP32 residual by the FP64
// true residual after its cycles and keeping the FP32 recycle data across
// systems.
#include "gmres.hpp"
#include "ilu.hpp"
#include "kernels.hpp"
#include "mstab.h"
#include "wg.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <new>
#include <string>
#include <atomic>
#include <thread>
#include <vector>

using namespace mstab;

namespace {

thread_local std::string g_tls_error;

struct HipError {
    hipError_t e;
    const char *what;
};

#define HIPCHK(call)                                              \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) throw HipError{e_, #call};          \
    } while (0)

struct StatusError {
    mstab_status st;
    std::string msg;
};

[[noreturn]] void fail(mstab_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    throw StatusError{st, buf};
}

uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// 32-bit key of P: low word of the start of splitmix64 stream 3 of the seed.
uint32_t p_key_from_seed(uint64_t seed)
{
    const uint64_t stream = 3;   // the P stream
    return (uint32_t)(mix64(seed ^ mix64(stream + 1)) & 0xFFFFFFFFull);
}

int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

int grid_for(int64_t work, int per_block, int cap)
{
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

#ifndef MSTAB_SPMV_MAX_BLOCKS
#define MSTAB_SPMV_MAX_BLOCKS 1024
#endif
constexpr int SPMV_MAX_BLOCKS = MSTAB_SPMV_MAX_BLOCKS;
// The constant-diagonal product: two workgroups per compute unit, all
// resident at once, eight rows per thread (24.1 us against 28.0 us with 1024
// workgroups at 128^3; fewer partials for its final reduction, too).
#ifndef MSTAB_SPMV_CONST_BLOCKS
#define MSTAB_SPMV_CONST_BLOCKS 512
#endif
constexpr int SPMV_CONST_MAX_BLOCKS = MSTAB_SPMV_CONST_BLOCKS;
constexpr int VEC_MAX_BLOCKS = 8192;
constexpr int GRAM_MAX_BLOCKS = 1024;
constexpr int POLY_MAX_BLOCKS = 1024;
constexpr int PART_STRIDE = MAX_PARTIAL_BLOCKS;  // >= every reduction grid
static_assert(SPMV_MAX_BLOCKS <= MAX_PARTIAL_BLOCKS && GRAM_MAX_BLOCKS <= MAX_PARTIAL_BLOCKS &&
                  POLY_MAX_BLOCKS <= MAX_PARTIAL_BLOCKS,
              "a reduction grid may not exceed the partials the final reduction reads");
constexpr int PART_VALUES = MAXS + MAXS * MAXS + 1;

// ---------------------------------------------------------------------------
// Kernel timing for the roofline report.
// ---------------------------------------------------------------------------
struct Profiler {
    bool on = false;
    int period = 1;                 // time one launch in `period` of each class
    int64_t seen[MSTAB_K_COUNT] = {};
    hipStream_t stream = nullptr;
    std::vector<hipEvent_t> ev;     // 2 per slot
    std::vector<int> cls;
    std::vector<double> bytes;
    int used = 0;
    int64_t launches[MSTAB_K_COUNT] = {};
    double ms[MSTAB_K_COUNT] = {};
    double nbytes[MSTAB_K_COUNT] = {};

    void init(hipStream_t s)
    {
        stream = s;
        ev.resize(2 * 512);
        cls.resize(512);
        bytes.resize(512);
        for (auto &e : ev) HIPCHK(hipEventCreate(&e));
    }
    void destroy()
    {
        for (auto &e : ev) (void)hipEventDestroy(e);
        ev.clear();
    }
    void reset()
    {
        used = 0;
        for (int c = 0; c < MSTAB_K_COUNT; ++c) { launches[c] = 0; ms[c] = 0; nbytes[c] = 0; seen[c] = 0; }
    }
    // returns slot or -1
    int begin(int c, double b)
    {
        if (!on) return -1;
        if (seen[c]++ % period != 0) return -1;
        if (used == (int)cls.size()) harvest();
        int i = used++;
        cls[i] = c;
        bytes[i] = b;
        HIPCHK(hipEventRecord(ev[2 * i], stream));
        return i;
    }
    void end(int i)
    {
        if (i >= 0) HIPCHK(hipEventRecord(ev[2 * i + 1], stream));
    }
    void harvest()
    {
        if (used == 0) return;
        HIPCHK(hipEventSynchronize(ev[2 * (used - 1) + 1]));
        for (int i = 0; i < used; ++i) {
            float t = 0.f;
            HIPCHK(hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]));
            launches[cls[i]] += 1;
            ms[cls[i]] += t;
            nbytes[cls[i]] += bytes[i];
        }
        used = 0;
    }
};

// CSR structure checks (the error contract: a malformed matrix is refused
// with E_INVALID before any kernel gathers through its indices).
// Host row pointer: rp[0] = 0, non-decreasing, rp[n] = nnz.
void check_row_ptr(int64_t n, int64_t nnz, const int32_t *rp)
{
    if (rp[0] != 0) fail(MSTAB_E_INVALID, "row_ptr[0] = %d, not 0", rp[0]);
    for (int64_t i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i]) fail(MSTAB_E_INVALID, "row_ptr decreases at row %lld", (long long)i);
    if (rp[n] != nnz)
        fail(MSTAB_E_INVALID, "row_ptr[n] = %d, not nnz = %lld", rp[n], (long long)nnz);
}

// Host column indices: in [0, n) and strictly increasing within each row
// (the row pointer checked first).
void check_columns_host(int64_t n, const int32_t *rp, const int32_t *ci)
{
    for (int64_t i = 0; i < n; ++i) {
        int64_t prev = -1;
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            if (ci[k] <= prev || ci[k] >= n)
                fail(MSTAB_E_INVALID, "row %lld: column index %d out of range or not increasing",
                     (long long)i, ci[k]);
            prev = ci[k];
        }
    }
}

// The same checks on a device CSR matrix: the row pointer on a host copy, the
// columns by one kernel that reads only the (then known-sized) index array.
void check_csr_dev(int64_t n, int64_t nnz, const int32_t *rp, const int32_t *ci, hipStream_t st)
{
    if (n < 1) return;
    std::vector<int32_t> h((size_t)n + 1);
    HIPCHK(hipMemcpyAsync(h.data(), rp, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    check_row_ptr(n, nnz, h.data());
    if (nnz == 0) return;
    int *bad = nullptr;
    int hbad = 0;
    HIPCHK(hipMalloc(&bad, sizeof(int)));
    hipError_t e = hipMemsetAsync(bad, 0, sizeof(int), st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_csr_check, dim3(grid_for(n, BLOCK, VEC_MAX_BLOCKS)), dim3(BLOCK), 0, st,
                           n, rp, ci, bad);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st);
    const hipError_t se = hipStreamSynchronize(st);
    (void)hipFree(bad);
    HIPCHK(e);
    HIPCHK(se);
    if (hbad) fail(MSTAB_E_INVALID, "a column index is outside [0, n) or not increasing within its row");
}

// Build the sliced ELLPACK copy of a device CSR matrix (setup only): slice
// widths from a host copy of the row pointer, then one scatter kernel.
// With share_col, the column array of `other` is reused.
// Diagonals of a CSR matrix (GPU table of MAX_DIAG slots): returns their
// number, ascending in *out, or 0 if there are more than MAX_DIAG or the
// diagonal storage would pad more than a quarter of the entries.
inline int detect_diagonals(int64_t n, int64_t nnz, const int32_t *rp, const int32_t *ci,
                            hipStream_t st, DiaOffsets *out)
{
    if (n < 1 || nnz < 1) return 0;
    unsigned long long *table = nullptr;
    int *overflow = nullptr;
    HIPCHK(hipMalloc(&table, sizeof(unsigned long long) * MAX_DIAG));
    HIPCHK(hipMalloc(&overflow, sizeof(int)));
    std::vector<unsigned long long> h(MAX_DIAG, DIA_EMPTY);
    int hov = 0;
    HIPCHK(hipMemcpyAsync(table, h.data(), sizeof(unsigned long long) * MAX_DIAG,
                          hipMemcpyHostToDevice, st));
    HIPCHK(hipMemsetAsync(overflow, 0, sizeof(int), st));
    hipLaunchKernelGGL(k_dia_offsets, dim3(grid_for(n, BLOCK, VEC_MAX_BLOCKS)), dim3(BLOCK), 0, st,
                       n, rp, ci, table, overflow);
    const hipError_t le = hipGetLastError();
    HIPCHK(hipMemcpyAsync(h.data(), table, sizeof(unsigned long long) * MAX_DIAG,
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&hov, overflow, sizeof(int), hipMemcpyDeviceToHost, st));
    const hipError_t se = hipStreamSynchronize(st);
    (void)hipFree(table);
    (void)hipFree(overflow);
    HIPCHK(le);
    HIPCHK(se);
    if (hov) return 0;
    std::vector<int64_t> offs;
    for (unsigned long long v : h)
        if (v != DIA_EMPTY) offs.push_back((int64_t)v);
    std::sort(offs.begin(), offs.end());
    const int nd = (int)offs.size();
    if (nd == 0 || (double)nd * (double)n > 1.25 * (double)nnz) return 0;
    for (int d = 0; d < MAX_DIAG; ++d) out->off[d] = d < nd ? offs[d] : 0;
    return nd;
}

// Reverse Cuthill-McKee order of the symmetrized pattern of a CSR matrix
// (host arrays): perm[new] = old.  Components are taken in order of their
// lowest-degree unvisited node; each is searched breadth-first from a
// minimum-degree node of the last level of a first search from that node (a
// pseudo-peripheral start), neighbours appended in order of degree, then
// index; the whole order is reversed at the end.
std::vector<int32_t> rcm_order(int64_t n, const int32_t *rp, const int32_t *ci)
{
    std::vector<int64_t> start((size_t)n + 1, 0);
    for (int64_t i = 0; i < n; ++i)
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
            if (ci[k] != i) { ++start[i + 1]; ++start[(size_t)ci[k] + 1]; }
    for (int64_t i = 0; i < n; ++i) start[i + 1] += start[i];
    std::vector<int32_t> adj((size_t)start[n]);
    {
        std::vector<int64_t> fill(start.begin(), start.end() - 1);
        for (int64_t i = 0; i < n; ++i)
            for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
                if (ci[k] != i) {
                    adj[(size_t)fill[i]++] = ci[k];
                    adj[(size_t)fill[ci[k]]++] = (int32_t)i;
                }
    }
    std::vector<int32_t> deg((size_t)n);
    std::vector<int64_t> end((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        auto b = adj.begin() + start[i], e = adj.begin() + start[i + 1];
        std::sort(b, e);
        end[i] = start[i] + (std::unique(b, e) - b);
        deg[i] = (int32_t)(end[i] - start[i]);
    }
    std::vector<int32_t> by_deg((size_t)n);
    for (int64_t i = 0; i < n; ++i) by_deg[i] = (int32_t)i;
    std::stable_sort(by_deg.begin(), by_deg.end(), [&](int32_t a, int32_t b) { return deg[a] < deg[b]; });
    std::vector<int32_t> order;
    order.reserve((size_t)n);
    std::vector<int32_t> mark((size_t)n, -1);   // component of the first search
    std::vector<char> seen((size_t)n, 0);
    std::vector<int32_t> q, nb;
    int32_t comp = 0;
    for (int32_t s0 : by_deg) {
        if (seen[s0]) continue;
        // first search: its last level holds the pseudo-peripheral start
        q.assign(1, s0);
        mark[s0] = comp;
        size_t head = 0, level_begin = 0;
        while (head < q.size()) {
            const size_t level_end = q.size();
            level_begin = head;
            for (; head < level_end; ++head) {
                const int32_t v = q[head];
                for (int64_t k = start[v]; k < end[v]; ++k)
                    if (mark[adj[k]] != comp) { mark[adj[k]] = comp; q.push_back(adj[k]); }
            }
        }
        int32_t root = q[level_begin];
        for (size_t k = level_begin; k < q.size(); ++k)
            if (deg[q[k]] < deg[root] || (deg[q[k]] == deg[root] && q[k] < root)) root = q[k];
        ++comp;
        // Cuthill-McKee search from the root
        const size_t first = order.size();
        order.push_back(root);
        seen[root] = 1;
        for (size_t h = first; h < order.size(); ++h) {
            const int32_t v = order[h];
            nb.clear();
            for (int64_t k = start[v]; k < end[v]; ++k)
                if (!seen[adj[k]]) { seen[adj[k]] = 1; nb.push_back(adj[k]); }
            std::sort(nb.begin(), nb.end(), [&](int32_t a, int32_t b) {
                return deg[a] != deg[b] ? deg[a] < deg[b] : a < b;
            });
            order.insert(order.end(), nb.begin(), nb.end());
        }
    }
    std::reverse(order.begin(), order.end());
    return order;
}

// A multicolour order of the symmetrized pattern of a CSR matrix (host
// arrays; diagonal ignored): nodes in index order take the smallest colour
// that none of their already coloured neighbours (in A or A^T) has.  Returns
// perm[new] = old, colour by colour, index order within a colour; cp receives
// the first new index of each colour and n.  No entry then couples two rows
// of one colour.
std::vector<int32_t> multicolour_order(int64_t n, const int32_t *rp, const int32_t *ci,
                                       std::vector<int64_t> &cp)
{
    // transposed pattern
    std::vector<int64_t> tptr((size_t)n + 1, 0);
    for (int64_t k = 0; k < rp[n]; ++k) tptr[(size_t)ci[k] + 1]++;
    for (int64_t i = 0; i < n; ++i) tptr[i + 1] += tptr[i];
    std::vector<int32_t> tcol((size_t)std::max<int64_t>(rp[n], 1));
    {
        std::vector<int64_t> pos(tptr.begin(), tptr.end() - 1);
        for (int64_t i = 0; i < n; ++i)
            for (int64_t k = rp[i]; k < rp[i + 1]; ++k) tcol[(size_t)pos[ci[k]]++] = (int32_t)i;
    }
    std::vector<int32_t> colour((size_t)n, 0);
    std::vector<int64_t> used;   // used[c] == i: colour c taken by a neighbour of node i
    int ncol = 0;
    for (int64_t i = 0; i < n; ++i) {
        auto take = [&](int32_t j) {
            if (j < i) {
                const int c = colour[j];
                if ((int)used.size() <= c) used.resize((size_t)c + 1, -1);
                used[c] = i;
            }
        };
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) take(ci[k]);
        for (int64_t k = tptr[i]; k < tptr[i + 1]; ++k) take(tcol[k]);
        int c = 0;
        while (c < (int)used.size() && used[c] == i) ++c;
        colour[i] = c;
        ncol = std::max(ncol, c + 1);
    }
    cp.assign((size_t)ncol + 1, 0);
    for (int64_t i = 0; i < n; ++i) cp[(size_t)colour[i] + 1]++;
    for (int c = 0; c < ncol; ++c) cp[c + 1] += cp[c];
    std::vector<int32_t> perm((size_t)n);
    std::vector<int64_t> pos(cp.begin(), cp.end() - 1);
    for (int64_t i = 0; i < n; ++i) perm[(size_t)pos[colour[i]]++] = (int32_t)i;
    return perm;
}

// The symmetrically permuted CSR matrix P A P^T (row new = row perm[new]),
// columns re-sorted, on the host.
void permute_csr(int64_t n, const std::vector<int32_t> &rp, const std::vector<int32_t> &ci,
                 const std::vector<double> &va, const std::vector<int32_t> &perm,
                 std::vector<int32_t> &prp, std::vector<int32_t> &pci, std::vector<double> &pva)
{
    std::vector<int32_t> iperm((size_t)n);
    for (int64_t i = 0; i < n; ++i) iperm[perm[i]] = (int32_t)i;
    prp.assign((size_t)n + 1, 0);
    pci.resize(ci.size());
    pva.resize(va.size());
    std::vector<std::pair<int32_t, double>> row;
    for (int64_t i = 0; i < n; ++i) {
        const int32_t o = perm[i];
        row.clear();
        for (int32_t k = rp[o]; k < rp[o + 1]; ++k) row.emplace_back(iperm[ci[k]], va[k]);
        std::sort(row.begin(), row.end(),
                  [](const std::pair<int32_t, double> &a, const std::pair<int32_t, double> &b) {
                      return a.first < b.first;
                  });
        int64_t w = prp[i];
        for (const auto &e : row) { pci[w] = e.first; pva[w] = e.second; ++w; }
        prp[i + 1] = (int32_t)w;
    }
}

// dst[i] = src[perm[i]] (times w[i] if w), and its inverse dst[perm[i]] = src[i] (times w[i]).
__global__ __launch_bounds__(BLOCK) void k_gather(int64_t n, const int32_t *__restrict__ perm,
                                                  const double *__restrict__ src,
                                                  const double *__restrict__ w,
                                                  double *__restrict__ dst)
{
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * BLOCK) {
        const double v = src[perm[i]];
        dst[i] = w ? v * w[i] : v;
    }
}

__global__ __launch_bounds__(BLOCK) void k_scatter(int64_t n, const int32_t *__restrict__ perm,
                                                   const double *__restrict__ src,
                                                   const double *__restrict__ w,
                                                   double *__restrict__ dst)
{
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * BLOCK) {
        const double v = src[i];
        dst[perm[i]] = w ? v * w[i] : v;
    }
}

// Split diagonal preconditioning: d, e (n doubles each) and the values of
// L^-1 A R^-1 in A's pattern (val_out, nnz doubles).  E_INVALID if a row has
// no stored, finite, nonzero diagonal entry.
inline void jacobi_split_dev(int64_t n, const int32_t *rp, const int32_t *ci, const double *va,
                             double *val_out, double *d, double *e, hipStream_t st)
{
    if (n < 1) return;
    int *bad = nullptr;
    int hbad = 0;
    HIPCHK(hipMalloc(&bad, sizeof(int)));
    hipError_t ce = hipMemsetAsync(bad, 0, sizeof(int), st);
    const int grid = grid_for(n, BLOCK, VEC_MAX_BLOCKS);
    if (ce == hipSuccess) {
        hipLaunchKernelGGL(k_jacobi_diag, dim3(grid), dim3(BLOCK), 0, st, n, rp, ci, va, d, e, bad);
        ce = hipGetLastError();
    }
    if (ce == hipSuccess) ce = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st);
    const hipError_t se = hipStreamSynchronize(st);
    (void)hipFree(bad);
    HIPCHK(ce);
    HIPCHK(se);
    if (hbad) fail(MSTAB_E_INVALID, "Jacobi splitting: a diagonal entry is missing, zero or not finite");
    hipLaunchKernelGGL(k_jacobi_scale, dim3(grid), dim3(BLOCK), 0, st, n, rp, ci, va, d, val_out);
    HIPCHK(hipGetLastError());
}

// The device copy of A used by the product kernels: diagonal storage when A
// is a stencil matrix (at most 16 diagonals), else sliced ELLPACK.  like: the
// FP64 copy whose column array (or diagonal mask) this copy shares.
template <typename T, typename TS>
Sell<T> make_sell(int64_t n, const int32_t *rp, const int32_t *ci, const TS *va, hipStream_t st,
                  const Sell<double> *like = nullptr, int format = MSTAB_FORMAT_AUTO)
{
    Sell<T> m;
    m.n = n;
    m.rp = rp;
    std::vector<int32_t> h((size_t)n + 1);
    HIPCHK(hipMemcpyAsync(h.data(), rp, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    m.nnz = h[n];
    const int grid = grid_for(n, BLOCK, VEC_MAX_BLOCKS);
    if (like) m.nd = like->nd;
    else if (format != MSTAB_FORMAT_SLICED) m.nd = detect_diagonals(n, m.nnz, rp, ci, st, &m.doff);
    if (m.nd > 0) {
        if (like) {
            m.doff = like->doff;
            m.dmask = like->dmask;
            if (like->dconst) {
                // the same constant diagonals, rounded to this copy's precision
                m.dconst = true;
                for (int d = 0; d < MAX_DIAG; ++d) m.cv.c[d] = (double)(T)like->cv.c[d];
                return m;
            }
        } else {
            HIPCHK(hipMalloc(&m.dmask, sizeof(uint16_t) * (size_t)n));
        }
        const size_t cnt = (size_t)m.nd * (size_t)round_up(n, 64);   // whole slices
        HIPCHK(hipMalloc(&m.dval, sizeof(T) * cnt));
        HIPCHK(hipMemsetAsync(m.dval, 0, sizeof(T) * cnt, st));
        hipLaunchKernelGGL((k_to_dia<T, TS>), dim3(grid), dim3(BLOCK), 0, st, n, rp, ci, va, m.nd,
                           m.doff, like ? nullptr : m.dmask, m.dval);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));
        if (!like && format == MSTAB_FORMAT_AUTO) {
            // constant diagonals: keep one value each instead of the value array
            unsigned long long *lohi = nullptr;
            std::vector<unsigned long long> hl(2 * MAX_DIAG);
            for (int d = 0; d < MAX_DIAG; ++d) { hl[d] = ~0ull; hl[MAX_DIAG + d] = 0ull; }
            HIPCHK(hipMalloc(&lohi, sizeof(unsigned long long) * 2 * MAX_DIAG));
            hipError_t e = hipMemcpyAsync(lohi, hl.data(), sizeof(unsigned long long) * 2 * MAX_DIAG,
                                          hipMemcpyHostToDevice, st);
            if (e == hipSuccess) {
                hipLaunchKernelGGL((k_dia_range<T>), dim3(grid), dim3(BLOCK), 0, st, n, m.nd,
                                   (const uint16_t *)m.dmask, (const T *)m.dval, lohi);
                e = hipGetLastError();
            }
            if (e == hipSuccess)
                e = hipMemcpyAsync(hl.data(), lohi, sizeof(unsigned long long) * 2 * MAX_DIAG,
                                   hipMemcpyDeviceToHost, st);
            const hipError_t se = hipStreamSynchronize(st);
            (void)hipFree(lohi);
            HIPCHK(e);
            HIPCHK(se);
            bool same = true;
            for (int d = 0; d < m.nd; ++d) same = same && hl[d] == hl[MAX_DIAG + d];
            if (same) {
                for (int d = 0; d < MAX_DIAG; ++d) {
                    T v = (T)0;
                    if (d < m.nd) {
                        if constexpr (sizeof(T) == 8) v = __builtin_bit_cast(T, (unsigned long long)hl[d]);
                        else v = __builtin_bit_cast(T, (uint32_t)hl[d]);
                    }
                    m.cv.c[d] = (double)v;
                }
                m.dconst = true;
                (void)hipFree(m.dval);
                m.dval = nullptr;
            }
        }
        return m;
    }
    const int64_t ns = (n + SLICE - 1) / SLICE;
    std::vector<int64_t> sp((size_t)ns + 1);
    sp[0] = 0;
    for (int64_t t = 0; t < ns; ++t) {
        int32_t w = 0;
        for (int64_t r = t * SLICE; r < std::min<int64_t>(n, (t + 1) * SLICE); ++r)
            w = std::max(w, h[r + 1] - h[r]);
        sp[t + 1] = sp[t] + (int64_t)w * SLICE;
    }
    m.padded = sp[ns];
    const size_t cnt = (size_t)std::max<int64_t>(m.padded, 1);
    HIPCHK(hipMalloc(&m.slice_ptr, sizeof(int64_t) * (ns + 1)));
    HIPCHK(hipMemcpyAsync(m.slice_ptr, sp.data(), sizeof(int64_t) * (ns + 1),
                          hipMemcpyHostToDevice, st));
    HIPCHK(hipMalloc(&m.val, sizeof(T) * cnt));
    HIPCHK(hipMemsetAsync(m.val, 0, sizeof(T) * cnt, st));        // padding: value 0
    const int32_t *share_col = like ? like->col : nullptr;
    if (share_col) {
        m.col = const_cast<int32_t *>(share_col);
    } else {
        HIPCHK(hipMalloc(&m.col, sizeof(int32_t) * cnt));
        HIPCHK(hipMemsetAsync(m.col, 0, sizeof(int32_t) * cnt, st)); // padding: column 0
    }
    hipLaunchKernelGGL((k_to_sell<T, TS>), dim3(grid), dim3(BLOCK), 0, st, n, rp, ci, va,
                       m.slice_ptr, share_col ? nullptr : m.col, m.val);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));   // sp (host) must outlive the copy
    return m;
}

template <typename T>
void free_sell(Sell<T> &m, bool own_col)
{
    (void)hipFree(m.slice_ptr);
    (void)hipFree(m.val);
    (void)hipFree(m.dval);
    if (own_col) {
        (void)hipFree(m.col);
        (void)hipFree(m.dmask);
    }
    m = Sell<T>();
}

// bytes a product must move: the matrix copy, x once, y (and b); vectors of
// vsize-byte elements
template <typename TM>
double spmv_bytes(const Sell<TM> &A, bool with_b, double vsize)
{
    const double n = (double)A.n;
    const double vecs = (with_b ? 3.0 : 2.0) * n * vsize;
    if (A.nd > 0) return (A.dconst ? 0.0 : (double)A.nd * n * sizeof(TM)) + 2.0 * n + vecs;
    return (n + 1) * 4 + (double)A.padded * (4 + sizeof(TM)) + (double)((A.n + SLICE - 1) / SLICE + 1) * 8 +
           vecs;
}

// The two-rows-per-thread product applies: diagonal storage, n even, the
// offsets -1, 0, +1 in the middle and the others even, and the vectors, the
// mask and the values aligned for pair loads.
template <typename T, typename TM>
bool pairs_ok(const Sell<TM> &A, const T *x, const T *y, const T *b)
{
    if (A.nd != 7 && A.nd != 5) return false;
    const int C = A.nd / 2;
    if (A.n % 2 || A.doff.off[C] != 0 || A.doff.off[C - 1] != -1 || A.doff.off[C + 1] != 1) return false;
    for (int d = 0; d < A.nd; ++d)
        if (d != C - 1 && d != C + 1 && (A.doff.off[d] % 2)) return false;
    const uintptr_t al = 2 * sizeof(T);
    return (uintptr_t)x % al == 0 && (uintptr_t)y % al == 0 && (!b || (uintptr_t)b % al == 0) &&
           (uintptr_t)A.dmask % 4 == 0 && (A.dconst || (uintptr_t)A.dval % (2 * sizeof(TM)) == 0);
}

// TM: value type of the stored matrix (T, or float for an FP32 copy used with
// FP64 vectors); PM: P from the generator (0) or the caller's matrix (1)
template <int PM, typename T, typename TM>
void launch_spmv_pm(int grid, hipStream_t stream, const Sell<TM> &A, const T *x, T *y, const T *b,
                    Ctl *ctl, double *part, SpmvArgs a)
{
    if ((A.nd == 7 || A.nd == 5) && pairs_ok(A, x, y, b)) {
        // two rows per thread (constant or streamed diagonals, 7 or 5 of them)
        switch (a.s) {
#define LAUNCH(S, CST, ND)                                                                            \
    hipLaunchKernelGGL((k_spmv_dia_pair<T, S, TM, CST, ND, PM>), dim3(grid), dim3(SPMV_BLOCK), 0, stream, \
                       A.n, A.doff, A.cv, A.dmask, (const TM *)A.dval, x, y, b, ctl, part, PART_STRIDE, a)
#define CASE(S)                                                                                       \
    case S:                                                                                           \
        if (A.dconst) {                                                                               \
            if (A.nd == 7) LAUNCH(S, true, 7); else LAUNCH(S, true, 5);                               \
        } else {                                                                                      \
            if (A.nd == 7) LAUNCH(S, false, 7); else LAUNCH(S, false, 5);                             \
        }                                                                                             \
        break;
            CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
#undef LAUNCH
        }
        return;
    }
    if (A.nd > 0 && A.dconst && (A.nd == 7 || A.nd == 5)) {
        switch (a.s) {
#define CASE(S)                                                                                      \
    case S:                                                                                          \
        if (A.nd == 7)                                                                               \
            hipLaunchKernelGGL((k_spmv_dia_const<T, S, 7, PM>), dim3(grid), dim3(SPMV_BLOCK), 0, stream, \
                               A.n, A.doff, A.cv, A.dmask, x, y, b, ctl, part, PART_STRIDE, a);      \
        else                                                                                         \
            hipLaunchKernelGGL((k_spmv_dia_const<T, S, 5, PM>), dim3(grid), dim3(SPMV_BLOCK), 0, stream, \
                               A.n, A.doff, A.cv, A.dmask, x, y, b, ctl, part, PART_STRIDE, a);      \
        break;
            CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        }
        return;
    }
    if (A.nd > 0) {
        switch (a.s) {
#define CASE(S)                                                                                   \
    case S:                                                                                       \
        if (A.dconst)                                                                             \
            hipLaunchKernelGGL((k_spmv_dia<T, S, TM, true, PM>), dim3(grid), dim3(SPMV_BLOCK), 0, stream, \
                               A.n, A.nd, A.doff, A.cv, A.dmask, (const TM *)A.dval, x, y, b, ctl,    \
                               part, PART_STRIDE, a);                                                 \
        else                                                                                      \
            hipLaunchKernelGGL((k_spmv_dia<T, S, TM, false, PM>), dim3(grid), dim3(SPMV_BLOCK), 0, stream,\
                               A.n, A.nd, A.doff, A.cv, A.dmask, (const TM *)A.dval, x, y, b, ctl,    \
                               part, PART_STRIDE, a);                                                 \
        break;
            CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        }
        return;
    }
    switch (a.s) {
#define CASE(S)                                                                                \
    case S:                                                                                    \
        hipLaunchKernelGGL((k_spmv<T, S, TM, PM>), dim3(grid), dim3(SPMV_BLOCK), 0, stream, A.n, A.rp, \
                           A.slice_ptr, A.col, A.val, x, y, b, ctl, part, PART_STRIDE, a);     \
        break;
        CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    }
}

template <typename T, typename TM = T>
void launch_spmv(int grid, hipStream_t stream, const Sell<TM> &A, const T *x, T *y, const T *b,
                 Ctl *ctl, double *part, SpmvArgs a)
{
    if (a.pkey.m)
        launch_spmv_pm<1>(grid, stream, A, x, y, b, ctl, part, a);
    else
        launch_spmv_pm<0>(grid, stream, A, x, y, b, ctl, part, a);
}

// The fetch point "shortly before the residual drops" (Section 5, how to
// choose the fetching point), estimated from a finished solve's history of
// recursive relative residuals (initial, then one per cycle): the cycle before
// the largest one-cycle reduction, res[k-1] / res[k] (the first on ties), at
// least cycle 1; -1 when no cycle ran.  FETCH_ESTIMATE applies it to the next
// solve of the sequence.
int64_t estimate_fetch_cycle(const std::vector<double> &h)
{
    int64_t best_k = -1;
    double best = -1.0;
    for (size_t k = 1; k < h.size(); ++k) {
        const double f = h[k] > 0.0 ? h[k - 1] / h[k] : INFINITY;
        if (f > best) { best = f; best_k = (int64_t)k; }
    }
    if (best_k < 0) return -1;
    return best_k > 1 ? best_k - 1 : 1;
}

struct SolveResult {
    int status = MSTAB_OK;
    bool converged = false;
    bool recycled = false;
    int restarts = 0;
    int replacements = 0;
    int64_t mv = 0, mv_check = 0, cycles = 0, level = 0, fetched = -1;
    double relres_rec = 0, relres_true = -1;
};

// ILU(0) factors of the multicolour-ordered matrix A' (device), for the
// preconditioned operator L^-1 A' U^-1.
struct IluData {
    int64_t n = 0, nnz = 0;
    const int32_t *rp = nullptr, *ci = nullptr;   // A''s CSR structure (device)
    double *lu = nullptr;                          // L below, U on and above the diagonal
    int32_t *dpos = nullptr;                       // position of each row's diagonal
    std::vector<int64_t> cp;                       // first row of each colour, and n
    double *t1 = nullptr, *t2 = nullptr;           // scratch vectors of the operator
    IluSell f;                                     // the factors sliced, for the solves
    // Eisenstat's form (the factors' off-diagonals are A''s): D_A - 2 D_U and D_U
    bool eis = false;
    double *dd = nullptr, *du = nullptr;

    int colours() const { return (int)cp.size() - 1; }
    // x := U^-1 z, colour by colour from the last (z and x distinct)
    void upper_solve(const double *z, double *x, hipStream_t st) const
    {
        for (int c = colours() - 1; c >= 0; --c) {
            const int64_t rows = cp[c + 1] - cp[c];
            hipLaunchKernelGGL(k_ilu_upper_sell, dim3(grid_for(rows, BLOCK, VEC_MAX_BLOCKS)), dim3(BLOCK), 0,
                               st, cp[c], cp[c + 1], rp, (const int32_t *)dpos, f, z, x);
            HIPCHK(hipGetLastError());
        }
    }
    // y := L^-1 y in place, colour by colour (colour 0 has no lower entries)
    void lower_solve(double *y, hipStream_t st) const
    {
        for (int c = 1; c < colours(); ++c) {
            const int64_t rows = cp[c + 1] - cp[c];
            hipLaunchKernelGGL(k_ilu_lower_sell, dim3(grid_for(rows, BLOCK, VEC_MAX_BLOCKS)), dim3(BLOCK), 0,
                               st, cp[c], cp[c + 1], rp, (const int32_t *)dpos, f, y);
            HIPCHK(hipGetLastError());
        }
    }
    // the sliced copies of the factors (host row pointer and diagonal
    // positions; lu final on the device)
    void make_sell(const std::vector<int32_t> &hrp, const std::vector<int32_t> &hdpos, hipStream_t st)
    {
        const int64_t ns = (n + SLICE - 1) / SLICE;
        std::vector<int64_t> lsp((size_t)ns + 1, 0), usp((size_t)ns + 1, 0);
        for (int64_t t = 0; t < ns; ++t) {
            int64_t lw = 0, uw = 0;
            for (int64_t r = t * SLICE; r < std::min(n, (t + 1) * SLICE); ++r) {
                lw = std::max<int64_t>(lw, hdpos[r] - hrp[r]);
                uw = std::max<int64_t>(uw, hrp[r + 1] - hdpos[r] - 1);
            }
            lsp[t + 1] = lsp[t] + lw * SLICE;
            usp[t + 1] = usp[t] + uw * SLICE;
        }
        const size_t ln = (size_t)std::max<int64_t>(lsp[ns], 1), un = (size_t)std::max<int64_t>(usp[ns], 1);
        HIPCHK(hipMalloc(&f.lsp, sizeof(int64_t) * (ns + 1)));
        HIPCHK(hipMalloc(&f.usp, sizeof(int64_t) * (ns + 1)));
        HIPCHK(hipMalloc(&f.lcol, sizeof(int32_t) * ln));
        HIPCHK(hipMalloc(&f.ucol, sizeof(int32_t) * un));
        HIPCHK(hipMalloc(&f.lval, sizeof(double) * ln));
        HIPCHK(hipMalloc(&f.uval, sizeof(double) * un));
        HIPCHK(hipMalloc(&f.udiag, sizeof(double) * (size_t)n));
        HIPCHK(hipMemsetAsync(f.lcol, 0, sizeof(int32_t) * ln, st));
        HIPCHK(hipMemsetAsync(f.ucol, 0, sizeof(int32_t) * un, st));
        HIPCHK(hipMemsetAsync(f.lval, 0, sizeof(double) * ln, st));
        HIPCHK(hipMemsetAsync(f.uval, 0, sizeof(double) * un, st));
        HIPCHK(hipMemcpyAsync(f.lsp, lsp.data(), sizeof(int64_t) * (ns + 1), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(f.usp, usp.data(), sizeof(int64_t) * (ns + 1), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_ilu_to_sell, dim3(grid_for(n, BLOCK, VEC_MAX_BLOCKS)), dim3(BLOCK), 0, st, n, rp, ci,
                           (const double *)lu, (const int32_t *)dpos, f);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));   // the host slice pointers go out of scope
    }
    void upper_mul(const double *x, double *y, hipStream_t st) const
    {
        hipLaunchKernelGGL(k_ilu_upper_mul, dim3(grid_for(n, BLOCK, VEC_MAX_BLOCKS)), dim3(BLOCK), 0, st, n,
                           rp, ci, (const double *)lu, (const int32_t *)dpos, x, y);
        HIPCHK(hipGetLastError());
    }
    void release()
    {
        (void)hipFree(lu); (void)hipFree(dpos); (void)hipFree(t1); (void)hipFree(t2);
        lu = nullptr; dpos = nullptr; t1 = t2 = nullptr;
        (void)hipFree(f.lsp); (void)hipFree(f.usp); (void)hipFree(f.lcol); (void)hipFree(f.ucol);
        (void)hipFree(f.lval); (void)hipFree(f.uval); (void)hipFree(f.udiag);
        f = IluSell{};
        (void)hipFree(dd); (void)hipFree(du);
        dd = du = nullptr;
        eis = false;
    }
};

// ---------------------------------------------------------------------------
// Engine<T>: Algorithm 1 with recycling, precision T, device-resident state.
// ---------------------------------------------------------------------------
template <typename T>
struct Engine {
    int s = 0, ell = 0;
    int64_t n = 0, ld = 0, nnz = 0;
    Sell<T> A;                          // sliced copy of the matrix
    bool own_col = true;
    PBasis pkey;
    hipStream_t stream = nullptr;

    T *W = nullptr, *R = nullptr, *X = nullptr, *Tv = nullptr;
    T *recU = nullptr, *recV = nullptr;
    double *rec_ptv = nullptr;         // device, MAXS*MAXS
    int64_t rec_level = 0;
    bool rec_have = false;
    // FETCH_ESTIMATE: the fetch cycle estimated from the last solve (-1: none)
    int64_t est_cycle = -1;

    Ctl *ctl = nullptr;
    Status *st_host = nullptr;         // pinned
    double *part = nullptr;
    Profiler *prof = nullptr;

    std::vector<int64_t> hist_mv;
    std::vector<double> hist_res;

    T *Wc(int lev, int q) const { return W + ((int64_t)(lev + 1) * s + q) * ld; }
    T *Rc(int i) const { return R + (int64_t)i * ld; }

    // full = false: only what the FP64 outer loop of the mixed mode needs
    void alloc(int64_t n_, int s_, int ell_, const Sell<T> &A_, bool own_col_, PBasis key,
               hipStream_t st, Profiler *pr, bool full = true)
    {
        n = n_; s = s_; ell = ell_; A = A_; own_col = own_col_; nnz = A_.nnz;
        pkey = key; stream = st; prof = pr;
        ld = round_up(n, 256);
        const size_t vb = (size_t)ld * sizeof(T);
        HIPCHK(hipMalloc(&X, vb));
        HIPCHK(hipMalloc(&Tv, vb));
        HIPCHK(hipMalloc(&ctl, sizeof(Ctl)));
        HIPCHK(hipMalloc(&part, sizeof(double) * (size_t)PART_STRIDE * PART_VALUES));
        HIPCHK(hipHostMalloc(&st_host, sizeof(Status), hipHostMallocDefault));
        HIPCHK(hipMemsetAsync(X, 0, vb, stream));
        HIPCHK(hipMemsetAsync(Tv, 0, vb, stream));
        HIPCHK(hipMemsetAsync(ctl, 0, sizeof(Ctl), stream));
        if (full) {
            HIPCHK(hipMalloc(&W, vb * s * (ell + 2)));
            HIPCHK(hipMalloc(&R, vb * (ell + 1)));
            HIPCHK(hipMalloc(&recU, vb * s));
            HIPCHK(hipMalloc(&recV, vb * s));
            HIPCHK(hipMalloc(&rec_ptv, sizeof(double) * MAXS * MAXS));
            HIPCHK(hipMemsetAsync(W, 0, vb * s * (ell + 2), stream));
            HIPCHK(hipMemsetAsync(R, 0, vb * (ell + 1), stream));
            HIPCHK(hipMemsetAsync(recU, 0, vb * s, stream));
            HIPCHK(hipMemsetAsync(recV, 0, vb * s, stream));
        }
        HIPCHK(hipStreamSynchronize(stream));
    }

    void release()
    {
        free_sell(A, own_col);
        if (use_low) free_sell(A_low, false);
        use_low = false;
        (void)hipFree(W); (void)hipFree(R); (void)hipFree(X); (void)hipFree(Tv);
        (void)hipFree(recU); (void)hipFree(recV); (void)hipFree(rec_ptv);
        (void)hipFree(ctl); (void)hipFree(part);
        (void)hipFree(gmV); (void)hipFree(gm_state);
        gmV = nullptr; gm_state = nullptr;
        if (st_host) (void)hipHostFree(st_host);
        W = R = X = Tv = recU = recV = nullptr;
        rec_ptv = nullptr; ctl = nullptr; part = nullptr; st_host = nullptr;
    }

    // ---- launches ---------------------------------------------------------
    double vbytes(double vectors) const { return vectors * (double)n * sizeof(T); }

    // FP32 copy of the matrix for the iteration's products (FP64 vectors; the
    // initial and true residuals keep the FP64 matrix), if set
    Sell<float> A_low{};
    bool use_low = false;
    // k > 0: replace the recursive residual by the true one after every k-th
    // cycle while it is above the tolerance (Section 5.1's ocean run, k = 1);
    // these replacements do not use up the budget of the final ones
    int replace_every = 0;
    // with A_low: replace the recursive residual by the true one whenever it
    // has fallen by this factor since the last true residual (the gap between
    // the two grows with the correction made since then)
    double low_drop = 1e-3;

    // ILU(0) split preconditioning: the products are L^-1 A U^-1 (FP64 only)
    const IluData *ilu = nullptr;

    // GMRES(m): basis v_1..v_{m+1} and the work vector w (m + 2 vectors of
    // ld), and the cycle's small state (GmLayout)
    T *gmV = nullptr;
    double *gm_state = nullptr;
    int gm_m = 0;
    void alloc_gmres(int m)
    {
        gm_m = m;
        HIPCHK(hipMalloc(&gmV, (size_t)ld * sizeof(T) * (size_t)(m + 2)));
        HIPCHK(hipMemsetAsync(gmV, 0, (size_t)ld * sizeof(T) * (size_t)(m + 2), stream));
        HIPCHK(hipMalloc(&gm_state, sizeof(double) * (size_t)GmLayout{m}.size()));
        HIPCHK(hipStreamSynchronize(stream));
    }

    template <int S>
    void vec_out_s(int grid, const T *t, const T *b, T *y, const SpmvArgs &a)
    {
        hipLaunchKernelGGL((k_vec_out<T, S>), dim3(grid), dim3(SPMV_BLOCK), 0, stream, n, t, b, y, ctl, part,
                           PART_STRIDE, a);
    }

    // y = L^-1 A U^-1 x (or b - that), then the product's epilogue for `act`
    template <int S>
    void vec_out_eis_s(int grid, const T *v, const T *t, const T *du, const T *b, T *y, const SpmvArgs &a)
    {
        hipLaunchKernelGGL((k_vec_out_eis<T, S>), dim3(grid), dim3(SPMV_BLOCK), 0, stream, n, v, t, du, b, y, ctl,
                           part, PART_STRIDE, a);
    }

    void ilu_product(const T *x, T *y, const T *b, const SpmvArgs &a)
    {
        if constexpr (sizeof(T) == 8) {
            if (ilu->eis) {
                // Eisenstat's form: t1 = U^-1 x, t2 = L^-1 (x + dd t1), y = t2 + du t1
                ilu->upper_solve(x, ilu->t1, stream);
                hipLaunchKernelGGL(k_ilu_eis_mid, dim3(grid_for(n, BLOCK, VEC_MAX_BLOCKS)), dim3(BLOCK), 0, stream,
                                   n, x, (const double *)ilu->t1, (const double *)ilu->dd, ilu->t2);
                HIPCHK(hipGetLastError());
                ilu->lower_solve(ilu->t2, stream);
                const int grid = grid_for(n, SPMV_BLOCK, SPMV_MAX_BLOCKS);
                const T *t1 = ilu->t1, *t2 = ilu->t2, *du = ilu->du;
                switch (s) {
                case 1: vec_out_eis_s<1>(grid, t2, t1, du, b, y, a); break;
                case 2: vec_out_eis_s<2>(grid, t2, t1, du, b, y, a); break;
                case 3: vec_out_eis_s<3>(grid, t2, t1, du, b, y, a); break;
                case 4: vec_out_eis_s<4>(grid, t2, t1, du, b, y, a); break;
                case 5: vec_out_eis_s<5>(grid, t2, t1, du, b, y, a); break;
                case 6: vec_out_eis_s<6>(grid, t2, t1, du, b, y, a); break;
                case 7: vec_out_eis_s<7>(grid, t2, t1, du, b, y, a); break;
                default: vec_out_eis_s<8>(grid, t2, t1, du, b, y, a); break;
                }
                HIPCHK(hipGetLastError());
                return;
            }
            ilu->upper_solve(x, ilu->t1, stream);
            SpmvArgs none{ACT_NONE, 0, 0, 0, 1, pkey};
            launch_spmv<T>(grid_for(n, SPMV_BLOCK, SPMV_MAX_BLOCKS), stream, A, ilu->t1, ilu->t2, nullptr,
                           ctl, part, none);
            HIPCHK(hipGetLastError());
            ilu->lower_solve(ilu->t2, stream);
            const int grid = grid_for(n, SPMV_BLOCK, SPMV_MAX_BLOCKS);
            switch (s) {
            case 1: vec_out_s<1>(grid, ilu->t2, b, y, a); break;
            case 2: vec_out_s<2>(grid, ilu->t2, b, y, a); break;
            case 3: vec_out_s<3>(grid, ilu->t2, b, y, a); break;
            case 4: vec_out_s<4>(grid, ilu->t2, b, y, a); break;
            case 5: vec_out_s<5>(grid, ilu->t2, b, y, a); break;
            case 6: vec_out_s<6>(grid, ilu->t2, b, y, a); break;
            case 7: vec_out_s<7>(grid, ilu->t2, b, y, a); break;
            default: vec_out_s<8>(grid, ilu->t2, b, y, a); break;
            }
            HIPCHK(hipGetLastError());
        }
    }

    void spmv(const T *x, T *y, const T *b, int act, int k, int q)
    {
        SpmvArgs a{act, k, q, s, ell, pkey};
        if (ilu) {
            // the sliced factors (12 B per off-diagonal entry, U's diagonal, the
            // row pointer and diagonal positions), then either the product and
            // the vectors x, t1 (write, read), t2 (write, read, write), y (and
            // b), or (Eisenstat) dd, du and x, t1 (write, 2 reads), t2 (write,
            // read, write, read), y (and b)
            const double lub = 12.0 * (double)(ilu->nnz - n) + 8.0 * (double)n + 16.0 * (double)n;
            const double bytes = ilu->eis ? lub + 16.0 * n + (b ? 10.0 : 9.0) * n * sizeof(T)
                                          : lub + spmv_bytes(A, false, sizeof(T)) + (b ? 8.0 : 6.0) * n * sizeof(T);
            int slot = prof ? prof->begin(MSTAB_K_SPMV, bytes) : -1;
            ilu_product(x, y, b, a);
            if (prof) prof->end(slot);
            return;
        }
        // the FP64 matrix for true residuals and the initial residual
        const bool low = use_low && act != ACT_TRUE && act != ACT_RESID;
        const bool cst = low ? A_low.dconst : A.dconst;
        const int grid = grid_for(n, SPMV_BLOCK, cst ? SPMV_CONST_MAX_BLOCKS : SPMV_MAX_BLOCKS);
        const double bytes = low ? spmv_bytes(A_low, b != nullptr, sizeof(T))
                                 : spmv_bytes(A, b != nullptr, sizeof(T));
        int slot = prof ? prof->begin(MSTAB_K_SPMV, bytes) : -1;
        if (low)
            launch_spmv<T, float>(grid, stream, A_low, x, y, b, ctl, part, a);
        else
            launch_spmv<T>(grid, stream, A, x, y, b, ctl, part, a);
        HIPCHK(hipGetLastError());
        if (prof) prof->end(slot);
    }

    void gamma(int k)
    {
        const int grid = grid_for(ld / Vec16<T>::W, BLOCK, VEC_MAX_BLOCKS);
        int slot = prof ? prof->begin(MSTAB_K_GAMMA, vbytes((k + 1) * (s + 2) + s + 2)) : -1;
        switch (s) {
#define CASE(S)                                                                              \
    case S:                                                                                  \
        hipLaunchKernelGGL((k_gamma<T, S>), dim3(grid), dim3(BLOCK), 0, stream, ld, W, R, X, \
                           k, ctl);                                                          \
        break;
            CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        }
        HIPCHK(hipGetLastError());
        if (prof) prof->end(slot);
    }

    void eta(int k, int q)
    {
        const int grid = grid_for(ld / Vec16<T>::W, BLOCK, VEC_MAX_BLOCKS);
        // r^(k+1) and s vectors read, v_q^(k) written
        int slot = prof ? prof->begin(MSTAB_K_ETA, vbytes(s + 2)) : -1;
        switch (s) {
#define CASE(S)                                                                               \
    case S:                                                                                   \
        hipLaunchKernelGGL((k_eta<T, S>), dim3(grid), dim3(BLOCK), 0, stream, ld, W, R, k, q, \
                           ctl);                                                              \
        break;
            CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        }
        HIPCHK(hipGetLastError());
        if (prof) prof->end(slot);
    }

    // levels -1..k-1 of all s steps of level k (after its last step)
    void eta_low(int k)
    {
        const int grid = grid_for(ld / Vec16<T>::W, BLOCK, VEC_MAX_BLOCKS);
        // level k (s), then per lower level r^(i+1) and s vectors read, s written
        int slot = prof ? prof->begin(MSTAB_K_ETA, vbytes(s + (k + 1) * (2 * s + 1))) : -1;
        switch (s) {
#define CASE(S)                                                                                \
    case S:                                                                                    \
        hipLaunchKernelGGL((k_eta_low<T, S>), dim3(grid), dim3(BLOCK), 0, stream, ld, W, R, k, \
                           ctl);                                                               \
        break;
            CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        }
        HIPCHK(hipGetLastError());
        if (prof) prof->end(slot);
    }

    // k_eta_low(k) fused with gamma(k + 1) (k + 1 < l)
    void eta_low_gamma(int k)
    {
        const int grid = grid_for(ld / Vec16<T>::W, BLOCK, VEC_MAX_BLOCKS);
        int slot = prof ? prof->begin(MSTAB_K_ETA, vbytes(2 * s + 4 + 2 * (k + 1) * (s + 1))) : -1;
        switch (s) {
#define CASE(S)                                                                                   \
    case S:                                                                                       \
        hipLaunchKernelGGL((k_eta_low_gamma<T, S>), dim3(grid), dim3(BLOCK), 0, stream, ld, W, R, \
                           X, k, ctl);                                                            \
        break;
            CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        }
        HIPCHK(hipGetLastError());
        if (prof) prof->end(slot);
    }

    template <int S>
    void eta_low_gram_s(int grid)
    {
        switch (ell) {
#define CASE(L)                                                                                  \
    case L:                                                                                      \
        hipLaunchKernelGGL((k_eta_low_gram<T, S, L>), dim3(grid), dim3(BLOCK), 0, stream, ld, W, \
                           (const T *)R, ctl, part, PART_STRIDE);                                \
        break;
            CASE(1) CASE(2) CASE(3) CASE(4)
#undef CASE
        }
    }

    // k_eta_low(l - 1) fused with the Gram matrix and the tau solve (l <= 4)
    void eta_low_gram()
    {
        const int grid = grid_for(ld / Vec16<T>::W, BLOCK, GRAM_MAX_BLOCKS);
        const int k = ell - 1;
        int slot = prof ? prof->begin(MSTAB_K_GRAM, vbytes(s + 1 + (k + 1) * (s + 1) + s * (k + 1))) : -1;
        switch (s) {
        case 1: eta_low_gram_s<1>(grid); break;
        case 2: eta_low_gram_s<2>(grid); break;
        case 3: eta_low_gram_s<3>(grid); break;
        case 4: eta_low_gram_s<4>(grid); break;
        case 5: eta_low_gram_s<5>(grid); break;
        case 6: eta_low_gram_s<6>(grid); break;
        case 7: eta_low_gram_s<7>(grid); break;
        default: eta_low_gram_s<8>(grid); break;
        }
        HIPCHK(hipGetLastError());
        if (prof) prof->end(slot);
    }

    void gram()
    {
        const int grid = grid_for(ld / Vec16<T>::W, BLOCK, GRAM_MAX_BLOCKS);
        int slot = prof ? prof->begin(MSTAB_K_GRAM, vbytes(ell + 1)) : -1;
        switch (ell) {
#define CASE(L)                                                                                 \
    case L:                                                                                     \
        hipLaunchKernelGGL((k_gram<T, L>), dim3(grid), dim3(BLOCK), 0, stream, ld, R, ctl, part, \
                           PART_STRIDE);                                                        \
        break;
            CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        }
        HIPCHK(hipGetLastError());
        if (prof) prof->end(slot);
    }

    template <int S, int PM>
    void poly_sp(int grid)
    {
        switch (ell) {
#define CASE(L)                                                                                  \
    case L:                                                                                      \
        hipLaunchKernelGGL((k_poly<T, S, L, PM>), dim3(grid), dim3(BLOCK), 0, stream, n, ld, ell, \
                           W, R, X, pkey, ctl, part, PART_STRIDE);                               \
        break;
            CASE(1) CASE(2) CASE(3) CASE(4)
#undef CASE
        default:
            hipLaunchKernelGGL((k_poly<T, S, 0, PM>), dim3(grid), dim3(BLOCK), 0, stream, n, ld, ell,
                               W, R, X, pkey, ctl, part, PART_STRIDE);
        }
    }

    // P's source (generator or the caller's matrix) picks the kernel variant
    template <int S>
    void poly_s(int grid)
    {
        if (pkey.m)
            poly_sp<S, 1>(grid);
        else
            poly_sp<S, 0>(grid);
    }

    void poly()
    {
        const int grid = grid_for(ld, BLOCK, POLY_MAX_BLOCKS);
        int slot = prof ? prof->begin(MSTAB_K_POLY,
                                      vbytes(1 + (ell + 1) + s * (ell + 2) + 2 * s + 2))
                        : -1;
        switch (s) {
        case 1: poly_s<1>(grid); break;
        case 2: poly_s<2>(grid); break;
        case 3: poly_s<3>(grid); break;
        case 4: poly_s<4>(grid); break;
        case 5: poly_s<5>(grid); break;
        case 6: poly_s<6>(grid); break;
        case 7: poly_s<7>(grid); break;
        default: poly_s<8>(grid); break;
        }
        HIPCHK(hipGetLastError());
        if (prof) prof->end(slot);
    }

    // P^T y (and ||y||^2): dst 0 -> ptv[0][q]; dst 1 -> ptt, tt
    // Called after every completed cycle with ||r||^2 when set (the FP32
    // solve of the mixed form replaces its recursive residual there).
    // HOOK_REPLACED: it has enqueued a replacement, which must leave the new
    // residual in Rc(0) and its P^T r, ||r||^2 and gamma in ctl;
    // HOOK_STOP: end the solve (not converged).
    enum { HOOK_NONE = 0, HOOK_REPLACED = 1, HOOK_STOP = 2 };
    std::function<int(double)> after_cycle;
    // After a replacement, with the new ||r||^2: false ends the solve (not
    // converged).
    std::function<bool(double)> after_replace;

    void project(const T *y, int dst, int q)
    {
        const int grid = grid_for(n, BLOCK, GRAM_MAX_BLOCKS);
        hipLaunchKernelGGL((k_project<T>), dim3(grid), dim3(BLOCK), 0, stream, n, y, pkey, s, dst,
                           q, ctl, part, PART_STRIDE);
        HIPCHK(hipGetLastError());
    }

    void small(int what)
    {
        hipLaunchKernelGGL(k_small, dim3(1), dim3(64), 0, stream, ctl, s, what);
        HIPCHK(hipGetLastError());
    }

    void dots(const T *U, int nu, const T *w, int first)
    {
        const int grid = grid_for(ld, BLOCK, GRAM_MAX_BLOCKS);
        hipLaunchKernelGGL((k_dots<T>), dim3(grid), dim3(BLOCK), 0, stream, ld, U, nu, w, first,
                           ctl, part, PART_STRIDE);
        HIPCHK(hipGetLastError());
    }

    void gs(const T *U, int nu, const T *w, T *out)
    {
        const int grid = grid_for(ld, BLOCK, VEC_MAX_BLOCKS);
        hipLaunchKernelGGL((k_gs<T>), dim3(grid), dim3(BLOCK), 0, stream, ld, U, nu, w, out, ctl);
        HIPCHK(hipGetLastError());
    }

    void normalize(const T *src, T *dst, int mode)
    {
        const int grid = grid_for(ld, BLOCK, VEC_MAX_BLOCKS);
        hipLaunchKernelGGL((k_normalize<T>), dim3(grid), dim3(BLOCK), 0, stream, ld, src, dst,
                           mode, ctl);
        HIPCHK(hipGetLastError());
    }

    void fill(T *dst, int64_t count, T v)
    {
        const int grid = grid_for(count, BLOCK, VEC_MAX_BLOCKS);
        hipLaunchKernelGGL((k_fill<T>), dim3(grid), dim3(BLOCK), 0, stream, count, dst, v);
        HIPCHK(hipGetLastError());
    }

    void sync_status()
    {
        HIPCHK(hipMemcpyAsync(st_host, &ctl->st, sizeof(Status), hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        if (prof) prof->harvest();
    }

    void set_thr2(double thr2)
    {
        hipLaunchKernelGGL(k_set_thr2, dim3(1), dim3(64), 0, stream, ctl, thr2);
        HIPCHK(hipGetLastError());
    }

    // Arnoldi basis of level s of r = R[0] (norm^2 in st.rr): U orthonormal, V = A U.
    void arnoldi()
    {
        normalize(Rc(0), Wc(-1, 0), 1);
        for (int q = 0; q < s; ++q) {
            spmv(Wc(-1, q), Wc(0, q), nullptr, ACT_ARN, 0, q);
            if (q + 1 < s) {
                T *w = Wc(-1, q + 1);
                dots(Wc(-1, 0), q + 1, Wc(0, q), 1);
                gs(Wc(-1, 0), q + 1, Wc(0, q), w);
                dots(Wc(-1, 0), q + 1, w, 0);
                gs(Wc(-1, 0), q + 1, w, w);
                dots(Wc(-1, 0), 0, w, 0);
                normalize(w, w, 0);
            }
        }
        small(SMALL_GAMMA0);
    }

    // One cycle of Algorithm 1: the level loop (gamma, the r product, the s
    // eta steps and v products), then the degree-l minimization and update.
    // Kernels that follow each other without a reduction between them are
    // fused: the lower levels' eta steps of level k with the gamma step of
    // level k + 1, and those of the last level with the Gram matrix and tau.
    void cycle()
    {
        // the fused Gram kernel holds all l + 1 residual levels and both V
        // levels of its pass in registers: used while that stays small
        const bool fuse_gram = ell <= 4 && s * ell * Vec16<T>::W <= 16;
        gamma(0);
        for (int k = 0; k < ell; ++k) {
            spmv(Rc(k), Rc(k + 1), nullptr, ACT_R, k, 0);
            for (int q = 0; q < s; ++q) {
                eta(k, q);
                spmv(Wc(k, q), Wc(k + 1, q), nullptr, ACT_V, k, q);
            }
            if (k + 1 < ell) {
                eta_low_gamma(k);
            } else if (fuse_gram) {
                eta_low_gram();
            } else {
                eta_low(k);
                gram();
            }
        }
        poly();
    }

    void copy_vecs(T *dst, const T *src, int count)
    {
        HIPCHK(hipMemcpyAsync(dst, src, (size_t)ld * sizeof(T) * count, hipMemcpyDeviceToDevice,
                              stream));
    }

    // Write out U, V at a cycle end.  With refresh_v (FP32 data), V := A U is
    // recomputed from the fetched U (s counted products), restoring Algorithm
    // 1's prior requirement V = A U, which FP32 rounding erodes over the
    // hundreds of cycles that chained recycle data live through.
    bool refresh_v = false;
    // Orthonormalize the fetched data (CholQR in FP64: U := U R^-1,
    // V := V R^-1 with U^T U = R^T R), and recompute their P^T V.
    bool orthonormalize = false;

    template <int S>
    void cholqr_s(T *V)
    {
        const int g = grid_for(ld, BLOCK, GRAM_MAX_BLOCKS);
        hipLaunchKernelGGL((k_chol_gram<T, S>), dim3(g), dim3(BLOCK), 0, stream, ld,
                           (const T *)recU, ctl, part, PART_STRIDE);
        HIPCHK(hipGetLastError());
        const int ga = grid_for(ld, BLOCK, VEC_MAX_BLOCKS);
        hipLaunchKernelGGL((k_chol_apply<T, S>), dim3(ga), dim3(BLOCK), 0, stream, ld, recU, V,
                           (const Ctl *)ctl);
        HIPCHK(hipGetLastError());
    }

    // recU (and V unless NULL) := B R^-1; unchanged if U^T U is not
    // numerically positive definite
    void cholqr(T *V)
    {
        switch (s) {
        case 1: cholqr_s<1>(V); break;
        case 2: cholqr_s<2>(V); break;
        case 3: cholqr_s<3>(V); break;
        case 4: cholqr_s<4>(V); break;
        case 5: cholqr_s<5>(V); break;
        case 6: cholqr_s<6>(V); break;
        case 7: cholqr_s<7>(V); break;
        default: cholqr_s<8>(V); break;
        }
    }

    void fetch(int64_t level)
    {
        copy_vecs(recU, Wc(-1, 0), s);
        if (refresh_v) {
            if (orthonormalize) cholqr(nullptr);
            for (int q = 0; q < s; ++q)
                spmv(recU + (int64_t)q * ld, recV + (int64_t)q * ld, nullptr, ACT_RECV, 0, q);
            HIPCHK(hipMemcpyAsync(rec_ptv, &ctl->prec[0][0], sizeof(double) * MAXS * MAXS,
                                  hipMemcpyDeviceToDevice, stream));
        } else if (orthonormalize) {
            copy_vecs(recV, Wc(0, 0), s);
            cholqr(recV);
            for (int q = 0; q < s; ++q) project(recV + (int64_t)q * ld, 2, q);
            HIPCHK(hipMemcpyAsync(rec_ptv, &ctl->prec[0][0], sizeof(double) * MAXS * MAXS,
                                  hipMemcpyDeviceToDevice, stream));
        } else {
            copy_vecs(recV, Wc(0, 0), s);
            HIPCHK(hipMemcpyAsync(rec_ptv, &ctl->ptv[0][0][0], sizeof(double) * MAXS * MAXS,
                                  hipMemcpyDeviceToDevice, stream));
        }
        rec_level = level;
        rec_have = true;
    }

    // Restarted GMRES(m) for A X = b from the current X (Section 5.1's
    // comparison method; the kernels are in gmres.hpp).  Every product counts
    // in res.mv (the true residual that starts each cycle and ends the solve
    // included); res.cycles counts Arnoldi steps, res.restarts the cycles
    // after the first; the history holds the initial residual and every
    // step's estimate.  A zero b gives x = 0 with no product.
    SolveResult gmres(const T *b, double tol, int64_t max_mv)
    {
        SolveResult res;
        hist_mv.clear();
        hist_res.clear();
        const int m = gm_m;
        const GmLayout L{m};
        T *w = gmV + (int64_t)(m + 1) * ld;
        auto V = [&](int j) { return gmV + (int64_t)j * ld; };
        const int gv = grid_for(ld, BLOCK, VEC_MAX_BLOCKS);
        const int gd = grid_for(ld, BLOCK, GRAM_MAX_BLOCKS);
        int64_t mv = 0, cycles = 0;
        double nb = 0.0, thr = 0.0, est = -1.0;
        double scal[GM_SCAL];
        // w += sign V[:, j0:j0+nv] coef[j0:j0+nv] (and ||w||^2 with norm)
        auto axpy = [&](int j0, int nv, const double *coef, double sign, T *y, int norm) {
            if (nv <= 8)
                hipLaunchKernelGGL((k_gm_axpy<T, 8>), dim3(norm ? gd : gv), dim3(BLOCK), 0, stream, ld,
                                   (const T *)gmV, j0, nv, coef, sign, y, ctl, norm, part, PART_STRIDE);
            else
                hipLaunchKernelGGL((k_gm_axpy<T, GM_CHUNK>), dim3(norm ? gd : gv), dim3(BLOCK), 0, stream, ld,
                                   (const T *)gmV, j0, nv, coef, sign, y, ctl, norm, part, PART_STRIDE);
            HIPCHK(hipGetLastError());
        };
        small(SMALL_CLEAR);
        for (;;) {
            // the true residual into v_1
            spmv(X, V(0), b, ACT_TRUE, 0, 0);
            ++mv;
            sync_status();
            if (st_host->flags & FLAG_NONFINITE) { res.status = MSTAB_E_NONFINITE; break; }
            if (cycles == 0) {
                nb = std::sqrt(st_host->bb);
                if (!std::isfinite(nb)) { res.status = MSTAB_E_NONFINITE; break; }
                if (nb == 0.0) {
                    fill(X, ld, (T)0);
                    HIPCHK(hipStreamSynchronize(stream));
                    mv = 0;
                    res.converged = true;
                    res.relres_true = 0.0;
                    est = 0.0;
                    break;
                }
                thr = tol * nb;
            }
            const double beta = std::sqrt(st_host->tt);
            if (!std::isfinite(beta)) { res.status = MSTAB_E_NONFINITE; break; }
            if (cycles == 0) {
                hist_mv.push_back(mv);
                hist_res.push_back(beta / nb);
            }
            res.relres_true = beta / nb;
            if (beta <= thr) { res.converged = true; break; }
            if (mv >= max_mv) break;
            hipLaunchKernelGGL((k_gm_start<T>), dim3(gv), dim3(BLOCK), 0, stream, ld, V(0), gm_state, m,
                               (const Ctl *)ctl);
            HIPCHK(hipGetLastError());
            int k = 0;
            for (int j = 0; j < m; ++j) {
                spmv(V(j), w, nullptr, ACT_NONE, 0, 0);
                ++mv;
                ++res.cycles;
                for (int pass = 0; pass < 2; ++pass) {
                    double *c = gm_state + L.c(pass);
                    for (int j0 = 0; j0 <= j; j0 += GM_CHUNK) {
                        const int nv = std::min(GM_CHUNK, j + 1 - j0);
                        if (nv <= 8)
                            hipLaunchKernelGGL((k_gm_dots<T, 8>), dim3(gd), dim3(BLOCK), 0, stream, ld,
                                               (const T *)gmV, j0, nv, (const T *)w, c, ctl, part, PART_STRIDE);
                        else
                            hipLaunchKernelGGL((k_gm_dots<T, GM_CHUNK>), dim3(gd), dim3(BLOCK), 0, stream, ld,
                                               (const T *)gmV, j0, nv, (const T *)w, c, ctl, part, PART_STRIDE);
                        HIPCHK(hipGetLastError());
                    }
                    for (int j0 = 0; j0 <= j; j0 += GM_CHUNK) {
                        const int nv = std::min(GM_CHUNK, j + 1 - j0);
                        // the last update of the second pass also gives ||w||^2
                        const int norm = pass == 1 && j0 + GM_CHUNK > j;
                        axpy(j0, nv, c, -1.0, w, norm);
                    }
                }
                hipLaunchKernelGGL(k_gm_column, dim3(1), dim3(64), 0, stream, gm_state, m, j, (const Ctl *)ctl);
                HIPCHK(hipGetLastError());
                HIPCHK(hipMemcpyAsync(scal, gm_state + L.scal(), sizeof scal, hipMemcpyDeviceToHost, stream));
                sync_status();
                if (st_host->flags & FLAG_NONFINITE) { res.status = MSTAB_E_NONFINITE; goto out; }
                if (scal[GM_SINGULAR] != 0.0) break;   // keep columns 0..j-1
                k = j + 1;
                est = scal[GM_EST];
                hist_mv.push_back(mv);
                hist_res.push_back(est / nb);
                if (est <= thr || !(scal[GM_HN] > 0.0) || mv >= max_mv) break;
                hipLaunchKernelGGL((k_gm_scale<T>), dim3(gv), dim3(BLOCK), 0, stream, ld, (const T *)w, V(j + 1),
                                   (const double *)gm_state, m);
                HIPCHK(hipGetLastError());
            }
            if (k == 0) { res.status = MSTAB_E_BREAKDOWN; break; }
            hipLaunchKernelGGL(k_gm_solve, dim3(1), dim3(64), 0, stream, gm_state, m, k);
            HIPCHK(hipGetLastError());
            for (int j0 = 0; j0 < k; j0 += GM_CHUNK)
                axpy(j0, std::min(GM_CHUNK, k - j0), gm_state + L.y(), 1.0, X, 0);
            ++cycles;
        }
        if (res.status == MSTAB_OK && !res.converged) res.status = MSTAB_NOT_CONVERGED;
    out:
        res.mv = mv;
        res.restarts = cycles > 0 ? (int)(cycles - 1) : 0;
        res.relres_rec = est < 0 ? -1.0 : est / (nb > 0 ? nb : 1.0);
        return res;
    }

    // Solve A X = b from the current X (b: n entries of T on the device).
    // check_true = false: stop on the recursive residual (inner solves of the
    // mixed mode, whose FP64 outer residual decides).
    SolveResult solve(const T *b, double tol, int64_t max_mv, int method, int fetch_policy,
                      double fetch_rel, int64_t fetch_level, int max_repl, bool check_true = true)
    {
        SolveResult res;
        hist_mv.clear();
        hist_res.clear();
        const double tol2 = tol * tol;
        int64_t mv0 = 0;

        small(SMALL_CLEAR);
        HIPCHK(hipMemsetAsync(&ctl->st.mv, 0, sizeof(int64_t), stream));
        set_thr2(0.0);
        spmv(X, Rc(0), b, ACT_RESID, 0, 0);
        sync_status();
        const double bb = st_host->bb;
        if (st_host->flags & FLAG_NONFINITE || !std::isfinite(bb)) {
            res.status = MSTAB_E_NONFINITE;
            return res;
        }
        if (bb == 0.0) {
            fill(X, ld, (T)0);
            HIPCHK(hipStreamSynchronize(stream));
            res.converged = true;
            res.relres_rec = 0.0;
            res.relres_true = 0.0;
            res.mv = 0;
            return res;
        }
        const double thr2 = tol2 * bb;
        set_thr2(thr2);
        double rr = st_host->rr;
        double rr_true_mark = rr;   // ||r||^2 at the last true residual
        int64_t since_true = 0;     // cycles since r was last the true residual
        int periodic_repl = 0;
        int64_t mv = st_host->mv;
        bool r_is_true = true;
        hist_mv.push_back(mv);
        hist_res.push_back(std::sqrt(rr / bb));

        bool have_uv = false;
        int64_t level = 0;
        if (method == MSTAB_METHOD_MSTAB && rec_have) {
            copy_vecs(Wc(-1, 0), recU, s);
            copy_vecs(Wc(0, 0), recV, s);
            HIPCHK(hipMemcpyAsync(&ctl->ptv[0][0][0], rec_ptv, sizeof(double) * MAXS * MAXS,
                                  hipMemcpyDeviceToDevice, stream));
            level = rec_level;
            have_uv = true;
            res.recycled = true;
            small(SMALL_GAMMA0);
        }
        const bool had_rec = rec_have;
        const int64_t est_in = est_cycle;
        int64_t fetched = -1;

        for (;;) {
            while (rr > thr2 && mv < max_mv) {
                if (!have_uv) {
                    arnoldi();
                    have_uv = true;
                    level = 0;
                    // the products are counted on the device; read them before deciding
                    sync_status();
                    mv = st_host->mv;
                    if (st_host->flags & FLAG_NONFINITE) { res.status = MSTAB_E_NONFINITE; goto out; }
                    if (st_host->flags & FLAG_BREAKDOWN && st_host->where == WHERE_ARNOLDI) {
                        res.status = MSTAB_E_BREAKDOWN;
                        goto out;
                    }
                    continue;
                }
                cycle();
                sync_status();
                mv = st_host->mv;
                if (st_host->flags & FLAG_NONFINITE) { res.status = MSTAB_E_NONFINITE; goto out; }
                if (st_host->flags & FLAG_BREAKDOWN) {
                    if (res.restarts < 2) {
                        ++res.restarts;
                        have_uv = false;
                        small(SMALL_CLEAR);
                        set_thr2(0.0);   // no gamma solve until the basis is rebuilt
                        spmv(X, Rc(0), b, ACT_RESID, 0, 0);
                        set_thr2(thr2);
                        sync_status();
                        mv = st_host->mv;
                        rr = st_host->rr;
                        rr_true_mark = rr;
                        r_is_true = true;
                        since_true = 0;
                        if (st_host->flags & FLAG_NONFINITE || !std::isfinite(rr)) {
                            res.status = MSTAB_E_NONFINITE;
                            goto out;
                        }
                        continue;
                    }
                    res.status = MSTAB_E_BREAKDOWN;
                    goto out;
                }
                ++res.cycles;
                level += ell;
                r_is_true = false;
                const int hook = after_cycle ? after_cycle(st_host->rr) : HOOK_NONE;
                if (hook == HOOK_STOP) {
                    res.status = MSTAB_NOT_CONVERGED;
                    rr = st_host->rr;
                    goto out;
                }
                if (hook == HOOK_REPLACED) {
                    sync_status();
                    mv = st_host->mv;
                    if (st_host->flags & FLAG_NONFINITE) { res.status = MSTAB_E_NONFINITE; goto out; }
                    if (st_host->flags & FLAG_BREAKDOWN) { res.status = MSTAB_E_BREAKDOWN; goto out; }
                    if (after_replace && !after_replace(st_host->rr)) {
                        res.status = MSTAB_NOT_CONVERGED;
                        rr = st_host->rr;
                        goto out;
                    }
                }
                rr = st_host->rr;
                ++since_true;
                const bool periodic = replace_every > 0 && since_true >= replace_every;
                const bool low_gap = use_low && rr <= low_drop * low_drop * rr_true_mark;
                if ((periodic || low_gap) && rr > thr2 && mv < max_mv) {
                    if (periodic) ++periodic_repl;
                    since_true = 0;
                    spmv(X, Tv, b, ACT_TRUE, 0, 0);
                    copy_vecs(Rc(0), Tv, 1);
                    small(SMALL_REPLACE);
                    sync_status();
                    ++res.mv_check;
                    ++res.replacements;
                    if (st_host->flags & FLAG_NONFINITE) { res.status = MSTAB_E_NONFINITE; goto out; }
                    if (st_host->flags & FLAG_BREAKDOWN) { res.status = MSTAB_E_BREAKDOWN; goto out; }
                    rr = st_host->rr;
                    rr_true_mark = rr;
                    r_is_true = true;
                }
                hist_mv.push_back(mv + res.mv_check);
                hist_res.push_back(std::sqrt(rr / bb));
                const double rel = std::sqrt(rr / bb);
                bool fire = false;
                switch (fetch_policy) {
                case MSTAB_FETCH_THRESHOLD: fire = (fetched < 0 && rel <= fetch_rel); break;
                case MSTAB_FETCH_AT_LEVEL: fire = (level == fetch_level); break;
                case MSTAB_FETCH_ONCE: fire = (!had_rec && fetched < 0 && rel <= fetch_rel); break;
                case MSTAB_FETCH_ESTIMATE: fire = (est_in > 0 && fetched < 0 && res.cycles == est_in); break;
                default: break;
                }
                if (fire) {
                    fetch(level);
                    fetched = level;
                }
            }
            // finish: the true residual decides
            if (r_is_true || !check_true) {
                res.relres_true = std::sqrt(rr / bb);
                res.converged = rr <= thr2;
                break;
            }
            spmv(X, Tv, b, ACT_TRUE, 0, 0);
            sync_status();
            ++res.mv_check;
            {
                const double tt = st_host->tt;
                res.relres_true = std::sqrt(tt / bb);
                if (!std::isfinite(tt)) { res.status = MSTAB_E_NONFINITE; goto out; }
                if (tt <= thr2) { res.converged = true; break; }
                if (rr <= thr2 && res.replacements - periodic_repl < max_repl && mv < max_mv) {
                    copy_vecs(Rc(0), Tv, 1);
                    small(SMALL_REPLACE);
                    rr = tt;
                    r_is_true = true;
                    since_true = 0;
                    ++res.replacements;
                    continue;
                }
            }
            break;
        }
        if (!res.converged) res.status = MSTAB_NOT_CONVERGED;
        if (res.cycles > 0 && fetched < 0 &&
            (fetch_policy == MSTAB_FETCH_AT_END || fetch_policy == MSTAB_FETCH_THRESHOLD ||
             (fetch_policy == MSTAB_FETCH_ONCE && !had_rec) ||
             (fetch_policy == MSTAB_FETCH_ESTIMATE && est_in > 0))) {
            fetch(level);
            fetched = level;
        }
        if (fetch_policy == MSTAB_FETCH_ESTIMATE) est_cycle = estimate_fetch_cycle(hist_res);
    out:
        sync_status();
        mv = st_host->mv;   // includes products of a fetch refresh after the last cycle
        res.mv = mv - mv0;
        res.level = level;
        res.fetched = fetched;
        res.relres_rec = std::sqrt(rr / bb);
        return res;
    }
};

}  // namespace

// ---------------------------------------------------------------------------
// The handle.
// ---------------------------------------------------------------------------
struct mstab_solver {
    mstab_options opt{};
    int s = 0, ell = 0;
    int64_t n = 0, nnz = 0;
    const int32_t *rp = nullptr, *ci = nullptr;
    const double *va = nullptr;
    hipStream_t stream = nullptr;
    int device = 0;         // the HIP device current at create
    uint32_t pkey = 0;
    // with the p_host option: the caller's cut-space basis (n x s, device copy)
    // and a 64-bit FNV-1a digest of its bytes (recycle blobs carry it)
    double *pmat = nullptr;
    uint64_t p_digest = 0;
    PBasis pbasis() const { return PBasis(pkey, pmat, n); }
    Engine<double> e64;
    Engine<float> e32;
    float *r32 = nullptr;   // F32_REFINE: scaled residual (right-hand side of the inner solve)
    double *xbak = nullptr; // F32_REFINE: x before the last fold of the FP32 iterate
    // PRECOND_JACOBI: d = |diag A|^-1/2, e = |diag A|^1/2, and L^-1 b
    double *pd = nullptr, *pe = nullptr, *bhat = nullptr;
    double *split_tmp = nullptr;  // create only: the split values while the copies are built
    // REORDER_RCM: perm[new] = old, the reordered CSR (its row pointer stays in
    // use by the sliced product), and the reordered iterate
    int32_t *perm = nullptr, *rp_perm = nullptr, *ci_perm = nullptr;
    double *va_perm = nullptr, *xwork = nullptr;
    // PRECOND_ILU0: the factors of the multicolour-ordered matrix (perm is that
    // order; rp_perm and ci_perm its structure)
    IluData ilu;
    // ENGINE_WORKGROUP: the job array and histories of the launches this
    // handle leads (as h[0] of a batch, or alone), grown on demand
    wg::Job *wg_jobs = nullptr;
    int64_t *wg_hmv = nullptr;
    double *wg_hres = nullptr;
    int wg_cap = 0;
    bool workgroup() const { return opt.engine == MSTAB_ENGINE_WORKGROUP; }
    bool transformed() const { return pd || perm; }
    Profiler prof;
    int64_t mv_total = 0, mv_last = 0;
    std::vector<int64_t> hist_mv;
    std::vector<double> hist_res;
    // the histories of every solve on the handle, in order
    std::vector<std::vector<int64_t>> hist_mv_all;
    std::vector<std::vector<double>> hist_res_all;
    std::string err;
    bool mixed() const { return opt.precision == MSTAB_PREC_F32_REFINE; }
};

namespace {

mstab_status record(mstab_solver *h, const StatusError &e)
{
    if (h) h->err = e.msg;
    g_tls_error = e.msg;
    return e.st;
}

mstab_status record_hip(mstab_solver *h, const HipError &e)
{
    char buf[512];
    snprintf(buf, sizeof buf, "HIP error %d (%s) in %s", (int)e.e, hipGetErrorString(e.e), e.what);
    if (h) h->err = buf;
    g_tls_error = buf;
    return MSTAB_E_HIP;
}

void release_handle(mstab_solver *h)
{
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    h->e64.release();
    h->e32.release();
    (void)hipFree(h->r32);
    (void)hipFree(h->xbak);
    (void)hipFree(h->pd);
    (void)hipFree(h->pe);
    (void)hipFree(h->bhat);
    (void)hipFree(h->split_tmp);
    (void)hipFree(h->perm);
    (void)hipFree(h->rp_perm);
    (void)hipFree(h->ci_perm);
    (void)hipFree(h->va_perm);
    (void)hipFree(h->xwork);
    h->ilu.release();
    (void)hipFree(h->pmat);
    (void)hipFree(h->wg_jobs);
    (void)hipFree(h->wg_hmv);
    (void)hipFree(h->wg_hres);
    h->prof.destroy();
    delete h;
}

#define API_BEGIN try {
#define API_END(h)                                                        \
    }                                                                     \
    catch (const StatusError &e) { return record((h), e); }               \
    catch (const HipError &e) { return record_hip((h), e); }              \
    catch (const std::bad_alloc &) {                                      \
        return record((h), StatusError{MSTAB_E_NOMEM, "host allocation failed"}); \
    }

void fill_info(mstab_info *info, const SolveResult &r, double secs)
{
    if (!info) return;
    memset(info, 0, sizeof *info);
    info->status = r.status;
    info->converged = r.converged;
    info->recycled = r.recycled;
    info->restarts = r.restarts;
    info->replacements = r.replacements;
    info->mv = r.mv;
    info->mv_check = r.mv_check;
    info->cycles = r.cycles;
    info->level = r.level;
    info->fetched_level = r.fetched;
    info->relres_recursive = r.relres_rec;
    info->relres_true = r.relres_true;
    info->seconds = secs;
}

int grid1(int64_t n) { return grid_for(n, BLOCK, VEC_MAX_BLOCKS); }

// true-residual replacements allowed with the FP32 matrix copy (each one a
// defect-correction step; two or three suffice in practice)
constexpr int LOW_MATRIX_REPLACEMENTS = 10;

// Files the history of the solve that ends with this guard's scope.
struct HistoryArchive {
    mstab_solver *h;
    ~HistoryArchive()
    {
        try {
            h->hist_mv_all.push_back(h->hist_mv);
            h->hist_res_all.push_back(h->hist_res);
        } catch (...) {
        }
    }
};

mstab_status wg_run(mstab_solver *const *h, int count, const double *const *b, double *const *x,
                    mstab_info *info, int extra_checks, int accepted);

mstab_status solve_f64(mstab_solver *h, const double *b, double *x, mstab_info *info,
                       int extra_checks, int accepted)
{
    if (h->workgroup()) return wg_run(&h, 1, &b, &x, info, extra_checks, accepted);
    HistoryArchive archive{h};
    h->hist_mv.clear();
    h->hist_res.clear();
    auto t0 = std::chrono::steady_clock::now();
    Engine<double> &E = h->e64;
    HIPCHK(hipMemcpyAsync(E.X, x, sizeof(double) * h->n, hipMemcpyDeviceToDevice, h->stream));
    // with the FP32 matrix copy the iteration solves a system O(eps32) away from
    // A: its recursive residual meets tol before the true one does, and each
    // true-residual replacement is a step of defect correction
    const bool low = h->opt.precision == MSTAB_PREC_F32_MATRIX;
    const int max_repl = low ? std::max(h->opt.max_replacements, LOW_MATRIX_REPLACEMENTS)
                             : h->opt.max_replacements;
    SolveResult r = h->opt.method == MSTAB_METHOD_GMRES
                        ? E.gmres(b, h->opt.tol, h->opt.max_mv)
                        : E.solve(b, h->opt.tol, h->opt.max_mv, h->opt.method, h->opt.fetch,
                                  h->opt.fetch_rel, h->opt.fetch_level, max_repl);
    HIPCHK(hipMemcpyAsync(x, E.X, sizeof(double) * h->n, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    r.mv_check += extra_checks;
    h->mv_last = r.mv + r.mv_check;
    h->mv_total += h->mv_last;
    h->hist_mv = E.hist_mv;
    h->hist_res = E.hist_res;
    double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    fill_info(info, r, secs);
    if (info) {
        info->guess_accepted = accepted;
        // products with the FP64 matrix: the initial residual (and one per
        // restart) and the true-residual checks
        if (low) info->mv_f64 = 1 + r.restarts + r.mv_check;
    }
    return (mstab_status)r.status;
}

// ENGINE_WORKGROUP: the next system of each handle, one workgroup each.
// Handles are grouped by s and a bound on l (template parameters of the
// kernel) into one launch per group on h[0]'s stream; every handle's stream is drained first,
// and the launch is synchronized before the results are filed.
int wg_lc(int ell) { return ell <= 2 ? 2 : (ell <= 4 ? 4 : 8); }

mstab_status wg_run(mstab_solver *const *h, int count, const double *const *b, double *const *x,
                    mstab_info *info, int extra_checks, int accepted)
{
    mstab_solver *h0 = h[0];
    auto t0 = std::chrono::steady_clock::now();
    for (int i = 0; i < count; ++i) {
        if (!h[i]->workgroup()) fail(MSTAB_E_INVALID, "handle %d is not of ENGINE_WORKGROUP", i);
        if (h[i]->device != h0->device) fail(MSTAB_E_INVALID, "handle %d is on another device", i);
    }
    std::vector<hipStream_t> streams;
    for (int i = 0; i < count; ++i)
        if (std::find(streams.begin(), streams.end(), h[i]->stream) == streams.end())
            streams.push_back(h[i]->stream);
    for (hipStream_t st : streams) HIPCHK(hipStreamSynchronize(st));
    if (h0->wg_cap < count) {
        (void)hipFree(h0->wg_jobs);
        (void)hipFree(h0->wg_hmv);
        (void)hipFree(h0->wg_hres);
        h0->wg_jobs = nullptr;
        h0->wg_hmv = nullptr;
        h0->wg_hres = nullptr;
        h0->wg_cap = 0;
        HIPCHK(hipMalloc(&h0->wg_jobs, sizeof(wg::Job) * (size_t)count));
        HIPCHK(hipMalloc(&h0->wg_hmv, sizeof(int64_t) * wg::HIST * (size_t)count));
        HIPCHK(hipMalloc(&h0->wg_hres, sizeof(double) * wg::HIST * (size_t)count));
        h0->wg_cap = count;
    }
    // job p is handle order[p]: grouped by s and the bound on l
    std::vector<int> order((size_t)count);
    for (int i = 0; i < count; ++i) order[(size_t)i] = i;
    // one launch per kernel variant: s, the bound on l, and the source of P
    auto key = [&](int i) { return (h[i]->s * 16 + wg_lc(h[i]->ell)) * 2 + (h[i]->pmat ? 1 : 0); };
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return key(a) < key(c); });
    std::vector<wg::Job> jobs((size_t)count);
    for (int p = 0; p < count; ++p) {
        const int i = order[(size_t)p];
        mstab_solver *hi = h[i];
        Engine<double> &E = hi->e64;
        wg::Job &J = jobs[(size_t)p];
        J.A = E.A;
        J.b = b[i]; J.x = x[i];
        J.W = E.W; J.R = E.R; J.T = E.Tv;
        J.recU = E.recU; J.recV = E.recV; J.rec_ptv = E.rec_ptv;
        // entry k of job p at k * count + p: the first entries of all jobs lie together
        J.hist_mv = h0->wg_hmv + p;
        J.hist_res = h0->wg_hres + p;
        J.hist_stride = count;
        J.n = hi->n; J.ld = E.ld;
        J.max_mv = hi->opt.max_mv; J.fetch_level = hi->opt.fetch_level;
        J.tol = hi->opt.tol; J.fetch_rel = hi->opt.fetch_rel;
        J.pkey = hi->pbasis();
        J.s = hi->s; J.ell = hi->ell; J.method = hi->opt.method; J.fetch = hi->opt.fetch;
        J.max_repl = hi->opt.max_replacements; J.replace_every = hi->opt.replace_every;
        J.rec_have = E.rec_have ? 1 : 0; J.rec_level = E.rec_level; J.est_cycle = E.est_cycle;
    }
    hipStream_t st = h0->stream;
    HIPCHK(hipMemcpyAsync(h0->wg_jobs, jobs.data(), sizeof(wg::Job) * (size_t)count, hipMemcpyHostToDevice, st));
    for (int p0 = 0; p0 < count;) {
        const int kv = key(order[(size_t)p0]);
        const int sv = h[order[(size_t)p0]]->s, lc = wg_lc(h[order[(size_t)p0]]->ell);
        int p1 = p0;
        while (p1 < count && key(order[(size_t)p1]) == kv) ++p1;
        wg::Job *jp = h0->wg_jobs + p0;
        wg::launch(sv, lc, h[order[(size_t)p0]]->pmat != nullptr, p1 - p0, jp, st);
        HIPCHK(hipGetLastError());
        p0 = p1;
    }
    HIPCHK(hipMemcpyAsync(jobs.data(), h0->wg_jobs, sizeof(wg::Job) * (size_t)count, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    // the histories: only the entries some job filled (one contiguous block)
    int64_t width = 1;
    for (int p = 0; p < count; ++p) width = std::max(width, std::min<int64_t>(jobs[(size_t)p].hist_len, wg::HIST));
    std::vector<int64_t> hmv((size_t)(width * count));
    std::vector<double> hres((size_t)(width * count));
    HIPCHK(hipMemcpyAsync(hmv.data(), h0->wg_hmv, sizeof(int64_t) * (size_t)(width * count), hipMemcpyDeviceToHost,
                          st));
    HIPCHK(hipMemcpyAsync(hres.data(), h0->wg_hres, sizeof(double) * (size_t)(width * count), hipMemcpyDeviceToHost,
                          st));
    HIPCHK(hipStreamSynchronize(st));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    mstab_status worst = MSTAB_OK;
    for (int p = 0; p < count; ++p) {
        const int i = order[(size_t)p];
        mstab_solver *hi = h[i];
        const wg::Job &J = jobs[(size_t)p];
        Engine<double> &E = hi->e64;
        E.rec_have = J.rec_have != 0;
        E.rec_level = J.rec_level;
        E.est_cycle = J.est_cycle;
        const int64_t kept = std::min<int64_t>(J.hist_len, wg::HIST);
        hi->hist_mv.resize((size_t)kept);
        hi->hist_res.resize((size_t)kept);
        for (int64_t k = 0; k < kept; ++k) {
            hi->hist_mv[(size_t)k] = hmv[(size_t)(k * count + p)];
            hi->hist_res[(size_t)k] = hres[(size_t)(k * count + p)];
        }
        hi->hist_mv_all.push_back(hi->hist_mv);
        hi->hist_res_all.push_back(hi->hist_res);
        SolveResult r;
        r.status = J.status;
        r.converged = J.converged != 0;
        r.recycled = J.recycled != 0;
        r.restarts = J.restarts;
        r.replacements = J.replacements;
        r.mv = J.mv;
        r.mv_check = J.mv_check + extra_checks;
        r.cycles = J.cycles;
        r.level = J.level;
        r.fetched = J.fetched;
        r.relres_rec = J.relres_rec;
        r.relres_true = J.relres_true;
        hi->mv_last = r.mv + r.mv_check;
        hi->mv_total += hi->mv_last;
        if (info) {
            fill_info(&info[i], r, secs);
            info[i].guess_accepted = accepted;
        }
        const mstab_status sti = (mstab_status)r.status;
        if (sti < 0) {
            hi->err = "solve failed with status " + std::to_string((int)sti);
            if (worst >= 0) worst = sti;
        } else if (sti == MSTAB_NOT_CONVERGED && worst == MSTAB_OK) {
            worst = MSTAB_NOT_CONVERGED;
        }
    }
    return worst;
}

// The F32_REFINE mode.
// Factor by which the FP32 residual must fall between two replacements
// (1: after every cycle, the paper's practice)
#ifndef MSTAB_REPLACE_DROP
#define MSTAB_REPLACE_DROP 1.0
#endif
constexpr double REPLACE_DROP = MSTAB_REPLACE_DROP;
// an FP32 process whose recursive residual grows by DIVERGED_GROWTH, or whose
// true residual grows by FOLD_GROWTH, over the smallest true residual it has
// reached has lost its accuracy and is ended (x returns to that point)
constexpr double DIVERGED_GROWTH = 1e3;
constexpr double FOLD_GROWTH = 1e2;

mstab_status solve_mixed(mstab_solver *h, const double *b, double *x, mstab_info *info,
                         int extra_checks, int accepted)
{
    HistoryArchive archive{h};
    // One FP32 Krylov process per refinement.  At the end of a cycle where
    // its residual has fallen far enough (reliable updating), its iterate is
    // folded into the FP64 x and its recursive residual is replaced by the
    // FP64 true residual b - A x (scaled by the fixed sigma, rounded to
    // FP32).  U, V and the Sonneveld space carry on across the replacement.
    // A refinement ends when the replaced residual meets the tolerance or the
    // FP32 process stops; the FP64 true residual then decides, and a further
    // refinement (fresh process) starts only if it is still too large.
    auto t0 = std::chrono::steady_clock::now();
    Engine<double> &E = h->e64;   // x64, true residuals; FP64 iterations on a stall
    Engine<float> &F = h->e32;
    const double tol2 = h->opt.tol * h->opt.tol;
    SolveResult tot;
    HIPCHK(hipMemcpyAsync(E.X, x, sizeof(double) * h->n, hipMemcpyDeviceToDevice, h->stream));
    h->hist_mv.clear();
    h->hist_res.clear();
    int64_t mv32 = 0, mvchk = extra_checks, mv64 = 0;
    int refinements = 0, abandoned = 0, stalls = 0, fallback = 0;
    double bb = 0.0;
    struct HookGuard {
        Engine<float> &F;
        ~HookGuard() { F.after_cycle = nullptr; F.after_replace = nullptr; }
    } guard{F};
    for (;;) {
        E.small(SMALL_CLEAR);
        E.spmv(E.X, E.Tv, b, ACT_TRUE, 0, 0);
        E.sync_status();
        ++mv64;
        bb = E.st_host->bb;
        const double tt = E.st_host->tt;
        if (!std::isfinite(bb) || !std::isfinite(tt)) { tot.status = MSTAB_E_NONFINITE; break; }
        if (bb == 0.0) {
            E.fill(E.X, E.ld, 0.0);
            tot.converged = true;
            tot.relres_true = 0.0;
            break;
        }
        tot.relres_true = std::sqrt(tt / bb);
        tot.relres_rec = tot.relres_true;
        if (h->hist_mv.empty()) {
            h->hist_mv.push_back(mv32 + mv64 + mvchk);
            h->hist_res.push_back(tot.relres_true);
        }
        if (tt <= tol2 * bb) { tot.converged = true; break; }
        if (stalls >= 2) break;   // FP64 iterations finish below
        if (refinements >= h->opt.max_refinements ||
            mv32 + mv64 + mvchk >= h->opt.max_mv) {
            tot.status = MSTAB_NOT_CONVERGED;
            break;
        }
        const double sigma = std::sqrt(tt);
        const double inv_sigma = 1.0 / sigma;
        hipLaunchKernelGGL(k_scale_to_f32, dim3(grid1(h->n)), dim3(BLOCK), 0, h->stream, h->n,
                           E.Tv, inv_sigma, h->r32);
        HIPCHK(hipGetLastError());
        F.fill(F.X, F.ld, 0.0f);
        // in units of sigma the FP64 tolerance is tol ||b|| / sigma (a
        // replaced residual is the true one, so the process may aim there)
        const double scale = std::sqrt(bb) / sigma;
        const double thr2_inner = tol2 * scale * scale;
        // Replace once the recursive residual has dropped by REPLACE_DROP
        // below the last true one, and whenever the process would stop on
        // it.  x at the smallest true residual so far is kept in xbak; a
        // process whose residual grows well past that is ended, and x returns
        // to the best point before the next refinement.
        double last_rr = 1.0, best_rr = 1.0;
        bool stopped = false, pending_fold = false;
        int64_t hook_mv = 0;
        HIPCHK(hipMemcpyAsync(h->xbak, E.X, sizeof(double) * h->n, hipMemcpyDeviceToDevice,
                              h->stream));
        F.after_cycle = [&, sigma, inv_sigma](double rr_now) -> int {
            if (!std::isfinite(rr_now) || rr_now > DIVERGED_GROWTH * DIVERGED_GROWTH * best_rr) {
                stopped = true;
                return Engine<float>::HOOK_STOP;
            }
            if (!(rr_now <= REPLACE_DROP * REPLACE_DROP * last_rr || rr_now <= thr2_inner))
                return Engine<float>::HOOK_NONE;
            pending_fold = true;
            hipLaunchKernelGGL(k_correct, dim3(grid1(h->n)), dim3(BLOCK), 0, h->stream, h->n, F.X,
                               sigma, E.X);
            F.fill(F.X, F.ld, 0.0f);
            E.spmv(E.X, E.Tv, b, ACT_TRUE, 0, 0);
            ++hook_mv;
            hipLaunchKernelGGL(k_scale_to_f32, dim3(grid1(h->n)), dim3(BLOCK), 0, h->stream, h->n,
                               E.Tv, inv_sigma, F.Rc(0));
            F.project(F.Rc(0), 1, 0);
            F.small(SMALL_REPLACE);
            return Engine<float>::HOOK_REPLACED;
        };
        F.after_replace = [&](double rr_true) -> bool {
            if (!std::isfinite(rr_true)) {
                stopped = true;
                return false;   // pending: x returns to the best point below
            }
            pending_fold = false;
            last_rr = rr_true;
            if (rr_true < best_rr) {
                best_rr = rr_true;
                HIPCHK(hipMemcpyAsync(h->xbak, E.X, sizeof(double) * h->n,
                                      hipMemcpyDeviceToDevice, h->stream));
            } else if (rr_true > FOLD_GROWTH * FOLD_GROWTH * best_rr) {
                stopped = true;
                return false;
            }
            return true;
        };
        SolveResult in = F.solve(h->r32, h->opt.tol * scale, h->opt.max_mv - (mv32 + mv64 + mvchk),
                                 h->opt.method, h->opt.fetch, h->opt.fetch_rel * scale,
                                 h->opt.fetch_level, 0, false);
        F.after_cycle = nullptr;
        F.after_replace = nullptr;
        if (pending_fold || last_rr > best_rr) {
            // x is not at the best true residual of this process: go back there
            HIPCHK(hipMemcpyAsync(E.X, h->xbak, sizeof(double) * h->n, hipMemcpyDeviceToDevice,
                                  h->stream));
            stopped = true;
        }
        ++refinements;
        mv32 += in.mv;
        mv64 += hook_mv;
        mvchk += in.mv_check;
        tot.cycles += in.cycles;
        tot.restarts += in.restarts;
        tot.replacements += in.replacements;
        tot.recycled = tot.recycled || in.recycled;
        tot.level = in.level;
        if (in.fetched >= 0) tot.fetched = in.fetched;
        // progress after the last confirmed replacement (at most one cycle
        // that did not lower the residual) is not folded: x stays at the
        // best confirmed point
        if (stopped) ++abandoned;
        // a process that ended without lowering the true residual tenfold
        // is a stall; after two, FP64 iterations finish the system from the
        // best x (FP32 cannot carry this (s, l) on this matrix)
        stalls = (best_rr > 1e-2) ? stalls + 1 : 0;
        const int64_t base = h->hist_mv.back();
        for (size_t i = 1; i < F.hist_mv.size(); ++i) {
            h->hist_mv.push_back(base + F.hist_mv[i] + (int64_t)i);
            h->hist_res.push_back(F.hist_res[i] / scale);
        }
        if (in.status < 0 && in.status != MSTAB_E_BREAKDOWN && in.status != MSTAB_E_NONFINITE) {
            tot.status = in.status;
            break;
        }
    }
    if (!tot.converged && tot.status != MSTAB_E_NONFINITE && stalls >= 2 &&
        mv32 + mv64 + mvchk < h->opt.max_mv) {
        fallback = 1;
        SolveResult in = E.solve(b, h->opt.tol, h->opt.max_mv - (mv32 + mv64 + mvchk),
                                 h->opt.method, h->opt.fetch, h->opt.fetch_rel, h->opt.fetch_level,
                                 h->opt.max_replacements);
        mv64 += in.mv + in.mv_check;
        tot.cycles += in.cycles;
        tot.restarts += in.restarts;
        tot.replacements += in.replacements;
        tot.converged = in.converged;
        tot.status = in.status;
        tot.relres_true = in.relres_true;
        tot.relres_rec = in.relres_rec;
        for (size_t i = 0; i < E.hist_mv.size(); ++i) {
            h->hist_mv.push_back(mv32 + mvchk + (mv64 - in.mv - in.mv_check) + E.hist_mv[i]);
            h->hist_res.push_back(E.hist_res[i]);
        }
    }
    if (tot.status == MSTAB_OK && !tot.converged) tot.status = MSTAB_NOT_CONVERGED;
    HIPCHK(hipMemcpyAsync(x, E.X, sizeof(double) * h->n, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    tot.mv = mv32;
    tot.mv_check = mvchk + mv64;
    h->mv_last = tot.mv + tot.mv_check;
    h->mv_total += h->mv_last;
    double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    fill_info(info, tot, secs);
    if (info) {
        info->refinements = refinements;
        info->mv_f64 = mv64;
        info->guess_accepted = accepted;
        info->restarts += abandoned;
        info->f64_fallback = fallback;
    }
    return (mstab_status)tot.status;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

mstab_status mstab_options_default(mstab_options *o)
{
    if (!o) return MSTAB_E_INVALID;
    memset(o, 0, sizeof *o);
    o->struct_size = (int32_t)sizeof(mstab_options);
    o->tol = 1e-8;
    o->max_mv = 100000;
    o->method = MSTAB_METHOD_MSTAB;
    o->precision = MSTAB_PREC_F64;
    o->fetch = MSTAB_FETCH_THRESHOLD;
    o->fetch_rel = 1e-4;
    o->fetch_level = -1;
    o->p_seed = 0;
    o->max_replacements = 3;
    o->max_refinements = 20;
    o->gmres_restart = 30;
    return MSTAB_OK;
}

mstab_status mstab_create(const mstab_csr *A, int32_t s, int32_t ell, const mstab_options *o,
                          void *hip_stream, mstab_solver **out)
{
    mstab_solver *h = nullptr;
    API_BEGIN
    if (!out) fail(MSTAB_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!A || !A->row_ptr || !A->col_idx || !A->val) fail(MSTAB_E_INVALID, "matrix pointer is NULL");
    if (s < 1 || s > MAXS) fail(MSTAB_E_INVALID, "s=%d outside 1..%d", s, MAXS);
    if (ell < 1 || ell > MAXL) fail(MSTAB_E_INVALID, "ell=%d outside 1..%d", ell, MAXL);
    if (A->n <= s) fail(MSTAB_E_INVALID, "n=%lld must exceed s=%d", (long long)A->n, s);
    if (A->n >= (int64_t)1 << 29) fail(MSTAB_E_INVALID, "n=%lld too large", (long long)A->n);
    if (A->nnz < 0 || A->nnz >= ((int64_t)1 << 31)) fail(MSTAB_E_INVALID, "nnz out of range");
    if (o && o->struct_size != (int32_t)sizeof(mstab_options))
        fail(MSTAB_E_INVALID, "options struct_size mismatch");
    h = new mstab_solver();
    if (o) h->opt = *o;
    else mstab_options_default(&h->opt);
    if (!(h->opt.tol > 0.0) || h->opt.max_mv < 1) fail(MSTAB_E_INVALID, "tol/max_mv invalid");
    if (h->opt.precision != MSTAB_PREC_F64 && h->opt.precision != MSTAB_PREC_F32_REFINE &&
        h->opt.precision != MSTAB_PREC_F32_MATRIX)
        fail(MSTAB_E_INVALID, "unknown precision");
    if (h->opt.precond != MSTAB_PRECOND_NONE && h->opt.precond != MSTAB_PRECOND_JACOBI &&
        h->opt.precond != MSTAB_PRECOND_ILU0)
        fail(MSTAB_E_INVALID, "unknown preconditioner");
    if (h->opt.precond == MSTAB_PRECOND_ILU0 && h->opt.precision != MSTAB_PREC_F64)
        fail(MSTAB_E_INVALID, "ILU(0) preconditioning runs in F64 precision only");
    if (h->opt.precond == MSTAB_PRECOND_ILU0 && h->opt.reorder != MSTAB_REORDER_NONE)
        fail(MSTAB_E_INVALID, "ILU(0) preconditioning orders the matrix itself; reorder must be NONE");
    if (h->opt.replace_every < 0) fail(MSTAB_E_INVALID, "replace_every < 0");
    if (h->opt.matrix_format < MSTAB_FORMAT_AUTO || h->opt.matrix_format > MSTAB_FORMAT_SLICED)
        fail(MSTAB_E_INVALID, "unknown matrix format");
    if (h->opt.reorder != MSTAB_REORDER_NONE && h->opt.reorder != MSTAB_REORDER_RCM)
        fail(MSTAB_E_INVALID, "unknown reordering");
    if (h->opt.fetch < MSTAB_FETCH_THRESHOLD || h->opt.fetch > MSTAB_FETCH_ESTIMATE)
        fail(MSTAB_E_INVALID, "unknown fetch policy");
    if (h->opt.orthonormalize_recycle != 0 && h->opt.orthonormalize_recycle != 1)
        fail(MSTAB_E_INVALID, "orthonormalize_recycle must be 0 or 1");
    if (h->opt.engine != MSTAB_ENGINE_GRID && h->opt.engine != MSTAB_ENGINE_WORKGROUP)
        fail(MSTAB_E_INVALID, "unknown engine");
    if (h->opt.method != MSTAB_METHOD_MSTAB && h->opt.method != MSTAB_METHOD_IDRSTAB &&
        h->opt.method != MSTAB_METHOD_GMRES)
        fail(MSTAB_E_INVALID, "unknown method");
    if (h->opt.method == MSTAB_METHOD_GMRES) {
        if (h->opt.gmres_restart < 1 || h->opt.gmres_restart > 1024)
            fail(MSTAB_E_INVALID, "gmres_restart=%d outside 1..1024", h->opt.gmres_restart);
        if (h->opt.precision != MSTAB_PREC_F64 || h->opt.engine != MSTAB_ENGINE_GRID)
            fail(MSTAB_E_INVALID, "GMRES: F64 precision and ENGINE_GRID only");
    }
    if (h->opt.engine == MSTAB_ENGINE_WORKGROUP) {
        if (A->n > wg::MAX_N) fail(MSTAB_E_INVALID, "ENGINE_WORKGROUP: n=%lld above 2^20", (long long)A->n);
        if (h->opt.precision != MSTAB_PREC_F64 || h->opt.precond != MSTAB_PRECOND_NONE ||
            h->opt.reorder != MSTAB_REORDER_NONE || h->opt.orthonormalize_recycle)
            fail(MSTAB_E_INVALID, "ENGINE_WORKGROUP: F64, no preconditioner, no reordering and "
                                  "no orthonormalization only");
    }
    h->s = s; h->ell = ell; h->n = A->n; h->nnz = A->nnz;
    h->rp = A->row_ptr; h->ci = A->col_idx; h->va = A->val;
    h->stream = (hipStream_t)hip_stream;
    HIPCHK(hipGetDevice(&h->device));
    h->pkey = p_key_from_seed(h->opt.p_seed);
    if (h->opt.p_host) {
        // the caller's cut-space basis: n x s, column q at p_host + q n, finite
        const double *ph = h->opt.p_host;
        uint64_t dg = 1469598103934665603ull;
        for (int64_t i = 0; i < h->n * (int64_t)s; ++i) {
            if (!std::isfinite(ph[i])) fail(MSTAB_E_INVALID, "p_host holds a non-finite value");
            unsigned char b8[8];
            memcpy(b8, &ph[i], 8);
            for (int k = 0; k < 8; ++k) dg = (dg ^ b8[k]) * 1099511628211ull;
        }
        h->p_digest = dg;
    }
    h->prof.init(h->stream);
    check_csr_dev(h->n, h->nnz, h->rp, h->ci, h->stream);
    const bool use_ilu = h->opt.precond == MSTAB_PRECOND_ILU0;
    std::vector<int32_t> host_perm;   // new row -> the caller's row, when the handle reorders
    if (h->opt.reorder == MSTAB_REORDER_RCM || use_ilu) {
        // host: the order (reverse Cuthill-McKee, or the multicolour order of
        // the ILU(0) splitting) and the symmetrically permuted CSR
        const int64_t n = h->n;
        std::vector<int32_t> rp((size_t)n + 1), ci((size_t)h->nnz);
        std::vector<double> va((size_t)h->nnz);
        HIPCHK(hipMemcpyAsync(rp.data(), h->rp, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipMemcpyAsync(ci.data(), h->ci, sizeof(int32_t) * h->nnz, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipMemcpyAsync(va.data(), h->va, sizeof(double) * h->nnz, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        std::vector<int64_t> cp;
        const std::vector<int32_t> perm = use_ilu ? multicolour_order(n, rp.data(), ci.data(), cp)
                                                  : rcm_order(n, rp.data(), ci.data());
        if ((int64_t)perm.size() != n) fail(MSTAB_E_INVALID, "reordering lost rows");
        host_perm = perm;
        std::vector<int32_t> prp, pci;
        std::vector<double> pva;
        permute_csr(n, rp, ci, va, perm, prp, pci, pva);
        HIPCHK(hipMalloc(&h->perm, sizeof(int32_t) * (size_t)n));
        HIPCHK(hipMalloc(&h->rp_perm, sizeof(int32_t) * (size_t)(n + 1)));
        HIPCHK(hipMalloc(&h->ci_perm, sizeof(int32_t) * (size_t)std::max<int64_t>(h->nnz, 1)));
        HIPCHK(hipMalloc(&h->va_perm, sizeof(double) * (size_t)std::max<int64_t>(h->nnz, 1)));
        HIPCHK(hipMalloc(&h->xwork, sizeof(double) * (size_t)round_up(n, 256)));
        if (!h->bhat) HIPCHK(hipMalloc(&h->bhat, sizeof(double) * (size_t)round_up(n, 256)));
        HIPCHK(hipMemcpyAsync(h->perm, perm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipMemcpyAsync(h->rp_perm, prp.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipMemcpyAsync(h->ci_perm, pci.data(), sizeof(int32_t) * h->nnz, hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipMemcpyAsync(h->va_perm, pva.data(), sizeof(double) * h->nnz, hipMemcpyHostToDevice, h->stream));
        if (use_ilu) {
            // diagonal positions, then the factorization colour by colour
            std::vector<int32_t> dpos((size_t)n, -1);
            for (int64_t i = 0; i < n; ++i)
                for (int32_t k = prp[i]; k < prp[i + 1]; ++k)
                    if (pci[k] == i) dpos[i] = k;
            for (int64_t i = 0; i < n; ++i)
                if (dpos[i] < 0) fail(MSTAB_E_INVALID, "ILU(0): row %lld has no diagonal entry", (long long)i);
            IluData &L = h->ilu;
            L.n = n;
            L.nnz = h->nnz;
            L.rp = h->rp_perm;
            L.ci = h->ci_perm;
            L.cp = cp;
            HIPCHK(hipMalloc(&L.lu, sizeof(double) * (size_t)std::max<int64_t>(h->nnz, 1)));
            HIPCHK(hipMalloc(&L.dpos, sizeof(int32_t) * (size_t)n));
            HIPCHK(hipMalloc(&L.t1, sizeof(double) * (size_t)round_up(n, 256)));
            HIPCHK(hipMalloc(&L.t2, sizeof(double) * (size_t)round_up(n, 256)));
            HIPCHK(hipMemcpyAsync(L.dpos, dpos.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, h->stream));
            HIPCHK(hipMemcpyAsync(L.lu, pva.data(), sizeof(double) * h->nnz, hipMemcpyHostToDevice, h->stream));
            int *bad = nullptr;
            HIPCHK(hipMalloc(&bad, sizeof(int)));
            int hbad = 0;
            hipError_t e = hipMemsetAsync(bad, 0, sizeof(int), h->stream);
            for (int c = 0; c < L.colours() && e == hipSuccess; ++c) {
                const int64_t rows = cp[c + 1] - cp[c];
                hipLaunchKernelGGL(k_ilu0_rows, dim3(grid_for(rows, BLOCK, VEC_MAX_BLOCKS)), dim3(BLOCK), 0,
                                   h->stream, cp[c], cp[c + 1], (const int32_t *)L.rp, (const int32_t *)L.ci,
                                   L.lu, (const int32_t *)L.dpos, bad);
                e = hipGetLastError();
            }
            if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, h->stream);
            const hipError_t se = hipStreamSynchronize(h->stream);
            (void)hipFree(bad);
            HIPCHK(e);
            HIPCHK(se);
            if (hbad) fail(MSTAB_E_INVALID, "ILU(0): a zero or non-finite pivot");
            L.make_sell(prp, dpos, h->stream);
            // Eisenstat's form where the factors allow it (no triangles in the pattern)
            {
                int *ebad = nullptr;
                HIPCHK(hipMalloc(&ebad, sizeof(int)));
                int hb = 1;
                hipError_t e2 = hipMemsetAsync(ebad, 0, sizeof(int), h->stream);
                if (e2 == hipSuccess) {
                    hipLaunchKernelGGL(k_ilu_check_eis, dim3(grid_for(n, BLOCK, VEC_MAX_BLOCKS)), dim3(BLOCK), 0,
                                       h->stream, n, (const int32_t *)L.rp, (const int32_t *)L.ci,
                                       (const double *)h->va_perm, (const double *)L.lu,
                                       (const int32_t *)L.dpos, ebad);
                    e2 = hipGetLastError();
                }
                if (e2 == hipSuccess) e2 = hipMemcpyAsync(&hb, ebad, sizeof(int), hipMemcpyDeviceToHost, h->stream);
                const hipError_t s2 = hipStreamSynchronize(h->stream);
                (void)hipFree(ebad);
                HIPCHK(e2);
                HIPCHK(s2);
                if (!hb) {
                    HIPCHK(hipMalloc(&L.dd, sizeof(double) * (size_t)round_up(n, 256)));
                    HIPCHK(hipMalloc(&L.du, sizeof(double) * (size_t)round_up(n, 256)));
                    hipLaunchKernelGGL(k_ilu_eis_diag, dim3(grid_for(n, BLOCK, VEC_MAX_BLOCKS)), dim3(BLOCK), 0,
                                       h->stream, n, (const double *)h->va_perm, (const double *)L.lu,
                                       (const int32_t *)L.dpos, L.dd, L.du);
                    HIPCHK(hipGetLastError());
                    L.eis = true;
                }
            }
        }
        HIPCHK(hipStreamSynchronize(h->stream));   // the host vectors go out of scope
        h->rp = h->rp_perm;
        h->ci = h->ci_perm;
        h->va = h->va_perm;
    }
    if (h->opt.p_host) {
        // the device copy of the caller's P, its rows permuted with A's when the
        // handle reorders (the method is invariant under the joint permutation)
        const double *ph = h->opt.p_host;
        const int64_t n = h->n;
        std::vector<double> pp;
        if (!host_perm.empty()) {
            pp.resize((size_t)n * (size_t)s);
            for (int q = 0; q < s; ++q)
                for (int64_t i = 0; i < n; ++i) pp[(size_t)q * n + i] = ph[(size_t)q * n + host_perm[i]];
            ph = pp.data();
        }
        HIPCHK(hipMalloc(&h->pmat, sizeof(double) * (size_t)n * (size_t)s));
        HIPCHK(hipMemcpyAsync(h->pmat, ph, sizeof(double) * (size_t)n * (size_t)s, hipMemcpyHostToDevice,
                              h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        h->opt.p_host = nullptr;   // the handle keeps its own copy, not the caller's pointer
    }
    double *split_val = nullptr;   // L^-1 A R^-1, needed only while the device copies are built
    if (h->opt.precond == MSTAB_PRECOND_JACOBI) {
        const size_t vb = sizeof(double) * (size_t)round_up(h->n, 256);
        HIPCHK(hipMalloc(&h->pd, vb));
        HIPCHK(hipMalloc(&h->pe, vb));
        if (!h->bhat) HIPCHK(hipMalloc(&h->bhat, vb));
        HIPCHK(hipMalloc(&split_val, sizeof(double) * (size_t)std::max<int64_t>(h->nnz, 1)));
        h->split_tmp = split_val;
        jacobi_split_dev(h->n, h->rp, h->ci, h->va, split_val, h->pd, h->pe, h->stream);
        h->va = split_val;
    }
    Sell<double> A64 = make_sell<double, double>(h->n, h->rp, h->ci, h->va, h->stream, nullptr,
                                                 h->opt.matrix_format);
    // the mixed form keeps a full FP64 engine for the FP64 fallback
    h->e64.alloc(h->n, s, ell, A64, true, h->pbasis(), h->stream, &h->prof);
    if (use_ilu) h->e64.ilu = &h->ilu;
    if (h->opt.method == MSTAB_METHOD_GMRES) h->e64.alloc_gmres(h->opt.gmres_restart);
    h->e64.replace_every = h->opt.replace_every;
    h->e64.orthonormalize = h->opt.orthonormalize_recycle != 0;
    if (h->opt.precision == MSTAB_PREC_F32_MATRIX) {
        h->e64.A_low = make_sell<float, double>(h->n, h->rp, h->ci, h->va, h->stream, &A64);
        h->e64.use_low = true;
    }
    if (h->mixed()) {
        HIPCHK(hipMalloc(&h->r32, sizeof(float) * (size_t)round_up(h->n, 256)));
        HIPCHK(hipMemsetAsync(h->r32, 0, sizeof(float) * (size_t)round_up(h->n, 256), h->stream));
        HIPCHK(hipMalloc(&h->xbak, sizeof(double) * (size_t)round_up(h->n, 256)));
        Sell<float> A32 = make_sell<float, double>(h->n, h->rp, h->ci, h->va, h->stream, &A64);
        h->e32.alloc(h->n, s, ell, A32, false, h->pbasis(), h->stream, &h->prof);
        h->e32.refresh_v = true;
        h->e32.orthonormalize = h->opt.orthonormalize_recycle != 0;
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    // the device copies hold the split (and reordered) values; the reordered
    // row pointer stays (the sliced product reads it); the rest is released
    (void)hipFree(h->split_tmp);
    h->split_tmp = nullptr;
    if (!use_ilu) {   // the ILU(0) solves keep reading the ordered structure
        (void)hipFree(h->ci_perm);
        h->ci_perm = nullptr;
    }
    (void)hipFree(h->va_perm);
    h->va_perm = nullptr;
    h->va = h->perm ? nullptr : A->val;
    h->ci = h->perm ? nullptr : A->col_idx;
    *out = h;
    return MSTAB_OK;
    }
    catch (const StatusError &e) {
        mstab_status st = record(h, e);
        release_handle(h);
        return st;
    }
    catch (const HipError &e) {
        mstab_status st = record_hip(h, e);
        release_handle(h);
        return (e.e == hipErrorOutOfMemory) ? MSTAB_E_NOMEM : st;
    }
    catch (const std::bad_alloc &) {
        g_tls_error = "host allocation failed";
        return MSTAB_E_NOMEM;
    }
}

mstab_status mstab_solve_next(mstab_solver *h, const double *b, double *x, mstab_info *info)
{
    if (!h) { g_tls_error = "handle is NULL"; return MSTAB_E_INVALID; }
    API_BEGIN
    if (!b || !x) fail(MSTAB_E_INVALID, "b or x is NULL");
    if (!h->transformed())
        return h->mixed() ? solve_mixed(h, b, x, info, 0, 0) : solve_f64(h, b, x, info, 0, 0);
    const int grid = grid1(h->n);
    if (h->ilu.lu) {
        // ILU(0) split system in the multicolour order: b^ = L^-1 b[perm],
        // y0 = U x0[perm]; afterwards x[perm] = U^-1 y (also after a failure)
        const IluData &L = h->ilu;
        hipLaunchKernelGGL(k_gather, dim3(grid), dim3(BLOCK), 0, h->stream, h->n, h->perm, b,
                           (const double *)nullptr, h->bhat);
        HIPCHK(hipGetLastError());
        L.lower_solve(h->bhat, h->stream);
        hipLaunchKernelGGL(k_gather, dim3(grid), dim3(BLOCK), 0, h->stream, h->n, h->perm, x,
                           (const double *)nullptr, L.t1);
        HIPCHK(hipGetLastError());
        L.upper_mul(L.t1, h->xwork, h->stream);
        auto finish = [&]() {
            L.upper_solve(h->xwork, L.t1, h->stream);
            hipLaunchKernelGGL(k_scatter, dim3(grid), dim3(BLOCK), 0, h->stream, h->n, h->perm,
                               (const double *)L.t1, (const double *)nullptr, x);
        };
        mstab_status st;
        try {
            st = solve_f64(h, h->bhat, h->xwork, info, 0, 0);
        } catch (...) {
            finish();
            throw;
        }
        finish();
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(h->stream));
        return st;
    }
    if (h->perm) {
        // reordered (and possibly split) system: b' = L^-1 b[perm], y0 = R x0[perm];
        // afterwards x[perm] = R^-1 y (also after a failure)
        hipLaunchKernelGGL(k_gather, dim3(grid), dim3(BLOCK), 0, h->stream, h->n, h->perm, b,
                           (const double *)h->pd, h->bhat);
        HIPCHK(hipGetLastError());
        hipLaunchKernelGGL(k_gather, dim3(grid), dim3(BLOCK), 0, h->stream, h->n, h->perm, x,
                           (const double *)h->pe, h->xwork);
        HIPCHK(hipGetLastError());
        mstab_status st;
        try {
            st = h->mixed() ? solve_mixed(h, h->bhat, h->xwork, info, 0, 0)
                            : solve_f64(h, h->bhat, h->xwork, info, 0, 0);
        } catch (...) {
            hipLaunchKernelGGL(k_scatter, dim3(grid), dim3(BLOCK), 0, h->stream, h->n, h->perm,
                               (const double *)h->xwork, (const double *)h->pd, x);
            throw;
        }
        hipLaunchKernelGGL(k_scatter, dim3(grid), dim3(BLOCK), 0, h->stream, h->n, h->perm,
                           (const double *)h->xwork, (const double *)h->pd, x);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(h->stream));
        return st;
    }
    // split system: L^-1 b, y0 = R x0; afterwards x = R^-1 y (also after a failure)
    hipLaunchKernelGGL(k_mul, dim3(grid), dim3(BLOCK), 0, h->stream, h->n, b, h->pd, h->bhat);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_mul, dim3(grid), dim3(BLOCK), 0, h->stream, h->n, x, h->pe, x);
    HIPCHK(hipGetLastError());
    mstab_status st;
    try {
        st = h->mixed() ? solve_mixed(h, h->bhat, x, info, 0, 0)
                        : solve_f64(h, h->bhat, x, info, 0, 0);
    } catch (...) {
        hipLaunchKernelGGL(k_mul, dim3(grid), dim3(BLOCK), 0, h->stream, h->n, x, h->pd, x);
        throw;
    }
    hipLaunchKernelGGL(k_mul, dim3(grid), dim3(BLOCK), 0, h->stream, h->n, x, h->pd, x);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->stream));
    return st;
    API_END(h)
}

mstab_status mstab_solve_batch(mstab_solver *const *h, int32_t count, const double *const *b,
                               double *const *x, mstab_info *info)
{
    API_BEGIN
    if (count < 0 || count > MSTAB_MAX_BATCH) fail(MSTAB_E_INVALID, "count=%d outside 0..%d", count, MSTAB_MAX_BATCH);
    if (count == 0) return MSTAB_OK;
    if (!h || !b || !x) fail(MSTAB_E_INVALID, "NULL array");
    for (int i = 0; i < count; ++i) {
        if (!h[i] || !b[i] || !x[i]) fail(MSTAB_E_INVALID, "NULL entry %d", i);
        for (int j = 0; j < i; ++j)
            if (h[j] == h[i]) fail(MSTAB_E_INVALID, "handle %d repeated", i);
    }
    if (h[0]->workgroup()) {
        for (int i = 0; i < count; ++i)
            if (!h[i]->workgroup()) fail(MSTAB_E_INVALID, "handle %d is not of ENGINE_WORKGROUP like handle 0", i);
        // the launch runs on h[0]'s device; the caller's current device is restored
        int prev = 0;
        HIPCHK(hipGetDevice(&prev));
        struct Restore {
            int dev;
            ~Restore() { (void)hipSetDevice(dev); }
        } restore{prev};
        HIPCHK(hipSetDevice(h[0]->device));
        const mstab_status w = wg_run(h, count, b, x, info, 0, 0);
        if (w < 0)
            for (int i = 0; i < count; ++i)
                if (info && info[i].status < 0) {
                    g_tls_error = "handle " + std::to_string(i) + ": " + h[i]->err;
                    break;
                }
        return w;
    }
    for (int i = 0; i < count; ++i)
        if (h[i]->workgroup()) fail(MSTAB_E_INVALID, "handle %d is of ENGINE_WORKGROUP, handle 0 is not", i);
    std::vector<mstab_status> st((size_t)count, MSTAB_OK);
    std::vector<std::thread> pool;
    // each worker takes the next handle; each handle's calls run on one host
    // thread at a time and on the handle's stream
    std::atomic<int> next{1};
    auto work = [&]() {
        for (int i = 0; i < count; i = next.fetch_add(1)) {
            if (i == 0) continue;   // handle 0 is the calling thread's
            if (hipSetDevice(h[i]->device) != hipSuccess) {
                h[i]->err = "hipSetDevice failed in a batch worker";
                st[i] = MSTAB_E_HIP;
                continue;
            }
            st[i] = mstab_solve_next(h[i], b[i], x[i], info ? &info[i] : nullptr);
        }
    };
    const int workers = std::min(count - 1, 15);
    pool.reserve((size_t)workers);
    try {
        for (int t = 0; t < workers; ++t) pool.emplace_back(work);
    } catch (...) {
        for (auto &t : pool) t.join();
        fail(MSTAB_E_NOMEM, "could not start %d host threads", workers);
    }
    st[0] = mstab_solve_next(h[0], b[0], x[0], info ? &info[0] : nullptr);
    work();
    for (auto &t : pool) t.join();
    mstab_status worst = MSTAB_OK;
    for (int i = 0; i < count; ++i) {
        if (st[i] < 0) {
            if (worst >= 0) {
                worst = st[i];
                g_tls_error = "handle " + std::to_string(i) + ": " + h[i]->err;
            }
        } else if (st[i] == MSTAB_NOT_CONVERGED && worst == MSTAB_OK) {
            worst = MSTAB_NOT_CONVERGED;
        }
    }
    return worst;
    API_END(nullptr)
}

mstab_status mstab_solve_next_guess(mstab_solver *h, const double *b, const double *x_prev,
                                    const double *x_guess, double *x, mstab_info *info)
{
    if (!h) { g_tls_error = "handle is NULL"; return MSTAB_E_INVALID; }
    API_BEGIN
    if (!b || !x_prev || !x_guess || !x) fail(MSTAB_E_INVALID, "NULL vector");
    if (h->transformed()) fail(MSTAB_E_INVALID, "guess gate on a preconditioned or reordered handle");
    Engine<double> &E = h->e64;
    E.small(SMALL_CLEAR);
    HIPCHK(hipMemcpyAsync(E.X, x_guess, sizeof(double) * h->n, hipMemcpyDeviceToDevice, h->stream));
    E.spmv(E.X, E.Tv, b, ACT_TRUE, 0, 0);
    E.sync_status();
    const double tg = E.st_host->tt;
    HIPCHK(hipMemcpyAsync(E.X, x_prev, sizeof(double) * h->n, hipMemcpyDeviceToDevice, h->stream));
    E.spmv(E.X, E.Tv, b, ACT_TRUE, 0, 0);
    E.sync_status();
    const double tp = E.st_host->tt;
    const int accept = (std::isfinite(tg) && tg < tp) ? 1 : 0;
    const double *x0 = accept ? x_guess : x_prev;
    if (x0 != x)
        HIPCHK(hipMemcpyAsync(x, x0, sizeof(double) * h->n, hipMemcpyDeviceToDevice, h->stream));
    return h->mixed() ? solve_mixed(h, b, x, info, 2, accept) : solve_f64(h, b, x, info, 2, accept);
    API_END(h)
}

mstab_status mstab_residual(mstab_solver *h, const double *b, const double *x, double *r,
                            double *norm2)
{
    if (!h) { g_tls_error = "handle is NULL"; return MSTAB_E_INVALID; }
    API_BEGIN
    if (!b || !x || !r) fail(MSTAB_E_INVALID, "NULL vector");
    if (r == b || r == x) fail(MSTAB_E_INVALID, "r must not alias b or x");
    if (h->transformed()) fail(MSTAB_E_INVALID, "residual on a preconditioned or reordered handle");
    Engine<double> &E = h->e64;
    E.small(SMALL_CLEAR);
    E.spmv(x, r, b, ACT_TRUE, 0, 0);
    E.sync_status();
    if (norm2) *norm2 = E.st_host->tt;
    h->mv_total += 1;
    return MSTAB_OK;
    API_END(h)
}

mstab_status mstab_solve_count(const mstab_solver *h, int64_t *count)
{
    if (!h || !count) return MSTAB_E_INVALID;
    *count = (int64_t)h->hist_mv_all.size();
    return MSTAB_OK;
}

mstab_status mstab_mv_count(const mstab_solver *h, int64_t *total, int64_t *last_system)
{
    if (!h) return MSTAB_E_INVALID;
    if (total) *total = h->mv_total;
    if (last_system) *last_system = h->mv_last;
    return MSTAB_OK;
}

mstab_status mstab_residual_history(const mstab_solver *h, int64_t system, int64_t *mv,
                                    double *relres, int64_t cap, int64_t *len)
{
    if (!h) { g_tls_error = "handle is NULL"; return MSTAB_E_INVALID; }
    if (!len || cap < 0 || (cap > 0 && (!mv || !relres))) {
        g_tls_error = "len NULL, cap < 0, or output arrays NULL";
        return MSTAB_E_INVALID;
    }
    const int64_t count = (int64_t)h->hist_mv_all.size();
    if (system < -1 || system >= count || (system == -1 && count == 0)) {
        char buf[128];
        snprintf(buf, sizeof buf, "system %lld outside -1..%lld", (long long)system, (long long)count - 1);
        g_tls_error = buf;
        const_cast<mstab_solver *>(h)->err = buf;
        return MSTAB_E_INVALID;
    }
    const size_t k = system < 0 ? (size_t)(count - 1) : (size_t)system;
    const std::vector<int64_t> &hm = h->hist_mv_all[k];
    const std::vector<double> &hr = h->hist_res_all[k];
    *len = (int64_t)hm.size();
    for (int64_t i = 0; i < std::min<int64_t>(cap, (int64_t)hm.size()); ++i) {
        mv[i] = hm[i];
        relres[i] = hr[i];
    }
    return MSTAB_OK;
}

mstab_status mstab_recycle_reset(mstab_solver *h)
{
    if (!h) return MSTAB_E_INVALID;
    h->e64.rec_have = false;
    h->e32.rec_have = false;
    h->e64.est_cycle = -1;
    h->e32.est_cycle = -1;
    return MSTAB_OK;
}

mstab_status mstab_recycle_get(const mstab_solver *h, double *U, double *V, int64_t *level,
                               int32_t *have)
{
    if (!h || !have || !level) return MSTAB_E_INVALID;
    mstab_solver *hh = const_cast<mstab_solver *>(h);
    API_BEGIN
    if (h->mixed()) fail(MSTAB_E_INVALID, "recycle_get needs F64 precision");
    *have = h->e64.rec_have ? 1 : 0;
    *level = h->e64.rec_level;
    if (h->e64.rec_have) {
        if (!U || !V) fail(MSTAB_E_INVALID, "U or V is NULL");
        HIPCHK(hipMemcpy2DAsync(U, sizeof(double) * h->n, h->e64.recU, sizeof(double) * h->e64.ld,
                                sizeof(double) * h->n, h->s, hipMemcpyDeviceToDevice, h->stream));
        HIPCHK(hipMemcpy2DAsync(V, sizeof(double) * h->n, h->e64.recV, sizeof(double) * h->e64.ld,
                                sizeof(double) * h->n, h->s, hipMemcpyDeviceToDevice, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
    }
    return MSTAB_OK;
    API_END(hh)
}

mstab_status mstab_recycle_set(mstab_solver *h, const double *U, const double *V, int64_t level)
{
    if (!h) return MSTAB_E_INVALID;
    API_BEGIN
    if (h->mixed()) fail(MSTAB_E_INVALID, "recycle_set needs F64 precision");
    if (!U || !V) fail(MSTAB_E_INVALID, "U or V is NULL");
    Engine<double> &E = h->e64;
    HIPCHK(hipMemcpy2DAsync(E.recU, sizeof(double) * E.ld, U, sizeof(double) * h->n,
                            sizeof(double) * h->n, h->s, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(hipMemcpy2DAsync(E.recV, sizeof(double) * E.ld, V, sizeof(double) * h->n,
                            sizeof(double) * h->n, h->s, hipMemcpyDeviceToDevice, h->stream));
    // P^T V of the installed data
    E.small(SMALL_CLEAR);
    for (int q = 0; q < h->s; ++q) E.project(E.recV + (int64_t)q * E.ld, 0, q);
    HIPCHK(hipMemcpyAsync(E.rec_ptv, &E.ctl->ptv[0][0][0], sizeof(double) * MAXS * MAXS,
                          hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    E.rec_level = level;
    E.rec_have = true;
    return MSTAB_OK;
    API_END(h)
}

namespace {
// Layout of an exported recycle state (host byte blob): this header, then
// the s x s P^T V cache (MAXS x MAXS doubles), then U and V (s columns of n
// doubles each, column-major), the last two only when have is set.
struct RecycleBlob {
    char magic[8];
    uint32_t version;
    int32_t s;
    int64_t n;
    uint64_t p_seed;
    uint64_t p_digest;   // of a caller's cut-space basis (p_host), else 0
    int32_t precond, reorder;
    int32_t have, pad;
    int64_t level;
    int64_t est_cycle;   // FETCH_ESTIMATE's fetch cycle for the next solve (-1: none)
};
constexpr char RECYCLE_MAGIC[8] = {'M', 'S', 'T', 'A', 'B', 'R', 'E', 'C'};
constexpr uint32_t RECYCLE_VERSION = 3;

size_t recycle_blob_size(const mstab_solver *h, bool have)
{
    return sizeof(RecycleBlob) + sizeof(double) * MAXS * MAXS +
           (have ? 2 * sizeof(double) * (size_t)h->s * (size_t)h->n : 0);
}
}  // namespace

mstab_status mstab_recycle_export(const mstab_solver *h, void *dst, size_t cap, size_t *len)
{
    if (!h || !len) return MSTAB_E_INVALID;
    mstab_solver *hh = const_cast<mstab_solver *>(h);
    API_BEGIN
    if (h->mixed()) fail(MSTAB_E_INVALID, "recycle_export needs F64 or F32_MATRIX precision");
    const Engine<double> &E = h->e64;
    const size_t need = recycle_blob_size(h, E.rec_have);
    *len = need;
    if (!dst) return MSTAB_OK;   // size query
    if (cap < need) fail(MSTAB_E_INVALID, "buffer of %zu bytes, %zu needed", cap, need);
    RecycleBlob hd{};
    memcpy(hd.magic, RECYCLE_MAGIC, sizeof hd.magic);
    hd.version = RECYCLE_VERSION;
    hd.s = h->s;
    hd.n = h->n;
    hd.p_seed = h->opt.p_seed;
    hd.p_digest = h->p_digest;
    hd.precond = h->opt.precond;
    hd.reorder = h->opt.reorder;
    hd.have = E.rec_have ? 1 : 0;
    hd.level = E.rec_level;
    hd.est_cycle = E.est_cycle;
    char *out = static_cast<char *>(dst);
    memcpy(out, &hd, sizeof hd);
    double *ptv = reinterpret_cast<double *>(out + sizeof hd);
    HIPCHK(hipMemcpyAsync(ptv, E.rec_ptv, sizeof(double) * MAXS * MAXS, hipMemcpyDeviceToHost, h->stream));
    if (E.rec_have) {
        double *U = ptv + MAXS * MAXS;
        double *V = U + (size_t)h->s * (size_t)h->n;
        HIPCHK(hipMemcpy2DAsync(U, sizeof(double) * h->n, E.recU, sizeof(double) * E.ld,
                                sizeof(double) * h->n, h->s, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipMemcpy2DAsync(V, sizeof(double) * h->n, E.recV, sizeof(double) * E.ld,
                                sizeof(double) * h->n, h->s, hipMemcpyDeviceToHost, h->stream));
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    return MSTAB_OK;
    API_END(hh)
}

mstab_status mstab_recycle_import(mstab_solver *h, const void *src, size_t len)
{
    if (!h) return MSTAB_E_INVALID;
    API_BEGIN
    if (h->mixed()) fail(MSTAB_E_INVALID, "recycle_import needs F64 or F32_MATRIX precision");
    if (!src || len < sizeof(RecycleBlob)) fail(MSTAB_E_INVALID, "no recycle blob");
    RecycleBlob hd;
    memcpy(&hd, src, sizeof hd);
    if (memcmp(hd.magic, RECYCLE_MAGIC, sizeof hd.magic) != 0 || hd.version != RECYCLE_VERSION)
        fail(MSTAB_E_INVALID, "not a recycle blob of this version");
    if (hd.s != h->s || hd.n != h->n || hd.p_seed != h->opt.p_seed || hd.p_digest != h->p_digest ||
        hd.precond != h->opt.precond || hd.reorder != h->opt.reorder)
        fail(MSTAB_E_INVALID, "recycle blob of another problem (s, n, P, preconditioner or order differ)");
    if (len < recycle_blob_size(h, hd.have != 0)) fail(MSTAB_E_INVALID, "recycle blob truncated");
    Engine<double> &E = h->e64;
    E.est_cycle = hd.est_cycle;
    if (!hd.have) {
        E.rec_have = false;
        return MSTAB_OK;
    }
    const double *ptv = reinterpret_cast<const double *>(static_cast<const char *>(src) + sizeof hd);
    const double *U = ptv + MAXS * MAXS;
    const double *V = U + (size_t)h->s * (size_t)h->n;
    HIPCHK(hipMemcpyAsync(E.rec_ptv, ptv, sizeof(double) * MAXS * MAXS, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpy2DAsync(E.recU, sizeof(double) * E.ld, U, sizeof(double) * h->n,
                            sizeof(double) * h->n, h->s, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpy2DAsync(E.recV, sizeof(double) * E.ld, V, sizeof(double) * h->n,
                            sizeof(double) * h->n, h->s, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    E.rec_level = hd.level;
    E.rec_have = true;
    return MSTAB_OK;
    API_END(h)
}

mstab_status mstab_destroy(mstab_solver *h)
{
    release_handle(h);
    return MSTAB_OK;
}

const char *mstab_status_str(mstab_status s)
{
    switch (s) {
    case MSTAB_OK: return "ok";
    case MSTAB_NOT_CONVERGED: return "not converged";
    case MSTAB_E_INVALID: return "invalid argument";
    case MSTAB_E_HIP: return "HIP runtime error";
    case MSTAB_E_NOMEM: return "out of memory";
    case MSTAB_E_BREAKDOWN: return "breakdown";
    case MSTAB_E_NONFINITE: return "non-finite value";
    }
    return "unknown status";
}

const char *mstab_last_error(const mstab_solver *h)
{
    if (h) return h->err.c_str();
    return g_tls_error.c_str();
}

mstab_status mstab_set_profiling(mstab_solver *h, int32_t enable)
{
    if (!h) return MSTAB_E_INVALID;
    API_BEGIN
    HIPCHK(hipStreamSynchronize(h->stream));
    h->prof.harvest();
    h->prof.reset();
    h->prof.on = enable > 0;
    h->prof.period = enable > 0 ? enable : 1;
    return MSTAB_OK;
    API_END(h)
}

mstab_status mstab_kernel_stats(const mstab_solver *h, int32_t kclass, int64_t *launches,
                                double *ms, double *bytes)
{
    if (!h || kclass < 0 || kclass >= MSTAB_K_COUNT) return MSTAB_E_INVALID;
    mstab_solver *hh = const_cast<mstab_solver *>(h);
    API_BEGIN
    HIPCHK(hipStreamSynchronize(h->stream));
    hh->prof.harvest();
    if (launches) *launches = h->prof.launches[kclass];
    if (ms) *ms = h->prof.ms[kclass];
    if (bytes) *bytes = h->prof.nbytes[kclass];
    return MSTAB_OK;
    API_END(hh)
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Standalone kernels (parity checks, time stepping)
// ---------------------------------------------------------------------------
namespace {

struct Scratch {
    Ctl *ctl = nullptr;
    double *part = nullptr;
    Status st{};
    ~Scratch()
    {
        (void)hipFree(ctl);
        (void)hipFree(part);
    }
    void init(hipStream_t s)
    {
        HIPCHK(hipMalloc(&ctl, sizeof(Ctl)));
        HIPCHK(hipMalloc(&part, sizeof(double) * (size_t)PART_STRIDE * PART_VALUES));
        HIPCHK(hipMemsetAsync(ctl, 0, sizeof(Ctl), s));
    }
};

}  // namespace

extern "C" {

mstab_status mstab_rcm_order(int64_t n, const int32_t *row_ptr, const int32_t *col_idx,
                             int32_t *perm)
{
    API_BEGIN
    if (n < 0 || n >= ((int64_t)1 << 29)) fail(MSTAB_E_INVALID, "n out of range");
    if (n == 0) return MSTAB_OK;
    if (!row_ptr || !col_idx || !perm) fail(MSTAB_E_INVALID, "NULL pointer");
    check_row_ptr(n, row_ptr[n], row_ptr);
    check_columns_host(n, row_ptr, col_idx);
    const std::vector<int32_t> p = rcm_order(n, row_ptr, col_idx);
    std::copy(p.begin(), p.end(), perm);
    return MSTAB_OK;
    API_END(nullptr)
}

mstab_status mstab_csr_check(int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx)
{
    API_BEGIN
    if (n < 0 || n >= ((int64_t)1 << 29)) fail(MSTAB_E_INVALID, "n out of range");
    if (nnz < 0 || nnz >= ((int64_t)1 << 31)) fail(MSTAB_E_INVALID, "nnz out of range");
    if (!row_ptr || (nnz > 0 && !col_idx)) fail(MSTAB_E_INVALID, "NULL pointer");
    check_row_ptr(n, nnz, row_ptr);
    check_columns_host(n, row_ptr, col_idx);
    return MSTAB_OK;
    API_END(nullptr)
}

mstab_status mstab_permutation(const mstab_solver *h, int32_t *perm)
{
    if (!h) { g_tls_error = "handle is NULL"; return MSTAB_E_INVALID; }
    if (!perm) return MSTAB_E_INVALID;
    API_BEGIN
    if (!h->perm) {
        for (int64_t i = 0; i < h->n; ++i) perm[i] = (int32_t)i;
        return MSTAB_OK;
    }
    HIPCHK(hipMemcpy(perm, h->perm, sizeof(int32_t) * (size_t)h->n, hipMemcpyDeviceToHost));
    return MSTAB_OK;
    API_END(const_cast<mstab_solver *>(h))
}

mstab_status mstab_jacobi_split(const mstab_csr *A, double *val_out, double *d, double *e,
                                void *hip_stream)
{
    double *td = nullptr, *te = nullptr;
    API_BEGIN
    if (!A || !A->row_ptr || !A->col_idx || !A->val || !val_out) fail(MSTAB_E_INVALID, "NULL pointer");
    if (A->n < 0 || A->n >= ((int64_t)1 << 29) || A->nnz < 0 || A->nnz >= ((int64_t)1 << 31))
        fail(MSTAB_E_INVALID, "size out of range");
    if (A->n == 0) return MSTAB_OK;
    hipStream_t st = (hipStream_t)hip_stream;
    check_csr_dev(A->n, A->nnz, A->row_ptr, A->col_idx, st);
    if (!d) HIPCHK(hipMalloc(&td, sizeof(double) * (size_t)A->n));
    if (!e) HIPCHK(hipMalloc(&te, sizeof(double) * (size_t)A->n));
    jacobi_split_dev(A->n, A->row_ptr, A->col_idx, A->val, val_out, d ? d : td, e ? e : te, st);
    HIPCHK(hipStreamSynchronize(st));
    (void)hipFree(td);
    (void)hipFree(te);
    return MSTAB_OK;
    }
    catch (const StatusError &ex) {
        (void)hipFree(td);
        (void)hipFree(te);
        g_tls_error = ex.msg;
        return ex.st;
    }
    catch (const HipError &ex) {
        (void)hipFree(td);
        (void)hipFree(te);
        mstab_status stt = record_hip(nullptr, ex);
        return (ex.e == hipErrorOutOfMemory) ? MSTAB_E_NOMEM : stt;
    }
}

mstab_status mstab_spmv(const mstab_csr *A, const double *x, double *y, void *hip_stream)
{
    API_BEGIN
    if (!A || !A->row_ptr || !A->col_idx || !A->val || !x || !y) fail(MSTAB_E_INVALID, "NULL pointer");
    if (A->n < 0 || A->n >= ((int64_t)1 << 29) || A->nnz < 0 || A->nnz >= ((int64_t)1 << 31))
        fail(MSTAB_E_INVALID, "size out of range");
    if (A->n == 0) return MSTAB_OK;
    hipStream_t st = (hipStream_t)hip_stream;
    check_csr_dev(A->n, A->nnz, A->row_ptr, A->col_idx, st);
    Scratch sc;
    sc.init(st);
    SpmvArgs a{ACT_NONE, 0, 0, 0, 1, 0u};
    Sell<double> M = make_sell<double, double>(A->n, A->row_ptr, A->col_idx, A->val, st);
    launch_spmv<double>(grid_for(A->n, SPMV_BLOCK, SPMV_MAX_BLOCKS), st, M, x, y,
                        (const double *)nullptr, sc.ctl, sc.part, a);
    const hipError_t le = hipGetLastError();
    const hipError_t se = hipStreamSynchronize(st);
    free_sell(M, true);
    HIPCHK(le);
    HIPCHK(se);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return MSTAB_OK;
    API_END(nullptr)
}

mstab_status mstab_project(int64_t n, int32_t s, uint64_t p_seed, const double *y, double *out,
                           void *hip_stream)
{
    API_BEGIN
    if (!y || !out) fail(MSTAB_E_INVALID, "NULL pointer");
    if (s < 1 || s > MAXS || n < 1 || n >= ((int64_t)1 << 29)) fail(MSTAB_E_INVALID, "size out of range");
    hipStream_t st = (hipStream_t)hip_stream;
    Scratch sc;
    sc.init(st);
    const int grid = grid_for(n, BLOCK, GRAM_MAX_BLOCKS);
    hipLaunchKernelGGL((k_project<double>), dim3(grid), dim3(BLOCK), 0, st, n, y,
                       p_key_from_seed(p_seed), s, 1, 0, sc.ctl, sc.part, PART_STRIDE);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(out, sc.ctl->ptt, sizeof(double) * s, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return MSTAB_OK;
    API_END(nullptr)
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Scratch of mstab_project_noalloc: a control block and the workgroup partials
// of one projection (s + 1 <= MAXS + 1 values from at most GRAM_MAX_BLOCKS
// workgroups), in a file-scope device array that each GPU holds from load
// until the process ends.  Host code uses the per-device address that
// hipGetSymbolAddress returns, never the array's name.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t NOALLOC_CTL_BYTES = (sizeof(Ctl) + 255) / 256 * 256;
constexpr size_t NOALLOC_PART_BYTES = sizeof(double) * (size_t)(MAXS + 1) * PART_STRIDE;
constexpr size_t NOALLOC_BYTES = NOALLOC_CTL_BYTES + NOALLOC_PART_BYTES;
static_assert(GRAM_MAX_BLOCKS <= PART_STRIDE, "projection grid exceeds the partials in scratch");

static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// The device address of scratch on the current device (looked up once per device).
unsigned char *scratch_on_current_device()
{
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) fail(MSTAB_E_INVALID, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) fail(MSTAB_E_HIP, "no device address for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    return (unsigned char *)g_scratch_ptr[dev];
}

// zero the last-workgroup counters of a control block (a kernel, not a
// memset, so that the call can be captured in a graph)
__global__ void k_clear_counters(Ctl *ctl)
{
    if (threadIdx.x < 4) ctl->counter[threadIdx.x] = 0u;
    for (int i = threadIdx.x; i < 4 * 8 * GROUP_PAD; i += blockDim.x) (&ctl->gcount[0][0])[i] = 0u;
}

}  // namespace

extern "C" {

mstab_status mstab_project_noalloc(int64_t n, int32_t s, uint64_t p_seed, const double *y,
                                   double *out, void *hip_stream)
{
    API_BEGIN
    if (!y || !out) fail(MSTAB_E_INVALID, "NULL pointer");
    if (s < 1 || s > MAXS) fail(MSTAB_E_INVALID, "s=%d outside 1..%d", s, MAXS);
    if (n < 1 || n >= ((int64_t)1 << 29))
        fail(MSTAB_E_INVALID, "n=%lld outside 1..2^29-1 (the largest size this call serves)", (long long)n);
    hipStream_t st = (hipStream_t)hip_stream;
    unsigned char *base = scratch_on_current_device();
    Ctl *ctl = (Ctl *)base;
    double *part = (double *)(base + NOALLOC_CTL_BYTES);
    hipLaunchKernelGGL(k_clear_counters, dim3(1), dim3(64), 0, st, ctl);
    HIPCHK(hipGetLastError());
    const int grid = grid_for(n, BLOCK, GRAM_MAX_BLOCKS);
    hipLaunchKernelGGL((k_project<double>), dim3(grid), dim3(BLOCK), 0, st, n, y,
                       p_key_from_seed(p_seed), s, 1, 0, ctl, part, PART_STRIDE);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(out, ctl->ptt, sizeof(double) * s, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return MSTAB_OK;
    API_END(nullptr)
}

mstab_status mstab_rhs_step(int64_t n, const double *x, double inv_dt, const double *f, double *b,
                            void *hip_stream)
{
    API_BEGIN
    if (!x || !f || !b) fail(MSTAB_E_INVALID, "NULL pointer");
    if (n < 0) fail(MSTAB_E_INVALID, "n < 0");
    if (n == 0) return MSTAB_OK;
    hipStream_t st = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(k_rhs_step, dim3(grid1(n)), dim3(BLOCK), 0, st, n, x, inv_dt, f, b);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return MSTAB_OK;
    API_END(nullptr)
}

}  // extern "C"
