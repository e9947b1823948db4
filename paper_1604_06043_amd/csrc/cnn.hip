// Learned initial guess: a 6-layer 3x3 convolutional network (2 -> 32 -> 32 ->
// 32 -> 32 -> 32 -> 1 channels, zero padding, ReLU after all but the last
// layer), BF16 weights and activations, FP32 accumulation, trained on the GPU
// by the kernels below (forward, backward, Adam).
//
// Layout: activations NHWC (channels contiguous), images of H x W pixels with
// W a multiple of 32, a batch stored image after image.  Parameters are one
// FP32 array in the order layer 0..5, each "w[co][ci][di][dj] then b[co]";
// the kernels read BF16 copies made from it after every update:
//   wf[l][tap][co][ci]  (forward A operand, tap = 3 di + dj)
//   wb[l][tap][ci][co]  (backward-data A operand: flipped taps, transposed)
// The four 32 -> 32 layers run as implicit GEMMs on the 32x32x16 BF16 MFMA:
// output rows = output channels, columns = 32 consecutive pixels of a row,
// K = 9 taps x 32 input channels.  Weight gradients are split-K MFMA products
// over pixel tiles staged in LDS, summed over workgroups in a fixed order.
#include "mstab.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

namespace {

constexpr int BLOCK = 256;
constexpr int LOSS_BLOCKS = 1024;

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int NL = 6;
constexpr int CH = 32;
constexpr int TAPS = 9;
constexpr int CIN[NL] = {2, 32, 32, 32, 32, 32};
constexpr int COUT[NL] = {32, 32, 32, 32, 32, 1};
constexpr int DW_BLOCKS = 1024;  // split-K workgroups of a weight gradient
constexpr int NXCD = 8;          // accelerator dies (XCDs) of an MI355X, each with its own L2
constexpr int DW_GROUPS = 32;    // pixel groups of a first/last-layer gradient workgroup (8 threads each)
static_assert(DW_GROUPS <= 32, "a pixel group's step must not exceed the narrowest row (W >= 32)");
constexpr int MAX_DIL = 32;      // largest dilation of a layer

constexpr int param_count_layer(int l) { return COUT[l] * CIN[l] * TAPS + COUT[l]; }
constexpr int param_offset(int l)
{
    int o = 0;
    for (int i = 0; i < l; ++i) o += param_count_layer(i);
    return o;
}
constexpr int NPARAM = param_offset(NL);

struct CnnCtl {
    double loss_sum;
    unsigned long long absmax_bits[2];   // max |r0|, max |x_prev| (bit patterns)
};

// ---------------------------------------------------------------------------
// Parameters -> BF16 working copies
// ---------------------------------------------------------------------------
__global__ void k_prep_weights(const float *__restrict__ p, bf16 *__restrict__ wf,
                               bf16 *__restrict__ wb, float *__restrict__ w0,
                               float *__restrict__ w5, float *__restrict__ bias)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    // middle layers: one thread per (l, tap, a, b)
    if (t < 4 * TAPS * CH * CH) {
        const int l = 1 + t / (TAPS * CH * CH);
        const int r = t % (TAPS * CH * CH);
        const int tap = r / (CH * CH), co = (r / CH) % CH, ci = r % CH;
        const float *w = p + param_offset(l);
        const bf16 v = (bf16)w[(co * CH + ci) * TAPS + tap];
        wf[(size_t)(l - 1) * TAPS * CH * CH + (tap * CH + co) * CH + ci] = v;
        // backward: tap' = 8 - tap, rows = ci, k = co
        wb[(size_t)(l - 1) * TAPS * CH * CH + ((8 - tap) * CH + ci) * CH + co] = v;
    }
    if (t < TAPS * 2 * CH) {   // layer 0: w0[tap][ci][co], values rounded to BF16
        const int tap = t / (2 * CH), ci = (t / CH) % 2, co = t % CH;
        w0[t] = (float)(bf16)p[param_offset(0) + (co * 2 + ci) * TAPS + tap];
    }
    if (t < TAPS * CH) {       // layer 5: w5[tap][ci]
        const int tap = t / CH, ci = t % CH;
        w5[t] = (float)(bf16)p[param_offset(5) + ci * TAPS + tap];
    }
    if (t < NL * CH) {         // biases bias[l][co] (FP32)
        const int l = t / CH, co = t % CH;
        bias[t] = co < COUT[l] ? p[param_offset(l) + COUT[l] * CIN[l] * TAPS + co] : 0.f;
    }
}

// ---------------------------------------------------------------------------
// Sample preparation.  With s = max |r0| and sx = max |x_prev|: input channels
// (r0 / s, x_prev / sx), target ((x_next - x_prev) unit) / s.  Quotients are
// divisions (not products with a reciprocal), rounded to FP32, then to BF16
// (round to nearest even); a zero scale gives a zero channel.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_absmax(int64_t n, const double *__restrict__ r0,
                                                  const double *__restrict__ xp, CnnCtl *ctl)
{
    double m0 = 0.0, m1 = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * BLOCK) {
        m0 = fmax(m0, fabs(r0[e]));
        m1 = fmax(m1, fabs(xp[e]));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        m0 = fmax(m0, __shfl_xor(m0, o));
        m1 = fmax(m1, __shfl_xor(m1, o));
    }
    // the maximum of non-negative doubles is the maximum of their bit
    // patterns, so the result does not depend on the order of the updates
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&ctl->absmax_bits[0], (unsigned long long)__double_as_longlong(m0));
        atomicMax(&ctl->absmax_bits[1], (unsigned long long)__double_as_longlong(m1));
    }
}

__device__ __forceinline__ double scale_of(const CnnCtl *ctl, int i)
{
    return __longlong_as_double((long long)ctl->absmax_bits[i]);
}

__global__ __launch_bounds__(BLOCK) void k_prep_sample(int64_t n, const double *__restrict__ r0,
                                                       const double *__restrict__ xp,
                                                       const double *__restrict__ xn, double unit,
                                                       const CnnCtl *ctl, bf16 *__restrict__ in,
                                                       float *__restrict__ target)
{
#pragma clang fp contract(off)
    const double s = scale_of(ctl, 0), sx = scale_of(ctl, 1);
    for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * BLOCK) {
        const double c0 = s > 0.0 ? r0[e] / s : 0.0;
        const double c1 = sx > 0.0 ? xp[e] / sx : 0.0;
        in[2 * e] = (bf16)(float)c0;
        in[2 * e + 1] = (bf16)(float)c1;
        if (target) target[e] = (float)(s > 0.0 ? ((xn[e] - xp[e]) * unit) / s : 0.0);
    }
}

// x_guess = x_prev + (s / unit) out, each operation rounded (no contraction).
// x_prev and x_guess may be the same array (each element is read, then written).
__global__ __launch_bounds__(BLOCK) void k_guess(int64_t n, const double *xp,
                                                 const float *__restrict__ out, double unit,
                                                 const CnnCtl *ctl, double *xg)
{
#pragma clang fp contract(off)
    const double q = scale_of(ctl, 0) / unit;
    for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * BLOCK)
        xg[e] = xp[e] + q * (double)out[e];
}

// ---------------------------------------------------------------------------
// Layer 0 (2 -> 32) and layer 5 (32 -> 1): one thread per pixel, FP32 FMA.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool inside(int y, int x, int H, int W)
{
    return y >= 0 && y < H && x >= 0 && x < W;
}

__global__ __launch_bounds__(BLOCK) void k_conv_first(int B, int H, int W, int d,
                                                      const bf16 *__restrict__ in,
                                                      const float *__restrict__ w0,
                                                      const float *__restrict__ bias,
                                                      bf16 *__restrict__ out)
{
    __shared__ float sw[TAPS * 2 * CH];
    __shared__ float sb[CH];
    for (int i = threadIdx.x; i < TAPS * 2 * CH; i += BLOCK) sw[i] = w0[i];
    if (threadIdx.x < CH) sb[threadIdx.x] = bias[threadIdx.x];
    __syncthreads();
    const int64_t npix = (int64_t)B * H * W;
    for (int64_t g = (int64_t)blockIdx.x * BLOCK + threadIdx.x; g < npix;
         g += (int64_t)gridDim.x * BLOCK) {
        const int64_t img = g / ((int64_t)H * W);
        const int y = (int)((g / W) % H), x = (int)(g % W);
        float acc[CH];
#pragma unroll
        for (int co = 0; co < CH; ++co) acc[co] = sb[co];
#pragma unroll 1
        for (int tap = 0; tap < TAPS; ++tap) {
            const int yy = y + (tap / 3 - 1) * d, xx = x + (tap % 3 - 1) * d;
            if (!inside(yy, xx, H, W)) continue;
            const int64_t q = (img * H + yy) * W + xx;
            const float a0 = (float)in[2 * q], a1 = (float)in[2 * q + 1];
#pragma unroll
            for (int co = 0; co < CH; ++co)
                acc[co] = fmaf(sw[(tap * 2 + 1) * CH + co], a1, fmaf(sw[(tap * 2) * CH + co], a0, acc[co]));
        }
        bf16x8 v[4];
#pragma unroll
        for (int co = 0; co < CH; ++co) v[co / 8][co % 8] = (bf16)fmaxf(acc[co], 0.f);
        bf16x8 *o = reinterpret_cast<bf16x8 *>(out + g * CH);
#pragma unroll
        for (int j = 0; j < 4; ++j) o[j] = v[j];
    }
}

__global__ __launch_bounds__(BLOCK) void k_conv_last(int B, int H, int W, int d,
                                                     const bf16 *__restrict__ in,
                                                     const float *__restrict__ w5,
                                                     const float *__restrict__ bias5,
                                                     float *__restrict__ out)
{
    __shared__ float sw[TAPS * CH];
    for (int i = threadIdx.x; i < TAPS * CH; i += BLOCK) sw[i] = w5[i];
    __syncthreads();
    const float b5 = bias5[0];
    const int64_t npix = (int64_t)B * H * W;
    for (int64_t g = (int64_t)blockIdx.x * BLOCK + threadIdx.x; g < npix;
         g += (int64_t)gridDim.x * BLOCK) {
        const int64_t img = g / ((int64_t)H * W);
        const int y = (int)((g / W) % H), x = (int)(g % W);
        float acc = b5;
        for (int tap = 0; tap < TAPS; ++tap) {
            const int yy = y + (tap / 3 - 1) * d, xx = x + (tap % 3 - 1) * d;
            if (!inside(yy, xx, H, W)) continue;
            const bf16x8 *src = reinterpret_cast<const bf16x8 *>(in + ((img * H + yy) * W + xx) * CH);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const bf16x8 v = src[j];
#pragma unroll
                for (int c = 0; c < 8; ++c) acc = fmaf(sw[tap * CH + 8 * j + c], (float)v[c], acc);
            }
        }
        out[g] = acc;
    }
}

// ---------------------------------------------------------------------------
// 32 -> 32 layers on MFMA.  MODE 0: forward (bias, ReLU).  MODE 1: backward
// data with the transposed, flipped weights, multiplied by the ReLU mask of the
// layer's input activation (mask > 0).
// One wavefront computes a 32 (channels) x 32 (pixels) tile per step.
// ---------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(BLOCK) void k_conv_mid(int B, int H, int W, int d,
                                                    const bf16 *__restrict__ in,
                                                    const bf16 *__restrict__ wt,
                                                    const float *__restrict__ bias,
                                                    const bf16 *__restrict__ mask,
                                                    bf16 *__restrict__ out)
{
    const int lane = threadIdx.x & 63, half = lane >> 5, col = lane & 31;
    // A operand of all 18 K-steps: row = lane % 32, k = 8 half + j
    bf16x8 a[18];
#pragma unroll
    for (int m = 0; m < 18; ++m) {
        const int tap = m >> 1, c0 = (m & 1) * 16 + 8 * half;
        a[m] = *reinterpret_cast<const bf16x8 *>(wt + (tap * CH + col) * CH + c0);
    }
    float bv[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) bv[r] = MODE == 0 ? bias[8 * (r / 4) + 4 * half + (r % 4)] : 0.f;

    const int64_t tiles_per_row = W / 32;
    const int64_t ntiles = (int64_t)B * H * tiles_per_row;
    // Workgroups go to the eight XCDs in turn (blockIdx.x mod 8), each XCD with
    // its own L2.  In the forward pass each XCD's workgroups take one
    // contiguous band of the tiles (whole image rows), so the rows y - d, y,
    // y + d that a tile reads are read by the tiles of that same XCD (512^2,
    // batch 8: HBM reads 318 -> 234 MB, 161.5 -> 152.8 us); the masked
    // backward pass measured 185 -> 196 us that way and keeps the plain order.
    // Which wavefront computes a tile changes nothing in its result.
    int64_t tile1 = ntiles, wave, nwaves;
    if (MODE == 0 && gridDim.x % NXCD == 0) {
        const int64_t xcd = blockIdx.x % NXCD, per = gridDim.x / NXCD;
        tile1 = ntiles * (xcd + 1) / NXCD;
        wave = ntiles * xcd / NXCD + (((int64_t)(blockIdx.x / NXCD) * BLOCK + threadIdx.x) >> 6);
        nwaves = (per * BLOCK) >> 6;
    } else {
        wave = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) >> 6;
        nwaves = ((int64_t)gridDim.x * BLOCK) >> 6;
    }
    for (int64_t tile = wave; tile < tile1; tile += nwaves) {
        const int64_t img = tile / ((int64_t)H * tiles_per_row);
        const int y = (int)((tile / tiles_per_row) % H);
        const int x = (int)(tile % tiles_per_row) * 32 + col;
        f32x16 acc = {};
#pragma unroll
        for (int m = 0; m < 18; ++m) {
            const int tap = m >> 1, c0 = (m & 1) * 16 + 8 * half;
            const int yy = y + (tap / 3 - 1) * d, xx = x + (tap % 3 - 1) * d;
            bf16x8 b;
            if (inside(yy, xx, H, W))
                b = *reinterpret_cast<const bf16x8 *>(in + ((img * H + yy) * W + xx) * CH + c0);
            else
                b = bf16x8{};
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[m], b, acc, 0, 0, 0);
        }
        const int64_t pix = (img * H + y) * W + x;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int c0 = 8 * g + 4 * half;
            typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
            bf16x4 o;
            if (MODE == 0) {
#pragma unroll
                for (int j = 0; j < 4; ++j) o[j] = (bf16)fmaxf(acc[4 * g + j] + bv[4 * g + j], 0.f);
            } else {
                const bf16x4 mk = *reinterpret_cast<const bf16x4 *>(mask + pix * CH + c0);
#pragma unroll
                for (int j = 0; j < 4; ++j) o[j] = (bf16)((float)mk[j] > 0.f ? acc[4 * g + j] : 0.f);
            }
            *reinterpret_cast<bf16x4 *>(out + pix * CH + c0) = o;
        }
    }
}

// ---------------------------------------------------------------------------
// Loss: out and target FP32; dout = 2 (out - target) / count.  The squared
// errors are summed per workgroup, then over workgroups in block order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_loss(int64_t n, const float *__restrict__ out,
                                                const float *__restrict__ target,
                                                float *__restrict__ dout, double *__restrict__ part)
{
    __shared__ double red[BLOCK / 64];
    double acc = 0.0;
    const float scale = 2.0f / (float)n;
    for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * BLOCK) {
        const float d = out[e] - target[e];
        dout[e] = scale * d;
        acc += (double)d * (double)d;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < BLOCK / 64; ++w) t += red[w];
        part[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(64) void k_loss_final(int nblocks, const double *__restrict__ part,
                                                   CnnCtl *ctl)
{
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 64) acc += part[b];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (threadIdx.x == 0) ctl->loss_sum = acc;
}

// ---------------------------------------------------------------------------
// Layer 5 backward.  Data: dZ4[p][ci] = (A5[p][ci] > 0) sum_tap w5[tap][ci]
// dout[p - off(tap)].  Weights: per-workgroup partials of
// dW5[ci][tap] = sum_p A5[p + off(tap)][ci] dout[p] and db5 = sum_p dout[p].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_last_bwd_data(int B, int H, int W, int d,
                                                         const float *__restrict__ dout,
                                                         const float *__restrict__ w5,
                                                         const bf16 *__restrict__ a5,
                                                         bf16 *__restrict__ dz)
{
    __shared__ float sw[TAPS * CH];
    for (int i = threadIdx.x; i < TAPS * CH; i += BLOCK) sw[i] = w5[i];
    __syncthreads();
    const int64_t npix = (int64_t)B * H * W;
    for (int64_t g = (int64_t)blockIdx.x * BLOCK + threadIdx.x; g < npix;
         g += (int64_t)gridDim.x * BLOCK) {
        const int64_t img = g / ((int64_t)H * W);
        const int y = (int)((g / W) % H), x = (int)(g % W);
        float acc[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) acc[c] = 0.f;
#pragma unroll 1
        for (int tap = 0; tap < TAPS; ++tap) {
            // p meets dout[p - off(tap)]
            const int yy = y - (tap / 3 - 1) * d, xx = x - (tap % 3 - 1) * d;
            if (!inside(yy, xx, H, W)) continue;
            const float d = dout[(img * H + yy) * W + xx];
#pragma unroll
            for (int c = 0; c < CH; ++c) acc[c] = fmaf(sw[tap * CH + c], d, acc[c]);
        }
        const bf16x8 *m = reinterpret_cast<const bf16x8 *>(a5 + g * CH);
        bf16x8 *o = reinterpret_cast<bf16x8 *>(dz + g * CH);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const bf16x8 mk = m[j];
            bf16x8 v;
#pragma unroll
            for (int c = 0; c < 8; ++c) v[c] = (bf16)((float)mk[c] > 0.f ? acc[8 * j + c] : 0.f);
            o[j] = v;
        }
    }
}

// Workgroup b takes a contiguous share of the pixels.  Thread (g, c4), g one
// of DW_GROUPS pixel groups and c4 one of eight channel quads, sums
// A5[p + off(tap)][4 c4 + j] dout[p] over every DW_GROUPS-th pixel of the
// share for all taps (one 8-byte load per tap gives its four channels); the
// groups are then added: the eight groups of a wavefront by a butterfly over
// the lanes (8, 16, 32 apart), the four wavefronts in order.  Partials
// part[block][289]: index ci * 9 + tap, and 288 the bias.
__global__ __launch_bounds__(256) void k_last_bwd_weight(int B, int H, int W, int d,
                                                         const float *__restrict__ dout,
                                                         const bf16 *__restrict__ a5,
                                                         float *__restrict__ part)
{
    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
    __shared__ float s_acc[4][CH * TAPS + 1];
    const int t = threadIdx.x, c4 = t % 8, g = t / 8, lane = t & 63, wave = t >> 6;
    const int64_t npix = (int64_t)B * H * W;
    const int64_t chunk = (npix + gridDim.x - 1) / gridDim.x;
    const int64_t p0 = (int64_t)blockIdx.x * chunk, p1 = min(npix, p0 + chunk);
    float acc[4][TAPS];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int k = 0; k < TAPS; ++k) acc[j][k] = 0.f;
    float bacc = 0.f;
    // the row and column of pixel p, advanced by DW_GROUPS <= W per step, and
    // the element offset of each tap from the pixel (a tap inside the image
    // lies in the pixel's own image)
    int y = (int)(((p0 + g) / W) % H), x = (int)((p0 + g) % W);
    int64_t toff[TAPS];
#pragma unroll
    for (int tap = 0; tap < TAPS; ++tap) toff[tap] = ((int64_t)(tap / 3 - 1) * d * W + (tap % 3 - 1) * d) * CH;
    for (int64_t p = p0 + g; p < p1; p += DW_GROUPS) {
        const float dv = dout[p];
        const bf16 *ap = a5 + p * CH + 4 * c4;
#pragma unroll
        for (int tap = 0; tap < TAPS; ++tap) {
            const int yy = y + (tap / 3 - 1) * d, xx = x + (tap % 3 - 1) * d;
            if (inside(yy, xx, H, W)) {
                const bf16x4 a = *reinterpret_cast<const bf16x4 *>(ap + toff[tap]);
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[j][tap] = fmaf((float)a[j], dv, acc[j][tap]);
            }
        }
        bacc += dv;
        x += DW_GROUPS;
        if (x >= W) {
            x -= W;
            if (++y == H) y = 0;   // the next image
        }
    }
    // the wavefront's eight pixel groups (lanes 8, 16, 32 apart), in a fixed order
#pragma unroll
    for (int o = 8; o < 64; o <<= 1) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int k = 0; k < TAPS; ++k) acc[j][k] += __shfl_xor(acc[j][k], o);
        bacc += __shfl_xor(bacc, o);
    }
    if (lane < 8) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int k = 0; k < TAPS; ++k) s_acc[wave][(4 * c4 + j) * TAPS + k] = acc[j][k];
        if (lane == 0) s_acc[wave][CH * TAPS] = bacc;
    }
    __syncthreads();
    for (int v = t; v <= CH * TAPS; v += 256)
        part[(size_t)blockIdx.x * (CH * TAPS + 1) + v] = ((s_acc[0][v] + s_acc[1][v]) + s_acc[2][v]) + s_acc[3][v];
}

// ---------------------------------------------------------------------------
// Weight gradient of a 32 -> 32 layer on MFMA:
//   dW[tap][co][ci] = sum_p dZ[p][co] * X[p + off(tap)][ci],  db[co] = sum_p dZ[p][co]
// A = dZ^T (rows co, k = pixels), B = shifted X (k = pixels, columns ci).  A
// workgroup stages one 32-pixel row segment of dZ and the 3 x 34 pixel halo of
// X in LDS per step; wavefront w accumulates the taps w, w+4, w+8.
// Partials part[block][tap][co][ci] and part_b[block][co].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_mid_bwd_weight(int B, int H, int W, int d,
                                                          const bf16 *__restrict__ dz,
                                                          const bf16 *__restrict__ x,
                                                          float *__restrict__ part,
                                                          float *__restrict__ part_b)
{
    __shared__ bf16 s_dz[32][CH];
    __shared__ bf16 s_x[3][32 + 2 * MAX_DIL][CH];   // rows y - d, y, y + d; columns x0 - d ..
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, half = lane >> 5, col = lane & 31;
    f32x16 acc[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) acc[i] = f32x16{};
    float bacc = 0.f;
    const int64_t tiles_per_row = W / 32;
    const int64_t ntiles = (int64_t)B * H * tiles_per_row;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t img = tile / ((int64_t)H * tiles_per_row);
        const int y = (int)((tile / tiles_per_row) % H);
        const int x0 = (int)(tile % tiles_per_row) * 32;
        __syncthreads();
        // stage dZ: 32 pixels x 32 channels = 128 vectors of 8
        if (threadIdx.x < 128) {
            const int p = threadIdx.x >> 2, c = (threadIdx.x & 3) * 8;
            *reinterpret_cast<bf16x8 *>(&s_dz[p][c]) =
                *reinterpret_cast<const bf16x8 *>(dz + ((img * H + y) * W + x0 + p) * CH + c);
        }
        // stage X halo: rows y - d, y, y + d, columns x0 - d .. x0 + 31 + d (zeros outside)
        const int cols = 32 + 2 * d;
        for (int v = threadIdx.x; v < 3 * cols * 4; v += BLOCK) {
            const int r = v / (cols * 4), pc = (v / 4) % cols, c = (v % 4) * 8;
            const int yy = y + (r - 1) * d, xx = x0 + pc - d;
            bf16x8 val = bf16x8{};
            if (inside(yy, xx, H, W))
                val = *reinterpret_cast<const bf16x8 *>(x + ((img * H + yy) * W + xx) * CH + c);
            *reinterpret_cast<bf16x8 *>(&s_x[r][pc][c]) = val;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            // A: row co = col, pixels k = 16 ks + 8 half + j
            bf16x8 a;
#pragma unroll
            for (int j = 0; j < 8; ++j) a[j] = s_dz[16 * ks + 8 * half + j][col];
            if (wave == 0) {
#pragma unroll
                for (int j = 0; j < 8; ++j) bacc += (float)a[j];
            }
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const int tap = wave + 4 * i;
                if (tap >= TAPS) break;
                const int dy = tap / 3 - 1, dx = tap % 3 - 1;
                // B: pixels k, column ci = col: X[y + dy d][x0 + k + dx d]
                bf16x8 b;
#pragma unroll
                for (int j = 0; j < 8; ++j) b[j] = s_x[1 + dy][d + 16 * ks + 8 * half + j + dx * d][col];
                acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[i], 0, 0, 0);
            }
        }
    }
    // D lane layout: column ci = col, row co = 8 (r / 4) + 4 half + r % 4
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int tap = wave + 4 * i;
        if (tap >= TAPS) break;
        float *dst = part + ((size_t)blockIdx.x * TAPS + tap) * CH * CH;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int co = 8 * (r / 4) + 4 * half + (r % 4);
            dst[co * CH + col] = acc[i][r];
        }
    }
    if (wave == 0) {
        // lanes l and l + 32 hold the two halves of channel col
        const float other = __shfl_xor(bacc, 32);
        if (half == 0) part_b[(size_t)blockIdx.x * CH + col] = bacc + other;
    }
}

// Layer 0 weight gradient, like the last layer's: thread (g, c4) sums
// in[p + off(tap)][ci] dz0[p][4 c4 + j] for both input channels (one 4-byte
// load per tap), all taps and its four output channels over every
// DW_GROUPS-th pixel of the workgroup's share; the groups are added by a
// butterfly over the lanes, then the wavefronts in order.  Partials
// part[block][608]: index (tap * 2 + ci) * 32 + co, then 576 + co the bias.
__global__ __launch_bounds__(256) void k_first_bwd_weight(int B, int H, int W, int d,
                                                          const bf16 *__restrict__ dz0,
                                                          const bf16 *__restrict__ in,
                                                          float *__restrict__ part)
{
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
    constexpr int NW = TAPS * 2 * CH;
    __shared__ float s_acc[4][NW + CH];
    const int t = threadIdx.x, c4 = t % 8, g = t / 8, lane = t & 63, wave = t >> 6;
    const int64_t npix = (int64_t)B * H * W;
    const int64_t chunk = (npix + gridDim.x - 1) / gridDim.x;
    const int64_t p0 = (int64_t)blockIdx.x * chunk, p1 = min(npix, p0 + chunk);
    float acc[4][2 * TAPS], bacc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        bacc[j] = 0.f;
#pragma unroll
        for (int k = 0; k < 2 * TAPS; ++k) acc[j][k] = 0.f;
    }
    // the row and column of pixel p, advanced by DW_GROUPS <= W per step, and
    // the element offset of each tap from the pixel (a tap inside the image
    // lies in the pixel's own image)
    int y = (int)(((p0 + g) / W) % H), x = (int)((p0 + g) % W);
    int64_t toff[TAPS];
#pragma unroll
    for (int tap = 0; tap < TAPS; ++tap) toff[tap] = ((int64_t)(tap / 3 - 1) * d * W + (tap % 3 - 1) * d) * 2;
    for (int64_t p = p0 + g; p < p1; p += DW_GROUPS) {
        const bf16x4 dz = *reinterpret_cast<const bf16x4 *>(dz0 + p * CH + 4 * c4);
        float dv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) dv[j] = (float)dz[j];
        const bf16 *ip = in + 2 * p;
#pragma unroll
        for (int tap = 0; tap < TAPS; ++tap) {
            const int yy = y + (tap / 3 - 1) * d, xx = x + (tap % 3 - 1) * d;
            if (inside(yy, xx, H, W)) {
                const bf16x2 v = *reinterpret_cast<const bf16x2 *>(ip + toff[tap]);
                const float v0 = (float)v[0], v1 = (float)v[1];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    acc[j][tap * 2] = fmaf(v0, dv[j], acc[j][tap * 2]);
                    acc[j][tap * 2 + 1] = fmaf(v1, dv[j], acc[j][tap * 2 + 1]);
                }
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) bacc[j] += dv[j];
        x += DW_GROUPS;
        if (x >= W) {
            x -= W;
            if (++y == H) y = 0;   // the next image
        }
    }
#pragma unroll
    for (int o = 8; o < 64; o <<= 1) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
#pragma unroll
            for (int k = 0; k < 2 * TAPS; ++k) acc[j][k] += __shfl_xor(acc[j][k], o);
            bacc[j] += __shfl_xor(bacc[j], o);
        }
    }
    if (lane < 8) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
#pragma unroll
            for (int k = 0; k < 2 * TAPS; ++k) s_acc[wave][k * CH + 4 * c4 + j] = acc[j][k];
            s_acc[wave][NW + 4 * c4 + j] = bacc[j];
        }
    }
    __syncthreads();
    for (int v = t; v < NW + CH; v += 256)
        part[(size_t)blockIdx.x * (NW + CH) + v] = ((s_acc[0][v] + s_acc[1][v]) + s_acc[2][v]) + s_acc[3][v];
}

// Sum per-workgroup partials into the FP32 gradient array in a fixed order:
// runs of RED_RUN blocks in sequence, then the run sums pairwise (a rounding
// chain of RED_RUN + log2(DW_BLOCKS / RED_RUN) additions).
// kind 0: middle layer (part[b][tap][co][ci], part_b[b][co]); 1: layer 0; 2: layer 5.
constexpr int RED_RUN = 32;
constexpr int RED_RUNS = DW_BLOCKS / RED_RUN;   // 32
constexpr int RED_VALS = BLOCK / RED_RUNS;      // values per reduce workgroup (8)
static_assert(RED_RUNS * RED_VALS == BLOCK && DW_BLOCKS % RED_RUN == 0, "reduce shape");

// Workgroup: RED_VALS values x RED_RUNS runs; thread (k, v) adds run k of
// value v, then one thread per value adds the runs pairwise.
__global__ __launch_bounds__(BLOCK) void k_grad_reduce(int kind, int layer, int nblocks,
                                                       const float *__restrict__ part,
                                                       const float *__restrict__ part_b,
                                                       float *__restrict__ grad)
{
    __shared__ float s_run[RED_RUNS][RED_VALS];
    const int vi = threadIdx.x % RED_VALS, k = threadIdx.x / RED_VALS;
    const int t = blockIdx.x * RED_VALS + vi;   // value index of this layer
    int nvals, stride;
    const float *src;
    int idx = t;
    if (kind == 0) {
        nvals = TAPS * CH * CH + CH;
        if (t < TAPS * CH * CH) { src = part; stride = TAPS * CH * CH; }
        else { src = part_b; stride = CH; idx = t - TAPS * CH * CH; }
    } else if (kind == 1) {
        nvals = TAPS * 2 * CH + CH; src = part; stride = nvals;
    } else {
        nvals = CH * TAPS + 1; src = part; stride = nvals;
    }
    float sacc = 0.f;
    if (t < nvals)
        for (int b = k * RED_RUN; b < min(nblocks, (k + 1) * RED_RUN); ++b)
            sacc += src[(size_t)b * stride + idx];
    s_run[k][vi] = sacc;
    __syncthreads();
    if (k != 0 || t >= nvals) return;
    float run[RED_RUNS];
#pragma unroll
    for (int j = 0; j < RED_RUNS; ++j) run[j] = s_run[j][vi];
#pragma unroll
    for (int h = RED_RUNS / 2; h > 0; h >>= 1)
#pragma unroll
        for (int j = 0; j < h; ++j) run[j] += run[j + h];
    const float sv = run[0];
    float *g = grad + param_offset(layer);
    if (kind == 0) {
        if (t < TAPS * CH * CH) {
            const int tap = t / (CH * CH), co = (t / CH) % CH, ci = t % CH;
            g[(co * CH + ci) * TAPS + tap] = sv;
        } else {
            g[CH * CH * TAPS + (t - TAPS * CH * CH)] = sv;
        }
    } else if (kind == 1) {
        const int nw = TAPS * 2 * CH;
        if (t < nw) {
            const int tap = t / (2 * CH), ci = (t / CH) % 2, co = t % CH;
            g[(co * 2 + ci) * TAPS + tap] = sv;
        } else {
            g[CH * 2 * TAPS + (t - nw)] = sv;
        }
    } else {
        const int nw = CH * TAPS;
        if (t < nw) {
            const int ci = t / TAPS, tap = t % TAPS;
            g[ci * TAPS + tap] = sv;
        } else {
            g[nw] = sv;
        }
    }
}

int reduce_grid(int nvals) { return (nvals + RED_VALS - 1) / RED_VALS; }

// Adam (Kingma and Ba) on the FP32 parameters.
__global__ __launch_bounds__(BLOCK) void k_adam(int n, float *__restrict__ p,
                                                const float *__restrict__ g, float *__restrict__ m,
                                                float *__restrict__ v, float lr, float b1, float b2,
                                                float eps, float c1, float c2)
{
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace

// ---------------------------------------------------------------------------
// Handle
// ---------------------------------------------------------------------------
struct mstab_cnn {
    int64_t H = 0, W = 0;
    int32_t max_batch = 0;
    double unit = 1.0;       // target = unit (x_next - x_prev) / s
    int dil[NL] = {1, 1, 1, 1, 1, 1};
    hipStream_t stream = nullptr;
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;   // FP32 parameters, grads, Adam
    bf16 *wf = nullptr, *wb = nullptr;
    float *w0 = nullptr, *w5 = nullptr, *bias = nullptr;
    bf16 *act[NL] = {};      // act[0] input (2 ch), act[1..5] hidden outputs (32 ch)
    float *out = nullptr, *dout = nullptr;
    bf16 *dz[NL - 1] = {};   // dz[l] = dL/dZ_l, pre-activation gradient of layer l (32 ch)
    float *part = nullptr, *part_b = nullptr;
    double *rpart = nullptr;
    CnnCtl *ctl = nullptr;
    CnnCtl *ctl_host = nullptr;
    int64_t t = 0;           // Adam step
    std::string err;
};

namespace {

thread_local std::string g_cnn_error;

#define CNNCHK(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            g_cnn_error = std::string(#call) + ": " + hipGetErrorString(e_);           \
            return e_ == hipErrorOutOfMemory ? MSTAB_E_NOMEM : MSTAB_E_HIP;            \
        }                                                                              \
    } while (0)

int grid_of(int64_t work, int cap)
{
    int64_t g = (work + BLOCK - 1) / BLOCK;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

mstab_status prep_weights(mstab_cnn *h)
{
    hipLaunchKernelGGL(k_prep_weights, dim3((4 * TAPS * CH * CH + BLOCK - 1) / BLOCK), dim3(BLOCK),
                       0, h->stream, h->p, h->wf, h->wb, h->w0, h->w5, h->bias);
    CNNCHK(hipGetLastError());
    return MSTAB_OK;
}

mstab_status run_forward(mstab_cnn *h, const bf16 *in, int B)
{
    const int H = (int)h->H, W = (int)h->W;
    const int64_t npix = (int64_t)B * H * W;
    hipLaunchKernelGGL(k_conv_first, dim3(grid_of(npix, 8192)), dim3(BLOCK), 0, h->stream, B, H, W,
                       h->dil[0], in, h->w0, h->bias, h->act[1]);
    const int64_t tiles = npix / 32;
    // a multiple of the XCD count, for the banded tile order of k_conv_mid
    const int mid_grid = (int)(((std::min<int64_t>((tiles + 3) / 4, 4096) + NXCD - 1) / NXCD) * NXCD);
    for (int l = 1; l <= 4; ++l)
        hipLaunchKernelGGL(k_conv_mid<0>, dim3(mid_grid), dim3(BLOCK), 0, h->stream, B, H, W,
                           h->dil[l], h->act[l], h->wf + (size_t)(l - 1) * TAPS * CH * CH, h->bias + l * CH,
                           (const bf16 *)nullptr, h->act[l + 1]);
    hipLaunchKernelGGL(k_conv_last, dim3(grid_of(npix, 8192)), dim3(BLOCK), 0, h->stream, B, H, W,
                       h->dil[5], h->act[5], h->w5, h->bias + 5 * CH, h->out);
    CNNCHK(hipGetLastError());
    return MSTAB_OK;
}

}  // namespace

extern "C" {

int64_t mstab_cnn_param_count(void) { return NPARAM; }

mstab_status mstab_cnn_create(int64_t H, int64_t W, int32_t max_batch, double unit,
                              const int32_t *dilation, void *hip_stream, mstab_cnn **out)
{
    if (!out) return MSTAB_E_INVALID;
    *out = nullptr;
    if (dilation) {
        for (int l = 0; l < NL; ++l)
            if (dilation[l] < 1 || dilation[l] > MAX_DIL) {
                g_cnn_error = "dilations must lie in 1..32";
                return MSTAB_E_INVALID;
            }
    }
    if (!(unit > 0.0) || !std::isfinite(unit)) {
        g_cnn_error = "unit must be positive and finite";
        return MSTAB_E_INVALID;
    }
    if (H < 1 || W < 32 || W % 32 != 0 || max_batch < 1 || H * W * (int64_t)max_batch > ((int64_t)1 << 31)) {
        g_cnn_error = "H >= 1, W a positive multiple of 32 and H*W*max_batch < 2^31 are required";
        return MSTAB_E_INVALID;
    }
    mstab_cnn *h = new mstab_cnn();
    h->H = H; h->W = W; h->max_batch = max_batch; h->unit = unit;
    if (dilation)
        for (int l = 0; l < NL; ++l) h->dil[l] = dilation[l];
    h->stream = (hipStream_t)hip_stream;
    const int64_t npix = H * W * max_batch;
    auto fail = [&](mstab_status st) { mstab_cnn_destroy(h); return st; };
#define ALLOC(ptr, bytes)                                                        \
    do {                                                                         \
        if (hipMalloc(&(ptr), (bytes)) != hipSuccess) {                          \
            g_cnn_error = "device allocation failed";                            \
            return fail(MSTAB_E_NOMEM);                                          \
        }                                                                        \
    } while (0)
    ALLOC(h->p, sizeof(float) * NPARAM);
    ALLOC(h->g, sizeof(float) * NPARAM);
    ALLOC(h->m, sizeof(float) * NPARAM);
    ALLOC(h->v, sizeof(float) * NPARAM);
    ALLOC(h->wf, sizeof(bf16) * 4 * TAPS * CH * CH);
    ALLOC(h->wb, sizeof(bf16) * 4 * TAPS * CH * CH);
    ALLOC(h->w0, sizeof(float) * TAPS * 2 * CH);
    ALLOC(h->w5, sizeof(float) * TAPS * CH);
    ALLOC(h->bias, sizeof(float) * NL * CH);
    ALLOC(h->act[0], sizeof(bf16) * 2 * npix);
    for (int l = 1; l < NL; ++l) ALLOC(h->act[l], sizeof(bf16) * CH * npix);
    ALLOC(h->out, sizeof(float) * npix);
    ALLOC(h->dout, sizeof(float) * npix);
    for (int l = 0; l < NL - 1; ++l) ALLOC(h->dz[l], sizeof(bf16) * CH * npix);
    ALLOC(h->part, sizeof(float) * (size_t)DW_BLOCKS * TAPS * CH * CH);
    ALLOC(h->part_b, sizeof(float) * (size_t)DW_BLOCKS * CH);
    ALLOC(h->rpart, sizeof(double) * LOSS_BLOCKS);
    ALLOC(h->ctl, sizeof(CnnCtl));
#undef ALLOC
    if (hipHostMalloc(&h->ctl_host, sizeof(CnnCtl), hipHostMallocDefault) != hipSuccess)
        return fail(MSTAB_E_NOMEM);
    if (hipMemsetAsync(h->ctl, 0, sizeof(CnnCtl), h->stream) != hipSuccess ||
        hipMemsetAsync(h->m, 0, sizeof(float) * NPARAM, h->stream) != hipSuccess ||
        hipMemsetAsync(h->v, 0, sizeof(float) * NPARAM, h->stream) != hipSuccess ||
        hipMemsetAsync(h->p, 0, sizeof(float) * NPARAM, h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess)
        return fail(MSTAB_E_HIP);
    *out = h;
    return MSTAB_OK;
}

mstab_status mstab_cnn_destroy(mstab_cnn *h)
{
    if (!h) return MSTAB_OK;
    (void)hipStreamSynchronize(h->stream);
    float *fl[] = {h->p, h->g, h->m, h->v, h->w0, h->w5, h->bias, h->out, h->dout, h->part, h->part_b};
    for (float *q : fl) (void)hipFree(q);
    (void)hipFree(h->wf);
    (void)hipFree(h->wb);
    for (int l = 0; l < NL; ++l) (void)hipFree(h->act[l]);
    for (int l = 0; l < NL - 1; ++l) (void)hipFree(h->dz[l]);
    (void)hipFree(h->rpart);
    (void)hipFree(h->ctl);
    if (h->ctl_host) (void)hipHostFree(h->ctl_host);
    delete h;
    return MSTAB_OK;
}

mstab_status mstab_cnn_set_params(mstab_cnn *h, const float *params_host, int64_t count)
{
    if (!h || !params_host || count != NPARAM) return MSTAB_E_INVALID;
    CNNCHK(hipMemcpyAsync(h->p, params_host, sizeof(float) * NPARAM, hipMemcpyHostToDevice, h->stream));
    CNNCHK(hipMemsetAsync(h->m, 0, sizeof(float) * NPARAM, h->stream));
    CNNCHK(hipMemsetAsync(h->v, 0, sizeof(float) * NPARAM, h->stream));
    h->t = 0;
    mstab_status st = prep_weights(h);
    if (st != MSTAB_OK) return st;
    CNNCHK(hipStreamSynchronize(h->stream));
    return MSTAB_OK;
}

mstab_status mstab_cnn_get_params(const mstab_cnn *h, float *params_host, float *grads_host,
                                  int64_t count)
{
    if (!h || count != NPARAM) return MSTAB_E_INVALID;
    if (params_host)
        CNNCHK(hipMemcpyAsync(params_host, h->p, sizeof(float) * NPARAM, hipMemcpyDeviceToHost, h->stream));
    if (grads_host)
        CNNCHK(hipMemcpyAsync(grads_host, h->g, sizeof(float) * NPARAM, hipMemcpyDeviceToHost, h->stream));
    CNNCHK(hipStreamSynchronize(h->stream));
    return MSTAB_OK;
}

mstab_status mstab_cnn_prepare(mstab_cnn *h, const double *x_prev, const double *r0,
                               const double *x_next, void *input_bf16, float *target,
                               double *scale)
{
    if (!h || !x_prev || !r0 || !input_bf16 || (target && !x_next)) return MSTAB_E_INVALID;
    const int64_t n = h->H * h->W;
    CNNCHK(hipMemsetAsync(h->ctl->absmax_bits, 0, sizeof(h->ctl->absmax_bits), h->stream));
    hipLaunchKernelGGL(k_absmax, dim3(grid_of(n, 1024)), dim3(BLOCK), 0, h->stream, n, r0, x_prev,
                       h->ctl);
    hipLaunchKernelGGL(k_prep_sample, dim3(grid_of(n, 8192)), dim3(BLOCK), 0, h->stream, n, r0,
                       x_prev, x_next, h->unit, h->ctl, (bf16 *)input_bf16, target);
    CNNCHK(hipGetLastError());
    if (scale) {
        CNNCHK(hipMemcpyAsync(h->ctl_host, h->ctl, sizeof(CnnCtl), hipMemcpyDeviceToHost, h->stream));
        CNNCHK(hipStreamSynchronize(h->stream));
        double sv;
        memcpy(&sv, &h->ctl_host->absmax_bits[0], sizeof sv);
        *scale = sv;
    }
    return MSTAB_OK;
}

mstab_status mstab_cnn_forward(mstab_cnn *h, const void *input_bf16, int32_t batch, float *out)
{
    if (!h || !input_bf16 || batch < 1 || batch > h->max_batch) return MSTAB_E_INVALID;
    mstab_status st = run_forward(h, (const bf16 *)input_bf16, batch);
    if (st != MSTAB_OK) return st;
    if (out)
        CNNCHK(hipMemcpyAsync(out, h->out, sizeof(float) * batch * h->H * h->W,
                              hipMemcpyDeviceToDevice, h->stream));
    CNNCHK(hipStreamSynchronize(h->stream));
    return MSTAB_OK;
}

mstab_status mstab_cnn_gradient(mstab_cnn *h, const void *input_bf16, const float *target,
                                int32_t batch, double *loss)
{
    if (!h || !input_bf16 || !target || batch < 1 || batch > h->max_batch) return MSTAB_E_INVALID;
    const int H = (int)h->H, W = (int)h->W, B = batch;
    const int64_t npix = (int64_t)B * H * W;
    mstab_status st = run_forward(h, (const bf16 *)input_bf16, B);
    if (st != MSTAB_OK) return st;
    const int loss_grid = grid_of(npix, LOSS_BLOCKS);
    hipLaunchKernelGGL(k_loss, dim3(loss_grid), dim3(BLOCK), 0, h->stream, npix, h->out, target,
                       h->dout, h->rpart);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, h->stream, loss_grid, h->rpart, h->ctl);
    // layer 5
    hipLaunchKernelGGL(k_last_bwd_weight, dim3(DW_BLOCKS), dim3(256), 0, h->stream, B, H, W,
                       h->dil[5], h->dout, h->act[5], h->part);
    hipLaunchKernelGGL(k_grad_reduce, dim3(reduce_grid(CH * TAPS + 1)), dim3(BLOCK), 0, h->stream, 2,
                       5, DW_BLOCKS, h->part,
                       (const float *)nullptr, h->g);
    hipLaunchKernelGGL(k_last_bwd_data, dim3(grid_of(npix, 8192)), dim3(BLOCK), 0, h->stream, B, H, W,
                       h->dil[5], h->dout, h->w5, h->act[5], h->dz[4]);
    // layers 4..1: weight gradient from dz[l], then dz[l - 1]
    const int64_t tiles = npix / 32;
    // a multiple of the XCD count, for the banded tile order of k_conv_mid
    const int mid_grid = (int)(((std::min<int64_t>((tiles + 3) / 4, 4096) + NXCD - 1) / NXCD) * NXCD);
    for (int l = 4; l >= 1; --l) {
        hipLaunchKernelGGL(k_mid_bwd_weight, dim3(DW_BLOCKS), dim3(BLOCK), 0, h->stream, B, H, W,
                           h->dil[l], h->dz[l], h->act[l], h->part, h->part_b);
        hipLaunchKernelGGL(k_grad_reduce, dim3(reduce_grid(TAPS * CH * CH + CH)), dim3(BLOCK),
                           0, h->stream, 0, l, DW_BLOCKS, h->part, h->part_b, h->g);
        hipLaunchKernelGGL(k_conv_mid<1>, dim3(mid_grid), dim3(BLOCK), 0, h->stream, B, H, W,
                           h->dil[l], h->dz[l], h->wb + (size_t)(l - 1) * TAPS * CH * CH, (const float *)nullptr,
                           h->act[l], h->dz[l - 1]);
    }
    // layer 0 (no input gradient needed)
    hipLaunchKernelGGL(k_first_bwd_weight, dim3(DW_BLOCKS), dim3(256), 0, h->stream, B, H, W,
                       h->dil[0], h->dz[0], (const bf16 *)input_bf16, h->part);
    hipLaunchKernelGGL(k_grad_reduce, dim3(reduce_grid(TAPS * 2 * CH + CH)), dim3(BLOCK), 0, h->stream,
                       1, 0, DW_BLOCKS, h->part,
                       (const float *)nullptr, h->g);
    CNNCHK(hipGetLastError());
    if (loss) {
        CNNCHK(hipMemcpyAsync(h->ctl_host, h->ctl, sizeof(CnnCtl), hipMemcpyDeviceToHost, h->stream));
        CNNCHK(hipStreamSynchronize(h->stream));
        *loss = h->ctl_host->loss_sum / (double)npix;
    } else {
        CNNCHK(hipStreamSynchronize(h->stream));
    }
    return MSTAB_OK;
}

mstab_status mstab_cnn_adam_step(mstab_cnn *h, double lr)
{
    if (!h || !(lr > 0.0)) return MSTAB_E_INVALID;
    h->t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)h->t), c2 = 1.f - powf(b2, (float)h->t);
    hipLaunchKernelGGL(k_adam, dim3((NPARAM + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, h->stream, NPARAM,
                       h->p, h->g, h->m, h->v, (float)lr, b1, b2, 1e-8f, c1, c2);
    CNNCHK(hipGetLastError());
    return prep_weights(h);
}

mstab_status mstab_cnn_guess(mstab_cnn *h, const double *x_prev, const double *r0,
                             double *x_guess)
{
    if (!h || !x_prev || !r0 || !x_guess) return MSTAB_E_INVALID;
    mstab_status st = mstab_cnn_prepare(h, x_prev, r0, nullptr, h->act[0], nullptr, nullptr);
    if (st != MSTAB_OK) return st;
    st = run_forward(h, h->act[0], 1);
    if (st != MSTAB_OK) return st;
    const int64_t n = h->H * h->W;
    hipLaunchKernelGGL(k_guess, dim3(grid_of(n, 8192)), dim3(BLOCK), 0, h->stream, n, x_prev, h->out,
                       h->unit, h->ctl, x_guess);
    CNNCHK(hipGetLastError());
    CNNCHK(hipStreamSynchronize(h->stream));
    return MSTAB_OK;
}

mstab_status mstab_cnn_tensor(const mstab_cnn *h, int32_t which, int32_t layer, void *dst,
                              int64_t bytes)
{
    if (!h || !dst) return MSTAB_E_INVALID;
    const int64_t npix = h->H * h->W * h->max_batch;
    const void *src = nullptr;
    int64_t need = 0;
    if (which == 0 && layer >= 0 && layer < NL) {
        src = h->act[layer];
        need = (int64_t)sizeof(bf16) * npix * (layer == 0 ? 2 : CH);
    } else if (which == 1) {
        src = h->out;
        need = (int64_t)sizeof(float) * npix;
    } else if (which == 2 && layer >= 0 && layer < NL - 1) {
        src = h->dz[layer];
        need = (int64_t)sizeof(bf16) * npix * CH;
    } else if (which == 3) {
        src = h->dout;
        need = (int64_t)sizeof(float) * npix;
    } else {
        return MSTAB_E_INVALID;
    }
    if (bytes < need) return MSTAB_E_INVALID;
    CNNCHK(hipMemcpyAsync(dst, src, need, hipMemcpyDeviceToDevice, h->stream));
    CNNCHK(hipStreamSynchronize(h->stream));
    return MSTAB_OK;
}

const char *mstab_cnn_last_error(void) { return g_cnn_error.c_str(); }

}  // extern "C"
