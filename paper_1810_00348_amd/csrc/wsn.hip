// Learned warm start of the DVM solver: a 3D U-Net on the matrix cores of
// gfx950.  Convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16 (BF16
// operands, FP32 accumulation); everything else (pooling, upsampling, ReLU,
// loss, Adam) is plain FP32 vector code.  C ABI: include/wsn.h.
//
// Activations are channels-last BF16 [V][stride] (V = D*H*W voxels, W
// fastest); a tensor "view" is a base pointer at its first channel plus a
// channel stride, so the skip activations are written straight into their
// slice of the decoder's concatenated input.  Gradients are FP32 with the
// same layout; the ReLU backward writes the BF16 pre-activation gradient
// that the two gradient GEMMs consume.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "wsn.h"

namespace wsn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef unsigned short bf16;

__device__ __forceinline__ bf16 f2bf(float f)
{
    // round to nearest, ties to even
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (bf16)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16 h) { return __uint_as_float(((uint32_t)h) << 16); }

__device__ __forceinline__ bf16x8 load8(const bf16* p)
{
    const uint4 u = *reinterpret_cast<const uint4*>(p);
    return __builtin_bit_cast(bf16x8, u);
}
__device__ __forceinline__ bf16x8 zero8()
{
    const uint4 u = {0u, 0u, 0u, 0u};
    return __builtin_bit_cast(bf16x8, u);
}

// tap t of a 3x3x3 stencil: (dz, dy, dx) = (t/9 - 1, (t/3)%3 - 1, t%3 - 1)
__device__ __forceinline__ void tap_offset(int taps, int t, int& dz, int& dy, int& dx)
{
    if (taps == 27) {
        dz = t / 9 - 1;
        dy = (t / 3) % 3 - 1;
        dx = t % 3 - 1;
    } else {
        dz = dy = dx = 0;
    }
}

// ---------------------------------------------------------------------------
// Convolution (forward, and input gradient with transformed weights):
//   out[v][o] = bias[o] + sum_k A[v][k] B[k][o],
//   A[v][k] = x[v + tap(k)][k mod cinp]  (zero outside the grid),
//   B[k][o] = w[tap(k)][o][k mod cinp],   k = tap * cinp + c.
// One wave computes a 16 (voxels) x 16 (output channels) tile with K in steps
// of 32; a lane supplies 8 consecutive k of one voxel row (A) / one channel
// column (B) -- 16-byte loads, since cinp is a multiple of 8.
// ---------------------------------------------------------------------------
struct ConvArgs {
    const bf16* x;
    int xs, cinp;
    const bf16* w;
    int coutp, taps;
    const float* bias;
    int D, H, W;
    float* yf;   // FP32 output or null
    int yfs;
    bf16* yb;    // BF16 output or null
    int ybs;
    int relu;
    int cout_valid;
};

// NT output-channel tiles per wave share each A fragment (one input load
// feeds NT matrix-core steps).
template <int NT>
__global__ __launch_bounds__(256) void conv_kernel(const ConvArgs A)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int V = A.D * A.H * A.W;
    const int v0 = (blockIdx.x * 4 + wv) * 16;
    if (v0 >= V) return;
    const int co0 = blockIdx.y * 16 * NT;
    const int r = lane & 15, g = lane >> 4;
    const int va = v0 + r;
    const int wa = va % A.W, ha = (va / A.W) % A.H, da = va / (A.W * A.H);
    const int K = A.taps * A.cinp;
    floatx4 acc[NT];
#pragma unroll
    for (int n = 0; n < NT; ++n) acc[n] = {0.f, 0.f, 0.f, 0.f};
    if (A.cinp % 32 == 0) {
        // every 32-wide K step lies in one tap: the tap's neighbour and
        // weight rows are set up once, the channel steps only add offsets
        for (int tap = 0; tap < A.taps; ++tap) {
            int dz, dy, dx;
            tap_offset(A.taps, tap, dz, dy, dx);
            const int zz = da + dz, yy = ha + dy, xx = wa + dx;
            const bool ok = va < V && zz >= 0 && zz < A.D && yy >= 0 && yy < A.H && xx >= 0 && xx < A.W;
            const bf16* xp = A.x + (size_t)(ok ? (zz * A.H + yy) * A.W + xx : 0) * A.xs + 8 * g;
            const bf16* wp = A.w + ((size_t)tap * A.coutp + co0 + r) * A.cinp + 8 * g;
            for (int c0 = 0; c0 < A.cinp; c0 += 32) {
                const bf16x8 a = ok ? load8(xp + c0) : zero8();
                bf16x8 b[NT];
#pragma unroll
                for (int n = 0; n < NT; ++n)
                    b[n] = co0 + 16 * n + r < A.coutp ? load8(wp + (size_t)16 * n * A.cinp + c0) : zero8();
#pragma unroll
                for (int n = 0; n < NT; ++n)
                    acc[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[n], acc[n], 0, 0, 0);
            }
        }
    } else
    for (int kb = 0; kb < K; kb += 32) {
        const int k = kb + 8 * g;
        bf16x8 a = zero8();
        bf16x8 b[NT];
#pragma unroll
        for (int n = 0; n < NT; ++n) b[n] = zero8();
        if (k < K) {
            const int tap = k / A.cinp, c0 = k - tap * A.cinp;
            int dz, dy, dx;
            tap_offset(A.taps, tap, dz, dy, dx);
            const int zz = da + dz, yy = ha + dy, xx = wa + dx;
            if (va < V && zz >= 0 && zz < A.D && yy >= 0 && yy < A.H && xx >= 0 && xx < A.W)
                a = load8(A.x + (size_t)((zz * A.H + yy) * A.W + xx) * A.xs + c0);
#pragma unroll
            for (int n = 0; n < NT; ++n) {
                const int col = co0 + 16 * n + r;
                if (col < A.coutp) b[n] = load8(A.w + ((size_t)tap * A.coutp + col) * A.cinp + c0);
            }
        }
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[n], acc[n], 0, 0, 0);
    }
    // lane holds rows 4g..4g+3 of column r of each tile
#pragma unroll
    for (int n = 0; n < NT; ++n) {
        const int c = co0 + 16 * n + r;
        if (c >= A.cout_valid) continue;
        const float bb = A.bias ? A.bias[c] : 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int v = v0 + 4 * g + i;
            if (v >= V) continue;
            float val = acc[n][i] + bb;
            if (A.relu) val = fmaxf(val, 0.f);
            if (A.yf) A.yf[(size_t)v * A.yfs + c] = val;
            if (A.yb) A.yb[(size_t)v * A.ybs + c] = f2bf(val);
        }
    }
}

// ---------------------------------------------------------------------------
// The same convolution for 3x3x3 stencils on inputs whose padded channel
// count is a multiple of 32, with the input tile in LDS.  A block computes an
// 8 (z) x 4 (y) x 4 (x) tile of voxels by 16 NT output channels; per 32
// input channels it stages the tile's 10 x 6 x 6 neighbourhood (zero outside
// the grid) and takes the A fragments of all 27 taps from there, so that an
// input value is read from memory about 2.8 times instead of 27.  Wave w
// covers z-planes 2w and 2w + 1 of the tile (16 voxels, 4 y x 4 x, each: one
// 16-row A fragment per plane, so that every B fragment feeds two steps).
// ---------------------------------------------------------------------------
constexpr int HZ = 10, HY = 6, HX = 6, HVOX = HZ * HY * HX;
constexpr int HST = 40;  // bf16 per staged voxel: 32 channels, 8 of padding (80 bytes)

template <int NT>
__global__ __launch_bounds__(256) void conv_halo_kernel(const ConvArgs A, int tx, int ty)
{
    __shared__ __align__(16) bf16 halo[HVOX * HST];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int bx = blockIdx.x % tx, by = (blockIdx.x / tx) % ty, bz = blockIdx.x / (tx * ty);
    const int x0 = bx * 4, y0 = by * 4, z0 = bz * 8;
    const int co0 = blockIdx.y * 16 * NT;
    const int r = lane & 15, g = lane >> 4;
    const int ry = r >> 2, rx = r & 3;
    floatx4 acc[2][NT];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[p][n] = {0.f, 0.f, 0.f, 0.f};
    for (int c0 = 0; c0 < A.cinp; c0 += 32) {
        // the neighbourhood, 8 channels (16 bytes) per thread and step
        for (int u = threadIdx.x; u < HVOX * 4; u += 256) {
            const int hv = u >> 2, gg = u & 3;
            const int hz = hv / (HY * HX), hy = (hv / HX) % HY, hx = hv % HX;
            const int zz = z0 - 1 + hz, yy = y0 - 1 + hy, xx = x0 - 1 + hx;
            bf16x8 val = zero8();
            if (zz >= 0 && zz < A.D && yy >= 0 && yy < A.H && xx >= 0 && xx < A.W)
                val = load8(A.x + ((size_t)(zz * A.H + yy) * A.W + xx) * A.xs + c0 + 8 * gg);
            *reinterpret_cast<bf16x8*>(&halo[hv * HST + 8 * gg]) = val;
        }
        __syncthreads();
        for (int tap = 0; tap < 27; ++tap) {
            // tap offsets (dz, dy, dx) + 1: positions in the neighbourhood
            const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
            const bf16* wp = A.w + ((size_t)tap * A.coutp + co0 + r) * A.cinp + c0 + 8 * g;
            bf16x8 b[NT];
#pragma unroll
            for (int n = 0; n < NT; ++n)
                b[n] = co0 + 16 * n + r < A.coutp ? load8(wp + (size_t)16 * n * A.cinp) : zero8();
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                const int hv = ((2 * wv + p + dz) * HY + ry + dy) * HX + rx + dx;
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(&halo[hv * HST + 8 * g]);
#pragma unroll
                for (int n = 0; n < NT; ++n)
                    acc[p][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[n], acc[p][n], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // lane holds rows 4g..4g+3 of column r of each tile: row 4g + i is the
    // tile voxel (y0 + g, x0 + i) of the plane
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const int z = z0 + 2 * wv + p, y = y0 + g;
        if (z >= A.D || y >= A.H) continue;
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            const int c = co0 + 16 * n + r;
            if (c >= A.cout_valid) continue;
            const float bb = A.bias ? A.bias[c] : 0.f;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int x = x0 + i;
                if (x >= A.W) continue;
                const size_t v = (size_t)(z * A.H + y) * A.W + x;
                float val = acc[p][n][i] + bb;
                if (A.relu) val = fmaxf(val, 0.f);
                if (A.yf) A.yf[v * A.yfs + c] = val;
                if (A.yb) A.yb[v * A.ybs + c] = f2bf(val);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Weight gradient: gw[tap][o][i] += sum_v gy[v][o] x[v + tap][i].
// GEMM with M = output channels, N = input channels, K = voxels; one wave per
// (tap, 16x16 channel tile, chunk of voxels), FP32 atomics into the flat
// (unpadded) gradient vector.
// ---------------------------------------------------------------------------
struct WgradArgs {
    const bf16* gy;
    int gys, coutp;
    const bf16* x;
    int xs, cinp;
    int taps, D, H, W;
    float* grad;   // flat: [tap][co][ci]
    int co, ci;    // valid channels
    int vchunk;
    int cotiles, citiles;
};

__global__ __launch_bounds__(64) void wgrad_kernel(const WgradArgs A)
{
    // Per step of 32 voxels the wave loads the gradient tile gy[32 v][16 o]
    // and the shifted input tile x[32 v + tap][16 i] with 16-byte loads along
    // the channels (lanes 2v and 2v+1 take the two halves of voxel v), and
    // transposes both through LDS into the MFMA's K = voxel order.
    constexpr int LS = 40;  // LDS row stride (bf16): 80-byte rows, 16-byte aligned
    __shared__ __align__(16) bf16 sa[16 * LS];
    __shared__ __align__(16) bf16 sb[16 * LS];
    const int lane = threadIdx.x;
    int t = blockIdx.x;
    const int cit = t % A.citiles;
    t /= A.citiles;
    const int cot = t % A.cotiles;
    const int tap = t / A.cotiles;
    const int V = A.D * A.H * A.W;
    const int vbeg = blockIdx.y * A.vchunk;
    const int vend = min(V, vbeg + A.vchunk);
    const int r = lane & 15, g = lane >> 4;
    const int o0 = cot * 16, i0 = cit * 16;
    const int lv = lane >> 1, hh = lane & 1;   // this lane's voxel in the step, channel half
    int dz, dy, dx;
    tap_offset(A.taps, tap, dz, dy, dx);
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int vb = vbeg; vb < vend; vb += 32) {
        const int v = vb + lv;
        uint4 ua = make_uint4(0, 0, 0, 0), ub = make_uint4(0, 0, 0, 0);
        if (v < vend) {
            if (o0 + 8 * hh < A.coutp)
                ua = *reinterpret_cast<const uint4*>(A.gy + (size_t)v * A.gys + o0 + 8 * hh);
            const int ww = v % A.W, yh = (v / A.W) % A.H, zd = v / (A.W * A.H);
            const int zz = zd + dz, yy = yh + dy, xx = ww + dx;
            if (i0 + 8 * hh < A.cinp && zz >= 0 && zz < A.D && yy >= 0 && yy < A.H && xx >= 0 && xx < A.W)
                ub = *reinterpret_cast<const uint4*>(A.x + (size_t)((zz * A.H + yy) * A.W + xx) * A.xs + i0 + 8 * hh);
        }
        bf16 ea[8], eb[8];
        __builtin_memcpy(ea, &ua, 16);
        __builtin_memcpy(eb, &ub, 16);
        __syncthreads();  // the previous step's reads are done
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            sa[(8 * hh + e) * LS + lv] = ea[e];
            sb[(8 * hh + e) * LS + lv] = eb[e];
        }
        __syncthreads();
        // lane (r, g): channel r of the tile, voxels 8g .. 8g+7 of the step
        const uint4 qa = *reinterpret_cast<const uint4*>(sa + r * LS + 8 * g);
        const uint4 qb = *reinterpret_cast<const uint4*>(sb + r * LS + 8 * g);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, qa),
                                                       __builtin_bit_cast(bf16x8, qb), acc, 0, 0, 0);
    }
    // lane holds rows (output channels) 4g..4g+3 of column (input channel) r
    const int ic = i0 + r;
    if (ic >= A.ci) return;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int oc = o0 + 4 * g + e;
        if (oc < A.co) atomicAdd(&A.grad[((size_t)tap * A.co + oc) * A.ci + ic], acc[e]);
    }
}

// bias gradient: gb[o] += sum_v gy[v][o].  The block's threads cover
// rows = 256 / gys voxels of all gys (padded) channels at a time, so that
// consecutive threads read consecutive channels of a voxel; the rows'
// partial sums are combined in LDS, one atomic per channel and block.
__global__ __launch_bounds__(256) void bgrad_kernel(const bf16* gy, int gys, int co, int V, int vchunk, float* gb)
{
    __shared__ float red[256];
    const int t = threadIdx.x;
    const int rows = 256 / gys;
    const int o = t % gys, r = t / gys;
    const int vbeg = blockIdx.x * vchunk, vend = min(V, vbeg + vchunk);
    float s = 0.f;
    if (r < rows)
        for (int v = vbeg + r; v < vend; v += rows) s += bf2f(gy[(size_t)v * gys + o]);
    red[t] = s;
    __syncthreads();
    if (r == 0 && o < co) {
        for (int k = 1; k < rows; ++k) s += red[k * gys + o];
        atomicAdd(&gb[o], s);
    }
}

// pre-activation gradient (BF16, padded channels zero): g * (act > 0) for a
// ReLU layer, g otherwise
__global__ void relu_bwd_kernel(const float* g, int gs, const bf16* act, int as, int c, int cp, int relu, int V,
                                bf16* out)
{
    const size_t n = (size_t)V * cp;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n; idx += (size_t)gridDim.x * blockDim.x) {
        const int v = (int)(idx / cp), ch = (int)(idx % cp);
        float val = 0.f;
        if (ch < c) {
            val = g[(size_t)v * gs + ch];
            if (relu && !(bf2f(act[(size_t)v * as + ch]) > 0.f)) val = 0.f;
        }
        out[idx] = f2bf(val);
    }
}

// 2x2x2 average pooling (BF16 in/out)
__global__ void pool_kernel(const bf16* x, int xs, int c, int D, int H, int W, bf16* y, int ys)
{
    const int D2 = D / 2, H2 = H / 2, W2 = W / 2;
    const size_t n = (size_t)D2 * H2 * W2 * c;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n; idx += (size_t)gridDim.x * blockDim.x) {
        const int ch = (int)(idx % c);
        const size_t v2 = idx / c;
        const int w2 = (int)(v2 % W2), h2 = (int)((v2 / W2) % H2), d2 = (int)(v2 / ((size_t)W2 * H2));
        float s = 0.f;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int e = 0; e < 2; ++e)
                    s += bf2f(x[(size_t)(((2 * d2 + a) * H + 2 * h2 + b) * W + 2 * w2 + e) * xs + ch]);
        y[v2 * ys + ch] = f2bf(0.125f * s);
    }
}

// pooling backward, accumulated: gx[child] += gy[parent] / 8
__global__ void pool_bwd_kernel(const float* gy, int gys, int c, int D, int H, int W, float* gx, int gxs)
{
    const size_t n = (size_t)D * H * W * c;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n; idx += (size_t)gridDim.x * blockDim.x) {
        const int ch = (int)(idx % c);
        const size_t v = idx / c;
        const int w = (int)(v % W), h = (int)((v / W) % H), d = (int)(v / ((size_t)W * H));
        const size_t p = ((size_t)(d / 2) * (H / 2) + h / 2) * (W / 2) + w / 2;
        gx[v * gxs + ch] += 0.125f * gy[p * gys + ch];
    }
}

// nearest x2 upsampling (BF16): y[v] = x[parent(v)]
__global__ void up_kernel(const bf16* x, int xs, int c, int D, int H, int W, bf16* y, int ys)
{
    const size_t n = (size_t)D * H * W * c;   // fine grid
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n; idx += (size_t)gridDim.x * blockDim.x) {
        const int ch = (int)(idx % c);
        const size_t v = idx / c;
        const int w = (int)(v % W), h = (int)((v / W) % H), d = (int)(v / ((size_t)W * H));
        const size_t p = ((size_t)(d / 2) * (H / 2) + h / 2) * (W / 2) + w / 2;
        y[v * ys + ch] = x[p * xs + ch];
    }
}

// upsampling backward: gx[parent] = sum over the 8 children of gy
__global__ void up_bwd_kernel(const float* gy, int gys, int c, int D, int H, int W, float* gx, int gxs)
{
    const int D2 = D / 2, H2 = H / 2, W2 = W / 2;
    const size_t n = (size_t)D2 * H2 * W2 * c;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n; idx += (size_t)gridDim.x * blockDim.x) {
        const int ch = (int)(idx % c);
        const size_t v2 = idx / c;
        const int w2 = (int)(v2 % W2), h2 = (int)((v2 / W2) % H2), d2 = (int)(v2 / ((size_t)W2 * H2));
        float s = 0.f;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int e = 0; e < 2; ++e)
                    s += gy[(size_t)(((2 * d2 + a) * H + 2 * h2 + b) * W + 2 * w2 + e) * gys + ch];
        gx[v2 * gxs + ch] = s;
    }
}

// FP32 [V][c] -> BF16 [V][cp] (padding zero)
__global__ void to_bf16_kernel(const float* x, int c, int cp, int V, bf16* y)
{
    const size_t n = (size_t)V * cp;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n; idx += (size_t)gridDim.x * blockDim.x) {
        const int ch = (int)(idx % cp);
        const size_t v = idx / cp;
        y[idx] = f2bf(ch < c ? x[v * c + ch] : 0.f);
    }
}

// masked squared error: acc[0] += mask, acc[1] += mask * sum_c (y - t)^2
__global__ void mse_sum_kernel(const float* y, const float* t, const float* mask, int c, int V, double* acc)
{
    __shared__ double red[2][256];
    double sm = 0, se = 0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < V; v += gridDim.x * blockDim.x) {
        const float m = mask[v];
        if (m == 0.f) continue;
        sm += m;
        for (int ch = 0; ch < c; ++ch) {
            const double d = (double)y[(size_t)v * c + ch] - (double)t[(size_t)v * c + ch];
            se += m * d * d;
        }
    }
    red[0][threadIdx.x] = sm;
    red[1][threadIdx.x] = se;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[0][threadIdx.x] += red[0][threadIdx.x + h];
            red[1][threadIdx.x] += red[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicAdd(&acc[0], red[0][0]);
        atomicAdd(&acc[1], red[1][0]);
    }
}

// dL/dy = weight * 2 (y - t) mask / (sum(mask) * c)
__global__ void mse_grad_kernel(const float* y, const float* t, const float* mask, int c, int V, const double* acc,
                                float weight, float* g)
{
    const double n = acc[0] * c;
    const float s = n > 0 ? (float)(2.0 * weight / n) : 0.f;
    const size_t tot = (size_t)V * c;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot; idx += (size_t)gridDim.x * blockDim.x) {
        const size_t v = idx / c;
        g[idx] = s * mask[v] * (y[idx] - t[idx]);
    }
}

__global__ void adam_kernel(float* th, float* m, float* v, const float* g, size_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// master FP32 weights of one layer -> BF16 forward form w[tap][co_p][ci_p] and
// input-gradient form wd[tap'][ci_p][co_p] = w[26 - tap'][o][i] (flipped
// stencil, channels transposed), bias -> padded FP32
__global__ void pack_kernel(const float* th, int taps, int co, int ci, int cop, int cip, bf16* w, bf16* wd, float* bias)
{
    const size_t n = (size_t)taps * cop * cip;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n; idx += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(idx % cip);
        const int o = (int)((idx / cip) % cop);
        const int t = (int)(idx / ((size_t)cip * cop));
        const float val = (o < co && i < ci) ? th[((size_t)t * co + o) * ci + i] : 0.f;
        const bf16 h = f2bf(val);
        w[idx] = h;
        const int tf = taps == 27 ? 26 - t : t;
        wd[((size_t)tf * cip + i) * cop + o] = h;
        if (t == 0 && i == 0) bias[o] = o < co ? th[(size_t)taps * co * ci + o] : 0.f;
    }
}

__global__ __launch_bounds__(64) void selftest_mfma_kernel(const bf16* a, const bf16* b, float* c)
{
    // a [16][32] row-major, b [32][16] row-major
    const int lane = threadIdx.x, r = lane & 15, g = lane >> 4;
    bf16 av[8], bv[8];
    for (int e = 0; e < 8; ++e) {
        av[e] = a[r * 32 + 8 * g + e];
        bv[e] = b[(8 * g + e) * 16 + r];
    }
    uint4 ua, ub;
    __builtin_memcpy(&ua, av, 16);
    __builtin_memcpy(&ub, bv, 16);
    const bf16x8 A = __builtin_bit_cast(bf16x8, ua);
    const bf16x8 B = __builtin_bit_cast(bf16x8, ub);
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B, acc, 0, 0, 0);
    for (int i = 0; i < 4; ++i) c[(4 * g + i) * 16 + r] = acc[i];
}

}  // namespace wsn

// ===========================================================================
// host side
// ===========================================================================
using namespace wsn;

namespace {
thread_local std::string g_err;
int wfail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}
#define WCHK(expr)                                                                          \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) return wfail(-4, "%s: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

int pad8(int c) { return (c + 7) / 8 * 8; }
unsigned nblk(size_t n) { return (unsigned)std::min<size_t>((n + 255) / 256, 65535 * 8); }

struct Layer {
    int taps, ci, co, cip, cop, relu;
    size_t woff, boff;     // offsets in the flat parameter vector
    bf16 *w, *wd;          // device BF16 weights (forward / input-gradient form)
    float* bias;           // device FP32 padded bias
};
}  // namespace

struct wsn_ctx {
    int cin, cout, base;
    int maxD, maxH, maxW;
    hipStream_t st;
    std::vector<Layer> L;
    size_t np = 0;
    float *th = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;  // master, Adam, grads
    int step = 0;
    // activations (BF16) and gradients (FP32), sized for the largest grid
    bf16 *xin, *a1, *cat1, *p1, *a3, *cat2, *p2, *a5, *a6, *a7, *a8, *a9, *a10, *gpre;
    float *y, *gy, *ga10, *ga9, *gcat1, *ga8, *ga7, *gcat2, *ga6, *ga5, *gp2, *ga3, *gp1, *ga1;
    double* acc;
    int D = 0, H = 0, W = 0;   // grid of the last forward
    std::vector<void*> allocs;
};

namespace {

template <typename T>
int dalloc(wsn_ctx* c, T** p, size_t n)
{
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T));
    if (e != hipSuccess) return wfail(-4, "hipMalloc(%zu): %s", n * sizeof(T), hipGetErrorString(e));
    c->allocs.push_back(q);
    *p = (T*)q;
    return 0;
}

int conv(wsn_ctx* c, const Layer& l, const bf16* x, int xs, int D, int H, int W, float* yf, int yfs, bf16* yb,
         int ybs, int cout_valid, bool grad_form, const bf16* wgt, int cinp, int coutp)
{
    ConvArgs a;
    a.x = x;
    a.xs = xs;
    a.cinp = cinp;
    a.w = wgt;
    a.coutp = coutp;
    a.taps = l.taps;
    a.bias = grad_form ? nullptr : l.bias;
    a.D = D;
    a.H = H;
    a.W = W;
    a.yf = yf;
    a.yfs = yfs;
    a.yb = yb;
    a.ybs = ybs;
    a.relu = grad_form ? 0 : l.relu;
    a.cout_valid = cout_valid;
    const int V = D * H * W;
    const int tiles = (coutp + 15) / 16;
    const int nt = tiles >= 4 ? 4 : tiles >= 2 ? 2 : 1;
    if (l.taps == 27 && cinp % 32 == 0) {
        const int tx = (W + 3) / 4, ty = (H + 3) / 4, tz = (D + 7) / 8;
        // fewer output-channel tiles per block on small grids, so that the
        // launch still has a few blocks per compute unit
        int nth = nt;
        while (nth > 1 && tx * ty * tz * ((tiles + nth - 1) / nth) < 512) nth /= 2;
        dim3 hgrid(tx * ty * tz, (tiles + nth - 1) / nth);
        if (nth == 4)
            conv_halo_kernel<4><<<hgrid, 256, 0, c->st>>>(a, tx, ty);
        else if (nth == 2)
            conv_halo_kernel<2><<<hgrid, 256, 0, c->st>>>(a, tx, ty);
        else
            conv_halo_kernel<1><<<hgrid, 256, 0, c->st>>>(a, tx, ty);
        WCHK(hipGetLastError());
        return 0;
    }
    dim3 grid((V / 16 + 3) / 4 + 1, (tiles + nt - 1) / nt);
    if (nt == 4)
        conv_kernel<4><<<grid, 256, 0, c->st>>>(a);
    else if (nt == 2)
        conv_kernel<2><<<grid, 256, 0, c->st>>>(a);
    else
        conv_kernel<1><<<grid, 256, 0, c->st>>>(a);
    WCHK(hipGetLastError());
    return 0;
}

int fwd_conv(wsn_ctx* c, int li, const bf16* x, int xs, int D, int H, int W, bf16* yb, int ybs)
{
    const Layer& l = c->L[li];
    return conv(c, l, x, xs, D, H, W, nullptr, 0, yb, ybs, l.co, false, l.w, l.cip, l.cop);
}

// gradients of layer li: gy (FP32 dL/d output activation) -> params, and
// (if gx) dL/d input
int bwd_conv(wsn_ctx* c, int li, const float* gy, int gys, const bf16* act, int as, const bf16* x, int xs, int D,
             int H, int W, float* gx, int gxs)
{
    const Layer& l = c->L[li];
    const int V = D * H * W;
    relu_bwd_kernel<<<nblk((size_t)V * l.cop), 256, 0, c->st>>>(gy, gys, act, as, l.co, l.cop, l.relu, V, c->gpre);
    WCHK(hipGetLastError());
    WgradArgs w;
    w.gy = c->gpre;
    w.gys = l.cop;
    w.coutp = l.cop;
    w.x = x;
    w.xs = xs;
    w.cinp = l.cip;
    w.taps = l.taps;
    w.D = D;
    w.H = H;
    w.W = W;
    w.grad = c->g + l.woff;
    w.co = l.co;
    w.ci = l.ci;
    w.vchunk = 1024;
    w.cotiles = (l.cop + 15) / 16;
    w.citiles = (l.cip + 15) / 16;
    dim3 grid(l.taps * w.cotiles * w.citiles, (V + w.vchunk - 1) / w.vchunk);
    wgrad_kernel<<<grid, 64, 0, c->st>>>(w);
    WCHK(hipGetLastError());
    bgrad_kernel<<<(V + 127) / 128, 256, 0, c->st>>>(c->gpre, l.cop, l.co, V, 128, c->g + l.boff);
    WCHK(hipGetLastError());
    if (gx) {
        // input gradient: convolution of the pre-activation gradient with the
        // flipped, transposed stencil
        int rc = conv(c, l, c->gpre, l.cop, D, H, W, gx, gxs, nullptr, 0, l.ci, true, l.wd, l.cop, l.cip);
        if (rc) return rc;
    }
    return 0;
}

int pack_all(wsn_ctx* c)
{
    for (const Layer& l : c->L) {
        pack_kernel<<<nblk((size_t)l.taps * l.cop * l.cip), 256, 0, c->st>>>(c->th + l.woff, l.taps, l.co, l.ci, l.cop,
                                                                              l.cip, l.w, l.wd, l.bias);
        WCHK(hipGetLastError());
    }
    return 0;
}

}  // namespace

extern "C" {

const char* wsn_last_error(void) { return g_err.c_str(); }

int wsn_create(int cin, int cout, int base, int max_d, int max_h, int max_w, void* hip_stream, wsn_ctx** out)
{
    if (!out) return wfail(-1, "out is NULL");
    *out = nullptr;
    if (cin < 1 || cin > 64 || cout < 1 || cout > 64 || base < 8 || base > 64 || base % 8)
        return wfail(-1, "bad channel counts (base must be a multiple of 8, at most 64)");
    if (max_d < 4 || max_h < 4 || max_w < 4 || max_d % 4 || max_h % 4 || max_w % 4)
        return wfail(-1, "grid sizes must be multiples of 4");
    wsn_ctx* c = new wsn_ctx();
    c->cin = cin;
    c->cout = cout;
    c->base = base;
    c->maxD = max_d;
    c->maxH = max_h;
    c->maxW = max_w;
    c->st = (hipStream_t)hip_stream;
    const int b1 = base, b2 = 2 * base, b3 = 4 * base;
    struct S { int taps, ci, co, relu; };
    const S spec[11] = {{27, cin, b1, 1}, {27, b1, b1, 1}, {27, b1, b2, 1}, {27, b2, b2, 1},
                        {27, b2, b3, 1},  {27, b3, b3, 1}, {27, b3 + b2, b2, 1}, {27, b2, b2, 1},
                        {27, b2 + b1, b1, 1}, {27, b1, b1, 1}, {1, b1, cout, 0}};
    size_t off = 0;
    int rc = 0;
    for (int i = 0; i < 11; ++i) {
        Layer l;
        l.taps = spec[i].taps;
        l.ci = spec[i].ci;
        l.co = spec[i].co;
        l.cip = pad8(l.ci);
        l.cop = pad8(l.co);
        l.relu = spec[i].relu;
        l.woff = off;
        off += (size_t)l.taps * l.co * l.ci;
        l.boff = off;
        off += l.co;
        rc |= dalloc(c, &l.w, (size_t)l.taps * l.cop * l.cip);
        rc |= dalloc(c, &l.wd, (size_t)l.taps * l.cop * l.cip);
        rc |= dalloc(c, &l.bias, l.cop);
        c->L.push_back(l);
    }
    c->np = off;
    rc |= dalloc(c, &c->th, off);
    rc |= dalloc(c, &c->m, off);
    rc |= dalloc(c, &c->v, off);
    rc |= dalloc(c, &c->g, off);
    const size_t V1 = (size_t)max_d * max_h * max_w, V2 = V1 / 8, V3 = V1 / 64;
    rc |= dalloc(c, &c->xin, V1 * pad8(cin));
    rc |= dalloc(c, &c->a1, V1 * b1);
    rc |= dalloc(c, &c->cat1, V1 * (b2 + b1));
    rc |= dalloc(c, &c->p1, V2 * b1);
    rc |= dalloc(c, &c->a3, V2 * b2);
    rc |= dalloc(c, &c->cat2, V2 * (b3 + b2));
    rc |= dalloc(c, &c->p2, V3 * b2);
    rc |= dalloc(c, &c->a5, V3 * b3);
    rc |= dalloc(c, &c->a6, V3 * b3);
    rc |= dalloc(c, &c->a7, V2 * b2);
    rc |= dalloc(c, &c->a8, V2 * b2);
    rc |= dalloc(c, &c->a9, V1 * b1);
    rc |= dalloc(c, &c->a10, V1 * b1);
    rc |= dalloc(c, &c->gpre, std::max(V1 * std::max(b1, pad8(cout)), std::max(V2 * b2, V3 * b3)));
    rc |= dalloc(c, &c->y, V1 * cout);
    rc |= dalloc(c, &c->gy, V1 * cout);
    rc |= dalloc(c, &c->ga10, V1 * b1);
    rc |= dalloc(c, &c->ga9, V1 * b1);
    rc |= dalloc(c, &c->gcat1, V1 * (b2 + b1));
    rc |= dalloc(c, &c->ga8, V2 * b2);
    rc |= dalloc(c, &c->ga7, V2 * b2);
    rc |= dalloc(c, &c->gcat2, V2 * (b3 + b2));
    rc |= dalloc(c, &c->ga6, V3 * b3);
    rc |= dalloc(c, &c->ga5, V3 * b3);
    rc |= dalloc(c, &c->gp2, V3 * b2);
    rc |= dalloc(c, &c->ga3, V2 * b2);
    rc |= dalloc(c, &c->gp1, V2 * b1);
    rc |= dalloc(c, &c->ga1, V1 * b1);
    rc |= dalloc(c, &c->acc, 2);
    if (rc) {
        wsn_destroy(c);
        return -4;
    }
    if (hipMemsetAsync(c->m, 0, sizeof(float) * off, c->st) != hipSuccess ||
        hipMemsetAsync(c->v, 0, sizeof(float) * off, c->st) != hipSuccess ||
        hipMemsetAsync(c->g, 0, sizeof(float) * off, c->st) != hipSuccess ||
        hipMemsetAsync(c->th, 0, sizeof(float) * off, c->st) != hipSuccess) {
        wsn_destroy(c);
        return wfail(-4, "memset failed");
    }
    *out = c;
    return 0;
}

size_t wsn_num_params(const wsn_ctx* c) { return c ? c->np : 0; }

int wsn_set_params(wsn_ctx* c, const float* p)
{
    if (!c || !p) return wfail(-1, "NULL");
    WCHK(hipMemcpyAsync(c->th, p, sizeof(float) * c->np, hipMemcpyHostToDevice, c->st));
    int rc = pack_all(c);
    if (rc) return rc;
    WCHK(hipStreamSynchronize(c->st));
    return 0;
}

int wsn_get_params(wsn_ctx* c, float* p)
{
    if (!c || !p) return wfail(-1, "NULL");
    WCHK(hipMemcpyAsync(p, c->th, sizeof(float) * c->np, hipMemcpyDeviceToHost, c->st));
    WCHK(hipStreamSynchronize(c->st));
    return 0;
}

int wsn_get_grads(wsn_ctx* c, float* p)
{
    if (!c || !p) return wfail(-1, "NULL");
    WCHK(hipMemcpyAsync(p, c->g, sizeof(float) * c->np, hipMemcpyDeviceToHost, c->st));
    WCHK(hipStreamSynchronize(c->st));
    return 0;
}

int wsn_zero_grad(wsn_ctx* c)
{
    if (!c) return wfail(-1, "NULL");
    WCHK(hipMemsetAsync(c->g, 0, sizeof(float) * c->np, c->st));
    return 0;
}

namespace {
// the forward pass; out (nullable) takes a copy of the network output
int forward_impl(wsn_ctx* c, const float* in, int D, int H, int W, float* out);
}  // namespace

int wsn_forward(wsn_ctx* c, const float* in, int D, int H, int W, float* out)
{
    if (!c || !in || !out) return wfail(-1, "NULL");
    return forward_impl(c, in, D, H, W, out);
}

namespace {
int forward_impl(wsn_ctx* c, const float* in, int D, int H, int W, float* out)
{
    if (D < 4 || H < 4 || W < 4 || D % 4 || H % 4 || W % 4 || D > c->maxD || H > c->maxH || W > c->maxW)
        return wfail(-1, "grid %dx%dx%d: must be multiples of 4 within the created maximum", D, H, W);
    c->D = D;
    c->H = H;
    c->W = W;
    const int b1 = c->base, b2 = 2 * b1, b3 = 4 * b1;
    const int V1 = D * H * W, D2 = D / 2, H2 = H / 2, W2 = W / 2, D3 = D / 4, H3 = H / 4, W3 = W / 4;
    const int c1 = b2 + b1, c2 = b3 + b2;
    int rc = 0;
    to_bf16_kernel<<<nblk((size_t)V1 * pad8(c->cin)), 256, 0, c->st>>>(in, c->cin, pad8(c->cin), V1, c->xin);
    WCHK(hipGetLastError());
    rc |= fwd_conv(c, 0, c->xin, pad8(c->cin), D, H, W, c->a1, b1);
    rc |= fwd_conv(c, 1, c->a1, b1, D, H, W, c->cat1 + b2, c1);          // s1 -> skip slice
    pool_kernel<<<nblk((size_t)V1 / 8 * b1), 256, 0, c->st>>>(c->cat1 + b2, c1, b1, D, H, W, c->p1, b1);
    rc |= fwd_conv(c, 2, c->p1, b1, D2, H2, W2, c->a3, b2);
    rc |= fwd_conv(c, 3, c->a3, b2, D2, H2, W2, c->cat2 + b3, c2);        // s2 -> skip slice
    pool_kernel<<<nblk((size_t)V1 / 64 * b2), 256, 0, c->st>>>(c->cat2 + b3, c2, b2, D2, H2, W2, c->p2, b2);
    rc |= fwd_conv(c, 4, c->p2, b2, D3, H3, W3, c->a5, b3);
    rc |= fwd_conv(c, 5, c->a5, b3, D3, H3, W3, c->a6, b3);
    up_kernel<<<nblk((size_t)V1 / 8 * b3), 256, 0, c->st>>>(c->a6, b3, b3, D2, H2, W2, c->cat2, c2);
    rc |= fwd_conv(c, 6, c->cat2, c2, D2, H2, W2, c->a7, b2);
    rc |= fwd_conv(c, 7, c->a7, b2, D2, H2, W2, c->a8, b2);
    up_kernel<<<nblk((size_t)V1 * b2), 256, 0, c->st>>>(c->a8, b2, b2, D, H, W, c->cat1, c1);
    rc |= fwd_conv(c, 8, c->cat1, c1, D, H, W, c->a9, b1);
    rc |= fwd_conv(c, 9, c->a9, b1, D, H, W, c->a10, b1);
    const Layer& lo = c->L[10];
    rc |= conv(c, lo, c->a10, b1, D, H, W, c->y, c->cout, nullptr, 0, c->cout, false, lo.w, lo.cip, lo.cop);
    if (rc) return rc;
    WCHK(hipGetLastError());
    if (out) WCHK(hipMemcpyAsync(out, c->y, sizeof(float) * V1 * c->cout, hipMemcpyDeviceToDevice, c->st));
    return 0;
}
}  // namespace

int wsn_backward_mse(wsn_ctx* c, const float* target, const float* mask, float weight, double* host_loss)
{
    if (!c || !target || !mask) return wfail(-1, "NULL");
    if (!c->D) return wfail(-1, "no forward pass yet");
    const int D = c->D, H = c->H, W = c->W;
    const int b1 = c->base, b2 = 2 * b1, b3 = 4 * b1;
    const int V1 = D * H * W, D2 = D / 2, H2 = H / 2, W2 = W / 2, D3 = D / 4, H3 = H / 4, W3 = W / 4;
    const int c1 = b2 + b1, c2 = b3 + b2;
    int rc = 0;
    WCHK(hipMemsetAsync(c->acc, 0, 2 * sizeof(double), c->st));
    mse_sum_kernel<<<256, 256, 0, c->st>>>(c->y, target, mask, c->cout, V1, c->acc);
    mse_grad_kernel<<<nblk((size_t)V1 * c->cout), 256, 0, c->st>>>(c->y, target, mask, c->cout, V1, c->acc, weight,
                                                                    c->gy);
    WCHK(hipGetLastError());
    // decoder, level 1
    rc |= bwd_conv(c, 10, c->gy, c->cout, nullptr, 0, c->a10, b1, D, H, W, c->ga10, b1);
    rc |= bwd_conv(c, 9, c->ga10, b1, c->a10, b1, c->a9, b1, D, H, W, c->ga9, b1);
    rc |= bwd_conv(c, 8, c->ga9, b1, c->a9, b1, c->cat1, c1, D, H, W, c->gcat1, c1);
    up_bwd_kernel<<<nblk((size_t)V1 / 8 * b2), 256, 0, c->st>>>(c->gcat1, c1, b2, D, H, W, c->ga8, b2);
    // decoder, level 2
    rc |= bwd_conv(c, 7, c->ga8, b2, c->a8, b2, c->a7, b2, D2, H2, W2, c->ga7, b2);
    rc |= bwd_conv(c, 6, c->ga7, b2, c->a7, b2, c->cat2, c2, D2, H2, W2, c->gcat2, c2);
    up_bwd_kernel<<<nblk((size_t)V1 / 64 * b3), 256, 0, c->st>>>(c->gcat2, c2, b3, D2, H2, W2, c->ga6, b3);
    // bottleneck
    rc |= bwd_conv(c, 5, c->ga6, b3, c->a6, b3, c->a5, b3, D3, H3, W3, c->ga5, b3);
    rc |= bwd_conv(c, 4, c->ga5, b3, c->a5, b3, c->p2, b2, D3, H3, W3, c->gp2, b2);
    // encoder, level 2: skip gradient += pooling backward
    pool_bwd_kernel<<<nblk((size_t)V1 / 8 * b2), 256, 0, c->st>>>(c->gp2, b2, b2, D2, H2, W2, c->gcat2 + b3, c2);
    rc |= bwd_conv(c, 3, c->gcat2 + b3, c2, c->cat2 + b3, c2, c->a3, b2, D2, H2, W2, c->ga3, b2);
    rc |= bwd_conv(c, 2, c->ga3, b2, c->a3, b2, c->p1, b1, D2, H2, W2, c->gp1, b1);
    // encoder, level 1
    pool_bwd_kernel<<<nblk((size_t)V1 * b1), 256, 0, c->st>>>(c->gp1, b1, b1, D, H, W, c->gcat1 + b2, c1);
    rc |= bwd_conv(c, 1, c->gcat1 + b2, c1, c->cat1 + b2, c1, c->a1, b1, D, H, W, c->ga1, b1);
    rc |= bwd_conv(c, 0, c->ga1, b1, c->a1, b1, c->xin, pad8(c->cin), D, H, W, nullptr, 0);
    if (rc) return rc;
    WCHK(hipGetLastError());
    if (host_loss) {
        double h[2];
        WCHK(hipMemcpyAsync(h, c->acc, sizeof h, hipMemcpyDeviceToHost, c->st));
        WCHK(hipStreamSynchronize(c->st));
        *host_loss += h[0] > 0 ? weight * h[1] / (h[0] * c->cout) : 0.0;
    }
    return 0;
}

int wsn_adam_step(wsn_ctx* c, float lr, float b1, float b2, float eps)
{
    if (!c) return wfail(-1, "NULL");
    c->step++;
    const float c1 = 1.f - powf(b1, (float)c->step), c2 = 1.f - powf(b2, (float)c->step);
    adam_kernel<<<nblk(c->np), 256, 0, c->st>>>(c->th, c->m, c->v, c->g, c->np, lr, b1, b2, eps, c1, c2);
    WCHK(hipGetLastError());
    return pack_all(c);
}

int wsn_train_step(wsn_ctx* c, int n, const float* const* inputs, const float* const* targets,
                   const float* const* masks, const int* dims, float lr, double* host_loss)
{
    if (!c || n < 1 || !inputs || !targets || !masks || !dims) return wfail(-1, "NULL or empty batch");
    for (int i = 0; i < n; ++i)
        if (!inputs[i] || !targets[i] || !masks[i]) return wfail(-1, "batch item %d: NULL array", i);
    int rc = wsn_zero_grad(c);
    if (rc) return rc;
    double loss = 0.0;
    for (int i = 0; i < n; ++i) {
        rc = forward_impl(c, inputs[i], dims[3 * i], dims[3 * i + 1], dims[3 * i + 2], nullptr);
        if (rc) return rc;
        rc = wsn_backward_mse(c, targets[i], masks[i], 1.0f / (float)n, &loss);
        if (rc) return rc;
    }
    rc = wsn_adam_step(c, lr, 0.9f, 0.999f, 1e-8f);
    if (rc) return rc;
    if (host_loss) *host_loss = loss;
    return 0;
}

namespace {
constexpr char kWsnMagic[8] = {'W', 'S', 'N', 'E', 'T', '0', '0', '1'};
}

int wsn_save(wsn_ctx* c, const char* path)
{
    if (!c || !path) return wfail(-1, "NULL");
    std::vector<float> buf(3 * c->np);
    WCHK(hipMemcpyAsync(buf.data(), c->th, sizeof(float) * c->np, hipMemcpyDeviceToHost, c->st));
    WCHK(hipMemcpyAsync(buf.data() + c->np, c->m, sizeof(float) * c->np, hipMemcpyDeviceToHost, c->st));
    WCHK(hipMemcpyAsync(buf.data() + 2 * c->np, c->v, sizeof(float) * c->np, hipMemcpyDeviceToHost, c->st));
    WCHK(hipStreamSynchronize(c->st));
    FILE* f = fopen(path, "wb");
    if (!f) return wfail(-1, "cannot open %s for writing", path);
    const int32_t hdr[4] = {c->cin, c->cout, c->base, c->step};
    const uint64_t np = c->np;
    bool ok = fwrite(kWsnMagic, 1, 8, f) == 8 && fwrite(hdr, sizeof hdr, 1, f) == 1 &&
              fwrite(&np, sizeof np, 1, f) == 1 && fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    ok = (fclose(f) == 0) && ok;
    if (!ok) return wfail(-1, "writing %s failed", path);
    return 0;
}

int wsn_load(wsn_ctx* c, const char* path)
{
    if (!c || !path) return wfail(-1, "NULL");
    FILE* f = fopen(path, "rb");
    if (!f) return wfail(-1, "cannot open %s", path);
    char magic[8];
    int32_t hdr[4];
    uint64_t np = 0;
    std::vector<float> buf(3 * c->np);
    bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, kWsnMagic, 8) == 0 && fread(hdr, sizeof hdr, 1, f) == 1 &&
              fread(&np, sizeof np, 1, f) == 1;
    if (ok && (hdr[0] != c->cin || hdr[1] != c->cout || hdr[2] != c->base || np != c->np)) {
        fclose(f);
        return wfail(-1, "%s holds a network (cin %d, cout %d, base %d, %llu parameters) of another shape", path,
                     hdr[0], hdr[1], hdr[2], (unsigned long long)np);
    }
    ok = ok && fread(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    fclose(f);
    if (!ok) return wfail(-1, "%s is not a complete network file", path);
    WCHK(hipMemcpyAsync(c->m, buf.data() + c->np, sizeof(float) * c->np, hipMemcpyHostToDevice, c->st));
    WCHK(hipMemcpyAsync(c->v, buf.data() + 2 * c->np, sizeof(float) * c->np, hipMemcpyHostToDevice, c->st));
    c->step = hdr[3];
    return wsn_set_params(c, buf.data());
}

int wsn_test_conv(int D, int H, int W, int ci, int co, int taps, const float* x, const float* w, const float* b,
                  const float* gy, float* y, float* gx, float* gw, float* gb)
{
    if (D < 1 || H < 1 || W < 1 || ci < 1 || co < 1 || (taps != 1 && taps != 27) || !x || !w)
        return wfail(-1, "bad arguments");
    wsn_ctx tmp;
    tmp.st = nullptr;
    Layer l;
    l.taps = taps;
    l.ci = ci;
    l.co = co;
    l.cip = pad8(ci);
    l.cop = pad8(co);
    l.relu = 0;
    l.woff = 0;
    l.boff = (size_t)taps * co * ci;
    tmp.L.push_back(l);
    const size_t V = (size_t)D * H * W, np = l.boff + co;
    std::vector<float> th(np, 0.f);
    memcpy(th.data(), w, sizeof(float) * taps * co * ci);
    if (b) memcpy(th.data() + l.boff, b, sizeof(float) * co);
    float *dth, *dy, *dgy, *dgx;
    bf16* dx;
    int rc = 0;
    rc |= dalloc(&tmp, &l.w, (size_t)taps * l.cop * l.cip);
    rc |= dalloc(&tmp, &l.wd, (size_t)taps * l.cop * l.cip);
    rc |= dalloc(&tmp, &l.bias, l.cop);
    rc |= dalloc(&tmp, &dth, np);
    rc |= dalloc(&tmp, &dx, V * l.cip);
    rc |= dalloc(&tmp, &dy, V * co);
    rc |= dalloc(&tmp, &dgy, V * co);
    rc |= dalloc(&tmp, &dgx, V * ci);
    rc |= dalloc(&tmp, &tmp.g, np);
    rc |= dalloc(&tmp, &tmp.gpre, V * l.cop);
    float* dxf;
    rc |= dalloc(&tmp, &dxf, V * ci);
    tmp.L[0] = l;
    auto cleanup = [&]() {
        for (void* p : tmp.allocs) (void)hipFree(p);
        tmp.allocs.clear();
    };
    if (rc) {
        cleanup();
        return -4;
    }
#define TCHK(expr)                                                                               \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess) {                                                                  \
            cleanup();                                                                           \
            return wfail(-4, "%s: %s", #expr, hipGetErrorString(e_));                           \
        }                                                                                        \
    } while (0)
    TCHK(hipMemcpy(dth, th.data(), sizeof(float) * np, hipMemcpyHostToDevice));
    TCHK(hipMemcpy(dxf, x, sizeof(float) * V * ci, hipMemcpyHostToDevice));
    TCHK(hipMemset(tmp.g, 0, sizeof(float) * np));
    pack_kernel<<<nblk((size_t)taps * l.cop * l.cip), 256>>>(dth, taps, co, ci, l.cop, l.cip, l.w, l.wd, l.bias);
    to_bf16_kernel<<<nblk(V * l.cip), 256>>>(dxf, ci, l.cip, (int)V, dx);
    TCHK(hipGetLastError());
    if (y) {
        if (conv(&tmp, l, dx, l.cip, D, H, W, dy, co, nullptr, 0, co, false, l.w, l.cip, l.cop)) {
            cleanup();
            return -4;
        }
        TCHK(hipMemcpy(y, dy, sizeof(float) * V * co, hipMemcpyDeviceToHost));
    }
    if (gy) {
        TCHK(hipMemcpy(dgy, gy, sizeof(float) * V * co, hipMemcpyHostToDevice));
        if (bwd_conv(&tmp, 0, dgy, co, nullptr, 0, dx, l.cip, D, H, W, gx ? dgx : nullptr, ci) != 0) {
            cleanup();
            return -4;
        }
        (void)0;
    }
    TCHK(hipDeviceSynchronize());
    if (gy) {
        std::vector<float> g(np);
        TCHK(hipMemcpy(g.data(), tmp.g, sizeof(float) * np, hipMemcpyDeviceToHost));
        if (gw) memcpy(gw, g.data(), sizeof(float) * taps * co * ci);
        if (gb) memcpy(gb, g.data() + l.boff, sizeof(float) * co);
        if (gx) TCHK(hipMemcpy(gx, dgx, sizeof(float) * V * ci, hipMemcpyDeviceToHost));
    }
    cleanup();
    return 0;
#undef TCHK
}

int wsn_selftest_mfma(const float* a, const float* b, float* c)
{
    if (!a || !b || !c) return wfail(-1, "NULL");
    std::vector<bf16> ha(16 * 32), hb(32 * 16);
    auto tobf = [](float f) {
        uint32_t u;
        memcpy(&u, &f, 4);
        u += 0x7FFFu + ((u >> 16) & 1u);
        return (bf16)(u >> 16);
    };
    for (int i = 0; i < 16 * 32; ++i) ha[i] = tobf(a[i]);
    for (int i = 0; i < 32 * 16; ++i) hb[i] = tobf(b[i]);
    bf16 *da, *db;
    float* dc;
    WCHK(hipMalloc(&da, sizeof(bf16) * 512));
    WCHK(hipMalloc(&db, sizeof(bf16) * 512));
    WCHK(hipMalloc(&dc, sizeof(float) * 256));
    WCHK(hipMemcpy(da, ha.data(), sizeof(bf16) * 512, hipMemcpyHostToDevice));
    WCHK(hipMemcpy(db, hb.data(), sizeof(bf16) * 512, hipMemcpyHostToDevice));
    selftest_mfma_kernel<<<1, 64>>>(da, db, dc);
    WCHK(hipGetLastError());
    WCHK(hipDeviceSynchronize());
    WCHK(hipMemcpy(c, dc, sizeof(float) * 256, hipMemcpyDeviceToHost));
    WCHK(hipFree(da));
    WCHK(hipFree(db));
    WCHK(hipFree(dc));
    return 0;
}

void wsn_destroy(wsn_ctx* c)
{
    if (!c) return;
    for (void* p : c->allocs) (void)hipFree(p);
    delete c;
}

}  // extern "C"
