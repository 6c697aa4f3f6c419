// surrogate.hip -- training and inference kernels of the occupancy surrogate
// (include/kl_surrogate.h): a BF16 matrix-core GEMM with FP32 accumulation,
// the column forms of the transposed convolutions (col2im / im2col), and
// the loss, optimiser, gate and IoU kernels, with their host orchestration.
//
// Activations are stored pixel-major: a layer with C channels on an H x W
// grid for B sets is a (B*H*W) x C row-major matrix, so a transposed
// convolution is one GEMM into "columns" Col = X K (K read as
// Cin x (Cout*4*4)) followed by a gather that sums, for every output pixel,
// the column entries of the input pixels that reach it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "kl_internal.hpp"
#include "kl_surrogate.h"

namespace kl {
namespace sur {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kImg = KL_SUR_IMG;

// parameter layout (offsets in floats)
struct Layout {
    size_t W1, b1, W2, b2, K1, c1, K2, c2, K3, c3, K4, c4, total;
};
static Layout layout() {
    Layout L;
    size_t o = 0;
    L.W1 = o; o += 4 * 256;
    L.b1 = o; o += 256;
    L.W2 = o; o += 256 * 256;
    L.b2 = o; o += 256;
    L.K1 = o; o += 16 * 64 * 16;
    L.c1 = o; o += 64;
    L.K2 = o; o += 64 * 32 * 16;
    L.c2 = o; o += 32;
    L.K3 = o; o += 32 * 16 * 16;
    L.c3 = o; o += 16;
    L.K4 = o; o += 16 * 1 * 16;
    L.c4 = o; o += 1;
    L.total = o;
    return L;
}

// ------------------------------------------------------------------ GEMM
// FP32 -> bfloat16, round to nearest even
__device__ __forceinline__ unsigned short to_bf16(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

// the value of x rounded to bfloat16, as FP32
__device__ __forceinline__ float bf16_value(float x) { return __uint_as_float((uint32_t)to_bf16(x) << 16); }

struct GemmArgs {
    int M, N, K;
    const float* A;
    int64_t lam, lak;
    const float* B;
    int64_t lbk, lbn;
    float* C;
    int64_t ldc;
    const float* bias;
    int relu, accumulate, ksplit, kchunk;
};

constexpr int kTM = 64, kTN = 64, kTK = 32, kPad = 8;

// 256 threads: 4 waves in a 2 x 2 arrangement of 32 x 32 wave tiles, each
// 2 x 2 MFMA 16x16x16 tiles.  A and B tiles are staged in LDS as bfloat16
// (B transposed, so both fragments are 4 consecutive k of one row).
// With ksplit > 1 each z-slice of the grid sums one chunk of K and adds it
// to C atomically.
__global__ __launch_bounds__(256) void gemm_bf16_kernel(const GemmArgs g) {
    __shared__ unsigned short As[kTM][kTK + kPad];
    __shared__ unsigned short Bs[kTN][kTK + kPad];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int bm = blockIdx.y * kTM, bn = blockIdx.x * kTN;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int kbeg = blockIdx.z * g.kchunk;
    const int kend = std::min(g.K, kbeg + g.kchunk);
    f32x4 acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = kbeg; k0 < kend; k0 += kTK) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = tid * 8 + u;
            const int r = e / kTK, k = e % kTK;   // A tile: 64 rows x 32 k
            const int gi = bm + r, gk = k0 + k;
            float va = 0.f;
            if (gi < g.M && gk < kend) va = g.A[(int64_t)gi * g.lam + (int64_t)gk * g.lak];
            As[r][k] = to_bf16(va);
            const int kb = e / kTN, c = e % kTN;  // B tile: 32 k x 64 cols
            const int gj = bn + c, gkb = k0 + kb;
            float vb = 0.f;
            if (gj < g.N && gkb < kend) vb = g.B[(int64_t)gkb * g.lbk + (int64_t)gj * g.lbn];
            Bs[c][kb] = to_bf16(vb);
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kTK; ks += 16) {
            bf16x4 af[2], bfr[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const unsigned short* pa = &As[wm + t * 16 + (lane & 15)][ks + 4 * (lane >> 4)];
                const unsigned short* pb = &Bs[wn + t * 16 + (lane & 15)][ks + 4 * (lane >> 4)];
                af[t] = bf16x4{(short)pa[0], (short)pa[1], (short)pa[2], (short)pa[3]};
                bfr[t] = bf16x4{(short)pb[0], (short)pb[1], (short)pb[2], (short)pb[3]};
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[a], bfr[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
    // D(i, j): lane holds column (lane & 15), rows 4 * (lane >> 4) + v
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = bm + wm + a * 16 + 4 * (lane >> 4) + v;
                const int j = bn + wn + b * 16 + (lane & 15);
                if (i >= g.M || j >= g.N) continue;
                float x = acc[a][b][v];
                float* dst = g.C + (int64_t)i * g.ldc + j;
                if (g.ksplit > 1) {
                    atomicAdd(dst, x);
                } else if (g.accumulate) {
                    *dst += x;
                } else {
                    if (g.bias) x += g.bias[j];
                    if (g.relu) x = fmaxf(x, 0.f);
                    *dst = x;
                }
            }
}

__global__ void zero_rows_kernel(float* C, int M, int N, int64_t ldc) {
    const int64_t n = (int64_t)M * N;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        C[(e / N) * ldc + (e % N)] = 0.f;
}

static hipError_t gemm(int M, int N, int K, const float* A, int64_t lam, int64_t lak, const float* B, int64_t lbk,
                       int64_t lbn, float* C, int64_t ldc, const float* bias, int relu, int accumulate,
                       hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    GemmArgs g{M, N, K, A, lam, lak, B, lbk, lbn, C, ldc, bias, relu, accumulate, 1, 0};
    const int tiles = ((M + kTM - 1) / kTM) * ((N + kTN - 1) / kTN);
    int ksplit = 1;
    // few output tiles and a long K: spread K over more workgroups
    if (!bias && !relu && tiles < 512 && K > 4 * kTK) {
        ksplit = std::min((K + 4 * kTK - 1) / (4 * kTK), std::max(1, 1024 / tiles));
    }
    int chunk = (K + ksplit - 1) / ksplit;
    chunk = ((chunk + kTK - 1) / kTK) * kTK;
    if (chunk < kTK) chunk = kTK;
    ksplit = std::max(1, (K + chunk - 1) / chunk);
    g.ksplit = ksplit;
    g.kchunk = K > 0 ? chunk : kTK;
    if (ksplit > 1 && !accumulate) {
        hipLaunchKernelGGL(zero_rows_kernel, dim3(std::min<int64_t>(4096, ((int64_t)M * N + 255) / 256)), dim3(256),
                           0, s, C, M, N, ldc);
    }
    if (K <= 0) return hipGetLastError();
    dim3 grid((N + kTN - 1) / kTN, (M + kTM - 1) / kTM, ksplit);
    hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

// ------------------------------------------------------------------ layer glue
__global__ void features_kernel(const kl_c64* ta, const kl_c64* tb, int B, float* u) {
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += gridDim.x * blockDim.x) {
        u[4 * b + 0] = (float)((ta[b].re - 2.4) / 0.6);
        u[4 * b + 1] = (float)(ta[b].im / 0.3);
        u[4 * b + 2] = (float)((tb[b].re - 2.4) / 0.6);
        u[4 * b + 3] = (float)(tb[b].im / 0.3);
    }
}

// h2 (B x 256, feature c*16 + q) <-> x0 ((B*16) x 16, row b*16 + q, column c)
__global__ void h2_to_x0_kernel(const float* h2, float* x0, int B) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < B * 256; e += gridDim.x * blockDim.x) {
        const int b = e / 256, f = e % 256, c = f / 16, q = f % 16;
        x0[(b * 16 + q) * 16 + c] = h2[e];
    }
}
__global__ void x0_to_h2_kernel(const float* x0, float* h2, int B) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < B * 256; e += gridDim.x * blockDim.x) {
        const int b = e / 256, f = e % 256, c = f / 16, q = f % 16;
        h2[e] = x0[(b * 16 + q) * 16 + c];
    }
}

struct ConvShape {
    int Hin, Hout, Co, s, p;  // square grids, 4 x 4 kernel
};

// Y[(b, oy, ox), o] = bias[o] + sum over taps (ky, kx) with oy = s*iy - p + ky,
// ox = s*ix - p + kx of Col[(b, iy, ix), o*16 + ky*4 + kx]; optional relu.
__global__ void col2im_kernel(const float* __restrict__ col, const float* __restrict__ bias, float* __restrict__ y,
                              int B, ConvShape c, int relu) {
    const int64_t n = (int64_t)B * c.Hout * c.Hout * c.Co;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int o = (int)(e % c.Co);
    int64_t t = e / c.Co;
    const int ox = (int)(t % c.Hout);
    t /= c.Hout;
    const int oy = (int)(t % c.Hout);
    const int b = (int)(t / c.Hout);
    float sum = 0.f;
    for (int ky = 0; ky < 4; ++ky) {
        const int ty = oy + c.p - ky;
        if (ty < 0 || ty % c.s) continue;
        const int iy = ty / c.s;
        if (iy >= c.Hin) continue;
        for (int kx = 0; kx < 4; ++kx) {
            const int tx = ox + c.p - kx;
            if (tx < 0 || tx % c.s) continue;
            const int ix = tx / c.s;
            if (ix >= c.Hin) continue;
            sum += col[(((int64_t)b * c.Hin + iy) * c.Hin + ix) * (c.Co * 16) + o * 16 + ky * 4 + kx];
        }
    }
    sum += bias[o];
    y[e] = relu ? fmaxf(sum, 0.f) : sum;
    }
}

// dCol[(b, iy, ix), o*16 + ky*4 + kx] = dY[(b, s*iy - p + ky, s*ix - p + kx), o], 0 outside
__global__ void im2col_kernel(const float* __restrict__ dy, float* __restrict__ dcol, int B, ConvShape c) {
    const int64_t n = (int64_t)B * c.Hin * c.Hin * c.Co * 16;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int tap = (int)(e % 16);
    const int o = (int)((e / 16) % c.Co);
    int64_t t = e / (16 * c.Co);
    const int ix = (int)(t % c.Hin);
    t /= c.Hin;
    const int iy = (int)(t % c.Hin);
    const int b = (int)(t / c.Hin);
    const int oy = c.s * iy - c.p + tap / 4, ox = c.s * ix - c.p + tap % 4;
    float v = 0.f;
    if (oy >= 0 && oy < c.Hout && ox >= 0 && ox < c.Hout)
        v = dy[(((int64_t)b * c.Hout + oy) * c.Hout + ox) * c.Co + o];
    dcol[e] = v;
    }
}

__global__ void relu_mask_kernel(float* d, const float* y, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        if (!(y[e] > 0.f)) d[e] = 0.f;
}

// Column sums of an M x C row-major matrix (C divides 256), two stages, fixed order.
__global__ void colsum_stage1(const float* __restrict__ x, int64_t M, int C, int64_t rows_per_block,
                              float* __restrict__ partial) {
    __shared__ float red[256];
    const int c = threadIdx.x % C, j = threadIdx.x / C, S = 256 / C;
    const int64_t r0 = blockIdx.x * rows_per_block;
    const int64_t r1 = std::min(M, r0 + rows_per_block);
    float acc = 0.f;
    for (int64_t r = r0 + j; r < r1; r += S) acc += x[r * C + c];
    red[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < C) {
        float sum = 0.f;
        for (int q = 0; q < S; ++q) sum += red[q * C + threadIdx.x];
        partial[(int64_t)blockIdx.x * C + threadIdx.x] = sum;
    }
}
// one workgroup per column: strided partial sums, then a fixed tree
__global__ void colsum_stage2(const float* __restrict__ partial, int blocks, int C, float* __restrict__ out,
                              int accumulate) {
    __shared__ float red[256];
    const int c = blockIdx.x;
    float sum = 0.f;
    for (int b = threadIdx.x; b < blocks; b += 256) sum += partial[(int64_t)b * C + c];
    red[threadIdx.x] = sum;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = accumulate ? out[c] + red[0] : red[0];
}

static hipError_t colsum(const float* x, int64_t M, int C, float* out, float* partial, hipStream_t s) {
    int blocks = (int)std::min<int64_t>(1024, (M + 255) / 256);
    if (blocks < 1) blocks = 1;
    const int64_t rpb = (M + blocks - 1) / blocks;
    hipLaunchKernelGGL(colsum_stage1, dim3(blocks), dim3(256), 0, s, x, M, C, rpb, partial);
    hipLaunchKernelGGL(colsum_stage2, dim3(C), dim3(256), 0, s, partial, blocks, C, out, 0);
    return hipGetLastError();
}

// BCE with logits: loss terms (summed in two fixed-order stages) and dz = (sigmoid(z) - t) / n
__global__ void bce_kernel(const float* __restrict__ z, const uint8_t* __restrict__ t, int64_t n,
                           float* __restrict__ dz, float* __restrict__ partial) {
    __shared__ float red[256];
    float acc = 0.f;
    const float inv = 1.0f / (float)n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const float x = z[e], y = t[e] ? 1.f : 0.f;
        acc += fmaxf(x, 0.f) - x * y + log1pf(expf(-fabsf(x)));
        dz[e] = (1.f / (1.f + expf(-x)) - y) * inv;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}
__global__ void loss_final_kernel(const float* partial, int blocks, int64_t n, float* loss) {
    __shared__ float red[256];
    float s = 0.f;
    for (int b = threadIdx.x; b < blocks; b += 256) s += partial[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0] / (float)n;
}

__global__ void adam_kernel(float* p, const float* g, float* m, float* v, int64_t n, float lr, float bc1, float bc2) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const float ge = g[e];
        const float me = b1 * m[e] + (1.f - b1) * ge;
        const float ve = b2 * v[e] + (1.f - b2) * ge * ge;
        m[e] = me;
        v[e] = ve;
        p[e] -= lr * (me / bc1) / (sqrtf(ve / bc2) + eps);
    }
}

__global__ void occupancy_kernel(const uint32_t* c, uint64_t n, uint8_t* o) {
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (uint64_t)gridDim.x * blockDim.x)
        o[e] = c[e] > 0u ? 1 : 0;
}

__global__ void predict_occupancy_kernel(const float* z, uint64_t n, uint8_t* o) {
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (uint64_t)gridDim.x * blockDim.x)
        o[e] = z[e] > 0.f ? 1 : 0;
}

// one block per set: mean binary entropy of sigmoid(z)
__global__ void uncertainty_kernel(const float* __restrict__ z, float* __restrict__ out) {
    __shared__ float red[256];
    const float* zs = z + (int64_t)blockIdx.x * kImg * kImg;
    float acc = 0.f;
    for (int e = threadIdx.x; e < kImg * kImg; e += 256) {
        const float x = zs[e];
        // H(sigmoid(x)) = log(1 + e^-|x|) + |x| sigmoid(-|x|)
        const float a = fabsf(x);
        acc += log1pf(expf(-a)) + a / (1.f + expf(a));
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0] / (float)(kImg * kImg);
}

__global__ void iou_kernel(const float* __restrict__ z, const uint8_t* __restrict__ pred,
                           const uint8_t* __restrict__ t, float* __restrict__ out) {
    __shared__ int ri[256], ru[256];
    const int64_t base = (int64_t)blockIdx.x * kImg * kImg;
    int inter = 0, uni = 0;
    for (int e = threadIdx.x; e < kImg * kImg; e += 256) {
        const bool p = z ? (z[base + e] > 0.f) : (pred[base + e] != 0);
        const bool q = t[base + e] != 0;
        inter += p && q;
        uni += p || q;
    }
    ri[threadIdx.x] = inter;
    ru[threadIdx.x] = uni;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            ri[threadIdx.x] += ri[threadIdx.x + w];
            ru[threadIdx.x] += ru[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = ru[0] == 0 ? 1.f : (float)ri[0] / (float)ru[0];
}

// ------------------------------------------------------------------ fused forward (inference)
// The whole network for one set in one workgroup, every activation held in
// LDS as bfloat16 -- the rounding the training path applies when it reads
// them as GEMM operands:
//   * u -> h1 (4 -> 256): four products per output on the vector ALUs;
//   * h1 -> h2 (256 -> 256): W2^T h1 on the matrix cores, h1 the only
//     non-zero column of the right operand;
//   * convT k4 s4 p0 (16 -> 64 channels, 4^2 -> 16^2): no two taps of one
//     input pixel overlap, so it is one product x0 (16 pixels x 16) K1
//     (16 x 1024) scattered to the output pixels;
//   * convT k4 s2 p1: output pixel (2m + py, 2n + px) gathers the input
//     pixels (m + dy, n + dx) over two row taps and two column taps fixed by
//     the phase (py, px) (tap_dy, tap_k below), so each of the four phases is
//     a 2 x 2 convolution: Cout x (4 taps * Cin) weights times (4 taps *
//     Cin) x (16 pixels) read straight from the padded input in LDS, one tap
//     and 32 channels per product step.  Taken this way round, a lane ends up
//     holding four consecutive channels of one output pixel;
//   * the last layer (16 -> 1 channel) in column form: col = y3 K4 (16 taps
//     per pixel).  A lane's four channels of y3 are exactly its operand of
//     that product, so y3 never leaves the registers; the columns of four
//     y3 rows at a time go to a ring of nine zero-padded LDS rows (tap-major,
//     so that the lanes of a wave read consecutive words), and each logit
//     sums its four column entries.
// Products: v_mfma_f32_16x16x32_bf16 (16x16x16 where K is 16), FP32 accumulation.
typedef unsigned short bf16_t;
typedef short bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kFwdThreads = 512;                      // 8 waves
constexpr int kY1S = 64 + 8, kY2S = 32 + 8;           // bf16 per pixel: 16-byte rows, padded against bank conflicts
constexpr int kY1Bytes = 18 * 18 * kY1S * 2;          // 16^2 grid with a zero border
constexpr int kY2Bytes = 34 * 34 * kY2S * 2;          // 32^2 grid with a zero border
constexpr int kRing = 9;                              // column rows m0-1 .. m0+7 never share a slot
constexpr int kRingW = 66;                            // x = -1 .. 64, the ends zero
constexpr int kRingBytes = kRing * kRingW * 16 * 4;
constexpr int kFwdLds = kY2Bytes + kY1Bytes + 256 * 2 + 256 * 2 + 16;
static_assert(kRingBytes <= kY1Bytes, "the column ring reuses the y1 space");

// packed bfloat16 weights: a lane's k values adjacent
constexpr size_t kK1p = 1024 * 16;          // [n = o*16 + ky*4 + kx][c]
constexpr size_t kK2p = 4 * 8 * 32 * 32;    // [phase][k step][o][32 k]; k step = tap * 2 + channel half
constexpr size_t kK3p = 4 * 4 * 16 * 32;    // [phase][tap][o][32 c]
constexpr size_t kK4p = 16 * 16;            // [tap = ky*4 + kx][c]
constexpr size_t kW2p = 16 * 8 * 16 * 32;   // [o / 16][k step][o % 16][32 k]
constexpr size_t kPackedElems = kK1p + kK2p + kK3p + kK4p + kW2p;

// Stride-2, pad-1 transposed convolution: for output phase p (0 even, 1
// odd) and tap a (0, 1), the input offset and kernel index.
__device__ __forceinline__ int tap_dy(int p, int a) { return p ? (a ? 0 : 1) : (a ? -1 : 0); }
__device__ __forceinline__ int tap_k(int p, int a) { return p ? (a ? 2 : 0) : (a ? 3 : 1); }

struct PackArgs {
    const float *W2, *K1, *K2, *K3, *K4;
    bf16_t* out;
};

__global__ void pack_weights_kernel(const PackArgs a) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < kPackedElems; e += (size_t)gridDim.x * blockDim.x) {
        float v;
        size_t i = e;
        if (i < kK1p) {
            const int n = (int)(i / 16), c = (int)(i % 16);
            v = a.K1[(c * 64 + n / 16) * 16 + n % 16];
        } else if ((i -= kK1p) < kK2p) {
            const int kk = (int)(i % 32), o = (int)((i / 32) % 32), ks = (int)((i / 1024) % 8), ph = (int)(i / 8192);
            const int tap = ks >> 1, c = (ks & 1) * 32 + kk;
            const int ky = tap_k(ph >> 1, tap >> 1), kx = tap_k(ph & 1, tap & 1);
            v = a.K2[((c * 32 + o) * 4 + ky) * 4 + kx];
        } else if ((i -= kK2p) < kK3p) {
            const int c = (int)(i % 32), o = (int)((i / 32) % 16), tap = (int)((i / 512) % 4), ph = (int)(i / 2048);
            const int ky = tap_k(ph >> 1, tap >> 1), kx = tap_k(ph & 1, tap & 1);
            v = a.K3[((c * 16 + o) * 4 + ky) * 4 + kx];
        } else if ((i -= kK3p) < kK4p) {
            const int tap = (int)(i / 16), c = (int)(i % 16);
            v = a.K4[c * 16 + tap];
        } else {
            i -= kK4p;
            const int kk = (int)(i % 32), oo = (int)((i / 32) % 16), ks = (int)((i / 512) % 8), mt = (int)(i / 4096);
            v = a.W2[(ks * 32 + kk) * 256 + mt * 16 + oo];
        }
        a.out[e] = to_bf16(v);
    }
}

struct FwdArgs {
    const kl_c64 *ta, *tb;
    const float *W1, *b1, *b2;                     // FP32 parameters
    const bf16_t *w2, *k1, *k2, *k3, *k4;          // packed weights
    const float *c1, *c2, *c3, *c4;                // biases
    float* logits;                                 // B x 128 x 128
    int B;
};

__device__ __forceinline__ bf16x4 frag4(const bf16_t* p) { return *(const bf16x4*)p; }
__device__ __forceinline__ bf16x8 frag8(const bf16_t* p) { return *(const bf16x8*)p; }
__device__ __forceinline__ f32x4 mma16(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mma32(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ bf16x4 relu_bf16(f32x4 d, const float* bias) {
    bf16x4 r;
#pragma unroll
    for (int v = 0; v < 4; ++v) r[v] = (short)to_bf16(fmaxf(d[v] + bias[v], 0.f));
    return r;
}

// One workgroup per set, sets dealt round robin over the grid.
__global__ __launch_bounds__(kFwdThreads) void forward_kernel(const FwdArgs a) {
    __shared__ __align__(16) unsigned char dsm[kFwdLds];
    bf16_t* y2p = (bf16_t*)dsm;                                // [34][34][kY2S]
    bf16_t* y1p = (bf16_t*)(dsm + kY2Bytes);                   // [18][18][kY1S]
    bf16_t* h1s = (bf16_t*)(dsm + kY2Bytes + kY1Bytes);        // [256]
    bf16_t* x0s = h1s + 256;                                   // [16 pixels][16 channels]
    float* us = (float*)(x0s + 256);                           // [4]
    float* ring = (float*)(dsm + kY2Bytes);                    // [kRing][16 taps][kRingW], once y1 is consumed
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lq = lane >> 4;
    const f32x4 zero4 = {0.f, 0.f, 0.f, 0.f};

    // weights that stay in registers
    const int ph2 = wave >> 1;                 // convT 2: phase, output rows 8 (wave & 1) .. + 8
    bf16x8 w2[2][8];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) w2[t][ks] = frag8(a.k2 + ((ph2 * 8 + ks) * 32 + 16 * t + lr) * 32 + 8 * lq);
    // convT 3 tiles of this wave: row r3 of each group of four, column phase px3, halves 0 and 1;
    // the row phase is r3 & 1 because groups start at multiples of four
    const int r3 = wave >> 1, px3 = wave & 1, ph3 = (r3 & 1) * 2 + px3;
    bf16x8 w3[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) w3[ks] = frag8(a.k3 + ((ph3 * 4 + ks) * 16 + lr) * 32 + 8 * lq);
    const bf16x4 w4 = frag4(a.k4 + lr * 16 + 4 * lq);
    float b2c[2][4], b3c[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        b2c[0][v] = a.c2[4 * lq + v];
        b2c[1][v] = a.c2[16 + 4 * lq + v];
        b3c[v] = a.c3[4 * lq + v];
    }
    const float b4 = a.c4[0];

    for (int i = tid; i < kY2Bytes / 4; i += kFwdThreads) ((uint32_t*)y2p)[i] = 0u;   // border stays zero

    for (int b = blockIdx.x; b < a.B; b += gridDim.x) {
        for (int i = tid; i < kY1Bytes / 4; i += kFwdThreads) ((uint32_t*)y1p)[i] = 0u;
        if (tid == 0) {
            us[0] = (float)((a.ta[b].re - 2.4) / 0.6);
            us[1] = (float)(a.ta[b].im / 0.3);
            us[2] = (float)((a.tb[b].re - 2.4) / 0.6);
            us[3] = (float)(a.tb[b].im / 0.3);
        }
        __syncthreads();
        // h1 = relu(u W1 + b1), operands rounded to bfloat16
        if (tid < 256) {
            float acc = 0.f;
#pragma unroll
            for (int k = 0; k < 4; ++k) acc = fmaf(bf16_value(us[k]), bf16_value(a.W1[k * 256 + tid]), acc);
            h1s[tid] = to_bf16(fmaxf(acc + a.b1[tid], 0.f));
        }
        __syncthreads();
        // h2 = relu(h1 W2 + b2): rows o of W2^T, 16 per tile, two tiles per wave; column 0 = h1
        {
            f32x4 d[2] = {zero4, zero4};
#pragma unroll
            for (int ks = 0; ks < 8; ++ks) {
                bf16x8 hb = {0, 0, 0, 0, 0, 0, 0, 0};
                if (lr == 0) hb = frag8(h1s + ks * 32 + 8 * lq);
#pragma unroll
                for (int u = 0; u < 2; ++u)
                    d[u] = mma32(frag8(a.w2 + (((2 * wave + u) * 8 + ks) * 16 + lr) * 32 + 8 * lq), hb, d[u]);
            }
            if (lr == 0) {
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int o = 16 * (2 * wave + u) + 4 * lq + v;   // feature c*16 + q -> x0 pixel q, channel c
                        x0s[(o % 16) * 16 + o / 16] = to_bf16(fmaxf(d[u][v] + a.b2[o], 0.f));
                    }
            }
        }
        __syncthreads();

        // convT 1: N tile t = output channel t (16 taps); rows = the 16 input pixels
        {
            const bf16x4 ax = frag4(x0s + lr * 16 + 4 * lq);
            const int ky = lr >> 2, kx = lr & 3;
            for (int t = wave; t < 64; t += kFwdThreads / 64) {
                const f32x4 d = mma16(ax, frag4(a.k1 + (16 * t + lr) * 16 + 4 * lq), zero4);
                const float bias = a.c1[t];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int p = 4 * lq + v, i = p >> 2, j = p & 3;
                    y1p[((4 * i + ky + 1) * 18 + 4 * j + kx + 1) * kY1S + t] = to_bf16(fmaxf(d[v] + bias, 0.f));
                }
            }
        }
        __syncthreads();

        // convT 2, phase ph2: tile = output row 2m + py, columns 2n + px for n = lane's lr
        {
            const int py = ph2 >> 1, px = ph2 & 1;
            for (int mi = 0; mi < 8; ++mi) {
                const int m = 8 * (wave & 1) + mi;
                bf16x8 ay[8];
#pragma unroll
                for (int ks = 0; ks < 8; ++ks) {
                    const int tap = ks >> 1;
                    const int iy = m + tap_dy(py, tap >> 1) + 1, ix = lr + tap_dy(px, tap & 1) + 1;
                    ay[ks] = frag8(y1p + (iy * 18 + ix) * kY1S + (ks & 1) * 32 + 8 * lq);
                }
                f32x4 d0 = zero4, d1 = zero4;
#pragma unroll
                for (int ks = 0; ks < 8; ++ks) {
                    d0 = mma32(w2[0][ks], ay[ks], d0);
                    d1 = mma32(w2[1][ks], ay[ks], d1);
                }
                // keep that order: the 8 LDS reads, then the 16 products
                __builtin_amdgcn_sched_group_barrier(0x100, 8, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, 16, 0);
                bf16_t* dst = y2p + ((2 * m + py + 1) * 34 + 2 * lr + px + 1) * kY2S + 4 * lq;
                *(bf16x4*)dst = relu_bf16(d0, b2c[0]);
                *(bf16x4*)(dst + 16) = relu_bf16(d1, b2c[1]);
            }
        }
        __syncthreads();
        // the ring: row -1 (slot 0) zero, the end pixels of every row zero
        for (int i = tid; i < kRingW * 16; i += kFwdThreads) ring[i] = 0.f;
        for (int i = tid; i < (kRing - 1) * 16 * 2; i += kFwdThreads) {
            const int slot = 1 + i / 32, tap = (i / 2) % 16, end = i & 1;
            ring[(slot * 16 + tap) * kRingW + (end ? kRingW - 1 : 0)] = 0.f;
        }

        // groups of four y3 rows m0 .. m0 + 3 (slot of row m: (m + 1) mod kRing);
        // the 17th group only closes the last logit row
        for (int g = 0; g <= 16; ++g) {
            const int m0 = 4 * g;
            if (g < 16) {
                const int Y = m0 + r3, m = Y >> 1, py = Y & 1;
                bf16x8 ay[2][4];
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const int iy = m + tap_dy(py, ks >> 1) + 1;
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int ix = 16 * h + lr + tap_dy(px3, ks & 1) + 1;
                        ay[h][ks] = frag8(y2p + (iy * 34 + ix) * kY2S + 8 * lq);
                    }
                }
                f32x4 d[2] = {zero4, zero4};
#pragma unroll
                for (int ks = 0; ks < 4; ++ks)
#pragma unroll
                    for (int h = 0; h < 2; ++h) d[h] = mma32(w3[ks], ay[h][ks], d[h]);
                __builtin_amdgcn_sched_group_barrier(0x100, 8, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, 8, 0);
                float* row = ring + ((Y + 1) % kRing) * 16 * kRingW;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const f32x4 c = mma16(w4, relu_bf16(d[h], b3c), zero4);   // taps 4 lq + v of pixel x
                    const int x = 2 * (16 * h + lr) + px3;
#pragma unroll
                    for (int v = 0; v < 4; ++v) row[(4 * lq + v) * kRingW + x + 1] = c[v];
                }
            } else {
                for (int i = tid; i < kRingW * 16; i += kFwdThreads) ring[(65 % kRing) * kRingW * 16 + i] = 0.f;  // row 64
            }
            __syncthreads();
            // logit row Z = 2 m0 - 1 + tid / 64 (those in range), columns 2u and 2u + 1 for u = tid % 64:
            // X = 2u takes pixels u (kx 1) and u - 1 (kx 3), X = 2u + 1 pixels u + 1 (kx 0) and u (kx 2)
            {
                const int Z = 2 * m0 - 1 + (tid >> 6), u = tid & 63;
                if (Z >= 0 && Z < 128) {
                    float e0 = 0.f, e1 = 0.f;
#pragma unroll
                    for (int ra = 0; ra < 2; ++ra) {
                        // taps (ky, 0..3) of y3 row (Z >> 1) + dy; ring x = pixel + 1
                        const float* t = ring + ((((Z >> 1) + tap_dy(Z & 1, ra) + 1) % kRing) * 16 +
                                                 4 * tap_k(Z & 1, ra)) * kRingW + u;
                        e0 += t[kRingW + 1] + t[3 * kRingW];
                        e1 += t[2] + t[2 * kRingW + 1];
                    }
                    float2 out = {e0 + b4, e1 + b4};
                    *(float2*)(a.logits + ((int64_t)b * 128 + Z) * 128 + 2 * u) = out;
                }
            }
        }
        __syncthreads();   // the next set's y1 clear overwrites the ring
    }
}

static unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(8192, (n + 255) / 256)); }

// ------------------------------------------------------------------ workspace
struct WS {
    float *u, *h1, *h2, *x0, *col1, *y1, *col2, *y2, *col3, *y3, *col4, *logits, *dlogits, *dy3, *dy2, *dy1, *dx0,
        *dh2, *dh1, *partial, *loss;
    bf16_t* packed;   // decoder weights of the fused inference path
    size_t bytes;
};

static const ConvShape kC1{4, 16, 64, 4, 0}, kC2{16, 32, 32, 2, 1}, kC3{32, 64, 16, 2, 1}, kC4{64, 128, 1, 2, 1};

static WS carve(void* base, int B) {
    WS w;
    size_t o = 0;
    auto take = [&](size_t nfloat) {
        float* p = base ? (float*)((char*)base + o) : nullptr;
        o += ((nfloat * sizeof(float) + 255) / 256) * 256;
        return p;
    };
    const size_t b = (size_t)B;
    w.u = take(b * 4);
    w.h1 = take(b * 256);
    w.h2 = take(b * 256);
    w.x0 = take(b * 256);
    w.col1 = take(b * 16 * 1024);
    w.y1 = take(b * 256 * 64);
    w.col2 = take(b * 256 * 512);
    w.y2 = take(b * 1024 * 32);
    w.col3 = take(b * 1024 * 256);
    w.y3 = take(b * 4096 * 16);
    w.col4 = take(b * 4096 * 16);
    w.logits = take(b * kImg * kImg);
    w.dlogits = take(b * kImg * kImg);
    w.dy3 = take(b * 4096 * 16);
    w.dy2 = take(b * 1024 * 32);
    w.dy1 = take(b * 256 * 64);
    w.dx0 = take(b * 256);
    w.dh2 = take(b * 256);
    w.dh1 = take(b * 256);
    w.partial = take(1024 * 256);
    w.loss = take(64);
    w.packed = (bf16_t*)take((kPackedElems + 1) / 2);
    w.bytes = o;
    return w;
}

#define CHECK_HIP(x)                                  \
    do {                                              \
        hipError_t e_ = (x);                          \
        if (e_ != hipSuccess) return e_;              \
    } while (0)

// forward pass into w (logits into `logits`)
static hipError_t forward(const float* P, const kl_c64* ta, const kl_c64* tb, int B, float* logits, const WS& w,
                          hipStream_t s) {
    const Layout L = layout();
    hipLaunchKernelGGL(features_kernel, dim3((B + 255) / 256), dim3(256), 0, s, ta, tb, B, w.u);
    CHECK_HIP(gemm(B, 256, 4, w.u, 4, 1, P + L.W1, 256, 1, w.h1, 256, P + L.b1, 1, 0, s));
    CHECK_HIP(gemm(B, 256, 256, w.h1, 256, 1, P + L.W2, 256, 1, w.h2, 256, P + L.b2, 1, 0, s));
    hipLaunchKernelGGL(h2_to_x0_kernel, dim3(grid_for(B * 256)), dim3(256), 0, s, w.h2, w.x0, B);
    // C1: (B*16) x 16 -> col1 (B*16) x 1024 -> y1 (B*256) x 64
    CHECK_HIP(gemm(B * 16, 1024, 16, w.x0, 16, 1, P + L.K1, 1024, 1, w.col1, 1024, nullptr, 0, 0, s));
    hipLaunchKernelGGL(col2im_kernel, dim3(grid_for((int64_t)B * 256 * 64)), dim3(256), 0, s, w.col1, P + L.c1,
                       w.y1, B, kC1, 1);
    CHECK_HIP(gemm(B * 256, 512, 64, w.y1, 64, 1, P + L.K2, 512, 1, w.col2, 512, nullptr, 0, 0, s));
    hipLaunchKernelGGL(col2im_kernel, dim3(grid_for((int64_t)B * 1024 * 32)), dim3(256), 0, s, w.col2, P + L.c2,
                       w.y2, B, kC2, 1);
    CHECK_HIP(gemm(B * 1024, 256, 32, w.y2, 32, 1, P + L.K3, 256, 1, w.col3, 256, nullptr, 0, 0, s));
    hipLaunchKernelGGL(col2im_kernel, dim3(grid_for((int64_t)B * 4096 * 16)), dim3(256), 0, s, w.col3, P + L.c3,
                       w.y3, B, kC3, 1);
    CHECK_HIP(gemm(B * 4096, 16, 16, w.y3, 16, 1, P + L.K4, 16, 1, w.col4, 16, nullptr, 0, 0, s));
    hipLaunchKernelGGL(col2im_kernel, dim3(grid_for((int64_t)B * kImg * kImg)), dim3(256), 0, s, w.col4, P + L.c4,
                       logits, B, kC4, 0);
    return hipGetLastError();
}

// Inference forward: the weights packed once per call, then the whole network
// per set in one kernel.
static hipError_t forward_fused(const float* P, const kl_c64* ta, const kl_c64* tb, int B, float* logits,
                                const WS& w, hipStream_t s) {
    const Layout L = layout();
    const PackArgs pa{P + L.W2, P + L.K1, P + L.K2, P + L.K3, P + L.K4, w.packed};
    hipLaunchKernelGGL(pack_weights_kernel, dim3(grid_for((int64_t)kPackedElems)), dim3(256), 0, s, pa);
    const bf16_t* k1 = w.packed;
    const bf16_t* k2 = k1 + kK1p;
    const bf16_t* k3 = k2 + kK2p;
    const bf16_t* k4 = k3 + kK3p;
    const bf16_t* w2 = k4 + kK4p;
    const FwdArgs f{ta, tb, P + L.W1, P + L.b1, P + L.b2, w2, k1, k2, k3, k4, P + L.c1, P + L.c2, P + L.c3, P + L.c4,
                    logits, B};
    hipLaunchKernelGGL(forward_kernel, dim3(std::min(B, 1024)), dim3(kFwdThreads), 0, s, f);
    return hipGetLastError();
}

// Backward of one transposed convolution: d_out (masked already) ->
// dbias, dK, d_in.  x_in: the layer input (Hin grid, Ci channels).
static hipError_t conv_backward(const float* dout, const float* x_in, const float* K, int Ci, ConvShape c, int B,
                                float* dcol, float* dK, float* dbias, float* din, const WS& w, hipStream_t s) {
    const int64_t rows_out = (int64_t)B * c.Hout * c.Hout;
    const int64_t rows_in = (int64_t)B * c.Hin * c.Hin;
    CHECK_HIP(colsum(dout, rows_out, c.Co, dbias, w.partial, s));
    hipLaunchKernelGGL(im2col_kernel, dim3(grid_for(rows_in * c.Co * 16)), dim3(256), 0, s, dout, dcol, B, c);
    const int N = c.Co * 16;
    // dK (Ci x N) = x_in^T (Ci x rows_in) dcol (rows_in x N)
    CHECK_HIP(gemm(Ci, N, (int)rows_in, x_in, 1, Ci, dcol, N, 1, dK, N, nullptr, 0, 0, s));
    // d_in (rows_in x Ci) = dcol (rows_in x N) K^T (N x Ci)
    if (din) CHECK_HIP(gemm((int)rows_in, Ci, N, dcol, N, 1, K, 1, N, din, Ci, nullptr, 0, 0, s));
    return hipGetLastError();
}

static hipError_t loss_grad(const float* P, const kl_c64* ta, const kl_c64* tb, const uint8_t* targets, int B,
                            float* G, float* loss, const WS& w, hipStream_t s) {
    const Layout L = layout();
    CHECK_HIP(forward(P, ta, tb, B, w.logits, w, s));
    const int64_t npx = (int64_t)B * kImg * kImg;
    const int bce_blocks = (int)std::min<int64_t>(1024, (npx + 255) / 256);
    hipLaunchKernelGGL(bce_kernel, dim3(bce_blocks), dim3(256), 0, s, w.logits, targets, npx, w.dlogits, w.partial);
    hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(256), 0, s, w.partial, bce_blocks, npx, loss);
    // C4 (no activation): d_out = dlogits
    CHECK_HIP(conv_backward(w.dlogits, w.y3, P + L.K4, 16, kC4, B, w.col4, G + L.K4, G + L.c4, w.dy3, w, s));
    hipLaunchKernelGGL(relu_mask_kernel, dim3(grid_for((int64_t)B * 4096 * 16)), dim3(256), 0, s, w.dy3, w.y3,
                       (int64_t)B * 4096 * 16);
    CHECK_HIP(conv_backward(w.dy3, w.y2, P + L.K3, 32, kC3, B, w.col3, G + L.K3, G + L.c3, w.dy2, w, s));
    hipLaunchKernelGGL(relu_mask_kernel, dim3(grid_for((int64_t)B * 1024 * 32)), dim3(256), 0, s, w.dy2, w.y2,
                       (int64_t)B * 1024 * 32);
    CHECK_HIP(conv_backward(w.dy2, w.y1, P + L.K2, 64, kC2, B, w.col2, G + L.K2, G + L.c2, w.dy1, w, s));
    hipLaunchKernelGGL(relu_mask_kernel, dim3(grid_for((int64_t)B * 256 * 64)), dim3(256), 0, s, w.dy1, w.y1,
                       (int64_t)B * 256 * 64);
    CHECK_HIP(conv_backward(w.dy1, w.x0, P + L.K1, 16, kC1, B, w.col1, G + L.K1, G + L.c1, w.dx0, w, s));
    hipLaunchKernelGGL(x0_to_h2_kernel, dim3(grid_for(B * 256)), dim3(256), 0, s, w.dx0, w.dh2, B);
    hipLaunchKernelGGL(relu_mask_kernel, dim3(grid_for(B * 256)), dim3(256), 0, s, w.dh2, w.h2, (int64_t)B * 256);
    CHECK_HIP(colsum(w.dh2, B, 256, G + L.b2, w.partial, s));
    CHECK_HIP(gemm(256, 256, B, w.h1, 1, 256, w.dh2, 256, 1, G + L.W2, 256, nullptr, 0, 0, s));   // h1^T dh2
    CHECK_HIP(gemm(B, 256, 256, w.dh2, 256, 1, P + L.W2, 1, 256, w.dh1, 256, nullptr, 0, 0, s));  // dh2 W2^T
    hipLaunchKernelGGL(relu_mask_kernel, dim3(grid_for(B * 256)), dim3(256), 0, s, w.dh1, w.h1, (int64_t)B * 256);
    CHECK_HIP(colsum(w.dh1, B, 256, G + L.b1, w.partial, s));
    CHECK_HIP(gemm(4, 256, B, w.u, 1, 4, w.dh1, 256, 1, G + L.W1, 256, nullptr, 0, 0, s));          // u^T dh1
    return hipGetLastError();
}

}  // namespace sur
}  // namespace kl

using namespace kl;
using namespace kl::sur;

static int sur_fail(int code, const char* m) { return set_error(code, "%s", m); }

extern "C" {

size_t kl_sur_num_params(void) { return layout().total; }

size_t kl_sur_workspace_bytes(int batch) { return batch > 0 ? carve(nullptr, batch).bytes : 0; }

int kl_sur_workspace_tensor(int batch, int which, size_t* offset_bytes, size_t* n_floats) {
    if (batch <= 0 || !offset_bytes || !n_floats) return sur_fail(KL_EINVAL, "bad workspace query");
    const WS w = carve(nullptr, batch);
    const WS z = carve((void*)(uintptr_t)256, batch);   // offsets relative to a nonzero base
    const size_t b = (size_t)batch;
    const float* p = nullptr;
    size_t n = 0;
    switch (which) {
        case KL_SUR_T_U: p = z.u; n = b * 4; break;
        case KL_SUR_T_H1: p = z.h1; n = b * 256; break;
        case KL_SUR_T_H2: p = z.h2; n = b * 256; break;
        case KL_SUR_T_X0: p = z.x0; n = b * 256; break;
        case KL_SUR_T_Y1: p = z.y1; n = b * 256 * 64; break;
        case KL_SUR_T_Y2: p = z.y2; n = b * 1024 * 32; break;
        case KL_SUR_T_Y3: p = z.y3; n = b * 4096 * 16; break;
        case KL_SUR_T_LOGITS: p = z.logits; n = b * kImg * kImg; break;
        case KL_SUR_T_DLOGITS: p = z.dlogits; n = b * kImg * kImg; break;
        case KL_SUR_T_DY3: p = z.dy3; n = b * 4096 * 16; break;
        case KL_SUR_T_DY2: p = z.dy2; n = b * 1024 * 32; break;
        case KL_SUR_T_DY1: p = z.dy1; n = b * 256 * 64; break;
        case KL_SUR_T_DX0: p = z.dx0; n = b * 256; break;
        case KL_SUR_T_DH2: p = z.dh2; n = b * 256; break;
        case KL_SUR_T_DH1: p = z.dh1; n = b * 256; break;
        default: return sur_fail(KL_EINVAL, "unknown workspace tensor");
    }
    (void)w;
    *offset_bytes = (size_t)((const char*)p - (const char*)(uintptr_t)256);
    *n_floats = n;
    return KL_OK;
}

int kl_gemm_bf16(int M, int N, int K, const float* A, int64_t lda_m, int64_t lda_k, const float* B, int64_t ldb_k,
                 int64_t ldb_n, float* C, int64_t ldc, const float* bias, int relu, int accumulate, void* stream) {
    if (M < 0 || N < 0 || K < 0) return sur_fail(KL_EINVAL, "negative GEMM size");
    if (M == 0 || N == 0) return KL_OK;
    if ((K > 0 && (!A || !B)) || !C) return sur_fail(KL_EINVAL, "NULL GEMM operand");
    if (accumulate && (bias || relu)) return sur_fail(KL_EINVAL, "accumulate excludes bias and relu");
    hipError_t e = gemm(M, N, K, A, lda_m, lda_k, B, ldb_k, ldb_n, C, ldc, bias, relu, accumulate, (hipStream_t)stream);
    return e == hipSuccess ? KL_OK : sur_fail(KL_EDEVICE, hipGetErrorString(e));
}

int kl_sur_forward(const float* params, const kl_c64* ta, const kl_c64* tb, int batch, float* logits_out,
                   void* workspace, size_t workspace_bytes, void* stream) {
    if (batch > 512) return sur_fail(KL_EINVAL, "batch above 512");
    if (batch <= 0 || !params || !ta || !tb || !logits_out || !workspace)
        return sur_fail(KL_EINVAL, "bad surrogate forward arguments");
    if (workspace_bytes < kl_sur_workspace_bytes(batch)) return sur_fail(KL_EINVAL, "workspace too small");
    const WS w = carve(workspace, batch);
    hipError_t e = forward_fused(params, ta, tb, batch, logits_out, w, (hipStream_t)stream);
    return e == hipSuccess ? KL_OK : sur_fail(KL_EDEVICE, hipGetErrorString(e));
}

int kl_sur_loss_grad(const float* params, const kl_c64* ta, const kl_c64* tb, const uint8_t* targets, int batch,
                     float* grad_out, float* loss_out, void* workspace, size_t workspace_bytes, void* stream) {
    if (batch > 512) return sur_fail(KL_EINVAL, "batch above 512");
    if (batch <= 0 || !params || !ta || !tb || !targets || !grad_out || !loss_out || !workspace)
        return sur_fail(KL_EINVAL, "bad surrogate gradient arguments");
    if (workspace_bytes < kl_sur_workspace_bytes(batch)) return sur_fail(KL_EINVAL, "workspace too small");
    const WS w = carve(workspace, batch);
    hipError_t e = loss_grad(params, ta, tb, targets, batch, grad_out, loss_out, w, (hipStream_t)stream);
    return e == hipSuccess ? KL_OK : sur_fail(KL_EDEVICE, hipGetErrorString(e));
}

int kl_sur_adam(float* params, const float* grad, float* m, float* v, int step, float lr, void* stream) {
    if (!params || !grad || !m || !v || step < 1) return sur_fail(KL_EINVAL, "bad Adam arguments");
    const int64_t n = (int64_t)layout().total;
    const float bc1 = 1.f - powf(0.9f, (float)step), bc2 = 1.f - powf(0.999f, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, params, grad, m, v, n, lr,
                       bc1, bc2);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? KL_OK : sur_fail(KL_EDEVICE, hipGetErrorString(e));
}

int kl_sur_train_step(float* params, float* m, float* v, float* grad_scratch, int step, float lr, const kl_c64* ta,
                      const kl_c64* tb, const uint8_t* targets, int batch, float* loss_out, void* workspace,
                      size_t workspace_bytes, void* stream) {
    if (!grad_scratch) return sur_fail(KL_EINVAL, "grad_scratch is NULL");
    int rc = kl_sur_loss_grad(params, ta, tb, targets, batch, grad_scratch, loss_out, workspace, workspace_bytes, stream);
    if (rc) return rc;
    return kl_sur_adam(params, grad_scratch, m, v, step, lr, stream);
}

int kl_occupancy(const uint32_t* counts, uint64_t n, uint8_t* occ_out, void* stream) {
    if (n == 0) return KL_OK;
    if (!counts || !occ_out) return sur_fail(KL_EINVAL, "NULL occupancy buffer");
    hipLaunchKernelGGL(occupancy_kernel, dim3(grid_for((int64_t)std::min<uint64_t>(n, 1ull << 40))), dim3(256), 0,
                       (hipStream_t)stream, counts, n, occ_out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? KL_OK : sur_fail(KL_EDEVICE, hipGetErrorString(e));
}

int kl_sur_predict_occupancy(const float* logits, uint64_t n, uint8_t* occ_out, void* stream) {
    if (n == 0) return KL_OK;
    if (!logits || !occ_out) return sur_fail(KL_EINVAL, "NULL occupancy buffer");
    hipLaunchKernelGGL(predict_occupancy_kernel, dim3(grid_for((int64_t)std::min<uint64_t>(n, 1ull << 40))), dim3(256),
                       0, (hipStream_t)stream, logits, n, occ_out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? KL_OK : sur_fail(KL_EDEVICE, hipGetErrorString(e));
}

int kl_sur_uncertainty(const float* logits, int batch, float* out, void* stream) {
    if (batch <= 0 || !logits || !out) return sur_fail(KL_EINVAL, "bad uncertainty arguments");
    hipLaunchKernelGGL(uncertainty_kernel, dim3(batch), dim3(256), 0, (hipStream_t)stream, logits, out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? KL_OK : sur_fail(KL_EDEVICE, hipGetErrorString(e));
}

int kl_iou(const float* logits, const uint8_t* pred_occ, const uint8_t* target_occ, int batch, float* iou_out,
           void* stream) {
    if (batch <= 0 || (!logits && !pred_occ) || !target_occ || !iou_out)
        return sur_fail(KL_EINVAL, "bad IoU arguments");
    hipLaunchKernelGGL(iou_kernel, dim3(batch), dim3(256), 0, (hipStream_t)stream, logits, pred_occ, target_occ,
                       iou_out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? KL_OK : sur_fail(KL_EDEVICE, hipGetErrorString(e));
}

}  // extern "C"
