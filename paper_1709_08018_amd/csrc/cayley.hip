// cayley.hip -- gfx950 kernels of libkl for words of an indexed Cayley
// table (Section 5 of the paper): decode, FP64 values and images.
#include <algorithm>

#include "kl_internal.hpp"

namespace kl {

constexpr uint32_t kCayleyOutside = 0xFFFFFFFFu;

// Bin of FP64 pixel coordinates, or kCayleyOutside when outside
// [0, W) x [0, H) or NaN (every comparison with NaN is false).
__device__ __forceinline__ uint32_t cayley_bin(double px, double py, uint32_t W, uint32_t H) {
    const bool ok = (px >= 0.0) & (px < (double)W) & (py >= 0.0) & (py < (double)H);
    const uint32_t col = ok ? (uint32_t)px : 0u;
    const uint32_t row = ok ? (uint32_t)py : 0u;
    return ok ? __umul24(row, W) + col : kCayleyOutside;
}

}  // namespace kl

namespace kl {

// Words of an indexed Cayley table (Section 5): symbols 1..m, states 0..S-1,
// a word x_1..x_d read right to left from state 0 and regular when no step
// lands in state 0 again; words numbered in lexicographic order, x_1 most
// significant.  C[L][s] counts the regular words of length L whose walk
// ends in state s.  A prefix is read after the rest of its word, from the
// state the rest ended in; `good` holds the states from which the prefix so
// far reads without a crash, and the words that begin with it number
// sum over s in good of C[remaining][s].  Choosing the next symbol x
// restricts good to the states s with T(s, x) != 0 and T(s, x) in good.
//
// The word's maps are multiplied left to right in FP64 while it is
// unranked, then applied to the seed: the attracting fixed point of its
// last symbol, or of one symbol for every word.
// pixel coordinates (or z itself under the identity fold) of the point (num : den)
__device__ inline void cayley_pixel(const CayleyJob& a, c64 num, c64 den, double& px, double& py) {
    const double n2 = fma_(den.re, den.re, den.im * den.im);
    const double re = fma_(num.re, den.re, num.im * den.im) / n2;
    const double im = fma_(num.im, den.re, -(num.re * den.im)) / n2;
    px = fma_(a.fold.s, re, a.fold.o.re) * a.fold.aniso;
    py = fma_(a.fold.s, im, a.fold.o.im);
}

constexpr int kCayleyRun = 16;   // consecutive words per thread in a render

// The good sets reachable from the set of all states form a deterministic
// automaton (next_set); CM[L][g] = sum over s in set g of C[L][s] counts the
// words that begin with a prefix of good set g and have L symbols to go.
// Choosing a symbol is then two table reads per candidate.  A word's
// symbols are packed 3 bits each (x - 1) into two registers and walked right
// to left in FP64 homogeneous coordinates from the seed.
template <int MODE>
__global__ __launch_bounds__(256) void cayley_kernel(const CayleyJob a) {
    __shared__ uint64_t C[KL_MAX_DEPTH + 1][kCayleyMaxStates];
    __shared__ uint64_t CM[KL_MAX_DEPTH + 1][kCayleyMaxSets];
    __shared__ uint8_t NX[kCayleyMaxSets * kCayleyMaxSymbols];
    __shared__ m64 G[kCayleyMaxSymbols];
    const int S = a.S, m = a.m, M = a.n_sets, D = a.max_depth;
    for (int i = threadIdx.x; i < M * m; i += blockDim.x) NX[i] = a.next_set[i];
    for (int i = threadIdx.x; i < m; i += blockDim.x) G[i] = a.maps[i];
    if (threadIdx.x < (unsigned)S) C[0][threadIdx.x] = threadIdx.x == 0 ? 1 : 0;
    __syncthreads();
    for (int L = 1; L <= D; ++L) {
        const int t = threadIdx.x;
        if (t < S) {
            uint64_t n = 0;
            if (t != 0)
                for (int s = 0; s < S; ++s)
                    for (int x = 1; x <= m; ++x)
                        if (a.table[s * (m + 1) + x] == t) n += C[L - 1][s];
            C[L][t] = n;
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < (D + 1) * M; i += blockDim.x) {
        const int L = i / M, g = i - L * M;
        uint64_t n = 0;
        for (int s = 0; s < S; ++s)
            if ((a.sets[g] >> s) & 1u) n += C[L][s];
        CM[L][g] = n;
    }
    __syncthreads();

    uint64_t drop = 0;
    uint32_t run_key = kCayleyOutside, run_len = 0;
    const uint64_t per = MODE == kCayleyRender ? kCayleyRun : 1;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * per;
    for (uint64_t k0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * per; k0 < a.count; k0 += stride) {
        const uint64_t k1 = k0 + per < a.count ? k0 + per : a.count;
        for (uint64_t k = k0; k < k1; ++k) {
            int d = D;
            uint64_t local;
            if (MODE == kCayleyEval) {
                local = a.idx[k];
                if (local >= a.depth_start[1]) {
                    a.z_out[k] = {__builtin_nan(""), __builtin_nan("")};
                    continue;
                }
            } else {
                const uint64_t i = a.first + k;
                d = a.min_depth;
                while (i >= a.depth_start[d - a.min_depth + 1]) ++d;
                local = i - a.depth_start[d - a.min_depth];
            }
            int g = 0;
            uint64_t lo = 0, hi = 0;   // symbols x - 1, 3 bits each: 0..20 in lo, 21..39 in hi
            for (int j = 0; j < d; ++j) {
                const uint64_t* row = CM[d - j - 1];
                int x = 1, gx = 0;
                for (; x <= m; ++x) {
                    gx = NX[g * m + x - 1];
                    const uint64_t n = row[gx];
                    if (local < n) break;
                    local -= n;
                }
                g = gx;
                if (MODE == kCayleyDecode) a.symbols_out[k * (uint64_t)d + j] = (uint8_t)x;
                else if (j < 21) lo |= (uint64_t)(x - 1) << (3 * j);
                else hi |= (uint64_t)(x - 1) << (3 * (j - 21));
            }
            if (MODE == kCayleyDecode) continue;
            const int last = (int)(((d - 1) < 21 ? lo >> (3 * (d - 1)) : hi >> (3 * (d - 22))) & 7u);
            const int sd = a.seed < 0 ? last : a.seed;
            c64 u = a.fix[sd], v = {1.0, 0.0};
            if ((a.inf_mask >> sd) & 1u) {
                u = {1.0, 0.0};
                v = {0.0, 0.0};
            }
            for (int j = d - 1; j >= 0; --j) {
                const int x = (int)((j < 21 ? lo >> (3 * j) : hi >> (3 * (j - 21))) & 7u);
                const m64& Gx = G[x];
                const c64 nu = cfma(Gx.a, u, cmul(Gx.b, v));
                const c64 nv = cfma(Gx.c, u, cmul(Gx.d, v));
                u = nu;
                v = nv;
            }
            double px, py;
            cayley_pixel(a, u, v, px, py);
            if (MODE == kCayleyEval) {
                a.z_out[k] = {px, py};
            } else {
                const uint32_t key = cayley_bin(px, py, a.W, a.H);
                if (key != run_key) {
                    if (run_key == kCayleyOutside) drop += run_len;
                    else if (run_len) atomicAdd(a.image + run_key, run_len);
                    run_key = key;
                    run_len = 0;
                }
                ++run_len;
            }
        }
    }
    if (MODE == kCayleyRender) {
        if (run_key == kCayleyOutside) drop += run_len;
        else if (run_len) atomicAdd(a.image + run_key, run_len);
        if (a.dropped) {
            for (int off = kWave / 2; off > 0; off >>= 1) drop += __shfl_down(drop, off, kWave);
            if ((threadIdx.x & (kWave - 1)) == 0 && drop)
                atomicAdd((unsigned long long*)a.dropped, (unsigned long long)drop);
        }
    }
}

hipError_t launch_cayley(const CayleyJob& j, int mode, hipStream_t s) {
    if (j.count == 0) return hipSuccess;
    const uint64_t per = mode == kCayleyRender ? kCayleyRun : 1;
    uint64_t blocks = (j.count + 256 * per - 1) / (256 * per);
    blocks = std::min<uint64_t>(blocks, (uint64_t)std::max(1, j.grid_blocks));
    if (mode == kCayleyDecode) hipLaunchKernelGGL(cayley_kernel<kCayleyDecode>, dim3((unsigned)blocks), dim3(256), 0, s, j);
    else if (mode == kCayleyEval) hipLaunchKernelGGL(cayley_kernel<kCayleyEval>, dim3((unsigned)blocks), dim3(256), 0, s, j);
    else hipLaunchKernelGGL(cayley_kernel<kCayleyRender>, dim3((unsigned)blocks), dim3(256), 0, s, j);
    return hipGetLastError();
}

}  // namespace kl
