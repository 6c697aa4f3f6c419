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
// 1 / x: v_rcp_f64 refined by two Newton steps r <- r + r (1 - x r), a
// full-precision reciprocal (x = 0 or an infinite x give NaN, a word that
// is dropped)
__device__ __forceinline__ double cayley_recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma_(-x, r, 1.0);
    r = fma_(r, e, r);
    e = fma_(-x, r, 1.0);
    return fma_(r, e, r);
}

// pixel coordinates (or z itself under the identity fold) of the point (num : den)
__device__ inline void cayley_pixel(const CayleyJob& a, c64 num, c64 den, double& px, double& py) {
    const double rc = cayley_recip(fma_(den.re, den.re, den.im * den.im));
    const double re = fma_(num.re, den.re, num.im * den.im) * rc;
    const double im = fma_(num.im, den.re, -(num.re * den.im)) * rc;
    px = fma_(a.fold.s, re, a.fold.o.re) * a.fold.aniso;
    py = fma_(a.fold.s, im, a.fold.o.im);
}

// consecutive words per thread in a render: enough threads to fill the grid,
// runs no shorter than 16 words and no longer than 256
constexpr int kCayleyRunMin = 16, kCayleyRunMax = 256;

// symbol j (0-based, x - 1) of a word packed 3 bits each into lo (0..20) and hi (21..39)
__device__ __forceinline__ int packed_symbol(uint64_t lo, uint64_t hi, int j) {
    return (int)((j < 21 ? lo >> (3 * j) : hi >> (3 * (j - 21))) & 7u);
}

// The good sets reachable from the set of all states form a deterministic
// automaton (next_set); CM[L][g] = sum over s in set g of C[L][s] counts the
// words that begin with a prefix of good set g and have L symbols to go.
// Choosing a symbol is then two table reads per candidate.  A word's
// symbols are packed 3 bits each (x - 1) into two registers.
//
// Words of depth d >= r are evaluated as head . tail, the tail being the
// last r symbols.  The tail read from state 0 ends in some state; the word
// is regular when the head reads from that state, i.e. the state is in the
// head's good set.  Every regular word of length r is a candidate tail: a
// table in LDS holds them in lexicographic order with their end states and
// their points (the maps of the tail applied right to left to the seed, FP64
// homogeneous).  The words of one head are then consecutive in index order
// and run over the candidate tails whose end state the head accepts, so a
// thread unranks the first word of its run once, keeps the head's product
// (FP64, left to right), and steps through the table: one Moebius map of a
// table point per word.  Shorter words are walked right to left in full.
template <int MODE>
__global__ __launch_bounds__(256) void cayley_kernel(const CayleyJob a) {
    __shared__ uint64_t C[KL_MAX_DEPTH + 1][kCayleyMaxStates];
    __shared__ uint64_t CM[KL_MAX_DEPTH + 1][kCayleyMaxSets];
    __shared__ uint8_t NX[kCayleyMaxSets * kCayleyMaxSymbols];
    __shared__ uint16_t SETS[kCayleyMaxSets];
    __shared__ m64 G[kCayleyMaxSymbols];
    __shared__ c64 TU[MODE == kCayleyDecode ? 1 : kCayleyMaxTails], TV[MODE == kCayleyDecode ? 1 : kCayleyMaxTails];
    __shared__ uint8_t TS[MODE == kCayleyDecode ? 1 : kCayleyMaxTails];
    const int S = a.S, m = a.m, M = a.n_sets, D = a.max_depth;
    const int r = MODE == kCayleyDecode ? 0 : a.r;
    for (int i = threadIdx.x; i < M * m; i += blockDim.x) NX[i] = a.next_set[i];
    for (int i = threadIdx.x; i < M; i += blockDim.x) SETS[i] = a.sets[i];
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

    // Unrank word `local` of length d (lexicographic, first symbol most
    // significant) from good set g0; symbol j chosen among the candidates
    // by the counts of their completions.  With hl >= 0 also the good set
    // after the first hl symbols and their product.
    auto unrank = [&](uint64_t local, int d, int g0, int hl, uint64_t& lo, uint64_t& hi, int& gh, m64& Mh,
                      uint64_t k) {
        int g = g0;
        lo = hi = 0;
        for (int j = 0; j < d; ++j) {
            if (j == hl) gh = g;
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
            if (j < hl) Mh = mmul(Mh, G[x - 1]);
        }
    };
    // the seed of a word whose last symbol is `last` (0-based), homogeneous
    auto seed_point = [&](int last, c64& u, c64& v) {
        const int sd = a.seed < 0 ? last : a.seed;
        u = a.fix[sd];
        v = {1.0, 0.0};
        if ((a.inf_mask >> sd) & 1u) {
            u = {1.0, 0.0};
            v = {0.0, 0.0};
        }
    };
    // the maps of symbols j0 .. j1 - 1 applied right to left to (u : v)
    auto walk = [&](uint64_t lo, uint64_t hi, int j0, int j1, c64& u, c64& v) {
        for (int j = j1 - 1; j >= j0; --j) {
            const m64& Gx = G[packed_symbol(lo, hi, j)];
            const c64 nu = cfma(Gx.a, u, cmul(Gx.b, v));
            const c64 nv = cfma(Gx.c, u, cmul(Gx.d, v));
            u = nu;
            v = nv;
        }
    };

    if (r > 0) {
        // the tail table: regular words of length r in lexicographic order
        for (int t = threadIdx.x; t < a.n_tails; t += blockDim.x) {
            uint64_t lo, hi;
            int gh = 0;
            m64 unused;
            unrank((uint64_t)t, r, 0, -1, lo, hi, gh, unused, 0);
            int s = 0;
            for (int j = r - 1; j >= 0; --j) s = a.table[s * (m + 1) + packed_symbol(lo, hi, j) + 1];
            TS[t] = (uint8_t)s;
            c64 u, v;
            seed_point(packed_symbol(lo, hi, r - 1), u, v);
            walk(lo, hi, 0, r, u, v);
            TU[t] = u;
            TV[t] = v;
        }
        __syncthreads();
    }

    uint64_t drop = 0;
    uint32_t run_key = kCayleyOutside, run_len = 0;
    auto emit = [&](uint64_t k, double px, double py) {
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
    };
    const uint64_t per = MODE == kCayleyRender ? (uint64_t)a.run : 1;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * per;
    for (uint64_t k0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * per; k0 < a.count; k0 += stride) {
        const uint64_t k1 = k0 + per < a.count ? k0 + per : a.count;
        uint64_t k = k0;
        while (k < k1) {
            int d = D;
            uint64_t local;
            if (MODE == kCayleyEval) {
                local = a.idx[k];
                if (local >= a.depth_start[1]) {
                    a.z_out[k] = {__builtin_nan(""), __builtin_nan("")};
                    ++k;
                    continue;
                }
            } else {
                const uint64_t i = a.first + k;
                d = a.min_depth;
                while (i >= a.depth_start[d - a.min_depth + 1]) ++d;
                local = i - a.depth_start[d - a.min_depth];
            }
            const int hl = (r > 0 && d >= r) ? d - r : -1;   // head length, -1: walk in full
            uint64_t lo, hi;
            int gh = 0;
            m64 Mh = {{1.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {1.0, 0.0}};
            unrank(local, d, 0, hl, lo, hi, gh, Mh, k);
            if (MODE == kCayleyDecode) {
                ++k;
                continue;
            }
            if (hl < 0) {
                c64 u, v;
                seed_point(packed_symbol(lo, hi, d - 1), u, v);
                walk(lo, hi, 0, d, u, v);
                double px, py;
                cayley_pixel(a, u, v, px, py);
                emit(k, px, py);
                ++k;
                continue;
            }
            // rank of the tail among the regular words of length r
            int t = 0;
            {
                int g = 0;
                for (int j = 0; j < r; ++j) {
                    const int y = packed_symbol(lo, hi, hl + j) + 1;
                    const uint64_t* row = CM[r - j - 1];
                    for (int x = 1; x < y; ++x) t += (int)row[NX[g * m + x - 1]];
                    g = NX[g * m + y - 1];
                }
            }
            const uint32_t accept = SETS[gh];   // end states after which the head reads
            while (true) {
                const c64 u = TU[t], v = TV[t];
                double px, py;
                cayley_pixel(a, cfma(Mh.a, u, cmul(Mh.b, v)), cfma(Mh.c, u, cmul(Mh.d, v)), px, py);
                emit(k, px, py);
                ++k;
                if (MODE == kCayleyEval || k >= k1) break;
                do {
                    ++t;
                } while (t < a.n_tails && !((accept >> TS[t]) & 1u));
                if (t >= a.n_tails) break;   // the head's words end here
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

hipError_t launch_cayley(const CayleyJob& job, int mode, hipStream_t s) {
    if (job.count == 0) return hipSuccess;
    CayleyJob j = job;
    const uint64_t threads = 256ull * (uint64_t)std::max(1, j.grid_blocks);
    j.run = (int)std::min<uint64_t>(kCayleyRunMax, std::max<uint64_t>(kCayleyRunMin, j.count / threads));
    const uint64_t per = mode == kCayleyRender ? (uint64_t)j.run : 1;
    uint64_t blocks = (j.count + 256 * per - 1) / (256 * per);
    blocks = std::min<uint64_t>(blocks, (uint64_t)std::max(1, j.grid_blocks));
    if (mode == kCayleyDecode) hipLaunchKernelGGL(cayley_kernel<kCayleyDecode>, dim3((unsigned)blocks), dim3(256), 0, s, j);
    else if (mode == kCayleyEval) hipLaunchKernelGGL(cayley_kernel<kCayleyEval>, dim3((unsigned)blocks), dim3(256), 0, s, j);
    else hipLaunchKernelGGL(cayley_kernel<kCayleyRender>, dim3((unsigned)blocks), dim3(256), 0, s, j);
    return hipGetLastError();
}

}  // namespace kl
