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

// A tail point (u : v) as stored in a tail table: (y : 1) with y = u / v
// where v != 0 and y is in range, else (u : v) unchanged (a point at or near
// infinity).  Tails stored as (y : 1) take the pole form.
__device__ inline void cayley_tail_normalize(c64& u, c64& v) {
    const double n2 = fma_(v.re, v.re, v.im * v.im);
    const c64 y = {fma_(u.re, v.re, u.im * v.im) / n2, fma_(u.im, v.re, -(u.re * v.im)) / n2};
    if (n2 > 0.0 && y.re <= 0x1p32 && y.re >= -0x1p32 && y.im <= 0x1p32 && y.im >= -0x1p32) {
        u = y;
        v = {1.0, 0.0};
    }
}

// A head's map [[a, b], [c, d]] in pole form, for c != 0:
//   h(y) = P + Q / (y + S),  P = a / c,  S = d / c,  Q = -(a d - b c) / c^2,
// with the pixel fold applied (P <- s P + o, Q <- s Q) and the x anisotropy
// folded into the real part's coefficients, so that with u = y + S
//   px = Px + (ax u.re + bx u.im) / |u|^2,  py = Py + (ay u.re + by u.im) / |u|^2;
// the map itself is kept for the ratio form.
struct CayleyHead {
    m64 M;
    c64 S;
    double Px, Py, ax, bx, ay, by;
    bool pole;
};

__device__ inline CayleyHead cayley_head(const CayleyJob& a, const m64& M) {
    CayleyHead h;
    h.M = M;
    const double cn = fma_(M.c.re, M.c.re, M.c.im * M.c.im);
    const double rn = cayley_recip(cn);
    const c64 ic = {M.c.re * rn, -(M.c.im * rn)};
    const c64 P = cmul(M.a, ic);
    h.S = cmul(M.d, ic);
    const c64 det = {fma_(M.a.re, M.d.re, -(M.a.im * M.d.im)) - fma_(M.b.re, M.c.re, -(M.b.im * M.c.im)),
                     fma_(M.a.re, M.d.im, M.a.im * M.d.re) - fma_(M.b.re, M.c.im, M.b.im * M.c.re)};
    const c64 q = cmul(det, cmul(ic, ic));
    const double s = a.fold.s, an = a.fold.aniso;
    h.Px = fma_(s, P.re, a.fold.o.re) * an;
    h.Py = fma_(s, P.im, a.fold.o.im);
    h.ax = -(s * q.re) * an;
    h.bx = -(s * q.im) * an;
    h.ay = -(s * q.im);
    h.by = s * q.re;
    auto in = [](double x, double lim) { return x <= lim && x >= -lim; };   // false for NaN
    h.pole = cn > 0.0 && cn <= 0x1p1000 && in(h.S.re, 0x1p40) && in(h.S.im, 0x1p40) && in(h.ax, 0x1p80) &&
             in(h.bx, 0x1p80) && in(h.ay, 0x1p80) && in(h.by, 0x1p80) && in(h.Px, 0x1p100) && in(h.Py, 0x1p100);
    return h;
}

// Pixel coordinates of head . tail from the tail's stored point (u : v): the
// pole form where the head has one and the point is (y : 1), else the ratio
// form.  Render and eval both come here, so their values agree bit for bit.
__device__ inline void cayley_word(const CayleyJob& a, const CayleyHead& h, c64 u, c64 v, double& px, double& py) {
    if (h.pole && v.re == 1.0 && v.im == 0.0) {
        const double ur = u.re + h.S.re, ui = u.im + h.S.im;
        const double rc = cayley_recip(fma_(ur, ur, ui * ui));
        px = fma_(fma_(h.ax, ur, h.bx * ui), rc, h.Px);
        py = fma_(fma_(h.ay, ur, h.by * ui), rc, h.Py);
    } else {
        cayley_pixel(a, cfma(h.M.a, u, cmul(h.M.b, v)), cfma(h.M.c, u, cmul(h.M.d, v)), px, py);
    }
}

// consecutive words per thread in a render: enough threads to fill the grid,
// runs no shorter than 16 words and no longer than 256
constexpr int kCayleyRunMin = 16, kCayleyRunMax = 256;

// symbol j (0-based, x - 1) of a word packed 3 bits each into lo (0..20) and hi (21..39)
__device__ __forceinline__ int packed_symbol(uint64_t lo, uint64_t hi, int j) {
    return (int)((j < 21 ? lo >> (3 * j) : hi >> (3 * (j - 21))) & 7u);
}

// Wave-level barrier for LDS written and read by the lanes of one wave.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Counts of the regular words by length and end state, C[L * stride + s]
// for L = 0..D, from the table copied to LDS (TB): A[t * S + s] counts the
// symbols that take state s to state t != 0, and C[L][t] = sum over s of
// A[t][s] C[L - 1][s].  The first wave forms the lengths one after another
// (one lane per state); the block is synchronised on return.
__device__ inline void cayley_counts(const uint8_t* TB, uint8_t* A, uint64_t* C, int stride, int S, int m, int D) {
    for (int i = threadIdx.x; i < S * S; i += blockDim.x) {
        const int t = i / S, s = i - t * S;
        int n = 0;
        if (t != 0)
            for (int x = 1; x <= m; ++x) n += TB[s * (m + 1) + x] == t ? 1 : 0;
        A[i] = (uint8_t)n;
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)kWave) {
        const int t = threadIdx.x;
        if (t < S) C[t] = t == 0 ? 1 : 0;
        wave_sync();
        for (int L = 1; L <= D; ++L) {
            if (t < S) {
                uint64_t n = 0;
                for (int s = 0; s < S; ++s) n += (uint64_t)A[t * S + s] * C[(L - 1) * stride + s];
                C[L * stride + t] = n;
            }
            wave_sync();
        }
    }
    __syncthreads();
}

// The good sets reachable from the set of all states form a deterministic
// automaton (next_set); CM[L][g] = sum over s in set g of C[L][s] counts the
// words that begin with a prefix of good set g and have L symbols to go.
// Choosing a symbol is then two table reads per candidate.  A word's
// symbols are packed 3 bits each (x - 1) into two registers.
//
// Decode, eval, and renders of words shorter than r (launch_cayley sends a
// render's words of depth >= r to cayley_head_kernel below).
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
    __shared__ uint8_t TB[kCayleyMaxStates * (kCayleyMaxSymbols + 1)];
    __shared__ uint8_t A[kCayleyMaxStates * kCayleyMaxStates];
    __shared__ uint64_t DS[KL_MAX_DEPTH + 2];
    const int S = a.S, m = a.m, M = a.n_sets, D = a.max_depth;
    const int r = MODE == kCayleyDecode ? 0 : a.r;
    for (int i = threadIdx.x; i < M * m; i += blockDim.x) NX[i] = a.next_set[i];
    for (int i = threadIdx.x; i < M; i += blockDim.x) SETS[i] = a.sets[i];
    for (int i = threadIdx.x; i < m; i += blockDim.x) G[i] = a.maps[i];
    for (int i = threadIdx.x; i < S * (m + 1); i += blockDim.x) TB[i] = a.table[i];
    for (int i = threadIdx.x; i < KL_MAX_DEPTH + 2; i += blockDim.x) DS[i] = a.depth_start[i];
    __syncthreads();
    cayley_counts(TB, A, &C[0][0], kCayleyMaxStates, S, m, D);
    for (int i = threadIdx.x; i < (D + 1) * M; i += blockDim.x) {
        const int L = i / M, g = i - L * M;
        uint64_t n = 0;
        for (int s = 0; s < S; ++s)
            if ((SETS[g] >> s) & 1u) n += C[L][s];
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
            for (int j = r - 1; j >= 0; --j) s = TB[s * (m + 1) + packed_symbol(lo, hi, j) + 1];
            TS[t] = (uint8_t)s;
            c64 u, v;
            seed_point(packed_symbol(lo, hi, r - 1), u, v);
            walk(lo, hi, 0, r, u, v);
            cayley_tail_normalize(u, v);
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
                if (local >= DS[1]) {
                    a.z_out[k] = {__builtin_nan(""), __builtin_nan("")};
                    ++k;
                    continue;
                }
            } else {
                const uint64_t i = a.first + k;
                d = a.min_depth;
                while (i >= DS[d - a.min_depth + 1]) ++d;
                local = i - DS[d - a.min_depth];
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
            const CayleyHead ch = cayley_head(a, Mh);
            while (true) {
                double px, py;
                cayley_word(a, ch, TU[t], TV[t], px, py);
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

// ------------------------------------------------------------------ one head per thread
// Render of the words of depths >= r: a thread takes a whole head (the
// first d - r symbols) and walks the list of tails its head's good set
// accepts (built per block in LDS), so no lane re-ranks in the middle of a
// run or steps over a tail it rejects.  Heads are ranked by their own
// counts: NH[L][g] heads of L more symbols from good set g accept at least
// one tail (NH[0][g] = [CM[r][g] > 0]), so head hh of a depth unranks as a
// word does, with NH in place of CM, while the skipped CM counts give the
// index of the head's first word.  The accepted tails of a head, in table
// (lexicographic) order, are its words in index order; an index range cuts
// the first and last of its heads.  The arithmetic of a word is that of
// cayley_kernel: the head's FP64 product left to right, then cayley_pixel.
//
// LDS, sized from the table (HeadLayout): C, CM and NH rows for lengths
// 0..D, the set automaton, the maps, the tail table, and per depth the
// range's head offsets.
struct HeadLayout {
    // byte offsets: C, CM, NH rows ([(D + 1) * S], [(D + 1) * M] twice); per
    // depth (index d - min_depth) the range's first head HA, the prefix of
    // head counts HS and the word range WA, WB; the tail points TU, TV; the
    // maps G; the sets SETS; the automaton NX; the tail end states TS; and
    // per good set g the tails it accepts, in table order, at AL[g * n_tails]
    uint32_t C, CM, NH, HA, HS, WA, WB, TU, TV, G, SETS, NX, TS, AL, TB, A, total;
};

__host__ __device__ inline HeadLayout cayley_head_layout(int S, int M, int m, int D, int n_tails, int n_seeds) {
    HeadLayout L;
    uint32_t off = 0;
    auto take = [&](uint32_t bytes) {
        const uint32_t at = off;
        off = (off + bytes + 15u) & ~15u;
        return at;
    };
    const uint32_t rows = (uint32_t)(D + 1);
    L.C = take(rows * (uint32_t)S * 8u);
    L.CM = take(rows * (uint32_t)M * 8u);
    L.NH = take(rows * (uint32_t)M * 8u);
    L.HA = take((KL_MAX_DEPTH + 1) * 8u);
    L.HS = take((KL_MAX_DEPTH + 2) * 8u);
    L.WA = take((KL_MAX_DEPTH + 1) * 8u);
    L.WB = take((KL_MAX_DEPTH + 1) * 8u);
    L.TU = take((uint32_t)n_seeds * (uint32_t)n_tails * (uint32_t)sizeof(c64));
    L.TV = take((uint32_t)n_seeds * (uint32_t)n_tails * (uint32_t)sizeof(c64));
    L.G = take((uint32_t)m * (uint32_t)sizeof(m64));
    L.SETS = take((uint32_t)M * 2u);
    L.NX = take((uint32_t)M * (uint32_t)m);
    L.TS = take((uint32_t)n_tails);
    L.AL = take((uint32_t)M * (uint32_t)n_tails * 2u);
    L.TB = take((uint32_t)S * (uint32_t)(m + 1));
    L.A = take((uint32_t)S * (uint32_t)S);
    L.total = off;
    return L;
}

// Workgroup of the head kernel.  Every workgroup builds the count tables
// and its seeds' tail tables in LDS, and two of them share a CU: 512 threads
// give 16 waves a CU to hide the latency of the FP64 head products and LDS
// reads.  On Table 2 at depth 16 and the PSL(2, Z) tiling, 256 threads took
// 0.215 / 0.225 ms, 512 threads 0.167 / 0.198 ms, 768 0.195 / 0.195 ms, 1024
// 0.19 / 0.26 ms; 512 threads with four workgroups a CU 0.169 / 0.236 ms.
constexpr unsigned kCayleyHeadBlock = 512;

__global__ __launch_bounds__(kCayleyHeadBlock) void cayley_head_kernel(const CayleyJob a) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int S = a.S, m = a.m, M = a.n_sets, D = a.max_depth, r = a.r;
    const int NT = a.n_tails, NS = a.n_seeds;
    const HeadLayout lay = cayley_head_layout(S, M, m, D, NT, NS);
    struct {
        uint64_t *C, *CM, *NH, *HA, *HS, *WA, *WB;
        c64 *TU, *TV;
        m64* G;
        uint16_t* SETS;
        uint8_t *NX, *TS;
        uint16_t* AL;
        uint8_t *TB, *A;
    } q = {(uint64_t*)(lds + lay.C), (uint64_t*)(lds + lay.CM), (uint64_t*)(lds + lay.NH), (uint64_t*)(lds + lay.HA),
           (uint64_t*)(lds + lay.HS), (uint64_t*)(lds + lay.WA), (uint64_t*)(lds + lay.WB), (c64*)(lds + lay.TU),
           (c64*)(lds + lay.TV), (m64*)(lds + lay.G), (uint16_t*)(lds + lay.SETS), (uint8_t*)(lds + lay.NX),
           (uint8_t*)(lds + lay.TS), (uint16_t*)(lds + lay.AL), (uint8_t*)(lds + lay.TB), (uint8_t*)(lds + lay.A)};
    for (int i = threadIdx.x; i < M * m; i += blockDim.x) q.NX[i] = a.next_set[i];
    for (int i = threadIdx.x; i < M; i += blockDim.x) q.SETS[i] = a.sets[i];
    for (int i = threadIdx.x; i < m; i += blockDim.x) q.G[i] = a.maps[i];
    for (int i = threadIdx.x; i < S * (m + 1); i += blockDim.x) q.TB[i] = a.table[i];
    __syncthreads();
    cayley_counts(q.TB, q.A, q.C, S, S, m, D);
    for (int i = threadIdx.x; i < (D + 1) * M; i += blockDim.x) {
        const int L = i / M, g = i - L * M;
        uint64_t n = 0;
        for (int s = 0; s < S; ++s)
            if ((q.SETS[g] >> s) & 1u) n += q.C[L * S + s];
        q.CM[i] = n;
    }
    __syncthreads();
    // heads of L more symbols that accept at least one tail: the first wave,
    // one lane per good set, one length after another
    static_assert(kCayleyMaxSets <= kWave, "one lane per good set");
    if (threadIdx.x < (unsigned)kWave) {
        const int g = threadIdx.x;
        if (g < M) q.NH[g] = q.CM[r * M + g] > 0 ? 1 : 0;
        wave_sync();
        for (int L = 1; L + r <= D; ++L) {
            if (g < M) {
                uint64_t n = 0;
                for (int x = 1; x <= m; ++x) n += q.NH[(L - 1) * M + q.NX[g * m + x - 1]];
                q.NH[L * M + g] = n;
            }
            wave_sync();
        }
    }
    __syncthreads();
    // the tail table: regular words of length r in lexicographic order, their
    // end states, and their points from each seed in turn (TU[slot * NT + t])
    for (int e = threadIdx.x; e < NS * NT; e += blockDim.x) {
        const int slot = e / NT, t = e - slot * NT;
        uint64_t local = (uint64_t)t, lo = 0, hi = 0;
        int g = 0;
        for (int j = 0; j < r; ++j) {
            int x = 1, gx = 0;
            for (; x <= m; ++x) {
                gx = q.NX[g * m + x - 1];
                const uint64_t n = q.CM[(r - j - 1) * M + gx];
                if (local < n) break;
                local -= n;
            }
            g = gx;
            if (j < 21) lo |= (uint64_t)(x - 1) << (3 * j);
            else hi |= (uint64_t)(x - 1) << (3 * (j - 21));
        }
        int s = 0;
        for (int j = r - 1; j >= 0; --j) s = q.TB[s * (m + 1) + packed_symbol(lo, hi, j) + 1];
        if (slot == 0) q.TS[t] = (uint8_t)s;
        const int last = packed_symbol(lo, hi, r - 1);
        const int sd = a.seed_list[slot] < 0 ? last : a.seed_list[slot];
        c64 u = a.fix[sd], v = {1.0, 0.0};
        if ((a.inf_mask >> sd) & 1u) {
            u = {1.0, 0.0};
            v = {0.0, 0.0};
        }
        for (int j = r - 1; j >= 0; --j) {
            const m64& Gx = q.G[packed_symbol(lo, hi, j)];
            const c64 nu = cfma(Gx.a, u, cmul(Gx.b, v));
            const c64 nv = cfma(Gx.c, u, cmul(Gx.d, v));
            u = nu;
            v = nv;
        }
        cayley_tail_normalize(u, v);
        q.TU[e] = u;
        q.TV[e] = v;
    }
    __syncthreads();
    // per good set, the tails it accepts in table order
    for (int g = threadIdx.x; g < M; g += blockDim.x) {
        int k = 0;
        for (int t = 0; t < a.n_tails; ++t)
            if ((q.SETS[g] >> q.TS[t]) & 1u) q.AL[g * a.n_tails + k++] = (uint16_t)t;
    }
    // per depth: the range's local word interval and the heads it touches
    const int d0 = r > a.min_depth ? r : a.min_depth;
    for (int e = threadIdx.x; e < 2 * (D - d0 + 1); e += blockDim.x) {
        const int d = d0 + e / 2, di = d - a.min_depth;
        const uint64_t s0 = a.depth_start[di], s1 = a.depth_start[di + 1];
        const uint64_t lo_w = a.first > s0 ? a.first - s0 : 0;
        const uint64_t end = a.first + a.count;
        const uint64_t hi_w = end < s1 ? (end > s0 ? end - s0 : 0) : s1 - s0;
        if (e % 2 == 0) {
            q.WA[di] = lo_w;
            q.WB[di] = hi_w;
        }
        // rank of the head of word lo_w (e even) or hi_w - 1 (e odd)
        uint64_t hr = 0;
        if (hi_w > lo_w) {
            uint64_t local = e % 2 == 0 ? lo_w : hi_w - 1;
            const int hl = d - r;
            int g = 0;
            for (int j = 0; j < hl; ++j) {
                int x = 1, gx = 0;
                for (; x <= m; ++x) {
                    gx = q.NX[g * m + x - 1];
                    const uint64_t n = q.CM[(d - j - 1) * M + gx];
                    if (local < n) break;
                    local -= n;
                    hr += q.NH[(hl - j - 1) * M + gx];
                }
                g = gx;
            }
        }
        if (e % 2 == 0) q.HA[di] = hr;
        else q.HS[di] = hr;   // the last head, turned into a count below
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t total = 0;
        for (int d = d0; d <= D; ++d) {
            const int di = d - a.min_depth;
            const uint64_t n = q.WB[di] > q.WA[di] ? q.HS[di] - q.HA[di] + 1 : 0;
            q.HS[di] = total;
            total += n;
        }
        q.HS[D - a.min_depth + 1] = total;
    }
    __syncthreads();

    // (seed, head) pairs, seed-major so that the lanes of a wave share a seed
    const uint64_t total = q.HS[D - a.min_depth + 1];
    uint64_t drop = 0;
    uint32_t run_key = kCayleyOutside, run_len = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t uu = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; uu < total * (uint64_t)NS; uu += stride) {
        const int slot = (int)(uu / total);
        const uint64_t u = uu - (uint64_t)slot * total;
        const c64* TU = q.TU + (size_t)slot * NT;
        const c64* TV = q.TV + (size_t)slot * NT;
        int d = d0;
        while (u >= q.HS[d + 1 - a.min_depth]) ++d;
        const int di = d - a.min_depth, hl = d - r;
        uint64_t hh = q.HA[di] + (u - q.HS[di]);
        // unrank the head by NH; the skipped CM counts give its first word
        int g = 0;
        uint64_t wstart = 0;
        m64 Mh = {{1.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {1.0, 0.0}};
        for (int j = 0; j < hl; ++j) {
            int x = 1, gx = 0;
            for (; x <= m; ++x) {
                gx = q.NX[g * m + x - 1];
                const uint64_t n = q.NH[(hl - j - 1) * M + gx];
                if (hh < n) break;
                hh -= n;
                wstart += q.CM[(d - j - 1) * M + gx];
            }
            g = gx;
            Mh = mmul(Mh, q.G[x - 1]);
        }
        // this head's accepted tails with ordinals in [o0, o1) are words of the range
        const uint64_t wa = q.WA[di], wb = q.WB[di], n_acc = q.CM[r * M + g];
        const uint32_t o0 = (uint32_t)(wa > wstart ? wa - wstart : 0);
        const uint32_t o1 = (uint32_t)(wb - wstart < n_acc ? wb - wstart : n_acc);
        const uint16_t* list = q.AL + (size_t)g * a.n_tails;
        const CayleyHead ch = cayley_head(a, Mh);
        for (uint32_t i = o0; i < o1; ++i) {
            const int t = list[i];
            double px, py;
            cayley_word(a, ch, TU[t], TV[t], px, py);
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
    if (run_key == kCayleyOutside) drop += run_len;
    else if (run_len) atomicAdd(a.image + run_key, run_len);
    if (a.dropped) {
        for (int off = kWave / 2; off > 0; off >>= 1) drop += __shfl_down(drop, off, kWave);
        if ((threadIdx.x & (kWave - 1)) == 0 && drop) atomicAdd((unsigned long long*)a.dropped, (unsigned long long)drop);
    }
}

hipError_t launch_cayley(const CayleyJob& job, int mode, hipStream_t s) {
    if (job.count == 0) return hipSuccess;
    CayleyJob j = job;
    const uint64_t threads = 256ull * (uint64_t)std::max(1, j.grid_blocks);
    j.run = (int)std::min<uint64_t>(kCayleyRunMax, std::max<uint64_t>(kCayleyRunMin, j.count / threads));
    if (mode == kCayleyRender && j.r > 0) {
        // words of depths >= r go one head per thread; shorter words keep the per-word path
        const uint64_t B = j.r > j.min_depth ? j.depth_start[j.r - j.min_depth] : 0;   // first word of depth r
        const uint64_t end = j.first + j.count;
        if (end > B) {
            CayleyJob h = j;
            h.first = j.first > B ? j.first : B;
            h.count = end - h.first;
            // as many seeds per launch as their tail tables fit the LDS of a CU
            const size_t cap = 160 * 1024;
            int per = j.n_seeds;
            while (per > 1 && cayley_head_layout(j.S, j.n_sets, j.m, j.max_depth, j.n_tails, per).total > cap) --per;
            for (int k0 = 0; k0 < j.n_seeds; k0 += per) {
                h.n_seeds = std::min(per, j.n_seeds - k0);
                for (int k = 0; k < h.n_seeds; ++k) h.seed_list[k] = j.seed_list[k0 + k];
                const size_t lds = cayley_head_layout(j.S, j.n_sets, j.m, j.max_depth, j.n_tails, h.n_seeds).total;
                if (lds > 65536) {
                    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(cayley_head_kernel),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
                    if (e != hipSuccess) return e;
                }
                hipLaunchKernelGGL(cayley_head_kernel, dim3((unsigned)std::max(1, j.grid_blocks)), dim3(kCayleyHeadBlock),
                                   lds, s, h);
                hipError_t e = hipGetLastError();
                if (e != hipSuccess) return e;
            }
        }
        if (j.first >= B) return hipSuccess;
        // the words shorter than r, each walked in full by a thread of its own
        // (no tail table), one launch per seed
        j.count = (end < B ? end : B) - j.first;
        j.r = 0;
        j.n_tails = 0;
        j.run = 1;
        const uint64_t blocks = std::min<uint64_t>((j.count + 255) / 256, (uint64_t)std::max(1, j.grid_blocks));
        for (int k = 0; k < j.n_seeds; ++k) {
            j.seed = j.seed_list[k];
            hipLaunchKernelGGL(cayley_kernel<kCayleyRender>, dim3((unsigned)blocks), dim3(256), 0, s, j);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    const uint64_t per = mode == kCayleyRender ? (uint64_t)j.run : 1;
    uint64_t blocks = (j.count + 256 * per - 1) / (256 * per);
    blocks = std::min<uint64_t>(blocks, (uint64_t)std::max(1, j.grid_blocks));
    if (mode == kCayleyDecode) hipLaunchKernelGGL(cayley_kernel<kCayleyDecode>, dim3((unsigned)blocks), dim3(256), 0, s, j);
    else if (mode == kCayleyEval) hipLaunchKernelGGL(cayley_kernel<kCayleyEval>, dim3((unsigned)blocks), dim3(256), 0, s, j);
    else hipLaunchKernelGGL(cayley_kernel<kCayleyRender>, dim3((unsigned)blocks), dim3(256), 0, s, j);
    return hipGetLastError();
}

}  // namespace kl
