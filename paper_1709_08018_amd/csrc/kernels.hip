// kernels.hip -- gfx950 kernels of libkl.
//
// Word model (Sections 1 and 3 of the paper): a reduced word w1..wd over
// {a, b, A, B}; its value is G_{w1}(G_{w2}(...G_{wd}(z0))) with z0 the
// attracting fixed point of wd.  Index order (Sections 4 and 6): the
// first letter is the most significant base-4 digit, every later letter a
// base-3 digit t read as the t-th letter that is not the inverse of its
// predecessor.
//
// Work split used here (not the paper's; the paper scans all 4^d strings
// and rejects crash words).  A depth-d word is head . tail, head = k + m
// letters, tail = r letters:
//   * the first k letters pick an FP64 prefix product from a table built
//     once per render (prefix_table_kernel);
//   * each lane of the renderer owns one head: it appends its m letters in
//     FP64, folds the window map into the product, scales it by a power of
//     two and rounds it once to the working precision;
//   * the r tail letters run through a table of suffix points
//     G_{y1}(...G_{y(r-1)}(fix(yr))) built right to left in the working
//     precision (tail_table_kernel), held in LDS; the lane walks the 3^r
//     tails allowed after its head's last letter in index order.
// The value of head . tail is then one Moebius map of one point, computed
// by eval_point() below, which every kernel shares.
#include <algorithm>
#include <type_traits>

#include "kl_internal.hpp"

namespace kl {

__device__ __forceinline__ int inv_letter(int c) { return c ^ 2; }

// ------------------------------------------------------------------ fill
__global__ void fill_u32_kernel(uint32_t* p, uint64_t n, uint32_t v) {
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}
__global__ void fill_u64_kernel(uint64_t* p, uint64_t n, uint64_t v) {
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}
hipError_t launch_fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// ------------------------------------------------------------------ digits
// x / 3 and x % 3 without a divide instruction sequence.
__device__ __forceinline__ uint64_t div3_u64(uint64_t x) { return __umul64hi(x, 0xAAAAAAAAAAAAAAABull) >> 1; }
__device__ __forceinline__ uint32_t div3_u32(uint32_t x) { return __umulhi(x, 0xAAAAAAABu) >> 1; }

// Letters of word `index` of length n (n <= 32), packed 2 bits per letter,
// letter j (leftmost = 0) at bits 2j..2j+1.
__device__ inline uint64_t decode_packed(uint64_t index, int n) {
    // base-3 digits from the least significant end; the remaining
    // quotient is the first letter (0..3).
    uint64_t digits = 0;
    uint64_t x = index;
    int j = n - 1;
    for (; j >= 1 && (x >> 32); --j) {
        uint64_t q = div3_u64(x);
        digits |= (x - 3 * q) << (2 * j);
        x = q;
    }
    uint32_t x32 = (uint32_t)x;
    for (; j >= 1; --j) {
        uint32_t q = div3_u32(x32);
        digits |= (uint64_t)(x32 - 3 * q) << (2 * j);
        x32 = q;
    }
    // digits -> letters, left to right
    uint64_t letters = x32;  // first letter
    int prev = (int)x32;
    for (int i = 1; i < n; ++i) {
        int t = (int)((digits >> (2 * i)) & 3);
        int c = t + (t >= inv_letter(prev));
        letters |= (uint64_t)c << (2 * i);
        prev = c;
    }
    return letters;
}

// ------------------------------------------------------------------ decode
// One thread per word; letters staged in LDS and written out as one
// contiguous, coalesced byte range per workgroup.
__global__ __launch_bounds__(256) void decode_kernel(uint64_t first, uint64_t count, int depth,
                                                     uint8_t* __restrict__ out) {
    __shared__ uint8_t stage[256 * KL_MAX_DEPTH];
    const uint64_t block_first = (uint64_t)blockIdx.x * 256;
    const int tid = threadIdx.x;
    const uint64_t rem = count - block_first;
    const int nw = rem < 256 ? (int)rem : 256;
    if (tid < nw) {
        const uint64_t index = first + block_first + tid;
        // digits from the least significant end into LDS, then letters
        uint8_t* w = stage + tid * depth;
        uint64_t x = index;
        int j = depth - 1;
        for (; j >= 1 && (x >> 32); --j) {
            uint64_t q = div3_u64(x);
            w[j] = (uint8_t)(x - 3 * q);
            x = q;
        }
        uint32_t x32 = (uint32_t)x;
        for (; j >= 1; --j) {
            uint32_t q = div3_u32(x32);
            w[j] = (uint8_t)(x32 - 3 * q);
            x32 = q;
        }
        int prev = (int)x32;
        w[0] = (uint8_t)prev;
        for (int i = 1; i < depth; ++i) {
            int t = w[i];
            int c = t + (t >= inv_letter(prev));
            w[i] = (uint8_t)c;
            prev = c;
        }
    }
    __syncthreads();
    const uint64_t nbytes = (uint64_t)nw * depth;
    uint8_t* dst = out + block_first * depth;
    // 4-byte stores where the destination is aligned, bytes at the edges
    const uintptr_t addr = (uintptr_t)dst;
    const uint32_t lead = (uint32_t)((4 - (addr & 3)) & 3);
    const uint32_t head = lead < nbytes ? lead : (uint32_t)nbytes;
    if ((uint32_t)tid < head) dst[tid] = stage[tid];
    const uint64_t body = (nbytes - head) / 4;
    uint32_t* dst32 = (uint32_t*)(dst + head);
    for (uint64_t i = tid; i < body; i += 256) {
        const uint8_t* s = stage + head + 4 * i;
        dst32[i] = (uint32_t)s[0] | ((uint32_t)s[1] << 8) | ((uint32_t)s[2] << 16) | ((uint32_t)s[3] << 24);
    }
    const uint64_t tail_start = head + body * 4;
    if ((uint64_t)tid < nbytes - tail_start) dst[tail_start + tid] = stage[tail_start + tid];
}

hipError_t launch_decode(uint64_t first, uint64_t count, int depth, uint8_t* out, hipStream_t s) {
    uint64_t blocks = (count + 255) / 256;
    // grid.x is limited to 2^31 - 1 blocks; kl_decode splits larger requests
    while (blocks) {
        uint64_t nb = blocks > 0x7FFFFFFFull ? 0x7FFFFFFFull : blocks;
        uint64_t words = nb * 256 < count ? nb * 256 : count;
        hipLaunchKernelGGL(decode_kernel, dim3((unsigned)nb), dim3(256), 0, s, first, words, depth, out);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        first += words;
        out += words * depth;
        count -= words;
        blocks -= nb;
    }
    return hipSuccess;
}

// ------------------------------------------------------------------ prefix table
// P_p = G_{w1} G_{w2} ... G_{wk} in FP64, left to right, for every prefix p
// of length k (k <= 14), and its last letter.
__device__ inline void prefix_entry(const Gens& g, int k, uint32_t p, m64* __restrict__ table,
                                    uint8_t* __restrict__ last) {
    const uint64_t w = decode_packed(p, k);
    int c = (int)(w & 3);
    m64 M = g.g[c];
    for (int j = 1; j < k; ++j) {
        c = (int)((w >> (2 * j)) & 3);
        M = mmul(M, g.g[c]);
    }
    table[p] = M;
    last[p] = (uint8_t)c;
}

__global__ __launch_bounds__(256) void prefix_table_kernel(Gens g, int k, uint32_t n,
                                                           m64* __restrict__ table,
                                                           uint8_t* __restrict__ last) {
    const uint32_t p = blockIdx.x * 256 + threadIdx.x;
    if (p < n) prefix_entry(g, k, p, table, last);
}

hipError_t launch_prefix_table(const Gens& g, int k, m64* prefix, uint8_t* last, hipStream_t s) {
    const uint32_t n = (uint32_t)num_words(k);
    hipLaunchKernelGGL(prefix_table_kernel, dim3((n + 255) / 256), dim3(256), 0, s, g, k, n, prefix, last);
    return hipGetLastError();
}

// ------------------------------------------------------------------ tail table
template <typename T>
__device__ inline void scale_pow2(cpx<T>& u, cpx<T>& v) {
    T m = fmax(fmax(fabs(u.re), fabs(u.im)), fmax(fabs(v.re), fabs(v.im)));
    if (m > T(0) && m <= T(1e300)) {
        int e;
        frexp((double)m, &e);
        const T f = (T)ldexp(1.0, -e);
        u.re *= f; u.im *= f; v.re *= f; v.im *= f;
    }
}

// Suffix point of tail t (length r, r <= 8): the homogeneous pair (u, v)
// of G_{y1}(...G_{y(r-1)}(fix(yr))) walked right to left in precision T
// from the rounded seed with the rounded generators (G_{yr} fixes its own
// seed and is not applied), rescaled by powers of two after every step;
// and its affine form y = u / v.
template <typename T>
__device__ inline void tail_entry(const Gens& g, int r, uint32_t t, cpx<T>* __restrict__ affine,
                                  cpx<T>* __restrict__ homog, uint32_t* __restrict__ flags, bool atomic = true) {
    const uint64_t w = decode_packed(t, r);
    const int last = (int)((w >> (2 * (r - 1))) & 3);
    cpx<T> u = {(T)g.fix[last].re, (T)g.fix[last].im};
    cpx<T> v = {T(1), T(0)};
    for (int j = r - 2; j >= 0; --j) {
        const m64& G = g.g[(w >> (2 * j)) & 3];
        const cpx<T> a = {(T)G.a.re, (T)G.a.im}, b = {(T)G.b.re, (T)G.b.im};
        const cpx<T> c = {(T)G.c.re, (T)G.c.im}, d = {(T)G.d.re, (T)G.d.im};
        const cpx<T> nu = cfma(a, u, cmul(b, v));
        const cpx<T> nv = cfma(c, u, cmul(d, v));
        u = nu;
        v = nv;
        scale_pow2(u, v);
    }
    homog[2 * t] = u;
    homog[2 * t + 1] = v;
    const T n2 = fma_(v.re, v.re, v.im * v.im);
    cpx<T> y = {(fma_(u.re, v.re, u.im * v.im)) / n2, (fma_(u.im, v.re, -(u.re * v.im))) / n2};
    const bool ok = n2 > T(0) && isfinite(y.re) && isfinite(y.im) && fabs(y.re) <= T(kAffineLimit) &&
                    fabs(y.im) <= T(kAffineLimit);
    if (!ok) {
        if (atomic) atomicOr(flags, 1u);
        else *flags = 1u;
        y = {T(0), T(0)};
    }
    affine[t] = y;
}

template <typename T>
__global__ __launch_bounds__(256) void tail_table_kernel(Gens g, int r, uint32_t n,
                                                         cpx<T>* __restrict__ affine,
                                                         cpx<T>* __restrict__ homog,
                                                         uint32_t* __restrict__ flags) {
    const uint32_t t = blockIdx.x * 256 + threadIdx.x;
    if (t < n) tail_entry<T>(g, r, t, affine, homog, flags);
}

hipError_t launch_tail_table(const Gens& g, int r, int precision, void* tail_affine, void* tail_homog,
                             uint32_t* flags, hipStream_t s) {
    const uint32_t n = (uint32_t)num_words(r);
    if (precision == KL_PREC_FP64)
        hipLaunchKernelGGL(tail_table_kernel<double>, dim3((n + 255) / 256), dim3(256), 0, s, g, r, n,
                           (c64*)tail_affine, (c64*)tail_homog, flags);
    else
        hipLaunchKernelGGL(tail_table_kernel<float>, dim3((n + 255) / 256), dim3(256), 0, s, g, r, n,
                           (c32*)tail_affine, (c32*)tail_homog, flags);
    return hipGetLastError();
}

// ------------------------------------------------------------------ fused set-up
// One launch that clears the image and the dropped counter, builds the
// FP64 prefix table (blocks 1..) and the suffix table (block 0, which also
// decides the suffix form without a separate clear of the flag).
struct SetupArgs {
    Gens g;
    int k, r;
    uint32_t n_prefix, n_tail;
    m64* prefix;
    uint8_t* last;
    void* aff;
    void* hom;
    uint32_t* flags;
    int force_homog;
    uint32_t* image;      // null: leave the image alone
    uint64_t bins;
    uint64_t* dropped;    // null: leave the counter alone
};

template <typename T>
__global__ __launch_bounds__(256) void setup_kernel(const SetupArgs a) {
    if (a.image) {
        const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
        const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
        if (((uintptr_t)a.image & 15) == 0) {
            const uint64_t n4 = a.bins / 4;
            uint4* p4 = (uint4*)a.image;
            for (uint64_t i = tid; i < n4; i += stride) p4[i] = make_uint4(0, 0, 0, 0);
            for (uint64_t i = n4 * 4 + tid; i < a.bins; i += stride) a.image[i] = 0;
        } else {
            for (uint64_t i = tid; i < a.bins; i += stride) a.image[i] = 0;
        }
    }
    if (blockIdx.x == 0) {
        uint32_t bad = 0;
        for (uint32_t t = threadIdx.x; t < a.n_tail; t += blockDim.x) {
            uint32_t f = 0;
            tail_entry<T>(a.g, a.r, t, (cpx<T>*)a.aff, (cpx<T>*)a.hom, &f, false);
            bad |= f;
        }
        bad = __syncthreads_or(bad);
        if (threadIdx.x == 0) {
            a.flags[0] = (bad || a.force_homog) ? 1u : 0u;
            if (a.dropped) a.dropped[0] = 0;
        }
    } else {
        const uint32_t p = (blockIdx.x - 1) * 256 + threadIdx.x;
        if (p < a.n_prefix) prefix_entry(a.g, a.k, p, a.prefix, a.last);
    }
}

// ------------------------------------------------------------------ shared arithmetic
template <typename T>
struct Head {
    cpx<T> A, B, C, D;  // window-folded head map, scaled by a power of two
    int e;              // last letter of the head, -1 for the empty head
};

template <typename T>
__device__ __forceinline__ T conv(double x) { return (T)x; }

// Head map of head index hidx: prefix-table product of its first k letters
// times its m lane letters (FP64, left to right), window folded
// (A, B) <- s (A, B) + o (C, D), scaled by a power of two, rounded to T.
template <typename T>
__device__ inline Head<T> compute_head(uint64_t hidx, const Split& sp, const m64* __restrict__ prefix,
                                       const uint8_t* __restrict__ plast, const m64* G, const Fold& f) {
    m64 M;
    int e;
    if (sp.k + sp.m == 0) {
        M = {{1.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {1.0, 0.0}};
        e = -1;
    } else {
        uint64_t p;
        uint64_t u;
        if (sp.m == 0) {
            p = hidx;
            u = 0;
        } else if (hidx >> 32) {
            p = hidx / sp.pow3_m;
            u = hidx - p * sp.pow3_m;
        } else {
            const uint32_t h32 = (uint32_t)hidx;
            const uint32_t p32 = h32 / sp.pow3_m;
            p = p32;
            u = h32 - p32 * sp.pow3_m;
        }
        M = prefix[p];
        e = plast[p];
        // lane letters: base-3 digits of u, most significant first
        uint64_t packed = 0;
        for (int j = 0; j < sp.m; ++j) {
            const uint64_t q = u / 3;
            packed |= (u - 3 * q) << (2 * j);
            u = q;
        }
        for (int j = sp.m - 1; j >= 0; --j) {
            const int t = (int)((packed >> (2 * j)) & 3);
            const int c = t + (t >= inv_letter(e));
            M = mmul(M, G[c]);
            e = c;
        }
    }
    const c64 sa = {f.s * M.a.re, f.s * M.a.im};
    const c64 sb = {f.s * M.b.re, f.s * M.b.im};
    c64 A = cfma(f.o, M.c, sa);
    c64 B = cfma(f.o, M.d, sb);
    c64 C = M.c, D = M.d;
    double mx = fmax(fmax(fmax(fabs(A.re), fabs(A.im)), fmax(fabs(B.re), fabs(B.im))),
                     fmax(fmax(fabs(C.re), fabs(C.im)), fmax(fabs(D.re), fabs(D.im))));
    if (mx > 0.0 && mx <= 1e300) {
        int ex;
        frexp(mx, &ex);
        const double sc = ldexp(1.0, -ex);
        A.re *= sc; A.im *= sc; B.re *= sc; B.im *= sc;
        C.re *= sc; C.im *= sc; D.re *= sc; D.im *= sc;
    }
    Head<T> h;
    h.A = {conv<T>(A.re), conv<T>(A.im)};
    h.B = {conv<T>(B.re), conv<T>(B.im)};
    h.C = {conv<T>(C.re), conv<T>(C.im)};
    h.D = {conv<T>(D.re), conv<T>(D.im)};
    h.e = e;
    return h;
}

__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// Value of one word: the head map applied to the suffix point y (affine
// form), in pixel coordinates when the head carries the window fold.
// x * y + z with the y.re products accumulated first, the order in which
// the matrix cores (v_mfma_f32_4x4x1f32, an exact FMA per K step) form it.
template <typename T>
__device__ __forceinline__ cpx<T> cfma_kre(cpx<T> x, cpx<T> y, cpx<T> z) {
    return {fma_(-x.im, y.im, fma_(x.re, y.re, z.re)), fma_(x.re, y.im, fma_(x.im, y.re, z.im))};
}

// The part of a word's value after its homogeneous numerator and
// denominator: complex division folded into pixel units.
template <typename T, bool ANISO>
__device__ __forceinline__ void finish_point(cpx<T> num, cpx<T> den, T aniso, T& px, T& py) {
    const T n2 = fma_(den.re, den.re, den.im * den.im);
    const T rc = recip(n2);
    const T re = fma_(num.re, den.re, num.im * den.im);
    const T im = fma_(num.im, den.re, -(num.re * den.im));
    px = re * rc;
    py = im * rc;
    if (ANISO) px = px * aniso;
}

template <typename T, bool ANISO>
__device__ __forceinline__ void eval_point(const Head<T>& h, cpx<T> y, T aniso, T& px, T& py) {
    finish_point<T, ANISO>(cfma_kre(h.A, y, h.B), cfma_kre(h.C, y, h.D), aniso, px, py);
}

// Same with the suffix point in homogeneous form (p : q).
template <typename T, bool ANISO>
__device__ __forceinline__ void eval_point_h(const Head<T>& h, cpx<T> p, cpx<T> q, T aniso, T& px, T& py) {
    const cpx<T> num = cfma(h.A, p, cmul(h.B, q));
    const cpx<T> den = cfma(h.C, p, cmul(h.D, q));
    const T n2 = fma_(den.re, den.re, den.im * den.im);
    const T rc = recip(n2);
    const T re = fma_(num.re, den.re, num.im * den.im);
    const T im = fma_(num.im, den.re, -(num.re * den.im));
    px = re * rc;
    py = im * rc;
    if (ANISO) px = px * aniso;
}

// Bin of pixel coordinates, or kOutside when outside [0,W) x [0,H) or NaN.
constexpr uint32_t kOutside = 0xFFFFFFFFu;

// floor(x) as int32, saturating (v_cvt_flr_i32_f32; NaN gives 0, which the
// caller rejects separately)
__device__ __forceinline__ int floor_i32(float x) {
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

__device__ __forceinline__ uint32_t bin_key(float px, float py, uint32_t W, uint32_t H) {
    const uint32_t col = (uint32_t)floor_i32(px);
    const uint32_t row = (uint32_t)floor_i32(py);
    const bool ok = !__builtin_isunordered(px, py) & (col < W) & (row < H);
    return ok ? __umul24(row, W) + col : kOutside;
}

__device__ __forceinline__ uint32_t bin_key(double px, double py, uint32_t W, uint32_t H) {
    const bool ok = (px >= 0.0) & (px < (double)W) & (py >= 0.0) & (py < (double)H);
    const uint32_t col = ok ? (uint32_t)px : 0u;
    const uint32_t row = ok ? (uint32_t)py : 0u;
    return ok ? __umul24(row, W) + col : kOutside;
}

// ------------------------------------------------------------------ persistent renderer
struct RenderArgs {
    Split sp;
    Fold fold;
    Gens gens;
    Tables tab;
    const void* tail_homog;
    uint32_t* image;
    uint32_t W, H;
    uint64_t* dropped;
    uint64_t head_begin;   // the heads [head_begin, head_begin + n_heads) are rendered,
    uint64_t n_heads;      // in n_units = ceil(n_heads / 64) units of 64
    uint32_t n_units;
    uint32_t n_units16;    // ceil(n_heads / 16): units of the matrix-core renderer
};

// Run-length binning state of one lane: the open run's bin and the word
// count at which it began.  The word counter itself is wave-uniform.
struct Runs {
    uint32_t cur, start;
    uint64_t drop;
};

// Where a closed run's count goes.  GlobalSink: one global atomic add per
// run.  TileSink: runs whose bin falls in the wave's 32 x 32 LDS tile are
// added there with an LDS atomic; the tile is merged into the image with
// one global add per non-zero bin whenever the wave moves its tile.
struct GlobalSink {
    uint32_t* image;
    __device__ __forceinline__ void add(uint32_t key, uint32_t cnt) const { atomicAdd(image + key, cnt); }
};

constexpr int kTile = 32;

struct TileSink {
    uint32_t* image;
    uint32_t* tile;   // LDS, kTile * kTile bins of this wave
    uint32_t W, H;
    int col0, row0;   // image position of tile bin (0, 0)
    __device__ __forceinline__ void add(uint32_t key, uint32_t cnt) const {
        const uint32_t row = key / W, col = key - row * W;
        const uint32_t tc = col - (uint32_t)col0, tr = row - (uint32_t)row0;
        if (tc < (uint32_t)kTile && tr < (uint32_t)kTile) atomicAdd(tile + tr * kTile + tc, cnt);
        else atomicAdd(image + key, cnt);
    }
    // merge the tile into the image and clear it (whole wave, uniform)
    __device__ __forceinline__ void merge(int lane) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int i = lane; i < kTile * kTile; i += kWave) {
            const uint32_t v = tile[i];
            if (v) {
                const uint32_t row = (uint32_t)row0 + (uint32_t)(i / kTile);
                const uint32_t col = (uint32_t)col0 + (uint32_t)(i % kTile);
                atomicAdd(image + row * W + col, v);
                tile[i] = 0;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
};

template <typename Sink>
__device__ __forceinline__ void close_run(Runs& s, uint32_t t_words, const Sink& sink) {
    const uint32_t cnt = t_words - s.start;
    if (s.cur == kOutside) s.drop += cnt;
    else if (cnt) sink.add(s.cur, cnt);
}

__device__ __forceinline__ void close_run(Runs& s, uint32_t t_words, uint32_t* image) {
    close_run(s, t_words, GlobalSink{image});
}

// All tails of one head: the 3 blocks of suffixes whose first letter may
// follow the head's last letter, each walked in index order, 9 suffix
// points loaded from LDS ahead of their use.
// With MASKED, lanes whose `live` is false walk along without binning
// (their bin stays kOutside; the caller discards their count).
template <typename T, bool AFFINE, bool ANISO, bool MASKED = false, typename Sink = GlobalSink>
__device__ __forceinline__ void walk_tails_s(const Head<T>& h, const unsigned char* tail_lds, uint32_t R1,
                                             T aniso, uint32_t W, uint32_t H, const Sink& sink, Runs& s,
                                             uint32_t& t_words, bool live = true) {
    const int ie = inv_letter(h.e);
    for (int j = 0; j < 3; ++j) {
        const uint32_t y1 = (uint32_t)(j + (j >= ie));
        for (uint32_t t0 = 0; t0 < R1; t0 += 9) {
            const uint32_t e0 = y1 * R1 + t0;
            cpx<T> ya[9], yb[9];
#pragma unroll
            for (uint32_t u = 0; u < 9; ++u) {
                if constexpr (AFFINE) {
                    ya[u] = ((const cpx<T>*)tail_lds)[e0 + u];
                } else {
                    ya[u] = ((const cpx<T>*)tail_lds)[2 * (e0 + u)];
                    yb[u] = ((const cpx<T>*)tail_lds)[2 * (e0 + u) + 1];
                }
            }
#pragma unroll
            for (uint32_t u = 0; u < 9; ++u) {
                T px, py;
                if constexpr (AFFINE) eval_point<T, ANISO>(h, ya[u], aniso, px, py);
                else eval_point_h<T, ANISO>(h, ya[u], yb[u], aniso, px, py);
                uint32_t key = bin_key(px, py, W, H);
                if (MASKED && !live) key = kOutside;
                if (key != s.cur) {
                    close_run(s, t_words, sink);
                    s.cur = key;
                    s.start = t_words;
                }
                ++t_words;
            }
        }
    }
}

template <typename T, bool AFFINE, bool ANISO, bool MASKED = false>
__device__ __forceinline__ void walk_tails(const Head<T>& h, const unsigned char* tail_lds, uint32_t R1,
                                           T aniso, uint32_t W, uint32_t H, uint32_t* image, Runs& s,
                                           uint32_t& t_words, bool live = true) {
    walk_tails_s<T, AFFINE, ANISO, MASKED>(h, tail_lds, R1, aniso, W, H, GlobalSink{image}, s, t_words, live);
}

// Bin of the head's first allowed word in some lane, wave-uniform; kOutside
// if no lane's first word is in the window.
template <typename T, bool AFFINE, bool ANISO>
__device__ __forceinline__ uint32_t first_key(const Head<T>& h, const unsigned char* tail_lds, uint32_t R1, T aniso,
                                              uint32_t W, uint32_t H) {
    const uint32_t y1 = (uint32_t)(0 + (0 >= inv_letter(h.e)));
    T px, py;
    if constexpr (AFFINE) eval_point<T, ANISO>(h, ((const cpx<T>*)tail_lds)[y1 * R1], aniso, px, py);
    else eval_point_h<T, ANISO>(h, ((const cpx<T>*)tail_lds)[2 * y1 * R1], ((const cpx<T>*)tail_lds)[2 * y1 * R1 + 1],
                                aniso, px, py);
    const uint32_t key = bin_key(px, py, W, H);
    const uint64_t m = __ballot(key != kOutside);
    if (!m) return kOutside;
    return __shfl(key, __ffsll((unsigned long long)m) - 1, kWave);
}

template <typename T, bool AFFINE, bool ANISO, bool LDSHIST>
__device__ __forceinline__ void render_units(const RenderArgs& a, const unsigned char* tail_lds, const m64* G,
                                             uint32_t* tile, Runs& s) {
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t waves = gridDim.x * (kBlock / kWave);
    const uint32_t gwave = blockIdx.x * (kBlock / kWave) + (threadIdx.x / kWave);
    const T aniso = (T)a.fold.aniso;
    uint32_t t_words = 0;
    TileSink ts{a.image, tile, a.W, a.H, -(1 << 30), -(1 << 30)};
    for (uint32_t unit = gwave; unit < a.n_units; unit += waves) {
        const uint64_t local = (uint64_t)unit * kWave + lane;
        const bool full = (uint64_t)(unit + 1) * kWave <= a.n_heads;
        const bool live = local < a.n_heads;
        const uint64_t hidx = a.head_begin + (live ? local : a.n_heads - 1);
        const Head<T> h = compute_head<T>(hidx, a.sp, a.tab.prefix, a.tab.prefix_last, G, a.fold);
        if constexpr (LDSHIST) {
            // move the tile to where this unit's words start
            const uint32_t k0 = first_key<T, AFFINE, ANISO>(h, tail_lds, a.sp.R1, aniso, a.W, a.H);
            ts.merge(lane);
            if (k0 != kOutside) {
                const uint32_t row = k0 / a.W;
                ts.row0 = (int)row - kTile / 2;
                ts.col0 = (int)(k0 - row * a.W) - kTile / 2;
            } else {
                ts.row0 = ts.col0 = -(1 << 30);
            }
        }
        if (full) {
            if constexpr (LDSHIST) walk_tails_s<T, AFFINE, ANISO, false>(h, tail_lds, a.sp.R1, aniso, a.W, a.H, ts, s, t_words);
            else walk_tails<T, AFFINE, ANISO>(h, tail_lds, a.sp.R1, aniso, a.W, a.H, a.image, s, t_words);
        } else {
            // last, partial unit: idle lanes walk a valid head without binning
            // and their count is discarded
            close_run(s, t_words, a.image);
            s.cur = kOutside;
            s.start = t_words;
            walk_tails<T, AFFINE, ANISO, true>(h, tail_lds, a.sp.R1, aniso, a.W, a.H, a.image, s, t_words, live);
            if (live) close_run(s, t_words, a.image);
            s.cur = kOutside;
            s.start = t_words;
        }
    }
    if constexpr (LDSHIST) {
        close_run(s, t_words, ts);
        ts.merge(lane);
    } else {
        close_run(s, t_words, a.image);
    }
}

// One wave per unit of 64 consecutive heads, units dealt round robin over
// the persistent waves.  Per word: one Moebius map of an LDS suffix point,
// the bin, and a run-length counter: a lane adds to the image only when its
// bin changes (consecutive tails of one head lie close together), and keeps
// its dropped words in a register until the end.
// LDS: suffix table (sized for the homogeneous form), generators, and with
// LDSHIST one 32 x 32 tile of uint32 bins per wave.
template <typename T, bool ANISO, bool LDSHIST>
__global__ __launch_bounds__(kBlock) void render_kernel(const RenderArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t n_tail = 4 * a.sp.R1;
    const bool affine = *a.tab.tail_flags == 0;
    const size_t entry = affine ? sizeof(cpx<T>) : 2 * sizeof(cpx<T>);
    const size_t tbytes = (n_tail * entry + 15) & ~size_t(15);
    const size_t tmax = (n_tail * 2 * sizeof(cpx<T>) + 15) & ~size_t(15);
    m64* G = (m64*)(smem + tbytes);
    uint32_t* tile = (uint32_t*)(smem + tmax + 4 * sizeof(m64)) + (threadIdx.x / kWave) * (kTile * kTile);
    {
        const uint4* src = (const uint4*)(affine ? a.tab.tail : a.tail_homog);
        uint4* dst = (uint4*)smem;
        const uint32_t n16 = (uint32_t)(tbytes / 16);
        for (uint32_t i = threadIdx.x; i < n16; i += blockDim.x) dst[i] = src[i];
        if (threadIdx.x < 4) G[threadIdx.x] = a.gens.g[threadIdx.x];
        if (LDSHIST)
            for (int i = threadIdx.x & (kWave - 1); i < kTile * kTile; i += kWave) tile[i] = 0;
    }
    __syncthreads();
    Runs s = {kOutside, 0, 0};
    if (affine) render_units<T, true, ANISO, LDSHIST>(a, smem, G, tile, s);
    else render_units<T, false, ANISO, LDSHIST>(a, smem, G, tile, s);
    if (a.dropped) {
        uint64_t drop = s.drop;
        for (int off = kWave / 2; off > 0; off >>= 1) drop += __shfl_down(drop, off, kWave);
        if ((threadIdx.x & (kWave - 1)) == 0 && drop)
            atomicAdd((unsigned long long*)a.dropped, (unsigned long long)drop);
    }
}

// ------------------------------------------------------------------ matrix-core renderer
// The map of a head applied to a suffix point is, over a block of 4 heads'
// rows and 4 suffix points, a 4 x 4 product with K = 2 (the point's real and
// imaginary part) plus the constant terms: v_mfma_f32_4x4x1f32 runs 16 such
// blocks per wave instruction, two instructions per 64 words.  Lane l holds
// row (l & 3) of head (l >> 2)'s coefficients, suffix column (l & 3), and
// receives (num.re, num.im, den.re, den.im) of word (head l >> 2, suffix
// l & 3).  The accumulation is an exact FMA per K step (y.re first), the
// order eval_point() uses, so this renderer and every other kernel agree
// bit for bit.
typedef float mf32x4 __attribute__((ext_vector_type(4)));

template <bool ANISO, bool MASKED>
__device__ __forceinline__ void mfma_bin(const mf32x4 d, float aniso, uint32_t W, uint32_t H, uint32_t* image,
                                         Runs& s, uint32_t& t_words, bool live, bool valid) {
    float px, py;
    finish_point<float, ANISO>({d[0], d[1]}, {d[2], d[3]}, aniso, px, py);
    uint32_t key = bin_key(px, py, W, H);
    if (MASKED && !live) key = kOutside;
    if (!valid) key = s.cur;
    if (key != s.cur) {
        close_run(s, t_words, image);
        s.cur = key;
        s.start = t_words;
    }
    if (!valid) s.start += 1;   // the repeated suffix is not a word
    ++t_words;
}

template <bool ANISO, bool MASKED>
__device__ __forceinline__ void walk_tails_mfma(const Head<float>& h, const cpx<float>* tail, uint32_t R1,
                                                float aniso, uint32_t W, uint32_t H, uint32_t* image, Runs& s,
                                                uint32_t& t_words, bool live, int col) {
    const float a0 = col == 0 ? h.A.re : col == 1 ? h.A.im : col == 2 ? h.C.re : h.C.im;
    const float a1 = col == 0 ? -h.A.im : col == 1 ? h.A.re : col == 2 ? -h.C.im : h.C.re;
    const mf32x4 c0 = {h.B.re, h.B.im, h.D.re, h.D.im};
    const int ie = inv_letter(h.e);
    const uint32_t full = R1 & ~3u, rem = R1 & 3u;
    for (int j = 0; j < 3; ++j) {
        const uint32_t y1 = (uint32_t)(j + (j >= ie));
        const cpx<float>* row = tail + y1 * R1;
#pragma unroll 4
        for (uint32_t t0 = 0; t0 < full; t0 += 4) {
            const cpx<float> y = row[t0 + col];
            mf32x4 d = __builtin_amdgcn_mfma_f32_4x4x1f32(a0, y.re, c0, 0, 0, 0);
            d = __builtin_amdgcn_mfma_f32_4x4x1f32(a1, y.im, d, 0, 0, 0);
            mfma_bin<ANISO, MASKED>(d, aniso, W, H, image, s, t_words, live, true);
        }
        if (rem) {
            // the block's last step: columns >= rem repeat its last suffix and do not count
            const bool valid = (uint32_t)col < rem;
            const cpx<float> y = row[full + (valid ? (uint32_t)col : rem - 1)];
            mf32x4 d = __builtin_amdgcn_mfma_f32_4x4x1f32(a0, y.re, c0, 0, 0, 0);
            d = __builtin_amdgcn_mfma_f32_4x4x1f32(a1, y.im, d, 0, 0, 0);
            mfma_bin<ANISO, MASKED>(d, aniso, W, H, image, s, t_words, live, valid);
        }
    }
}

template <bool ANISO>
__device__ __forceinline__ void render_units_mfma(const RenderArgs& a, const cpx<float>* tail, const m64* G, Runs& s) {
    const int lane = threadIdx.x & (kWave - 1);
    const int blk = lane >> 2, col = lane & 3;
    const uint32_t waves = gridDim.x * (kBlock / kWave);
    const uint32_t gwave = blockIdx.x * (kBlock / kWave) + (threadIdx.x / kWave);
    const float aniso = (float)a.fold.aniso;
    uint32_t t_words = 0;
    for (uint32_t unit = gwave; unit < a.n_units16; unit += waves) {
        const uint64_t local = (uint64_t)unit * 16 + blk;
        const bool full = (uint64_t)(unit + 1) * 16 <= a.n_heads;
        const bool live = local < a.n_heads;
        const uint64_t hidx = a.head_begin + (live ? local : a.n_heads - 1);
        const Head<float> h = compute_head<float>(hidx, a.sp, a.tab.prefix, a.tab.prefix_last, G, a.fold);
        if (full) {
            walk_tails_mfma<ANISO, false>(h, tail, a.sp.R1, aniso, a.W, a.H, a.image, s, t_words, true, col);
        } else {
            close_run(s, t_words, a.image);
            s.cur = kOutside;
            s.start = t_words;
            walk_tails_mfma<ANISO, true>(h, tail, a.sp.R1, aniso, a.W, a.H, a.image, s, t_words, live, col);
            if (live) close_run(s, t_words, a.image);
            s.cur = kOutside;
            s.start = t_words;
        }
    }
    close_run(s, t_words, a.image);
}

// FP32 renderer on the matrix cores (affine suffix points); a homogeneous
// suffix table falls back to the VALU walk in the same launch.
template <bool ANISO>
__global__ __launch_bounds__(kBlock) void render_kernel_mfma(const RenderArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t n_tail = 4 * a.sp.R1;
    const bool affine = *a.tab.tail_flags == 0;
    const size_t entry = affine ? sizeof(c32) : 2 * sizeof(c32);
    const size_t tbytes = (n_tail * entry + 15) & ~size_t(15);
    m64* G = (m64*)(smem + tbytes);
    {
        const uint4* src = (const uint4*)(affine ? a.tab.tail : a.tail_homog);
        uint4* dst = (uint4*)smem;
        const uint32_t n16 = (uint32_t)(tbytes / 16);
        for (uint32_t i = threadIdx.x; i < n16; i += blockDim.x) dst[i] = src[i];
        if (threadIdx.x < 4) G[threadIdx.x] = a.gens.g[threadIdx.x];
    }
    __syncthreads();
    Runs s = {kOutside, 0, 0};
    if (affine) render_units_mfma<ANISO>(a, (const cpx<float>*)smem, G, s);
    else render_units<float, false, ANISO, false>(a, smem, G, nullptr, s);
    if (a.dropped) {
        uint64_t drop = s.drop;
        for (int off = kWave / 2; off > 0; off >>= 1) drop += __shfl_down(drop, off, kWave);
        if ((threadIdx.x & (kWave - 1)) == 0 && drop)
            atomicAdd((unsigned long long*)a.dropped, (unsigned long long)drop);
    }
}

// ------------------------------------------------------------------ per-word kernel
struct PerWordArgs {
    Split sp;
    Fold fold;
    Gens gens;
    Tables tab;
    const void* tail_homog;
    uint64_t n_words;      // words of depth sp.depth
    // render mode: words [first0, first0+count0) then [first1, first1+count1)
    uint64_t first0, count0, first1, count1;
    uint32_t* image;
    uint32_t W, H;
    uint64_t* dropped;
    // eval mode
    const uint64_t* idx;
    c64* out;
    uint64_t n;
};

// Value of word i of depth sp.depth, with the renderer's arithmetic.
template <typename T, bool ANISO>
__device__ inline void word_point(uint64_t i, const PerWordArgs& a, const m64* G, T& px, T& py) {
    const Split& sp = a.sp;
    Head<T> h;
    uint64_t entry;
    if (sp.k + sp.m == 0) {
        h = compute_head<T>(0, sp, nullptr, nullptr, G, a.fold);
        entry = i;
    } else {
        const uint64_t hidx = i / sp.R;
        const uint32_t t = (uint32_t)(i - hidx * sp.R);
        h = compute_head<T>(hidx, sp, a.tab.prefix, a.tab.prefix_last, G, a.fold);
        const uint32_t j = t / sp.R1;
        const uint32_t tt = t - j * sp.R1;
        const int y1 = (int)j + ((int)j >= inv_letter(h.e));
        entry = (uint64_t)y1 * sp.R1 + tt;
    }
    const T aniso = (T)a.fold.aniso;
    if (*a.tab.tail_flags == 0) {
        const cpx<T> y = ((const cpx<T>*)a.tab.tail)[entry];
        eval_point<T, ANISO>(h, y, aniso, px, py);
    } else {
        const cpx<T>* hm = (const cpx<T>*)a.tail_homog;
        eval_point_h<T, ANISO>(h, hm[2 * entry], hm[2 * entry + 1], aniso, px, py);
    }
}

template <typename T, bool ANISO>
__global__ __launch_bounds__(256) void perword_render_kernel(const PerWordArgs a) {
    __shared__ m64 G[4];
    if (threadIdx.x < 4) G[threadIdx.x] = a.gens.g[threadIdx.x];
    __syncthreads();
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t drop = 0;
    if (tid < a.count0 + a.count1) {
        const uint64_t i = tid < a.count0 ? a.first0 + tid : a.first1 + (tid - a.count0);
        T px, py;
        word_point<T, ANISO>(i, a, G, px, py);
        const uint32_t key = bin_key(px, py, a.W, a.H);
        if (key == kOutside) drop = 1;
        else atomicAdd(a.image + key, 1u);
    }
    if (a.dropped) {
        for (int off = kWave / 2; off > 0; off >>= 1) drop += __shfl_down(drop, off, kWave);
        if ((threadIdx.x & (kWave - 1)) == 0 && drop)
            atomicAdd((unsigned long long*)a.dropped, (unsigned long long)drop);
    }
}

template <typename T, bool ANISO>
__global__ __launch_bounds__(256) void eval_kernel(const PerWordArgs a) {
    __shared__ m64 G[4];
    if (threadIdx.x < 4) G[threadIdx.x] = a.gens.g[threadIdx.x];
    __syncthreads();
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= a.n) return;
    const uint64_t i = a.idx[tid];
    if (i >= a.n_words) {
        a.out[tid] = {__builtin_nan(""), __builtin_nan("")};
        return;
    }
    T px, py;
    word_point<T, ANISO>(i, a, G, px, py);
    a.out[tid] = {(double)px, (double)py};
}

}  // namespace kl

namespace kl {

template <typename T, bool ANISO>
static hipError_t launch_render_t(const RenderJob& job, hipStream_t s) {
    if (job.n_units > 0) {
        RenderArgs a;
        a.sp = job.sp;
        a.fold = job.fold;
        a.gens = job.gens;
        a.tab = job.tab;
        a.tail_homog = job.tail_homog;
        a.image = job.image;
        a.W = job.width;
        a.H = job.height;
        a.dropped = job.dropped;
        a.head_begin = job.head_begin;
        a.n_heads = job.n_heads;
        a.n_units = job.n_units;
        a.n_units16 = (uint32_t)((job.n_heads + 15) / 16);
        const size_t n_tail = 4 * (size_t)job.sp.R1;
        const bool ldsh = job.hist_mode == KL_HIST_LDS;
        const size_t lds = ((n_tail * 2 * sizeof(cpx<T>) + 15) & ~size_t(15)) + 4 * sizeof(m64) +
                           (ldsh ? (kBlock / kWave) * kTile * kTile * sizeof(uint32_t) : 0);
        const void* fn = ldsh ? reinterpret_cast<const void*>(&render_kernel<T, ANISO, true>)
                              : reinterpret_cast<const void*>(&render_kernel<T, ANISO, false>);
        if (lds > 65536) {
            hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        uint32_t grid = (uint32_t)job.grid_blocks;
        const uint32_t need = (job.n_units + (kBlock / kWave) - 1) / (kBlock / kWave);
        if (grid > need) grid = need;
        if (grid < 1) grid = 1;
        const bool mfma = std::is_same<T, float>::value && job.engine == KL_ENGINE_MATRIX;
        if (mfma) {
            const uint32_t need16 = (a.n_units16 + (kBlock / kWave) - 1) / (kBlock / kWave);
            uint32_t g16 = std::min<uint32_t>((uint32_t)job.grid_blocks, need16);
            if (g16 < 1) g16 = 1;
            const size_t lds16 = ((n_tail * 2 * sizeof(c32) + 15) & ~size_t(15)) + 4 * sizeof(m64);
            if (lds16 > 65536) {
                hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&render_kernel_mfma<ANISO>),
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds16);
                if (e != hipSuccess) return e;
            }
            hipLaunchKernelGGL((render_kernel_mfma<ANISO>), dim3(g16), dim3(kBlock), lds16, s, a);
        } else if (ldsh) {
            hipLaunchKernelGGL((render_kernel<T, ANISO, true>), dim3(grid), dim3(kBlock), lds, s, a);
        } else {
            hipLaunchKernelGGL((render_kernel<T, ANISO, false>), dim3(grid), dim3(kBlock), lds, s, a);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const uint64_t rag = job.rag_count[0] + job.rag_count[1];
    if (rag > 0) {
        PerWordArgs p = {};
        p.sp = job.sp;
        p.fold = job.fold;
        p.gens = job.gens;
        p.tab = job.tab;
        p.tail_homog = job.tail_homog;
        p.n_words = num_words(job.sp.depth);
        p.first0 = job.rag_first[0];
        p.count0 = job.rag_count[0];
        p.first1 = job.rag_first[1];
        p.count1 = job.rag_count[1];
        p.image = job.image;
        p.W = job.width;
        p.H = job.height;
        p.dropped = job.dropped;
        const uint64_t blocks = (rag + 255) / 256;
        if (blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
        hipLaunchKernelGGL((perword_render_kernel<T, ANISO>), dim3((unsigned)blocks), dim3(256), 0, s, p);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_render(const RenderJob& job, hipStream_t s) {
    const bool an = job.fold.use_aniso != 0;
    if (job.precision == KL_PREC_FP64)
        return an ? launch_render_t<double, true>(job, s) : launch_render_t<double, false>(job, s);
    return an ? launch_render_t<float, true>(job, s) : launch_render_t<float, false>(job, s);
}

template <typename T, bool ANISO>
static hipError_t launch_eval_t(const EvalJob& job, hipStream_t s) {
    PerWordArgs p = {};
    p.sp = job.sp;
    p.fold = job.fold;
    p.gens = job.gens;
    p.tab = job.tab;
    p.tail_homog = job.tail_homog;
    p.n_words = num_words(job.sp.depth);
    p.idx = job.idx;
    p.out = job.out;
    p.n = job.n;
    const uint64_t blocks = (job.n + 255) / 256;
    if (blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
    hipLaunchKernelGGL((eval_kernel<T, ANISO>), dim3((unsigned)blocks), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_eval(const EvalJob& job, hipStream_t s) {
    if (job.n == 0) return hipSuccess;
    const bool an = job.fold.use_aniso != 0;
    if (job.precision == KL_PREC_FP64)
        return an ? launch_eval_t<double, true>(job, s) : launch_eval_t<double, false>(job, s);
    return an ? launch_eval_t<float, true>(job, s) : launch_eval_t<float, false>(job, s);
}

}  // namespace kl

// ====================================================================== batched renderer
namespace kl {

__global__ __launch_bounds__(256) void prefix_table_batch_kernel(const SetDesc* __restrict__ sets) {
    const SetDesc& S = sets[blockIdx.y];
    const uint32_t p = blockIdx.x * 256 + threadIdx.x;
    if (S.sp.k == 0 || p >= S.n_prefix) return;
    const Gens g = S.gens;
    prefix_entry(g, S.sp.k, p, (m64*)S.tab.prefix, (uint8_t*)S.tab.prefix_last);
}

template <typename T>
__global__ __launch_bounds__(256) void tail_table_batch_kernel(const SetDesc* __restrict__ sets, int force_homog) {
    const SetDesc& S = sets[blockIdx.y];
    const uint32_t t = blockIdx.x * 256 + threadIdx.x;
    if (t >= S.n_tail) return;
    const Gens g = S.gens;
    uint32_t* flags = (uint32_t*)S.tab.tail_flags;
    tail_entry<T>(g, S.sp.r, t, (cpx<T>*)S.tab.tail, (cpx<T>*)S.tail_homog, flags);
    if (force_homog && t == 0) atomicOr(flags, 1u);
}

hipError_t launch_batch_tables(const BatchJob& job, hipStream_t s) {
    if (job.max_prefix > 0) {
        dim3 grid((job.max_prefix + 255) / 256, job.n_sets);
        hipLaunchKernelGGL(prefix_table_batch_kernel, grid, dim3(256), 0, s, job.sets);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    dim3 grid((job.max_tail + 255) / 256, job.n_sets);
    if (job.precision == KL_PREC_FP64)
        hipLaunchKernelGGL(tail_table_batch_kernel<double>, grid, dim3(256), 0, s, job.sets, job.force_homog);
    else
        hipLaunchKernelGGL(tail_table_batch_kernel<float>, grid, dim3(256), 0, s, job.sets, job.force_homog);
    return hipGetLastError();
}

struct BatchArgs {
    const SetDesc* sets;
    const uint64_t* unit_offsets;
    int n_sets;
    uint64_t total_units;
    Fold fold;
    uint32_t W, H;
    uint32_t lds_per_wave;
};

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void flush_drop(uint64_t& drop, uint64_t* dst) {
    uint64_t d = drop;
    for (int off = kWave / 2; off > 0; off >>= 1) d += __shfl_down(d, off, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0 && d && dst) atomicAdd((unsigned long long*)dst, (unsigned long long)d);
    drop = 0;
}

// Units of 64 heads from every set form one queue dealt round robin over
// the persistent waves; each wave keeps the suffix table and generators of
// the set it is working on in its own LDS slice and reloads them when its
// next unit belongs to another set.  The last unit of a set may be partial:
// its idle lanes walk a valid head without binning.
template <typename T, bool ANISO>
__global__ __launch_bounds__(kBlock) void render_batch_kernel(const BatchArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int wid = threadIdx.x / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    unsigned char* slice = smem + (size_t)wid * a.lds_per_wave;
    m64* G = (m64*)(slice + a.lds_per_wave - 4 * sizeof(m64));
    const uint32_t waves = gridDim.x * (kBlock / kWave);
    const uint32_t gwave = blockIdx.x * (kBlock / kWave) + wid;
    const T aniso = (T)a.fold.aniso;

    int cur = -1;
    bool affine = true;
    Split sp{};
    const m64* prefix = nullptr;
    const uint8_t* plast = nullptr;
    uint32_t* image = nullptr;
    uint64_t* dropped = nullptr;
    uint64_t base = 0;
    Runs s = {kOutside, 0, 0};
    uint32_t t_words = 0;

    for (uint64_t unit = gwave; unit < a.total_units; unit += waves) {
        // set of this unit: the last set whose first unit is <= unit
        int lo = 0, hi = a.n_sets - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.unit_offsets[mid] <= unit) lo = mid;
            else hi = mid - 1;
        }
        if (lo != cur) {
            if (cur >= 0) {
                close_run(s, t_words, image);
                flush_drop(s.drop, dropped);
            }
            s.cur = kOutside;
            s.start = t_words;
            cur = lo;
            const SetDesc& S = a.sets[cur];
            sp = S.sp;
            prefix = S.tab.prefix;
            plast = S.tab.prefix_last;
            image = S.image;
            dropped = S.dropped;
            base = a.unit_offsets[cur];
            affine = *S.tab.tail_flags == 0;
            const size_t bytes = (size_t)S.n_tail * (affine ? 1 : 2) * sizeof(cpx<T>);
            const uint4* src = (const uint4*)(affine ? S.tab.tail : S.tail_homog);
            wave_lds_sync();
            for (uint32_t i = lane; i < (uint32_t)((bytes + 15) / 16); i += kWave) ((uint4*)slice)[i] = src[i];
            if (lane < 4) G[lane] = S.gens.g[lane];
            wave_lds_sync();
        }
        const uint64_t local = unit - base;
        uint64_t hidx = local * kWave + lane;
        const bool partial = (local + 1) * kWave > sp.n_heads;
        if (!partial) {
            const Head<T> h = compute_head<T>(hidx, sp, prefix, plast, G, a.fold);
            if (affine) walk_tails<T, true, ANISO>(h, slice, sp.R1, aniso, a.W, a.H, image, s, t_words);
            else walk_tails<T, false, ANISO>(h, slice, sp.R1, aniso, a.W, a.H, image, s, t_words);
        } else {
            const bool live = hidx < sp.n_heads;
            if (!live) hidx = sp.n_heads - 1;
            close_run(s, t_words, image);
            s.cur = kOutside;
            s.start = t_words;
            const Head<T> h = compute_head<T>(hidx, sp, prefix, plast, G, a.fold);
            if (affine) walk_tails<T, true, ANISO, true>(h, slice, sp.R1, aniso, a.W, a.H, image, s, t_words, live);
            else walk_tails<T, false, ANISO, true>(h, slice, sp.R1, aniso, a.W, a.H, image, s, t_words, live);
            if (live) close_run(s, t_words, image);
            s.cur = kOutside;
            s.start = t_words;
        }
    }
    if (cur >= 0) {
        close_run(s, t_words, image);
        flush_drop(s.drop, dropped);
    }
}

hipError_t launch_render_batch(const BatchJob& job, hipStream_t s) {
    if (job.total_units == 0) return hipSuccess;
    BatchArgs a;
    a.sets = job.sets;
    a.unit_offsets = job.unit_offsets;
    a.n_sets = job.n_sets;
    a.total_units = job.total_units;
    a.fold = job.fold;
    a.W = job.width;
    a.H = job.height;
    a.lds_per_wave = job.lds_per_wave;
    const size_t lds = (size_t)job.lds_per_wave * (kBlock / kWave);
    uint64_t need = (job.total_units + (kBlock / kWave) - 1) / (kBlock / kWave);
    uint32_t grid = (uint32_t)std::min<uint64_t>(need, (uint64_t)job.grid_blocks);
    if (grid < 1) grid = 1;
    const bool an = job.fold.use_aniso != 0;
    if (lds > 65536) {
        const void* fn = job.precision == KL_PREC_FP64
                             ? (an ? reinterpret_cast<const void*>(&render_batch_kernel<double, true>)
                                   : reinterpret_cast<const void*>(&render_batch_kernel<double, false>))
                             : (an ? reinterpret_cast<const void*>(&render_batch_kernel<float, true>)
                                   : reinterpret_cast<const void*>(&render_batch_kernel<float, false>));
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    if (job.precision == KL_PREC_FP64) {
        if (an) hipLaunchKernelGGL((render_batch_kernel<double, true>), dim3(grid), dim3(kBlock), lds, s, a);
        else hipLaunchKernelGGL((render_batch_kernel<double, false>), dim3(grid), dim3(kBlock), lds, s, a);
    } else {
        if (an) hipLaunchKernelGGL((render_batch_kernel<float, true>), dim3(grid), dim3(kBlock), lds, s, a);
        else hipLaunchKernelGGL((render_batch_kernel<float, false>), dim3(grid), dim3(kBlock), lds, s, a);
    }
    return hipGetLastError();
}

}  // namespace kl

namespace kl {

hipError_t launch_setup(const SetupJob& j, hipStream_t s) {
    SetupArgs a;
    a.g = j.gens;
    a.k = j.k;
    a.r = j.r;
    a.n_prefix = j.k ? (uint32_t)num_words(j.k) : 0;
    a.n_tail = (uint32_t)num_words(j.r);
    a.prefix = j.prefix;
    a.last = j.last;
    a.aff = j.aff;
    a.hom = j.hom;
    a.flags = j.flags;
    a.force_homog = j.force_homog;
    a.image = j.image;
    a.bins = j.bins;
    a.dropped = j.dropped;
    uint64_t blocks = 1 + (a.n_prefix + 255) / 256;
    if (a.image) blocks = std::max<uint64_t>(blocks, std::min<uint64_t>(2048, (a.bins / 4 + 255) / 256));
    if (j.precision == KL_PREC_FP64)
        hipLaunchKernelGGL(setup_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(setup_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace kl
