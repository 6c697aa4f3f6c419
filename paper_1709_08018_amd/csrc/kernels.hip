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
//     once per render (setup_kernel);
//   * each lane of the renderer owns one head: it appends its m letters in
//     FP64, folds the window map into the product, scales it by a power of
//     two and rounds it once to the working precision;
//   * the r tail letters run through a table of suffix points
//     G_{y1}(...G_{y(r-1)}(fix(yr))) built right to left in the working
//     precision (setup_kernel), held in LDS; the lane walks the 3^r
//     tails allowed after its head's last letter in index order.
// The value of head . tail is then one Moebius map of one point, in the
// pole form of the head (compute_head, word_value below), which every
// kernel shares.
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
// of G_{y1}(...G_{yr}(z0)) walked right to left in precision T from the
// rounded seed with the rounded generators, rescaled by powers of two after
// every step; and its affine form y = u / v.  seed < 0: z0 is the attracting
// fixed point of the tail's last letter yr, which G_{yr} fixes, so that map
// is not applied; seed = 0..3: z0 is that generator's attracting fixed
// point and every map is applied.  A seed at infinity starts as (1, 0).
template <typename T>
__device__ inline void tail_entry(const Gens& g, int r, uint32_t t, int seed, cpx<T>* __restrict__ affine,
                                  cpx<T>* __restrict__ homog, uint32_t* __restrict__ flags, bool atomic = true) {
    const uint64_t w = decode_packed(t, r);
    const int last = (int)((w >> (2 * (r - 1))) & 3);
    const int s = seed < 0 ? last : seed;
    cpx<T> u = {(T)g.fix[s].re, (T)g.fix[s].im};
    cpx<T> v = {T(1), T(0)};
    if ((g.inf_mask >> s) & 1u) {
        u = {T(1), T(0)};
        v = {T(0), T(0)};
    }
    for (int j = seed < 0 ? r - 2 : r - 1; j >= 0; --j) {
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

// ------------------------------------------------------------------ fused set-up
// One launch that clears the image and the dropped counter and builds the
// suffix table (blocks 0 .. nb_tail-1, one point per thread) and the FP64
// prefix table (the next blocks).  Each suffix block writes one word of the
// form flags: nonzero when one of its points needs the homogeneous form (or
// that form is forced), so no flag has to be cleared beforehand.
struct SetupArgs {
    Gens g;
    int k, r, seed;
    uint32_t n_prefix, n_tail, nb_tail;
    m64* prefix;
    uint8_t* last;
    void* aff;
    void* hom;
    uint32_t* flags;      // nb_tail words
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
    if (blockIdx.x < a.nb_tail) {
        const uint32_t t = blockIdx.x * 256 + threadIdx.x;
        uint32_t bad = 0;
        if (t < a.n_tail) tail_entry<T>(a.g, a.r, t, a.seed, (cpx<T>*)a.aff, (cpx<T>*)a.hom, &bad, false);
        bad = __syncthreads_or(bad);
        if (threadIdx.x == 0) {
            a.flags[blockIdx.x] = (bad || a.force_homog) ? 1u : 0u;
            if (blockIdx.x == 0 && a.dropped) a.dropped[0] = 0;
        }
    } else {
        const uint32_t p = (blockIdx.x - a.nb_tail) * 256 + threadIdx.x;
        if (p < a.n_prefix) prefix_entry(a.g, a.k, p, a.prefix, a.last);
    }
}

// Whether the suffix table is used in its affine form: no flag word is set.
// Uniform over the block; every thread of the block must call it.
__device__ inline bool tail_affine_block(const Tables& t) {
    uint32_t bad = 0;
    for (uint32_t i = threadIdx.x; i < t.n_flags; i += blockDim.x) bad |= t.tail_flags[i];
    return !__syncthreads_or(bad);
}

// Same, uniform over the wave; every lane of the wave must call it.
__device__ inline bool tail_affine_wave(const Tables& t) {
    uint32_t bad = 0;
    for (uint32_t i = threadIdx.x & (kWave - 1); i < t.n_flags; i += kWave) bad |= t.tail_flags[i];
    return __ballot(bad != 0) == 0;
}

// ------------------------------------------------------------------ shared arithmetic
// Map of one head, rounded once to T, in two forms.
//
// Pole form, for a head matrix [[a, b], [c, d]] of determinant 1 with c != 0:
//   h(y) = P + Q / (y + S),   P = a / c,  Q = -1 / c^2,  S = d / c,
// with the window fold F(z) = s z + o applied (P <- F(P), Q <- s Q) and the
// x anisotropy folded into the coefficients of the real part, so that with
// u = y + S
//   px = Px + (ax u.re + bx u.im) / |u|^2,   py = Py + (ay u.re + by u.im) / |u|^2.
// That is eleven operations per word: two adds, |u|^2, one reciprocal and
// per coordinate a product and two FMAs.  Its rounding error is of the
// order of eps (|P| + |h(y) - P|), like that of the ratio below.
//
// General form, for heads whose c is 0 or whose pole form leaves T's range:
// the folded matrix (A, B) = s (a, b) + o (c, d), (C, D) = (c, d), scaled by
// a power of two and evaluated as (A y + B) / (C y + D).
template <typename T>
struct Head {
    cpx<T> S;
    T Px, Py, ax, bx, ay, by;
    cpx<T> A, B, C, D;
    T aniso;
    bool pole;          // the pole form is valid
    int e;              // last letter of the head, -1 for the empty head
};

template <typename T>
__device__ __forceinline__ T conv(double x) { return (T)x; }

// |x| <= lim (false for NaN)
template <typename T>
__device__ __forceinline__ bool bounded(T x, double lim) { return x <= (T)lim && x >= -(T)lim; }

// Head map of head index hidx: prefix-table product of its first k letters
// times its m lane letters (FP64, left to right), in both forms.
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
    Head<T> h;
    h.e = e;
    h.aniso = conv<T>(f.aniso);
    {
        const double cn = fma_(M.c.re, M.c.re, M.c.im * M.c.im);
        const c64 ic = {M.c.re / cn, -M.c.im / cn};
        const c64 pm = cmul(M.a, ic), sm = cmul(M.d, ic), q = cmul(ic, ic);
        const double Pre = fma_(f.s, pm.re, f.o.re), Pim = fma_(f.s, pm.im, f.o.im);
        const double Qre = -(f.s * q.re), Qim = -(f.s * q.im);
        h.S = {conv<T>(sm.re), conv<T>(sm.im)};
        h.Px = conv<T>(f.aniso * Pre);
        h.Py = conv<T>(Pim);
        h.ax = conv<T>(f.aniso * Qre);
        h.bx = conv<T>(f.aniso * Qim);
        h.ay = conv<T>(Qim);
        h.by = conv<T>(-Qre);
        // bounds keep |u|^2 and the products of one word finite for affine
        // suffix points (|y| <= 2^32)
        h.pole = cn > 0.0 && cn <= 0x1p1000 && bounded(h.S.re, 0x1p40) && bounded(h.S.im, 0x1p40) &&
                 bounded(h.ax, 0x1p80) && bounded(h.bx, 0x1p80) && bounded(h.ay, 0x1p80) &&
                 bounded(h.by, 0x1p80) && bounded(h.Px, 0x1p100) && bounded(h.Py, 0x1p100);
        if (f.head_form == 1 || (f.head_form == 2 && (hidx & 1))) h.pole = false;
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
    h.A = {conv<T>(A.re), conv<T>(A.im)};
    h.B = {conv<T>(B.re), conv<T>(B.im)};
    h.C = {conv<T>(C.re), conv<T>(C.im)};
    h.D = {conv<T>(D.re), conv<T>(D.im)};
    return h;
}

__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
// v_rcp_f64 refined by two Newton steps r <- r + r (1 - x r), each of which
// doubles the number of correct bits: a full-precision reciprocal in five
// instructions instead of an IEEE division's dozen.  x = 0 gives NaN (a word
// at infinity, dropped like any non-finite value).
__device__ __forceinline__ double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma_(-x, r, 1.0);
    r = fma_(r, e, r);
    e = fma_(-x, r, 1.0);
    return fma_(r, e, r);
}

// The smallest normal number of T.  The pole forms add it to |u|^2 (inside
// the FMA that forms it, so at no cost): |u|^2 is then a normal number, its
// reciprocal finite, and with finite, bounded head and suffix data (the pole
// form's guards) a coordinate is finite or an infinity, never NaN.  It
// changes |u|^2 only where |u| < 2^-50 in FP32, far below the rounding error
// of u = y + S itself.
template <typename T> struct MinNormal;
template <> struct MinNormal<float> { static constexpr float v = 0x1p-126f; };
template <> struct MinNormal<double> { static constexpr double v = 0x1p-1022; };

// Pole form at an affine suffix point y.
template <typename T>
__device__ __forceinline__ void eval_pole(const Head<T>& h, cpx<T> y, T& px, T& py) {
    const T ur = y.re + h.S.re, ui = y.im + h.S.im;
    const T rc = recip(fma_(ur, ur, fma_(ui, ui, MinNormal<T>::v)));
    px = fma_(fma_(h.ax, ur, h.bx * ui), rc, h.Px);
    py = fma_(fma_(h.ay, ur, h.by * ui), rc, h.Py);
}

// Pole form at a homogeneous suffix point (p : q): with u = p + S q and
// v = q conj(u), Q q / u = Q v / |u|^2.  (p : 0) is infinity, whose image is P.
template <typename T>
__device__ __forceinline__ void eval_pole_h(const Head<T>& h, cpx<T> p, cpx<T> q, T& px, T& py) {
    const cpx<T> u = cfma(h.S, q, p);
    const T vr = fma_(q.re, u.re, q.im * u.im);
    const T vi = fma_(q.im, u.re, -(q.re * u.im));
    const T rc = recip(fma_(u.re, u.re, fma_(u.im, u.im, MinNormal<T>::v)));
    px = fma_(fma_(h.ax, vr, -(h.bx * vi)), rc, h.Px);
    py = fma_(fma_(h.ay, vr, -(h.by * vi)), rc, h.Py);
}

// General form: num / den in pixel units.
template <typename T>
__device__ __forceinline__ void finish_point(cpx<T> num, cpx<T> den, T aniso, T& px, T& py) {
    const T n2 = fma_(den.re, den.re, den.im * den.im);
    const T rc = recip(n2);
    const T re = fma_(num.re, den.re, num.im * den.im);
    const T im = fma_(num.im, den.re, -(num.re * den.im));
    px = (re * rc) * aniso;
    py = im * rc;
}

template <typename T>
__device__ __forceinline__ void eval_general(const Head<T>& h, cpx<T> y, T& px, T& py) {
    finish_point(cfma(h.A, y, h.B), cfma(h.C, y, h.D), h.aniso, px, py);
}

template <typename T>
__device__ __forceinline__ void eval_general_h(const Head<T>& h, cpx<T> p, cpx<T> q, T& px, T& py) {
    finish_point(cfma(h.A, p, cmul(h.B, q)), cfma(h.C, p, cmul(h.D, q)), h.aniso, px, py);
}

// Value of head . tail in pixel units, the suffix point being y (AFFINE) or
// (y : q).  A lane uses its head's pole form when valid, else the general
// form.  DUAL: some lane of the wave holds a head without a pole form, so
// every lane evaluates both and keeps its own head's; without DUAL every
// head of the wave has one.  All kernels evaluate words through these
// functions, so they agree bit for bit on every word under the same split.
template <typename T, bool AFFINE, bool DUAL>
__device__ __forceinline__ void word_value(const Head<T>& h, cpx<T> y, cpx<T> q, T& px, T& py) {
    if constexpr (AFFINE) eval_pole(h, y, px, py);
    else eval_pole_h(h, y, q, px, py);
    if constexpr (DUAL) {
        T gx, gy;
        if constexpr (AFFINE) eval_general(h, y, gx, gy);
        else eval_general_h(h, y, q, gx, gy);
        px = h.pole ? px : gx;
        py = h.pole ? py : gy;
    }
}

// Bin of pixel coordinates: row floor(py), column floor(px) when 0 <= px <
// W and 0 <= py < H, else kOutside.  The comparisons are IEEE ones, as the
// oracle's: -0 counts as 0, and a NaN is outside.  The range test is taken
// on the floors as integers: floor(px) lies in [0, W) exactly when px does
// (W an integer), and a saturated or negative floor is outside.
constexpr uint32_t kOutside = 0xFFFFFFFFu;

// floor(x) as int32, saturating, NaN to 0 (v_cvt_flr_i32_f32)
__device__ __forceinline__ int floor_i32(float x) {
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// floor(x) as int32 for x in [-1, 2^31 - 1] after clamping; NaN to -1
// (the clamp's maxNum keeps the number), so a NaN is outside
__device__ __forceinline__ int floor_i32(double x) {
    return (int)__builtin_floor(__builtin_fmin(__builtin_fmax(x, -1.0), 2147483647.0));
}

__device__ __forceinline__ uint32_t bin_key(float px, float py, uint32_t W, uint32_t H) {
    const uint32_t col = (uint32_t)floor_i32(px);
    const uint32_t row = (uint32_t)floor_i32(py);
    const bool ok = (col < W) & (row < H) & (px == px) & (py == py);
    return ok ? __umul24(row, W) + col : kOutside;
}

__device__ __forceinline__ uint32_t bin_key(double px, double py, uint32_t W, uint32_t H) {
    const uint32_t col = (uint32_t)floor_i32(px);
    const uint32_t row = (uint32_t)floor_i32(py);
    const bool ok = (col < W) & (row < H);
    return ok ? __umul24(row, W) + col : kOutside;
}

// Run keys of the persistent walks.  A lane counts runs of consecutive
// words that share a bin.  The key of a word is the pair (floor(px),
// floor(py)) of saturating int32 floors in one 64-bit value, so consecutive
// words are compared with one 64-bit compare; whether a run lies in the
// window (both floors in range, bin_key's rule) and its bin are worked out
// only when the run closes.  v_cvt_flr_i32_f32 maps NaN to 0, so a word
// whose coordinates may be NaN (the general form of DUAL waves) takes the
// outside key explicitly; the pole form's coordinates are never NaN
// (MinNormal).
constexpr uint64_t kOutsideKey = ~0ull;        // floors (-1, -1): outside
constexpr uint64_t kSpanKey = ~0ull - 1;       // bounded walk: a node waiting in the span queue; outside

__device__ __forceinline__ uint64_t run_key(float px, float py) {
    return (uint64_t)(uint32_t)floor_i32(px) | ((uint64_t)(uint32_t)floor_i32(py) << 32);
}

// floor(x) as int32, saturating, NaN to 0 (v_cvt_i32_f64 of the floor), as
// v_cvt_flr_i32_f32 does in FP32
__device__ __forceinline__ int floor_sat_i32(double x) {
    int r;
    asm("v_cvt_i32_f64 %0, %1" : "=v"(r) : "v"(__builtin_floor(x)));
    return r;
}

__device__ __forceinline__ uint64_t run_key(double px, double py) {
    return (uint64_t)(uint32_t)floor_sat_i32(px) | ((uint64_t)(uint32_t)floor_sat_i32(py) << 32);
}

// the key of bin (row, col) of the window
__device__ __forceinline__ uint64_t bin_run_key(uint32_t row, uint32_t col) {
    return (uint64_t)col | ((uint64_t)row << 32);
}

// The window of a run key.
struct KeyRange {
    uint32_t W, H;
};

__device__ __forceinline__ KeyRange key_range(uint32_t W, uint32_t H) { return {W, H}; }

__device__ __forceinline__ bool key_inside(uint64_t k, const KeyRange& kr) {
    return ((uint32_t)k < kr.W) & ((uint32_t)(k >> 32) < kr.H);
}

__device__ __forceinline__ uint32_t key_col(uint64_t k) { return (uint32_t)k; }
__device__ __forceinline__ uint32_t key_row(uint64_t k) { return (uint32_t)(k >> 32); }

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
};

// Run-length binning state of one lane: the open run's key (run_key) and
// the word count at which it began.  The word counter itself is
// wave-uniform.  With DROP the lane also counts the words of its runs
// outside the image.
template <bool DROP>
struct Runs {
    uint64_t key;
    uint32_t start;
    uint64_t drop;
};

// Where a closed run's count goes.  GlobalSink: one global atomic add per
// run.  TileSink: runs whose bin falls in the wave's 32 x 32 LDS tile are
// added there with an LDS atomic; the tile is merged into the image with
// one global add per non-zero bin whenever the wave moves its tile.
struct GlobalSink {
    uint32_t* image;
    KeyRange kr;
    __device__ __forceinline__ void add(uint32_t row, uint32_t col, uint32_t cnt) const {
        const uint32_t bin = row * kr.W + col;
        atomicAdd(image + bin, cnt);
    }
};

constexpr int kTile = 32;

struct TileSink {
    uint32_t* image;
    uint32_t* tile;   // LDS, kTile * kTile bins of this wave
    uint32_t W, H;
    int col0, row0;   // image position of tile bin (0, 0)
    KeyRange kr;
    __device__ __forceinline__ void add(uint32_t row, uint32_t col, uint32_t cnt) const {
        const uint32_t tc = col - (uint32_t)col0, tr = row - (uint32_t)row0;
        if (tc < (uint32_t)kTile && tr < (uint32_t)kTile) atomicAdd(tile + tr * kTile + tc, cnt);
        else atomicAdd(image + row * W + col, cnt);
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

// A run is closed at a later word count than it was opened at, so a run
// inside the image always has a count of at least 1.
template <bool DROP, typename Sink>
__device__ __forceinline__ void close_run(Runs<DROP>& s, uint32_t t_words, const Sink& sink) {
    const uint32_t cnt = t_words - s.start;
    if (key_inside(s.key, sink.kr)) sink.add(key_row(s.key), key_col(s.key), cnt);
    else if (DROP) s.drop += cnt;
}

// close_run for a run whose key is `key` (the lane's state already holds the
// next run's key)
template <bool DROP, typename Sink>
__device__ __forceinline__ void close_run_key(Runs<DROP>& s, uint64_t key, uint32_t t_words, const Sink& sink) {
    const uint32_t cnt = t_words - s.start;
    if (key_inside(key, sink.kr)) sink.add(key_row(key), key_col(key), cnt);
    else if (DROP) s.drop += cnt;
}

// open a new run at word count t_words (its key outside until a word sets it)
template <bool DROP>
__device__ __forceinline__ void reset_run(Runs<DROP>& s, uint32_t t_words) {
    s.key = kOutsideKey;
    s.start = t_words;
}

// All tails of one head: the 3 blocks of suffixes whose first letter may
// follow the head's last letter, each walked in index order, 9 suffix
// points loaded from LDS ahead of their use.
// With MASKED, lanes whose `live` is false walk along without binning
// (their key stays kOutsideKey; the caller discards their count).
template <typename T, bool AFFINE, bool DUAL, bool MASKED = false, typename Sink = GlobalSink, bool DROP = false>
__device__ __forceinline__ void walk_tails_s(const Head<T>& h, const unsigned char* tail_lds, uint32_t R1,
                                             uint32_t W, uint32_t H, const Sink& sink, Runs<DROP>& s,
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
                    yb[u] = {T(1), T(0)};
                } else {
                    ya[u] = ((const cpx<T>*)tail_lds)[2 * (e0 + u)];
                    yb[u] = ((const cpx<T>*)tail_lds)[2 * (e0 + u) + 1];
                }
            }
            // the word counter is wave-uniform: keep it in a scalar register
            const uint32_t tw = __builtin_amdgcn_readfirstlane(t_words);
#pragma unroll
            for (uint32_t u = 0; u < 9; ++u) {
                T px, py;
                word_value<T, AFFINE, DUAL>(h, ya[u], yb[u], px, py);
                uint64_t key = run_key(px, py);
                if constexpr (DUAL)   // the general form can give NaN
                    if (!((px == px) & (py == py))) key = kOutsideKey;
                if (MASKED && !live) key = kOutsideKey;
                // the new key replaces the open run's unconditionally (a
                // rename, no copy); the run closes with the key it had
                const uint64_t open = s.key;
                s.key = key;
                if (key != open) {
                    close_run_key(s, open, tw + u, sink);
                    s.start = tw + u;
                }
            }
            t_words = tw + 9;
        }
    }
}

template <typename T, bool AFFINE, bool DUAL, bool MASKED = false, bool DROP = false>
__device__ __forceinline__ void walk_tails(const Head<T>& h, const unsigned char* tail_lds, uint32_t R1,
                                           uint32_t W, uint32_t H, uint32_t* image, Runs<DROP>& s,
                                           uint32_t& t_words, bool live = true) {
    walk_tails_s<T, AFFINE, DUAL, MASKED>(h, tail_lds, R1, W, H, GlobalSink{image, key_range(W, H)}, s, t_words,
                                          live);
}

// Whether some lane of the wave holds a head without a pole form (uniform).
template <typename T>
__device__ __forceinline__ bool wave_needs_dual(const Head<T>& h) { return __ballot(!h.pole) != 0; }

// Bin of the head's first allowed word in some lane, wave-uniform; kOutside
// if no lane's first word is in the window.
template <typename T, bool AFFINE>
__device__ __forceinline__ uint32_t first_key(const Head<T>& h, const unsigned char* tail_lds, uint32_t R1,
                                              uint32_t W, uint32_t H) {
    const uint32_t y1 = (uint32_t)(0 + (0 >= inv_letter(h.e)));
    T px, py;
    if constexpr (AFFINE)
        word_value<T, true, true>(h, ((const cpx<T>*)tail_lds)[y1 * R1], cpx<T>{T(1), T(0)}, px, py);
    else
        word_value<T, false, true>(h, ((const cpx<T>*)tail_lds)[2 * y1 * R1],
                                   ((const cpx<T>*)tail_lds)[2 * y1 * R1 + 1], px, py);
    const uint32_t key = bin_key(px, py, W, H);
    const uint64_t m = __ballot(key != kOutside);
    if (!m) return kOutside;
    return __shfl(key, __ffsll((unsigned long long)m) - 1, kWave);
}

// ------------------------------------------------------------------ block bounds
// Suffix nodes: the suffixes that share their first r - 3 letters, 27 of
// them, consecutive in the suffix table (node q holds entries 27q .. 27q +
// 26).  A head with last letter e walks the 3^(r-3) nodes under its three
// allowed first letters.
constexpr uint32_t kNodeWords = 27;
constexpr uint32_t kQueue = 128;          // span queue entries per wave
constexpr uint32_t kNodeGroup = 3;        // nodes classified together

template <typename T>
struct NodeDisk {
    T cr, ci, rho, pad;
};

// Per-precision constants of the bounds below, with eps the unit roundoff
// (2^-24 in FP32, 2^-53 in FP64): `sum` covers the rounding of c + S (4 and
// 8 eps), `up` enlarges a radius, `p` and `g` are the margin's coefficients
// (64 eps, and 1024 eps in FP32 and FP64 alike), and the guards keep every
// product of a word's evaluation finite and normal.
template <typename T> struct BoundK;
template <> struct BoundK<float> {
    static constexpr float sum = 0x1p-22f, up = 1.0f + 0x1p-20f, p = 0x1p-18f, g = 0x1p-14f, tiny = 0x1p-100f;
    static constexpr float umin_abs = 0x1p-30f, umax = 0x1p40f, gmax = 0x1p60f, pmax = 0x1p100f;
};
template <> struct BoundK<double> {
    static constexpr double sum = 0x1p-50, up = 1.0 + 0x1p-40, p = 0x1p-47, g = 0x1p-43, tiny = 0x1p-900;
    static constexpr double umin_abs = 0x1p-100, umax = 0x1p100, gmax = 0x1p300, pmax = 0x1p100;
};

__device__ __forceinline__ float babs(float x) { return __builtin_fabsf(x); }
__device__ __forceinline__ double babs(double x) { return __builtin_fabs(x); }
__device__ __forceinline__ float bmin(float x, float y) { return __builtin_fminf(x, y); }
__device__ __forceinline__ double bmin(double x, double y) { return __builtin_fmin(x, y); }
__device__ __forceinline__ float bmax(float x, float y) { return __builtin_fmaxf(x, y); }
__device__ __forceinline__ double bmax(double x, double y) { return __builtin_fmax(x, y); }
__device__ __forceinline__ float bound_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double bound_sqrt(double x) { return sqrt(x); }

// floor of a bound known to lie in (0, 2^31) where it is used; any value otherwise
__device__ __forceinline__ int bound_floor(float x) { return floor_i32(x); }
__device__ __forceinline__ int bound_floor(double x) {
    return (int)__builtin_floor(__builtin_fmin(__builtin_fmax(x, -1.0), 2147483647.0));
}

// Bounding disk of node q's suffix points: the centre c is the midpoint of
// their bounding box rounded to T; the radius is their largest distance
// from c, computed in FP64 and enlarged by 2^-40, plus BoundK<T>::sum
// (|c.re| + |c.im|), which covers the rounding of c + S in node_class; in
// FP32 it is rounded up.
template <typename T>
__device__ inline void node_disk(const cpx<T>* tail, uint32_t q, NodeDisk<T>* out) {
    const cpx<T>* p = tail + q * kNodeWords;
    T x0 = p[0].re, x1 = p[0].re, y0 = p[0].im, y1 = p[0].im;
    for (uint32_t t = 1; t < kNodeWords; ++t) {
        x0 = bmin(x0, p[t].re);
        x1 = bmax(x1, p[t].re);
        y0 = bmin(y0, p[t].im);
        y1 = bmax(y1, p[t].im);
    }
    const T cr = (T)(0.5 * ((double)x0 + (double)x1));
    const T ci = (T)(0.5 * ((double)y0 + (double)y1));
    double r2 = 0.0;
    for (uint32_t t = 0; t < kNodeWords; ++t) {
        const double dx = (double)p[t].re - (double)cr, dy = (double)p[t].im - (double)ci;
        r2 = fmax(r2, dx * dx + dy * dy);
    }
    const double rho = sqrt(r2) * (1.0 + 0x1p-40) + (double)BoundK<T>::sum * (fabs((double)cr) + fabs((double)ci)) +
                       0x1p-900;
    T rho_t;
    if constexpr (std::is_same<T, float>::value) rho_t = __double2float_ru(rho);
    else rho_t = rho;
    out[q] = {cr, ci, rho_t, T(0)};
}

// Constants of node_class for one head, formed once per unit.
template <typename T>
struct HeadBound {
    T gx, gy;       // |ax| + |bx|, |ay| + |by|
    T gxg, gyg;     // BoundK<T>::g times those
    T mPx, mPy;     // BoundK<T>::p |Px| + tiny, likewise Py
    T sS;           // covers the rounding of c + S: sum (1 + up) (|S.re| + |S.im|)
    bool ok;        // the products of one word stay finite (a NaN fails this too)
};

template <typename T>
__device__ __forceinline__ HeadBound<T> head_bound(const Head<T>& h) {
    using K = BoundK<T>;
    HeadBound<T> b;
    b.gx = babs(h.ax) + babs(h.bx);
    b.gy = babs(h.ay) + babs(h.by);
    b.gxg = b.gx * K::g;
    b.gyg = b.gy * K::g;
    b.mPx = fma_(babs(h.Px), K::p, K::tiny);
    b.mPy = fma_(babs(h.Py), K::p, K::tiny);
    b.sS = (babs(h.S.re) + babs(h.S.im)) * (K::sum * K::up);
    b.ok = bmax(b.gx, b.gy) <= K::gmax && babs(h.Px) <= K::pmax && babs(h.Py) <= K::pmax;
    return b;
}

// Where a pole-form head sends the 27 words of a node, as eval_pole computes
// them in T: kOutsideKey when every word's bin is outside the window, that bin's key
// when every word falls in one bin, kSpanKey when neither can be shown.
//
// For y in the disk D(c, rho) and w = c + S with |w| > rho, u = y + S lies
// in D(w, rho), so 1/u lies in the disk of centre conj(w) / den and radius
// rho / den, den = |w|^2 - rho^2, and the exact pole form px = Px + Re((ax
// + i bx) / u) lies within (|ax| + |bx|) rho / den of cx = Px + (ax w.re +
// bx w.im) / den; likewise py with ay, by.
//
// Margins, eps the unit roundoff of T.  (1) The evaluation at the same
// inputs (two sums, |u|^2 from a product and an FMA, a reciprocal within
// about one ulp, the numerator from a product and an FMA, the closing FMA)
// differs from the exact value by at most about eps (|Px| + 12 |ax + i bx| /
// |u|), with |u| >= |w| - rho.  (2) This function computes in T too: w's
// rounding is inside rho (node_disk, sS); with |w| - rho >= |w| / 64 (a
// guard) the computed |w| - rho is within about 200 eps of its value, and
// cx - Px, the radius and the reciprocal within about 420 eps of theirs,
// all relative to (|ax| + |bx|) / (|w| - rho).  The margin 64 eps |Px| +
// 1024 eps (|ax| + |bx|) / (|w| - rho) holds both with room.  Guards keep
// every product of the evaluation finite and normal, else kSpanKey; NaN fails
// them.
template <typename T>
__device__ __forceinline__ uint64_t node_class(const Head<T>& h, const HeadBound<T>& b, const NodeDisk<T>& d, T Wf,
                                               T Hf) {
    using K = BoundK<T>;
    const T wr = d.cr + h.S.re, wi = d.ci + h.S.im;
    const T rp = fma_(d.rho, K::up, b.sS);
    const T aw = bound_sqrt(fma_(wr, wr, wi * wi));
    const T umin = aw - rp, umax = aw + rp;
    const T inv = recip(umin * umax);
    const T kr = wr * inv, ki = wi * inv, kap = rp * inv, iu = umax * inv;
    const T cx = fma_(h.ax, kr, fma_(h.bx, ki, h.Px));
    const T cy = fma_(h.ay, kr, fma_(h.by, ki, h.Py));
    const T hx = fma_(b.gx, kap, fma_(b.gxg, iu, b.mPx));
    const T hy = fma_(b.gy, kap, fma_(b.gyg, iu, b.mPy));
    const T lx = cx - hx, ux = cx + hx, ly = cy - hy, uy = cy + hy;
    const bool ok = b.ok & (umin >= bmax(aw * T(0x1p-6), K::umin_abs)) & (umax <= K::umax);
    const bool out = (ux < T(0)) | (lx >= Wf) | (uy < T(0)) | (ly >= Hf);
    const int c0 = bound_floor(lx), c1 = bound_floor(ux), r0 = bound_floor(ly), r1 = bound_floor(uy);
    const bool one = (lx > T(0)) & (ux < Wf) & (ly > T(0)) & (uy < Hf) & (c0 == c1) & (r0 == r1);
    const uint64_t key = one ? bin_run_key((uint32_t)r0, (uint32_t)c0) : kSpanKey;
    return !ok ? kSpanKey : out ? kOutsideKey : key;
}

// Close a run of the bounded walk: bins add their count, runs outside the
// window are dropped words, kSpanKey runs were queued and add nothing here.
template <bool DROP>
__device__ __forceinline__ void close_bounded(Runs<DROP>& s, uint32_t t_words, const GlobalSink& sink) {
    const uint32_t cnt = t_words - s.start;
    if (key_inside(s.key, sink.kr)) sink.add(key_row(s.key), key_col(s.key), cnt);
    else if (DROP && s.key != kSpanKey) s.drop += cnt;
}

// Lanes q < c evaluate the 27 words of span-queue entry q (the head of lane
// entry >> 8, its node entry & 255) word by word, with eval_pole and
// bin_key as every other kernel, and run-length counts of their own.
template <typename T, bool DROP>
__device__ inline void drain_span_queue(const Head<T>& h, int lane, const uint16_t* queue, uint32_t c,
                                        const unsigned char* tail_lds, uint32_t per, uint32_t W, uint32_t H,
                                        uint32_t* image, Runs<DROP>& s) {
    const uint32_t entry = (uint32_t)lane < c ? queue[lane] : 0u;
    const int src = (int)(entry >> 8);
    Head<T> g;
    g.S.re = __shfl(h.S.re, src, kWave);
    g.S.im = __shfl(h.S.im, src, kWave);
    g.ax = __shfl(h.ax, src, kWave);
    g.bx = __shfl(h.bx, src, kWave);
    g.ay = __shfl(h.ay, src, kWave);
    g.by = __shfl(h.by, src, kWave);
    g.Px = __shfl(h.Px, src, kWave);
    g.Py = __shfl(h.Py, src, kWave);
    const int e = __shfl(h.e, src, kWave);
    if ((uint32_t)lane < c) {
        const uint32_t n = entry & 255u;
        const uint32_t j = n / per, sub = n - j * per;
        const uint32_t y1 = j + (j >= (uint32_t)inv_letter(e));
        const uint32_t base = (y1 * per + sub) * kNodeWords;
        uint32_t cur = kOutside, cnt = 0;
        for (uint32_t t0 = 0; t0 < kNodeWords; t0 += 9) {
            cpx<T> ya[9];
#pragma unroll
            for (uint32_t u = 0; u < 9; ++u) ya[u] = ((const cpx<T>*)tail_lds)[base + t0 + u];
#pragma unroll
            for (uint32_t u = 0; u < 9; ++u) {
                T px, py;
                eval_pole(g, ya[u], px, py);
                const uint32_t key = bin_key(px, py, W, H);
                if (key != cur) {
                    if (cur != kOutside) atomicAdd(image + cur, cnt);
                    else if (DROP) s.drop += cnt;
                    cur = key;
                    cnt = 0;
                }
                ++cnt;
            }
        }
        if (cur != kOutside) atomicAdd(image + cur, cnt);
        else if (DROP) s.drop += cnt;
    }
}

// One full unit of 64 pole-form heads over an affine suffix table, node by
// node: each lane classifies its head's node (node_class); bins and
// outside nodes extend the lane's run like single words, spanning nodes go
// to the wave's queue, which lanes drain 64 entries at a time and at the
// end of the unit.  The word counter advances 27 per node, so the runs
// count exactly the words the per-word walk would.
template <typename T, bool DROP>
__device__ inline void bounded_unit(const Head<T>& h, int lane, const unsigned char* tail_lds,
                                    const NodeDisk<T>* nodes, uint16_t* queue, uint32_t per, uint32_t W, uint32_t H,
                                    uint32_t* image, Runs<DROP>& s, uint32_t& t_words) {
    const int ie = inv_letter(h.e);
    const HeadBound<T> hb = head_bound(h);
    const T Wf = (T)W, Hf = (T)H;
    const GlobalSink sink{image, key_range(W, H)};
    // a word's key can equal kSpanKey: close the run the per-word walk left
    // open, so that close_bounded sees only node_class's keys
    close_run(s, t_words, sink);
    reset_run(s, t_words);
    uint32_t qn = 0;   // queued entries (wave-uniform)
    auto drain = [&](uint32_t c) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        drain_span_queue<T, DROP>(h, lane, queue, c, tail_lds, per, W, H, image, s);
        const uint32_t rest = qn - c;
        const uint16_t v = (uint32_t)lane < rest ? queue[c + lane] : (uint16_t)0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if ((uint32_t)lane < rest) queue[lane] = v;
        qn = rest;
    };
    // one node's verdict: extend or close the lane's run, queue a spanning node
    auto step = [&](uint64_t key, uint32_t n) {
        const uint32_t tw = __builtin_amdgcn_readfirstlane(t_words);
        if (key != s.key) {
            close_bounded(s, tw, sink);
            s.key = key;
            s.start = tw;
        }
        const uint64_t span = __ballot(key == kSpanKey);
        if (span) {
            if (key == kSpanKey) {
                const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(span >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)span, 0u));
                queue[qn + below] = (uint16_t)(((uint32_t)lane << 8) | n);
            }
            qn += (uint32_t)__popcll(span);
            if (qn >= (uint32_t)kWave) drain((uint32_t)kWave);
        }
        t_words = tw + kNodeWords;
    };
    for (uint32_t j = 0; j < 3; ++j) {
        const uint32_t y1 = j + (j >= (uint32_t)ie);
        const NodeDisk<T>* nd = nodes + y1 * per;
        if (per % kNodeGroup == 0) {
            // kNodeGroup nodes at a time: their disks read together, their verdicts independent
            for (uint32_t sub0 = 0; sub0 < per; sub0 += kNodeGroup) {
                NodeDisk<T> dk[kNodeGroup];
#pragma unroll
                for (uint32_t u = 0; u < kNodeGroup; ++u) dk[u] = nd[sub0 + u];
                uint64_t key[kNodeGroup];
#pragma unroll
                for (uint32_t u = 0; u < kNodeGroup; ++u) key[u] = node_class(h, hb, dk[u], Wf, Hf);
#pragma unroll
                for (uint32_t u = 0; u < kNodeGroup; ++u) step(key[u], j * per + sub0 + u);
            }
        } else {
            for (uint32_t sub = 0; sub < per; ++sub) step(node_class(h, hb, nd[sub], Wf, Hf), j * per + sub);
        }
    }
    // the words of a queued node are counted by the drain, not by the run
    if (s.key == kSpanKey) reset_run(s, t_words);
    while (qn > 0) drain(qn < (uint32_t)kWave ? qn : (uint32_t)kWave);
}

template <typename T, bool AFFINE, bool LDSHIST, bool DROP, bool BOUNDED>
__device__ __forceinline__ void render_units(const RenderArgs& a, const unsigned char* tail_lds, const m64* G,
                                             uint32_t* tile, const NodeDisk<T>* nodes, uint16_t* queue,
                                             Runs<DROP>& s) {
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t waves = gridDim.x * (kBlock / kWave);
    const uint32_t gwave = blockIdx.x * (kBlock / kWave) + (threadIdx.x / kWave);
    uint32_t t_words = 0;
    const KeyRange kr = key_range(a.W, a.H);
    const GlobalSink gs{a.image, kr};
    TileSink ts{a.image, tile, a.W, a.H, -(1 << 30), -(1 << 30), kr};
    for (uint32_t unit = gwave; unit < a.n_units; unit += waves) {
        const uint64_t local = (uint64_t)unit * kWave + lane;
        const bool full = (uint64_t)(unit + 1) * kWave <= a.n_heads;
        const bool live = local < a.n_heads;
        const uint64_t hidx = a.head_begin + (live ? local : a.n_heads - 1);
        const Head<T> h = compute_head<T>(hidx, a.sp, a.tab.prefix, a.tab.prefix_last, G, a.fold);
        const bool dual = wave_needs_dual(h);
        if constexpr (BOUNDED && AFFINE && !LDSHIST) {
            if (full && !dual) {
                bounded_unit<T, DROP>(h, lane, tail_lds, nodes, queue, a.sp.R1 / kNodeWords, a.W, a.H, a.image, s,
                                      t_words);
                continue;
            }
        }
        if constexpr (LDSHIST) {
            // move the tile to where this unit's words start
            const uint32_t k0 = first_key<T, AFFINE>(h, tail_lds, a.sp.R1, a.W, a.H);
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
            if constexpr (LDSHIST) {
                if (dual) walk_tails_s<T, AFFINE, true>(h, tail_lds, a.sp.R1, a.W, a.H, ts, s, t_words);
                else walk_tails_s<T, AFFINE, false>(h, tail_lds, a.sp.R1, a.W, a.H, ts, s, t_words);
            } else {
                if (dual) walk_tails<T, AFFINE, true>(h, tail_lds, a.sp.R1, a.W, a.H, a.image, s, t_words);
                else walk_tails<T, AFFINE, false>(h, tail_lds, a.sp.R1, a.W, a.H, a.image, s, t_words);
            }
        } else {
            // last, partial unit: idle lanes walk a valid head without binning
            // and their count is discarded
            close_run(s, t_words, gs);
            reset_run(s, t_words);
            walk_tails<T, AFFINE, true, true>(h, tail_lds, a.sp.R1, a.W, a.H, a.image, s, t_words, live);
            if (live) close_run(s, t_words, gs);
            reset_run(s, t_words);
        }
    }
    if constexpr (LDSHIST) {
        close_run(s, t_words, ts);
        ts.merge(lane);
    } else {
        close_run(s, t_words, gs);
    }
}

// One wave per unit of 64 consecutive heads, units dealt round robin over
// the persistent waves.  Per word: one Moebius map of an LDS suffix point,
// the bin, and a run-length counter: a lane adds to the image only when its
// bin changes (consecutive tails of one head lie close together), and keeps
// its dropped words in a register until the end.
// LDS: suffix table (sized for the homogeneous form), generators, and with
// LDSHIST one 32 x 32 tile of uint32 bins per wave.  With BOUNDED (FP32,
// affine suffix tables, r >= 4) full units of pole-form heads go node by
// node (bounded_unit); LDS then also holds the nodes' bounding disks and
// one span queue per wave.
template <typename T, bool LDSHIST, bool DROP, bool BOUNDED>
__device__ __forceinline__ void render_body(const RenderArgs& a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t n_tail = 4 * a.sp.R1;
    const bool affine = tail_affine_block(a.tab);
    const size_t entry = affine ? sizeof(cpx<T>) : 2 * sizeof(cpx<T>);
    const size_t tbytes = (n_tail * entry + 15) & ~size_t(15);
    const size_t tmax = (n_tail * 2 * sizeof(cpx<T>) + 15) & ~size_t(15);
    m64* G = (m64*)(smem + tbytes);
    uint32_t* tile = (uint32_t*)(smem + tmax + 4 * sizeof(m64)) + (threadIdx.x / kWave) * (kTile * kTile);
    NodeDisk<T>* nodes = (NodeDisk<T>*)(smem + tmax + 4 * sizeof(m64));
    const uint32_t n_nodes = BOUNDED ? n_tail / kNodeWords : 0u;
    uint16_t* queue = (uint16_t*)(nodes + n_nodes) + (threadIdx.x / kWave) * kQueue;
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
    if constexpr (BOUNDED) {
        if (affine) {
            for (uint32_t q = threadIdx.x; q < n_nodes; q += blockDim.x) node_disk((const cpx<T>*)smem, q, nodes);
            __syncthreads();
        }
    }
    Runs<DROP> s = {kOutsideKey, 0, 0};
    if (affine) render_units<T, true, LDSHIST, DROP, BOUNDED>(a, smem, G, tile, nodes, queue, s);
    else render_units<T, false, LDSHIST, DROP, false>(a, smem, G, tile, nodes, queue, s);
    if (DROP) {
        uint64_t drop = s.drop;
        for (int off = kWave / 2; off > 0; off >>= 1) drop += __shfl_down(drop, off, kWave);
        if ((threadIdx.x & (kWave - 1)) == 0 && drop)
            atomicAdd((unsigned long long*)a.dropped, (unsigned long long)drop);
    }
}

template <typename T, bool LDSHIST, bool DROP>
__global__ __launch_bounds__(kBlock) void render_kernel(const RenderArgs a) {
    render_body<T, LDSHIST, DROP, false>(a);
}

// The block-bounds variant (run-length histogram).  Its node
// classification and span drains are chains of dependent operations, so it
// is held to at least kBoundedWaves waves per SIMD to hide their latency
// (fewer in FP64, whose values take two registers each).
template <typename T>
constexpr int kBoundedWaves = std::is_same<T, float>::value ? 5 : 3;

template <typename T, bool DROP>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kBoundedWaves<T>)))
void render_bounded_kernel(const RenderArgs a) {
    render_body<T, false, DROP, true>(a);
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
template <typename T>
__device__ inline void word_point(uint64_t i, const Split& sp, const Tables& tab, const void* tail_homog,
                                  const Fold& fold, const m64* G, bool affine, T& px, T& py) {
    Head<T> h;
    uint64_t entry;
    if (sp.k + sp.m == 0) {
        h = compute_head<T>(0, sp, nullptr, nullptr, G, fold);
        entry = i;
    } else {
        const uint64_t hidx = i / sp.R;
        const uint32_t t = (uint32_t)(i - hidx * sp.R);
        h = compute_head<T>(hidx, sp, tab.prefix, tab.prefix_last, G, fold);
        const uint32_t j = t / sp.R1;
        const uint32_t tt = t - j * sp.R1;
        const int y1 = (int)j + ((int)j >= inv_letter(h.e));
        entry = (uint64_t)y1 * sp.R1 + tt;
    }
    if (affine) {
        const cpx<T> y = ((const cpx<T>*)tab.tail)[entry];
        if (h.pole) eval_pole(h, y, px, py);
        else eval_general(h, y, px, py);
    } else {
        const cpx<T>* hm = (const cpx<T>*)tail_homog;
        if (h.pole) eval_pole_h(h, hm[2 * entry], hm[2 * entry + 1], px, py);
        else eval_general_h(h, hm[2 * entry], hm[2 * entry + 1], px, py);
    }
}

template <typename T>
__device__ inline void word_point(uint64_t i, const PerWordArgs& a, const m64* G, bool affine, T& px, T& py) {
    word_point<T>(i, a.sp, a.tab, a.tail_homog, a.fold, G, affine, px, py);
}

// Runs of equal bins among consecutive lanes of a wave (consecutive words of
// one head mostly share a bin): the first lane of a run gets the run's
// length, the others 0.  `tag` separates runs that must not merge (the set
// of a batched word); kDead marks a lane without a word.  All lanes of the
// wave take part.
constexpr uint32_t kDead = 0xFFFFFFFEu;

__device__ __forceinline__ uint32_t lane_run_length(uint32_t key, uint32_t tag) {
    const int lane = (int)(threadIdx.x & (kWave - 1));
    const uint32_t pk = __shfl_up(key, 1, kWave), pt = __shfl_up(tag, 1, kWave);
    const bool first = lane == 0 || key != pk || tag != pt;
    const uint64_t starts = __ballot(first);
    const uint64_t later = lane == kWave - 1 ? 0ull : starts & (~0ull << (lane + 1));
    const int next = later ? __ffsll((unsigned long long)later) - 1 : kWave;
    return first ? (uint32_t)(next - lane) : 0u;
}

template <typename T>
__global__ __launch_bounds__(256) void perword_render_kernel(const PerWordArgs a) {
    __shared__ m64 G[4];
    if (threadIdx.x < 4) G[threadIdx.x] = a.gens.g[threadIdx.x];
    const bool affine = tail_affine_block(a.tab);  // also orders the G stores before their use
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t key = kDead;
    if (tid < a.count0 + a.count1) {
        const uint64_t i = tid < a.count0 ? a.first0 + tid : a.first1 + (tid - a.count0);
        T px, py;
        word_point<T>(i, a, G, affine, px, py);
        key = bin_key(px, py, a.W, a.H);
    }
    // one atomic per run of equal bins
    const uint32_t len = lane_run_length(key, 0u);
    uint64_t drop = 0;
    if (len && key == kOutside) drop = len;
    else if (len && key != kDead) atomicAdd(a.image + key, len);
    if (a.dropped) {
        for (int off = kWave / 2; off > 0; off >>= 1) drop += __shfl_down(drop, off, kWave);
        if ((threadIdx.x & (kWave - 1)) == 0 && drop)
            atomicAdd((unsigned long long*)a.dropped, (unsigned long long)drop);
    }
}

// Words of several sets (their tables built by the batch table kernels, one
// form flag word per set), one per thread.  A run of equal bins of one set
// among consecutive lanes is added with one atomic, to its image or to its
// dropped counter.
template <typename T>
__global__ __launch_bounds__(256) void perword_batch_kernel(const PerWordBatchJob a) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    // every lane of a block takes part in every round (lane_run_length)
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < a.total; base += stride) {
        const uint64_t w = base + threadIdx.x;
        uint32_t key = kDead, tag = 0xFFFFFFFFu;
        const SetDesc* S = nullptr;
        if (w < a.total) {
            int lo = 0, hi = a.n - 1;   // the last q with word_offsets[q] <= w
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (a.word_offsets[mid] <= w) lo = mid;
                else hi = mid - 1;
            }
            S = &a.sets[a.set_ids[lo]];
            const bool affine = S->tab.tail_flags[0] == 0u;
            T px, py;
            word_point<T>(w - a.word_offsets[lo], S->sp, S->tab, S->tail_homog, a.fold, S->gens.g, affine, px, py);
            key = bin_key(px, py, a.width, a.height);
            tag = (uint32_t)lo;
        }
        // one atomic per run of equal bins of one set
        const uint32_t len = lane_run_length(key, tag);
        if (len && key != kDead) {
            if (key != kOutside) atomicAdd(S->image + key, len);
            else if (S->dropped) atomicAdd((unsigned long long*)S->dropped, (unsigned long long)len);
        }
    }
}

hipError_t launch_perword_batch(const PerWordBatchJob& job, hipStream_t s) {
    if (job.total == 0) return hipSuccess;
    const uint64_t blocks = std::min<uint64_t>((job.total + 255) / 256, 8192);
    if (job.precision == KL_PREC_FP64)
        hipLaunchKernelGGL(perword_batch_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s, job);
    else
        hipLaunchKernelGGL(perword_batch_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s, job);
    return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void eval_kernel(const PerWordArgs a) {
    __shared__ m64 G[4];
    if (threadIdx.x < 4) G[threadIdx.x] = a.gens.g[threadIdx.x];
    const bool affine = tail_affine_block(a.tab);  // also orders the G stores before their use
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= a.n) return;
    const uint64_t i = a.idx[tid];
    if (i >= a.n_words) {
        a.out[tid] = {__builtin_nan(""), __builtin_nan("")};
        return;
    }
    T px, py;
    word_point<T>(i, a, G, affine, px, py);
    a.out[tid] = {(double)px, (double)py};
}

}  // namespace kl

namespace kl {

template <typename T>
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
        const size_t n_tail = 4 * (size_t)job.sp.R1;
        const bool ldsh = job.hist_mode == KL_HIST_LDS;
        const bool bounded = job.bounded && !ldsh && job.sp.r >= 4;
        const size_t lds = ((n_tail * 2 * sizeof(cpx<T>) + 15) & ~size_t(15)) + 4 * sizeof(m64) +
                           (ldsh ? (kBlock / kWave) * kTile * kTile * sizeof(uint32_t) : 0) +
                           (bounded ? n_tail / kNodeWords * sizeof(NodeDisk<T>) + (kBlock / kWave) * kQueue * 2 : 0);
        const bool drop = job.dropped != nullptr;
        void (*kern)(RenderArgs) = ldsh ? (drop ? render_kernel<T, true, true> : render_kernel<T, true, false>)
                                        : (drop ? render_kernel<T, false, true> : render_kernel<T, false, false>);
        if (bounded) kern = drop ? render_bounded_kernel<T, true> : render_bounded_kernel<T, false>;
        const void* fn = reinterpret_cast<const void*>(kern);
        if (lds > 65536) {
            hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        uint32_t grid = (uint32_t)job.grid_blocks;
        const uint32_t need = (job.n_units + (kBlock / kWave) - 1) / (kBlock / kWave);
        if (grid > need) grid = need;
        if (grid < 1) grid = 1;
        hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), lds, s, a);
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
        hipLaunchKernelGGL((perword_render_kernel<T>), dim3((unsigned)blocks), dim3(256), 0, s, p);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_render(const RenderJob& job, hipStream_t s) {
    return job.precision == KL_PREC_FP64 ? launch_render_t<double>(job, s) : launch_render_t<float>(job, s);
}

template <typename T>
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
    hipLaunchKernelGGL((eval_kernel<T>), dim3((unsigned)blocks), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_eval(const EvalJob& job, hipStream_t s) {
    if (job.n == 0) return hipSuccess;
    return job.precision == KL_PREC_FP64 ? launch_eval_t<double>(job, s) : launch_eval_t<float>(job, s);
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
    tail_entry<T>(g, S.sp.r, t, S.seed, (cpx<T>*)S.tab.tail, (cpx<T>*)S.tail_homog, flags);
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
    const uint64_t* unit_offsets;  // n_sets + 1 prefix sums of block units
    int n_sets;
    uint64_t total_units;
    Fold fold;
    uint32_t W, H;
    uint32_t table_bytes;          // LDS bytes of the largest suffix table (homogeneous form)
    uint32_t max_nodes;            // block bounds: suffix nodes of the largest table
};

__device__ __forceinline__ void flush_drop(uint64_t& drop, uint64_t* dst) {
    uint64_t d = drop;
    for (int off = kWave / 2; off > 0; off >>= 1) d += __shfl_down(d, off, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0 && d && dst) atomicAdd((unsigned long long*)dst, (unsigned long long)d);
    drop = 0;
}

// Block units of kBlock heads (64 per wave) from every set form one queue
// dealt round robin over the persistent blocks.  A block keeps the suffix
// table and generators of the set it is working on in LDS, shared by its
// waves, and reloads them between two barriers when its next unit belongs
// to another set.  The last unit of a set may be partial: waves past the
// set's last head skip it, and the idle lanes of a partly filled wave walk a
// valid head without binning.
template <typename T, bool DROP, bool BOUNDED = false>
__global__ __launch_bounds__(kBlock) void render_batch_kernel(const BatchArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    m64* G = (m64*)(smem + a.table_bytes);
    const uint64_t wid = threadIdx.x / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    // with BOUNDED: the set's node disks and one span queue per wave (bounded_unit)
    NodeDisk<T>* nodes = (NodeDisk<T>*)(smem + a.table_bytes + 4 * sizeof(m64));
    uint16_t* queue = (uint16_t*)(nodes + a.max_nodes) + wid * kQueue;

    int cur = -1;
    bool affine = true;
    Split sp{};
    const m64* prefix = nullptr;
    const uint8_t* plast = nullptr;
    uint32_t* image = nullptr;
    uint64_t* dropped = nullptr;
    uint64_t base = 0;
    Runs<DROP> s = {kOutsideKey, 0, 0};
    uint32_t t_words = 0;
    const KeyRange kr = key_range(a.W, a.H);

    for (uint64_t unit = blockIdx.x; unit < a.total_units; unit += gridDim.x) {
        // set of this unit: the last set whose first unit is <= unit (uniform over the block)
        int lo = 0, hi = a.n_sets - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.unit_offsets[mid] <= unit) lo = mid;
            else hi = mid - 1;
        }
        if (lo != cur) {
            if (cur >= 0) {
                close_run(s, t_words, GlobalSink{image, kr});
                if (DROP) flush_drop(s.drop, dropped);
            }
            reset_run(s, t_words);
            cur = lo;
            const SetDesc& S = a.sets[cur];
            sp = S.sp;
            prefix = S.tab.prefix;
            plast = S.tab.prefix_last;
            image = S.image;
            dropped = S.dropped;
            base = a.unit_offsets[cur];
            __syncthreads();  // every wave is done with the previous set's table
            affine = tail_affine_block(S.tab);
            const size_t bytes = (size_t)S.n_tail * (affine ? 1 : 2) * sizeof(cpx<T>);
            const uint4* src = (const uint4*)(affine ? S.tab.tail : S.tail_homog);
            for (uint32_t i = threadIdx.x; i < (uint32_t)((bytes + 15) / 16); i += kBlock) ((uint4*)smem)[i] = src[i];
            if (threadIdx.x < 4) G[threadIdx.x] = S.gens.g[threadIdx.x];
            if constexpr (BOUNDED) {
                if (affine && sp.r >= 4) {
                    __syncthreads();
                    for (uint32_t q = threadIdx.x; q < S.n_tail / kNodeWords; q += kBlock)
                        node_disk((const cpx<T>*)smem, q, nodes);
                }
            }
            __syncthreads();
        }
        const uint64_t wunit = (unit - base) * (kBlock / kWave) + wid;  // this wave's 64 heads of the set
        if (wunit * kWave >= sp.n_heads) continue;
        uint64_t hidx = wunit * kWave + lane;
        const bool partial = (wunit + 1) * kWave > sp.n_heads;
        if (!partial) {
            const Head<T> h = compute_head<T>(hidx, sp, prefix, plast, G, a.fold);
            const bool dual = wave_needs_dual(h);
            if constexpr (BOUNDED) {
                if (affine && !dual && sp.r >= 4) {
                    bounded_unit<T, DROP>(h, lane, smem, nodes, queue, sp.R1 / kNodeWords, a.W, a.H, image, s,
                                          t_words);
                    continue;
                }
            }
            if (dual) {
                if (affine) walk_tails<T, true, true>(h, smem, sp.R1, a.W, a.H, image, s, t_words);
                else walk_tails<T, false, true>(h, smem, sp.R1, a.W, a.H, image, s, t_words);
            } else {
                if (affine) walk_tails<T, true, false>(h, smem, sp.R1, a.W, a.H, image, s, t_words);
                else walk_tails<T, false, false>(h, smem, sp.R1, a.W, a.H, image, s, t_words);
            }
        } else {
            const bool live = hidx < sp.n_heads;
            if (!live) hidx = sp.n_heads - 1;
            close_run(s, t_words, GlobalSink{image, kr});
            reset_run(s, t_words);
            const Head<T> h = compute_head<T>(hidx, sp, prefix, plast, G, a.fold);
            if (affine) walk_tails<T, true, true, true>(h, smem, sp.R1, a.W, a.H, image, s, t_words, live);
            else walk_tails<T, false, true, true>(h, smem, sp.R1, a.W, a.H, image, s, t_words, live);
            if (live) close_run(s, t_words, GlobalSink{image, kr});
            reset_run(s, t_words);
        }
    }
    if (cur >= 0) {
        close_run(s, t_words, GlobalSink{image, kr});
        if (DROP) flush_drop(s.drop, dropped);
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
    a.table_bytes = job.table_bytes;
    const bool fp64 = job.precision == KL_PREC_FP64;
    const size_t esz = fp64 ? sizeof(cpx<double>) : sizeof(cpx<float>);
    // the largest table's suffix nodes (the table bytes hold its homogeneous form)
    a.max_nodes = job.bounded ? (uint32_t)(job.table_bytes / (2 * esz) / kNodeWords) : 0u;
    const size_t lds = (size_t)job.table_bytes + 4 * sizeof(m64) +
                       (job.bounded ? (size_t)a.max_nodes * (fp64 ? sizeof(NodeDisk<double>) : sizeof(NodeDisk<float>)) +
                                          (kBlock / kWave) * kQueue * 2
                                    : 0);
    uint32_t grid = (uint32_t)std::min<uint64_t>(job.total_units, (uint64_t)job.grid_blocks);
    if (grid < 1) grid = 1;
    const bool drop = job.count_dropped != 0;
    void (*kern)(BatchArgs) =
        job.bounded ? (fp64 ? (drop ? render_batch_kernel<double, true, true> : render_batch_kernel<double, false, true>)
                            : (drop ? render_batch_kernel<float, true, true> : render_batch_kernel<float, false, true>))
                    : (fp64 ? (drop ? render_batch_kernel<double, true> : render_batch_kernel<double, false>)
                            : (drop ? render_batch_kernel<float, true> : render_batch_kernel<float, false>));
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), lds, s, a);
    return hipGetLastError();
}

}  // namespace kl

namespace kl {

hipError_t launch_setup(const SetupJob& j, hipStream_t s) {
    SetupArgs a;
    a.g = j.gens;
    a.k = j.k;
    a.r = j.r;
    a.seed = j.seed;
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
    a.nb_tail = (a.n_tail + 255) / 256;
    uint64_t blocks = a.nb_tail + (a.n_prefix + 255) / 256;
    if (a.image) blocks = std::max<uint64_t>(blocks, std::min<uint64_t>(2048, (a.bins / 4 + 255) / 256));
    if (j.precision == KL_PREC_FP64)
        hipLaunchKernelGGL(setup_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(setup_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace kl
