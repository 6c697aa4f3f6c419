// walk.hip -- the probabilistic approach of Section 4: random walks on the
// group, one orbit per walker, drawn into the density image.
//
// The paper describes this approach only in words: one word grows as
// generators are appended through random picks under some probability law,
// and the orbit of a point under it is drawn.  Here a walker takes a
// uniform first letter c_0, starts at that generator's attracting fixed
// point, and at step k picks c_k uniformly among the three letters that do
// not undo c_{k-1} (so the word stays reduced) and maps its point:
// z_k = G_{c_k}(z_{k-1}).  z_k is then the value of the reduced word
// c_k ... c_1 c_0 from the fixed point of its last letter (Section 1).
// After burn_in steps the walker draws its next n_steps points.  The
// commutator "boost" of the Fig. 3 caption is not applied.
//
// Random numbers: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel
// random numbers: as easy as 1, 2, 3", SC'11), counter-based, so that any
// walker's stream is reached without running the others.  Walker w's k-th
// 32-bit value is half k % 2 (low first) of output (k % 8) / 2 of the block
// at the counter (k / 8, w, 0, 0) under the key (seed, 0).  c_0 is the top
// two bits of value 0; c_k (k >= 1) is the floor(3 x / 2^32)-th letter, in
// code order, other than the inverse of c_{k-1}.
//
// Kernel: one thread per walker.  A Philox block gives the thread its next
// eight decisions; the point moves as a homogeneous pair (u : v), the four
// maps read from LDS, rescaled by a power of two (exact) every eight steps;
// each drawn point is u / v, folded into pixel coordinates and binned with
// the renderer's rule (0 <= px < W, 0 <= py < H as IEEE comparisons, NaN and
// infinity outside), one global atomic per point in the window: the points
// of a walk jump across the limit set, so there are no runs to merge.
#include <hip/hip_runtime.h>

#include "kl_internal.hpp"

namespace kl {

namespace {

constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull, kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull, kPhiloxW1 = 0xBB67AE8584CAA73Bull;

// Ten Philox4x64 rounds: each takes the 128-bit products of words 0 and 2
// with the two multipliers and mixes their halves with words 1 and 3 and
// the key; the key advances by the two Weyl constants between rounds.
__device__ __forceinline__ void philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                              uint64_t k1, uint64_t out[4]) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += kPhiloxW0;
            k1 += kPhiloxW1;
        }
        const uint64_t hi0 = __umul64hi(kPhiloxM0, c0), lo0 = kPhiloxM0 * c0;
        const uint64_t hi1 = __umul64hi(kPhiloxM1, c2), lo1 = kPhiloxM1 * c2;
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// bin of pixel coordinates, the renderer's rule; kWalkOutside when outside
constexpr uint32_t kWalkOutside = 0xFFFFFFFFu;

__device__ __forceinline__ uint32_t walk_bin(float px, float py, uint32_t W, uint32_t H) {
    const bool ok = (px >= 0.0f) & (px < (float)W) & (py >= 0.0f) & (py < (float)H);
    return ok ? (uint32_t)__builtin_floorf(py) * W + (uint32_t)__builtin_floorf(px) : kWalkOutside;
}

__device__ __forceinline__ uint32_t walk_bin(double px, double py, uint32_t W, uint32_t H) {
    const bool ok = (px >= 0.0) & (px < (double)W) & (py >= 0.0) & (py < (double)H);
    return ok ? (uint32_t)__builtin_floor(py) * W + (uint32_t)__builtin_floor(px) : kWalkOutside;
}

__device__ __forceinline__ float wabs(float x) { return __builtin_fabsf(x); }
__device__ __forceinline__ double wabs(double x) { return __builtin_fabs(x); }
__device__ __forceinline__ float wmax(float x, float y) { return __builtin_fmaxf(x, y); }
__device__ __forceinline__ double wmax(double x, double y) { return __builtin_fmax(x, y); }
__device__ __forceinline__ float wldexp(float x, int e) { return __builtin_ldexpf(x, e); }
__device__ __forceinline__ double wldexp(double x, int e) { return __builtin_ldexp(x, e); }
__device__ __forceinline__ int wexp(float x) { return __builtin_amdgcn_frexp_expf(x); }
__device__ __forceinline__ int wexp(double x) { return __builtin_amdgcn_frexp_exp(x); }

// (u : v) scaled by the power of two that brings its largest component into
// [0.5, 1); exact, and the point u / v is unchanged
template <typename T>
__device__ __forceinline__ void walk_rescale(cpx<T>& u, cpx<T>& v) {
    const T m = wmax(wmax(wabs(u.re), wabs(u.im)), wmax(wabs(v.re), wabs(v.im)));
    if (m > T(0) && m < T(INFINITY)) {
        const int e = -wexp(m);
        u = {wldexp(u.re, e), wldexp(u.im, e)};
        v = {wldexp(v.re, e), wldexp(v.im, e)};
    }
}

template <typename T>
__device__ __forceinline__ T walk_recip(T x) { return T(1) / x; }

template <typename T>
__global__ __launch_bounds__(256) void walk_kernel(const WalkJob j) {
    __shared__ mat<T> G[4];
    __shared__ cpx<T> SU[4], SV[4];
    if (threadIdx.x < 4) {
        const m64& g = j.gens.g[threadIdx.x];
        G[threadIdx.x] = {{(T)g.a.re, (T)g.a.im}, {(T)g.b.re, (T)g.b.im}, {(T)g.c.re, (T)g.c.im},
                          {(T)g.d.re, (T)g.d.im}};
        const bool inf = (j.gens.inf_mask >> threadIdx.x) & 1u;
        SU[threadIdx.x] = inf ? cpx<T>{T(1), T(0)} : cpx<T>{(T)j.gens.fix[threadIdx.x].re, (T)j.gens.fix[threadIdx.x].im};
        SV[threadIdx.x] = inf ? cpx<T>{T(0), T(0)} : cpx<T>{T(1), T(0)};
    }
    __syncthreads();
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t drop = 0;
    if (tid < j.n_walkers) {
        const uint64_t walker = j.first_walker + tid;
        const uint32_t n_total = 1 + j.burn_in + j.n_steps;
        const T s = (T)j.fold.s, ox = (T)j.fold.o.re, oy = (T)j.fold.o.im, an = (T)j.fold.aniso;
        cpx<T> u = {T(0), T(0)}, v = {T(1), T(0)};
        int prev = 0;
        uint32_t k = 0;
        for (uint64_t blk = 0; k < n_total; ++blk) {
            uint64_t r[4];
            philox4x64_10(blk, walker, 0, 0, j.seed, 0, r);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                if (k < n_total) {
                    const uint32_t x = (uint32_t)(r[i >> 1] >> (32 * (i & 1)));
                    int c;
                    if (k == 0) {
                        c = (int)(x >> 30);
                        u = SU[c];
                        v = SV[c];
                    } else {
                        const int t = (int)__umulhi(x, 3u);
                        c = t + (t >= (prev ^ 2));
                        const mat<T> g = G[c];
                        const cpx<T> nu = cfma(g.a, u, cmul(g.b, v));
                        const cpx<T> nv = cfma(g.c, u, cmul(g.d, v));
                        u = nu;
                        v = nv;
                    }
                    if (j.mode == kWalkLetters) j.letters[tid * n_total + k] = (uint8_t)c;
                    if (k > j.burn_in && j.mode != kWalkLetters) {
                        // z = u / v, then the window's affine map s z + o (x anisotropy on the real part)
                        const T n2 = fma_(v.re, v.re, v.im * v.im);
                        const T rc = walk_recip(n2);
                        const T zr = fma_(u.re, v.re, u.im * v.im) * rc;
                        const T zi = fma_(u.im, v.re, -(u.re * v.im)) * rc;
                        const T px = fma_(s, zr, ox) * an, py = fma_(s, zi, oy);
                        const uint64_t p = tid * j.n_steps + (k - j.burn_in - 1);
                        if (j.mode == kWalkEval) {
                            j.z_out[p] = {(double)px, (double)py};
                        } else {
                            const uint32_t b = walk_bin(px, py, j.W, j.H);
                            if (b != kWalkOutside) atomicAdd(j.image + b, 1u);
                            else ++drop;
                        }
                    }
                    prev = c;
                    ++k;
                }
            }
            walk_rescale(u, v);
        }
    }
    if (j.mode == kWalkRender && j.dropped) {
        for (int off = 32; off > 0; off >>= 1) drop += __shfl_down(drop, off, 64);
        if ((threadIdx.x & 63) == 0 && drop) atomicAdd((unsigned long long*)j.dropped, (unsigned long long)drop);
    }
}

}  // namespace

// Walkers go in launches of at most 2^30 (2^22 blocks), each with its
// outputs advanced to its first walker.
hipError_t launch_walk(const WalkJob& j, hipStream_t s) {
    const uint64_t per = 1ull << 30;
    const uint64_t n_total = 1ull + j.burn_in + j.n_steps;
    for (uint64_t off = 0; off < j.n_walkers; off += per) {
        WalkJob c = j;
        c.first_walker = j.first_walker + off;
        c.n_walkers = j.n_walkers - off < per ? j.n_walkers - off : per;
        if (c.letters) c.letters += off * n_total;
        if (c.z_out) c.z_out += off * j.n_steps;
        const unsigned blocks = (unsigned)((c.n_walkers + 255) / 256);
        if (j.precision == KL_PREC_FP64)
            hipLaunchKernelGGL(walk_kernel<double>, dim3(blocks), dim3(256), 0, s, c);
        else
            hipLaunchKernelGGL(walk_kernel<float>, dim3(blocks), dim3(256), 0, s, c);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace kl
