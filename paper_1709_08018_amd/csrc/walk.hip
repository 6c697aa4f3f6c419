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
// infinity outside).  The points of a walk jump across the limit set, so
// there are no runs to merge, and a global atomic per point (walk_kernel)
// costs a cache line per lane.  The binned path (walk_bin_kernel,
// walk_tile_hist_kernel) instead sorts each workgroup's points of 8 steps
// by image tile of 2^15 bins in LDS and writes them out as 16-bit offsets
// within their tiles; a second kernel counts each tile's offsets in an LDS
// histogram and adds its non-zero bins to the image.
#include <hip/hip_runtime.h>

#include "kl_internal.hpp"

namespace kl {

namespace {

constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull, kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull, kPhiloxW1 = 0xBB67AE8584CAA73Bull;

// The 128-bit product a m of 64-bit words, from the four 32 x 32-bit
// partial products (each a multiply-add into 64 bits that cannot overflow):
// both halves come from the same four multiply-adds.
template <uint64_t M>
__device__ __forceinline__ void mul128(uint64_t a, uint64_t& hi, uint64_t& lo) {
    constexpr uint32_t m0 = (uint32_t)M, m1 = (uint32_t)(M >> 32);
    const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
    const uint64_t p0 = (uint64_t)a0 * m0;
    const uint64_t p1 = (uint64_t)a0 * m1 + (p0 >> 32);
    const uint64_t p2 = (uint64_t)a1 * m0 + (uint32_t)p1;
    hi = (uint64_t)a1 * m1 + (p1 >> 32) + (p2 >> 32);
    lo = (p2 << 32) | (uint32_t)p0;
}

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
        uint64_t hi0, lo0, hi1, lo1;
        mul128<kPhiloxM0>(c0, hi0, lo0);
        mul128<kPhiloxM1>(c2, hi1, lo1);
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

// 1 / x as the renderer takes it: v_rcp_f32 in FP32 (within an ulp), and in
// FP64 v_rcp_f64 refined by two Newton steps r <- r + r (1 - x r), a
// full-precision reciprocal.  x = 0 (a point at infinity) gives infinity or
// NaN, and the point is dropped.
__device__ __forceinline__ float walk_recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double walk_recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma_(-x, r, 1.0);
    r = fma_(r, e, r);
    e = fma_(-x, r, 1.0);
    return fma_(r, e, r);
}

// The four maps and the seeds (u : v) in LDS, one entry per letter.
template <typename T>
struct WalkMaps {
    mat<T> G[4];
    cpx<T> SU[4], SV[4];
};

template <typename T>
__device__ __forceinline__ void load_walk_maps(const WalkJob& j, WalkMaps<T>& m) {
    if (threadIdx.x < 4) {
        const m64& g = j.gens.g[threadIdx.x];
        m.G[threadIdx.x] = {{(T)g.a.re, (T)g.a.im}, {(T)g.b.re, (T)g.b.im}, {(T)g.c.re, (T)g.c.im},
                            {(T)g.d.re, (T)g.d.im}};
        const bool inf = (j.gens.inf_mask >> threadIdx.x) & 1u;
        m.SU[threadIdx.x] = inf ? cpx<T>{T(1), T(0)} : cpx<T>{(T)j.gens.fix[threadIdx.x].re, (T)j.gens.fix[threadIdx.x].im};
        m.SV[threadIdx.x] = inf ? cpx<T>{T(0), T(0)} : cpx<T>{T(1), T(0)};
    }
}

// The walk of one walker: letters c_0 .. c_{n_total - 1} (letter(k, c)),
// and after each step k > burn_in its drawn point in the window's pixel
// coordinates (point(d, px, py), d = k - burn_in - 1).  All walkers of a
// launch take the same steps, so calls happen at the same k in every lane
// (`active` lanes without a walker step along on walker 0's stream and
// report nothing).
template <typename T, typename Letter, typename Point>
__device__ __forceinline__ void walk_walker(const WalkJob& j, const WalkMaps<T>& m, uint64_t walker, bool active,
                                            Letter letter, Point point) {
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
                    u = m.SU[c];
                    v = m.SV[c];
                } else {
                    const int t = (int)__umulhi(x, 3u);
                    c = t + (t >= (prev ^ 2));
                    const mat<T> g = m.G[c];
                    const cpx<T> nu = cfma(g.a, u, cmul(g.b, v));
                    const cpx<T> nv = cfma(g.c, u, cmul(g.d, v));
                    u = nu;
                    v = nv;
                }
                if (active) letter(k, c);
                if (k > j.burn_in) {
                    // z = u / v, then the window's affine map s z + o (x anisotropy on the real part)
                    const T n2 = fma_(v.re, v.re, v.im * v.im);
                    const T rc = walk_recip(n2);
                    const T zr = fma_(u.re, v.re, u.im * v.im) * rc;
                    const T zi = fma_(u.im, v.re, -(u.re * v.im)) * rc;
                    const T px = fma_(s, zr, ox) * an, py = fma_(s, zi, oy);
                    point(k - j.burn_in - 1, px, py, active);
                }
                prev = c;
                ++k;
            }
        }
        walk_rescale(u, v);
    }
}

// Letters, points or a render with one global atomic per point.
template <typename T>
__global__ __launch_bounds__(256) void walk_kernel(const WalkJob j) {
    __shared__ WalkMaps<T> m;
    load_walk_maps(j, m);
    __syncthreads();
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t drop = 0;
    if (tid < j.n_walkers) {
        const uint32_t n_total = 1 + j.burn_in + j.n_steps;
        walk_walker<T>(j, m, j.first_walker + tid, true,
                       [&](uint32_t k, int c) {
                           if (j.mode == kWalkLetters) j.letters[tid * n_total + k] = (uint8_t)c;
                       },
                       [&](uint32_t d, T px, T py, bool) {
                           const uint64_t p = tid * j.n_steps + d;
                           if (j.mode == kWalkEval) {
                               j.z_out[p] = {(double)px, (double)py};
                           } else if (j.mode == kWalkRender) {
                               const uint32_t b = walk_bin(px, py, j.W, j.H);
                               if (b != kWalkOutside) atomicAdd(j.image + b, 1u);
                               else ++drop;
                           }
                       });
    }
    if (j.mode == kWalkRender && j.dropped) {
        for (int off = 32; off > 0; off >>= 1) drop += __shfl_down(drop, off, 64);
        if ((threadIdx.x & 63) == 0 && drop) atomicAdd((unsigned long long*)j.dropped, (unsigned long long)drop);
    }
}

// ---- binned render
constexpr uint32_t kWalkTileBits = 15;                    // a tile: 2^15 bins
constexpr uint32_t kWalkTileBins = 1u << kWalkTileBits;
// Drawn steps per region.  Eight keep a workgroup's LDS near 14 KB, so that
// eight workgroups (32 waves) fit a CU and hide the sort's barriers and
// LDS atomics behind each other's arithmetic; sixteen steps (26 KB, six
// workgroups) took 15% longer on 2^30 points, thirty-two 72% longer, and
// four no shorter.
constexpr uint32_t kWalkChunk = 8;
constexpr uint32_t kWalkRegion = 256 * kWalkChunk;        // points of a region at most
constexpr uint32_t kNoKey = 0xFFFFFFFFu;

// One region per (workgroup, chunk of kWalkChunk drawn steps): its points
// in the window as offsets within their tiles, tile by tile (ids, kWalkRegion
// slots a region), and where each tile's offsets start (starts, T + 1
// entries a region: starts[T] is the region's count).
template <typename T>
__global__ __launch_bounds__(256) void walk_bin_kernel(const WalkJob j, uint16_t* __restrict__ ids,
                                                       uint32_t* __restrict__ starts, uint32_t T_tiles,
                                                       uint32_t n_chunks) {
    __shared__ WalkMaps<T> m;
    __shared__ uint32_t keys[kWalkRegion];
    __shared__ uint16_t sorted[kWalkRegion];
    __shared__ uint32_t cnt[kMaxWalkTiles + 1], cur[kMaxWalkTiles];
    load_walk_maps(j, m);
    for (uint32_t t = threadIdx.x; t <= kMaxWalkTiles; t += blockDim.x) cnt[t] = 0;
    __syncthreads();
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = tid < j.n_walkers;
    const uint32_t lane_slot = threadIdx.x * kWalkChunk;
    uint64_t drop = 0;
    walk_walker<T>(j, m, j.first_walker + (active ? tid : 0), active, [](uint32_t, int) {},
                   [&](uint32_t d, T px, T py, bool act) {
                       const uint32_t slot = d % kWalkChunk;
                       const uint32_t b = walk_bin(px, py, j.W, j.H);
                       uint32_t key = kNoKey;
                       if (act) {
                           if (b != kWalkOutside) key = b;
                           else ++drop;
                       }
                       keys[lane_slot + slot] = key;
                       if (key != kNoKey) atomicAdd(&cnt[key >> kWalkTileBits], 1u);
                       // the chunk is full, or the walk ends: sort it into its region
                       if (slot == kWalkChunk - 1 || d == j.n_steps - 1) {
                           const uint32_t nk = slot + 1;
                           __syncthreads();
                           if (threadIdx.x < 64) {
                               // exclusive scan of cnt[0 .. T) by one wave, into cnt, with cnt[T] the total
                               uint32_t carry = 0;
                               for (uint32_t base = 0; base < T_tiles; base += 64) {
                                   const uint32_t t = base + threadIdx.x;
                                   const uint32_t c = t < T_tiles ? cnt[t] : 0u;
                                   uint32_t x = c;
                                   for (int off = 1; off < 64; off <<= 1) {
                                       const uint32_t y = __shfl_up(x, off, 64);
                                       if ((int)threadIdx.x >= off) x += y;
                                   }
                                   if (t < T_tiles) {
                                       cnt[t] = carry + x - c;
                                       cur[t] = carry + x - c;
                                   }
                                   carry += __shfl(x, 63, 64);
                               }
                               if (threadIdx.x == 0) cnt[T_tiles] = carry;
                           }
                           __syncthreads();
                           for (uint32_t q = 0; q < nk; ++q) {
                               const uint32_t kq = keys[lane_slot + q];
                               if (kq != kNoKey)
                                   sorted[atomicAdd(&cur[kq >> kWalkTileBits], 1u)] = (uint16_t)(kq & (kWalkTileBins - 1));
                           }
                           __syncthreads();
                           const uint64_t region = (uint64_t)blockIdx.x * n_chunks + d / kWalkChunk;
                           const uint32_t n_in = cnt[T_tiles];
                           uint16_t* out = ids + region * kWalkRegion;
                           for (uint32_t i = threadIdx.x; i < n_in; i += blockDim.x) out[i] = sorted[i];
                           uint32_t* st = starts + region * (T_tiles + 1);
                           for (uint32_t t = threadIdx.x; t <= T_tiles; t += blockDim.x) st[t] = cnt[t];
                           __syncthreads();
                           for (uint32_t t = threadIdx.x; t <= T_tiles; t += blockDim.x) cnt[t] = 0;
                           __syncthreads();
                       }
                   });
    if (j.dropped) {
        for (int off = 32; off > 0; off >>= 1) drop += __shfl_down(drop, off, 64);
        if ((threadIdx.x & 63) == 0 && drop) atomicAdd((unsigned long long*)j.dropped, (unsigned long long)drop);
    }
}

// The tile histogram reads a region's offsets of one tile (its segment) in
// 16-byte chunks of 8 offsets, 8 lanes to a region, so that one load
// instruction of a wave covers the first 64 offsets of 8 regions; a wave
// loads the first chunks of kHistPasses such groups of 8 regions before
// counting them, and loads the segment bounds of its next 64 regions while
// it counts the current ones.
constexpr uint32_t kHistLanes = 8;    // lanes per region
constexpr uint32_t kHistPasses = 4;   // groups of 8 regions loaded before counting

// count the offsets of chunk c (offsets 8c .. 8c + 7 of the region) that
// lie in the segment [a, b)
__device__ __forceinline__ void hist_chunk(uint32_t* hist, uint4 v, uint32_t c, uint32_t a, uint32_t b) {
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (uint32_t e = 0; e < 8; ++e) {
        const uint32_t i = 8 * c + e;
        if (i >= a && i < b) atomicAdd(&hist[(w[e / 2] >> (16 * (e % 2))) & 0xFFFFu], 1u);
    }
}

// Tile blockIdx.x / split over its share of the regions: every offset
// counted in an LDS histogram, then each non-zero bin added to the image.
__global__ __launch_bounds__(1024) void walk_tile_hist_kernel(const uint16_t* __restrict__ ids,
                                                              const uint32_t* __restrict__ starts,
                                                              uint64_t n_regions, uint32_t T_tiles, uint32_t split,
                                                              uint32_t* __restrict__ image) {
    __shared__ uint32_t hist[kWalkTileBins];
    const uint32_t tile = blockIdx.x / split, part = blockIdx.x % split;
    for (uint32_t i = threadIdx.x; i < kWalkTileBins; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    const uint64_t r0 = n_regions * part / split, r1 = n_regions * (part + 1) / split;
    const uint32_t wave = threadIdx.x / 64, lane = threadIdx.x % 64, waves = blockDim.x / 64;
    const uint32_t grp = lane / kHistLanes, sub = lane % kHistLanes;
    // a wave takes a contiguous slice of the regions, 64 at a time; lane l
    // holds the segment bounds [a, b) of region base + l (0, 0 past the slice)
    const uint64_t per = (r1 - r0 + waves - 1) / waves;
    const uint64_t w0 = r0 + wave * per, w1 = w0 + per < r1 ? w0 + per : r1;
    uint32_t na = 0, nb_ = 0;
    if (w0 + lane < w1) {
        const uint32_t* st = starts + (w0 + lane) * (T_tiles + 1);
        na = st[tile];
        nb_ = st[tile + 1];
    }
    for (uint64_t base = w0; base < w1; base += 64) {
        const uint32_t a = na, b = nb_;
        na = 0;
        nb_ = 0;
        if (base + 64 + lane < w1) {
            const uint32_t* st = starts + (base + 64 + lane) * (T_tiles + 1);
            na = st[tile];
            nb_ = st[tile + 1];
        }
        const uint32_t n = w1 - base < 64 ? (uint32_t)(w1 - base) : 64u;
        for (uint32_t j = 0; j < n; j += kHistLanes * kHistPasses) {
            uint4 v[kHistPasses];
            uint32_t aq[kHistPasses], bq[kHistPasses], cq[kHistPasses];
            const uint16_t* seg[kHistPasses];
#pragma unroll
            for (uint32_t q = 0; q < kHistPasses; ++q) {
                const uint32_t r = j + kHistLanes * q + grp;   // < 64
                aq[q] = __shfl(a, (int)r, 64);
                bq[q] = __shfl(b, (int)r, 64);
                cq[q] = aq[q] / 8 + sub;
                seg[q] = ids + (base + r) * kWalkRegion;
                v[q] = 8 * cq[q] < bq[q] ? *(const uint4*)(seg[q] + 8 * cq[q]) : make_uint4(0, 0, 0, 0);
            }
#pragma unroll
            for (uint32_t q = 0; q < kHistPasses; ++q)
                if (8 * cq[q] < bq[q]) hist_chunk(hist, v[q], cq[q], aq[q], bq[q]);
            // segments longer than the group's first 8 chunks
#pragma unroll
            for (uint32_t q = 0; q < kHistPasses; ++q)
                for (uint32_t c = cq[q] + kHistLanes; 8 * c < bq[q]; c += kHistLanes)
                    hist_chunk(hist, *(const uint4*)(seg[q] + 8 * c), c, aq[q], bq[q]);
        }
    }
    __syncthreads();
    uint32_t* img = image + (uint64_t)tile * kWalkTileBins;
    for (uint32_t i = threadIdx.x; i < kWalkTileBins; i += blockDim.x) {
        const uint32_t v = hist[i];
        if (v) atomicAdd(img + i, v);
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

uint32_t walk_tiles(uint32_t W, uint32_t H) {
    const uint64_t bins = (uint64_t)W * H;
    return (uint32_t)((bins + kWalkTileBins - 1) / kWalkTileBins);
}

uint64_t walk_region_points(uint32_t n_steps) {
    return 256ull * kWalkChunk * ((n_steps + kWalkChunk - 1) / kWalkChunk);
}

// The binned render: walkers in launches whose regions hold at most
// kWalkBinnedPoints points, each launch binning its walkers' points
// (walk_bin_kernel) and then counting them tile by tile
// (walk_tile_hist_kernel), in temporaries allocated on the stream.
hipError_t launch_walk_binned(const WalkJob& j, hipStream_t s) {
    if (j.n_walkers == 0 || j.n_steps == 0) return hipSuccess;
    const uint32_t T_tiles = walk_tiles(j.W, j.H);
    const uint32_t n_chunks = (j.n_steps + kWalkChunk - 1) / kWalkChunk;
    const uint64_t block_points = walk_region_points(j.n_steps);   // one block of 256 walkers
    uint64_t blocks_per = kWalkBinnedPoints / block_points;
    if (blocks_per == 0) return hipErrorInvalidValue;
    const uint64_t total_blocks = (j.n_walkers + 255) / 256;
    if (blocks_per > total_blocks) blocks_per = total_blocks;
    uint16_t* ids = nullptr;
    uint32_t* starts = nullptr;
    const uint64_t regions_per = blocks_per * n_chunks;
    hipError_t e = hipMallocAsync((void**)&ids, regions_per * kWalkRegion * sizeof(uint16_t), s);
    if (e != hipSuccess) return e;
    e = hipMallocAsync((void**)&starts, regions_per * (T_tiles + 1) * sizeof(uint32_t), s);
    if (e != hipSuccess) {
        (void)hipFreeAsync(ids, s);
        return e;
    }
    int cus = device_cu_count();
    for (uint64_t b0 = 0; b0 < total_blocks && e == hipSuccess; b0 += blocks_per) {
        const uint64_t nb = total_blocks - b0 < blocks_per ? total_blocks - b0 : blocks_per;
        WalkJob c = j;
        c.first_walker = j.first_walker + b0 * 256;
        c.n_walkers = j.n_walkers - b0 * 256 < nb * 256 ? j.n_walkers - b0 * 256 : nb * 256;
        if (j.precision == KL_PREC_FP64)
            hipLaunchKernelGGL(walk_bin_kernel<double>, dim3((unsigned)nb), dim3(256), 0, s, c, ids, starts, T_tiles,
                               n_chunks);
        else
            hipLaunchKernelGGL(walk_bin_kernel<float>, dim3((unsigned)nb), dim3(256), 0, s, c, ids, starts, T_tiles,
                               n_chunks);
        if ((e = hipGetLastError()) != hipSuccess) break;
        const uint64_t n_regions = nb * n_chunks;
        // enough workgroups to fill the GPU twice over, each tile split evenly
        uint64_t split = (2ull * (uint64_t)cus + T_tiles - 1) / T_tiles;
        if (split > n_regions) split = n_regions;
        if (split < 1) split = 1;
        hipLaunchKernelGGL(walk_tile_hist_kernel, dim3((unsigned)(T_tiles * split)), dim3(1024), 0, s, ids, starts,
                           n_regions, T_tiles, (uint32_t)split, j.image);
        e = hipGetLastError();
    }
    const hipError_t f1 = hipFreeAsync(ids, s), f2 = hipFreeAsync(starts, s);
    return e != hipSuccess ? e : f1 != hipSuccess ? f1 : f2;
}

}  // namespace kl
