// kl_internal.hpp -- shared declarations of libkl (host planner, launchers,
// device arithmetic).  Every floating-point step of a word value is written
// with explicit fma / mul / add and the library is built with
// -ffp-contract=off, so the persistent renderer, the per-word kernel and
// kl_eval produce bit-identical values for the same word and split.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kl.h"

namespace kl {

constexpr int kMaxTail = 8;         // LDS suffix tables hold 4*3^(r-1) <= 8748 entries
constexpr int kMaxTailFp64 = 7;     // FP64: the homogeneous table of r = 8 exceeds a CU's LDS
constexpr int kMaxLane = 20;        // letters a lane appends to its prefix (3^20 < 2^32)
constexpr int kMaxPrefix = 14;      // prefix table depth (4*3^13 entries of 64 B at most)
constexpr int kWave = 64;
constexpr int kBlock = 256;         // threads per workgroup of the renderer
constexpr double kAffineLimit = 4294967296.0;  // |tail point| above this -> homogeneous form

// ---------------------------------------------------------------- complex
template <typename T>
struct cpx {
    T re, im;
};
using c32 = cpx<float>;
using c64 = cpx<double>;

template <typename T>
struct mat {  // [[a, b], [c, d]]
    cpx<T> a, b, c, d;
};
using m64 = mat<double>;
using m32 = mat<float>;

__host__ __device__ inline double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }
__host__ __device__ inline float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// x * y (complex), fixed operation order
template <typename T>
__host__ __device__ inline cpx<T> cmul(cpx<T> x, cpx<T> y) {
    return {fma_(x.re, y.re, -(x.im * y.im)), fma_(x.re, y.im, x.im * y.re)};
}
// x * y + z (complex), fixed operation order
template <typename T>
__host__ __device__ inline cpx<T> cfma(cpx<T> x, cpx<T> y, cpx<T> z) {
    return {fma_(x.re, y.re, fma_(-x.im, y.im, z.re)), fma_(x.re, y.im, fma_(x.im, y.re, z.im))};
}

template <typename T>
__host__ __device__ inline mat<T> mmul(const mat<T>& x, const mat<T>& y) {
    return {cfma(x.a, y.a, cmul(x.b, y.c)), cfma(x.a, y.b, cmul(x.b, y.d)),
            cfma(x.c, y.a, cmul(x.d, y.c)), cfma(x.c, y.b, cmul(x.d, y.d))};
}

// ---------------------------------------------------------------- launch args
struct Gens {
    m64 g[4];           // a, b, A, B  (FP64, determinant 1)
    c64 fix[4];         // attracting fixed points (FP64); 0 where at infinity
    uint32_t inf_mask;  // bit k: generator k's attracting fixed point is infinity
};

// Affine map folded into the head so the word value comes out in pixel
// coordinates: pixel = s * z + o (with aniso applied to the real part).
struct Fold {
    double s;        // bins per unit along y
    c64 o;           // -(x0, y0) * s
    double aniso;    // (bins per unit along x) / s; 1 for square bins
    int head_form;   // kl_opts.head_form
};

struct Split {
    int depth, r, m, k;        // depth = k + m + r (k = 0 only when m = 0 and r = depth)
    uint32_t pow3_m;           // 3^m
    uint32_t R1;               // 3^(r-1): suffixes per first suffix letter
    uint64_t R;                // 3^r: suffixes after a given letter
    uint64_t n_heads;          // 4*3^(k+m-1) (1 when k+m = 0)
};

struct Tables {                // device pointers of one parameter set
    const m64* prefix;         // N_k prefix products (k >= 1)
    const uint8_t* prefix_last;// last letter of each prefix
    const void* tail;          // N_r suffix points: affine (T) or homogeneous (2 T)
    const uint32_t* tail_flags;// n_flags words; the suffix table is used in its
    uint32_t n_flags;          // homogeneous form when any of them is nonzero
};

// Host-side planning and validation helpers (abi.cpp)
int set_error(int code, const char* fmt, ...);  // records kl_last_error(), returns code
// Where a split is used: a render of one depth (and kl_eval and kl_plan,
// which must agree with it word for word); a depth of a tiling render
// (min_depth < depth, whole or by index ranges); or one set of a batched
// render of many parameter sets.  Prefix tables of at most 9, 6 and 8
// letters respectively: a tiling builds one table for every depth and seed
// in one launch, and smaller tables pay there (the Maskit tiling to depth
// 14: 0.160 against 0.182 ms with 9 letters; the depth-16 tiling of the
// quasi-Fuchsian group: 0.153 against 0.167 ms).  A word's value depends
// on the tail only, not on how the head divides into prefix and lane
// letters.
enum PlanContext { kPlanSingle, kPlanTiling, kPlanBatch };
int plan_split(int depth, int precision, int r_req, int m_req, Split* out, PlanContext ctx = kPlanSingle);
uint64_t num_words(int depth);
uint64_t pow3_u64(int n);

// Launchers (kernels.hip).  All enqueue on `stream` and return a hipError_t.
hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s);
hipError_t launch_fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t s);
hipError_t launch_decode(uint64_t first, uint64_t count, int depth, uint8_t* out, hipStream_t s);

// Fused set-up of one render or evaluation: image / dropped clear, FP64
// prefix table, suffix table and its form flags (one word per 256 points).
struct SetupJob {
    Gens gens;
    int precision, k, r, force_homog;
    int seed;              // -1: each suffix from its last letter's fixed point; 0..3: that generator's
    m64* prefix;
    uint8_t* last;
    void* aff;
    void* hom;
    uint32_t* flags;
    uint32_t* image;       // null: not cleared
    uint64_t bins;
    uint64_t* dropped;     // null: not cleared
};
hipError_t launch_setup(const SetupJob& j, hipStream_t s);

struct RenderJob {
    Split sp;
    int precision;
    Gens gens;
    Fold fold;
    Tables tab;
    const void* tail_homog;
    uint32_t* image;
    uint32_t width, height;
    uint64_t* dropped;         // device u64 (may be null)
    // persistent kernel: heads [head_begin, head_begin + n_heads), n_units = ceil(n_heads / 64)
    uint64_t head_begin;
    uint64_t n_heads;
    uint32_t n_units;
    // per-word kernel: word indices (within this depth) of the ragged ends
    uint64_t rag_first[2], rag_count[2];
    int hist_mode;
    int grid_blocks;
    int bounded;               // FP32 persistent kernel with per-node bounds (kl_opts::block_bounds)
};
hipError_t launch_render(const RenderJob& job, hipStream_t s);

struct EvalJob {
    Split sp;
    int precision;
    Gens gens;
    Fold fold;
    Tables tab;
    const void* tail_homog;
    const uint64_t* idx;
    uint64_t n;
    c64* out;
};
hipError_t launch_eval(const EvalJob& job, hipStream_t s);

// Batched renderer: one descriptor per parameter set (device array).
struct SetDesc {
    Gens gens;
    Split sp;
    Tables tab;
    const void* tail_homog;
    uint32_t* image;
    uint64_t* dropped;         // device u64 of this set (may be null)
    uint32_t n_prefix;         // 4*3^(k-1)
    uint32_t n_tail;           // 4*3^(r-1)
    int seed;                  // as SetupJob::seed
};
struct BatchJob {
    const SetDesc* sets;           // device, n_sets entries
    const uint64_t* unit_offsets;  // device, n_sets + 1 prefix sums of block units (kBlock heads each)
    int n_sets;
    uint64_t total_units;
    int precision;
    Fold fold;
    uint32_t width, height;
    int grid_blocks;
    uint32_t table_bytes;          // LDS bytes of the largest suffix table (homogeneous form)
    uint32_t max_prefix, max_tail; // largest n_prefix / n_tail over the sets
    int force_homog;
    int count_dropped;             // the sets' dropped counters are set
    int bounded;                   // block bounds in the persistent batch kernel (kl_opts::block_bounds)
};
hipError_t launch_batch_tables(const BatchJob& job, hipStream_t s);
hipError_t launch_render_batch(const BatchJob& job, hipStream_t s);

// Every word of the sets too shallow for the persistent kernel, one per
// thread: word w of the launch is word w - word_offsets[q] of set set_ids[q].
struct PerWordBatchJob {
    const SetDesc* sets;           // device (the batch's descriptors)
    const uint64_t* word_offsets;  // device, n + 1 prefix sums of the sets' words
    const int* set_ids;            // device, n indices into sets
    int n;
    uint64_t total;
    int precision;
    Fold fold;
    uint32_t width, height;
};
hipError_t launch_perword_batch(const PerWordBatchJob& job, hipStream_t s);

// Words of an indexed Cayley table (Section 5), one per thread.  Every field
// is passed by value: the table, the maps and the seeds are small.
constexpr int kCayleyMaxStates = 16;
constexpr int kCayleyMaxSymbols = 8;
constexpr int kCayleyMaxSets = 64;      // good-state sets reachable from the set of all states
constexpr int kCayleyMaxTails = 1024;   // entries of the tail table
// The tail table's size in use: a render goes one head per thread, so
// shorter tails give more heads to spread over the GPU (the once-punctured
// torus table: 324 tails of 5 symbols, three times the heads of 972 tails of
// 6, at 0.31 against 0.42 ms for depth 16), while longer tails spread each
// head's ranking over more words.
constexpr int kCayleyHeadTails = 400;
constexpr int kCayleyMaxTail = 12;      // its longest tails
enum { kCayleyDecode = 0, kCayleyEval = 1, kCayleyRender = 2 };
struct CayleyJob {
    uint8_t table[kCayleyMaxStates * (kCayleyMaxSymbols + 1)];
    // good sets: set 0 holds every state; next_set[g * m + x - 1] is the set
    // after choosing symbol x with set g
    uint16_t sets[kCayleyMaxSets];
    uint8_t next_set[kCayleyMaxSets * kCayleyMaxSymbols];
    int n_sets;
    m64 maps[kCayleyMaxSymbols];        // determinant 1
    c64 fix[kCayleyMaxSymbols];         // attracting fixed points; 0 where at infinity
    uint32_t inf_mask;                  // bit x - 1: symbol x's fixed point is infinity
    int S, m, min_depth, max_depth;
    int seed;                           // -1: each word's last symbol's fixed point; else symbol seed + 1's
    int n_seeds;                        // render: the seeds drawn in turn (each as `seed`), n_seeds >= 1
    int8_t seed_list[kCayleyMaxSymbols];
    uint64_t first, count;              // decode / render: words [first, first + count) of the combined
    uint64_t depth_start[KL_MAX_DEPTH + 2];  // index space; depth_start[d - min_depth] = its first word
    Fold fold;
    uint32_t* image;
    uint32_t W, H;
    uint64_t* dropped;                  // render: device u64 or null
    uint8_t* symbols_out;               // decode: count * max_depth bytes
    const uint64_t* idx;                // eval: count indices of words of max_depth
    c64* z_out;                         // eval
    int grid_blocks;
    // head/tail evaluation of words of depth >= r (r = 0: none): a table of the
    // n_tails regular words of length r, their end states and their points
    int r, n_tails;
    int run;                            // render: consecutive words per thread
};
hipError_t launch_cayley(const CayleyJob& j, int mode, hipStream_t s);

// Random walks (Section 4, the probabilistic approach), one thread per
// walker: the letters of each walker, or its drawn points (values, or pixel
// coordinates with a window), or its points binned into an image.
enum { kWalkLetters = 0, kWalkEval = 1, kWalkRender = 2 };
struct WalkJob {
    Gens gens;
    Fold fold;                 // identity without a window
    int precision, mode;
    uint64_t seed, first_walker, n_walkers;
    uint32_t burn_in, n_steps;
    uint8_t* letters;          // letters: n_walkers * (1 + burn_in + n_steps), walker-major
    c64* z_out;                // eval: n_walkers * n_steps, walker-major
    uint32_t* image;           // render
    uint32_t W, H;
    uint64_t* dropped;         // render: device u64 or null
};
hipError_t launch_walk(const WalkJob& j, hipStream_t s);
// Binned walk render: points sorted by image tile of 2^15 bins, counted in
// LDS; images of at most kMaxWalkTiles tiles, at most kWalkBinnedPoints
// points staged per launch (walk_region_points(n_steps) per 256 walkers).
constexpr uint32_t kMaxWalkTiles = 256;
constexpr uint64_t kWalkBinnedPoints = 1ull << 27;
uint32_t walk_tiles(uint32_t W, uint32_t H);
uint64_t walk_region_points(uint32_t n_steps);
hipError_t launch_walk_binned(const WalkJob& j, hipStream_t s);

int device_cu_count();

}  // namespace kl
