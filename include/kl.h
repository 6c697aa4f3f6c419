/*
 * kl.h -- C ABI of libkl, an indexed renderer for the attractors (limit
 * sets) of once-punctured-torus Kleinian groups on AMD Instinct MI355X
 * (gfx950), after A. Rosa, "A new indexed approach to render the attractors
 * of Kleinian groups", arXiv:1709.08018.
 *
 * The paper's problem statement (abstract, Section 4 and Section 6): words
 * over the alphabet {a, b, A, B} are not stored in a dictionary but pulled
 * out of integer indices; every reduced word (no crash pair aA, Aa, bB, Bb:
 * Sections 1 and 3, Table 1) of the requested depth is visited, its
 * Moebius maps are applied right to left to a seed point (Section 1: for
 * W = abA, z1 = A(z0), z2 = b(z1), z3 = a(z2); the last orbit point is the
 * word value) and the value is drawn (Section 6, index search).
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 * letters   0 = a, 1 = b, 2 = A, 3 = B; A = a^-1, B = b^-1, so the inverse of
 *           letter c is c ^ 2.  Letter 0 of a word is its LEFTMOST letter,
 *           the one applied last.
 * index     the reduced words of depth d are numbered 0 .. 4*3^(d-1) - 1 in
 *           lexicographic order with the letter order above (first letter
 *           most significant).  This is the order in which the paper's scan
 *           of all 4^d digit strings (Section 6) meets the words that pass
 *           its Cayley-table check (Section 5), renumbered densely.
 * tiling    with min_depth < depth (kl_opts), every word of every depth
 *           min_depth .. depth is drawn ("tiling" render mode of Section 6);
 *           the index space is then all words of depth min_depth, followed
 *           by all of depth min_depth + 1, ..., followed by all of depth.
 *           Otherwise only words of length depth are drawn ("limit set").
 * group     ta = tr a, tb = tr b; the generators come from the trace recipe
 *           (Indra's Pearls' "Grandma's recipe", which the paper cites for
 *           its generators): tab = tr ab is the root (ta tb + s)/2 of
 *           tab^2 - ta tb tab + ta^2 + tb^2 = 0 with s in the closed upper
 *           half plane, so that tr abAB = -2.
 * seed      the attracting fixed point of the word's last letter.
 * window    [x0, x1) x [y0, y1) split into width x height bins; row 0 holds
 *           y in [y0, y0 + (y1 - y0)/height); bin index row * width + col.
 *           Values outside the window or not finite are dropped.  The
 *           bin is taken from the word's pixel coordinates (kl_eval_ex
 *           with the window): column floor(px) when 0 <= px < width,
 *           row likewise, compared as IEEE numbers (-0.0 counts as 0, a
 *           NaN is outside), as the oracle bins.
 * images    uint32 counts, row-major; additions wrap modulo 2^32.
 * memory    pointers named *_out, idx, letters_out, image_out and images_out
 *           are DEVICE pointers (memory of the current HIP device); all
 *           others are host pointers.  The caller owns every buffer; the
 *           library never frees caller memory.  The library allocates its
 *           own temporaries with hipMallocAsync on the call's stream; calls
 *           on the null stream keep their prefix and suffix tables in one
 *           buffer per device instead (1 MiB growing to at most 64 MiB,
 *           held until the process ends), which calls on other streams,
 *           or on another host thread while one holds it, do not touch.
 * streams   the plain entry points run on the null stream and return after
 *           the device has finished; the *_ex entry points enqueue on
 *           opts->stream (a hipStream_t, NULL = null stream) and return at
 *           once, except where a host output is requested.  Batched renders
 *           (kl_render_many_ex, and a tiling render of its whole index
 *           space) upload their set descriptors from host memory and return
 *           once that upload has finished, before the renders have.
 * errors    0 on success, a negative KL_E* code otherwise.  Every argument
 *           is validated before anything is enqueued, and on error no
 *           output is touched.  kl_strerror() names a code;
 *           kl_last_error() describes the last failure of the calling
 *           thread.
 */
#ifndef KL_H
#define KL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KL_OK 0
#define KL_EINVAL (-1)     /* null pointer, depth outside 1..40, bad window, bad option */
#define KL_ERANGE (-2)     /* index range beyond the words of the requested depth(s) */
#define KL_ESINGULAR (-3)  /* traces for which the recipe or a seed is undefined */
#define KL_EDEVICE (-4)    /* a HIP call failed */
#define KL_ENOMEM (-5)     /* device memory for temporaries could not be allocated */

#define KL_MAX_DEPTH 40

/* precision of the word values */
#define KL_PREC_FP32 0  /* FP64 generators, seeds and prefix products; FP32 suffix maps */
#define KL_PREC_FP64 1  /* every step in FP64 */

/* where each word's orbit starts (Section 6, index search: the paper feeds
 * every generator's fixed point to every word, each word's maps applied to
 * it in turn) */
#define KL_SEED_OWN 0     /* the attracting fixed point of the word's last letter */
#define KL_SEED_ALL 1     /* each of the four below in turn: four values per word (renders only) */
#define KL_SEED_A 2       /* the attracting fixed point of a, fed to every word; */
#define KL_SEED_B 3       /*   of b; */
#define KL_SEED_INV_A 4   /*   of A; */
#define KL_SEED_INV_B 5   /*   of B */

/* histogram strategy of the renderer */
#define KL_HIST_AUTO 0    /* planner's choice */
#define KL_HIST_RUNS 1    /* per-lane run-length counts, flushed with global atomics */
#define KL_HIST_LDS 2     /* per-lane runs flushed into an LDS tile, merged per work unit */

typedef struct { double re, im; } kl_c64;

typedef struct {
    double x0, x1, y0, y1;
    uint32_t width, height;
} kl_window;

/* Options of the *_ex entry points.  A zero-initialised struct gives the
 * defaults of the plain entry points (limit set, FP32 suffix path, whole
 * index space, image cleared first, null stream, planner's split). */
typedef struct {
    int min_depth;        /* 0 or depth: limit set; 1 .. depth-1: tiling */
    int precision;        /* KL_PREC_FP32 or KL_PREC_FP64 */
    int use_range;        /* 0: every index; 1: only [first_idx, first_idx + count) */
    uint64_t first_idx;
    uint64_t count;
    int accumulate;       /* 0: image cleared before drawing; 1: counts added */
    void *stream;         /* hipStream_t; NULL = null stream */
    uint64_t *dropped_out;/* device pointer to one uint64 or NULL: receives
                             (or, with accumulate, is increased by) the number
                             of words dropped as outside or not finite */
    int tail_len;         /* r: letters per suffix table, 0 = planner (1..8 in
                             FP32, 1..7 in FP64, whose r = 8 table would not
                             fit a CU's LDS: KL_EINVAL).  The planner takes 6
                             letters, fewer below depth 7, and for a render
                             of one depth of 13..16 letters (and kl_eval and
                             kl_plan of such a depth) 4 letters at depths
                             13-14 and 5 at 15-16; a word's value depends on
                             r, so renders compared bit for bit across these
                             contexts pass the same r */
    int lane_len;         /* m: letters each lane adds to its prefix, 0 = planner (1..20) */
    int hist_mode;        /* KL_HIST_* */
    int waves_per_cu;     /* persistent grid size, 0 = planner */
    int suffix_form;      /* 0: affine suffix points unless one needs the
                             homogeneous form; 1: homogeneous form always */
    int seed_mode;        /* KL_SEED_*; with KL_SEED_ALL the image and the
                             dropped count hold four points per word */
    int head_form;        /* how each head's map is applied to its suffix
                             points: 0: as P + Q / (y + S) (c != 0, det 1)
                             wherever that form fits the working precision,
                             else as the ratio (A y + B) / (C y + D);
                             1: the ratio for every head; 2: the ratio for
                             heads of odd index (waves then mix both forms).
                             1 and 2 exist to test the ratio path. */
    void *kernel_events[2];/* instrumentation: two hipEvent_t created by the
                             caller, or NULL; recorded on the stream right
                             before and right after the persistent renderer's
                             launches (of the deepest depth rendered) */
    int block_bounds;     /* 0: the renderer evaluates every word.  1: the
                             persistent renderer first bounds, for each head
                             and each group of 27 suffixes sharing their
                             leading letters, the bins those words can reach
                             (the head is a linear fractional map, Section
                             3, so it sends the group's bounding disk to a
                             disk; a margin covers the FP32 arithmetic).  A
                             group whose bound lies outside the window is
                             counted as dropped, one inside a single bin is
                             added to it, and only the others are evaluated
                             word by word.  Images and dropped counts are
                             bit for bit those of 0.  Applies where a
                             persistent renderer runs: renders of one depth
                             whose whole heads number at least 128 x 64,
                             and the sets of kl_render_many and the depths
                             and seeds of a tiling render that reach that
                             size; FP32 or FP64, with tail_len >= 4 and
                             KL_HIST_RUNS or AUTO; ignored elsewhere. */
} kl_opts;

/* The split the renderer uses for one depth (see kl_plan). */
typedef struct {
    int depth;
    int tail_len;      /* r: suffix letters enumerated from the LDS suffix table */
    int lane_len;      /* m: letters a lane appends to its table prefix in FP64 */
    int prefix_len;    /* k = depth - r - m: letters of the FP64 prefix table */
    int hist_mode;
    int waves_per_cu;
} kl_plan_t;

/* Number of reduced words of length depth, 4 * 3^(depth-1); 0 when depth
 * is outside 1..40. */
uint64_t kl_num_words(int depth);

/* kl_decode: the words with indices first_idx .. first_idx + count - 1 of
 * depth `depth` (Section 4, digital and indexed trees; Section 6, the
 * index-to-word routine), without any stored word list.
 *   letters_out  device buffer of count * depth bytes, word-major: letter j
 *                of word first_idx + i is letters_out[i * depth + j].
 * Errors: KL_EINVAL (depth, null pointer with count > 0), KL_ERANGE
 * (first_idx + count exceeds the number of words, including overflow; the
 * paper's routine silently wraps such indices, this one refuses them). */
int kl_decode(uint64_t first_idx, uint64_t count, int depth, uint8_t *letters_out);
int kl_decode_ex(uint64_t first_idx, uint64_t count, int depth, uint8_t *letters_out,
                 void *stream);

/* kl_render: limit-set image of the group with traces (ta, tb) at depth
 * `depth` (Section 6, index search, limit-set mode): every reduced word of
 * that length is decoded from its index, evaluated right to left from its
 * seed and counted in its bin of image_out (device, width * height uint32,
 * cleared first).  FP32 suffix path (see KL_PREC_FP32).
 * Errors: KL_EINVAL, KL_ESINGULAR, KL_EDEVICE, KL_ENOMEM. */
int kl_render(kl_c64 ta, kl_c64 tb, int depth, const kl_window *window, uint32_t *image_out);

/* kl_render_ex: as kl_render with options: tiling mode (min_depth), FP64
 * path, an index sub-range (streaming: rendering [0, x) then [x, N) with
 * accumulate gives exactly the image of [0, N)), accumulation, a stream,
 * the dropped-word count, and explicit split/histogram choices. */
int kl_render_ex(kl_c64 ta, kl_c64 tb, int depth, const kl_window *window,
                 uint32_t *image_out, const kl_opts *opts);

/* Bytes of the library's per-device scratch array (kl_render_noalloc). */
#define KL_NOALLOC_SCRATCH_BYTES (4u << 20)

/* kl_render_noalloc: for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, options and result as kl_render_ex for a
 * render of one depth: image_out (and opts->dropped_out) as there, bit for
 * bit the same image.  It allocates nothing: the prefix and suffix tables
 * that kl_render_ex puts in a library buffer or temporary go to a
 * library-owned device array of KL_NOALLOC_SCRATCH_BYTES, one per device,
 * held until the process ends, whose address is taken once per device on
 * its first call.  Every call on a device shares that device's array and
 * rewrites the tables it uses before reading them, so nothing carries over
 * between calls; calls that overlap on one device (two streams, or two host
 * threads) race on it and must be serialised by the caller, while calls on
 * one stream are ordered by it.  It enqueues only kernels on opts->stream,
 * so a HIP graph can capture it once a first call outside capture has taken
 * the array's address on the device.
 * Errors: as kl_render_ex; KL_EINVAL for a tiling render (min_depth other
 * than 0 or depth); KL_ENOMEM when the split's tables exceed the array
 * (prefix tables of 10 or more letters: depths above 35 under the planner's
 * splits), before anything is enqueued. */
int kl_render_noalloc(kl_c64 ta, kl_c64 tb, int depth, const kl_window *window,
                      uint32_t *image_out, const kl_opts *opts);

/* kl_render_many: n independent limit-set renders in one persistent launch
 * (parameter sets of uneven depth share one work queue).
 *   ta, tb, depth  host arrays of n entries
 *   images_out     device, n * width * height uint32; image i starts at
 *                  images_out + i * width * height; each is cleared first.
 * Image i equals kl_render(ta[i], tb[i], depth[i], window, ...) bit for bit.
 * Errors: as kl_render; the message of kl_last_error() names the first bad
 * set. */
int kl_render_many(int n, const kl_c64 *ta, const kl_c64 *tb, const int *depth,
                   const kl_window *window, uint32_t *images_out);
/* opts: precision, accumulate, stream, hist_mode, waves_per_cu, tail_len
 * and lane_len apply to every set (0 = planner per set);
 * min_depth and use_range must be 0.  dropped_out, if set, points to n
 * device uint64 counters, one per set. */
int kl_render_many_ex(int n, const kl_c64 *ta, const kl_c64 *tb, const int *depth,
                      const kl_window *window, uint32_t *images_out, const kl_opts *opts);

/* kl_eval: values of the words with the given indices, computed with
 * exactly the arithmetic the renderer uses for the same depth, precision
 * and split (Section 1, word value).
 *   idx     device, n uint64 word indices of depth `depth`
 *   z_out   device, n complex values (re, im as doubles)
 * kl_eval_ex additionally takes a window: with one, z_out receives the
 * continuous pixel coordinates (col + fraction, row + fraction) the
 * renderer floors into a bin, bit for bit; and options (precision, split,
 * stream, suffix form, head form, seed mode -- one seed per word, so
 * KL_SEED_ALL is KL_EINVAL; the other fields are ignored).
 * An index beyond the words of that depth yields NaN (the indices live in
 * device memory and are checked there).
 * Errors: KL_EINVAL, KL_ESINGULAR, KL_EDEVICE. */
int kl_eval(kl_c64 ta, kl_c64 tb, int depth, const uint64_t *idx, uint64_t n,
            int precision, kl_c64 *z_out);
int kl_eval_ex(kl_c64 ta, kl_c64 tb, int depth, const uint64_t *idx, uint64_t n,
               const kl_window *window, kl_c64 *z_out, const kl_opts *opts);

/* kl_generators: host-side trace recipe and seeds, FP64.
 *   tab_out     tr ab
 *   gens_out    16 entries: generator g (0=a 1=b 2=A 3=B) entry (row, col)
 *               at gens_out[g * 4 + row * 2 + col]
 *   fix_out     4 entries: attracting fixed point of each generator; a
 *               seed at infinity is written as (HUGE_VAL, 0).  On a curve of
 *               traces, among them ta = tb = 2 (the double cusp, whose
 *               limit set is the Apollonian gasket), a has c = 0: it is a
 *               translation, and a and A take infinity as their seed.
 *               Words whose value is infinity are dropped like any
 *               non-finite value.
 * Any output pointer may be NULL.  Errors: KL_ESINGULAR. */
int kl_generators(kl_c64 ta, kl_c64 tb, kl_c64 *tab_out, kl_c64 *gens_out, kl_c64 *fix_out);

/* Groups given by two generators instead of traces (Section 3: the maps
 * are linear fractional, z -> (a z + b)/(c z + d)).
 *   ab   host, 8 entries: a = [[ab[0], ab[1]], [ab[2], ab[3]]], then b
 *        likewise in ab[4..7].  Each is scaled to determinant 1, which
 *        leaves its map unchanged; A and B are the inverses.
 * A generator's seed is its attracting fixed point on the Riemann sphere,
 * which may be infinity (a map with c = 0, as for a translation).  Words
 * whose value is infinity are dropped like any non-finite value.
 *
 * kl_group_seeds: the four normalised maps (gens_out, 16 entries, laid out
 * as in kl_generators) and their seeds as homogeneous pairs (seeds_out, 8
 * entries: seed k = seeds_out[2k] / seeds_out[2k+1], infinity when the
 * second is 0).  Host pointers, either may be NULL.
 * Errors: KL_EINVAL (NULL ab, non-finite entries), KL_ESINGULAR (a zero
 * determinant, a map without an attracting fixed point: the identity). */
int kl_group_seeds(const kl_c64 *ab, kl_c64 *gens_out, kl_c64 *seeds_out);

/* kl_maskit_generators: Maskit's parametrisation of the once-punctured
 * torus groups, the embedding of the paper's figures (Fig. 1, Fig. 6 use
 * mu = -0.097 + 1.838i): a = [[-i mu, -i], [-i, 0]], b = [[1, 2], [0, 1]]
 * into ab_out (host, 8 entries, as kl_group_seeds takes them).
 * Errors: KL_EINVAL (NULL ab_out, non-finite mu). */
int kl_maskit_generators(kl_c64 mu, kl_c64 *ab_out);

/* kl_render_group_ex / kl_eval_group_ex: kl_render_ex / kl_eval_ex for a
 * group given by its two generators; every option applies the same way.
 * Errors: as kl_render_ex / kl_eval_ex, and as kl_group_seeds. */
int kl_render_group_ex(const kl_c64 *ab, int depth, const kl_window *window, uint32_t *image_out,
                       const kl_opts *opts);
int kl_eval_group_ex(const kl_c64 *ab, int depth, const uint64_t *idx, uint64_t n,
                     const kl_window *window, kl_c64 *z_out, const kl_opts *opts);

/* Random walks: the probabilistic approach of Section 4 (the rendering of
 * Fig. 3), the paper's alternative to its indexed method.  One word grows by
 * random picks of generators and the orbit of a point under it is drawn.
 * Walker w (first_walker <= w < first_walker + n_walkers) takes letters c_0,
 * c_1, ... (codes as everywhere: 0=a 1=b 2=A 3=B):
 *   c_0       uniform over the four letters: the top two bits of value 0;
 *   c_k       (k >= 1) uniform over the three letters other than the
 *             inverse of c_{k-1} (the word stays reduced): the
 *             floor(3 x / 2^32)-th of them in code order, x = value k;
 * where value k is the 32-bit half k % 2 (low half first) of 64-bit output
 * (k % 8) / 2 of Philox4x64-10 (Salmon et al., SC'11) at the counter
 * (k / 8, w, 0, 0) under the key (seed, 0).  The walker starts at the
 * attracting fixed point of c_0 and applies G_{c_k} at step k, so its point
 * after step k is the value of the reduced word c_k ... c_1 c_0 (Section 1).
 * It draws its points after steps burn_in + 1 .. burn_in + n_steps.  The
 * commutator "boost" of Fig. 3's caption is not applied.
 * A group is given by its generators a, b as for kl_render_group_ex. */
typedef struct {
    uint64_t seed;          /* Philox key (seed, 0) */
    uint64_t first_walker;  /* walkers first_walker .. first_walker + n_walkers - 1 */
    uint64_t n_walkers;
    uint32_t burn_in;       /* steps taken before the first drawn point */
    uint32_t n_steps;       /* points drawn per walker */
} kl_walk;

/* kl_walk_letters: letters c_0 .. c_{burn_in + n_steps} of each walker into
 * letters_out (device, n_walkers * (1 + burn_in + n_steps) bytes,
 * walker-major), asynchronously on `stream` (a hipStream_t).
 * Errors: KL_EINVAL (NULL walk or letters_out, 1 + burn_in + n_steps above
 * 2^32 - 1), KL_ERANGE (walker indices past 2^64), KL_EDEVICE. */
int kl_walk_letters(const kl_walk *walk, uint8_t *letters_out, void *stream);

/* kl_walk_eval_ex: the drawn points (z_out: device, n_walkers * n_steps,
 * walker-major), or with a window their pixel coordinates, computed as
 * kl_walk_render_ex computes them.  opts: precision, stream.
 * Errors: as kl_walk_letters, KL_EINVAL (bad window or option), and as
 * kl_group_seeds. */
int kl_walk_eval_ex(const kl_c64 *ab, const kl_walk *walk, const kl_window *window, kl_c64 *z_out,
                    const kl_opts *opts);

/* kl_walk_render_ex: the drawn points binned into image_out (device,
 * width * height uint32, cleared first unless accumulate) as every render
 * bins; dropped_out (if set) receives the points outside the window or not
 * finite.  image + dropped = n_walkers * n_steps.  opts: precision,
 * accumulate, stream, dropped_out, hist_mode:
 *   KL_HIST_RUNS  one global atomic add per point in the window;
 *   KL_HIST_LDS   each workgroup's points of 8 steps sorted by image tile
 *                 (2^15 bins) in LDS and staged in device temporaries
 *                 (2 bytes a point, allocated on the stream), then counted
 *                 tile by tile in LDS; images of at most 256 tiles
 *                 (8,388,608 bins), at most 524,288 drawn points a walker;
 *   KL_HIST_AUTO  KL_HIST_LDS from 2^18 points up where it applies, else
 *                 KL_HIST_RUNS.
 * Both give the same image and dropped count.
 * Errors: as kl_walk_eval_ex; KL_EINVAL for KL_HIST_LDS beyond its limits. */
int kl_walk_render_ex(const kl_c64 *ab, const kl_walk *walk, const kl_window *window, uint32_t *image_out,
                      const kl_opts *opts);

/* Indexed Cayley tables (Section 5, Tables 2 and 3): words over any finite
 * presentation the table encodes, drawn with one Moebius map per symbol.
 *   n_states   2..16; state 0 is where a walk starts and, reached again,
 *              the crash state
 *   n_symbols  1..8; symbols are 1..n_symbols (0 is the identity column)
 *   table      host, n_states * (n_symbols + 1) bytes: table[s * (n_symbols
 *              + 1) + x] is the state after reading symbol x in state s
 *   maps       host, 4 * n_symbols entries: symbol x's map [[m0, m1], [m2,
 *              m3]] at maps[4 (x - 1)]; scaled to determinant 1; NULL is
 *              allowed for kl_cayley_num_words and kl_cayley_decode_ex
 * A word x_1..x_d is read right to left from state 0 (Section 5's table
 * walk) and is regular when no step lands in state 0; the regular words of
 * each length are numbered in lexicographic order, x_1 most significant --
 * the order in which the paper's scan of all digit strings (Section 6)
 * meets them.  With the once-punctured torus table (Table 2) and letter x
 * = symbol x + 1, these are exactly the words and indices of kl_decode.
 * A word's value applies its maps right to left to its seed: the
 * attracting fixed point of its last symbol (KL_SEED_OWN), of symbol q + 1
 * for every word (KL_SEED_A + q, q < n_symbols), or each symbol's in turn
 * (KL_SEED_ALL, renders).  This path computes in FP64 throughout.
 * A table is refused (KL_EINVAL) when ranking its words needs more than 64
 * good-state sets: the sets of states a word's prefix can be read from,
 * which the kernels keep in LDS. */
typedef struct {
    int n_states;
    int n_symbols;
    const uint8_t *table;
    const kl_c64 *maps;
} kl_cayley;

/* Number of regular words of length depth; 0 for an invalid table or depth,
 * or when a count of words by length and end state reaches 2^63, or the
 * total 2^64. */
uint64_t kl_cayley_num_words(const kl_cayley *t, int depth);

/* symbols_out: device, count * depth bytes, word-major (symbol j of word
 * first_idx + i at symbols_out[i * depth + j]).  Asynchronous on stream.
 * Errors: KL_EINVAL (table, depth, NULL output with count > 0), KL_ERANGE. */
int kl_cayley_decode_ex(const kl_cayley *t, uint64_t first_idx, uint64_t count, int depth,
                        uint8_t *symbols_out, void *stream);

/* As kl_eval_ex: word values, or with a window continuous pixel
 * coordinates, bit for bit those kl_cayley_render_ex bins.  opts: stream
 * and seed_mode (not KL_SEED_ALL).  An index beyond the words gives NaN.
 * Errors: KL_EINVAL, KL_ESINGULAR (a map of determinant 0 or without an
 * attracting fixed point). */
int kl_cayley_eval_ex(const kl_cayley *t, int depth, const uint64_t *idx, uint64_t n,
                      const kl_window *window, kl_c64 *z_out, const kl_opts *opts);

/* As kl_render_ex for the table's words: limit set or tiling (min_depth),
 * an index range of the combined index space, accumulate, stream,
 * dropped_out and seed_mode apply; the other options are ignored. */
int kl_cayley_render_ex(const kl_cayley *t, int depth, const kl_window *window, uint32_t *image_out,
                        const kl_opts *opts);

/* kl_plan: the split and histogram strategy the renderer would use for a
 * render of this one depth and precision on the current device, after the
 * options' overrides (kl_eval takes the same split).  A tiling render
 * (min_depth < depth) that leaves the split to the planner takes its
 * deepest depth's tail_len from this plan at every depth longer than it
 * when that tail is not 6 letters and no tuned plan covers the deepest
 * depth; otherwise each depth takes 6 letters (fewer below depth 7) or its
 * tuned plan.  Errors: KL_EINVAL. */
int kl_plan(int depth, int precision, const kl_window *window, const kl_opts *opts,
            kl_plan_t *plan_out);

/* kl_autotune: times the candidate splits, histogram strategies and grid
 * sizes for (ta, tb, depth, window, precision) on the current device,
 * keeps the fastest as the plan for every later render and evaluation
 * of one depth with the same (device architecture, depth, precision) in
 * this process that leaves tail_len and lane_len to the planner, and
 * appends it to the file named by the environment variable
 * KL_AUTOTUNE_CACHE, if set (that file is read at the first plan lookup of
 * the process; lines "arch context depth precision width height tail_len
 * lane_len waves_per_cu hist_mode ms", context 0 for these plans with width
 * and height 0, arch "*" for any device; a line the planner rejects is
 * skipped).  scratch_image: device, width * height uint32, overwritten.
 * best_out may be NULL; best_ms_out (host, may be NULL) receives the
 * winner's median time.
 * Errors: as kl_render_ex. */
int kl_autotune(kl_c64 ta, kl_c64 tb, int depth, const kl_window *window, int precision,
                uint32_t *scratch_image, kl_plan_t *best_out, double *best_ms_out);

/* kl_autotune_many: tunes the plans of a batched render as a whole, timing
 * whole kl_render_many_ex launches of the given sets (n, ta, tb, depth,
 * window, precision; scratch_images: device, n * width * height uint32,
 * overwritten).  From the planner's plans it tries, for each depth of the
 * batch, deepest first, the splits with tails of 4..7 letters and prefix
 * tables of 1..9 letters, the other depths fixed, then persistent grids of
 * 16 and 24 waves per CU; a change is kept only when the batch gets at least
 * 1% faster, and the result only when, timed alternately with the planner's
 * plans three times more, it is still 1% faster (else the planner's plans
 * are kept).  The kept plans apply to every later kl_render_many_ex on a
 * device of the same architecture with the same image size and precision
 * that leaves tail_len and lane_len to the planner (kl_render_ex and kl_eval
 * keep their own plans), and are appended to KL_AUTOTUNE_CACHE as context 1
 * lines keyed by (arch, depth, width, height, precision).
 * plans_out (host, n entries, may be NULL): each set's plan;
 * best_ms_out / default_ms_out (host, may be NULL): the median batch time
 * with the kept plans / with the planner's.
 * Errors: as kl_render_many_ex. */
int kl_autotune_many(int n, const kl_c64 *ta, const kl_c64 *tb, const int *depth, const kl_window *window,
                     int precision, uint32_t *scratch_images, kl_plan_t *plans_out, double *best_ms_out,
                     double *default_ms_out);

/* kl_plan_many: the plan a set of this depth takes in kl_render_many_ex on
 * the current device with this window and precision (tuned by
 * kl_autotune_many, else the planner's).  Errors: KL_EINVAL. */
int kl_plan_many(int depth, int precision, const kl_window *window, kl_plan_t *plan_out);

const char *kl_strerror(int code);
const char *kl_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* KL_H */
