/*
 * kl_oracle.h -- CPU reference ("oracle") for the indexed Kleinian-attractor
 * renderer of Rosa, "A new indexed approach to render the attractors of
 * Kleinian groups" (arXiv:1709.08018).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain, obviously
 * correct definition that the GPU path is checked against.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header, table or constant with the GPU library.
 *
 * Conventions (all FP64):
 *   letters  0=a 1=b 2=A 3=B; A = a^-1, B = b^-1 (Section 3: the group is
 *            free on a, b; the only crash pairs are aA, Aa, bB, Bb).
 *   word     w[0..d-1], w[0] is the LEFTMOST letter, applied LAST
 *            (Section 1: right-to-left reading, W = abA gives
 *            z1 = A(z0), z2 = b(z1), z3 = a(z2); the last orbit point is
 *            the word value).
 *   index    rank of a reduced word of length d in lexicographic order of
 *            (w[0], ..., w[d-1]) with the letter order above; equivalently
 *            the rank among the survivors of the paper's scan of all m^d
 *            digit strings in numeric order (Section 6, index search).
 *   seed     attracting fixed point of the word's last (rightmost) letter;
 *            the *_group functions also feed one generator's fixed point to
 *            every word (seed 0..3), or each of the four in turn (seed 4,
 *            renders only): the paper's index-search loop (Section 6).
 *   complex  interleaved (re, im) doubles.
 *   matrix   gens[((letter*2 + row)*2 + col)*2 + part], part 0=re 1=im.
 *   window   [x0,x1) x [y0,y1), width x height bins, row 0 at y0,
 *            bin index row*width + col; non-finite values are dropped.
 *
 *   group    gens: 32 doubles, the four matrices laid out as above;
 *            seeds: 16 doubles, each generator's attracting fixed point as
 *            a homogeneous pair (u, v) of complex numbers, the point u / v
 *            (v = 0: infinity).  Matrices have determinant 1.
 *
 *   fix      oracle_generators writes each seed as a point, infinity as
 *            (inf, 0): the recipe's a fixes infinity on a curve of traces,
 *            among them ta = tb = 2, where it is the translation z + 2i;
 *            oracle_word_value reads such a value back as infinity.
 *
 * Return codes: 0 ok, -1 bad argument, -2 singular parameters.
 */
#ifndef KL_ORACLE_H
#define KL_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

uint64_t oracle_num_words(int depth);
uint64_t oracle_num_tree_nodes(int m, int depth, int tiling);
int oracle_unrank(uint64_t index, int depth, uint8_t *word);
int oracle_enumerate(int depth, uint64_t first, uint64_t count, uint8_t *words);
int oracle_generators(double ta_re, double ta_im, double tb_re, double tb_im,
                      double *tab_out, double *gens_out, double *fix_out);
int oracle_word_value(const uint8_t *word, int depth, const double *gens,
                      const double *fix, int literal, double *z_out);
int oracle_eval(double ta_re, double ta_im, double tb_re, double tb_im,
                int depth, const uint64_t *idx, uint64_t n, int literal,
                double *z_out);
int oracle_render(double ta_re, double ta_im, double tb_re, double tb_im,
                  int depth, int min_depth,
                  double x0, double x1, double y0, double y1,
                  uint32_t width, uint32_t height,
                  uint64_t first, uint64_t count, int nthreads,
                  double edge_tol, uint32_t *image, uint64_t *dropped,
                  uint64_t *near_edge);

/* groups: by the trace recipe; from two explicit matrices a, b (16 doubles,
 * a then b, each row-major complex; scaled to determinant 1, A and B are
 * their inverses); by Maskit's parametrisation with parameter mu */
int oracle_group_recipe(double ta_re, double ta_im, double tb_re, double tb_im,
                        double *gens_out, double *seeds_out);
int oracle_group_explicit(const double *ab, double *gens_out, double *seeds_out);
int oracle_group_maskit(double mu_re, double mu_im, double *gens_out, double *seeds_out);
/* seed: -1 the word's own, 0..3 that generator's fixed point for every word */
int oracle_eval_group(const double *gens, const double *seeds, int seed, int depth,
                      const uint64_t *idx, uint64_t n, int literal, double *z_out);
/* seed: as oracle_eval_group, or 4 for each generator's fixed point in turn */
int oracle_render_group(const double *gens, const double *seeds, int seed,
                        int depth, int min_depth,
                        double x0, double x1, double y0, double y1,
                        uint32_t width, uint32_t height,
                        uint64_t first, uint64_t count, int nthreads,
                        double edge_tol, uint32_t *image, uint64_t *dropped,
                        uint64_t *near_edge);

/* Indexed Cayley tables (Section 5): table[s * (n_symbols + 1) + x] is the
 * state after reading symbol x (1..n_symbols) in state s (0..n_states-1);
 * state 0 is the start and, reached again, the crash state.  Words
 * x_1..x_d are read right to left and are regular when no step lands in
 * state 0; they are numbered in lexicographic order, x_1 most significant.
 * maps: n_symbols matrices of 8 doubles (a, b, c, d complex); each symbol's
 * seed is its map's attracting fixed point; seed -1 takes the last
 * symbol's, 0..n_symbols-1 that symbol's for every word, and (renders
 * only) n_symbols each symbol's in turn. */
uint64_t oracle_cayley_num_words(const uint8_t *table, int n_states, int n_symbols, int depth);
int oracle_cayley_unrank(const uint8_t *table, int n_states, int n_symbols, uint64_t index, int depth,
                         uint8_t *symbols);
int oracle_cayley_scan(const uint8_t *table, int n_states, int n_symbols, int depth, uint8_t *out,
                       uint64_t cap, uint64_t *n_out);
int oracle_cayley_eval(const uint8_t *table, int n_states, int n_symbols, const double *maps, int seed,
                       int depth, const uint64_t *idx, uint64_t n, int literal, double *z_out);
int oracle_cayley_render(const uint8_t *table, int n_states, int n_symbols, const double *maps, int seed,
                         int depth, int min_depth, double x0, double x1, double y0, double y1,
                         uint32_t width, uint32_t height, double edge_tol, uint32_t *image,
                         uint64_t *dropped, uint64_t *near_edge);

/* Probabilistic rendering (Section 4): random walks.  Walker w's letters
 * come from Philox4x64-10 under the key (seed, 0), block j at the counter
 * (j, w, 0, 0), eight 32-bit values a block (low, high half of each output);
 * c_0 = value >> 30, and c_k (k >= 1) is the floor(3 value / 2^32)-th letter
 * other than the inverse of c_{k-1}.  The walk starts at the attracting
 * fixed point of c_0 and applies G_{c_k} at step k; points z_{burn_in+1} ..
 * z_{burn_in+n_steps} are drawn (walker-major in z_out). */
int oracle_philox4x64_10(const uint64_t *ctr, const uint64_t *key, uint64_t *out);
int oracle_walk_letters(uint64_t seed, uint64_t walker, uint32_t n, uint8_t *letters);
int oracle_walk_points(const double *gens, const double *seeds, uint64_t seed, uint64_t first_walker,
                       uint64_t n_walkers, uint32_t burn_in, uint32_t n_steps, double *z_out);
int oracle_walk_render(const double *gens, const double *seeds, uint64_t seed, uint64_t first_walker,
                       uint64_t n_walkers, uint32_t burn_in, uint32_t n_steps,
                       double x0, double x1, double y0, double y1, uint32_t width, uint32_t height,
                       double edge_tol, uint32_t *image, uint64_t *dropped, uint64_t *near_edge);

#ifdef __cplusplus
}
#endif
#endif
