/*
 * kl_oracle.c -- CPU reference ("oracle") for the indexed Kleinian-attractor
 * renderer (Rosa, arXiv:1709.08018).  TEST INFRASTRUCTURE ONLY: the test
 * suite, the smoke check and the benchmark's CPU-baseline leg are its only
 * users.  Plain C99, FP64 complex arithmetic, no blocking or reordering
 * beyond what the definitions below state.  See kl_oracle.h for the
 * conventions (letters, word order, index order, window).
 *
 * What is computed, and where it comes from:
 *   - reduced words: strings over {a,b,A,B} with no adjacent inverse pair
 *     (Section 1, crash words; Section 3, pruned tree and Table 1);
 *   - their order: a depth-first walk of the pruned tree visiting children
 *     in letter order; this equals the order of the survivors in the
 *     paper's numeric scan of all 4^d digit strings (Section 4, digital and
 *     indexed trees; Section 6, index search);
 *   - word value: the word's maps applied right to left to the seed
 *     (Section 1); the DFS evaluator carries the product of the maps from
 *     the left, one 2x2 product per tree node, the literal evaluator walks
 *     the point itself;
 *   - render modes: "limit set" draws words of depth D only, "tiling"
 *     draws every word of depth 1..D (Section 6);
 *   - generators: the trace recipe (Indra's Pearls' "Grandma's recipe",
 *     the paper's reference for generator construction), with the root of
 *     the trace quadratic taken in the closed upper half plane; or two
 *     explicit matrices; or Maskit's parametrisation of the once-punctured
 *     torus groups (the embedding of the paper's figures);
 *   - seed: attracting fixed point of the word's last letter; or, as in the
 *     paper's index-search loop (Section 6), one generator's attracting
 *     fixed point fed to every word, all of the word's maps applied, for
 *     each generator in turn.  Seeds are points of the Riemann sphere,
 *     kept as homogeneous pairs (u : v) so that infinity is one of them.
 */
#include "kl_oracle.h"

#include <complex.h>
#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;
typedef struct { cplx a, b, c, d; } mat2; /* [[a, b], [c, d]] */

/* a <-> A, b <-> B */
static const int INVERSE[4] = {2, 3, 0, 1};

#define MAX_DEPTH 40

/* ------------------------------------------------------------------ */
/* counting                                                            */
/* ------------------------------------------------------------------ */

static uint64_t pow3(int n)
{
    uint64_t p = 1;
    for (int i = 0; i < n; i++) p *= 3;
    return p;
}

/* Reduced words of length d: 4 choices for the first letter, then 3 for
 * each later letter (anything but the inverse of the previous one). */
uint64_t oracle_num_words(int depth)
{
    if (depth < 1 || depth > MAX_DEPTH) return 0;
    return 4 * pow3(depth - 1);
}

/* Node counts of the unpruned m-branched tree (Section 6): m^D nodes at
 * depth D ("limit set"), or the sum over depths 1..D ("tiling"). */
uint64_t oracle_num_tree_nodes(int m, int depth, int tiling)
{
    uint64_t total = 0, level = 1;
    for (int d = 1; d <= depth; d++) {
        level *= (uint64_t)m;
        if (tiling || d == depth) total += level;
    }
    return total;
}

/* ------------------------------------------------------------------ */
/* words                                                               */
/* ------------------------------------------------------------------ */

/* Random access by subtree sizes: below the root every node has 3
 * children, so a child at depth j heads 3^(d-j) leaves.  At each level
 * take the (rank / subtree)-th allowed child in letter order. */
int oracle_unrank(uint64_t index, int depth, uint8_t *word)
{
    if (depth < 1 || depth > MAX_DEPTH || !word) return -1;
    if (index >= oracle_num_words(depth)) return -1;
    uint64_t rank = index;
    int prev = -1;
    for (int j = 1; j <= depth; j++) {
        uint64_t subtree = pow3(depth - j);
        uint64_t pick = rank / subtree;
        rank = rank % subtree;
        int seen = 0, chosen = -1;
        for (int c = 0; c < 4; c++) {
            if (prev >= 0 && c == INVERSE[prev]) continue;
            if ((uint64_t)seen == pick) { chosen = c; break; }
            seen++;
        }
        if (chosen < 0) return -1;
        word[j - 1] = (uint8_t)chosen;
        prev = chosen;
    }
    return 0;
}

typedef struct {
    int depth;
    uint64_t first, last; /* leaf index range [first, last) */
    uint64_t next;        /* index of the next leaf the walk reaches */
    uint8_t *out;
    uint8_t word[MAX_DEPTH];
} enum_ctx;

static void enumerate_rec(enum_ctx *e, int j)
{
    if (j == e->depth) {
        if (e->next >= e->first && e->next < e->last)
            memcpy(e->out + (e->next - e->first) * (uint64_t)e->depth,
                   e->word, (size_t)e->depth);
        e->next++;
        return;
    }
    for (int c = 0; c < 4; c++) {
        if (j > 0 && c == INVERSE[e->word[j - 1]]) continue;
        e->word[j] = (uint8_t)c;
        enumerate_rec(e, j + 1);
    }
}

/* Depth-first walk of the pruned tree with the explicit word on a stack;
 * writes the words whose visiting rank lies in [first, first+count). */
int oracle_enumerate(int depth, uint64_t first, uint64_t count, uint8_t *words)
{
    if (depth < 1 || depth > 20 || (!words && count)) return -1;
    uint64_t n = oracle_num_words(depth);
    if (first > n || count > n - first) return -1;
    enum_ctx e;
    memset(&e, 0, sizeof e);
    e.depth = depth;
    e.first = first;
    e.last = first + count;
    e.out = words;
    enumerate_rec(&e, 0);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Moebius maps                                                        */
/* ------------------------------------------------------------------ */

static mat2 mat_mul(mat2 x, mat2 y)
{
    mat2 r;
    r.a = x.a * y.a + x.b * y.c;
    r.b = x.a * y.b + x.b * y.d;
    r.c = x.c * y.a + x.d * y.c;
    r.d = x.c * y.b + x.d * y.d;
    return r;
}

/* The point (u : v) of the Riemann sphere, infinity when v = 0. */
static cplx point_of(cplx u, cplx v)
{
    if (v == 0) return INFINITY;
    return u / v;
}

/* z -> (a z + b) / (c z + d)   (Section 3, linear fractional maps), for
 * z = (u : v) on the Riemann sphere: (a u + b v) / (c u + d v). */
static cplx mobius_h(mat2 m, cplx u, cplx v)
{
    return point_of(m.a * u + m.b * v, m.c * u + m.d * v);
}

static mat2 mat_inverse(mat2 m)
{
    cplx det = m.a * m.d - m.b * m.c;
    mat2 r = {m.d / det, -m.b / det, -m.c / det, m.a / det};
    return r;
}

/* ------------------------------------------------------------------ */
/* generators and seeds                                                */
/* ------------------------------------------------------------------ */

typedef struct {
    cplx tab;
    mat2 g[4];         /* a, b, A, B */
    cplx fu[4], fv[4]; /* attracting fixed point of each generator: fu / fv, fv = 0 at infinity */
} group;

static int finite_c(cplx z) { return isfinite(creal(z)) && isfinite(cimag(z)); }

/* Attracting fixed point of z -> (a z + b)/(c z + d) on the Riemann sphere,
 * as a homogeneous pair (u : v).
 * c != 0: the roots of c z^2 + (d - a) z - b = 0; |g'(z)| = |det| / |c z + d|^2,
 *   so the attracting root is the one with the larger |c z + d|.  A tie (one
 *   parabolic root, or an elliptic pair) takes the "+" root.
 * c == 0: the map is z -> (a z + b) / d.  Infinity is fixed; when a != d so is
 *   b / (d - a), where the derivative is a / d: it attracts iff |a / d| < 1,
 *   else infinity does.  When a == d infinity is the only fixed point
 *   (parabolic), and the identity (b == 0 too) has no attracting point. */
static int attracting_fixed_point(mat2 m, cplx *u, cplx *v)
{
    if (m.c == 0) {
        if (m.d == 0) return -2;
        *u = 1;
        *v = 0;
        if (m.a == m.d) return m.b == 0 ? -2 : 0;
        if (cabs(m.a / m.d) < 1) {
            *u = m.b / (m.d - m.a);
            *v = 1;
        }
        return finite_c(*u) ? 0 : -2;
    }
    cplx disc = (m.a - m.d) * (m.a - m.d) + 4.0 * m.b * m.c;
    cplx root = csqrt(disc);
    cplx zp = ((m.a - m.d) + root) / (2.0 * m.c);
    cplx zm = ((m.a - m.d) - root) / (2.0 * m.c);
    double kp = cabs(m.c * zp + m.d);
    double km = cabs(m.c * zm + m.d);
    *u = (km > kp) ? zm : zp;
    *v = 1;
    return finite_c(*u) ? 0 : -2;
}

/* The four maps a, b, A = a^-1, B = b^-1 from a and b, each scaled to
 * determinant 1 (the Moebius map is unchanged), and their seeds. */
static int complete_group(mat2 a, mat2 b, group *g)
{
    mat2 ab[2] = {a, b};
    for (int k = 0; k < 2; k++) {
        cplx det = ab[k].a * ab[k].d - ab[k].b * ab[k].c;
        if (det == 0 || !finite_c(det)) return -2;
        cplx r = csqrt(det);
        ab[k].a /= r;
        ab[k].b /= r;
        ab[k].c /= r;
        ab[k].d /= r;
    }
    g->g[0] = ab[0];
    g->g[1] = ab[1];
    g->g[2] = mat_inverse(ab[0]);
    g->g[3] = mat_inverse(ab[1]);
    for (int k = 0; k < 4; k++) {
        mat2 m = g->g[k];
        if (!finite_c(m.a) || !finite_c(m.b) || !finite_c(m.c) || !finite_c(m.d))
            return -2;
        if (attracting_fixed_point(m, &g->fu[k], &g->fv[k]) != 0) return -2;
    }
    return 0;
}

/* Trace recipe: given tr a = ta and tr b = tb, tab = tr ab is a root of
 * tab^2 - ta tb tab + ta^2 + tb^2 = 0 (which makes tr abAB = -2), taken
 * as (ta tb + s)/2 with s^2 the discriminant and s in the closed upper
 * half plane; then
 *   z0 = (tab - 2) tb / (tb tab - 2 ta + 2i tab)
 *   a  = [[ta/2, (ta tab - 2 tb + 4i) / ((2 tab + 4) z0)],
 *         [(ta tab - 2 tb - 4i) z0 / (2 tab - 4), ta/2]]
 *   b  = [[(tb - 2i)/2, tb/2], [tb/2, (tb + 2i)/2]]
 *   A  = a^-1, B = b^-1. */
static int build_group(cplx ta, cplx tb, group *g)
{
    const cplx I2 = 2.0 * I, I4 = 4.0 * I;
    cplx disc = (ta * tb) * (ta * tb) - 4.0 * (ta * ta + tb * tb);
    cplx s = csqrt(disc);
    if (cimag(s) < 0 || (cimag(s) == 0 && creal(s) < 0)) s = -s;
    cplx tab = (ta * tb + s) / 2.0;
    cplx den_z0 = tb * tab - 2.0 * ta + I2 * tab;
    if (den_z0 == 0 || 2.0 * tab + 4.0 == 0 || 2.0 * tab - 4.0 == 0) return -2;
    cplx z0 = (tab - 2.0) * tb / den_z0;
    if (z0 == 0) return -2;
    mat2 a, b;
    a.a = ta / 2.0;
    a.b = (ta * tab - 2.0 * tb + I4) / ((2.0 * tab + 4.0) * z0);
    a.c = (ta * tab - 2.0 * tb - I4) * z0 / (2.0 * tab - 4.0);
    a.d = ta / 2.0;
    b.a = (tb - I2) / 2.0;
    b.b = tb / 2.0;
    b.c = tb / 2.0;
    b.d = (tb + I2) / 2.0;
    g->tab = tab;
    g->g[0] = a;
    g->g[1] = b;
    g->g[2] = mat_inverse(a);
    g->g[3] = mat_inverse(b);
    for (int k = 0; k < 4; k++) {
        mat2 m = g->g[k];
        if (!finite_c(m.a) || !finite_c(m.b) || !finite_c(m.c) || !finite_c(m.d))
            return -2;
        /* a seed may be infinity: a has c = 0 on a curve of traces, among
         * them ta = tb = 2 (the double cusp), where it is a translation */
        if (attracting_fixed_point(m, &g->fu[k], &g->fv[k]) != 0) return -2;
    }
    return 0;
}

/* Maskit's parametrisation of the once-punctured torus groups (the Maskit
 * embedding of the paper's figures), as in Indra's Pearls:
 *   a = [[-i mu, -i], [-i, 0]],  b = [[1, 2], [0, 1]],
 * so tr a = -i mu, b is the translation z -> z + 2 (parabolic, fixed at
 * infinity) and tr abAB = -2. */
static int build_maskit(cplx mu, group *g)
{
    mat2 a = {-I * mu, -I, -I, 0};
    mat2 b = {1, 2, 0, 1};
    g->tab = 0;
    return complete_group(a, b, g);
}

static void put_c(double *dst, cplx z)
{
    dst[0] = creal(z);
    dst[1] = cimag(z);
}

static cplx get_c(const double *src) { return src[0] + src[1] * I; }

int oracle_generators(double ta_re, double ta_im, double tb_re, double tb_im,
                      double *tab_out, double *gens_out, double *fix_out)
{
    group g;
    int rc = build_group(ta_re + ta_im * I, tb_re + tb_im * I, &g);
    if (rc) return rc;
    if (tab_out) put_c(tab_out, g.tab);
    if (gens_out) {
        for (int k = 0; k < 4; k++) {
            put_c(gens_out + ((k * 2 + 0) * 2 + 0) * 2, g.g[k].a);
            put_c(gens_out + ((k * 2 + 0) * 2 + 1) * 2, g.g[k].b);
            put_c(gens_out + ((k * 2 + 1) * 2 + 0) * 2, g.g[k].c);
            put_c(gens_out + ((k * 2 + 1) * 2 + 1) * 2, g.g[k].d);
        }
    }
    if (fix_out)
        for (int k = 0; k < 4; k++) put_c(fix_out + 2 * k, g.fv[k] == 0 ? INFINITY : g.fu[k] / g.fv[k]);
    return 0;
}

static void put_group(const group *g, double *gens_out, double *seeds_out)
{
    for (int k = 0; k < 4; k++) {
        put_c(gens_out + ((k * 2 + 0) * 2 + 0) * 2, g->g[k].a);
        put_c(gens_out + ((k * 2 + 0) * 2 + 1) * 2, g->g[k].b);
        put_c(gens_out + ((k * 2 + 1) * 2 + 0) * 2, g->g[k].c);
        put_c(gens_out + ((k * 2 + 1) * 2 + 1) * 2, g->g[k].d);
        put_c(seeds_out + 4 * k, g->fu[k]);
        put_c(seeds_out + 4 * k + 2, g->fv[k]);
    }
}

int oracle_group_recipe(double ta_re, double ta_im, double tb_re, double tb_im,
                        double *gens_out, double *seeds_out)
{
    if (!gens_out || !seeds_out) return -1;
    group g;
    int rc = build_group(ta_re + ta_im * I, tb_re + tb_im * I, &g);
    if (rc) return rc;
    put_group(&g, gens_out, seeds_out);
    return 0;
}

int oracle_group_explicit(const double *ab, double *gens_out, double *seeds_out)
{
    if (!ab || !gens_out || !seeds_out) return -1;
    group g;
    mat2 a = {get_c(ab + 0), get_c(ab + 2), get_c(ab + 4), get_c(ab + 6)};
    mat2 b = {get_c(ab + 8), get_c(ab + 10), get_c(ab + 12), get_c(ab + 14)};
    g.tab = 0;
    int rc = complete_group(a, b, &g);
    if (rc) return rc;
    put_group(&g, gens_out, seeds_out);
    return 0;
}

int oracle_group_maskit(double mu_re, double mu_im, double *gens_out, double *seeds_out)
{
    if (!gens_out || !seeds_out) return -1;
    group g;
    int rc = build_maskit(mu_re + mu_im * I, &g);
    if (rc) return rc;
    put_group(&g, gens_out, seeds_out);
    return 0;
}

/* ------------------------------------------------------------------ */
/* word values                                                         */
/* ------------------------------------------------------------------ */

/* seed < 0: the attracting fixed point of the word's last letter (the
 * default); seed = 0..3: that generator's attracting fixed point, fed to
 * every word (the paper's index-search loop, Section 6). */
static cplx value_product(const group *g, const uint8_t *w, int d, int seed)
{
    /* M = G_{w1} G_{w2} ... G_{wd}, then M applied to the seed */
    mat2 m = g->g[w[0]];
    for (int j = 1; j < d; j++) m = mat_mul(m, g->g[w[j]]);
    int s = seed < 0 ? w[d - 1] : seed;
    return mobius_h(m, g->fu[s], g->fv[s]);
}

static cplx value_literal(const group *g, const uint8_t *w, int d, int seed)
{
    /* (u : v) = seed; (u : v) <- G_{wj} (u : v) for j = d, d-1, ..., 1 */
    const int k = (seed >= 0) ? seed : w[d - 1];
    cplx u = g->fu[k], v = g->fv[k];
    for (int j = d - 1; j >= 0; j--) {
        mat2 m = g->g[w[j]];
        cplx nu = m.a * u + m.b * v;
        v = m.c * u + m.d * v;
        u = nu;
    }
    return point_of(u, v);
}

static int group_from_arrays(const double *gens, const double *fix, group *g)
{
    for (int k = 0; k < 4; k++) {
        g->g[k].a = get_c(gens + ((k * 2 + 0) * 2 + 0) * 2);
        g->g[k].b = get_c(gens + ((k * 2 + 0) * 2 + 1) * 2);
        g->g[k].c = get_c(gens + ((k * 2 + 1) * 2 + 0) * 2);
        g->g[k].d = get_c(gens + ((k * 2 + 1) * 2 + 1) * 2);
        g->fu[k] = get_c(fix + 2 * k);
        g->fv[k] = 1;
        if (isinf(creal(g->fu[k])) || isinf(cimag(g->fu[k]))) {  /* infinity, as oracle_generators writes it */
            g->fu[k] = 1;
            g->fv[k] = 0;
        }
    }
    return 0;
}

/* gens as oracle_generators lays them out; seeds: 4 homogeneous pairs (u, v) */
static void group_from_group_arrays(const double *gens, const double *seeds, group *g)
{
    group_from_arrays(gens, seeds, g);  /* matrices */
    for (int k = 0; k < 4; k++) {
        g->fu[k] = get_c(seeds + 4 * k);
        g->fv[k] = get_c(seeds + 4 * k + 2);
    }
    g->tab = 0;
}

int oracle_word_value(const uint8_t *word, int depth, const double *gens,
                      const double *fix, int literal, double *z_out)
{
    if (!word || !gens || !fix || !z_out || depth < 1 || depth > MAX_DEPTH)
        return -1;
    for (int j = 0; j < depth; j++) {
        if (word[j] > 3) return -1;
        if (j > 0 && word[j] == INVERSE[word[j - 1]]) return -1;
    }
    group g;
    group_from_arrays(gens, fix, &g);
    put_c(z_out, literal ? value_literal(&g, word, depth, -1)
                         : value_product(&g, word, depth, -1));
    return 0;
}

static int eval_words(const group *g, int seed, int depth, const uint64_t *idx, uint64_t n,
                      int literal, double *z_out)
{
    uint8_t w[MAX_DEPTH];
    for (uint64_t i = 0; i < n; i++) {
        if (oracle_unrank(idx[i], depth, w) != 0) return -1;
        put_c(z_out + 2 * i, literal ? value_literal(g, w, depth, seed)
                                     : value_product(g, w, depth, seed));
    }
    return 0;
}

int oracle_eval(double ta_re, double ta_im, double tb_re, double tb_im,
                int depth, const uint64_t *idx, uint64_t n, int literal,
                double *z_out)
{
    if (depth < 1 || depth > MAX_DEPTH || (n && (!idx || !z_out))) return -1;
    group g;
    int rc = build_group(ta_re + ta_im * I, tb_re + tb_im * I, &g);
    if (rc) return rc;
    return eval_words(&g, -1, depth, idx, n, literal, z_out);
}

int oracle_eval_group(const double *gens, const double *seeds, int seed, int depth,
                      const uint64_t *idx, uint64_t n, int literal, double *z_out)
{
    if (!gens || !seeds || seed < -1 || seed > 3) return -1;
    if (depth < 1 || depth > MAX_DEPTH || (n && (!idx || !z_out))) return -1;
    group g;
    group_from_group_arrays(gens, seeds, &g);
    return eval_words(&g, seed, depth, idx, n, literal, z_out);
}

/* ------------------------------------------------------------------ */
/* rendering                                                           */
/* ------------------------------------------------------------------ */

typedef struct {
    double x0, x1, y0, y1;
    uint32_t width, height;
    double edge_tol;
} window;

/* col = floor((x - x0) W / (x1 - x0)), row = floor((y - y0) H / (y1 - y0));
 * kept iff both are in range; NaN and infinities are dropped. */
static int bin_point(const window *w, cplx z, uint32_t *bin, int *near_edge)
{
    double x = creal(z), y = cimag(z);
    *near_edge = 0;
    if (!isfinite(x) || !isfinite(y)) return 0;
    double fx = (x - w->x0) * (double)w->width / (w->x1 - w->x0);
    double fy = (y - w->y0) * (double)w->height / (w->y1 - w->y0);
    if (w->edge_tol > 0) {
        double t = w->edge_tol;
        int in_reach = fx > -t && fx < w->width + t && fy > -t && fy < w->height + t;
        int close = fabs(fx - nearbyint(fx)) < t || fabs(fy - nearbyint(fy)) < t;
        *near_edge = in_reach && close;
    }
    if (!(fx >= 0 && fx < (double)w->width && fy >= 0 && fy < (double)w->height))
        return 0;
    uint32_t col = (uint32_t)floor(fx), row = (uint32_t)floor(fy);
    *bin = row * w->width + col;
    return 1;
}

typedef struct {
    const group *g;
    const window *win;
    int depth, seed;
    uint64_t first, last; /* leaf range [first, last) of this depth */
    uint32_t *image;
    uint64_t dropped, near_edge;
    uint8_t word[MAX_DEPTH];
} render_ctx;

/* Node at depth j with word[0..j-1] and product m = G_{w1}...G_{wj};
 * its subtree holds the leaves [base, base + 3^(d-j)) (4 * 3^(d-1) for
 * the root).  Subtrees entirely outside [first, last) are not entered. */
static void render_rec(render_ctx *r, int j, mat2 m, uint64_t base)
{
    int d = r->depth;
    if (j == d) {
        const int s = r->seed < 0 ? r->word[d - 1] : r->seed;
        cplx z = mobius_h(m, r->g->fu[s], r->g->fv[s]);
        uint32_t bin;
        int near;
        if (bin_point(r->win, z, &bin, &near))
            r->image[bin] += 1u;
        else
            r->dropped++;
        r->near_edge += (uint64_t)near;
        return;
    }
    uint64_t child_leaves = pow3(d - j - 1);
    for (int c = 0; c < 4; c++) {
        if (j > 0 && c == INVERSE[r->word[j - 1]]) continue;
        uint64_t lo = base, hi = base + child_leaves;
        base = hi;
        if (hi <= r->first || lo >= r->last) continue;
        r->word[j] = (uint8_t)c;
        mat2 child = (j == 0) ? r->g->g[c] : mat_mul(m, r->g->g[c]);
        render_rec(r, j + 1, child, lo);
    }
}

/* Render the words with combined index in [first, first+count) of the
 * index space "all words of depth min_depth, then all of min_depth+1, ...,
 * then all of depth" into image (added to what it holds).  seed: as in
 * value_product, or 4 for every generator's fixed point in turn, each word
 * drawn once from each (the paper's index-search loop, Section 6). */
static void render_range(const group *g, const window *win, int seed, int min_depth,
                         int depth, uint64_t first, uint64_t count,
                         uint32_t *image, uint64_t *dropped, uint64_t *near_edge)
{
    if (seed == 4) {
        for (int p = 0; p < 4; p++)
            render_range(g, win, p, min_depth, depth, first, count, image, dropped, near_edge);
        return;
    }
    uint64_t offset = 0, end = first + count;
    for (int d = min_depth; d <= depth; d++) {
        uint64_t n = oracle_num_words(d);
        uint64_t lo = first > offset ? first - offset : 0;
        uint64_t hi = end - offset < n ? end - offset : n;
        if (end > offset && first < offset + n && lo < hi) {
            render_ctx r;
            memset(&r, 0, sizeof r);
            r.g = g;
            r.win = win;
            r.depth = d;
            r.seed = seed;
            r.first = lo;
            r.last = hi;
            r.image = image;
            mat2 identity = {1, 0, 0, 1};
            render_rec(&r, 0, identity, 0);
            *dropped += r.dropped;
            *near_edge += r.near_edge;
        }
        offset += n;
    }
}

typedef struct {
    const group *g;
    const window *win;
    int seed, min_depth, depth;
    uint64_t first, count;
    uint32_t *image;
    uint64_t dropped, near_edge;
} thread_job;

static void *thread_main(void *arg)
{
    thread_job *t = (thread_job *)arg;
    render_range(t->g, t->win, t->seed, t->min_depth, t->depth, t->first, t->count,
                 t->image, &t->dropped, &t->near_edge);
    return NULL;
}

static int render_group(const group *g, int seed, int depth, int min_depth,
                        double x0, double x1, double y0, double y1,
                        uint32_t width, uint32_t height,
                        uint64_t first, uint64_t count, int nthreads,
                        double edge_tol, uint32_t *image, uint64_t *dropped,
                        uint64_t *near_edge)
{
    if (depth < 1 || depth > MAX_DEPTH || min_depth < 1 || min_depth > depth || seed < -1 || seed > 4)
        return -1;
    if (!image || width == 0 || height == 0 || !(x1 > x0) || !(y1 > y0))
        return -1;
    uint64_t total = 0;
    for (int d = min_depth; d <= depth; d++) total += oracle_num_words(d);
    if (first > total || count > total - first) return -1;
    if (nthreads < 1) nthreads = 1;
    int rc = 0;
    window win = {x0, x1, y0, y1, width, height, edge_tol};
    uint64_t bins = (uint64_t)width * height;

    /* contiguous sub-ranges, one private image per thread, summed after */
    thread_job *jobs = (thread_job *)calloc((size_t)nthreads, sizeof(thread_job));
    pthread_t *tids = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !tids) { free(jobs); free(tids); return -1; }
    uint64_t start = first;
    for (int t = 0; t < nthreads; t++) {
        uint64_t share = count / (uint64_t)nthreads + ((uint64_t)t < count % (uint64_t)nthreads);
        jobs[t].g = g;
        jobs[t].win = &win;
        jobs[t].seed = seed;
        jobs[t].min_depth = min_depth;
        jobs[t].depth = depth;
        jobs[t].first = start;
        jobs[t].count = share;
        start += share;
        jobs[t].image = (t == 0) ? image : (uint32_t *)calloc(bins, sizeof(uint32_t));
        if (!jobs[t].image) { nthreads = t; rc = -1; break; }
    }
    for (int t = 1; t < nthreads; t++) pthread_create(&tids[t], NULL, thread_main, &jobs[t]);
    if (nthreads > 0) thread_main(&jobs[0]);
    for (int t = 1; t < nthreads; t++) pthread_join(tids[t], NULL);
    uint64_t drop = 0, near = 0;
    for (int t = 0; t < nthreads; t++) {
        drop += jobs[t].dropped;
        near += jobs[t].near_edge;
        if (t > 0) {
            for (uint64_t i = 0; i < bins; i++) image[i] += jobs[t].image[i];
            free(jobs[t].image);
        }
    }
    free(jobs);
    free(tids);
    if (dropped) *dropped = drop;
    if (near_edge) *near_edge = near;
    return rc;
}

int oracle_render(double ta_re, double ta_im, double tb_re, double tb_im,
                  int depth, int min_depth,
                  double x0, double x1, double y0, double y1,
                  uint32_t width, uint32_t height,
                  uint64_t first, uint64_t count, int nthreads,
                  double edge_tol, uint32_t *image, uint64_t *dropped,
                  uint64_t *near_edge)
{
    group g;
    int rc = build_group(ta_re + ta_im * I, tb_re + tb_im * I, &g);
    if (rc) return rc;
    return render_group(&g, -1, depth, min_depth, x0, x1, y0, y1, width, height, first, count,
                        nthreads, edge_tol, image, dropped, near_edge);
}

int oracle_render_group(const double *gens, const double *seeds, int seed,
                        int depth, int min_depth,
                        double x0, double x1, double y0, double y1,
                        uint32_t width, uint32_t height,
                        uint64_t first, uint64_t count, int nthreads,
                        double edge_tol, uint32_t *image, uint64_t *dropped,
                        uint64_t *near_edge)
{
    if (!gens || !seeds) return -1;
    group g;
    group_from_group_arrays(gens, seeds, &g);
    return render_group(&g, seed, depth, min_depth, x0, x1, y0, y1, width, height, first, count,
                        nthreads, edge_tol, image, dropped, near_edge);
}

/* ------------------------------------------------------------------ */
/* indexed Cayley tables (Section 5)                                   */
/* ------------------------------------------------------------------ */
/*
 * A table has states 0..S-1 and symbols 1..m; next = table[s * (m + 1) + x]
 * (column 0, the identity symbol, is not read).  State 0 is where a walk
 * starts and, reached again, the crash state.  A word x_1 ... x_d is read
 * right to left (x_d first, Section 5's table walk); it is regular when no
 * step of that walk lands in state 0.  Regular words are numbered in
 * lexicographic order of (x_1, ..., x_d), x_1 most significant, which is the
 * order in which the paper's scan of all m^d digit strings (Section 6)
 * meets them.
 *
 * Counting: C[L][s] is the number of regular words of length L whose walk
 * ends in state s (C[0][0] = 1: the empty walk stays in the start state).
 * A prefix p of a word is read after the rest of the word, starting in the
 * state the rest ended in; good_p is the set of states from which p can be
 * read without a crash, with good_(p x)(s) = [T(s, x) != 0] and
 * good_p(T(s, x)).  The words that begin with p number
 * sum over s in good_p of C[d - |p|][s].
 */

#define MAX_STATES 16
#define MAX_SYMBOLS 8

typedef struct {
    int S, m;
    const uint8_t *t;
    uint64_t C[MAX_DEPTH + 1][MAX_STATES];
    int depth;
} cayley;

static int cayley_next(const cayley *c, int s, int x) { return c->t[s * (c->m + 1) + x]; }

static int cayley_init(const uint8_t *table, int S, int m, int depth, cayley *c)
{
    if (!table || S < 2 || S > MAX_STATES || m < 1 || m > MAX_SYMBOLS || depth < 1 || depth > MAX_DEPTH)
        return -1;
    for (int i = 0; i < S * (m + 1); i++)
        if (table[i] >= S) return -1;
    c->S = S;
    c->m = m;
    c->t = table;
    c->depth = depth;
    memset(c->C, 0, sizeof c->C);
    c->C[0][0] = 1;
    for (int L = 1; L <= depth; L++) {
        for (int s = 0; s < S; s++) {
            if (!c->C[L - 1][s]) continue;
            for (int x = 1; x <= m; x++) {
                int t = cayley_next(c, s, x);
                if (t == 0) continue;
                if (c->C[L][t] > UINT64_MAX / 2 - c->C[L - 1][s]) return -1;  /* too many words */
                c->C[L][t] += c->C[L - 1][s];
            }
        }
        /* every word of a length gets a 64-bit index: their total, which
         * bounds every count by a good set, must fit */
        uint64_t total = 0;
        for (int s = 0; s < S; s++) {
            if (total > UINT64_MAX - c->C[L][s]) return -1;
            total += c->C[L][s];
        }
    }
    return 0;
}

/* words beginning with a prefix whose good set is `good`, with L symbols to go */
static uint64_t cayley_count(const cayley *c, int L, uint32_t good)
{
    uint64_t n = 0;
    for (int s = 0; s < c->S; s++)
        if ((good >> s) & 1u) n += c->C[L][s];
    return n;
}

static uint32_t cayley_extend(const cayley *c, uint32_t good, int x)
{
    uint32_t g = 0;
    for (int s = 0; s < c->S; s++) {
        int t = cayley_next(c, s, x);
        if (t != 0 && ((good >> t) & 1u)) g |= 1u << s;
    }
    return g;
}

uint64_t oracle_cayley_num_words(const uint8_t *table, int n_states, int n_symbols, int depth)
{
    cayley c;
    if (cayley_init(table, n_states, n_symbols, depth, &c)) return 0;
    return cayley_count(&c, depth, (1u << n_states) - 1);
}

int oracle_cayley_unrank(const uint8_t *table, int n_states, int n_symbols, uint64_t index, int depth,
                         uint8_t *symbols)
{
    cayley c;
    if (!symbols || cayley_init(table, n_states, n_symbols, depth, &c)) return -1;
    uint32_t good = (1u << n_states) - 1;
    if (index >= cayley_count(&c, depth, good)) return -1;
    for (int j = 0; j < depth; j++) {
        int L = depth - j - 1;
        int x;
        for (x = 1; x <= n_symbols; x++) {
            uint32_t g = cayley_extend(&c, good, x);
            uint64_t n = cayley_count(&c, L, g);
            if (index < n) {
                good = g;
                break;
            }
            index -= n;
        }
        symbols[j] = (uint8_t)x;
    }
    return 0;
}

/* the paper's scan: every m^d digit string in numeric order (digit x - 1
 * for symbol x, most significant leftmost), kept when its right-to-left
 * table walk never reaches state 0; writes the first `cap` survivors */
int oracle_cayley_scan(const uint8_t *table, int n_states, int n_symbols, int depth, uint8_t *out,
                       uint64_t cap, uint64_t *n_out)
{
    if (!table || !n_out || depth < 1 || depth > 12 || n_symbols < 1 || n_symbols > MAX_SYMBOLS) return -1;
    uint64_t total = 1, kept = 0;
    for (int j = 0; j < depth; j++) total *= (uint64_t)n_symbols;
    uint8_t w[16];
    for (uint64_t n = 0; n < total; n++) {
        uint64_t q = n;
        for (int j = depth - 1; j >= 0; j--) {
            w[j] = (uint8_t)(q % (uint64_t)n_symbols + 1);
            q /= (uint64_t)n_symbols;
        }
        int s = 0, ok = 1;
        for (int j = depth - 1; j >= 0 && ok; j--) {
            s = table[s * (n_symbols + 1) + w[j]];
            ok = s != 0;
        }
        if (!ok) continue;
        if (out && kept < cap) memcpy(out + kept * depth, w, (size_t)depth);
        kept++;
    }
    *n_out = kept;
    return 0;
}

/* maps: m matrices of 8 doubles (a, b, c, d complex); each symbol's seed is
 * its map's attracting fixed point (homogeneous) */
static int cayley_maps(const double *maps, int m, mat2 *g, cplx *fu, cplx *fv)
{
    for (int k = 0; k < m; k++) {
        mat2 a = {get_c(maps + 8 * k), get_c(maps + 8 * k + 2), get_c(maps + 8 * k + 4), get_c(maps + 8 * k + 6)};
        if (!finite_c(a.a) || !finite_c(a.b) || !finite_c(a.c) || !finite_c(a.d)) return -1;
        cplx det = a.a * a.d - a.b * a.c;
        if (det == 0) return -2;
        cplx r = csqrt(det);
        a.a /= r;
        a.b /= r;
        a.c /= r;
        a.d /= r;
        g[k] = a;
        if (attracting_fixed_point(a, &fu[k], &fv[k]) != 0) return -2;
    }
    return 0;
}

/* value of symbols x_1..x_d: maps applied right to left to the seed (the
 * last symbol's fixed point, or symbol seed + 1's) */
static cplx cayley_value(const mat2 *g, const cplx *fu, const cplx *fv, const uint8_t *w, int d, int seed,
                         int literal)
{
    int s = seed < 0 ? w[d - 1] - 1 : seed;
    if (literal) {
        cplx u = fu[s], v = fv[s];
        for (int j = d - 1; j >= 0; j--) {
            mat2 a = g[w[j] - 1];
            cplx nu = a.a * u + a.b * v;
            v = a.c * u + a.d * v;
            u = nu;
        }
        return point_of(u, v);
    }
    mat2 p = g[w[0] - 1];
    for (int j = 1; j < d; j++) p = mat_mul(p, g[w[j] - 1]);
    return mobius_h(p, fu[s], fv[s]);
}

int oracle_cayley_eval(const uint8_t *table, int n_states, int n_symbols, const double *maps, int seed,
                       int depth, const uint64_t *idx, uint64_t n, int literal, double *z_out)
{
    if (!maps || seed < -1 || seed >= n_symbols || (n && (!idx || !z_out))) return -1;
    mat2 g[MAX_SYMBOLS];
    cplx fu[MAX_SYMBOLS], fv[MAX_SYMBOLS];
    int rc = cayley_maps(maps, n_symbols, g, fu, fv);
    if (rc) return rc;
    uint8_t w[MAX_DEPTH];
    for (uint64_t i = 0; i < n; i++) {
        if (oracle_cayley_unrank(table, n_states, n_symbols, idx[i], depth, w)) return -1;
        put_c(z_out + 2 * i, cayley_value(g, fu, fv, w, depth, seed, literal));
    }
    return 0;
}

typedef struct {
    const cayley *c;
    const mat2 *g;
    const cplx *fu, *fv;
    const window *win;
    int seed;
    uint64_t first, last;
    uint32_t *image;
    uint64_t dropped, near_edge;
    uint8_t word[MAX_DEPTH];
} cayley_ctx;

/* depth-first walk over the regular words of one depth in index order;
 * the node at depth j has prefix word[0..j-1], product m and good set
 * `good`; its words are [base, base + count) */
static void cayley_rec(cayley_ctx *r, int j, mat2 m, uint32_t good, uint64_t base)
{
    const cayley *c = r->c;
    int d = c->depth;
    if (j == d) {
        int s = r->seed < 0 ? r->word[d - 1] - 1 : r->seed;
        cplx z = mobius_h(m, r->fu[s], r->fv[s]);
        uint32_t bin;
        int near;
        if (bin_point(r->win, z, &bin, &near))
            r->image[bin] += 1u;
        else
            r->dropped++;
        r->near_edge += (uint64_t)near;
        return;
    }
    for (int x = 1; x <= c->m; x++) {
        uint32_t g = cayley_extend(c, good, x);
        uint64_t n = cayley_count(c, d - j - 1, g);
        uint64_t lo = base, hi = base + n;
        base = hi;
        if (n == 0 || hi <= r->first || lo >= r->last) continue;
        r->word[j] = (uint8_t)x;
        mat2 child = (j == 0) ? r->g[x - 1] : mat_mul(m, r->g[x - 1]);
        cayley_rec(r, j + 1, child, g, lo);
    }
}

/* seed: -1 own, 0..m-1 that symbol's fixed point, m: each symbol's in turn */
int oracle_cayley_render(const uint8_t *table, int n_states, int n_symbols, const double *maps, int seed,
                         int depth, int min_depth, double x0, double x1, double y0, double y1,
                         uint32_t width, uint32_t height, double edge_tol, uint32_t *image,
                         uint64_t *dropped, uint64_t *near_edge)
{
    if (!maps || !image || seed < -1 || seed > n_symbols || min_depth < 1 || min_depth > depth) return -1;
    if (width == 0 || height == 0 || !(x1 > x0) || !(y1 > y0)) return -1;
    mat2 g[MAX_SYMBOLS];
    cplx fu[MAX_SYMBOLS], fv[MAX_SYMBOLS];
    int rc = cayley_maps(maps, n_symbols, g, fu, fv);
    if (rc) return rc;
    window win = {x0, x1, y0, y1, width, height, edge_tol};
    uint64_t drop = 0, near = 0;
    for (int s0 = (seed == n_symbols ? 0 : seed); s0 <= (seed == n_symbols ? n_symbols - 1 : seed); s0++) {
        for (int d = min_depth; d <= depth; d++) {
            cayley c;
            if (cayley_init(table, n_states, n_symbols, d, &c)) return -1;
            cayley_ctx r;
            memset(&r, 0, sizeof r);
            r.c = &c;
            r.g = g;
            r.fu = fu;
            r.fv = fv;
            r.win = &win;
            r.seed = s0;
            r.first = 0;
            r.last = UINT64_MAX;
            r.image = image;
            mat2 identity = {1, 0, 0, 1};
            cayley_rec(&r, 0, identity, (1u << n_states) - 1, 0);
            drop += r.dropped;
            near += r.near_edge;
        }
    }
    if (dropped) *dropped = drop;
    if (near_edge) *near_edge = near;
    return 0;
}

/* ------------------------------------------------------------------ */
/* probabilistic rendering: one orbit per walker (Section 4)           */
/* ------------------------------------------------------------------ */

/* Section 4 describes the probabilistic approach only in words: a single
 * word grows as generators are appended through random picks under some
 * probability law, and its orbit is drawn.  The reading taken here:
 *   - a walker's first letter c_0 is uniform over a, b, A, B, and its
 *     orbit starts at the attracting fixed point of c_0;
 *   - step n >= 1 picks c_n uniformly among the three letters that do not
 *     undo c_{n-1} (the word stays reduced) and maps the point:
 *     z_n = G_{c_n}(z_{n-1});
 *   - after burn_in steps, the next n_steps points are drawn.
 * So z_n is the value of the reduced word c_n ... c_1 c_0 (rightmost letter
 * applied first, from the fixed point of its last letter), the word value of
 * Section 1.  The commutator "boost" of the Fig. 3 caption is not applied.
 *
 * Random numbers: Philox4x64-10 (J. Salmon, M. Moraes, R. Dror, D. Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11).  A counter of four
 * 64-bit words is encrypted under a key of two by ten rounds; a round takes
 * the 128-bit products of words 0 and 2 with two multipliers and mixes their
 * halves with words 1 and 3 and the key, and the key is advanced by two
 * Weyl constants between rounds. */
static const uint64_t PHILOX_M0 = 0xD2E7470EE14C6C93ull, PHILOX_M1 = 0xCA5A826395121157ull;
static const uint64_t PHILOX_W0 = 0x9E3779B97F4A7C15ull, PHILOX_W1 = 0xBB67AE8584CAA73Bull;

static void mul_full64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    __extension__ unsigned __int128 p = (unsigned __int128)a * b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

int oracle_philox4x64_10(const uint64_t *ctr, const uint64_t *key, uint64_t *out)
{
    if (!ctr || !key || !out) return -1;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t hi0, lo0, hi1, lo1;
        mul_full64(PHILOX_M0, x0, &hi0, &lo0);
        mul_full64(PHILOX_M1, x2, &hi1, &lo1);
        uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
        x0 = y0;
        x1 = y1;
        x2 = y2;
        x3 = y3;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
    return 0;
}

/* The n-th 32-bit random value of walker `walker`: block n / 8 is Philox4x64-10
 * of the counter (n / 8, walker, 0, 0) under the key (seed, 0); its 64-bit
 * outputs r0..r3 give the values r0 low, r0 high, r1 low, ..., r3 high. */
static uint32_t walk_value(uint64_t seed, uint64_t walker, uint64_t n)
{
    uint64_t ctr[4] = {n / 8, walker, 0, 0}, key[2] = {seed, 0}, r[4];
    oracle_philox4x64_10(ctr, key, r);
    uint64_t w = r[(n % 8) / 2];
    return (uint32_t)((n % 2) ? (w >> 32) : w);
}

/* Letters c_0 .. c_{n-1} of a walker: c_0 = the value's top two bits (a
 * uniform letter); for k >= 1 the value x picks t = floor(3 x / 2^32) in
 * {0, 1, 2} and c_k is the t-th letter, in code order, other than the
 * inverse of c_{k-1}. */
int oracle_walk_letters(uint64_t seed, uint64_t walker, uint32_t n, uint8_t *letters)
{
    if (!letters && n) return -1;
    for (uint32_t k = 0; k < n; k++) {
        uint32_t x = walk_value(seed, walker, k);
        if (k == 0) {
            letters[0] = (uint8_t)(x >> 30);
            continue;
        }
        uint32_t t = (uint32_t)(((uint64_t)x * 3u) >> 32);
        int skip = INVERSE[letters[k - 1]];
        int c = -1;
        for (int cand = 0, seen = 0; cand < 4; cand++) {
            if (cand == skip) continue;
            if (seen == (int)t) {
                c = cand;
                break;
            }
            seen++;
        }
        letters[k] = (uint8_t)c;
    }
    return 0;
}

/* Points of walkers first_walker .. first_walker + n_walkers - 1: for each,
 * z_{burn_in + 1} .. z_{burn_in + n_steps}, walker-major, each step applied
 * to the previous point literally, z <- (a z + b) / (c z + d) on the
 * Riemann sphere (infinity as (1 : 0)). */
static int walk_run(const group *g, uint64_t seed, uint64_t walker, uint32_t burn_in, uint32_t n_steps,
                    cplx *z_out)
{
    const uint32_t n = 1 + burn_in + n_steps;
    uint8_t *c = (uint8_t *)malloc(n);
    if (!c) return -1;
    oracle_walk_letters(seed, walker, n, c);
    cplx u = g->fu[c[0]], v = g->fv[c[0]];
    for (uint32_t k = 1; k < n; k++) {
        cplx z = mobius_h(g->g[c[k]], u, v);
        if (finite_c(z)) {
            u = z;
            v = 1;
        } else {
            u = 1;
            v = 0;
        }
        if (k > burn_in) z_out[k - burn_in - 1] = point_of(u, v);
    }
    free(c);
    return 0;
}

int oracle_walk_points(const double *gens, const double *seeds, uint64_t seed, uint64_t first_walker,
                       uint64_t n_walkers, uint32_t burn_in, uint32_t n_steps, double *z_out)
{
    if (!gens || !seeds || (!z_out && n_walkers && n_steps)) return -1;
    if (n_walkers && n_walkers - 1 > UINT64_MAX - first_walker) return -1;
    group g;
    group_from_group_arrays(gens, seeds, &g);
    cplx *z = (cplx *)malloc((size_t)(n_steps ? n_steps : 1) * sizeof(cplx));
    if (!z) return -1;
    for (uint64_t w = 0; w < n_walkers; w++) {
        if (walk_run(&g, seed, first_walker + w, burn_in, n_steps, z)) {
            free(z);
            return -1;
        }
        for (uint32_t s = 0; s < n_steps; s++) put_c(z_out + 2 * (w * n_steps + s), z[s]);
    }
    free(z);
    return 0;
}

/* The walkers' points binned as every render bins (bin_point). */
int oracle_walk_render(const double *gens, const double *seeds, uint64_t seed, uint64_t first_walker,
                       uint64_t n_walkers, uint32_t burn_in, uint32_t n_steps,
                       double x0, double x1, double y0, double y1, uint32_t width, uint32_t height,
                       double edge_tol, uint32_t *image, uint64_t *dropped, uint64_t *near_edge)
{
    if (!gens || !seeds || !image || width == 0 || height == 0) return -1;
    if (n_walkers && n_walkers - 1 > UINT64_MAX - first_walker) return -1;
    group g;
    group_from_group_arrays(gens, seeds, &g);
    window win = {x0, x1, y0, y1, width, height, edge_tol};
    cplx *z = (cplx *)malloc((size_t)(n_steps ? n_steps : 1) * sizeof(cplx));
    if (!z) return -1;
    uint64_t drop = 0, near = 0;
    for (uint64_t w = 0; w < n_walkers; w++) {
        if (walk_run(&g, seed, first_walker + w, burn_in, n_steps, z)) {
            free(z);
            return -1;
        }
        for (uint32_t s = 0; s < n_steps; s++) {
            uint32_t bin;
            int ne;
            if (bin_point(&win, z[s], &bin, &ne)) image[bin] += 1;
            else drop++;
            near += (uint64_t)ne;
        }
    }
    free(z);
    if (dropped) *dropped = drop;
    if (near_edge) *near_edge = near;
    return 0;
}
