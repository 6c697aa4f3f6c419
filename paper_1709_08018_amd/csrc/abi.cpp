// abi.cpp -- host side of libkl: argument validation, the trace recipe and
// seeds in FP64, planning of the head/tail split, device temporaries, and
// the extern "C" entry points declared in include/kl.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "kl_internal.hpp"

namespace kl {

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;

int set_error(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}
#define fail set_error

static int hip_fail(hipError_t e, const char* what) {
    return fail(e == hipErrorOutOfMemory ? KL_ENOMEM : KL_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ------------------------------------------------------------------ counting
uint64_t pow3_u64(int n) {
    uint64_t p = 1;
    for (int i = 0; i < n; ++i) p *= 3;
    return p;
}

uint64_t num_words(int depth) {
    if (depth < 1 || depth > KL_MAX_DEPTH) return 0;
    return 4 * pow3_u64(depth - 1);
}

// ------------------------------------------------------------------ recipe
using cd = std::complex<double>;

static bool finite(cd z) { return std::isfinite(z.real()) && std::isfinite(z.imag()); }

// Attracting fixed point of [[a, b], [c, d]] (det 1) on the Riemann sphere.
// c != 0: of the two roots z of c z^2 + (d - a) z - b = 0, the one where
// |c z + d| is larger, since |g'(z)| = 1 / |c z + d|^2; equal moduli
// (parabolic, elliptic) take the "+" root.  c == 0: z -> (a z + b) / d
// fixes infinity, and b / (d - a) when a != d, where g' = a / d; that point
// attracts iff |a / d| < 1, else infinity does; with a == d infinity is the
// only fixed point, and the identity has no attracting one.
static int attracting_point(const cd m[4], cd* out, bool* at_inf) {
    const cd a = m[0], b = m[1], c = m[2], d = m[3];
    *at_inf = false;
    *out = cd(0.0);
    if (c == cd(0.0)) {
        if (d == cd(0.0)) return KL_ESINGULAR;
        if (a == d) {
            if (b == cd(0.0)) return KL_ESINGULAR;
            *at_inf = true;
            return KL_OK;
        }
        if (std::abs(a / d) < 1.0) {
            *out = b / (d - a);
            return finite(*out) ? KL_OK : KL_ESINGULAR;
        }
        *at_inf = true;
        return KL_OK;
    }
    const cd disc = (a - d) * (a - d) + 4.0 * b * c;
    const cd root = std::sqrt(disc);
    const cd zp = ((a - d) + root) / (2.0 * c);
    const cd zm = ((a - d) - root) / (2.0 * c);
    const double kp = std::abs(c * zp + d), km = std::abs(c * zm + d);
    *out = km > kp ? zm : zp;
    return finite(*out) ? KL_OK : KL_ESINGULAR;
}

static void inverse2(const cd m[4], cd out[4]) {
    const cd det = m[0] * m[3] - m[1] * m[2];
    out[0] = m[3] / det;
    out[1] = -m[1] / det;
    out[2] = -m[2] / det;
    out[3] = m[0] / det;
}

static void store_gens(const cd g[4][4], const cd fix[4], const bool inf[4], Gens* G) {
    G->inf_mask = 0;
    for (int k = 0; k < 4; ++k) {
        G->g[k].a = {g[k][0].real(), g[k][0].imag()};
        G->g[k].b = {g[k][1].real(), g[k][1].imag()};
        G->g[k].c = {g[k][2].real(), g[k][2].imag()};
        G->g[k].d = {g[k][3].real(), g[k][3].imag()};
        G->fix[k] = {fix[k].real(), fix[k].imag()};
        if (inf[k]) G->inf_mask |= 1u << k;
    }
}

// Trace recipe: tab solves tab^2 - ta tb tab + ta^2 + tb^2 = 0, root
// (ta tb + s)/2 with s in the closed upper half plane.  On a curve of
// traces, among them ta = tb = 2 (the double cusp), a comes out with c = 0,
// a translation whose seed (and A's) is infinity (inf[k]).
static int recipe(cd ta, cd tb, cd* tab_out, cd g[4][4], cd fix[4], bool inf[4]) {
    const cd i1(0.0, 1.0);
    const cd p = ta * tb;
    cd s = std::sqrt(p * p - 4.0 * (ta * ta + tb * tb));
    if (s.imag() < 0.0 || (s.imag() == 0.0 && s.real() < 0.0)) s = -s;
    const cd tab = (p + s) / 2.0;
    const cd q_den = tb * tab - 2.0 * ta + 2.0 * i1 * tab;
    const cd tp = 2.0 * tab + 4.0, tm = 2.0 * tab - 4.0;
    if (q_den == cd(0.0) || tp == cd(0.0) || tm == cd(0.0))
        return fail(KL_ESINGULAR, "trace recipe undefined for ta=(%g,%g) tb=(%g,%g)", ta.real(), ta.imag(),
                    tb.real(), tb.imag());
    const cd q = (tab - 2.0) * tb / q_den;
    if (q == cd(0.0)) return fail(KL_ESINGULAR, "trace recipe degenerate (tab = 2 or tb = 0)");
    const cd a[4] = {ta / 2.0, (ta * tab - 2.0 * tb + 4.0 * i1) / (tp * q),
                     (ta * tab - 2.0 * tb - 4.0 * i1) * q / tm, ta / 2.0};
    const cd b[4] = {(tb - 2.0 * i1) / 2.0, tb / 2.0, tb / 2.0, (tb + 2.0 * i1) / 2.0};
    for (int j = 0; j < 4; ++j) {
        g[0][j] = a[j];
        g[1][j] = b[j];
    }
    inverse2(a, g[2]);
    inverse2(b, g[3]);
    for (int k = 0; k < 4; ++k) {
        for (int j = 0; j < 4; ++j)
            if (!finite(g[k][j])) return fail(KL_ESINGULAR, "generator %d not finite", k);
        if (attracting_point(g[k], &fix[k], &inf[k]) != KL_OK)
            return fail(KL_ESINGULAR, "generator %d has no attracting fixed point", k);
    }
    *tab_out = tab;
    return KL_OK;
}

static int make_gens(kl_c64 ta, kl_c64 tb, Gens* G, cd* tab_out = nullptr) {
    cd g[4][4], fix[4], tab;
    bool inf[4];
    if (!std::isfinite(ta.re) || !std::isfinite(ta.im) || !std::isfinite(tb.re) || !std::isfinite(tb.im))
        return fail(KL_EINVAL, "traces must be finite");
    int rc = recipe(cd(ta.re, ta.im), cd(tb.re, tb.im), &tab, g, fix, inf);
    if (rc) return rc;
    store_gens(g, fix, inf, G);
    if (tab_out) *tab_out = tab;
    return KL_OK;
}

// Group of two explicit generators a = ab[0..3], b = ab[4..7] (row major),
// each scaled by 1/sqrt(det) to determinant 1, with A, B their inverses.
static int make_gens_ab(const kl_c64* ab, Gens* G) {
    if (!ab) return fail(KL_EINVAL, "generator array is NULL");
    cd g[4][4], fix[4];
    bool inf[4];
    for (int k = 0; k < 2; ++k) {
        for (int j = 0; j < 4; ++j) {
            g[k][j] = cd(ab[4 * k + j].re, ab[4 * k + j].im);
            if (!finite(g[k][j])) return fail(KL_EINVAL, "generator entries must be finite");
        }
        const cd det = g[k][0] * g[k][3] - g[k][1] * g[k][2];
        if (det == cd(0.0)) return fail(KL_ESINGULAR, "generator %c has determinant 0", k ? 'b' : 'a');
        const cd r = std::sqrt(det);
        for (int j = 0; j < 4; ++j) g[k][j] /= r;
    }
    inverse2(g[0], g[2]);
    inverse2(g[1], g[3]);
    for (int k = 0; k < 4; ++k) {
        for (int j = 0; j < 4; ++j)
            if (!finite(g[k][j])) return fail(KL_ESINGULAR, "generator %d not finite", k);
        if (attracting_point(g[k], &fix[k], &inf[k]) != KL_OK)
            return fail(KL_ESINGULAR, "generator %d has no attracting fixed point", k);
    }
    store_gens(g, fix, inf, G);
    return KL_OK;
}

// ------------------------------------------------------------------ window
static int check_window(const kl_window* w) {
    if (!w) return fail(KL_EINVAL, "window is NULL");
    if (!std::isfinite(w->x0) || !std::isfinite(w->x1) || !std::isfinite(w->y0) || !std::isfinite(w->y1))
        return fail(KL_EINVAL, "window bounds must be finite");
    if (!(w->x1 > w->x0) || !(w->y1 > w->y0)) return fail(KL_EINVAL, "window must have x1 > x0 and y1 > y0");
    if (w->width < 1 || w->height < 1 || w->width > 32768 || w->height > 32768 ||
        (uint64_t)w->width * w->height >= (1ull << 31))
        return fail(KL_EINVAL, "window size %ux%u outside 1..32768 per side, < 2^31 bins", w->width, w->height);
    return KL_OK;
}

static Fold make_fold(const kl_window* w, int head_form) {
    Fold f;
    f.head_form = head_form;
    if (!w) {
        f.s = 1.0;
        f.o = {0.0, 0.0};
        f.aniso = 1.0;
        return f;
    }
    const double sy = (double)w->height / (w->y1 - w->y0);
    const double sx = (double)w->width / (w->x1 - w->x0);
    f.s = sy;
    f.o = {-w->x0 * sy, -w->y0 * sy};
    f.aniso = sx / sy;
    return f;
}

// ------------------------------------------------------------------ devices
// Table buffer that single-set calls on a device's null stream reuse (Temp::tables).
struct TableCache {
    void* base = nullptr;
    size_t bytes = 0;
    bool busy = false;   // leased to a call that is still enqueuing its kernels
};

struct DeviceInfo {
    int cus = 0;
    void* scratch = nullptr;   // device address of this device's copy of `scratch` (kl_render_noalloc)
    TableCache tables;
    char arch[32] = {0};       // architecture name up to its first ':' (tuned-plan keys)
};
constexpr int kMaxDevices = 64;
static std::mutex g_dev_mutex;
static DeviceInfo g_devs[kMaxDevices];

int device_cu_count() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 256;
    std::lock_guard<std::mutex> lk(g_dev_mutex);
    if (g_devs[dev].cus == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        g_devs[dev].cus = cus;
    }
    return g_devs[dev].cus;
}

// ------------------------------------------------------------------ allocation-free scratch
// The tables of kl_render_noalloc: one array per device, held until the
// process ends.  Host code never uses the array's name as an address: the
// device address of the current device's copy comes from
// hipGetSymbolAddress, taken once per device on its first call.
static __device__ __align__(256) unsigned char scratch[KL_NOALLOC_SCRATCH_BYTES];

static int scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(KL_EDEVICE, "device %d beyond the %d the library tracks", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_dev_mutex);
    if (!g_devs[dev].scratch) {
        void* p = nullptr;
        if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess) return hip_fail(e, "scratch address");
        if (!p) return fail(KL_EDEVICE, "scratch array has no device address");
        g_devs[dev].scratch = p;
    }
    *out = g_devs[dev].scratch;
    return KL_OK;
}

// ------------------------------------------------------------------ planning
static const int kDefaultTail = 6;
static const int kDefaultWavesPerCU = 32;

int plan_split(int depth, int precision, int r_req, int m_req, Split* sp, PlanContext ctx) {
    const int prefix_cap = ctx == kPlanBatch ? 8 : ctx == kPlanTiling ? 6 : 9;
    int r;
    if (r_req > 0) {
        if (r_req > kMaxTail || r_req > depth) return fail(KL_EINVAL, "tail_len %d outside 1..min(8, depth)", r_req);
        // the persistent kernels hold the homogeneous suffix table in LDS,
        // 8 * 3^(r-1) points: in FP64 (16 B a point) r = 8 needs 280 KB,
        // more than a CU's 160 KB
        if (precision == KL_PREC_FP64 && r_req > kMaxTailFp64)
            return fail(KL_EINVAL, "tail_len %d exceeds %d in FP64 (LDS suffix table)", r_req, kMaxTailFp64);
        r = r_req;
    } else {
        r = depth <= 4 ? depth : std::min(kDefaultTail, depth - 1);
        // A render of one depth from 13 to 16 letters has few heads for
        // the persistent kernel's 8,192 waves with 6-letter tails (137
        // units of 64 heads at depth 14), so it takes shorter ones: 4
        // letters at depths 13-14, 5 at 15-16.  Measured, FP32, 6-letter
        // tails against these: 2048^2 image over [-1.5, 1.5]^2, 33 / 21,
        // 104 / 26, 101 / 47, 109 / 59 us at depths 13..16; 512^2 over
        // [-2, 2]^2, 34 / 19, 86 / 32, 88 / 42, 93 / 87 us.  Still shorter
        // tails lose there (depth 16 with 4 letters: 231 us), many more
        // heads flushing their runs into the same coarse bins; depths 17 and
        // up keep 6.  A batch of many sets fills the GPU with its sets and
        // keeps 6 letters, which its many small images favour; so do the
        // depths of a tiling, which go in one batched launch whose units
        // of 256 heads are dealt round robin: mixing 4- and 6-letter tails
        // there leaves units of unequal work (the tiling of Maskit's group
        // to depth 14 took 0.25 ms against 0.215 ms with 6 letters throughout).
        if (ctx == kPlanSingle && depth >= 13 && depth <= 16) r = depth <= 14 ? 4 : 5;
        // the deepest words need a longer tail: k <= 14 and m <= 20
        r = std::max(r, std::min(kMaxTail, depth - kMaxLane - kMaxPrefix));
    }
    const int h = depth - r;
    int m, k;
    if (h == 0) {
        if (m_req > 0) return fail(KL_EINVAL, "lane_len %d needs a head (tail_len < depth)", m_req);
        m = 0;
        k = 0;
    } else {
        if (m_req > 0) {
            if (m_req > kMaxLane || m_req > h - 1) return fail(KL_EINVAL, "lane_len %d outside 1..min(20, %d)", m_req, h - 1);
            m = m_req;
        } else {
            m = std::min(std::max(h - prefix_cap, std::min(2, h - 1)), kMaxLane);
        }
        k = h - m;
        if (k > kMaxPrefix) return fail(KL_EINVAL, "prefix table depth %d exceeds %d", k, kMaxPrefix);
        if (m > kMaxLane) return fail(KL_EINVAL, "lane_len %d exceeds %d", m, kMaxLane);
    }
    sp->depth = depth;
    sp->r = r;
    sp->m = m;
    sp->k = k;
    sp->pow3_m = (uint32_t)pow3_u64(m);
    sp->R1 = (uint32_t)pow3_u64(r - 1);
    sp->R = pow3_u64(r);
    sp->n_heads = (k + m == 0) ? 1 : num_words(k + m);
    return KL_OK;
}

// ------------------------------------------------------------------ temporaries
// Largest table set that the per-device table cache holds.
constexpr size_t kTableCacheMax = size_t(64) << 20;

// Stream-ordered temporaries of one call, freed on its stream when the call
// returns.  tables() lends the call its device's cached table buffer instead
// when the call runs on the null stream: every user of that buffer enqueues
// on the null stream, which lives as long as the process, so the set-up
// kernel that rewrites the tables runs after every kernel that read them
// before, and the steady state of repeated renders enqueues no allocation
// (a hipMallocAsync / hipFreeAsync pair costs the GPU some 3 us of idle
// time per call).  The lease ends with the call, once its kernels are
// enqueued; a call that finds the buffer leased to another thread, or that
// runs on another stream, or that needs more than kTableCacheMax bytes,
// takes a temporary.
struct Temp {
    hipStream_t s;
    std::vector<void*> ptrs;
    int lease = -1;   // device whose table cache this call holds
    explicit Temp(hipStream_t st) : s(st) {}
    hipError_t alloc(void** p, size_t bytes) {
        *p = nullptr;
        if (bytes == 0) bytes = 16;
        hipError_t e = hipMallocAsync(p, bytes, s);
        if (e == hipSuccess) ptrs.push_back(*p);
        return e;
    }
    hipError_t tables(void** p, size_t bytes) {
        int dev = -1;
        if (s == nullptr && lease < 0 && bytes <= kTableCacheMax && hipGetDevice(&dev) == hipSuccess && dev >= 0 &&
            dev < kMaxDevices) {
            std::lock_guard<std::mutex> lk(g_dev_mutex);
            TableCache& c = g_devs[dev].tables;
            if (!c.busy) {
                if (c.bytes < bytes) {
                    if (c.base) (void)hipFreeAsync(c.base, s);
                    c.base = nullptr;
                    c.bytes = 0;
                    const size_t want = std::max(bytes, size_t(1) << 20);
                    if (hipMallocAsync(&c.base, want, s) == hipSuccess) {
                        c.bytes = want;
                    } else {
                        // a temporary of the exact size may still fit; clear the
                        // error so that the next launch check does not report it
                        c.base = nullptr;
                        (void)hipGetLastError();
                    }
                }
                if (c.base) {
                    c.busy = true;
                    lease = dev;
                    *p = c.base;
                    return hipSuccess;
                }
            }
        }
        return alloc(p, bytes);
    }
    ~Temp() {
        for (void* p : ptrs) (void)hipFreeAsync(p, s);
        if (lease >= 0) {
            std::lock_guard<std::mutex> lk(g_dev_mutex);
            g_devs[lease].tables.busy = false;
        }
    }
};

// Device tables of one parameter set for one split, in one temporary
// allocation, built by the fused set-up kernel (which also clears the image
// and the dropped counter when asked to).
struct SetTables {
    Tables tab{};
    const void* tail_homog = nullptr;
};

static size_t round16(size_t x) { return (x + 15) & ~size_t(15); }

// Layout of one set's tables in one buffer.
struct TableLayout {
    uint64_t np, nt;
    size_t off_last, off_aff, off_hom, off_flags, total;
    uint32_t n_flags;
};

static TableLayout table_layout(const Split& sp, int precision) {
    TableLayout L;
    L.np = sp.k ? num_words(sp.k) : 0;
    L.nt = num_words(sp.r);
    const size_t esz = precision == KL_PREC_FP64 ? sizeof(c64) : sizeof(c32);
    L.off_last = round16(L.np * sizeof(m64));
    L.off_aff = L.off_last + round16(L.np);
    L.off_hom = L.off_aff + round16(L.nt * esz + 16);
    L.off_flags = L.off_hom + round16(2 * L.nt * esz + 16);
    L.n_flags = (uint32_t)((L.nt + 255) / 256);  // one per set-up block of suffix points
    L.total = L.off_flags + round16(L.n_flags * sizeof(uint32_t));
    return L;
}

// A caller-provided table buffer (kl_render_noalloc): base and capacity.
struct TableBuf {
    unsigned char* base = nullptr;
    size_t bytes = 0;
};

static int build_tables(const Gens& G, const Split& sp, int precision, int force_homog, int seed, Temp& tmp,
                        SetTables* out, uint32_t* clear_image = nullptr, uint64_t bins = 0,
                        uint64_t* clear_dropped = nullptr, const TableBuf* buf = nullptr) {
    const TableLayout L = table_layout(sp, precision);
    const uint64_t np = L.np;
    const size_t off_last = L.off_last, off_aff = L.off_aff, off_hom = L.off_hom, off_flags = L.off_flags;
    const uint32_t n_flags = L.n_flags;
    unsigned char* base = nullptr;
    hipError_t e = hipSuccess;
    if (buf) {
        if (L.total > buf->bytes)
            return fail(KL_ENOMEM, "tables of %zu bytes exceed the %zu-byte scratch array", L.total, buf->bytes);
        base = buf->base;
    } else if ((e = tmp.tables((void**)&base, L.total)) != hipSuccess) {
        return hip_fail(e, "tables");
    }
    SetupJob j{};
    j.gens = G;
    j.precision = precision;
    j.k = sp.k;
    j.r = sp.r;
    j.force_homog = force_homog;
    j.seed = seed;
    j.prefix = np ? (m64*)base : nullptr;
    j.last = np ? base + off_last : nullptr;
    j.aff = base + off_aff;
    j.hom = base + off_hom;
    j.flags = (uint32_t*)(base + off_flags);
    j.image = clear_image;
    j.bins = bins;
    j.dropped = clear_dropped;
    if ((e = launch_setup(j, tmp.s)) != hipSuccess) return hip_fail(e, "set-up kernel");
    out->tab.prefix = j.prefix;
    out->tab.prefix_last = j.last;
    out->tab.tail = j.aff;
    out->tab.tail_flags = j.flags;
    out->tab.n_flags = n_flags;
    out->tail_homog = j.hom;
    return KL_OK;
}

static int grid_for(int waves_per_cu) {
    if (waves_per_cu <= 0) waves_per_cu = kDefaultWavesPerCU;
    return std::max(1, device_cu_count() * waves_per_cu / (kBlock / kWave));
}

static bool persistent_ok(const Split& sp) { return sp.k + sp.m > 0 && sp.r >= 3 && sp.n_heads >= (uint64_t)kWave; }

// Units of 64 heads below which a launch leaves the persistent kernel for the
// per-word kernel.  With u units only u waves walk 3^r words each, one after
// another (a unit of 729 words takes some 30 us at one wave per SIMD), while
// the per-word kernel spreads the same words one per thread; the two break
// even near a hundred units.  Both compute every word the same way.
constexpr uint64_t kMinPersistentUnits = 128;

// ------------------------------------------------------------------ tuned plans
// Plans chosen by the autotuners, in two contexts:
//   single (kl_autotune): renders and evaluations of one depth, keyed by
//     (device architecture, depth, precision) -- the split decides the
//     arithmetic of every word, so kl_eval (which may have no window) and
//     every render of that depth and precision share it;
//   batch (kl_autotune_many): the sets of batched renders, keyed by
//     (architecture, depth, image width and height, precision).
// KL_AUTOTUNE_CACHE names a text file of lines
//   "arch context depth precision width height tail_len lane_len
//    waves_per_cu hist_mode ms"
// (context 0 single with width = height = 0, 1 batch; arch "*" matches any
// device) read at the first lookup and appended to by the tuners.
enum { kTuneSingle = 0, kTuneBatch = 1 };
struct Tuned {
    char arch[32];
    int ctx, depth, precision;
    uint32_t W, H;
    int r, m, wpc, hist;
    double ms;
};
static std::mutex g_tune_mutex;
static std::vector<Tuned> g_tuned;
static bool g_tune_loaded = false;

// "gfx950" for the current device (up to the first ':' of its architecture
// name), "none" without one
static void device_arch(char* out, size_t n) {
    snprintf(out, n, "none");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return;
    std::lock_guard<std::mutex> lk(g_dev_mutex);
    if (!g_devs[dev].arch[0]) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return;
        size_t i = 0;
        for (; i + 1 < sizeof g_devs[dev].arch && prop.gcnArchName[i] && prop.gcnArchName[i] != ':'; ++i)
            g_devs[dev].arch[i] = prop.gcnArchName[i];
        g_devs[dev].arch[i] = 0;
    }
    snprintf(out, n, "%s", g_devs[dev].arch);
}

static bool same_key(const Tuned& a, const Tuned& b) {
    return strcmp(a.arch, b.arch) == 0 && a.ctx == b.ctx && a.depth == b.depth && a.precision == b.precision &&
           a.W == b.W && a.H == b.H;
}

static void put_tuned_locked(const Tuned& t) {
    auto it = std::find_if(g_tuned.begin(), g_tuned.end(), [&](const Tuned& x) { return same_key(x, t); });
    if (it != g_tuned.end()) *it = t;
    else g_tuned.push_back(t);
}

static void load_tuned_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = getenv("KL_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    char line[256];
    while (fgets(line, sizeof line, f)) {
        Tuned t;
        Split sp;
        // a line is kept only if the planner accepts its split: a stale or
        // foreign line must not make every render of its depth fail
        if (sscanf(line, "%31s %d %d %d %u %u %d %d %d %d %lf", t.arch, &t.ctx, &t.depth, &t.precision, &t.W,
                   &t.H, &t.r, &t.m, &t.wpc, &t.hist, &t.ms) == 11 &&
            (t.ctx == kTuneSingle || t.ctx == kTuneBatch) && t.hist >= KL_HIST_AUTO && t.hist <= KL_HIST_LDS &&
            (t.precision == KL_PREC_FP32 || t.precision == KL_PREC_FP64) &&
            t.depth >= 1 && t.depth <= KL_MAX_DEPTH && t.r >= 1 && t.r <= kMaxTail && t.r < t.depth && t.m >= 0 &&
            t.m <= kMaxLane && t.wpc >= 0 && t.wpc <= 32 && t.W <= 32768 && t.H <= 32768 &&
            plan_split(t.depth, t.precision, t.r, t.m, &sp, t.ctx == kTuneBatch ? kPlanBatch : kPlanSingle) == KL_OK)
            put_tuned_locked(t);
    }
    fclose(f);
}

// The tuned plan of a context, depth, image size (batch only) and precision
// on the current device.
static bool find_tuned(int ctx, int depth, int precision, const kl_window* w, Tuned* out) {
    Tuned key{};
    device_arch(key.arch, sizeof key.arch);
    key.ctx = ctx;
    key.depth = depth;
    key.precision = precision;
    if (ctx == kTuneBatch) {
        if (!w) return false;
        key.W = w->width;
        key.H = w->height;
    }
    std::lock_guard<std::mutex> lk(g_tune_mutex);
    load_tuned_locked();
    for (int pass = 0; pass < 2; ++pass)   // this device's architecture, then "*"
        for (const Tuned& t : g_tuned) {
            Tuned k2 = key;
            if (pass) snprintf(k2.arch, sizeof k2.arch, "*");
            if (same_key(t, k2)) {
                *out = t;
                return true;
            }
        }
    return false;
}

static void store_tuned(const Tuned& t) {
    std::lock_guard<std::mutex> lk(g_tune_mutex);
    load_tuned_locked();
    put_tuned_locked(t);
    const char* path = getenv("KL_AUTOTUNE_CACHE");
    if (path && *path) {
        FILE* f = fopen(path, "a");
        if (f) {
            fprintf(f, "%s %d %d %d %u %u %d %d %d %d %.6f\n", t.arch, t.ctx, t.depth, t.precision, t.W, t.H, t.r,
                    t.m, t.wpc, t.hist, t.ms);
            fclose(f);
        }
    }
}

// Seed of every word for the suffix tables: -1 (each word's own) or a generator.
static int seed_index(const kl_opts& o) { return o.seed_mode >= KL_SEED_A ? o.seed_mode - KL_SEED_A : -1; }

// Options with the tuned plan filled in where the caller left the planner's
// choice: the single-render plan, or with `batch` the batched one.
static kl_opts apply_tuned(const kl_opts& o, int depth, const kl_window* w, bool batch = false) {
    kl_opts r = o;
    Tuned t;
    if (o.tail_len == 0 && o.lane_len == 0 && find_tuned(batch ? kTuneBatch : kTuneSingle, depth, o.precision, w, &t)) {
        r.tail_len = t.r;
        r.lane_len = t.m;
        if (r.waves_per_cu == 0) r.waves_per_cu = t.wpc;
        if (r.hist_mode == KL_HIST_AUTO) r.hist_mode = t.hist;
    }
    return r;
}

// Render the words [lo, hi) of one depth; with `clear`, the set-up kernel
// also clears the image and the dropped counter first.
static int render_depth(const Gens& G, const Fold& f, int depth, uint64_t lo, uint64_t hi, const kl_opts& o_in,
                        const kl_window* w, uint32_t* image, uint64_t* dropped, hipStream_t s, bool clear,
                        const TableBuf* buf = nullptr, PlanContext ctx = kPlanSingle) {
    if (lo >= hi && !clear) return KL_OK;
    const kl_opts o = apply_tuned(o_in, depth, w);
    Split sp;
    int rc = plan_split(depth, o.precision, o.tail_len, o.lane_len, &sp, ctx);
    if (rc) return rc;
    Temp tmp(s);
    SetTables st;
    const uint64_t bins = (uint64_t)w->width * w->height;
    if ((rc = build_tables(G, sp, o.precision, o.suffix_form, seed_index(o), tmp, &st, clear ? image : nullptr, bins,
                           clear ? dropped : nullptr, buf)))
        return rc;
    if (lo >= hi) return KL_OK;
    RenderJob job{};
    job.sp = sp;
    job.precision = o.precision;
    job.gens = G;
    job.fold = f;
    job.tab = st.tab;
    job.tail_homog = st.tail_homog;
    job.image = image;
    job.width = w->width;
    job.height = w->height;
    job.dropped = dropped;
    job.hist_mode = o.hist_mode;
    job.grid_blocks = grid_for(o.waves_per_cu);
    job.bounded = o.block_bounds && sp.r >= 4 && o.hist_mode != KL_HIST_LDS;
    uint64_t rag_lo = lo, rag_hi = hi;  // default: every word by the per-word kernel
    if (persistent_ok(sp)) {
        // whole heads inside [lo, hi) go to the persistent kernel, when they fill enough units
        const uint64_t hb = (lo + sp.R - 1) / sp.R, he = hi / sp.R;
        if (he > hb && he - hb >= kMinPersistentUnits * kWave) {
            if (o.kernel_events[0]) (void)hipEventRecord((hipEvent_t)o.kernel_events[0], s);
            const uint64_t max_heads = (uint64_t)kWave << 30;
            for (uint64_t h0 = hb; h0 < he;) {
                const uint64_t nh = std::min(he - h0, max_heads);
                RenderJob part = job;
                part.head_begin = h0;
                part.n_heads = nh;
                part.n_units = (uint32_t)((nh + kWave - 1) / kWave);
                hipError_t e = launch_render(part, s);
                if (e != hipSuccess) return hip_fail(e, "render kernel");
                h0 += nh;
            }
            if (o.kernel_events[1]) (void)hipEventRecord((hipEvent_t)o.kernel_events[1], s);
            rag_hi = hb * sp.R;
            job.rag_first[1] = he * sp.R;
            job.rag_count[1] = hi - he * sp.R;
        }
    }
    job.n_units = 0;
    job.rag_first[0] = rag_lo;
    job.rag_count[0] = rag_hi - rag_lo;
    if (job.rag_count[0] + job.rag_count[1] > 0) {
        hipError_t e = launch_render(job, s);
        if (e != hipSuccess) return hip_fail(e, "per-word kernel");
    }
    return KL_OK;
}

// max_seed_mode: KL_SEED_INV_B for the four letters; a Cayley table names
// up to eight symbols, KL_SEED_A + 7.
static int check_opts_common(const kl_opts& o, int max_seed_mode = KL_SEED_INV_B) {
    if (o.precision != KL_PREC_FP32 && o.precision != KL_PREC_FP64)
        return fail(KL_EINVAL, "precision %d is neither KL_PREC_FP32 nor KL_PREC_FP64", o.precision);
    if (o.tail_len < 0 || o.tail_len > kMaxTail) return fail(KL_EINVAL, "tail_len %d outside 0..8", o.tail_len);
    if (o.lane_len < 0 || o.lane_len > kMaxLane) return fail(KL_EINVAL, "lane_len %d outside 0..20", o.lane_len);
    if (o.hist_mode < KL_HIST_AUTO || o.hist_mode > KL_HIST_LDS) return fail(KL_EINVAL, "hist_mode %d", o.hist_mode);
    if (o.waves_per_cu < 0 || o.waves_per_cu > 32) return fail(KL_EINVAL, "waves_per_cu %d outside 0..32", o.waves_per_cu);
    if (o.head_form < 0 || o.head_form > 2) return fail(KL_EINVAL, "head_form %d outside 0..2", o.head_form);
    if (o.seed_mode < KL_SEED_OWN || o.seed_mode > max_seed_mode)
        return fail(KL_EINVAL, "seed_mode %d outside 0..%d", o.seed_mode, max_seed_mode);
    if (o.block_bounds != 0 && o.block_bounds != 1)
        return fail(KL_EINVAL, "block_bounds %d is neither 0 nor 1", o.block_bounds);
    return KL_OK;
}

// The tail_len / lane_len overrides apply to the depths that can take them;
// shallower depths of a tiling render use the planner.
static kl_opts opts_for_depth(const kl_opts& o, int d) {
    kl_opts od = o;
    if (od.tail_len >= d || (od.lane_len > 0 && od.lane_len > d - (od.tail_len ? od.tail_len : 1) - 1)) {
        od.tail_len = 0;
        od.lane_len = 0;
    }
    return od;
}

static kl_opts default_opts() {
    kl_opts o;
    memset(&o, 0, sizeof o);
    return o;
}

}  // namespace kl

using namespace kl;

// ====================================================================== C ABI
extern "C" {

uint64_t kl_num_words(int depth) { return num_words(depth); }

const char* kl_strerror(int code) {
    switch (code) {
        case KL_OK: return "success";
        case KL_EINVAL: return "invalid argument";
        case KL_ERANGE: return "index range beyond the words of the requested depth";
        case KL_ESINGULAR: return "singular parameters: generators or seeds undefined";
        case KL_EDEVICE: return "HIP device error";
        case KL_ENOMEM: return "out of device memory";
        default: return "unknown error";
    }
}

const char* kl_last_error(void) { return g_last_error.c_str(); }

int kl_generators(kl_c64 ta, kl_c64 tb, kl_c64* tab_out, kl_c64* gens_out, kl_c64* fix_out) {
    Gens G;
    cd tab;
    int rc = make_gens(ta, tb, &G, &tab);
    if (rc) return rc;
    if (tab_out) *tab_out = {tab.real(), tab.imag()};
    if (gens_out)
        for (int k = 0; k < 4; ++k) {
            gens_out[4 * k + 0] = {G.g[k].a.re, G.g[k].a.im};
            gens_out[4 * k + 1] = {G.g[k].b.re, G.g[k].b.im};
            gens_out[4 * k + 2] = {G.g[k].c.re, G.g[k].c.im};
            gens_out[4 * k + 3] = {G.g[k].d.re, G.g[k].d.im};
        }
    if (fix_out)
        for (int k = 0; k < 4; ++k)
            fix_out[k] = (G.inf_mask >> k) & 1u ? kl_c64{HUGE_VAL, 0.0} : kl_c64{G.fix[k].re, G.fix[k].im};
    return KL_OK;
}

int kl_decode_ex(uint64_t first_idx, uint64_t count, int depth, uint8_t* letters_out, void* stream) {
    if (depth < 1 || depth > KL_MAX_DEPTH) return fail(KL_EINVAL, "depth %d outside 1..40", depth);
    if (count == 0) return KL_OK;
    if (!letters_out) return fail(KL_EINVAL, "letters_out is NULL");
    const uint64_t n = num_words(depth);
    if (first_idx > n || count > n - first_idx)
        return fail(KL_ERANGE, "indices [%llu, %llu + %llu) exceed the %llu words of depth %d",
                    (unsigned long long)first_idx, (unsigned long long)first_idx, (unsigned long long)count,
                    (unsigned long long)n, depth);
    hipError_t e = launch_decode(first_idx, count, depth, letters_out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "decode kernel");
    return KL_OK;
}

int kl_decode(uint64_t first_idx, uint64_t count, int depth, uint8_t* letters_out) {
    int rc = kl_decode_ex(first_idx, count, depth, letters_out, nullptr);
    if (rc || count == 0) return rc;
    hipError_t e = hipStreamSynchronize(nullptr);
    return e == hipSuccess ? KL_OK : hip_fail(e, "decode");
}

int kl_plan(int depth, int precision, const kl_window* window, const kl_opts* opts, kl_plan_t* plan_out) {
    (void)window;
    if (depth < 1 || depth > KL_MAX_DEPTH) return fail(KL_EINVAL, "depth %d outside 1..40", depth);
    if (!plan_out) return fail(KL_EINVAL, "plan_out is NULL");
    kl_opts o = opts ? *opts : default_opts();
    o.precision = precision;
    int rc = check_opts_common(o);
    if (rc) return rc;
    o = apply_tuned(o, depth, window);
    Split sp;
    if ((rc = plan_split(depth, precision, o.tail_len, o.lane_len, &sp))) return rc;
    plan_out->depth = depth;
    plan_out->tail_len = sp.r;
    plan_out->lane_len = sp.m;
    plan_out->prefix_len = sp.k;
    plan_out->hist_mode = o.hist_mode ? o.hist_mode : KL_HIST_RUNS;
    (void)window;
    plan_out->waves_per_cu = o.waves_per_cu ? o.waves_per_cu : kDefaultWavesPerCU;
    return KL_OK;
}

}  // extern "C"

namespace kl {

// Index space of a render: words [first, first + count) of depths min_depth..depth.
struct RenderSpan {
    int min_depth;
    uint64_t first, count;
};

// Every check of a render that needs no group; nothing is enqueued.
static int check_render(int depth, const kl_window* window, const uint32_t* image_out, const kl_opts& o,
                        RenderSpan* span) {
    if (depth < 1 || depth > KL_MAX_DEPTH) return fail(KL_EINVAL, "depth %d outside 1..40", depth);
    int rc = check_window(window);
    if (rc) return rc;
    if (!image_out) return fail(KL_EINVAL, "image_out is NULL");
    if ((rc = check_opts_common(o))) return rc;
    const int min_depth = o.min_depth == 0 ? depth : o.min_depth;
    if (min_depth < 1 || min_depth > depth) return fail(KL_EINVAL, "min_depth %d outside 1..%d", o.min_depth, depth);
    uint64_t total = 0;
    for (int d = min_depth; d <= depth; ++d) {
        const uint64_t n = num_words(d);
        if (total > UINT64_MAX - n) return fail(KL_ERANGE, "index space of depths %d..%d exceeds 2^64", min_depth, depth);
        total += n;
    }
    uint64_t first = 0, count = total;
    if (o.use_range) {
        first = o.first_idx;
        count = o.count;
        if (first > total || count > total - first)
            return fail(KL_ERANGE, "range [%llu, +%llu) exceeds the %llu words", (unsigned long long)first,
                        (unsigned long long)count, (unsigned long long)total);
    }
    // every split must be plannable before anything is enqueued
    for (int d = min_depth; d <= depth; ++d) {
        Split sp;
        const kl_opts od = d == depth ? o : opts_for_depth(o, d);
        if ((rc = plan_split(d, od.precision, od.tail_len, od.lane_len, &sp,
                             min_depth < depth ? kPlanTiling : kPlanSingle)))
            return rc;
    }
    *span = {min_depth, first, count};
    return KL_OK;
}

// One set of a batched render: its generators, split, seed and outputs.
struct SetSpec {
    Gens gens;
    Split sp;
    int seed;
    uint32_t* image;
    uint64_t* dropped;
};

// Many sets in a few launches: one table launch builds every set's prefix
// and suffix tables, one persistent launch renders the sets the persistent
// kernel takes (whole heads), one per-word launch renders the rest.  Sets
// may share an image and a dropped counter.  Every word is evaluated with
// its set's split and tables, bit for bit as a single render of that set.
// The descriptors are uploaded from host memory; the call waits for those
// copies (not for the renders) before it returns.
static int render_sets(const std::vector<SetSpec>& specs, const kl_window* w, const kl_opts& o, int wpc,
                       hipStream_t s) {
    const int nb = (int)specs.size();
    if (nb == 0) return KL_OK;
    const size_t esz = o.precision == KL_PREC_FP64 ? sizeof(c64) : sizeof(c32);
    uint64_t n_prefix = 0, n_tail = 0;
    uint32_t max_prefix = 0, max_tail = 0;
    for (const SetSpec& q : specs) {
        const uint32_t np = q.sp.k ? (uint32_t)num_words(q.sp.k) : 0;
        const uint32_t nt = (uint32_t)num_words(q.sp.r);
        n_prefix += np;
        n_tail += nt;
        max_prefix = std::max(max_prefix, np);
        max_tail = std::max(max_tail, nt);
    }
    // every temporary in one allocation: the descriptors (uploaded together)
    // then the tables
    std::vector<SetDesc> h_sets(nb), h_psets;
    std::vector<uint64_t> h_off(1, 0), h_woff(1, 0);
    std::vector<int> h_ids;
    // the persistent kernel takes the deep sets when together they fill enough units
    uint64_t units = 0;
    for (int j = 0; j < nb; ++j)
        if (persistent_ok(specs[j].sp)) units += (specs[j].sp.n_heads + kWave - 1) / kWave;
    const bool persist = units >= kMinPersistentUnits;
    auto persistent = [&](const Split& sp) { return persist && persistent_ok(sp); };
    for (int j = 0; j < nb; ++j) {
        if (persistent(specs[j].sp)) {
            h_off.push_back(h_off.back() + (specs[j].sp.n_heads + kBlock - 1) / kBlock);  // block units: one head per thread
        } else {
            h_ids.push_back(j);
            h_woff.push_back(h_woff.back() + num_words(specs[j].sp.depth));
        }
    }
    const int np_sets = (int)h_off.size() - 1, nw_sets = (int)h_ids.size();
    size_t off = 0;
    auto place = [&](size_t bytes) {
        const size_t at = off;
        off += round16(bytes);
        return at;
    };
    const size_t o_sets = place(nb * sizeof(SetDesc)), o_psets = place(np_sets * sizeof(SetDesc));
    const size_t o_off = place(h_off.size() * sizeof(uint64_t)), o_woff = place(h_woff.size() * sizeof(uint64_t));
    const size_t o_ids = place(nw_sets * sizeof(int)), o_flags = place(nb * sizeof(uint32_t));
    const size_t upload = off;
    const size_t o_prefix = place(n_prefix * sizeof(m64)), o_last = place(n_prefix + 16);
    const size_t o_aff = place(n_tail * esz + 16 * nb), o_hom = place(2 * n_tail * esz + 16 * nb);
    Temp tmp(s);
    unsigned char* base = nullptr;
    hipError_t e;
    if ((e = tmp.alloc((void**)&base, off)) != hipSuccess) return hip_fail(e, "batch temporaries");
    SetDesc* d_sets = (SetDesc*)(base + o_sets);
    SetDesc* d_psets = (SetDesc*)(base + o_psets);
    uint64_t* d_off = (uint64_t*)(base + o_off);
    uint64_t* d_woff = (uint64_t*)(base + o_woff);
    int* d_ids = (int*)(base + o_ids);
    uint32_t* d_flags = (uint32_t*)(base + o_flags);
    m64* d_prefix = (m64*)(base + o_prefix);
    uint8_t* d_last = base + o_last;
    unsigned char* d_aff = base + o_aff;
    unsigned char* d_hom = base + o_hom;
    uint64_t po = 0, to_aff = 0, to_hom = 0;
    uint32_t max_bytes = 0;
    for (int j = 0; j < nb; ++j) {
        const SetSpec& q = specs[j];
        SetDesc& D = h_sets[j];
        memset(&D, 0, sizeof D);
        D.gens = q.gens;
        D.sp = q.sp;
        D.seed = q.seed;
        D.n_prefix = q.sp.k ? (uint32_t)num_words(q.sp.k) : 0;
        D.n_tail = (uint32_t)num_words(q.sp.r);
        D.tab.prefix = d_prefix + po;
        D.tab.prefix_last = d_last + po;
        D.tab.tail = d_aff + to_aff;
        D.tail_homog = d_hom + to_hom;
        D.tab.tail_flags = d_flags + j;
        D.tab.n_flags = 1;
        D.image = q.image;
        D.dropped = q.dropped;
        po += D.n_prefix;
        to_aff += ((D.n_tail * esz + 15) / 16) * 16;
        to_hom += ((2 * D.n_tail * esz + 15) / 16) * 16;
        if (persistent(q.sp)) {
            max_bytes = std::max<uint32_t>(max_bytes, (uint32_t)(((2 * D.n_tail * esz + 15) / 16) * 16));
            h_psets.push_back(D);
        }
    }
    std::vector<unsigned char> blob(upload, 0);   // the form flags start at zero
    memcpy(blob.data() + o_sets, h_sets.data(), nb * sizeof(SetDesc));
    if (np_sets) memcpy(blob.data() + o_psets, h_psets.data(), np_sets * sizeof(SetDesc));
    memcpy(blob.data() + o_off, h_off.data(), h_off.size() * sizeof(uint64_t));
    memcpy(blob.data() + o_woff, h_woff.data(), h_woff.size() * sizeof(uint64_t));
    if (nw_sets) memcpy(blob.data() + o_ids, h_ids.data(), nw_sets * sizeof(int));
    if ((e = hipMemcpyAsync(base, blob.data(), upload, hipMemcpyHostToDevice, s)) != hipSuccess)
        return hip_fail(e, "batch descriptors");
    hipEvent_t copied;
    if ((e = hipEventCreateWithFlags(&copied, hipEventDisableTiming)) != hipSuccess) return hip_fail(e, "event");
    e = hipEventRecord(copied, s);
    int rc = KL_OK;
    BatchJob job{};
    job.sets = d_sets;
    job.n_sets = nb;
    job.precision = o.precision;
    job.fold = make_fold(w, o.head_form);
    job.width = w->width;
    job.height = w->height;
    job.grid_blocks = grid_for(wpc);
    job.max_prefix = max_prefix;
    job.max_tail = max_tail;
    job.force_homog = o.suffix_form;
    job.count_dropped = o.dropped_out != nullptr;
    job.bounded = o.block_bounds;
    if (e == hipSuccess) e = launch_batch_tables(job, s);
    if (e == hipSuccess && np_sets) {
        BatchJob pj = job;
        pj.sets = d_psets;
        pj.n_sets = np_sets;
        pj.unit_offsets = d_off;
        pj.total_units = h_off.back();
        pj.table_bytes = max_bytes;
        e = launch_render_batch(pj, s);
    }
    if (e == hipSuccess && nw_sets) {
        PerWordBatchJob wj{};
        wj.sets = d_sets;
        wj.word_offsets = d_woff;
        wj.set_ids = d_ids;
        wj.n = nw_sets;
        wj.total = h_woff.back();
        wj.precision = o.precision;
        wj.fold = job.fold;
        wj.width = w->width;
        wj.height = w->height;
        e = launch_perword_batch(wj, s);
    }
    if (e != hipSuccess) rc = hip_fail(e, "batch render");
    // the descriptors live in host vectors: wait for their copies before they go
    const hipError_t e2 = hipEventSynchronize(copied);
    (void)hipEventDestroy(copied);
    if (rc == KL_OK && e2 != hipSuccess) rc = hip_fail(e2, "batch descriptors");
    return rc;
}

// A tiling render of its whole index space: every depth of every seed is one
// set of a batched render into the one image, each set planned as a single
// render of its depth would be, so the image is the same.
static int render_tiling(const Gens& G, int depth, const kl_window* w, uint32_t* image, const kl_opts& o,
                         int min_depth) {
    hipStream_t s = (hipStream_t)o.stream;
    std::vector<int> seeds;
    if (o.seed_mode == KL_SEED_ALL) seeds = {0, 1, 2, 3};
    else seeds = {seed_index(o)};
    std::vector<SetSpec> specs;
    int wpc = o.waves_per_cu;
    for (int sd : seeds)
        for (int d = min_depth; d <= depth; ++d) {
            const kl_opts od = apply_tuned(d == depth ? o : opts_for_depth(o, d), d, w);
            Split sp;
            int rc = plan_split(d, od.precision, od.tail_len, od.lane_len, &sp, kPlanTiling);
            if (rc) return rc;
            if (!wpc && d == depth) wpc = od.waves_per_cu;
            specs.push_back({G, sp, sd, image, o.dropped_out});
        }
    if (!o.accumulate) {
        hipError_t e;
        if ((e = launch_fill_u32(image, (uint64_t)w->width * w->height, 0, s)) != hipSuccess)
            return hip_fail(e, "clear image");
        if (o.dropped_out && (e = launch_fill_u64(o.dropped_out, 1, 0, s)) != hipSuccess)
            return hip_fail(e, "clear dropped");
    }
    return render_sets(specs, w, o, wpc, s);
}

// The render itself, once every argument has been checked.  KL_SEED_ALL is
// four renders of the same words, one per generator's fixed point (the
// paper's index-search loop), accumulated.
static int render_run(const Gens& G, int depth, const kl_window* window, uint32_t* image_out, const kl_opts& o,
                      const RenderSpan& span, const TableBuf* buf = nullptr) {
    int rc;
    if (!buf && span.min_depth < depth && !o.kernel_events[0] && !o.kernel_events[1]) {
        uint64_t total = 0;
        for (int d = span.min_depth; d <= depth; ++d) total += num_words(d);
        if (span.first == 0 && span.count == total) return render_tiling(G, depth, window, image_out, o, span.min_depth);
    }
    if (o.seed_mode == KL_SEED_ALL) {
        for (int q = 0; q < 4; ++q) {
            kl_opts oq = o;
            oq.seed_mode = KL_SEED_A + q;
            oq.accumulate = o.accumulate || q > 0;
            if ((rc = render_run(G, depth, window, image_out, oq, span, buf))) return rc;
        }
        return KL_OK;
    }
    const Fold f = make_fold(window, o.head_form);
    hipStream_t s = (hipStream_t)o.stream;
    bool clear = !o.accumulate;
    uint64_t offset = 0;
    const uint64_t first = span.first, end = span.first + span.count;
    for (int d = span.min_depth; d <= depth; ++d) {
        const uint64_t n = num_words(d);
        const uint64_t lo = first > offset ? first - offset : 0;
        const uint64_t hi = end - offset < n ? end - offset : n;
        if ((end > offset && first < offset + n && lo < hi) || (clear && d == depth)) {
            const kl_opts od = d == depth ? o : opts_for_depth(o, d);
            const bool any = end > offset && first < offset + n && lo < hi;
            if ((rc = render_depth(G, f, d, any ? lo : 0, any ? hi : 0, od, window, image_out, o.dropped_out, s,
                                   clear, buf, span.min_depth < depth ? kPlanTiling : kPlanSingle)))
                return rc;
            clear = false;
        }
        offset += n;
    }
    return KL_OK;
}

// Every check of an evaluation that needs no group.
static int check_eval(int depth, const uint64_t* idx, uint64_t n, const kl_window* window, const kl_c64* z_out,
                      const kl_opts& o, Split* sp) {
    if (depth < 1 || depth > KL_MAX_DEPTH) return fail(KL_EINVAL, "depth %d outside 1..40", depth);
    int rc = check_opts_common(o);
    if (rc) return rc;
    if (o.seed_mode == KL_SEED_ALL) return fail(KL_EINVAL, "KL_SEED_ALL gives four values per word; evaluate one seed at a time");
    if (window && (rc = check_window(window))) return rc;
    if (n && (!idx || !z_out)) return fail(KL_EINVAL, "idx and z_out must not be NULL");
    return plan_split(depth, o.precision, o.tail_len, o.lane_len, sp);
}

static int eval_run(const Gens& G, const Split& sp, const uint64_t* idx, uint64_t n, const kl_window* window,
                    kl_c64* z_out, const kl_opts& o) {
    if (n == 0) return KL_OK;
    hipStream_t s = (hipStream_t)o.stream;
    Temp tmp(s);
    SetTables st;
    int rc;
    if ((rc = build_tables(G, sp, o.precision, o.suffix_form, seed_index(o), tmp, &st))) return rc;
    EvalJob job{};
    job.sp = sp;
    job.precision = o.precision;
    job.gens = G;
    job.fold = make_fold(window, o.head_form);
    job.tab = st.tab;
    job.tail_homog = st.tail_homog;
    job.idx = idx;
    job.n = n;
    job.out = (c64*)z_out;
    hipError_t e = launch_eval(job, s);
    if (e != hipSuccess) return hip_fail(e, "eval kernel");
    return KL_OK;
}

// A tiling render (min_depth < depth) that leaves the split to the planner
// takes its deepest depth's tail -- the tail a render of that depth alone
// would take -- at every depth long enough for it, so that the units of its
// batched launch carry equal work and its index ranges split their words
// the same way.  (The tiling of Maskit's group to depth 14, 4-letter tails
// throughout: 0.18 ms, against 0.215 ms with 6 letters throughout and
// 0.25 ms with 4 letters at depths 13-14 only.)
// That applies where the two differ (deepest depths 13-16) and no tuned
// plan covers the deepest depth; tuned plans keep their depths' splits.
static kl_opts tiling_opts(const kl_opts& o, int min_depth, int depth, const kl_window* w) {
    if (min_depth >= depth || o.tail_len != 0 || o.lane_len != 0) return o;
    if (apply_tuned(o, depth, w).tail_len != 0) return o;
    Split single, tiling;
    if (plan_split(depth, o.precision, 0, 0, &single, kPlanSingle) != KL_OK ||
        plan_split(depth, o.precision, 0, 0, &tiling, kPlanTiling) != KL_OK || single.r == tiling.r)
        return o;
    kl_opts r = o;
    r.tail_len = single.r;
    return r;
}

}  // namespace kl

extern "C" {

int kl_render_ex(kl_c64 ta, kl_c64 tb, int depth, const kl_window* window, uint32_t* image_out,
                 const kl_opts* opts) {
    const kl_opts o = opts ? *opts : default_opts();
    RenderSpan span;
    int rc = check_render(depth, window, image_out, o, &span);
    if (rc) return rc;
    Gens G;
    if ((rc = make_gens(ta, tb, &G))) return rc;
    return render_run(G, depth, window, image_out, tiling_opts(o, span.min_depth, depth, window), span);
}

int kl_render_noalloc(kl_c64 ta, kl_c64 tb, int depth, const kl_window* window, uint32_t* image_out,
                      const kl_opts* opts) {
    const kl_opts o = opts ? *opts : default_opts();
    RenderSpan span;
    int rc = check_render(depth, window, image_out, o, &span);
    if (rc) return rc;
    if (span.min_depth != depth)
        return fail(KL_EINVAL, "kl_render_noalloc renders one depth: min_depth must be 0 or %d", depth);
    // the split's tables must fit the scratch array, checked before anything is enqueued
    const kl_opts ot = apply_tuned(o, depth, window);
    Split sp;
    if ((rc = plan_split(depth, ot.precision, ot.tail_len, ot.lane_len, &sp))) return rc;
    const size_t need = table_layout(sp, ot.precision).total;
    if (need > (size_t)KL_NOALLOC_SCRATCH_BYTES)
        return fail(KL_ENOMEM, "depth %d (prefix %d, tail %d letters) needs %zu bytes of tables; the scratch array "
                    "holds %zu", depth, sp.k, sp.r, need, (size_t)KL_NOALLOC_SCRATCH_BYTES);
    Gens G;
    if ((rc = make_gens(ta, tb, &G))) return rc;
    void* p = nullptr;
    if ((rc = scratch_address(&p))) return rc;
    const TableBuf buf{(unsigned char*)p, (size_t)KL_NOALLOC_SCRATCH_BYTES};
    return render_run(G, depth, window, image_out, o, span, &buf);
}

int kl_render_group_ex(const kl_c64* ab, int depth, const kl_window* window, uint32_t* image_out,
                       const kl_opts* opts) {
    const kl_opts o = opts ? *opts : default_opts();
    RenderSpan span;
    int rc = check_render(depth, window, image_out, o, &span);
    if (rc) return rc;
    Gens G;
    if ((rc = make_gens_ab(ab, &G))) return rc;
    return render_run(G, depth, window, image_out, tiling_opts(o, span.min_depth, depth, window), span);
}

int kl_render(kl_c64 ta, kl_c64 tb, int depth, const kl_window* window, uint32_t* image_out) {
    int rc = kl_render_ex(ta, tb, depth, window, image_out, nullptr);
    if (rc) return rc;
    hipError_t e = hipStreamSynchronize(nullptr);
    return e == hipSuccess ? KL_OK : hip_fail(e, "render");
}

int kl_eval_ex(kl_c64 ta, kl_c64 tb, int depth, const uint64_t* idx, uint64_t n, const kl_window* window,
               kl_c64* z_out, const kl_opts* opts) {
    kl_opts o = opts ? *opts : default_opts();
    if (depth >= 1 && depth <= KL_MAX_DEPTH) o = apply_tuned(o, depth, window);
    Split sp;
    int rc = check_eval(depth, idx, n, window, z_out, o, &sp);
    if (rc || n == 0) return rc;
    Gens G;
    if ((rc = make_gens(ta, tb, &G))) return rc;
    return eval_run(G, sp, idx, n, window, z_out, o);
}

int kl_eval_group_ex(const kl_c64* ab, int depth, const uint64_t* idx, uint64_t n, const kl_window* window,
                     kl_c64* z_out, const kl_opts* opts) {
    kl_opts o = opts ? *opts : default_opts();
    if (depth >= 1 && depth <= KL_MAX_DEPTH) o = apply_tuned(o, depth, window);
    Split sp;
    int rc = check_eval(depth, idx, n, window, z_out, o, &sp);
    if (rc) return rc;
    Gens G;
    if ((rc = make_gens_ab(ab, &G))) return rc;
    return eval_run(G, sp, idx, n, window, z_out, o);
}

// ------------------------------------------------------------------ random walks (Section 4)
}  // extern "C"

namespace kl {

// The walk's shape, checked before anything is enqueued; n_total letters per
// walker and n_points drawn points in all.
static int check_walk(const kl_walk* walk, uint64_t* n_total, uint64_t* n_points) {
    if (!walk) return fail(KL_EINVAL, "walk is NULL");
    // the last walker, first_walker + n_walkers - 1, must be below 2^64
    if (walk->n_walkers && walk->n_walkers - 1 > UINT64_MAX - walk->first_walker)
        return fail(KL_ERANGE, "walkers [%llu, +%llu) pass 2^64", (unsigned long long)walk->first_walker,
                    (unsigned long long)walk->n_walkers);
    const uint64_t nt = 1ull + walk->burn_in + walk->n_steps;
    if (nt > 0xFFFFFFFFull) return fail(KL_EINVAL, "1 + burn_in + n_steps exceeds 2^32 - 1");
    if (walk->n_walkers && (walk->n_walkers > UINT64_MAX / nt))
        return fail(KL_ERANGE, "walkers times letters exceeds 2^64");
    *n_total = nt;
    *n_points = walk->n_walkers * walk->n_steps;
    return KL_OK;
}

static WalkJob walk_job(const Gens& G, const kl_walk* walk, const kl_window* window, int precision, int mode) {
    WalkJob j{};
    j.gens = G;
    j.fold = make_fold(window, 0);
    j.precision = precision;
    j.mode = mode;
    j.seed = walk->seed;
    j.first_walker = walk->first_walker;
    j.n_walkers = walk->n_walkers;
    j.burn_in = walk->burn_in;
    j.n_steps = walk->n_steps;
    return j;
}

}  // namespace kl

extern "C" {

int kl_walk_letters(const kl_walk* walk, uint8_t* letters_out, void* stream) {
    uint64_t nt, np;
    int rc = check_walk(walk, &nt, &np);
    if (rc) return rc;
    if (walk->n_walkers && !letters_out) return fail(KL_EINVAL, "letters_out is NULL");
    Gens G{};
    for (int k = 0; k < 4; ++k) G.g[k] = {{1.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {1.0, 0.0}};
    WalkJob j = walk_job(G, walk, nullptr, KL_PREC_FP32, kWalkLetters);
    j.letters = letters_out;
    hipError_t e = launch_walk(j, (hipStream_t)stream);
    return e == hipSuccess ? KL_OK : hip_fail(e, "walk kernel");
}

int kl_walk_eval_ex(const kl_c64* ab, const kl_walk* walk, const kl_window* window, kl_c64* z_out,
                    const kl_opts* opts) {
    const kl_opts o = opts ? *opts : default_opts();
    uint64_t nt, np;
    int rc = check_walk(walk, &nt, &np);
    if (rc) return rc;
    if ((rc = check_opts_common(o))) return rc;
    if (window && (rc = check_window(window))) return rc;
    if (np && !z_out) return fail(KL_EINVAL, "z_out is NULL");
    Gens G;
    if ((rc = make_gens_ab(ab, &G))) return rc;
    WalkJob j = walk_job(G, walk, window, o.precision, kWalkEval);
    j.z_out = (c64*)z_out;
    hipError_t e = launch_walk(j, (hipStream_t)o.stream);
    return e == hipSuccess ? KL_OK : hip_fail(e, "walk kernel");
}

int kl_walk_render_ex(const kl_c64* ab, const kl_walk* walk, const kl_window* window, uint32_t* image_out,
                      const kl_opts* opts) {
    const kl_opts o = opts ? *opts : default_opts();
    uint64_t nt, np;
    int rc = check_walk(walk, &nt, &np);
    if (rc) return rc;
    if ((rc = check_opts_common(o))) return rc;
    if ((rc = check_window(window))) return rc;
    if (!image_out) return fail(KL_EINVAL, "image_out is NULL");
    if (o.hist_mode == KL_HIST_LDS && walk_tiles(window->width, window->height) > kMaxWalkTiles)
        return fail(KL_EINVAL, "hist_mode KL_HIST_LDS takes images of at most %u x 32768 bins", kMaxWalkTiles);
    if (o.hist_mode == KL_HIST_LDS && walk_region_points(walk->n_steps) > kWalkBinnedPoints)
        return fail(KL_EINVAL, "hist_mode KL_HIST_LDS takes at most %llu drawn points per walker",
                    (unsigned long long)(kWalkBinnedPoints / 256));
    Gens G;
    if ((rc = make_gens_ab(ab, &G))) return rc;
    hipStream_t s = (hipStream_t)o.stream;
    hipError_t e;
    if (!o.accumulate) {
        if ((e = launch_fill_u32(image_out, (uint64_t)window->width * window->height, 0, s)) != hipSuccess)
            return hip_fail(e, "clear image");
        if (o.dropped_out && (e = launch_fill_u64(o.dropped_out, 1, 0, s)) != hipSuccess)
            return hip_fail(e, "clear dropped");
    }
    WalkJob j = walk_job(G, walk, window, o.precision, kWalkRender);
    j.image = image_out;
    j.W = window->width;
    j.H = window->height;
    j.dropped = o.dropped_out;
    e = o.hist_mode == KL_HIST_LDS || (o.hist_mode == KL_HIST_AUTO && np >= (1ull << 18) &&
                                       walk_tiles(j.W, j.H) <= kMaxWalkTiles &&
                                       walk_region_points(walk->n_steps) <= kWalkBinnedPoints)
            ? launch_walk_binned(j, s)
            : launch_walk(j, s);
    return e == hipSuccess ? KL_OK : hip_fail(e, "walk kernel");
}

int kl_group_seeds(const kl_c64* ab, kl_c64* gens_out, kl_c64* seeds_out) {
    Gens G;
    int rc = make_gens_ab(ab, &G);
    if (rc) return rc;
    for (int k = 0; k < 4; ++k) {
        if (gens_out) {
            gens_out[4 * k + 0] = {G.g[k].a.re, G.g[k].a.im};
            gens_out[4 * k + 1] = {G.g[k].b.re, G.g[k].b.im};
            gens_out[4 * k + 2] = {G.g[k].c.re, G.g[k].c.im};
            gens_out[4 * k + 3] = {G.g[k].d.re, G.g[k].d.im};
        }
        if (seeds_out) {
            const bool inf = (G.inf_mask >> k) & 1u;
            seeds_out[2 * k] = inf ? kl_c64{1.0, 0.0} : kl_c64{G.fix[k].re, G.fix[k].im};
            seeds_out[2 * k + 1] = inf ? kl_c64{0.0, 0.0} : kl_c64{1.0, 0.0};
        }
    }
    return KL_OK;
}

// Maskit's parametrisation: a = [[-i mu, -i], [-i, 0]], b = [[1, 2], [0, 1]].
int kl_maskit_generators(kl_c64 mu, kl_c64* ab_out) {
    if (!ab_out) return fail(KL_EINVAL, "ab_out is NULL");
    if (!std::isfinite(mu.re) || !std::isfinite(mu.im)) return fail(KL_EINVAL, "mu must be finite");
    ab_out[0] = {mu.im, -mu.re};  // -i mu
    ab_out[1] = {0.0, -1.0};
    ab_out[2] = {0.0, -1.0};
    ab_out[3] = {0.0, 0.0};
    ab_out[4] = {1.0, 0.0};
    ab_out[5] = {2.0, 0.0};
    ab_out[6] = {0.0, 0.0};
    ab_out[7] = {1.0, 0.0};
    return KL_OK;
}

int kl_eval(kl_c64 ta, kl_c64 tb, int depth, const uint64_t* idx, uint64_t n, int precision, kl_c64* z_out) {
    kl_opts o = default_opts();
    o.precision = precision;
    int rc = kl_eval_ex(ta, tb, depth, idx, n, nullptr, z_out, &o);
    if (rc) return rc;
    hipError_t e = hipStreamSynchronize(nullptr);
    return e == hipSuccess ? KL_OK : hip_fail(e, "eval");
}

}  // extern "C"

namespace kl {

// A table with its maps and seeds, checked, and the start of each depth in
// the combined index space of depths min_depth..max_depth.  need_maps:
// evaluation and rendering (decoding reads the table only).
static int make_cayley(const kl_cayley* t, int min_depth, int max_depth, bool need_maps, CayleyJob* j) {
    if (!t || !t->table) return fail(KL_EINVAL, "Cayley table is NULL");
    const int S = t->n_states, m = t->n_symbols;
    if (S < 2 || S > kCayleyMaxStates) return fail(KL_EINVAL, "n_states %d outside 2..16", S);
    if (m < 1 || m > kCayleyMaxSymbols) return fail(KL_EINVAL, "n_symbols %d outside 1..8", m);
    if (min_depth < 1 || max_depth > KL_MAX_DEPTH || min_depth > max_depth)
        return fail(KL_EINVAL, "depths %d..%d outside 1..40", min_depth, max_depth);
    memset(j, 0, sizeof *j);
    j->S = S;
    j->m = m;
    j->min_depth = min_depth;
    j->max_depth = max_depth;
    for (int i = 0; i < S * (m + 1); ++i) {
        if (t->table[i] >= S) return fail(KL_EINVAL, "table entry %d = %d is not a state", i, t->table[i]);
        j->table[i] = t->table[i];
    }
    // counts of regular words by length and end state, as the kernel forms them
    std::vector<std::array<uint64_t, kCayleyMaxStates>> C(max_depth + 1);
    for (auto& row : C) row.fill(0);
    C[0][0] = 1;
    // every count below 2^63, every sum of counts within 64 bits
    const uint64_t cap = (1ull << 63) - 1;
    for (int L = 1; L <= max_depth; ++L)
        for (int s = 0; s < S; ++s)
            for (int x = 1; x <= m; ++x) {
                const int nx = t->table[s * (m + 1) + x];
                if (nx == 0) continue;
                if (C[L][nx] > cap - C[L - 1][s]) return fail(KL_EINVAL, "the words of length %d exceed 2^63", L);
                C[L][nx] += C[L - 1][s];
            }
    uint64_t start = 0;
    for (int d = min_depth; d <= max_depth; ++d) {
        j->depth_start[d - min_depth] = start;
        uint64_t n = 0;
        for (int s = 1; s < S; ++s) {
            if (n > UINT64_MAX - C[d][s]) return fail(KL_EINVAL, "the words of depth %d exceed 2^64", d);
            n += C[d][s];
        }
        if (start > UINT64_MAX - n) return fail(KL_EINVAL, "the words of depths %d..%d exceed 2^64", min_depth, max_depth);
        start += n;
    }
    j->depth_start[max_depth - min_depth + 1] = start;
    // tail length of the head/tail evaluation: the longest r <= 12 (and <= the
    // largest depth) with at most kCayleyHeadTails regular words, which the
    // render spreads one head per thread
    for (int r = std::min(kCayleyMaxTail, max_depth); r >= 1; --r) {
        uint64_t n = 0;
        for (int s = 1; s < S; ++s) n += C[r][s];
        if (n <= (uint64_t)kCayleyHeadTails) {
            j->r = r;
            j->n_tails = (int)n;
            break;
        }
    }
    // the good sets reachable from the set of all states, and their transitions
    auto extend = [&](uint32_t good, int x) {
        uint32_t g = 0;
        for (int s = 0; s < S; ++s) {
            const int nx = t->table[s * (m + 1) + x];
            if (nx != 0 && ((good >> nx) & 1u)) g |= 1u << s;
        }
        return g;
    };
    j->sets[0] = (uint16_t)((1u << S) - 1u);
    j->n_sets = 1;
    for (int g = 0; g < j->n_sets; ++g)
        for (int x = 1; x <= m; ++x) {
            const uint32_t nxt = extend(j->sets[g], x);
            int h = 0;
            while (h < j->n_sets && j->sets[h] != nxt) ++h;
            if (h == j->n_sets) {
                if (h == kCayleyMaxSets)
                    return fail(KL_EINVAL, "the table's prefixes need more than %d good-state sets", kCayleyMaxSets);
                j->sets[h] = (uint16_t)nxt;
                ++j->n_sets;
            }
            j->next_set[g * m + x - 1] = (uint8_t)h;
        }
    if (!need_maps) return KL_OK;
    if (!t->maps) return fail(KL_EINVAL, "Cayley maps are NULL");
    for (int x = 0; x < m; ++x) {
        cd g[4];
        for (int e = 0; e < 4; ++e) {
            g[e] = cd(t->maps[4 * x + e].re, t->maps[4 * x + e].im);
            if (!finite(g[e])) return fail(KL_EINVAL, "map of symbol %d is not finite", x + 1);
        }
        const cd det = g[0] * g[3] - g[1] * g[2];
        if (det == cd(0.0)) return fail(KL_ESINGULAR, "map of symbol %d has determinant 0", x + 1);
        const cd r = std::sqrt(det);
        for (auto& e : g) e /= r;
        cd fix;
        bool inf;
        if (attracting_point(g, &fix, &inf) != KL_OK)
            return fail(KL_ESINGULAR, "map of symbol %d has no attracting fixed point", x + 1);
        j->maps[x].a = {g[0].real(), g[0].imag()};
        j->maps[x].b = {g[1].real(), g[1].imag()};
        j->maps[x].c = {g[2].real(), g[2].imag()};
        j->maps[x].d = {g[3].real(), g[3].imag()};
        j->fix[x] = {fix.real(), fix.imag()};
        if (inf) j->inf_mask |= 1u << x;
    }
    return KL_OK;
}

static int cayley_seed(const kl_opts& o, int m, int* seed) {
    if (o.seed_mode == KL_SEED_OWN) *seed = -1;
    else if (o.seed_mode >= KL_SEED_A && o.seed_mode - KL_SEED_A < m)
        *seed = o.seed_mode - KL_SEED_A;
    else return fail(KL_EINVAL, "seed_mode %d does not name one of the %d symbols", o.seed_mode, m);
    return KL_OK;
}

}  // namespace kl

extern "C" {

uint64_t kl_cayley_num_words(const kl_cayley* t, int depth) {
    CayleyJob j;
    if (depth < 1 || depth > KL_MAX_DEPTH || make_cayley(t, depth, depth, false, &j) != KL_OK) return 0;
    return j.depth_start[1];
}

int kl_cayley_decode_ex(const kl_cayley* t, uint64_t first_idx, uint64_t count, int depth, uint8_t* symbols_out,
                        void* stream) {
    CayleyJob j;
    int rc = make_cayley(t, depth, depth, false, &j);
    if (rc) return rc;
    const uint64_t n = j.depth_start[1];
    if (first_idx > n || count > n - first_idx)
        return fail(KL_ERANGE, "indices [%llu, +%llu) exceed the %llu words", (unsigned long long)first_idx,
                    (unsigned long long)count, (unsigned long long)n);
    if (count == 0) return KL_OK;
    if (!symbols_out) return fail(KL_EINVAL, "symbols_out is NULL");
    j.first = first_idx;
    j.count = count;
    j.symbols_out = symbols_out;
    j.grid_blocks = device_cu_count() * 8;
    hipError_t e = launch_cayley(j, kCayleyDecode, (hipStream_t)stream);
    return e == hipSuccess ? KL_OK : hip_fail(e, "Cayley decode kernel");
}

int kl_cayley_eval_ex(const kl_cayley* t, int depth, const uint64_t* idx, uint64_t n, const kl_window* window,
                      kl_c64* z_out, const kl_opts* opts) {
    const kl_opts o = opts ? *opts : default_opts();
    CayleyJob j;
    int rc = make_cayley(t, depth, depth, true, &j);
    if (rc) return rc;
    if ((rc = check_opts_common(o, KL_SEED_A + kCayleyMaxSymbols - 1)) || (rc = cayley_seed(o, j.m, &j.seed)))
        return rc;
    if (window && (rc = check_window(window))) return rc;
    if (n == 0) return KL_OK;
    if (!idx || !z_out) return fail(KL_EINVAL, "idx and z_out must not be NULL");
    j.fold = make_fold(window, 0);
    j.count = n;
    j.idx = idx;
    j.z_out = (c64*)z_out;
    j.grid_blocks = device_cu_count() * 8;
    hipError_t e = launch_cayley(j, kCayleyEval, (hipStream_t)o.stream);
    return e == hipSuccess ? KL_OK : hip_fail(e, "Cayley eval kernel");
}

int kl_cayley_render_ex(const kl_cayley* t, int depth, const kl_window* window, uint32_t* image_out,
                        const kl_opts* opts) {
    const kl_opts o = opts ? *opts : default_opts();
    int rc = check_window(window);
    if (rc) return rc;
    if (!image_out) return fail(KL_EINVAL, "image_out is NULL");
    if ((rc = check_opts_common(o, KL_SEED_A + kCayleyMaxSymbols - 1))) return rc;
    if (depth < 1 || depth > KL_MAX_DEPTH) return fail(KL_EINVAL, "depth %d outside 1..40", depth);
    const int min_depth = o.min_depth == 0 ? depth : o.min_depth;
    CayleyJob j;
    if ((rc = make_cayley(t, min_depth, depth, true, &j))) return rc;
    const uint64_t total = j.depth_start[depth - min_depth + 1];
    uint64_t first = 0, count = total;
    if (o.use_range) {
        first = o.first_idx;
        count = o.count;
        if (first > total || count > total - first)
            return fail(KL_ERANGE, "range [%llu, +%llu) exceeds the %llu words", (unsigned long long)first,
                        (unsigned long long)count, (unsigned long long)total);
    }
    std::vector<int> seeds;
    if (o.seed_mode == KL_SEED_ALL) {
        for (int x = 0; x < j.m; ++x) seeds.push_back(x);
    } else {
        int sd;
        if ((rc = cayley_seed(o, j.m, &sd))) return rc;
        seeds.push_back(sd);
    }
    hipStream_t s = (hipStream_t)o.stream;
    hipError_t e;
    if (!o.accumulate) {
        if ((e = launch_fill_u32(image_out, (uint64_t)window->width * window->height, 0, s)) != hipSuccess)
            return hip_fail(e, "clear image");
        if (o.dropped_out && (e = launch_fill_u64(o.dropped_out, 1, 0, s)) != hipSuccess)
            return hip_fail(e, "clear dropped");
    }
    j.fold = make_fold(window, 0);
    j.first = first;
    j.count = count;
    j.image = image_out;
    j.W = window->width;
    j.H = window->height;
    j.dropped = o.dropped_out;
    j.grid_blocks = device_cu_count() * 2;   // the tail table fits two workgroups per CU
    // every seed in one render: one tail table per seed in the head kernel
    j.n_seeds = (int)seeds.size();
    for (int k = 0; k < j.n_seeds; ++k) j.seed_list[k] = (int8_t)seeds[k];
    j.seed = seeds[0];
    if ((e = launch_cayley(j, kCayleyRender, s)) != hipSuccess) return hip_fail(e, "Cayley render kernel");
    return KL_OK;
}

}  // extern "C"

namespace kl {

// Explicit per-depth splits of a batched render (the batch tuner's
// candidates): tail and lane lengths by depth, 0 for the planner's or the
// tuned plan; wpc 0 for the planner's grid.
struct BatchPlans {
    int r[KL_MAX_DEPTH + 1] = {};
    int m[KL_MAX_DEPTH + 1] = {};
    int wpc = 0;
};

static int render_many_run(int n, const kl_c64* ta, const kl_c64* tb, const int* depth, const kl_window* window,
                           uint32_t* images_out, const kl_opts& o_in, const BatchPlans* bp);

}  // namespace kl

extern "C" {

int kl_render_many_ex(int n, const kl_c64* ta, const kl_c64* tb, const int* depth, const kl_window* window,
                      uint32_t* images_out, const kl_opts* opts) {
    return render_many_run(n, ta, tb, depth, window, images_out, opts ? *opts : default_opts(), nullptr);
}

}  // extern "C"

namespace kl {

static int render_many_run(int n, const kl_c64* ta, const kl_c64* tb, const int* depth, const kl_window* window,
                           uint32_t* images_out, const kl_opts& o_in, const BatchPlans* bp) {
    kl_opts o = o_in;
    if (n <= 0) return fail(KL_EINVAL, "n = %d must be positive", n);
    if (!ta || !tb || !depth) return fail(KL_EINVAL, "ta, tb and depth must not be NULL");
    int rc = check_window(window);
    if (rc) return rc;
    if (!images_out) return fail(KL_EINVAL, "images_out is NULL");
    if ((rc = check_opts_common(o))) return rc;
    if (o.min_depth != 0 || o.use_range) return fail(KL_EINVAL, "min_depth and use_range must be 0 for kl_render_many");
    if (o.seed_mode == KL_SEED_ALL) {
        // the paper's loop over the generators' fixed points: four batches, accumulated
        for (int q = 0; q < 4; ++q) {
            kl_opts oq = o;
            oq.seed_mode = KL_SEED_A + q;
            oq.accumulate = o.accumulate || q > 0;
            if ((rc = render_many_run(n, ta, tb, depth, window, images_out, oq, bp))) return rc;
        }
        return KL_OK;
    }
    const uint64_t bins = (uint64_t)window->width * window->height;
    std::vector<Gens> gens(n);
    std::vector<Split> splits(n);
    std::vector<kl_opts> per(n);
    for (int i = 0; i < n; ++i) {
        if (depth[i] < 1 || depth[i] > KL_MAX_DEPTH) return fail(KL_EINVAL, "set %d: depth %d outside 1..40", i, depth[i]);
        per[i] = apply_tuned(opts_for_depth(o, depth[i]), depth[i], window, true);
        if (bp && bp->r[depth[i]]) {
            per[i].tail_len = bp->r[depth[i]];
            per[i].lane_len = bp->m[depth[i]];
        }
        if ((rc = plan_split(depth[i], o.precision, per[i].tail_len, per[i].lane_len, &splits[i], kPlanBatch))) {
            std::string m = g_last_error;
            return fail(rc, "set %d: %s", i, m.c_str());
        }
        if ((rc = make_gens(ta[i], tb[i], &gens[i]))) {
            std::string m = g_last_error;
            return fail(rc, "set %d: %s", i, m.c_str());
        }
    }
    hipStream_t s = (hipStream_t)o.stream;
    hipError_t e;
    if (!o.accumulate) {
        if ((e = launch_fill_u32(images_out, bins * (uint64_t)n, 0, s)) != hipSuccess) return hip_fail(e, "clear images");
        if (o.dropped_out && (e = launch_fill_u64(o.dropped_out, (uint64_t)n, 0, s)) != hipSuccess)
            return hip_fail(e, "clear dropped");
    }
    std::vector<SetSpec> specs(n);
    int wpc = o.waves_per_cu ? o.waves_per_cu : (bp ? bp->wpc : 0);
    for (int i = 0; i < n; ++i) {
        specs[i] = {gens[i], splits[i], seed_index(o), images_out + bins * i, o.dropped_out ? o.dropped_out + i : nullptr};
        if (!wpc && persistent_ok(splits[i])) wpc = per[i].waves_per_cu;
    }
    return render_sets(specs, window, o, wpc, s);
}

// Median time of a batched render with plans bp (one untimed run first).
static int time_batch(int n, const kl_c64* ta, const kl_c64* tb, const int* depth, const kl_window* window,
                      uint32_t* images, const kl_opts& o, const BatchPlans& bp, hipEvent_t e0, hipEvent_t e1,
                      double* ms_out) {
    std::vector<float> times;
    for (int rep = 0; rep < 4; ++rep) {
        (void)hipEventRecord(e0, nullptr);
        int rc = render_many_run(n, ta, tb, depth, window, images, o, &bp);
        (void)hipEventRecord(e1, nullptr);
        if (rc) return rc;
        if (hipEventSynchronize(e1) != hipSuccess) return fail(KL_EDEVICE, "batch autotune timing failed");
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep) times.push_back(ms);
    }
    std::sort(times.begin(), times.end());
    *ms_out = times[times.size() / 2];
    return KL_OK;
}

}  // namespace kl

extern "C" {

int kl_autotune_many(int n, const kl_c64* ta, const kl_c64* tb, const int* depth, const kl_window* window,
                     int precision, uint32_t* scratch_images, kl_plan_t* plans_out, double* best_ms_out,
                     double* default_ms_out) {
    if (n <= 0) return fail(KL_EINVAL, "n = %d must be positive", n);
    if (!ta || !tb || !depth) return fail(KL_EINVAL, "ta, tb and depth must not be NULL");
    int rc = check_window(window);
    if (rc) return rc;
    if (!scratch_images) return fail(KL_EINVAL, "scratch_images is NULL");
    if (precision != KL_PREC_FP32 && precision != KL_PREC_FP64) return fail(KL_EINVAL, "precision %d", precision);
    bool present[KL_MAX_DEPTH + 1] = {};
    for (int i = 0; i < n; ++i) {
        if (depth[i] < 1 || depth[i] > KL_MAX_DEPTH) return fail(KL_EINVAL, "set %d: depth %d outside 1..40", i, depth[i]);
        present[depth[i]] = true;
    }
    kl_opts o = default_opts();
    o.precision = precision;
    // the planner's plans, whatever was tuned before
    BatchPlans cur;
    for (int d = 1; d <= KL_MAX_DEPTH; ++d) {
        if (!present[d]) continue;
        Split sp;
        if ((rc = plan_split(d, precision, 0, 0, &sp, kPlanBatch))) return rc;
        cur.r[d] = sp.r;
        cur.m[d] = sp.m;
    }
    cur.wpc = kDefaultWavesPerCU;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(KL_EDEVICE, "hipEventCreate failed");
    double def_ms = 0, best = 0;
    rc = time_batch(n, ta, tb, depth, window, scratch_images, o, cur, e0, e1, &def_ms);
    best = def_ms;
    // coordinate descent: each depth's split, deepest first, then the grid;
    // a change is kept only when the whole batch gets at least 1% faster
    for (int d = KL_MAX_DEPTH; d >= 1 && rc == KL_OK; --d) {
        if (!present[d]) continue;
        for (int r = 4; r <= std::min(7, d - 1) && rc == KL_OK; ++r)
            for (int m = 1; m <= 6 && rc == KL_OK; ++m) {
                const int k = d - r - m;
                if (k < 1 || k > 9 || (r == cur.r[d] && m == cur.m[d])) continue;
                BatchPlans trial = cur;
                trial.r[d] = r;
                trial.m[d] = m;
                double t = 0;
                if ((rc = time_batch(n, ta, tb, depth, window, scratch_images, o, trial, e0, e1, &t))) break;
                if (t < 0.99 * best) {
                    best = t;
                    cur = trial;
                }
            }
    }
    for (int wpc : {16, 24}) {
        if (rc) break;
        BatchPlans trial = cur;
        trial.wpc = wpc;
        double t = 0;
        if ((rc = time_batch(n, ta, tb, depth, window, scratch_images, o, trial, e0, e1, &t))) break;
        if (t < 0.99 * best) {
            best = t;
            cur = trial;
        }
    }
    // confirmation: the kept plans and the planner's, timed alternately;
    // the planner's stay unless the kept ones still win by 1%
    BatchPlans def;
    for (int d = 1; d <= KL_MAX_DEPTH; ++d) {
        def.r[d] = 0;
        def.m[d] = 0;
        if (!present[d]) continue;
        Split sp;
        if (rc == KL_OK && (rc = plan_split(d, precision, 0, 0, &sp, kPlanBatch)) == KL_OK) {
            def.r[d] = sp.r;
            def.m[d] = sp.m;
        }
    }
    def.wpc = kDefaultWavesPerCU;
    if (rc == KL_OK && best < def_ms) {
        double td[3] = {}, tt[3] = {};
        for (int q = 0; q < 3 && rc == KL_OK; ++q) {
            if ((rc = time_batch(n, ta, tb, depth, window, scratch_images, o, def, e0, e1, &td[q]))) break;
            rc = time_batch(n, ta, tb, depth, window, scratch_images, o, cur, e0, e1, &tt[q]);
        }
        std::sort(td, td + 3);
        std::sort(tt, tt + 3);
        def_ms = td[1];
        best = tt[1];
        if (best >= 0.99 * def_ms) {
            cur = def;
            best = def_ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    for (int d = 1; d <= KL_MAX_DEPTH; ++d) {
        if (!present[d]) continue;
        Tuned t{};
        device_arch(t.arch, sizeof t.arch);
        t.ctx = kTuneBatch;
        t.depth = d;
        t.precision = precision;
        t.W = window->width;
        t.H = window->height;
        t.r = cur.r[d];
        t.m = cur.m[d];
        t.wpc = cur.wpc;
        t.hist = KL_HIST_RUNS;
        t.ms = best;
        store_tuned(t);
    }
    if (plans_out)
        for (int i = 0; i < n; ++i) {
            const int d = depth[i];
            plans_out[i].depth = d;
            plans_out[i].tail_len = cur.r[d];
            plans_out[i].lane_len = cur.m[d];
            plans_out[i].prefix_len = d - cur.r[d] - cur.m[d];
            plans_out[i].hist_mode = KL_HIST_RUNS;
            plans_out[i].waves_per_cu = cur.wpc;
        }
    if (best_ms_out) *best_ms_out = best;
    if (default_ms_out) *default_ms_out = def_ms;
    return KL_OK;
}

int kl_plan_many(int depth, int precision, const kl_window* window, kl_plan_t* plan_out) {
    if (depth < 1 || depth > KL_MAX_DEPTH) return fail(KL_EINVAL, "depth %d outside 1..40", depth);
    if (!plan_out) return fail(KL_EINVAL, "plan_out is NULL");
    if (precision != KL_PREC_FP32 && precision != KL_PREC_FP64) return fail(KL_EINVAL, "precision %d", precision);
    int rc = check_window(window);
    if (rc) return rc;
    kl_opts o = default_opts();
    o.precision = precision;
    o = apply_tuned(o, depth, window, true);
    Split sp;
    if ((rc = plan_split(depth, precision, o.tail_len, o.lane_len, &sp, kPlanBatch))) return rc;
    plan_out->depth = depth;
    plan_out->tail_len = sp.r;
    plan_out->lane_len = sp.m;
    plan_out->prefix_len = sp.k;
    plan_out->hist_mode = KL_HIST_RUNS;
    plan_out->waves_per_cu = o.waves_per_cu ? o.waves_per_cu : kDefaultWavesPerCU;
    return KL_OK;
}

int kl_render_many(int n, const kl_c64* ta, const kl_c64* tb, const int* depth, const kl_window* window,
                   uint32_t* images_out) {
    int rc = kl_render_many_ex(n, ta, tb, depth, window, images_out, nullptr);
    if (rc) return rc;
    hipError_t e = hipStreamSynchronize(nullptr);
    return e == hipSuccess ? KL_OK : hip_fail(e, "render_many");
}

int kl_autotune(kl_c64 ta, kl_c64 tb, int depth, const kl_window* window, int precision, uint32_t* scratch_image,
                kl_plan_t* best_out, double* best_ms_out) {
    if (depth < 2 || depth > KL_MAX_DEPTH) return fail(KL_EINVAL, "depth %d outside 2..40", depth);
    int rc = check_window(window);
    if (rc) return rc;
    if (!scratch_image) return fail(KL_EINVAL, "scratch_image is NULL");
    if (precision != KL_PREC_FP32 && precision != KL_PREC_FP64) return fail(KL_EINVAL, "precision %d", precision);
    Gens G;
    if ((rc = make_gens(ta, tb, &G))) return rc;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(KL_EDEVICE, "hipEventCreate failed");
    Tuned best{};
    device_arch(best.arch, sizeof best.arch);
    best.ctx = kTuneSingle;
    best.depth = depth;
    best.precision = precision;
    best.hist = KL_HIST_RUNS;
    best.ms = 1e300;
    const int wpcs[] = {8, 16, 24, 32};
    for (int r = 3; r <= std::min(kMaxTail - 1, depth - 1); ++r) {
        for (int m = 1; m <= std::min(6, depth - r - 1); ++m) {
            if (depth - r - m > kMaxPrefix) continue;
            for (int wpc : wpcs) for (int hist : {KL_HIST_RUNS, KL_HIST_LDS}) {
                kl_opts o = default_opts();
                o.precision = precision;
                o.tail_len = r;
                o.lane_len = m;
                o.waves_per_cu = wpc;
                o.hist_mode = hist;
                std::vector<float> times;
                for (int rep = 0; rep < 4; ++rep) {
                    (void)hipEventRecord(e0, nullptr);
                    rc = kl_render_ex(ta, tb, depth, window, scratch_image, &o);
                    (void)hipEventRecord(e1, nullptr);
                    if (rc) break;
                    if (hipEventSynchronize(e1) != hipSuccess) {
                        rc = fail(KL_EDEVICE, "autotune timing failed");
                        break;
                    }
                    float ms = 0;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    if (rep) times.push_back(ms);
                }
                if (rc) {
                    (void)hipEventDestroy(e0);
                    (void)hipEventDestroy(e1);
                    return rc;
                }
                std::sort(times.begin(), times.end());
                const double med = times[times.size() / 2];
                if (med < best.ms) {
                    best.r = r;
                    best.m = m;
                    best.wpc = wpc;
                    best.hist = hist;
                    best.ms = med;
                }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best.r == 0) return fail(KL_EINVAL, "no candidate plan for depth %d", depth);
    store_tuned(best);
    if (best_out) {
        best_out->depth = depth;
        best_out->tail_len = best.r;
        best_out->lane_len = best.m;
        best_out->prefix_len = depth - best.r - best.m;
        best_out->hist_mode = best.hist;
        best_out->waves_per_cu = best.wpc;
    }
    if (best_ms_out) *best_ms_out = best.ms;
    return KL_OK;
}

}  // extern "C"
