// decode.hip -- kl_decode: the words with given indices, with no stored
// list (Sections 4 and 6 of the paper: the index is read as the first
// letter, a base-4 digit, followed by base-3 digits, each the rank of a
// letter among those that do not undo its predecessor).
#include <algorithm>
#include <array>
#include <atomic>
#include <utility>

#include "kl_internal.hpp"

namespace kl {

namespace {

__device__ __forceinline__ int inv_letter(int c) { return c ^ 2; }
__device__ __forceinline__ uint64_t div3_u64(uint64_t x) { return __umul64hi(x, 0xAAAAAAAAAAAAAAABull) >> 1; }

}  // namespace

// ------------------------------------------------------------------ decode
// A word of depth d is its first letter index / 3^(d-1) followed by the
// d - 1 base-3 digits of the rest, most significant first; letter j is the
// t_j-th letter that is not the inverse of letter j - 1.  The digits go six
// at a time through a table, built once per workgroup in LDS, that maps
// (previous letter, six digits) to the next six letters, 2 bits each (the
// last of them in bits 10..11).  A shorter group is padded with zero digits
// at its end, whose letters are not kept.
constexpr uint32_t kDigitGroup = 729;   // 3^6

__device__ void build_next6(uint16_t* next6) {
    for (uint32_t e = threadIdx.x; e < 4 * kDigitGroup; e += blockDim.x) {
        int prev = (int)(e / kDigitGroup);
        uint32_t v = e - (uint32_t)prev * kDigitGroup;
        int dg[6];
        for (int j = 5; j >= 0; --j) {
            const uint32_t q = v / 3;
            dg[j] = (int)(v - 3 * q);
            v = q;
        }
        uint32_t bits = 0;
        for (int j = 0; j < 6; ++j) {
            const int c = dg[j] + (dg[j] >= inv_letter(prev));
            bits |= (uint32_t)c << (2 * j);
            prev = c;
        }
        next6[e] = (uint16_t)bits;
    }
}

// Byte path (any depth, any destination): one word per thread, staged as
// bytes, 256 words a tile, written as one contiguous byte range.
__device__ __forceinline__ void put_letters(uint64_t& lo, uint64_t& hi, int pos, uint64_t bits) {
    const int sh = 2 * pos;   // pos <= 39, bits < 2^12
    if (sh < 64) {
        lo |= bits << sh;
        if (sh > 52) hi |= bits >> (64 - sh);
    } else {
        hi |= bits << (sh - 64);
    }
}

__device__ __forceinline__ uint8_t letter_at(uint64_t lo, uint64_t hi, int j) {
    return (uint8_t)((j < 32 ? lo >> (2 * j) : hi >> (2 * j - 64)) & 3u);
}

__global__ __launch_bounds__(256) void decode_bytes_kernel(uint64_t first, uint64_t count, int depth,
                                                           uint8_t* __restrict__ out) {
    __shared__ uint16_t next6[4 * kDigitGroup];
    __shared__ __align__(16) uint8_t stage[256 * KL_MAX_DEPTH];
    const int tid = threadIdx.x;
    build_next6(next6);
    __syncthreads();
    const int n = depth - 1, groups = n / 6, p = n - 6 * groups;   // p digits in a last, shorter group
    uint32_t pow_p = 1;
    for (int j = 0; j < p; ++j) pow_p *= 3;
    const uint32_t pad = kDigitGroup / pow_p;   // 3^(6 - p)
    const uint64_t tiles = (count + 255) / 256;
    for (uint64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const uint64_t tfirst = tile * 256;
        const uint64_t rem = count - tfirst;
        const uint32_t nw = rem < 256 ? (uint32_t)rem : 256u;
        uint8_t* dst = out + tfirst * (uint64_t)depth;
        if ((uint32_t)tid < nw) {
            uint64_t r = first + tfirst + tid;
            uint32_t last = 0;
            if (p) {
                uint64_t q = r;
                for (int j = 0; j < p; ++j) q = div3_u64(q);
                last = (uint32_t)(r - q * pow_p);
                r = q;
            }
            uint32_t g[6];   // groups of six digits, least significant first
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                g[k] = 0;
                if (k < groups) {
                    const uint64_t q = r / kDigitGroup;
                    g[k] = (uint32_t)(r - q * kDigitGroup);
                    r = q;
                }
            }
            int prev = (int)r;   // the first letter (an index below first + count: <= 3)
            uint64_t lo = (uint64_t)prev, hi = 0;
            int pos = 1;
#pragma unroll
            for (int kk = 5; kk >= 0; --kk) {
                if (kk < groups) {
                    const uint32_t bits = next6[prev * kDigitGroup + g[kk]];
                    put_letters(lo, hi, pos, bits);
                    prev = (int)(bits >> 10);
                    pos += 6;
                }
            }
            if (p) put_letters(lo, hi, pos, next6[prev * kDigitGroup + last * pad] & ((1u << (2 * p)) - 1u));
            uint8_t* w = stage + tid * depth;
            for (int j = 0; j < depth; ++j) w[j] = letter_at(lo, hi, j);
        }
        __syncthreads();
        const uint32_t nbytes = nw * (uint32_t)depth;
        if (((uintptr_t)dst & 15u) == 0) {
            const uint32_t n16 = nbytes / 16;
            for (uint32_t i = tid; i < n16; i += 256) ((uint4*)dst)[i] = ((const uint4*)stage)[i];
            for (uint32_t i = n16 * 16 + tid; i < nbytes; i += 256) dst[i] = stage[i];
        } else {
            for (uint32_t i = tid; i < nbytes; i += 256) dst[i] = stage[i];
        }
        __syncthreads();
    }
}

// Packed path: depths 16 .. 32 into a 16-byte aligned destination, one
// kernel per depth D, so that every digit group, position and shift is a
// constant.  The letters of a tile are staged in LDS as one stream, 2 bits a
// letter, 16 letters a dword, in the order of the output bytes: dword i of
// the stream is output piece i (bytes 16 i .. 16 i + 15).
//   * A thread takes K consecutive words, 2 D K bits of the stream: a whole
//     number of dwords (K = 8 for even D, 16 for odd D).
//   * The digits split into the first letter, HIGH groups of six, and a low
//     part of LOW digits (3 .. 8: the short group, widened by six when it
//     has fewer than three digits), so that the low part takes 3^LOW >= 27 >
//     K values and carries out of it at most once among a thread's words.
//     The thread unranks its first word once, forms the letters above the
//     low part for its high digits and for those plus one, and per word
//     reads the low part's letters from the table and picks the high
//     letters on whether the low digits have wrapped.
//   * A piece spreads its 16 letters to 16 bytes: bytes q of x and of
//     x >> 4 go to bytes 0 and 2 of a dword, and (v | v << 6) & 0x03030303
//     moves letters 1 and 3 of the four into bytes 1 and 3.
constexpr uint32_t pow3u(int e) {
    uint32_t v = 1;
    for (int i = 0; i < e; ++i) v *= 3;
    return v;
}

template <int D>
struct PackedDecode {
    static constexpr int N = D - 1;                         // base-3 digits after the first letter
    static constexpr int P = N % 6;
    static constexpr int LOW = P >= 3 ? P : P + 6;          // digits of the low part
    static constexpr uint32_t RADIX = pow3u(LOW);
    static constexpr int HIGH = (N - LOW) / 6;              // groups of six above it
    static constexpr int LOWPOS = 1 + 6 * HIGH;             // position of its first letter
    static constexpr int K = D % 2 ? 16 : 8;                // words per thread
    static constexpr int SEG = D * K / 16;                  // stream dwords per thread
    static constexpr uint32_t TILE = 256u * K;              // words per tile
    static_assert(D >= 16 && D <= 32 && HIGH >= 2 && RADIX > (uint32_t)K && 2 * D <= 64, "packed decode layout");
};

// Letters 0 .. LOWPOS - 1 (first letter and the HIGH groups, g[HIGH - 1]
// most significant), and the last of them.
template <int HIGH>
__device__ __forceinline__ uint64_t high_letters(uint32_t f, const uint32_t (&g)[HIGH], const uint16_t* next6,
                                                 uint32_t& last) {
    uint64_t L = f;
    uint32_t prev = f;
#pragma unroll
    for (int k = HIGH - 1; k >= 0; --k) {
        const uint32_t bits = next6[prev * kDigitGroup + g[k]];
        L |= (uint64_t)bits << (2 * (1 + 6 * (HIGH - 1 - k)));
        prev = bits >> 10;
    }
    last = prev;
    return L;
}

// Letters of the low part (2 LOW bits) of word k of a thread, from the
// table entry e of its first six digits (LOW <= 6: the entry's last 6 - LOW
// letters, of padding digits, are cut off; LOW = 7, 8: a second entry gives
// the last LOW - 6 letters).
template <int LOW>
__device__ __forceinline__ uint32_t low_letters(const uint16_t* next6, uint32_t e, uint32_t l2) {
    const uint32_t a = next6[e];
    if constexpr (LOW <= 6) {
        return a & ((1u << (2 * LOW)) - 1u);
    } else {
        const uint32_t b = next6[(a >> 10) * kDigitGroup + l2 * pow3u(12 - LOW)] & ((1u << (2 * (LOW - 6))) - 1u);
        return a | (b << 12);
    }
}

// 16 letters, 2 bits each, as 16 bytes.  v_perm_b32 puts byte q of x
// (letters 4q .. 4q + 3) in byte 0 and byte q of x >> 4 (letters 4q + 2 ..
// 4q + 5) in byte 2, zeros in bytes 1 and 3; then v | v << 6 copies letters
// 4q + 1 and 4q + 3 into bytes 1 and 3, and the mask keeps 2 bits a byte.
__device__ __forceinline__ uint32_t spread_quarter(uint32_t x, uint32_t y, uint32_t q) {
    const uint32_t v = __builtin_amdgcn_perm(y, x, 0x0C040C00u + 0x00010001u * q);
    return (v | (v << 6)) & 0x03030303u;
}

__device__ __forceinline__ uint4 spread16(uint32_t x) {
    const uint32_t y = x >> 4;
    return make_uint4(spread_quarter(x, y, 0), spread_quarter(x, y, 1), spread_quarter(x, y, 2), spread_quarter(x, y, 3));
}

template <int D>
__global__ __launch_bounds__(256) void decode_packed_kernel(uint64_t first, uint64_t count, uint8_t* __restrict__ out) {
    using L = PackedDecode<D>;
    __shared__ uint16_t next6[4 * kDigitGroup];
    __shared__ __align__(16) uint32_t stream[256 * L::SEG];
    const uint32_t tid = threadIdx.x;
    build_next6(next6);
    __syncthreads();
    const uint64_t tiles = (count + L::TILE - 1) / L::TILE;
    for (uint64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const uint64_t tfirst = tile * L::TILE;
        const uint64_t rem = count - tfirst;
        const uint32_t nw = rem < L::TILE ? (uint32_t)rem : L::TILE;
        const uint32_t w0 = tid * L::K;
        if (w0 < nw) {
            // first word: high digits h and low digits l0
            const uint64_t r = first + tfirst + w0;
            const uint64_t h = r / L::RADIX;
            const uint32_t l0 = (uint32_t)(r - h * L::RADIX);
            uint32_t g[L::HIGH], g1[L::HIGH], f;
            if constexpr (L::HIGH <= 3) {   // h < 4 * 729^3 < 2^32
                uint32_t x = (uint32_t)h;
#pragma unroll
                for (int k = 0; k < L::HIGH; ++k) {
                    const uint32_t q = x / kDigitGroup;
                    g[k] = x - q * kDigitGroup;
                    x = q;
                }
                f = x;
            } else {
                uint64_t x = h;
#pragma unroll
                for (int k = 0; k < L::HIGH; ++k) {
                    const uint64_t q = x / kDigitGroup;
                    g[k] = (uint32_t)(x - q * kDigitGroup);
                    x = q;
                }
                f = (uint32_t)x;
            }
            // the high digits plus one (their first letter kept <= 3: past
            // the last word those letters are never used)
            uint32_t c = 1;
#pragma unroll
            for (int k = 0; k < L::HIGH; ++k) {
                const uint32_t v = g[k] + c;
                c = v == kDigitGroup ? 1u : 0u;
                g1[k] = c ? 0u : v;
            }
            const uint32_t f1 = f + c < 3u ? f + c : 3u;
            uint32_t prev0, prev1;
            const uint64_t H0 = high_letters<L::HIGH>(f, g, next6, prev0);
            const uint64_t H1 = high_letters<L::HIGH>(f1, g1, next6, prev1);
            // Table entry of the low part's first six digits: before the
            // wrap e0 + k S (S = 3^(6 - LOW), or per six-digit step for LOW >
            // 6), after it e1 + k S, so a word's entry is a select plus a
            // constant offset.
            constexpr uint32_t R2 = L::LOW > 6 ? pow3u(L::LOW - 6) : 1;
            constexpr uint32_t S = L::LOW > 6 ? 1 : pow3u(6 - L::LOW);
            const uint32_t e0 = prev0 * kDigitGroup, e1 = prev1 * kDigitGroup;
            // LOW <= 6: entry (wrap ? b1 : b0) + k S, with the wrap folded in
            // (b1 wraps around as an unsigned number; b1 + k S does not)
            const uint32_t b0 = e0 + l0 * S, b1 = e1 + l0 * S - L::RADIX * S;
            uint32_t seg[L::SEG];
#pragma unroll
            for (int j = 0; j < L::SEG; ++j) seg[j] = 0;
#pragma unroll
            for (int k = 0; k < L::K; ++k) {
                // words past the range's end are formed too (from clamped
                // digits) and never written out
                const bool wrap = l0 >= L::RADIX - (uint32_t)k;
                uint32_t lowb;
                if constexpr (L::LOW <= 6) {
                    lowb = low_letters<L::LOW>(next6, (wrap ? b1 : b0) + (uint32_t)k * S, 0);
                } else {
                    const uint32_t l = wrap ? l0 + (uint32_t)k - L::RADIX : l0 + (uint32_t)k;
                    const uint32_t h6 = l / R2;
                    lowb = low_letters<L::LOW>(next6, (wrap ? e1 : e0) + h6, l - h6 * R2);
                }
                const uint64_t W = (wrap ? H1 : H0) | ((uint64_t)lowb << (2 * L::LOWPOS));
                const int s = 2 * D * k;   // the word's first bit in the thread's segment
#pragma unroll
                for (int j = s / 32; j <= (s + 2 * D - 1) / 32; ++j) {
                    const int sh = 32 * j - s;
                    seg[j] |= sh >= 0 ? (uint32_t)(W >> sh) : (uint32_t)(W << -sh);
                }
            }
            uint32_t* mine = stream + tid * L::SEG;
#pragma unroll
            for (int j = 0; j < L::SEG; ++j) mine[j] = seg[j];
        }
        __syncthreads();
        uint8_t* dst = out + tfirst * (uint64_t)D;
        if (nw == L::TILE) {
            // a whole tile: SEG pieces a thread, at uniform bases
#pragma unroll
            for (int j = 0; j < L::SEG; ++j) ((uint4*)dst + 256 * j)[tid] = spread16(stream[256 * j + tid]);
        } else {
            const uint32_t nbytes = nw * (uint32_t)D;
            const uint32_t n16 = nbytes / 16;
            for (uint32_t i = tid; i < n16; i += 256) ((uint4*)dst)[i] = spread16(stream[i]);
            for (uint32_t b = n16 * 16 + tid; b < nbytes; b += 256)
                dst[b] = (uint8_t)((stream[b / 16] >> (2 * (b % 16))) & 3u);
        }
        __syncthreads();
    }
}

using DecodeKernel = void (*)(uint64_t, uint64_t, uint8_t*);

template <int... I>
static constexpr std::array<DecodeKernel, sizeof...(I)> packed_decode_kernels(std::integer_sequence<int, I...>) {
    return {{decode_packed_kernel<16 + I>...}};
}

template <int... I>
static constexpr std::array<uint32_t, sizeof...(I)> packed_tile_words(std::integer_sequence<int, I...>) {
    return {{PackedDecode<16 + I>::TILE...}};
}

hipError_t launch_decode(uint64_t first, uint64_t count, int depth, uint8_t* out, hipStream_t s) {
    if (count == 0) return hipSuccess;
    static constexpr std::array<DecodeKernel, 17> kPacked = packed_decode_kernels(std::make_integer_sequence<int, 17>{});
    static constexpr std::array<uint32_t, 17> kTile = packed_tile_words(std::make_integer_sequence<int, 17>{});
    const bool pack = depth >= 16 && depth <= 32 && ((uintptr_t)out & 15u) == 0;
    const void* fn = pack ? reinterpret_cast<const void*>(kPacked[depth - 16])
                          : reinterpret_cast<const void*>(decode_bytes_kernel);
    const uint64_t tile_words = pack ? kTile[depth - 16] : 256;
    const uint64_t tiles = (count + tile_words - 1) / tile_words;
    // as many workgroups as fit on a CU at once, so that none waits for a
    // second round (the same on every gfx950 device; asked once per kernel)
    static std::atomic<int> fits[18];
    const int slot = pack ? depth - 16 : 17;
    int resident = fits[slot].load(std::memory_order_relaxed);
    if (resident == 0) {
        int n = 0;
        resident = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, 256, 0) == hipSuccess && n > 0 ? n : 1;
        fits[slot].store(resident, std::memory_order_relaxed);
    }
    const uint64_t blocks = std::min<uint64_t>(tiles, (uint64_t)device_cu_count() * (uint64_t)resident);
    hipError_t e;
    if (pack) {
        void* args[] = {&first, &count, &out};
        e = hipLaunchKernel(fn, dim3((unsigned)blocks), dim3(256), args, 0, s);
    } else {
        void* args[] = {&first, &count, &depth, &out};
        e = hipLaunchKernel(fn, dim3((unsigned)blocks), dim3(256), args, 0, s);
    }
    return e != hipSuccess ? e : hipGetLastError();
}

}  // namespace kl
