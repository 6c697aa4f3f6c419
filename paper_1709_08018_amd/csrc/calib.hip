// calib.hip -- libkl_calib.so: instruction-throughput microbenchmarks that
// calibrate the renderer's VALU roofline on gfx950, and store-pattern
// microbenchmarks beside the decode kernel's HBM roofline.  Not part of the
// renderer's ABI; bench.py --workload calib and --workload decode call it.
//
// Each kernel runs 8 independent dependency chains of one instruction class
// per lane for a fixed trip count on 32 waves per CU, and stores one value
// per thread at the end.  From the event-timed duration and the device
// clock follows the cost of one wave64 instruction group per SIMD, in cycles:
//   cycles = ms * clock * (CUs * 4 SIMDs) / (waves * groups per wave).
// The integer and compare classes are written as single ALU instructions so
// that the compiler cannot fold their chains.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kIters = 4096;
constexpr int kChains = 8;
constexpr int kClasses = 9;

template <int OP>
__global__ __launch_bounds__(256) void rate_kernel(float* out, float s, float t, unsigned su) {
    float a[kChains];
    unsigned u[kChains];
    double d[kChains];
    for (int i = 0; i < kChains; ++i) {
        a[i] = threadIdx.x * 1e-3f + i;
        u[i] = threadIdx.x + i;
        d[i] = threadIdx.x * 1e-3 + i;
    }
    for (int it = 0; it < kIters; ++it) {
#pragma unroll
        for (int i = 0; i < kChains; ++i) {
            if constexpr (OP == 0) a[i] = __builtin_fmaf(a[i], s, t);
            if constexpr (OP == 1) a[i] = a[i] * s;
            if constexpr (OP == 2) a[i] = a[i] + s;
            if constexpr (OP == 3) asm volatile("v_add_u32 %0, %0, %1" : "+v"(u[i]) : "s"(su));
            if constexpr (OP == 4) a[i] = __builtin_amdgcn_rcpf(a[i]);
            if constexpr (OP == 5) asm volatile("v_mad_u32_u24 %0, %0, %1, 7" : "+v"(u[i]) : "s"(su));
            if constexpr (OP == 6) {
                int r;
                asm volatile("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(a[i]));
                a[i] = __int_as_float(r) + s;
            }
            if constexpr (OP == 7)
                asm volatile("v_cmp_gt_u32 vcc, %1, %0\n\tv_cndmask_b32 %0, %1, %0, vcc" : "+v"(u[i]) : "v"(su) : "vcc");
            if constexpr (OP == 8) d[i] = __builtin_fma(d[i], (double)s, (double)t);
        }
    }
    float acc = 0;
    for (int i = 0; i < kChains; ++i) acc += a[i] + (float)u[i] + (float)d[i];
    out[blockIdx.x * 256 + threadIdx.x] = acc;
}

template <int OP>
hipError_t time_class(float* out, int blocks, hipEvent_t e0, hipEvent_t e1, float* ms) {
    for (int w = 0; w < 3; ++w) hipLaunchKernelGGL(rate_kernel<OP>, dim3(blocks), dim3(256), 0, 0, out, 1.0001f, 0.5f, 123u);
    hipError_t e = hipEventRecord(e0, nullptr);
    for (int w = 0; w < 5; ++w) hipLaunchKernelGGL(rate_kernel<OP>, dim3(blocks), dim3(256), 0, 0, out, 1.0001f, 0.5f, 123u);
    if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    *ms /= 5;
    return e == hipSuccess ? hipGetLastError() : e;
}

// ---- store patterns
// The same bytes written in different orders, 16 bytes a thread and store.
// Chunks: workgroup c writes chunk c (per_thread stores a thread, 4 KB
// apart), one chunk a workgroup, in launch order.
__global__ __launch_bounds__(256) void store_chunks(uint4* __restrict__ p, uint64_t n16, uint32_t per_thread) {
    const uint64_t base = (uint64_t)blockIdx.x * 256u * per_thread;
    for (uint32_t k = 0; k < per_thread; ++k) {
        const uint64_t i = base + (uint64_t)k * 256u + threadIdx.x;
        if (i < n16) p[i] = make_uint4((uint32_t)i, 1u, 2u, 3u);
    }
}

// Tiles: a persistent grid, workgroup b writing tiles b, b + grid, ... of
// tile16 16-byte pieces each, as the decode kernel writes its letters.
__global__ __launch_bounds__(256) void store_tiles(uint4* __restrict__ p, uint64_t n16, uint32_t tile16) {
    const uint64_t tiles = (n16 + tile16 - 1) / tile16;
    for (uint64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        const uint64_t base = t * tile16;
        for (uint32_t k = threadIdx.x; k < tile16; k += 256) {
            const uint64_t i = base + k;
            if (i < n16) p[i] = make_uint4((uint32_t)i, 1u, 2u, 3u);
        }
    }
}

}  // namespace

extern "C" {

// Store patterns: `bytes` (a multiple of 16) written to the device buffer
// `buf` (16-byte aligned) in each of kl_calib_store_patterns orders, 2
// warm-up and 5 timed launches each; gbs_out[i] (host) receives GB/s:
//   0..2  one chunk of 4, 16, 64 KB a workgroup, non-persistent;
//   3..5  persistent, 8 workgroups a CU, tiles of 4 KB, 36,864 B (the
//         decode's tile at depth 18: 2048 words of 18 letters) and 144 KB.
// Returns 0, -1 for a misaligned or unsized buffer, or -4 on a HIP error.
int kl_calib_store_patterns(void) { return 6; }

int kl_calib_store(void* buf, uint64_t bytes, double* gbs_out) {
    if (!buf || !gbs_out || bytes == 0 || (bytes & 15) || ((uintptr_t)buf & 15)) return -1;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return -4;
    uint4* p = (uint4*)buf;
    const uint64_t n16 = bytes / 16;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -4;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -4;
    }
    hipError_t e = hipSuccess;
    for (int pat = 0; pat < 6 && e == hipSuccess; ++pat) {
        auto launch = [&]() {
            if (pat < 3) {
                const uint32_t per = pat == 0 ? 1u : pat == 1 ? 4u : 16u;
                const uint64_t blocks = (n16 + 256ull * per - 1) / (256ull * per);
                hipLaunchKernelGGL(store_chunks, dim3((unsigned)blocks), dim3(256), 0, 0, p, n16, per);
            } else {
                const uint32_t tile16 = pat == 3 ? 256u : pat == 4 ? 2304u : 9216u;
                hipLaunchKernelGGL(store_tiles, dim3((unsigned)(cus * 8)), dim3(256), 0, 0, p, n16, tile16);
            }
        };
        for (int w = 0; w < 2; ++w) launch();
        e = hipEventRecord(e0, nullptr);
        for (int w = 0; w < 5 && e == hipSuccess; ++w) launch();
        if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess) e = hipGetLastError();
        gbs_out[pat] = e == hipSuccess && ms > 0.0f ? (double)bytes * 5 / (ms * 1e-3) / 1e9 : 0.0;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return e == hipSuccess ? 0 : -4;
}

// Instruction classes, in the order of the outputs:
//   0 v_fma_f32, 1 v_mul_f32, 2 v_add_f32, 3 v_add_u32, 4 v_rcp_f32,
//   5 v_mad_u32_u24, 6 v_cvt_flr_i32_f32 + v_add_f32 (a group of two),
//   7 v_cmp_gt_u32 + v_cndmask_b32 (a group of two), 8 v_fma_f64.
// ms_out[9]: kernel milliseconds; cycles_out[9]: SIMD cycles per wave64
// group at clock_ghz_out (the device's reported maximum clock).  Host
// pointers.  Returns 0, or -4 on a HIP error.
int kl_calib_valu(double* ms_out, double* cycles_out, double* clock_ghz_out) {
    int dev = 0, cus = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeClockRate, dev) != hipSuccess)
        return -4;
    const int blocks = cus * 8;  // 32 waves per CU
    float* out = nullptr;
    if (hipMalloc(&out, (size_t)blocks * 256 * sizeof(float)) != hipSuccess) return -4;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipFree(out);
        return -4;
    }
    float ms[kClasses] = {};
    hipError_t e = time_class<0>(out, blocks, e0, e1, &ms[0]);
    if (e == hipSuccess) e = time_class<1>(out, blocks, e0, e1, &ms[1]);
    if (e == hipSuccess) e = time_class<2>(out, blocks, e0, e1, &ms[2]);
    if (e == hipSuccess) e = time_class<3>(out, blocks, e0, e1, &ms[3]);
    if (e == hipSuccess) e = time_class<4>(out, blocks, e0, e1, &ms[4]);
    if (e == hipSuccess) e = time_class<5>(out, blocks, e0, e1, &ms[5]);
    if (e == hipSuccess) e = time_class<6>(out, blocks, e0, e1, &ms[6]);
    if (e == hipSuccess) e = time_class<7>(out, blocks, e0, e1, &ms[7]);
    if (e == hipSuccess) e = time_class<8>(out, blocks, e0, e1, &ms[8]);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(out);
    if (e != hipSuccess) return -4;
    const double ghz = khz * 1e-6;
    const double groups = (double)blocks * 4 * kIters * kChains;  // wave-groups
    for (int i = 0; i < kClasses; ++i) {
        ms_out[i] = ms[i];
        cycles_out[i] = ms[i] * 1e-3 * ghz * 1e9 * (cus * 4.0) / groups;
    }
    *clock_ghz_out = ghz;
    return 0;
}

}  // extern "C"
