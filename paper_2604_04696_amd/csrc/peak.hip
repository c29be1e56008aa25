// Issue-rate microbenchmarks (include/pir_peak.h): the INT8 MFMA and
// v_mad_u64_u32 rates and a streaming HBM read, measured on this GPU.
//
// Every kernel reads the shader clock counter (s_memtime) and the 100 MHz
// constant clock (s_memrealtime) at the start and end of each wave's loop;
// lane 0 of every wave adds its two deltas into a pair of 64-bit counters,
// from which the host takes the average shader clock.  Results of the loops
// are folded into one word per wave and stored, so the compiler keeps the
// work.
#include <algorithm>
#include <functional>

#include "common.h"
#include "modarith.h"

namespace pir {

typedef int p_i32x4 __attribute__((ext_vector_type(4)));
typedef int p_i32x16 __attribute__((ext_vector_type(16)));

struct ClockSums {
    unsigned long long shader, real;
};

__device__ __forceinline__ void add_clock(ClockSums *c, uint64_t s0, uint64_t r0) {
    const uint64_t s1 = __builtin_amdgcn_s_memtime(), r1 = __builtin_amdgcn_s_memrealtime();
    if (threadIdx.x % 64 == 0) {
        atomicAdd(&c->shader, (unsigned long long)(s1 - s0));
        atomicAdd(&c->real, (unsigned long long)(r1 - r0));
    }
}

__global__ void __launch_bounds__(256) peak_mfma_kernel(uint32_t iters, int random_operands, int *sink,
                                                        ClockSums *clk) {
    const uint32_t tid = blockIdx.x * 256 + threadIdx.x;
    p_i32x16 acc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = (p_i32x16){};
    uint64_t s0, r0;
    if (!random_operands) {
        // zero operands, no other instruction in the loop
        const p_i32x4 z = {0, 0, 0, 0};
        s0 = __builtin_amdgcn_s_memtime();
        r0 = __builtin_amdgcn_s_memrealtime();
        for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(z, z, acc[j], 0, 0, 0);
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(z, z, acc[j], 0, 0, 0);
        }
    } else {
        // operands that change every 16 MFMAs: one 32-bit LCG step per word
        // (per lane), two operand pairs used in turn
        const uint32_t sa = tid * 2654435761u + 1, sb = tid * 2246822519u + 7;
        p_i32x4 a = {(int)sa, (int)(sa ^ 0x5bd1e995u), (int)(sa * 3u), (int)(sa + 0x27d4eb2fu)};
        p_i32x4 b = {(int)sb, (int)(sb ^ 0x68e31da4u), (int)(sb * 5u), (int)(sb + 0x165667b1u)};
        s0 = __builtin_amdgcn_s_memtime();
        r0 = __builtin_amdgcn_s_memrealtime();
        for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc[j], 0, 0, 0);
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(b, a, acc[j], 0, 0, 0);
            a = a * 1664525 + 1013904223;
            b = b * 22695477 + 1;
        }
    }
    add_clock(clk, s0, r0);
    int x = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) x ^= acc[j][r];
    sink[tid] = x;
}

__global__ void __launch_bounds__(256) peak_mad64_kernel(uint32_t iters, uint64_t *sink, ClockSums *clk) {
    const uint32_t tid = blockIdx.x * 256 + threadIdx.x;
    const uint32_t y = 0x9E3779B1u ^ tid;
    uint64_t acc[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[j] = (uint64_t)(tid + 1) * (2 * j + 1);
    const uint64_t s0 = __builtin_amdgcn_s_memtime(), r0 = __builtin_amdgcn_s_memrealtime();
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < 16; ++j)   // the multiplicand is the chain's own high word
            acc[j] = (uint64_t)(uint32_t)(acc[j] >> 32) * y + acc[j];
    }
    add_clock(clk, s0, r0);
    uint64_t x = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) x ^= acc[j];
    sink[tid] = x;
}

__global__ void __launch_bounds__(256) peak_read_kernel(const uint4 *__restrict__ src, uint64_t n16, uint32_t *sink) {
    uint32_t x = 0;
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += stride) {
        const uint4 v = ld_nt(src + i);
        x ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    // one word per block (any lane's value serves; the XOR only keeps the loads)
    if (x == 0x9E3779B9u) sink[blockIdx.x] = x;
}

static double run_timed(hipStream_t st, const std::function<void()> &launch) {
    hipEvent_t a = nullptr, b = nullptr;
    PIR_HIP(hipEventCreate(&a));
    const hipError_t e = hipEventCreate(&b);
    if (e != hipSuccess) {
        (void)hipEventDestroy(a);
        PIR_FAIL(PIR_EDEVICE, "hipEventCreate failed: %s", hipGetErrorString(e));
    }
    float ms = 0.0f;
    hipError_t r = hipEventRecord(a, st);
    if (r == hipSuccess) {
        launch();
        r = hipEventRecord(b, st);
    }
    if (r == hipSuccess) r = hipEventSynchronize(b);
    if (r == hipSuccess) r = hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (r != hipSuccess) PIR_FAIL(PIR_EDEVICE, "timing failed: %s", hipGetErrorString(r));
    return ms;
}

static int cus() {
    int dev = 0, n = 0;
    PIR_HIP(hipGetDevice(&dev));
    PIR_HIP(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev));
    return std::max(1, n);
}

}  // namespace pir

using namespace pir;

extern "C" {

pir_status pir_peak_mfma_i8(uint32_t iters, int random_operands, double *tops, double *mhz, void *stream) {
    return guarded([&] {
        PIR_REQUIRE(tops && mhz, "NULL argument");
        PIR_REQUIRE(iters >= 1 && iters <= (1u << 24), "iters must be 1..2^24");
        hipStream_t st = reinterpret_cast<hipStream_t>(stream);
        const uint32_t blocks = 2 * (uint32_t)cus();   // 8 waves per CU
        DevBuf sink((size_t)blocks * 256 * 4 + sizeof(ClockSums));
        ClockSums *clk = reinterpret_cast<ClockSums *>(sink.as<int8_t>() + (size_t)blocks * 256 * 4);
        PIR_HIP(hipMemsetAsync(clk, 0, sizeof(ClockSums), st));
        const double ms = run_timed(st, [&] {
            peak_mfma_kernel<<<blocks, 256, 0, st>>>(iters, random_operands ? 1 : 0, sink.as<int>(), clk);
        });
        PIR_LAUNCH_CHECK();
        ClockSums h{};
        PIR_HIP(hipMemcpy(&h, clk, sizeof(h), hipMemcpyDeviceToHost));
        const double mfmas = (double)blocks * 4 * iters * 16;
        *tops = mfmas * 65536.0 / (ms * 1e-3) / 1e12;
        *mhz = h.real ? 100.0 * (double)h.shader / (double)h.real : 0.0;
    });
}

pir_status pir_peak_valu_mad64(uint32_t iters, double *gops, double *mhz, void *stream) {
    return guarded([&] {
        PIR_REQUIRE(gops && mhz, "NULL argument");
        PIR_REQUIRE(iters >= 1 && iters <= (1u << 24), "iters must be 1..2^24");
        hipStream_t st = reinterpret_cast<hipStream_t>(stream);
        const uint32_t blocks = 4 * (uint32_t)cus();   // 16 waves per CU
        DevBuf sink((size_t)blocks * 256 * 8 + sizeof(ClockSums));
        ClockSums *clk = reinterpret_cast<ClockSums *>(sink.as<int8_t>() + (size_t)blocks * 256 * 8);
        PIR_HIP(hipMemsetAsync(clk, 0, sizeof(ClockSums), st));
        const double ms = run_timed(st, [&] {
            peak_mad64_kernel<<<blocks, 256, 0, st>>>(iters, sink.as<uint64_t>(), clk);
        });
        PIR_LAUNCH_CHECK();
        ClockSums h{};
        PIR_HIP(hipMemcpy(&h, clk, sizeof(h), hipMemcpyDeviceToHost));
        *gops = (double)blocks * 256 * iters * 16 / (ms * 1e-3) / 1e9;
        *mhz = h.real ? 100.0 * (double)h.shader / (double)h.real : 0.0;
    });
}

pir_status pir_peak_hbm_read(const void *src, uint64_t bytes, double *gbs, void *stream) {
    return guarded([&] {
        PIR_REQUIRE(src && gbs, "NULL argument");
        PIR_REQUIRE(bytes >= 16 && bytes % 16 == 0, "bytes must be a positive multiple of 16");
        PIR_REQUIRE(reinterpret_cast<uintptr_t>(src) % 16 == 0, "src must be 16-byte aligned");
        hipStream_t st = reinterpret_cast<hipStream_t>(stream);
        const uint32_t blocks = 8 * (uint32_t)cus();
        DevBuf sink((size_t)blocks * 4);
        const double ms = run_timed(st, [&] {
            peak_read_kernel<<<blocks, 256, 0, st>>>(static_cast<const uint4 *>(src), bytes / 16,
                                                     sink.as<uint32_t>());
        });
        PIR_LAUNCH_CHECK();
        *gbs = (double)bytes / (ms * 1e-3) / 1e9;
    });
}

}  // extern "C"
