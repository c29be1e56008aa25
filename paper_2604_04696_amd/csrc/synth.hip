// Seeded synthetic inputs on the device (SplitMix64 as a counter-based
// stream; Steele, Lea and Flood, OOPSLA 2014).  Not part of RowSel: these
// kernels only let benchmarks and tests fill multi-GiB buffers in HBM.
#include <algorithm>

#include "common.h"
#include "../../include/pir_synth.h"

namespace pir {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t draw(uint64_t key, uint64_t i) {
    return mix64(key + (i + 1) * 0x9E3779B97F4A7C15ull);
}

__global__ void synth_query_kernel(uint32_t *out, uint64_t key, uint64_t base, uint64_t count,
                                   uint32_t n, uint32_t nprimes, uint32_t q0, uint32_t q1,
                                   uint32_t q2, uint32_t q3) {
    const uint32_t qs[4] = {q0, q1, q2, q3};
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t f = base + i;
        const uint32_t q = qs[(f / n) % nprimes];
        out[i] = (uint32_t)__umul64hi(draw(key, f), (uint64_t)q);
    }
}

__global__ void synth_db_kernel(uint32_t *out, uint64_t key, uint32_t row0, uint64_t count,
                                uint32_t d1, uint32_t nprimes, uint32_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t t = (uint32_t)(i % n);
        const uint64_t rec = i / ((uint64_t)n * nprimes);   // local (row, column) record
        const uint64_t k = row0 + rec / d1, col = rec % d1;
        out[i] = (uint32_t)(draw(key, (k * d1 + col) * n + t) & 0xFFFFu);
    }
}

__global__ void synth_draw_kernel(uint64_t *out, uint64_t key, uint64_t i0, uint64_t count) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = draw(key, i0 + i);
}

static uint32_t grid_for(uint64_t count) {
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((count + 255) / 256, 1u << 16));
}

}  // namespace pir

using namespace pir;

extern "C" {

pir_status pir_synth_query(uint32_t *out, uint64_t key, uint32_t b0, uint32_t nb, uint32_t d0,
                           uint32_t nprimes, uint32_t n, const uint32_t *q, void *stream) {
    return guarded([&] {
        PIR_REQUIRE(nprimes >= 1 && nprimes <= PIR_MAX_PRIMES && q != nullptr, "bad primes");
        PIR_REQUIRE(n >= 1, "bad n");
        for (uint32_t l = 0; l < nprimes; ++l) PIR_REQUIRE(q[l] >= 1, "q[%u] must be positive", l);
        const uint64_t per = 2ull * d0 * nprimes * n;
        const uint64_t count = per * nb;
        if (!count) return;
        PIR_REQUIRE(out != nullptr, "out is NULL");
        uint32_t qq[4] = {1, 1, 1, 1};
        for (uint32_t l = 0; l < nprimes; ++l) qq[l] = q[l];
        synth_query_kernel<<<grid_for(count), 256, 0, (hipStream_t)stream>>>(
            out, key, per * b0, count, n, nprimes, qq[0], qq[1], qq[2], qq[3]);
        PIR_LAUNCH_CHECK();
    });
}

pir_status pir_synth_db_coeffs(uint32_t *out, uint64_t key, uint32_t row0, uint32_t nrows,
                               uint32_t d1, uint32_t nprimes, uint32_t n, void *stream) {
    return guarded([&] {
        PIR_REQUIRE(nprimes >= 1 && nprimes <= PIR_MAX_PRIMES && n >= 1 && d1 >= 1, "bad shape");
        const uint64_t count = (uint64_t)nrows * d1 * nprimes * n;
        if (!count) return;
        PIR_REQUIRE(out != nullptr, "out is NULL");
        synth_db_kernel<<<grid_for(count), 256, 0, (hipStream_t)stream>>>(out, key, row0, count, d1,
                                                                          nprimes, n);
        PIR_LAUNCH_CHECK();
    });
}

pir_status pir_synth_draw(uint64_t *out, uint64_t key, uint64_t i0, uint64_t count, void *stream) {
    return guarded([&] {
        if (!count) return;
        PIR_REQUIRE(out != nullptr, "out is NULL");
        synth_draw_kernel<<<grid_for(count), 256, 0, (hipStream_t)stream>>>(out, key, i0, count);
        PIR_LAUNCH_CHECK();
    });
}

}  // extern "C"
