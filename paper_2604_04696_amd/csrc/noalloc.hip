// pir_rowsel_noalloc: the streaming RowSel (VALU path, one to four clients)
// with its staging in a file-scope device array instead of allocated memory,
// for callers that cannot allocate (code under stream capture, serving loops,
// harnesses that forbid allocation).
//
// `scratch` is a device symbol: every GPU the library runs on holds its own
// copy from module load until the process ends.  Host code never uses the
// symbol's name as an address: at a device's first call its address is taken
// once with hipGetSymbolAddress (that device current) and kept per device,
// and the kernels receive that pointer.  All calls on one device share the
// array, so calls that overlap on one device race.
#include <mutex>

#include "common.h"

namespace pir {

static __device__ __align__(256) uint8_t scratch[PIR_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[MAX_DEVICES];

// Address of this device's copy of `scratch` (the device must be current).
static void *device_scratch(int dev) {
    PIR_REQUIRE(dev >= 0 && dev < MAX_DEVICES, "device %d beyond the %d this library tracks", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        PIR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        PIR_REQUIRE(p != nullptr, "hipGetSymbolAddress returned no address");
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace pir

using namespace pir;

extern "C" pir_status pir_rowsel_noalloc(const pir_db *db, const uint32_t *q_dev, uint32_t B, uint32_t *out_dev,
                                         void *hip_stream) {
    return guarded([&] {
        check_rowsel_args(db, q_dev, B, out_dev);
        if (B == 0) return;
        PIR_REQUIRE(db->layouts & PIR_LAYOUT_VALU, "pir_rowsel_noalloc needs a DB with the VALU layout");
        PIR_REQUIRE(B <= 4, "pir_rowsel_noalloc serves 1..4 clients (got %u)", B);
        const size_t need = stream_staging_bytes(*db, B);
        PIR_REQUIRE(need <= PIR_NOALLOC_SCRATCH_BYTES,
                    "pir_rowsel_noalloc: %zu bytes of staging needed, above its %u-byte maximum "
                    "(L*N*D1*2B*4 bytes; two clients per pass with primes of 2^30 or more)",
                    need, (unsigned)PIR_NOALLOC_SCRATCH_BYTES);
        DeviceGuard dg(db->device);
        void *stage = device_scratch(db->device);
        launch_rowsel_stream(*db, q_dev, B, out_dev, reinterpret_cast<hipStream_t>(hip_stream), stage);
    });
}
