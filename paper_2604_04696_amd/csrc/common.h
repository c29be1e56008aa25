// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/pir.h"

namespace pir {

// ------------------------------------------------------------------ errors
void set_error(const std::string &msg);
void clear_error();

struct Error {
    pir_status status;
    std::string msg;
};

#define PIR_FAIL(st, ...)                                                     \
    do {                                                                      \
        char _buf[512];                                                       \
        std::snprintf(_buf, sizeof(_buf), __VA_ARGS__);                       \
        throw ::pir::Error{st, std::string(_buf)};                            \
    } while (0)

#define PIR_REQUIRE(cond, ...)                                                \
    do {                                                                      \
        if (!(cond)) PIR_FAIL(PIR_EINVAL, __VA_ARGS__);                       \
    } while (0)

#define PIR_HIP(call)                                                         \
    do {                                                                      \
        hipError_t _e = (call);                                               \
        if (_e != hipSuccess)                                                 \
            PIR_FAIL(PIR_EDEVICE, "%s failed: %s (%s:%d)", #call,             \
                     hipGetErrorString(_e), __FILE__, __LINE__);              \
    } while (0)

// After a kernel launch: catches launch-configuration errors.
#define PIR_LAUNCH_CHECK() PIR_HIP(hipGetLastError())

// Runs `body` and converts exceptions into a status + thread-local message.
template <class F>
pir_status guarded(F &&body) {
    try {
        clear_error();
        body();
        return PIR_OK;
    } catch (const Error &e) {
        set_error(e.msg);
        return e.status;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return PIR_ENOMEM;
    } catch (const std::exception &e) {
        set_error(std::string("internal error: ") + e.what());
        return PIR_EDEVICE;
    } catch (...) {
        set_error("internal error");
        return PIR_EDEVICE;
    }
}

// --------------------------------------------------------- modular constants
// Per-prime constants passed to kernels by value.
//   q      the prime, < 2^32 (below 2^30 for the lazy VALU sums and the MFMA path)
//   r32    2^32 mod q           (folding a 64-bit sum: hi*2^32 + lo = hi*r32 + lo)
//   r64    2^64 mod q           (wide primes: wraps of a 64-bit sum)
//   mu     floor(2^64 / q)      (Barrett reduction of a 64-bit value)
//   qd, qinv    q and 1/q in binary64 (exact-integer reductions, see modarith.h)
//   c32, c47    2^32 mod q and 2^47 mod q in binary64
struct ModQ {
    uint32_t q;
    uint32_t r32;
    uint64_t mu;
    uint32_t fold2;   // 1 when r32 >= 2^28: two folds keep fifteen more products exact
    uint32_t r64;
    double qd, qinv, c32, c47;
};

// Primes at or above this bound take the wide forms (64-bit intermediates,
// no lazy sums) on the VALU path and in the NTTs, and on the MFMA path the
// digit window and the wide recombination.
constexpr uint32_t WIDE_Q = 1u << 30;

ModQ make_modq(uint32_t q);
bool is_prime_u32(uint32_t q);
uint32_t pow_mod(uint64_t a, uint64_t e, uint32_t q);

// Tables for the on-device negacyclic NTT of one prime.
struct NttTables {
    uint32_t q = 0, n = 0;
    uint32_t *fwd = nullptr;      // [n] psi^brv(i) and Shoup companions [n]
    uint32_t *inv = nullptr;      // [n] psi^-brv(i) and companions [n]
    uint32_t n_inv = 0, n_inv_shoup = 0;
};

// Tables are built once per (q, n) and kept for the process lifetime.
const NttTables &ntt_tables(uint32_t q, uint32_t n);

// ------------------------------------------------------------------ the DB
struct DbLayoutValu {
    // [L][N/4][S][D0][W][4] uint32: for a group of four consecutive NTT
    // points of one prime, the D1 columns are cut into S strips of
    // VALU_STRIP columns (the last one narrower, W = its width), and the D0
    // rows of one strip are one contiguous run of D0*W 16-byte vectors.
    uint32_t *data = nullptr;
};

constexpr uint32_t VALU_STRIP = 256;

// Offset (in 16-byte vectors) of strip `strip` of point group gg, and the
// strip's width; element (row k, column n) of the strip is at
// valu_strip_base(...) + k * width + (n % VALU_STRIP).
__host__ __device__ inline uint64_t valu_strip_base(uint64_t gg, uint32_t strip, uint32_t d0, uint32_t d1) {
    return gg * d0 * d1 + (uint64_t)strip * VALU_STRIP * d0;
}
__host__ __device__ inline uint32_t valu_strip_width(uint32_t strip, uint32_t d1) {
    const uint32_t left = d1 - strip * VALU_STRIP;
    return left < VALU_STRIP ? left : VALU_STRIP;
}

struct DbLayoutMfma {
    // [L*N][4][Kp/64][D1][64] int8: per point p and digit d, chunk c of
    // column n holds the d-th signed 8-bit digits of DB[64c .. 64c+63][n]
    // (zero for D0 <= k < Kp).
    int8_t *data = nullptr;
    uint32_t kp = 0;   // D0 rounded up to a multiple of 64
};

}  // namespace pir

struct pir_db {
    pir_params p{};
    uint32_t layouts = 0;
    int device = 0;
    bool wide = false;   // some prime is >= 2^30 (see WIDE_Q)
    pir::ModQ mod[PIR_MAX_PRIMES]{};
    pir::DbLayoutValu valu;
    pir::DbLayoutMfma mfma;
    uint64_t slots() const { return (uint64_t)p.n * p.nprimes; }
};

namespace pir {

// Validation shared by the entry points.
void validate_params(const pir_params &p);

// Device buffer that frees itself (used for temporaries).
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    explicit DevBuf(size_t n);
    ~DevBuf();
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

// Makes `dev` current for the guard's scope and restores the caller's
// current device afterwards (entry points never leave it changed).
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) PIR_HIP(hipSetDevice(dev));
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
    DeviceGuard(const DeviceGuard &) = delete;
    DeviceGuard &operator=(const DeviceGuard &) = delete;
};

void *dev_alloc(size_t bytes);   // throws PIR_ENOMEM
void dev_free(void *p);

// Stream-ordered temporary: hipMallocAsync on `st` at construction,
// hipFreeAsync on the same stream when the scope ends (also when a later
// step of the call throws).  Allocation failure throws PIR_ENOMEM.
struct StreamScratch {
    void *ptr = nullptr;
    hipStream_t st = nullptr;
    StreamScratch(size_t bytes, hipStream_t s);
    ~StreamScratch();
    StreamScratch(const StreamScratch &) = delete;
    StreamScratch &operator=(const StreamScratch &) = delete;
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

// Timing of each RowSel path's main kernel (pir_kernel_timing): while
// enabled, a Scope records a pair of HIP events on the launch stream around
// the launches made during its lifetime.
struct KernelTimer {
    struct Scope {
        explicit Scope(hipStream_t st);
        ~Scope();
        Scope(const Scope &) = delete;
        Scope &operator=(const Scope &) = delete;
        hipStream_t st;
        hipEvent_t start = nullptr;
    };
};

bool env_flag(const char *name);

// ---------------------------------------------------------------- launchers
// Defined in the kernel translation units; all enqueue on `st`.
void launch_ntt(const uint32_t *in, uint32_t *out, uint64_t count, uint64_t in_stride,
                uint64_t out_stride, const NttTables &t, bool inverse, hipStream_t st);
void launch_db_layout_valu(const pir_db &db, const uint32_t *ntt_src, uint32_t row0,
                           uint32_t nrows, hipStream_t st);
void launch_db_layout_mfma(const pir_db &db, const uint32_t *ntt_src, uint32_t row0,
                           uint32_t nrows, hipStream_t st);
void launch_rowsel_valu(const pir_db &db, const uint32_t *q, uint32_t B, uint32_t *out,
                        hipStream_t st);
// 2B <= 8.  stage_buf: staging of stream_staging_bytes(db, B) bytes supplied by
// the caller (NULL: stream-ordered scratch, and the kernel is timed when
// kernel timing is on)
void launch_rowsel_stream(const pir_db &db, const uint32_t *q, uint32_t B, uint32_t *out,
                          hipStream_t st, void *stage_buf = nullptr);
size_t stream_staging_bytes(const pir_db &db, uint32_t B);
// q_coeff: the query is in the coefficient domain (transformed first)
void launch_rowsel_mfma(const pir_db &db, const uint32_t *q, uint32_t B, uint32_t *out,
                        hipStream_t st, bool q_coeff = false);
// Query front end: coefficient-domain query -> NTT-domain query, both in the
// boundary layout [B][2][D0][L][N].
void launch_query_ntt(const pir_db &db, const uint32_t *q_coeff, uint32_t B, uint32_t *q_ntt, hipStream_t st);

// First ColTor stage (coltor.hip).
void coltor_check_gadget(const pir_params &ring, uint32_t log2z, uint32_t ell);
void launch_coltor_stage(const pir_params &ring, const uint32_t *ct, uint32_t B, uint32_t ncols,
                         const uint32_t *rgsw, uint32_t log2z, uint32_t ell, uint32_t *out, hipStream_t st);
size_t mfma_query_scratch_bytes(const pir_db &db, uint32_t B);
void launch_rowsel_mfma_grouped(const pir_rowsel_item *items, uint32_t count, hipStream_t st);
// Drops every cached grouped plan whose item list names `db`.
void release_group_plans(const pir_db *db);
// Tile of every item of the cached grouped plan of an item set, as (points,
// rows, columns) triples (zeros for B = 0 items); false if there is no plan.
bool group_plan_tiles(const pir_rowsel_item *items, uint32_t count, uint32_t *tiles);
void check_rowsel_args(const pir_db *db, const uint32_t *q, uint32_t B, const uint32_t *out);
void rowsel_one(const pir_db &db, const uint32_t *q, uint32_t B, uint32_t *out, pir_path path,
                hipStream_t st, bool q_coeff = false);
void launch_validate_residues(const uint32_t *x, uint64_t count_per_limb_block, uint32_t n,
                              uint32_t nprimes, const uint32_t *q, uint64_t total,
                              uint32_t *flag, hipStream_t st);

}  // namespace pir
