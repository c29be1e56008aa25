// C-ABI entry points of libpir.so: validation, DB management and dispatch.
#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "common.h"
#include "mfma.h"
#include "modarith.h"

namespace pir {

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

// ------------------------------------------------------------------ memory
void *dev_alloc(size_t bytes) {
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes ? bytes : 1);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        PIR_FAIL(PIR_ENOMEM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    }
    return p;
}

void dev_free(void *p) {
    if (p) (void)hipFree(p);
}

DevBuf::DevBuf(size_t n) : ptr(dev_alloc(n)), bytes(n) {}
DevBuf::~DevBuf() { dev_free(ptr); }

StreamScratch::StreamScratch(size_t bytes, hipStream_t s) : st(s) {
    if (bytes == 0) return;
    const hipError_t e = hipMallocAsync(&ptr, bytes, st);
    if (e != hipSuccess) {
        ptr = nullptr;
        (void)hipGetLastError();
        PIR_FAIL(e == hipErrorOutOfMemory ? PIR_ENOMEM : PIR_EDEVICE, "hipMallocAsync(%zu bytes) failed: %s",
                 bytes, hipGetErrorString(e));
    }
}
StreamScratch::~StreamScratch() {
    if (ptr) (void)hipFreeAsync(ptr, st);
}

// ------------------------------------------------------------- kernel timer
// Recorded (start, stop) pairs wait here until pir_kernel_time_read.
static std::atomic<bool> g_timing{false};
static std::mutex g_timing_mu;
static std::vector<std::pair<hipEvent_t, hipEvent_t>> g_timed;

static void drop_timed_locked() {
    for (auto &e : g_timed) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    g_timed.clear();
}

KernelTimer::Scope::Scope(hipStream_t s) : st(s) {
    if (!g_timing.load(std::memory_order_relaxed)) return;
    PIR_HIP(hipEventCreate(&start));
    const hipError_t e = hipEventRecord(start, st);
    if (e != hipSuccess) {
        (void)hipEventDestroy(start);
        start = nullptr;
        PIR_FAIL(PIR_EDEVICE, "hipEventRecord failed: %s", hipGetErrorString(e));
    }
}
KernelTimer::Scope::~Scope() {
    if (!start) return;
    hipEvent_t stop = nullptr;
    if (hipEventCreate(&stop) != hipSuccess || hipEventRecord(stop, st) != hipSuccess) {
        if (stop) (void)hipEventDestroy(stop);
        (void)hipEventDestroy(start);
        return;
    }
    std::lock_guard<std::mutex> lk(g_timing_mu);
    g_timed.emplace_back(start, stop);
}

bool env_flag(const char *name) {
    const char *v = std::getenv(name);
    return v && *v && std::strcmp(v, "0") != 0;
}

// ---------------------------------------------------------------- numbers
static uint64_t mulmod64(uint64_t a, uint64_t b, uint64_t m) {
    return (uint64_t)((unsigned __int128)a * b % m);
}

// Deterministic Miller-Rabin: bases 2, 7, 61 decide every n < 4,759,123,141.
bool is_prime_u32(uint32_t n) {
    if (n < 2) return false;
    for (uint32_t p : {2u, 3u, 5u, 7u, 11u, 13u, 61u})
        if (n % p == 0) return n == p;
    uint64_t d = n - 1;
    int r = 0;
    while ((d & 1) == 0) { d >>= 1; ++r; }
    for (uint64_t a : {2ull, 7ull, 61ull}) {
        uint64_t x = 1, b = a % n, e = d;
        while (e) {
            if (e & 1) x = mulmod64(x, b, n);
            b = mulmod64(b, b, n);
            e >>= 1;
        }
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int i = 1; i < r; ++i) {
            x = mulmod64(x, x, n);
            if (x == n - 1) { comp = false; break; }
        }
        if (comp) return false;
    }
    return true;
}

ModQ make_modq(uint32_t q) {
    ModQ m{};
    m.q = q;
    m.r32 = (uint32_t)((1ull << 32) % q);
    m.r64 = (uint32_t)(((unsigned __int128)1 << 64) % q);
    m.mu = (uint64_t)(((unsigned __int128)1 << 64) / q);
    m.fold2 = m.r32 >= (1u << 28) ? 1u : 0u;
    m.qd = (double)q;
    m.qinv = 1.0 / (double)q;
    m.c32 = (double)m.r32;
    m.c47 = (double)(uint32_t)((1ull << 47) % q);
    return m;
}

void validate_params(const pir_params &p) {
    PIR_REQUIRE(p.n >= 8 && p.n <= 16384 && (p.n & (p.n - 1)) == 0,
                "n must be a power of two in [8, 16384] (got %u)", p.n);
    PIR_REQUIRE(p.nprimes >= 1 && p.nprimes <= PIR_MAX_PRIMES, "nprimes must be 1..%d (got %u)",
                PIR_MAX_PRIMES, p.nprimes);
    for (uint32_t l = 0; l < p.nprimes; ++l) {
        const uint32_t q = p.q[l];
        PIR_REQUIRE(q >= 3, "q[%u] = %u is too small", l, q);
        PIR_REQUIRE(q % (2 * p.n) == 1, "q[%u] = %u is not 1 mod 2N = %u", l, q, 2 * p.n);
        PIR_REQUIRE(is_prime_u32(q), "q[%u] = %u is not prime", l, q);
    }
    PIR_REQUIRE(p.d0 >= 1 && p.d0 <= 65536, "d0 must be 1..65536 (got %u)", p.d0);
    PIR_REQUIRE(p.d1 >= 1 && p.d1 <= 65536, "d1 must be 1..65536 (got %u)", p.d1);
}

static hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

static bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
    auto x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + nb && y < x + na;
}

// Input check behind PIR_VALIDATE=1: counts residues >= q_l.
__global__ void validate_kernel(const uint32_t *x, uint64_t total, uint32_t n, uint32_t nprimes,
                                uint32_t q0, uint32_t q1, uint32_t q2, uint32_t q3, uint32_t *flag) {
    const uint32_t qs[4] = {q0, q1, q2, q3};
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t l = (uint32_t)((i / n) % nprimes);
        if (x[i] >= qs[l]) atomicOr(flag, 1u);
    }
}

static void check_residues(const uint32_t *x, uint64_t total, const pir_params &p, hipStream_t st) {
    DevBuf flag(sizeof(uint32_t));
    PIR_HIP(hipMemsetAsync(flag.ptr, 0, sizeof(uint32_t), st));
    uint32_t blocks = (uint32_t)std::min<uint64_t>((total + 255) / 256, 65536);
    validate_kernel<<<blocks, 256, 0, st>>>(x, total, p.n, p.nprimes, p.q[0], p.q[1], p.q[2], p.q[3],
                                            flag.as<uint32_t>());
    PIR_LAUNCH_CHECK();
    uint32_t h = 0;
    PIR_HIP(hipMemcpyAsync(&h, flag.ptr, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    PIR_HIP(hipStreamSynchronize(st));
    PIR_REQUIRE(h == 0, "input holds a value >= its prime (PIR_VALIDATE)");
}

static pir_path resolve_path(const pir_db &db, uint32_t B, pir_path path) {
    const bool has_v = db.layouts & PIR_LAYOUT_VALU, has_m = db.layouts & PIR_LAYOUT_MFMA;
    if (path == PIR_PATH_AUTO) {
        // one or two clients are HBM bound: the streaming VALU kernel reads the
        // DB once at full bandwidth; beyond that the matrix cores win.  With a
        // prime of 2^30 or more every client is its own streaming pass (two
        // 64-bit words per sum), so the matrix cores win from two clients on
        // (8 GiB DB, two 32-bit primes: 1.9 ms on MFMA against 2.8 ms)
        if (has_v && (!has_m || B <= (db.wide ? 1u : 2u))) return PIR_PATH_VALU;
        return PIR_PATH_MFMA_I8;
    }
    PIR_REQUIRE(path == PIR_PATH_VALU || path == PIR_PATH_MFMA_I8, "unknown path %d", (int)path);
    PIR_REQUIRE(path != PIR_PATH_VALU || has_v, "the DB holds no VALU layout");
    PIR_REQUIRE(path != PIR_PATH_MFMA_I8 || has_m, "the DB holds no MFMA layout");
    return path;
}

void check_rowsel_args(const pir_db *db, const uint32_t *q, uint32_t B, const uint32_t *out) {
    PIR_REQUIRE(db != nullptr, "db is NULL");
    if (B == 0) return;
    PIR_REQUIRE(B <= 65536, "B must be <= 65536 (got %u)", B);
    PIR_REQUIRE(q != nullptr && out != nullptr, "query or output pointer is NULL");
    PIR_REQUIRE(reinterpret_cast<uintptr_t>(q) % 16 == 0 && reinterpret_cast<uintptr_t>(out) % 16 == 0,
                "query and output must be 16-byte aligned");
    const auto &p = db->p;
    const size_t qb = (size_t)B * 2 * p.d0 * db->slots() * 4;
    const size_t ob = (size_t)B * 2 * p.d1 * db->slots() * 4;
    PIR_REQUIRE(!overlaps(q, qb, out, ob), "output overlaps the query");
}

void rowsel_one(const pir_db &db, const uint32_t *q, uint32_t B, uint32_t *out, pir_path path,
                hipStream_t st, bool q_coeff) {
    if (B == 0) return;
    DeviceGuard dg(db.device);
    const uint64_t qwords = (uint64_t)B * 2 * db.p.d0 * db.slots();
    if (!q_coeff && env_flag("PIR_VALIDATE")) check_residues(q, qwords, db.p, st);
    const pir_path use = resolve_path(db, B, path);
    if (use == PIR_PATH_VALU) {
        if (q_coeff) {
            StreamScratch qn(qwords * 4, st);   // NTT-domain copy of the query
            launch_query_ntt(db, q, B, qn.as<uint32_t>(), st);
            launch_rowsel_valu(db, qn.as<uint32_t>(), B, out, st);
        } else {
            launch_rowsel_valu(db, q, B, out, st);
        }
    } else {
        launch_rowsel_mfma(db, q, B, out, st, q_coeff);
    }
}

}  // namespace pir

using namespace pir;

extern "C" {

pir_status pir_kernel_timing(int enable) {
    return pir::guarded([&] {
        std::lock_guard<std::mutex> lk(pir::g_timing_mu);
        pir::g_timing.store(enable != 0);
        if (!enable) pir::drop_timed_locked();
    });
}

pir_status pir_kernel_time_read(uint32_t *launches, double *total_ms) {
    return pir::guarded([&] {
        PIR_REQUIRE(launches && total_ms, "launches and total_ms must not be NULL");
        std::vector<std::pair<hipEvent_t, hipEvent_t>> timed;
        {
            std::lock_guard<std::mutex> lk(pir::g_timing_mu);
            timed.swap(pir::g_timed);
        }
        double sum = 0;
        hipError_t err = hipSuccess;
        for (auto &e : timed) {
            float ms = 0;
            hipError_t r = hipEventSynchronize(e.second);
            if (r == hipSuccess) r = hipEventElapsedTime(&ms, e.first, e.second);
            if (r != hipSuccess && err == hipSuccess) err = r;
            sum += ms;
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        if (err != hipSuccess) PIR_FAIL(PIR_EDEVICE, "reading kernel timing events failed: %s", hipGetErrorString(err));
        *launches = (uint32_t)timed.size();
        *total_ms = sum;
    });
}

const char *pir_last_error(void) { return g_last_error.c_str(); }

const char *pir_version(void) { return "pir-rowsel-mi355x 0.1 (gfx950)"; }

pir_status pir_db_create(const pir_params *params, uint32_t layouts, pir_db **out) {
    return guarded([&] {
        PIR_REQUIRE(params != nullptr && out != nullptr, "NULL argument");
        *out = nullptr;
        validate_params(*params);
        PIR_REQUIRE(layouts != 0 && (layouts & ~(PIR_LAYOUT_VALU | PIR_LAYOUT_MFMA)) == 0,
                    "layouts must be a non-empty subset of PIR_LAYOUT_VALU | PIR_LAYOUT_MFMA");
        auto *db = new pir_db();
        try {
            db->p = *params;
            for (uint32_t l = db->p.nprimes; l < PIR_MAX_PRIMES; ++l) db->p.q[l] = 0;
            db->layouts = layouts;
            for (uint32_t l = 0; l < db->p.nprimes; ++l) {
                db->mod[l] = make_modq(db->p.q[l]);
                if (db->p.q[l] >= WIDE_Q) db->wide = true;
            }
            PIR_HIP(hipGetDevice(&db->device));
            const uint64_t words = db->slots() * db->p.d0 * db->p.d1;
            if (layouts & PIR_LAYOUT_VALU) {
                db->valu.data = static_cast<uint32_t *>(dev_alloc(words * 4));
                PIR_HIP(hipMemset(db->valu.data, 0, words * 4));
            }
            if (layouts & PIR_LAYOUT_MFMA) {
                db->mfma.kp = (db->p.d0 + 63) / 64 * 64;
                const uint64_t bytes = db->slots() * 4ull * db->p.d1 * db->mfma.kp;
                db->mfma.data = static_cast<int8_t *>(dev_alloc(bytes));
                PIR_HIP(hipMemset(db->mfma.data, 0, bytes));
            }
            PIR_HIP(hipDeviceSynchronize());
        } catch (...) {
            dev_free(db->valu.data);
            dev_free(db->mfma.data);
            delete db;
            throw;
        }
        *out = db;
    });
}

pir_status pir_db_params(const pir_db *db, pir_params *out) {
    return guarded([&] {
        PIR_REQUIRE(db && out, "NULL argument");
        *out = db->p;
    });
}

uint32_t pir_db_layouts(const pir_db *db) { return db ? db->layouts : 0; }

void pir_db_free(pir_db *db) {
    if (!db) return;
    try {
        DeviceGuard dg(db->device);
        (void)hipDeviceSynchronize();
        release_group_plans(db);
    } catch (...) {
    }
    dev_free(db->valu.data);
    dev_free(db->mfma.data);
    delete db;
}

pir_status pir_db_load_ntt(pir_db *db, const uint32_t *src, uint32_t row0, uint32_t nrows,
                           pir_domain domain, void *stream) {
    return guarded([&] {
        PIR_REQUIRE(db != nullptr, "db is NULL");
        PIR_REQUIRE(domain == PIR_DOMAIN_COEFF || domain == PIR_DOMAIN_NTT, "unknown domain %d",
                    (int)domain);
        PIR_REQUIRE((uint64_t)row0 + nrows <= db->p.d0, "rows [%u, %u) exceed d0 = %u", row0,
                    row0 + nrows, db->p.d0);
        if (nrows == 0) return;
        PIR_REQUIRE(src != nullptr, "src is NULL");
        PIR_REQUIRE(reinterpret_cast<uintptr_t>(src) % 16 == 0, "src must be 16-byte aligned");
        DeviceGuard dg(db->device);
        hipStream_t st = as_stream(stream);
        const auto &p = db->p;
        const uint64_t poly = (uint64_t)p.nprimes * p.n;          // words per record
        const uint64_t row_words = (uint64_t)p.d1 * poly;
        if (domain == PIR_DOMAIN_NTT) {
            if (env_flag("PIR_VALIDATE")) check_residues(src, nrows * row_words, p, st);
            if (db->layouts & PIR_LAYOUT_VALU) launch_db_layout_valu(*db, src, row0, nrows, st);
            if (db->layouts & PIR_LAYOUT_MFMA) launch_db_layout_mfma(*db, src, row0, nrows, st);
            return;
        }
        // coefficient domain: NTT into a stream-ordered temporary, in row chunks
        // of at most ~1 GiB, then build the layouts from it
        const uint32_t chunk = (uint32_t)std::max<uint64_t>(1, (1ull << 30) / (row_words * 4));
        const uint32_t rows_tmp = std::min(chunk, nrows);
        StreamScratch buf((size_t)rows_tmp * row_words * 4, st);
        uint32_t *tmp = buf.as<uint32_t>();
        for (uint32_t r = 0; r < nrows; r += rows_tmp) {
            const uint32_t nr = std::min(rows_tmp, nrows - r);
            const uint32_t *s = src + (uint64_t)r * row_words;
            for (uint32_t l = 0; l < p.nprimes; ++l) {
                const NttTables &t = ntt_tables(p.q[l], p.n);
                launch_ntt(s + (uint64_t)l * p.n, tmp + (uint64_t)l * p.n, (uint64_t)nr * p.d1, poly, poly,
                           t, false, st);
            }
            if (db->layouts & PIR_LAYOUT_VALU) launch_db_layout_valu(*db, tmp, row0 + r, nr, st);
            if (db->layouts & PIR_LAYOUT_MFMA) launch_db_layout_mfma(*db, tmp, row0 + r, nr, st);
        }
    });
}

pir_status pir_rowsel(const pir_db *db, const uint32_t *q, uint32_t B, uint32_t *out, pir_path path,
                      void *stream) {
    return guarded([&] {
        check_rowsel_args(db, q, B, out);
        rowsel_one(*db, q, B, out, path, as_stream(stream));
    });
}

pir_status pir_rowsel_coeff(const pir_db *db, const uint32_t *q_coeff, uint32_t B, uint32_t *out, pir_path path,
                            void *stream) {
    return guarded([&] {
        check_rowsel_args(db, q_coeff, B, out);
        rowsel_one(*db, q_coeff, B, out, path, as_stream(stream), true);
    });
}

pir_status pir_coltor_stage(const pir_params *ring, const uint32_t *ct, uint32_t B, uint32_t ncols,
                            const uint32_t *rgsw, uint32_t log2z, uint32_t ell, uint32_t *out, void *stream) {
    return guarded([&] {
        PIR_REQUIRE(ring != nullptr, "ring is NULL");
        pir_params r = *ring;
        r.d0 = r.d1 = 1;
        validate_params(r);
        coltor_check_gadget(r, log2z, ell);
        if (B == 0) return;
        PIR_REQUIRE(ncols >= 1, "ncols must be at least 1");
        PIR_REQUIRE(ct && rgsw && out, "ct, rgsw and out must not be NULL");
        const size_t LN = (size_t)r.n * r.nprimes * 4;
        const size_t nct = (size_t)B * 2 * ncols * LN, nrg = (size_t)B * 4 * ell * LN,
                     nout = (size_t)B * 2 * ((ncols + 1) / 2) * LN;
        PIR_REQUIRE(!overlaps(out, nout, ct, nct), "out overlaps ct");
        PIR_REQUIRE(!overlaps(out, nout, rgsw, nrg), "out overlaps rgsw");
        if (env_flag("PIR_VALIDATE")) {
            check_residues(ct, nct / 4, r, as_stream(stream));
            check_residues(rgsw, nrg / 4, r, as_stream(stream));
        }
        launch_coltor_stage(r, ct, B, ncols, rgsw, log2z, ell, out, as_stream(stream));
    });
}

pir_status pir_rowsel_grouped(const pir_rowsel_item *items, uint32_t count, pir_path path, void *stream) {
    return guarded([&] {
        PIR_REQUIRE(count == 0 || items != nullptr, "items is NULL");
        PIR_REQUIRE(count <= 4096, "at most 4096 items");
        int dev = 0;
        PIR_HIP(hipGetDevice(&dev));
        bool all_mfma = true;
        for (uint32_t i = 0; i < count; ++i) {
            check_rowsel_args(items[i].db, items[i].q_dev, items[i].B, items[i].out_dev);
            PIR_REQUIRE(items[i].db->device == dev, "item %u: DB lives on another device", i);
            all_mfma = all_mfma && (items[i].db->layouts & PIR_LAYOUT_MFMA);
        }
        // outputs must not overlap each other or any query
        for (uint32_t i = 0; i < count; ++i) {
            if (!items[i].B) continue;
            const auto &pi = items[i].db->p;
            const size_t oi = (size_t)items[i].B * 2 * pi.d1 * items[i].db->slots() * 4;
            for (uint32_t j = 0; j < count; ++j) {
                if (!items[j].B) continue;
                const auto &pj = items[j].db->p;
                const size_t qj = (size_t)items[j].B * 2 * pj.d0 * items[j].db->slots() * 4;
                PIR_REQUIRE(!overlaps(items[i].out_dev, oi, items[j].q_dev, qj),
                            "item %u output overlaps item %u query", i, j);
                if (j > i) {
                    const size_t oj = (size_t)items[j].B * 2 * pj.d1 * items[j].db->slots() * 4;
                    PIR_REQUIRE(!overlaps(items[i].out_dev, oi, items[j].out_dev, oj),
                                "outputs of items %u and %u overlap", i, j);
                }
            }
        }
        if (!count) return;
        hipStream_t st = as_stream(stream);
        PIR_REQUIRE(path == PIR_PATH_AUTO || path == PIR_PATH_VALU || path == PIR_PATH_MFMA_I8,
                    "unknown path %d", (int)path);
        const bool mfma = path == PIR_PATH_MFMA_I8 || (path == PIR_PATH_AUTO && all_mfma);
        if (mfma) {
            PIR_REQUIRE(all_mfma, "every DB of an MFMA grouped call needs the MFMA layout");
            if (env_flag("PIR_VALIDATE"))
                for (uint32_t i = 0; i < count; ++i)
                    check_residues(items[i].q_dev, (uint64_t)items[i].B * 2 * items[i].db->p.d0 * items[i].db->slots(),
                                   items[i].db->p, st);
            launch_rowsel_mfma_grouped(items, count, st);
        } else {
            for (uint32_t i = 0; i < count; ++i)
                rowsel_one(*items[i].db, items[i].q_dev, items[i].B, items[i].out_dev, PIR_PATH_VALU, st);
        }
    });
}

pir_status pir_rowsel_grouped_tiles(const pir_rowsel_item *items, uint32_t count, uint32_t *tiles) {
    return guarded([&] {
        PIR_REQUIRE(tiles != nullptr && (count == 0 || items != nullptr), "NULL argument");
        PIR_REQUIRE(group_plan_tiles(items, count, tiles), "no grouped plan for this item list");
    });
}

static pir_status ntt_entry(const uint32_t *in, uint32_t *out, uint32_t count, uint32_t n, uint32_t q,
                            void *stream, bool inverse) {
    return guarded([&] {
        PIR_REQUIRE(n >= 8 && n <= 16384 && (n & (n - 1)) == 0, "n must be a power of two in [8, 16384]");
        PIR_REQUIRE(q % (2 * n) == 1 && is_prime_u32(q), "q must be a prime with q = 1 mod 2n");
        if (count == 0) return;
        PIR_REQUIRE(in && out, "NULL pointer");
        const NttTables &t = ntt_tables(q, n);
        launch_ntt(in, out, count, n, n, t, inverse, as_stream(stream));
    });
}

pir_status pir_ntt_forward(const uint32_t *in, uint32_t *out, uint32_t count, uint32_t n, uint32_t q,
                           void *stream) {
    return ntt_entry(in, out, count, n, q, stream, false);
}

pir_status pir_ntt_inverse(const uint32_t *in, uint32_t *out, uint32_t count, uint32_t n, uint32_t q,
                           void *stream) {
    return ntt_entry(in, out, count, n, q, stream, true);
}

}  // extern "C"
