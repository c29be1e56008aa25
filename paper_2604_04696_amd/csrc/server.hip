// Continuous-batching RowSel server: a native host loop around the MFMA
// kernels.
//
// The DB's L*N/4 point groups are swept in `chunks` steps.  Client slot s
// owns rows 2s and 2s+1 of one shared set of query digit planes
// [L*N][4][Kp/64][mstride][64]; a step runs the persistent MFMA RowSel on one
// chunk of point groups for rows [0, 2*(highest active slot + 1)) and
// scatters each row's results to its request's output buffer.  A request is
// admitted into a free slot at a step boundary, takes part in the next
// `chunks` steps (one full sweep, starting wherever the sweep is) and then
// completes; every output word depends only on its own slot's rows, so
// results do not depend on the mix.  Slots pass FREE -> ACTIVE -> DRAINING
// (last step launched; its output pointers are cleared on the stream right
// away, so later steps cannot write to it) -> FREE (last step retired).
#include <chrono>
#include <deque>
#include <unordered_set>
#include <vector>

#include "common.h"
#include "mfma.h"
#include "modarith.h"

namespace pir {

// Staging [cp][mp][ss] of one step (cp points, starting at point p_begin of
// the DB; ss = d1 rounded up to a multiple of 4) -> per-row destinations.
// Row m holds slot m/2, component m%2; row_dst[m] is that component's
// [D1][L*N] array (0 = discard).  A block takes one row, SC_C columns and
// SC_P points and moves 16-byte vectors through a padded LDS tile: 256-byte
// read runs and 512-byte write runs (the shape the output transpose of
// single calls measured fastest; cp, p_begin and pall are multiples of 4).
constexpr int SC_P = 128, SC_C = 64;

__global__ void __launch_bounds__(256)
serve_scatter_kernel(const uint32_t *__restrict__ stage, const uint64_t *__restrict__ row_dst, uint32_t mp,
                     uint32_t d1, uint32_t ss, uint32_t cp, uint32_t p_begin, uint32_t pall, uint32_t nblk_n,
                     uint32_t nblk_p) {
    __shared__ __attribute__((aligned(16))) uint32_t tile[SC_C][SC_P + 4];   // [column][point]
    constexpr int NQ = SC_C / 4, PQ = SC_P / 4, LOADS = SC_P * NQ / 256, STORES = SC_C * PQ / 256;
    static_assert(LOADS * 256 == SC_P * NQ && STORES * 256 == SC_C * PQ, "tile divides among the threads");
    const uint32_t tid = threadIdx.x;
    uint32_t b = blockIdx.x;
    const uint32_t pb = b % nblk_p;
    b /= nblk_p;
    const uint32_t nb = b % nblk_n;
    const uint32_t m = b / nblk_n;
    uint32_t *dst = reinterpret_cast<uint32_t *>(row_dst[m]);
    if (!dst) return;   // uniform for the block
    const uint32_t p0 = pb * SC_P, n0 = nb * SC_C;
    uint4 v[LOADS];
#pragma unroll
    for (int j = 0; j < LOADS; ++j) {
        const uint32_t e = tid + 256 * j, pi = e / NQ, nq = e % NQ;
        v[j] = p0 + pi < cp && n0 + 4 * nq < d1
                   ? ld_nt(reinterpret_cast<const uint4 *>(stage + ((uint64_t)(p0 + pi) * mp + m) * ss + n0 + 4 * nq))
                   : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < LOADS; ++j) {
        const uint32_t e = tid + 256 * j, pi = e / NQ, nq = e % NQ;
        tile[4 * nq + 0][pi] = v[j].x;
        tile[4 * nq + 1][pi] = v[j].y;
        tile[4 * nq + 2][pi] = v[j].z;
        tile[4 * nq + 3][pi] = v[j].w;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < STORES; ++j) {
        const uint32_t e = tid + 256 * j, ni = e / PQ, pq = e % PQ;
        if (n0 + ni < d1 && p0 + 4 * pq < cp)
            st_nt(reinterpret_cast<uint4 *>(dst + (uint64_t)(n0 + ni) * pall + p_begin + p0 + 4 * pq),
                  *reinterpret_cast<const uint4 *>(&tile[ni][4 * pq]));
    }
}

// Writes up to ROW_UPDATES entries of the row-pointer table; the values travel
// as kernel arguments, so no host buffer has to outlive the launch.
constexpr int ROW_UPDATES = 32;
struct RowUpdates {
    uint32_t n;
    uint32_t row[ROW_UPDATES];
    uint64_t val[ROW_UPDATES];
};

__global__ void set_rows_kernel(uint64_t *row_dst, RowUpdates u) {
    const uint32_t i = threadIdx.x;
    if (i < u.n) row_dst[u.row[i]] = u.val[i];
}

static double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace pir

using namespace pir;

struct pir_server {
    enum State : uint8_t { FREE, ACTIVE, DRAINING };
    struct Slot {
        State state = FREE;
        uint64_t id = 0;
        uint32_t remaining = 0;
        double t_submit = 0, t_admit = 0;
    };
    struct Pending {
        pir_request r;
        double t_submit;
    };
    struct Step {
        hipEvent_t ev;
        std::vector<uint32_t> finishing;
    };

    const pir_db *db = nullptr;
    int device = 0;
    hipStream_t st = nullptr;
    uint32_t capacity = 0, chunks = 0, pipeline = 1, cg = 0, gall = 0, mstride = 0, max_waiting = 0;
    uint64_t device_bytes = 0;
    int8_t *qd = nullptr;
    uint32_t *stage = nullptr;
    uint64_t *row_dst_dev = nullptr;    // per row: destination of its results (0 = discard)
    RowUpdates pending_rows{};          // table updates not yet launched
    std::vector<Slot> slots;
    std::deque<Pending> waitq;
    std::deque<Step> inflight;
    std::deque<pir_completion> done;
    std::unordered_set<uint64_t> live_ids;   // ids submitted whose completion is not yet returned
    std::vector<hipEvent_t> spare_events;
    uint64_t next_chunk = 0, steps = 0, admitted = 0, completed = 0;

    ~pir_server() {
        int prev = -1;
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (device_bytes || st) {
            (void)hipSetDevice(device);
            if (st) (void)hipStreamSynchronize(st);
        }
        for (auto &s : inflight) (void)hipEventDestroy(s.ev);
        for (auto e : spare_events) (void)hipEventDestroy(e);
        dev_free(qd);
        dev_free(stage);
        dev_free(row_dst_dev);
        if (st) (void)hipStreamDestroy(st);
        if (prev >= 0) (void)hipSetDevice(prev);
    }

    // device bytes for `cap` client slots
    uint64_t bytes_for(uint32_t cap) const {
        const uint64_t P = db->slots(), ms = (2ull * cap + 127) / 128 * 128;
        return P * 4 * db->mfma.kp * ms + (uint64_t)cg * ms * staging_stride(db->p.d1) * 16 + ms * 8 + 4096;
    }

    void flush_rows() {
        if (!pending_rows.n) return;
        set_rows_kernel<<<1, ROW_UPDATES, 0, st>>>(row_dst_dev, pending_rows);
        PIR_LAUNCH_CHECK();
        pending_rows.n = 0;
    }

    void set_rows(uint32_t s, const uint32_t *out) {
        const uint64_t comp = out ? (uint64_t)db->p.d1 * db->slots() : 0;   // words per component
        if (pending_rows.n + 2 > ROW_UPDATES) flush_rows();
        RowUpdates &u = pending_rows;
        u.row[u.n] = 2 * s;
        u.val[u.n++] = out ? reinterpret_cast<uint64_t>(out) : 0;
        u.row[u.n] = 2 * s + 1;
        u.val[u.n++] = out ? reinterpret_cast<uint64_t>(out + comp) : 0;
    }

    void retire() {
        while (!inflight.empty()) {
            const hipError_t e = hipEventQuery(inflight.front().ev);
            if (e == hipErrorNotReady) {
                (void)hipGetLastError();   // not an error: clear it
                break;
            }
            if (e != hipSuccess) PIR_FAIL(PIR_EDEVICE, "serving step failed: %s", hipGetErrorString(e));
            const double t = now_s();
            for (uint32_t s : inflight.front().finishing) {
                Slot &sl = slots[s];
                done.push_back(pir_completion{sl.id, PIR_OK, 0, sl.t_submit, sl.t_admit, t});
                sl.state = FREE;
                ++completed;
            }
            spare_events.push_back(inflight.front().ev);
            inflight.pop_front();
        }
    }

    void admit() {
        for (uint32_t s = 0; s < capacity && !waitq.empty(); ++s) {
            if (slots[s].state != FREE) continue;
            const Pending pr = waitq.front();
            waitq.pop_front();
            Slot &sl = slots[s];
            sl.state = ACTIVE;
            sl.id = pr.r.id;
            sl.remaining = chunks;
            sl.t_submit = pr.t_submit;
            sl.t_admit = now_s();
            launch_query_digits_rows(*db, pr.r.q_dev, 2, qd, mstride, 2 * s, st);
            set_rows(s, pr.r.out_dev);
            ++admitted;
        }
        flush_rows();
    }

    // launches the next step if any client is active; returns false otherwise
    bool launch_step() {
        uint32_t hi = 0;
        bool any = false;
        for (uint32_t s = 0; s < capacity; ++s)
            if (slots[s].state == ACTIVE) {
                hi = s;
                any = true;
            }
        if (!any) return false;
        const uint32_t rows = 2 * (hi + 1);
        const uint32_t c = (uint32_t)(next_chunk++ % chunks);
        const uint32_t g_begin = c * cg, ng = std::min(cg, gall - g_begin);
        // the tile shape that pads the fewest output words for this many rows
        // (32 x 256 while at most 16 clients are active: all eight waves on
        // useful sub-tiles, 256 DB columns per pipeline stage)
        // (or the query-resident kernel when the rows fill its units)
        const uint32_t mp = (rows + 31) / 32 * 32;
        MfmaJob job;
        if (qres_preferred(mp, db->mfma.kp / 64)) {
            job = make_qres_job(*db, qd, mstride, stage, hi + 1, qres_shape_for(mp));
            job.g_begin = g_begin;
            job.groups = ng;
            job.tiles = 4 * ng * job.nblk_m * job.nblk_n;
            KernelTimer::Scope timed(st);
            launch_mfma_qres(job, st);
        } else {
            uint32_t pts = 1, wm = 2;
            bool deep = true;
            pick_shape(mp, db->p.d1, &pts, &wm, &deep);
            job = make_shaped_job(*db, qd, stage, hi + 1, pts, wm);
            job.mstride = mstride;
            job.g_begin = g_begin;
            job.groups = ng;
            job.tiles = ng * job.nblk_m * job.nblk_n;
            KernelTimer::Scope timed(st);
            launch_mfma_grouped(job, nullptr, 1, job.tiles, job.split, deep, st);
        }
        const uint32_t cp = 4 * ng, nblk_n = (db->p.d1 + SC_C - 1) / SC_C, nblk_p = (cp + SC_P - 1) / SC_P;
        const uint64_t blocks = (uint64_t)rows * nblk_n * nblk_p;
        PIR_REQUIRE(blocks < (1ull << 31), "scatter launch too large");
        serve_scatter_kernel<<<(uint32_t)blocks, 256, 0, st>>>(stage, row_dst_dev, job.mp, db->p.d1, job.sstride,
                                                               cp, 4 * g_begin, 4 * gall, nblk_n, nblk_p);
        PIR_LAUNCH_CHECK();
        Step step;
        for (uint32_t s = 0; s < capacity; ++s) {
            Slot &sl = slots[s];
            if (sl.state != ACTIVE) continue;
            if (--sl.remaining == 0) {
                sl.state = DRAINING;
                step.finishing.push_back(s);
                set_rows(s, nullptr);   // later steps must not write to this request any more
            }
        }
        flush_rows();
        if (spare_events.empty()) {
            hipEvent_t e;
            PIR_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            spare_events.push_back(e);
        }
        step.ev = spare_events.back();
        spare_events.pop_back();
        PIR_HIP(hipEventRecord(step.ev, st));
        inflight.push_back(std::move(step));
        ++steps;
        return true;
    }
};

extern "C" {

double pir_clock(void) { return now_s(); }

pir_status pir_server_create(const pir_db *db, const pir_server_opts *opts, pir_server **out) {
    return guarded([&] {
        PIR_REQUIRE(db && out, "NULL argument");
        *out = nullptr;
        PIR_REQUIRE(db->layouts & PIR_LAYOUT_MFMA, "the server needs a DB with the MFMA layout");
        pir_server_opts o{};
        if (opts) o = *opts;
        const uint32_t max_clients = o.max_clients ? o.max_clients : 256;
        PIR_REQUIRE(max_clients <= 4096, "max_clients must be <= 4096");
        PIR_REQUIRE(o.pipeline <= 4, "pipeline must be 1..4");
        DeviceGuard dg(db->device);
        auto *srv = new pir_server();
        try {
            srv->db = db;
            srv->device = db->device;
            srv->pipeline = o.pipeline ? o.pipeline : 1;
            srv->max_waiting = o.max_waiting;
            srv->gall = (uint32_t)(db->slots() / 4);
            uint32_t chunks = o.chunks ? o.chunks : 16;
            PIR_REQUIRE(chunks <= srv->gall, "chunks must be <= L*N/4 = %u", srv->gall);
            srv->cg = (srv->gall + chunks - 1) / chunks;
            srv->chunks = (srv->gall + srv->cg - 1) / srv->cg;
            uint64_t budget = o.hbm_budget;
            if (!budget) {
                size_t fr = 0, tot = 0;
                PIR_HIP(hipMemGetInfo(&fr, &tot));
                budget = (uint64_t)(fr * 0.9);
            }
            uint32_t cap = max_clients;
            while (cap > 0 && srv->bytes_for(cap) > budget) cap = cap > 64 ? cap - cap / 16 : cap - 1;
            if (!cap) PIR_FAIL(PIR_ENOMEM, "budget of %llu bytes holds no client (one needs %llu)",
                               (unsigned long long)budget, (unsigned long long)srv->bytes_for(1));
            srv->capacity = cap;
            srv->mstride = (2 * cap + 127) / 128 * 128;
            const uint64_t P = db->slots();
            srv->qd = static_cast<int8_t *>(dev_alloc(P * 4 * db->mfma.kp * srv->mstride));
            srv->stage = static_cast<uint32_t *>(
                dev_alloc((uint64_t)srv->cg * srv->mstride * staging_stride(db->p.d1) * 16));
            srv->row_dst_dev = static_cast<uint64_t *>(dev_alloc((uint64_t)srv->mstride * 8));
            srv->device_bytes = srv->bytes_for(cap);
            // every row starts as "discard"; query rows start zeroed
            PIR_HIP(hipMemset(srv->qd, 0, P * 4 * db->mfma.kp * srv->mstride));
            PIR_HIP(hipMemset(srv->row_dst_dev, 0, (size_t)srv->mstride * 8));
            PIR_HIP(hipDeviceSynchronize());
            PIR_HIP(hipStreamCreateWithFlags(&srv->st, hipStreamNonBlocking));
            srv->slots.resize(cap);
        } catch (...) {
            delete srv;
            throw;
        }
        *out = srv;
    });
}

pir_status pir_serve_step(pir_server *srv, const pir_request *arrivals, uint32_t n_arrivals,
                          pir_completion *done, uint32_t cap, uint32_t *n_done) {
    return guarded([&] {
        PIR_REQUIRE(srv != nullptr, "server is NULL");
        PIR_REQUIRE(n_arrivals == 0 || arrivals != nullptr, "arrivals is NULL");
        PIR_REQUIRE(cap == 0 || done != nullptr, "done is NULL");
        if (n_done) *n_done = 0;
        DeviceGuard dg(srv->device);
        const double t = now_s();
        const auto &p = srv->db->p;
        const size_t qb = (size_t)2 * p.d0 * srv->db->slots() * 4, ob = (size_t)2 * p.d1 * srv->db->slots() * 4;
        {
            // ids must be unique among live requests: checked before anything is queued
            std::unordered_set<uint64_t> fresh;
            for (uint32_t i = 0; i < n_arrivals; ++i)
                PIR_REQUIRE(!srv->live_ids.count(arrivals[i].id) && fresh.insert(arrivals[i].id).second,
                            "request id %llu is already live", (unsigned long long)arrivals[i].id);
        }
        for (uint32_t i = 0; i < n_arrivals; ++i) {
            const pir_request &r = arrivals[i];
            srv->live_ids.insert(r.id);   // every arrival gets exactly one completion
            const auto qa = reinterpret_cast<uintptr_t>(r.q_dev), oa = reinterpret_cast<uintptr_t>(r.out_dev);
            const bool bad = !r.q_dev || !r.out_dev || qa % 16 || oa % 16 || (qa < oa + ob && oa < qa + qb);
            if (bad) {
                srv->done.push_back(pir_completion{r.id, PIR_EINVAL, 0, t, t, t});
                continue;
            }
            if (srv->max_waiting && srv->waitq.size() >= srv->max_waiting) {
                srv->done.push_back(pir_completion{r.id, PIR_EBUSY, 0, t, t, t});
                continue;
            }
            // the query's producer: later reads on the server stream wait for it
            if (r.ready_event) PIR_HIP(hipStreamWaitEvent(srv->st, reinterpret_cast<hipEvent_t>(r.ready_event), 0));
            srv->waitq.push_back({r, t});
        }
        srv->retire();
        while (srv->inflight.size() < srv->pipeline) {
            srv->admit();
            if (!srv->launch_step()) break;
        }
        uint32_t k = 0;
        while (k < cap && !srv->done.empty()) {
            done[k++] = srv->done.front();
            srv->live_ids.erase(srv->done.front().id);
            srv->done.pop_front();
        }
        if (n_done) *n_done = k;
    });
}

pir_status pir_server_get_stats(const pir_server *srv, pir_server_stats *out) {
    return guarded([&] {
        PIR_REQUIRE(srv && out, "NULL argument");
        pir_server_stats s{};
        s.capacity = srv->capacity;
        for (const auto &sl : srv->slots) s.active += sl.state == pir_server::ACTIVE;
        s.waiting = (uint32_t)srv->waitq.size();
        s.inflight = (uint32_t)srv->inflight.size();
        s.steps = srv->steps;
        s.admitted = srv->admitted;
        s.completed = srv->completed;
        s.device_bytes = srv->device_bytes;
        *out = s;
    });
}

void pir_server_destroy(pir_server *srv) { delete srv; }

}  // extern "C"
