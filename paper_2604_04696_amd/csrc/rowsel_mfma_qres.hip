// RowSel on the INT8 matrix cores, query-resident form, for 64 query rows
// and more (2B >= 33; above 128 rows in blocks of the unit's height).
//
// The arithmetic is that of rowsel_mfma.hip (four balanced signed digits per
// residue, sixteen digit products summed per weight class s = i + j in int32,
// exact binary64 recombination per output, a class flush every 2048 rows of
// k).  What differs is the data flow and the MFMA shape.  A work unit is one
// point, BM query rows and BN DB columns; every wave owns RS x RN sub-tiles
// of 16 x 16 outputs (RS along m, RN along n) and multiplies its B fragments
// (per DB digit, one per 16 columns) against the RS query fragments of each
// query digit with v_mfma_i32_16x16x64_i8, so a DB fragment feeds RS and a
// query fragment RN MFMAs per digit pair.  Per 64-row chunk of k the block
// copies the query chunk (four digits x BM rows) and the DB chunk into LDS
// rings; with one row group of waves (units of 32 or 64 rows x 128 columns)
// each wave loads its own 16 columns into a ring of its own, with several
// (96 x 64 and 128 x 64 units) the block shares one DB ring, since every row
// group reads the same columns.  The 32 x 128 unit is kept for tuning and
// grouped plans: with 32 rows it ties with the tiled kernel.  Every wave
// holds seven class accumulators per sub-tile: 112 registers for the four
// sub-tiles of the 64- and 128-row units, as in the tiled kernel.
//
// Operand layout of v_mfma_i32_16x16x64_i8: lane l supplies row (A) or
// column (B) l % 16 and the 16 bytes of k-group l / 16 of the 64-row chunk;
// the same k mapping holds for both operands, so a 16-byte run of k per lane
// on both sides pairs every query digit with the DB digit of the same k.
// Element r of a lane's result is row 4 (l / 16) + r, column l % 16.
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "common.h"
#include "modarith.h"
#include "mfma.h"

namespace pir {

namespace {

typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;

constexpr int QKCH = 64;                            // k rows per chunk
constexpr int QWAVES = 8;                           // waves per block
constexpr int DBCH = 4 * 1024;                      // bytes of one wave's DB chunk (4 digits x 16 columns)
constexpr int LDS_BYTES = 160 * 1024;
constexpr uint32_t QKSUPER = 2048;                  // rows of k per int32 accumulation

// RS 16-row sub-tiles per wave, WR row groups of waves, NQ query chunk
// buffers per block, RING DB chunks per wave (RING - 1 = PF in flight).
// SHDB: one DB ring for the block (the row groups share the columns),
// else one per wave.
template <int RS_, int WR_, int NQ_, int RING_, bool SHDB_ = false, int RN_ = 1>
struct QShape {
    static constexpr int RS = RS_;
    static constexpr int RN = RN_;                       // 16-column sub-tiles per wave
    static constexpr int WR = WR_;
    static constexpr int NQ = NQ_;
    static constexpr int RING = RING_;
    static constexpr bool SHDB = SHDB_;
    static constexpr int PF = RING - 1;
    static constexpr int BM = 16 * RS * WR;              // query rows of a unit
    static constexpr int WC = QWAVES / WR;               // waves per row group
    static constexpr int BN = 16 * RN * WC;              // DB columns of a unit
    static constexpr int QCH = 4 * BM * QKCH;            // bytes of one query chunk (four digits)
    static constexpr int QL = QCH / 1024 / QWAVES;       // 1 KiB query loads per wave and chunk
    static constexpr int DBS = SHDB ? 4 * BN * QKCH : QWAVES * DBCH;   // bytes of one DB ring slot, all waves
    static constexpr int DL = SHDB ? DBS / 1024 / QWAVES : 4;          // 1 KiB DB loads per wave and chunk
    static constexpr int DB_LDS = NQ * QCH;              // offset of the DB ring
    static_assert(QL >= 1 && QL * QWAVES * 1024 == QCH, "query chunk loads");
    static_assert(DL >= 1 && (!SHDB || DL * QWAVES * 1024 == DBS), "DB chunk loads");
    static_assert(DB_LDS + RING * DBS <= LDS_BYTES, "LDS");
    static_assert(PF >= 1 && (SHDB || (PF <= NQ && PF >= NQ - 1)) && NQ >= 2, "pipeline depths");
    static_assert(RN == 1 || SHDB, "a wave's own DB ring holds 16 columns");
};

template <int N>
__device__ __forceinline__ void qwait_vmcnt() {
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

__device__ __forceinline__ void qbarrier() { asm volatile("s_barrier" ::: "memory"); }

// Unit u of a job: u = (point * nblk_m + mb) * nblk_n + nb, points in the
// job's order (4 * group + s, groups from g_begin), as in the staging layout.
struct QUnit {
    uint64_t p;       // global point l * N + j
    uint32_t pl;      // point index inside the job (staging row block)
    uint32_t l;       // prime
    uint32_t m0, n0;  // first query row, first DB column
};

__device__ __forceinline__ QUnit decode_unit(uint32_t u, const MfmaJob &J, uint32_t bm, uint32_t bn) {
    QUnit r;
    const uint32_t nb = u % J.nblk_n;
    u /= J.nblk_n;
    const uint32_t mb = u % J.nblk_m;
    r.pl = u / J.nblk_m;
    const uint32_t G = J.N / 4, gg = J.g_begin + r.pl / 4;
    r.l = gg / G;
    r.p = (uint64_t)r.l * J.N + 4 * (gg % G) + r.pl % 4;
    r.m0 = mb * bm;
    r.n0 = nb * bn;
    return r;
}

// Persistent block (one per CU): units T = (i*8 + x)*per_xcd + y for
// i = 0, 1, ..., x the block's XCD, y its index there, so the units in flight
// on one XCD are consecutive and the blocks working on one point share its
// query planes in that XCD's L2.
//
// LDS: a ring of NQ query chunks (all four digits of BM rows for 64 rows of
// k) shared by the block and a ring of RING DB chunks (four digits of the
// unit's columns; per wave, its 16 columns, or shared).  Every operand moves
// global -> LDS with global_load_lds_dwordx4 and every wait for those loads
// is explicit: a wave's vector-memory operations retire in issue order, so a
// wave waits for a load by waiting until no more than the count issued after
// it are outstanding.  Chunk step t of a block:
//   1. waits for its loads of query chunk t (issued NQ - 1 steps earlier;
//      everything issued before them is then done too, which is at most
//      DB chunk t - NQ + PF <= t: nothing the step does not need anyway) --
//      with the shared DB ring also for its loads of DB chunk t -- and meets
//      the block at a barrier, after which the buffers read in step t - 1
//      are free;
//   2. issues its loads of query chunk t + NQ - 1 and of DB chunk t + PF
//      (PF = RING - 1) into those buffers;
//   3. with its own DB ring, waits for its DB chunk t (PF steps' loads were
//      issued after it; in the first PF steps it waits for everything);
//   4. reads the four digits' B fragments and, per query digit, the RS A
//      fragments (the next digit's read while the MFMAs of this one run),
//      and issues 16 RS v_mfma_i32_16x16x64_i8 into the seven class
//      accumulators.
// A wave's own DB ring streams PF chunks ahead with no barrier of its own.
// Both load cursors run over the block's units ahead of the MFMAs; the host
// requires nkc >= NQ - 1 and nkc >= PF so that neither is more than one unit
// ahead, and past the last unit they reload their last chunk into buffers
// nobody reads.
template <class S, int MODE>
__global__ void __launch_bounds__(64 * QWAVES) __attribute__((amdgpu_waves_per_eu(2, 2)))
rowsel_mfma_qres_kernel(const MfmaJob J) {
    constexpr int RS = S::RS, RN = S::RN, WR = S::WR, BM = S::BM, BN = S::BN, NQ = S::NQ, RING = S::RING,
                  PF = S::PF;
    constexpr int QCH = S::QCH, QL = S::QL, DBL = S::DL, DBS = S::DBS;
    constexpr bool SHDB = S::SHDB;
    __shared__ __attribute__((aligned(1024))) int8_t lds[LDS_BYTES];

    const uint32_t lane = threadIdx.x % 64;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    const uint32_t wr = wv / S::WC, wc = wv % S::WC;
    const uint32_t per_xcd = gridDim.x / 8, xcd = blockIdx.x % 8, yi = blockIdx.x / 8;
    auto unit_of = [&](uint32_t i) { return (i * 8 + xcd) * per_xcd + yi; };
    const uint32_t units = J.tiles, nkc = J.nkc, d1 = J.d1;
    if (unit_of(0) >= units) return;   // uniform over the block
    const uint64_t qplane = (uint64_t)J.mstride * QKCH, dplane = (uint64_t)d1 * QKCH;
    const uint64_t qstride = (uint64_t)nkc * qplane, dstride = (uint64_t)nkc * dplane;   // digit plane sets

    // Query load j of a chunk moves 16 rows of one digit, placed at byte
    // v * 1024 of the buffer, v = wv + j * QWAVES = d * (BM / 16) + rb.  A
    // lane moves 16 bytes; chunk c of local row r sits at position
    // c ^ ((r >> 1) & 3), hence the lane's source offset.  A fragment read
    // (16 rows at one chunk index) is then free of bank conflicts; with
    // c ^ ((r >> 2) & 3), the tiled kernel's swizzle for its 32-row
    // fragments, every read here took two passes (counters: 4 conflict
    // cycles per read, none with this one).
    const uint32_t qlane = (lane / 4) * QKCH + ((lane % 4) ^ ((lane / 8) & 3)) * 16;
    const uint32_t arow = wr * 16 * RS + lane % 16;
    const uint32_t a_lane = arow * QKCH + ((lane / 16) ^ ((arow >> 1) & 3)) * 16;
    // DB ring: per wave, slot k of wave w at k * DBS + w * 4 KiB, digit d
    // at + d KiB, the lane's 16 bytes at + lane * 16 (what it loaded itself);
    // shared, slot k at k * DBS, digit d at + d * BN * 64, column c at + c * 64
    // with the same chunk swizzle as the query (load v of a chunk is 16
    // columns of one digit: v = d * (BN / 16) + cq).
    int8_t *const ring = lds + S::DB_LDS + (SHDB ? 0 : wv * DBCH);
    const uint32_t bcol = wc * 16 * RN + lane % 16;
    const uint32_t b_lane = SHDB ? bcol * QKCH + ((lane / 16) ^ ((bcol >> 1) & 3)) * 16 : lane * 16;
    auto q_base = [&](const QUnit &u) { return J.qd + u.p * 4 * qstride + (uint64_t)u.m0 * QKCH + qlane; };
    // per-lane source of DB load j (columns past D1 are never stored); a
    // wave's own ring takes the four digits at one source plus j digit planes
    constexpr int DP = SHDB ? DBL : 1;
    auto d_base = [&](const QUnit &u, int j) {
        if (SHDB) {
            const uint32_t v = wv + j * QWAVES, d = v / (BN / 16), cq = v % (BN / 16);
            const uint32_t n = u.n0 + cq * 16 + lane / 4;
            return J.dbd + u.p * 4 * dstride + d * dstride + (uint64_t)min(n, d1 - 1) * QKCH + (qlane % QKCH);
        }
        const uint32_t n = u.n0 + wc * 16 * RN + lane % 16;
        return J.dbd + u.p * 4 * dstride + (uint64_t)min(n, d1 - 1) * QKCH + (lane / 16) * 16;
    };
    // the unit after iteration i (iteration i's own past the last one)
    auto next_unit = [&](uint32_t i) {
        const uint32_t u = unit_of(i + 1);
        return decode_unit(u < units ? u : unit_of(i), J, BM, BN);
    };

    uint32_t ci = 0;
    QUnit cu = decode_unit(unit_of(0), J, BM, BN);
    QUnit nu = next_unit(0);

    // ---- query cursor: chunk q_kc of the unit at q_cur, into buffer q_buf.
    // q_kc == nkc: past the unit's end; the next issue moves to q_nxt unless
    // q_last (the unit after q_cur is not known yet, or there is none), and
    // with no unit to move to it reloads the last chunk.
    const int8_t *q_cur = q_base(cu), *q_nxt = q_base(nu);
    uint32_t q_kc = 0, q_buf = 0;
    bool q_last = unit_of(1) >= units;
    auto q_issue = [&]() {
        if (q_kc == nkc && !q_last) {
            q_cur = q_nxt;
            q_kc = 0;
            q_last = true;   // until the compute cursor names the unit after it
        }
        const int8_t *src = q_cur + min(q_kc, nkc - 1) * qplane;
        int8_t *dst = lds + q_buf * QCH;
#pragma unroll
        for (int j = 0; j < QL; ++j) {
            const uint32_t v = wv + j * QWAVES, d = v / (BM / 16), rb = v % (BM / 16);
            const int8_t *from = src + d * qstride + rb * 1024;
            lds_void *to = (lds_void *)(dst + v * 1024);
            __builtin_amdgcn_global_load_lds(from, to, 16, 0, 0);
        }
        q_buf = q_buf + 1 == NQ ? 0 : q_buf + 1;
        q_kc += q_kc < nkc;
    };

    // ---- DB cursor: chunk d_kc of the unit at d_cur, into ring slot d_slot
    // (as the query cursor)
    const int8_t *d_cur[DP], *d_nxt[DP];
#pragma unroll
    for (int j = 0; j < DP; ++j) {
        d_cur[j] = d_base(cu, j);
        d_nxt[j] = d_base(nu, j);
    }
    uint32_t d_kc = 0, d_slot = 0;
    bool d_last = q_last;
    auto d_issue = [&]() {
        if (d_kc == nkc && !d_last) {
#pragma unroll
            for (int j = 0; j < DP; ++j) d_cur[j] = d_nxt[j];
            d_kc = 0;
            d_last = true;
        }
        const uint64_t off = min(d_kc, nkc - 1) * dplane;
        int8_t *dst = ring + d_slot * DBS;
#pragma unroll
        for (int j = 0; j < DBL; ++j) {
            const int8_t *from = SHDB ? d_cur[j % DP] + off : d_cur[0] + off + j * dstride;
            lds_void *to = (lds_void *)(dst + (SHDB ? (wv + j * QWAVES) : j) * 1024);
            __builtin_amdgcn_global_load_lds(from, to, 16, 0, 0);
        }
        d_slot = d_slot + 1 == RING ? 0 : d_slot + 1;
        d_kc += d_kc < nkc;
    };

    i32x4 acc[7][RS * RN];
    auto zero_acc = [&]() {
#pragma unroll
        for (int c = 0; c < 7; ++c)
#pragma unroll
            for (int t = 0; t < RS * RN; ++t) acc[c][t] = (i32x4){0, 0, 0, 0};
    };
    zero_acc();

    // Recombination of the classes into the staging layout [point][mp][sstride]
    // (every QKSUPER rows of k and at the unit's end; a later flush of the
    // unit adds to what the earlier ones stored); each store moves four
    // 64-byte row pieces.
    auto flush = [&](bool first, bool last) {
        const EpiQ mq = J.q[cu.l];
        uint32_t *pt = J.out + (uint64_t)cu.pl * J.mp * J.sstride;
#pragma unroll
        for (int t = 0; t < RS * RN; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint32_t rs = t / RN, n = cu.n0 + wc * 16 * RN + (t % RN) * 16 + lane % 16;
                int gr[7];
#pragma unroll
                for (int c = 0; c < 7; ++c) gr[c] = acc[c][t][r];
                uint32_t v = combine_classes<MODE>(gr, mq);
                const uint32_t m = cu.m0 + wr * 16 * RS + rs * 16 + 4 * (lane / 16) + r;
                if (m < J.mp && n < d1) {
                    uint32_t *o = pt + (uint64_t)m * J.sstride + n;
                    if (!first) v = MODE == RECOMB_WIDE ? add_mod_w(*o, v, mq.q) : add_mod(*o, v, mq.q);
                    if (last) __builtin_nontemporal_store(v, o);
                    else *o = v;
                }
            }
        zero_acc();
    };

    // ---- prologue: query chunks 0 .. NQ - 2, then DB chunks 0 .. PF - 1
#pragma unroll
    for (int k = 0; k + 1 < NQ; ++k) q_issue();
#pragma unroll
    for (int k = 0; k < PF; ++k) d_issue();

    uint32_t c_buf = 0, c_slot = 0;   // query buffer and LDS ring slot of the chunk being computed
    uint32_t gstep = 0;               // chunk steps of this block so far

    // loads issued after the later of this wave's loads of query chunk t
    // (step t - NQ + 1, first in its step) and of DB chunk t (step t - PF,
    // second): with a shared DB ring both must have landed at the barrier
    constexpr int AFTER_BOTH = PF > NQ - 1 ? DBL + (NQ - 2) * (QL + DBL) : (PF - 1) * (QL + DBL);
    auto step = [&]() {
        if constexpr (SHDB) {
            // 1. this wave's loads of query and DB chunk t, then everybody's
            if (gstep < (uint32_t)(PF > NQ ? PF : NQ)) qwait_vmcnt<0>();
            else qwait_vmcnt<AFTER_BOTH>();
            ++gstep;
            qbarrier();
            // 2.
            q_issue();
            d_issue();
        } else {
            // 1. query chunk t: after its loads, this wave issued one step's
            //    DB loads and NQ - 2 steps' query and DB loads
            qwait_vmcnt<DBL + (NQ - 2) * (QL + DBL)>();
            qbarrier();
            // 2.
            q_issue();
            d_issue();
            // 3. DB chunk t: PF steps' loads were issued after it
            if (gstep < PF) qwait_vmcnt<0>();
            else qwait_vmcnt<PF * (QL + DBL)>();
            ++gstep;
        }
        // 4.
        const int8_t *bb = ring + c_slot * DBS + b_lane;
        c_slot = c_slot + 1 == RING ? 0 : c_slot + 1;
        i32x4 b[4][RN];
#pragma unroll
        for (int d = 0; d < 4; ++d)
#pragma unroll
            for (int rn = 0; rn < RN; ++rn)
                b[d][rn] = *reinterpret_cast<const i32x4 *>(bb + d * (SHDB ? BN * QKCH : 1024) + rn * 16 * QKCH);
        // query digit i's RS fragments go to buffer i % 2, two digits ahead
        // of their MFMAs, so each digit's reads overlap the previous digit's
        // MFMAs
        const int8_t *ab = lds + c_buf * QCH + a_lane;
        c_buf = c_buf + 1 == NQ ? 0 : c_buf + 1;
        i32x4 a[2][RS];
        auto read_a = [&](int i) {
#pragma unroll
            for (int rs = 0; rs < RS; ++rs)
                a[i % 2][rs] = *reinterpret_cast<const i32x4 *>(ab + (i * BM + rs * 16) * QKCH);
        };
        read_a(0);
        read_a(1);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int rs = 0; rs < RS; ++rs)
#pragma unroll
                    for (int rn = 0; rn < RN; ++rn)
                        acc[i + j][rs * RN + rn] = __builtin_amdgcn_mfma_i32_16x16x64_i8(
                            a[i % 2][rs], b[j][rn], acc[i + j][rs * RN + rn], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
            if (i + 2 < 4) {
                read_a(i + 2);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    };

    constexpr uint32_t SUPER = QKSUPER / QKCH;
    while (true) {
        // the unit's k in runs of SUPER chunks, each ending in a flush
        for (uint32_t kc1 = 0; kc1 < nkc; kc1 += SUPER) {
            const uint32_t kend = min(kc1 + SUPER, nkc);
            for (uint32_t kc = kc1; kc < kend; ++kc) step();
            flush(kc1 == 0, kend == nkc);
        }
        if (unit_of(++ci) >= units) break;
        // the load cursors are in unit ci by now (they moved into it while
        // the MFMAs were in unit ci - 1 and wait for the unit after it)
        cu = nu;
        nu = next_unit(ci);
        const bool more = unit_of(ci + 1) < units;
        q_nxt = q_base(nu);
#pragma unroll
        for (int j = 0; j < DP; ++j) d_nxt[j] = d_base(nu, j);
        q_last = !more;
        d_last = !more;
    }
    qwait_vmcnt<0>();   // the trailing loads land before the block ends
}

int qres_cu_count() {
    static int cached = 0;
    if (!cached) {
        int dev = 0;
        PIR_HIP(hipGetDevice(&dev));
        PIR_HIP(hipDeviceGetAttribute(&cached, hipDeviceAttributeMultiprocessorCount, dev));
    }
    return cached;
}

}  // namespace

// Unit shapes (sub-tiles per wave RS x RN, WR row groups; query buffers, DB
// ring slots): 32 x 128, 64 x 128, 96 x 64 and 128 x 64, the last two with one
// DB ring for the block.  Measured on the 512 x 512, N = 4096 DB (GEMM
// alone): the 128-row unit with 4 x 1 sub-tiles per wave (each wave all 64
// rows of 16 columns) and per-wave DB rings, which load each column twice,
// took 4.28 ms for 64 clients, with one shared ring 4.16 ms, and with 2 x 2
// sub-tiles per wave (a fifth fewer LDS fragment reads) 4.05-4.14 ms against
// 4.18-4.26 ms on the same boxes; the 96-row unit took 3.15-3.30 ms for 33 to
// 48 clients, where 128-row units took 3.71-4.18 ms.  A 64 x 128 unit with
// 2 x 2 sub-tiles and a shared ring tied with the 4 x 1 form.
struct QVariant {
    uint32_t rs, wr, nq, ring, rn;
    uint32_t rows() const { return 16 * rs * wr; }
    uint32_t cols() const { return 16 * rn * (QWAVES / wr); }
    uint32_t min_chunks() const { return std::max(nq - 1, ring - 1); }
};
static const QVariant QRES[] = {{2, 1, 3, 4, 1}, {4, 1, 3, 3, 1}, {3, 2, 3, 3, 1}, {2, 4, 2, 3, 2}};
constexpr uint32_t NQRES = sizeof(QRES) / sizeof(QRES[0]);
uint32_t qres_shape_count() { return NQRES; }
uint32_t qres_min_chunks(uint32_t shape) { return QRES[shape].min_chunks(); }

// PIR_MFMA_KERNEL=qres or tile forces a kernel, else the query-resident one
// from 64 rows up (measured on the 512 x 512, N = 4096 DB: 64 rows 2.17 ms
// against 2.43 ms tiled, 96 rows 3.3 against 4.0, 128 rows 4.1 against 4.6;
// with 32 rows the two tie).
bool qres_preferred(uint32_t mp, uint32_t nkc) {
    if (nkc < qres_min_chunks(qres_shape_for(mp))) return false;
    if (const char *e = std::getenv("PIR_MFMA_KERNEL")) {
        if (!std::strcmp(e, "qres")) return true;
        if (!std::strcmp(e, "tile")) return false;
    }
    return mp >= 64;
}

// The unit for mp rows: the one of mp's height up to 128 rows; above, the
// 64-, 96- or 128-row unit with the fewest rows computed (the taller one on
// a tie: the GEMM's time per computed row is about the same for the three).
uint32_t qres_shape_for(uint32_t mp) {
    if (const char *e = std::getenv("PIR_QRES_VARIANT")) {   // tuning runs
        const int v = std::atoi(e);
        if (v >= 0 && (uint32_t)v < NQRES && QRES[v].rows() >= std::min(mp, 128u)) return (uint32_t)v;
    }
    if (mp <= 128) return mp <= 32 ? 0u : mp <= 64 ? 1u : mp <= 96 ? 2u : 3u;
    auto computed = [&](uint32_t s2) { return (mp + QRES[s2].rows() - 1) / QRES[s2].rows() * QRES[s2].rows(); };
    uint32_t best = 3;
    for (uint32_t s2 : {2u, 1u})
        if (computed(s2) < computed(best)) best = s2;
    return best;
}
uint32_t qres_rows(uint32_t shape) { return QRES[shape].rows(); }
uint32_t qres_cols(uint32_t shape) { return QRES[shape].cols(); }

MfmaJob make_qres_job(const pir_db &db, const int8_t *qd, uint32_t mstride, uint32_t *stage, uint32_t B,
                      uint32_t shape) {
    MfmaJob j = make_mfma_job(db, qd, stage, B, 0, 2);
    const uint32_t bm = qres_rows(shape), bn = qres_cols(shape);
    j.wm = shape;
    j.pts = 1;
    j.mstride = mstride;
    j.nblk_m = (j.mp + bm - 1) / bm;
    j.nblk_n = (j.d1 + bn - 1) / bn;
    j.tiles = 4 * j.groups * j.nblk_m * j.nblk_n;
    if (j.nkc < qres_min_chunks(shape))
        PIR_FAIL(PIR_EINVAL, "D0 of %u rows is below the kernel's %u chunks of 64", db.p.d0, qres_min_chunks(shape));
    if ((uint64_t)j.nblk_m * bm > mstride)
        PIR_FAIL(PIR_EINVAL, "query planes of %u rows hold no %u-row units", mstride, bm);
    if ((uint64_t)4 * j.groups * j.nblk_m * j.nblk_n >= (1ull << 32))
        PIR_FAIL(PIR_EINVAL, "too many work units");
    return j;
}

void launch_mfma_qres(const MfmaJob &job, hipStream_t st) {
    if (!job.tiles) return;
    const uint32_t grid = 8 * (uint32_t)std::max(1, qres_cu_count() / 8);
    auto go = [&](auto shape, auto mode) {
        using S = decltype(shape);
        constexpr int MODE = decltype(mode)::value;
        rowsel_mfma_qres_kernel<S, MODE><<<grid, 64 * QWAVES, 0, st>>>(job);
    };
    auto go_mode = [&](auto shape) {
        switch (job.split) {
            case RECOMB_DIRECT: go(shape, std::integral_constant<int, RECOMB_DIRECT>{}); break;
            case RECOMB_SPLIT: go(shape, std::integral_constant<int, RECOMB_SPLIT>{}); break;
            default: go(shape, std::integral_constant<int, RECOMB_WIDE>{}); break;
        }
    };
    switch (job.wm) {
        case 0: go_mode(QShape<2, 1, 3, 4>{}); break;
        case 1: go_mode(QShape<4, 1, 3, 3>{}); break;
        case 2: go_mode(QShape<3, 2, 3, 3, true>{}); break;
        default: go_mode(QShape<2, 4, 2, 3, true, 2>{}); break;
    }
    PIR_LAUNCH_CHECK();
}

}  // namespace pir
