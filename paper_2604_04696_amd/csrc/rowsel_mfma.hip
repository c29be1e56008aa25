// RowSel on the INT8 matrix cores, exact.
//
// Every residue x < 2^30 is written as four balanced signed 8-bit digits,
// x = sum_i d_i 2^(8i), d_i in [-128, 127].  A point's GEMM (sec. 2.3)
//   out[m][n] = sum_k Q[m][k] DB[k][n]  mod q
// then splits into sixteen digit products
//   P_ij[m][n] = sum_k dQ_i[m][k] dDB_j[k][n]
// computed by v_mfma_i32_32x32x32_i8 and summed per weight class s = i + j
// in int32: G_s = sum_{i+j=s} P_ij.  With |d| <= 128 and at most four pairs
// per class, |G_s| <= 4 * K * 2^14, so a K chunk of 2048 rows keeps
// |G_s| <= 2^27 (no int32 overflow, and small enough for the exact binary64
// recombination sum_s G_s 2^(8s) mod q of combine_classes): bit-identical to
// the 64-bit VALU path.
//
// Layouts (k contiguous within 64-byte chunks, "k-major" in the paper's
// terms, sec. 5.2.1), chunk-major so that a block's operand tile for one
// 64-row step of k is one contiguous run:
//   DB digits    [L*N][4][Kp/64][D1][64] int8   built once at load time
//   query digits [L*N][4][Kp/64][Mp][64] int8   built per call (ingest kernel)
// with Kp = D0 rounded up to 64 (rows D0 <= k < Kp hold zero digits) and
// Mp = 2B rounded up to 32 (query rows 2B <= m < Mp are not written: their
// GEMM rows are computed and never transposed out).
#include <algorithm>
#include <list>
#include <mutex>
#include <vector>
#include <type_traits>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "common.h"
#include "modarith.h"
#include "mfma.h"

namespace pir {

typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x16 __attribute__((ext_vector_type(16)));

struct ModQ4m {
    ModQ m[PIR_MAX_PRIMES];
};

// ----------------------------------------------------------- digit planes
// Generic transpose + digit split:  element (r, k, p) of a uint32 source at
// src[r*s_r + (k - klo)*s_k + p] (points p contiguous) goes to byte k%64 of
// row r of chunk k/64 of plane [p][d]:
//   dst[(((p*4 + d)*Kp/64 + k/64)*RS + row0 + r)*64 + k%64].
// A block takes two rows r, r+1, 64 k (aligned) and 64 points: it reads 128
// runs of 256 bytes, splits in LDS, and writes one 128-byte run (the two
// rows' 64-byte chunk rows, adjacent in dst) per point and digit.  k outside
// [klo, khi) and rows r >= r_valid read as zero; rows r >= R are not
// written; 16-byte chunks that straddle [klo, khi) (only when loading a DB
// in row ranges) are written byte by byte so neighbouring ranges are not
// overwritten.  CENTER (DBs with a prime of 2^30 or more): a residue above
// 0x7F7F7F7F is taken as x - q_l, so that four balanced digits cover every
// prime below 2^32 (point p belongs to prime p / N).
struct DigitCenter {
    uint32_t q[PIR_MAX_PRIMES];
    uint32_t n;
};

template <bool CENTER>
__global__ void __launch_bounds__(256)
digit_planes_kernel(const uint32_t *__restrict__ src, uint64_t s_r, uint64_t s_k,
                    int8_t *__restrict__ dst, uint32_t R, uint32_t r_valid, uint32_t P,
                    uint32_t kp, uint32_t klo, uint32_t khi, uint32_t kvalid, uint32_t kblk0,
                    uint32_t nkblk, uint32_t RS, uint32_t row0, DigitCenter dc) {
    __shared__ uint32_t tile[2][64][65];
    const uint32_t tid = threadIdx.x;
    uint64_t b = blockIdx.x;
    const uint32_t npb = (P + 63) / 64;
    const uint32_t pb = (uint32_t)(b % npb);
    b /= npb;
    const uint32_t kb = kblk0 + (uint32_t)(b % nkblk);
    const uint32_t r0 = 2 * (uint32_t)(b / nkblk);
    const uint32_t k0 = kb * 64, p0 = pb * 64;

    // all 32 loads of a thread are issued before the first LDS store
    uint32_t v[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) {
        const uint32_t e = tid + 256 * j, rr = e / 4096, kk = (e / 64) % 64, pp = e % 64;
        const uint32_t k = k0 + kk, r = r0 + rr;
        const bool in = r < r_valid && k >= klo && k < khi && p0 + pp < P;
        v[j] = in ? __builtin_nontemporal_load(src + (uint64_t)r * s_r + (uint64_t)(k - klo) * s_k + p0 + pp)
                  : 0u;
    }
#pragma unroll
    for (int j = 0; j < 32; ++j) {
        const uint32_t e = tid + 256 * j;
        uint32_t w;
        if (CENTER) {
            // the prime of this point (a point past P holds 0, any prime serves)
            const uint32_t li = (p0 + e % 64) / dc.n;
            w = split_digits_window(v[j], dc.q[li < PIR_MAX_PRIMES ? li : 0]);
        } else {
            w = split_digits(v[j]);
        }
        tile[e / 4096][(e / 64) % 64][e % 64] = w;
    }
    __syncthreads();

#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const uint32_t c = tid + 256 * j;
        const uint32_t kq = c % 4, rr = (c / 4) % 2, d = (c / 8) % 4, pp = c / 32;
        const uint32_t kc = k0 + kq * 16, r = r0 + rr;
        if (r >= R || kc >= kp || p0 + pp >= P) continue;
        const uint32_t hv = std::min(kc + 16, kvalid);   // k >= kvalid is padding
        const bool inside = kc >= klo && hv <= khi;
        uint32_t w[4];
#pragma unroll
        for (int i4 = 0; i4 < 4; ++i4) {
            uint32_t x = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                x |= ((tile[rr][kq * 16 + i4 * 4 + i][pp] >> (8 * d)) & 0xFFu) << (8 * i);
            w[i4] = x;
        }
        int8_t *o = dst + ((((uint64_t)(p0 + pp) * 4 + d) * (kp / 64) + kc / 64) * RS + row0 + r) * 64 + kc % 64;
        if (inside) {
            st_nt(reinterpret_cast<uint4 *>(o), make_uint4(w[0], w[1], w[2], w[3]));
        } else {
            for (int i = 0; i < 16; ++i) {
                const uint32_t k = kc + i;
                if (k >= klo && k < khi && k < kvalid) o[i] = (int8_t)(w[i / 4] >> (8 * (i % 4)));
            }
        }
    }
}

static void launch_digit_planes(const pir_db &db, const uint32_t *src, uint64_t s_r, uint64_t s_k, int8_t *dst,
                                uint32_t R, uint32_t r_valid, uint32_t P, uint32_t kp,
                                uint32_t klo, uint32_t khi, uint32_t kvalid, hipStream_t st,
                                uint32_t RS = 0, uint32_t row0 = 0) {
    if (!RS) RS = R;
    if (klo >= khi || R == 0) return;
    // blocks cover [klo, khi); when khi = D0 the last block also zero-fills
    // the padding up to Kp (Kp is D0 rounded up to 64)
    const uint32_t kb0 = klo / 64, kb1 = (khi + 63) / 64;
    const uint32_t nkb = kb1 - kb0;
    const uint64_t blocks = (uint64_t)((P + 63) / 64) * nkb * ((R + 1) / 2);
    if (blocks >= (1ull << 31)) PIR_FAIL(PIR_EINVAL, "digit-plane launch too large");
    DigitCenter dc{};
    for (uint32_t l = 0; l < db.p.nprimes; ++l) dc.q[l] = db.p.q[l];
    dc.n = db.p.n;
    if (db.wide)
        digit_planes_kernel<true><<<(uint32_t)blocks, 256, 0, st>>>(src, s_r, s_k, dst, R, r_valid, P, kp, klo,
                                                                    khi, kvalid, kb0, nkb, RS, row0, dc);
    else
        digit_planes_kernel<false><<<(uint32_t)blocks, 256, 0, st>>>(src, s_r, s_k, dst, R, r_valid, P, kp, klo,
                                                                     khi, kvalid, kb0, nkb, RS, row0, dc);
    PIR_LAUNCH_CHECK();
}

// DB rows [row0, row0+nrows) of an NTT-domain source [nrows][D1][L][N]:
// the GEMM's k is the DB row, r the DB column.
void launch_db_layout_mfma(const pir_db &db, const uint32_t *ntt_src, uint32_t row0,
                           uint32_t nrows, hipStream_t st) {
    const auto &p = db.p;
    const uint32_t P = p.n * p.nprimes;
    // src index = (k - row0)*D1*P + n*P + point
    launch_digit_planes(db, ntt_src, P, (uint64_t)p.d1 * P, db.mfma.data, p.d1, p.d1, P, db.mfma.kp,
                        row0, row0 + nrows, p.d0, st);
}

size_t mfma_query_scratch_bytes(const pir_db &db, uint32_t B) {
    const uint64_t mp = (2ull * B + 31) / 32 * 32;
    return (size_t)db.slots() * 4 * mp * db.mfma.kp;
}

// ------------------------------------------------------------- the GEMM
constexpr int KCH = 64;             // k bytes per pipeline step (two MFMA k-steps of 32)
constexpr uint32_t KSUPER = 2048;   // rows per int32 accumulation (bound above)
constexpr int NWAVE = 8;            // waves per block
constexpr int ROWS = 192;           // BM + BN of every tile shape (128 x 64 or 64 x 128)
constexpr int STAGE_BYTES = 4 * ROWS * KCH;            // 48 KiB: A and B digit planes of one step
constexpr int NSTAGE = 3;                              // LDS pipeline depth
constexpr int LPW = (4 * ROWS / 16) / NWAVE;           // 16-row, 1 KiB load instructions per wave per step
static_assert(LPW * NWAVE * 16 == 4 * ROWS, "loads must divide among the waves");

// LDS rows are 64 bytes (four 16-byte chunks).  Chunk c of row r is stored at
// position c ^ swz(r): rows r and r + 4 (which map to the same banks at a
// 256-byte bank period) then use different chunk positions, so a fragment
// read (32 consecutive rows at one chunk index) is conflict free; measured on
// gfx950 it moves ~230 B/clk per CU against ~125 for a (r >> 1) swizzle.
__device__ __forceinline__ uint32_t swz(uint32_t r) { return (r >> 2) & 3u; }

// Waits until at most N vector-memory operations of this wave are
// outstanding (they complete in issue order for this count).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// Workgroup barrier without the memory fences of __syncthreads(): those make
// the compiler wait for every outstanding global load, which would drain the
// operand pipeline.  LDS visibility is handled explicitly: each wave waits
// for its own direct-to-LDS loads (wait_vmcnt) before the barrier, and its
// LDS reads of a buffer complete (their values are consumed) before it
// reaches the barrier after which that buffer is refilled.
__device__ __forceinline__ void block_barrier() { asm volatile("s_barrier" ::: "memory"); }

// Wave-uniform description of one output tile.
struct Tile {
    const int8_t *qd, *dbd;
    uint32_t *out;
    uint32_t m_rows, mp, mstride, d1, sstride, nkc, L, N, bm, bn, wn, l, g, m0, n0, job, gl;
};

// Global tile index -> tile.  Within a job the (m, n) blocks of one point
// group are numbered consecutively, so the tiles that run at the same time
// on one XCD share that group's query digit planes in its L2.
__device__ __forceinline__ Tile decode_tile(uint32_t T, const MfmaJob &J, uint32_t j) {
    const uint32_t loc = T - J.tile0;
    const uint32_t tiles = J.nblk_m * J.nblk_n;
    uint32_t gg = loc / tiles;
    const uint32_t tile = loc % tiles;
    Tile t;
    t.gl = gg;            // group index inside the job (staging points 4*gl .. 4*gl+3)
    gg += J.g_begin;
    t.qd = J.qd;
    t.dbd = J.dbd;
    t.out = J.out;
    t.m_rows = J.m_rows;
    t.mp = J.mp;
    t.mstride = J.mstride;
    t.d1 = J.d1;
    t.sstride = J.sstride;
    t.nkc = J.nkc;
    t.L = J.L;
    t.N = J.N;
    t.bm = 32 * J.wm;
    t.bn = ROWS - t.bm;
    t.wn = NWAVE / J.wm;
    const uint32_t G = J.N / 4;
    t.l = gg / G;
    t.g = gg % G;
    t.m0 = (tile / J.nblk_n) * t.bm;
    t.n0 = (tile % J.nblk_n) * t.bn;
    t.job = j;
    return t;
}

// Load side of the pipeline for one wave and tile shape BM x BN: which
// operand, digit plane and 16-row block each of the wave's LPW load
// instructions covers is fixed by (wave, instruction).  The first QL
// instructions of every wave read query planes, the rest DB planes (A_INST
// is a multiple of NWAVE), so the per-step advance of each instruction's
// address is a compile-time choice between two plane sizes.  Each lane keeps
// the full 64-bit address of each of its loads, set when a tile starts and
// advanced by one add per step.  Byte offset of (point s, digit d, chunk kc,
// row r) in a plane set: ((s*4 + d)*nkc + kc)*plane + r*64, plane = rows*64.
template <int BM>
struct LoadCursor {
    static constexpr int BN = ROWS - BM;
    static constexpr int A_INST = 4 * BM / 16;   // query instructions (16 rows each)
    static constexpr int QL = A_INST / NWAVE;     // query loads of each wave
    static_assert(A_INST % NWAVE == 0, "query loads must split evenly among the waves");
    const int8_t *src[LPW];                       // per lane: address of each load's next step
    uint64_t qplane, dplane;                      // bytes of one query / DB plane chunk
    uint32_t lds[LPW];                            // LDS offset of each load inside a stage
    uint32_t kc, s, nkc;

    // LDS destination of instruction i inside a stage
    static __device__ __forceinline__ uint32_t lds_off(int i, uint32_t wv) {
        const uint32_t ii = wv + i * NWAVE;
        if (i < QL) return (ii / (BM / 16)) * BM * KCH + (ii % (BM / 16)) * 1024;
        const uint32_t jj = ii - A_INST;
        return 4 * BM * KCH + (jj / (BN / 16)) * BN * KCH + (jj % (BN / 16)) * 1024;
    }

    __device__ __forceinline__ void init(uint32_t wv) {
#pragma unroll
        for (int i = 0; i < LPW; ++i) lds[i] = lds_off(i, wv);
    }

    __device__ __forceinline__ void start(const Tile &t, uint32_t wv, uint32_t lane) {
        const uint64_t p0 = (uint64_t)t.l * t.N + 4 * t.g;
        qplane = (uint64_t)t.mstride * KCH;
        dplane = (uint64_t)t.d1 * KCH;
        const int8_t *qbase = t.qd + p0 * 4 * t.nkc * qplane;
        const int8_t *dbase = t.dbd + p0 * 4 * t.nkc * dplane;
        kc = s = 0;
        nkc = t.nkc;
        const uint32_t lrow = lane / 4, lchunk = lane % 4;
#pragma unroll
        for (int i = 0; i < LPW; ++i) {
            const uint32_t ii = wv + i * NWAVE;
            const bool q = i < QL;
            const uint32_t jj = q ? ii : ii - A_INST, rbn = q ? BM / 16 : BN / 16;
            const uint32_t d = jj / rbn, rb = jj % rbn, r = rb * 16 + lrow;
            uint32_t off = q ? min(t.m0 + r, t.mp - 1) * KCH : min(t.n0 + r, t.d1 - 1) * KCH;
            off += 16 * (lchunk ^ swz(r));
            src[i] = (q ? qbase + (uint64_t)d * t.nkc * qplane : dbase + (uint64_t)d * t.nkc * dplane) + off;
        }
    }

    // Issues this wave's loads of the current step into `stage`; returns
    // true when the tile's last step has been issued.
    __device__ __forceinline__ bool issue(int8_t *stage) {
#pragma unroll
        for (int i = 0; i < LPW; ++i) {
            // (a named pointer: an arithmetic expression as the builtin's
            // argument stops the host pass from emitting the kernel stub)
            const int8_t *from = src[i];
            __builtin_amdgcn_global_load_lds(from, (__attribute__((address_space(3))) void *)(stage + lds[i]), 16,
                                             0, 0);
            src[i] += i < QL ? qplane : dplane;
        }
        if (++kc == nkc) {
            kc = 0;
#pragma unroll
            for (int i = 0; i < LPW; ++i) src[i] += 3ull * nkc * (i < QL ? qplane : dplane);
            if (++s == 4) return true;
        }
        return false;
    }
};

// Persistent block: processes global tiles T = (i*8 + x)*per_xcd + y for
// i = 0, 1, ..., where x is the block's XCD (blocks are dealt to the XCDs
// round-robin) and y its index there; at any moment the tiles in flight on
// one XCD are consecutive in the tile order.  Each tile runs 4 points x nkc
// steps; the LDS pipeline runs over the concatenated steps of all the
// block's tiles without draining at tile boundaries.
//
// Per step a wave owns a 32 x 32 sub-tile and issues 2 k-steps x 16 MFMAs
// (four query digits x four DB digits) into seven int32 class accumulators.
//
// A single instance travels by value in `one` (ONE = true); a grouped launch
// passes a device array of jobs sorted by tile0.
template <bool ONE, int BM, int MODE>
__global__ void __launch_bounds__(64 * NWAVE) __attribute__((amdgpu_waves_per_eu(2, 2)))
rowsel_mfma_persistent(const MfmaJob one, const MfmaJob *__restrict__ jobs, uint32_t njobs,
                       uint32_t total_tiles) {
    __shared__ __attribute__((aligned(1024))) int8_t lds[NSTAGE * STAGE_BYTES];
    auto decode = [&](uint32_t T) {
        uint32_t j = 0;
        if (!ONE)
            while (j + 1 < njobs && T >= jobs[j + 1].tile0) ++j;
        return decode_tile(T, ONE ? one : jobs[j], j);
    };

    const uint32_t tid = threadIdx.x, lane = tid % 64;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(tid / 64);
    const uint32_t per_xcd = gridDim.x / 8;
    const uint32_t xcd = blockIdx.x % 8, yi = blockIdx.x / 8;
    auto tile_index = [&](uint32_t i) { return (i * 8 + xcd) * per_xcd + yi; };
    const uint32_t half = lane / 32;

    // ---- load cursor
    uint32_t li = 0;
    bool l_done = tile_index(0) >= total_tiles;
    Tile lt{};
    LoadCursor<BM> lc;
    lc.init(wv);
    if (!l_done) {
        lt = decode(tile_index(0));
        lc.start(lt, wv, lane);
    }
    uint32_t lbuf = 0;   // stage of the next issue
    auto issue_next = [&]() {
        const bool tile_end = lc.issue(lds + lbuf * STAGE_BYTES);
        lbuf = lbuf + 1 == NSTAGE ? 0 : lbuf + 1;
        if (tile_end) {
            ++li;
            l_done = tile_index(li) >= total_tiles;
            if (!l_done) {
                lt = decode(tile_index(li));
                lc.start(lt, wv, lane);
            }
        }
    };

    // ---- compute cursor (per-tile values refreshed when a tile starts)
    uint32_t ci = 0, s = 0, kc = 0, cbuf = 0;
    bool c_done = l_done;
    Tile ct = lt;
    uint32_t wmi = 0, wni = 0, abase = 0, bbase = 0, a_stride = 0, b_stride = 0;
    bool active = false;
    auto start_compute = [&]() {
        wmi = wv / ct.wn;
        wni = wv % ct.wn;
        active = ct.m0 + wmi * 32 < ct.mp && ct.n0 + wni * 32 < ct.d1;
        a_stride = ct.bm * KCH;
        b_stride = ct.bn * KCH;
        abase = (wmi * 32 + lane % 32) * KCH;
        bbase = 4 * a_stride + (wni * 32 + lane % 32) * KCH;
    };
    if (!c_done) start_compute();
    uint32_t achunk[2], bchunk[2];   // swizzled 16-byte chunk of each k-step
    auto chunks = [&]() {
        const uint32_t ar = wmi * 32 + lane % 32, br = wni * 32 + lane % 32;
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            achunk[ks] = 16 * ((2 * ks + half) ^ swz(ar));
            bchunk[ks] = 16 * ((2 * ks + half) ^ swz(br));
        }
    };
    chunks();

    i32x16 acc[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) acc[c] = (i32x16){};
    uint32_t res[16];   // this point's result (summed over K chunks of KSUPER rows)

    uint32_t outstanding = 0;   // steps issued beyond the one being computed
    for (int k = 0; k < NSTAGE - 1 && !l_done; ++k) {
        issue_next();
        ++outstanding;
    }

    bool after_store = false;
    while (!c_done) {
        // the loads of the current step are done once at most the NSTAGE-2
        // later steps' loads are outstanding (after output stores, or near
        // the end, wait for everything)
        --outstanding;
        if (!after_store && outstanding == NSTAGE - 2) wait_vmcnt<(NSTAGE - 2) * LPW>();
        else wait_vmcnt<0>();
        after_store = false;
        block_barrier();

        // Fragments go to distinct registers and are read ahead of their
        // use: k-step 0's eight, then (after its first MFMA group and this
        // step's operand loads) k-step 1's eight, which overlap k-step 0's
        // remaining MFMAs.  At most eleven reads are outstanding, within the
        // LDS wait counter's range, so each group waits only for its own
        // fragments.  The loads' address arithmetic is issued while the
        // first group's MFMAs run.  The scheduling barriers keep the
        // compiler from sinking the reads back to their uses and keep the
        // MFMAs in groups of four distinct classes (no back-to-back
        // accumulator dependence).
        const int8_t *abuf = lds + cbuf * STAGE_BYTES + abase, *bbuf = lds + cbuf * STAGE_BYTES + bbase;
        i32x4 a[2][4], b[2][4];
        auto read_frags = [&](int ks) {
#pragma unroll
            for (int d = 0; d < 4; ++d)
                a[ks][d] = *reinterpret_cast<const i32x4 *>(abuf + d * a_stride + achunk[ks]);
#pragma unroll
            for (int d = 0; d < 4; ++d)
                b[ks][d] = *reinterpret_cast<const i32x4 *>(bbuf + d * b_stride + bchunk[ks]);
            __builtin_amdgcn_sched_barrier(0);
        };
        auto mfma_group = [&](int ks, int j) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                acc[i + j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[ks][i], b[ks][j], acc[i + j], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
        };
        if (active) {
            read_frags(0);
            mfma_group(0, 0);
        }
        if (!l_done) {
            issue_next();
            ++outstanding;
        }
        if (active) {
            read_frags(1);
#pragma unroll
            for (int j = 1; j < 4; ++j) mfma_group(0, j);
#pragma unroll
            for (int j = 0; j < 4; ++j) mfma_group(1, j);
        }
        cbuf = cbuf + 1 == NSTAGE ? 0 : cbuf + 1;
        const bool last = kc + 1 == ct.nkc;
        if (last || ((kc + 1) * KCH) % KSUPER == 0) {
            // recombine the seven classes of this point: sum_s G_s 2^(8s) mod q
            const EpiQ mq = ONE ? one.q[ct.l] : jobs[ct.job].q[ct.l];
            const bool first = kc + 1 <= KSUPER / KCH;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                int gr[7];
#pragma unroll
                for (int c = 0; c < 7; ++c) gr[c] = acc[c][r];
                const uint32_t part = combine_classes<MODE>(gr, mq);
                // a sum of two residues of a prime above 2^31 needs 33 bits
                res[r] = first ? part : MODE == RECOMB_WIDE ? add_mod_w(res[r], part, mq.q)
                                                            : add_mod(res[r], part, mq.q);
            }
#pragma unroll
            for (int c = 0; c < 7; ++c) acc[c] = (i32x16){};
            if (last) {
                // the point is done: its rows go to the staging layout
                // [point][mp][sstride]; accumulator element r of a lane is row
                // 8*(r/4) + 4*(lane/32) + r%4, column lane%32 of the wave's
                // 32 x 32 sub-tile, so each store moves two 128-byte runs
                const uint32_t n = ct.n0 + wni * 32 + lane % 32;
                if (active && n < ct.d1) {
                    uint32_t *pt = ct.out + (uint64_t)(4 * ct.gl + s) * ct.mp * ct.sstride + n;
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const uint32_t m = ct.m0 + wmi * 32 + 8 * (r / 4) + 4 * half + (r % 4);
                        __builtin_nontemporal_store(res[r], pt + (uint64_t)m * ct.sstride);
                    }
                }
                after_store = true;
            }
        }
        if (++kc == ct.nkc) {
            kc = 0;
            if (++s == 4) {
                s = 0;
                ++ci;
                c_done = tile_index(ci) >= total_tiles;
                if (!c_done) {
                    ct = decode(tile_index(ci));
                    start_compute();
                    chunks();
                }
            }
        }
    }
}

// Output transpose: staging [P][mp][ss] (P = L*N points, ss = d1 rounded up
// to a multiple of 4) -> boundary layout [B][2][d1][L][N], i.e. for every row
// m < m_rows a P x d1 -> d1 x P transpose.  A block takes one row m, 64
// points and 64 columns: it reads 64 runs of 256 bytes (columns contiguous)
// and writes 64 runs of 256 bytes (points contiguous), 16-byte vectors on
// both sides through a padded LDS tile (the paper's output transposition of
// sec. 5.2.2, here one coalesced pass).  P is a multiple of 4 (N >= 4).
__global__ void __launch_bounds__(256)
out_transpose_kernel(const uint32_t *__restrict__ stage, uint32_t *__restrict__ out, uint32_t mp, uint32_t d1,
                     uint32_t ss, uint32_t P, uint32_t nblk_n, uint32_t nblk_p) {
    __shared__ __attribute__((aligned(16))) uint32_t tile[64][68];   // [column][point]
    const uint32_t tid = threadIdx.x;
    uint32_t b = blockIdx.x;
    const uint32_t pb = b % nblk_p;
    b /= nblk_p;
    const uint32_t nb = b % nblk_n;
    const uint32_t m = b / nblk_n;
    const uint32_t p0 = pb * 64, n0 = nb * 64;
    uint4 v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t e = tid + 256 * j, pi = e / 16, nq = e % 16;
        v[j] = p0 + pi < P && n0 + 4 * nq < d1
                   ? ld_nt(reinterpret_cast<const uint4 *>(stage + ((uint64_t)(p0 + pi) * mp + m) * ss + n0 + 4 * nq))
                   : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t e = tid + 256 * j, pi = e / 16, nq = e % 16;
        tile[4 * nq + 0][pi] = v[j].x;
        tile[4 * nq + 1][pi] = v[j].y;
        tile[4 * nq + 2][pi] = v[j].z;
        tile[4 * nq + 3][pi] = v[j].w;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t e = tid + 256 * j, ni = e / 16, pq = e % 16;
        if (n0 + ni < d1 && p0 + 4 * pq < P)
            st_nt(reinterpret_cast<uint4 *>(out + ((uint64_t)m * d1 + n0 + ni) * P + p0 + 4 * pq),
                  *reinterpret_cast<const uint4 *>(&tile[ni][4 * pq]));
    }
}

void launch_out_transpose(const uint32_t *stage, uint32_t *out, uint32_t m_rows, uint32_t mp, uint32_t d1,
                          uint32_t slots, hipStream_t st) {
    const uint32_t nblk_n = (d1 + 63) / 64, nblk_p = (slots + 63) / 64;
    const uint64_t blocks = (uint64_t)m_rows * nblk_n * nblk_p;
    if (!blocks) return;
    if (blocks >= (1ull << 31)) PIR_FAIL(PIR_EINVAL, "transpose launch too large");
    out_transpose_kernel<<<(uint32_t)blocks, 256, 0, st>>>(stage, out, mp, d1, staging_stride(d1), slots, nblk_n,
                                                           nblk_p);
    PIR_LAUNCH_CHECK();
}

static int cu_count() {
    static int cached = 0;
    if (!cached) {
        int dev = 0;
        PIR_HIP(hipGetDevice(&dev));
        PIR_HIP(hipDeviceGetAttribute(&cached, hipDeviceAttributeMultiprocessorCount, dev));
    }
    return cached;
}

// Fills a job for one instance; `tile0` is its first global tile index.
MfmaJob make_mfma_job(const pir_db &db, const int8_t *qd, uint32_t *out, uint32_t B, uint32_t tile0,
                      uint32_t wm) {
    const auto &p = db.p;
    MfmaJob j{};
    j.qd = qd;
    j.dbd = db.mfma.data;
    j.out = out;
    j.m_rows = 2 * B;
    j.mp = (j.m_rows + 31) / 32 * 32;
    j.mstride = j.mp;
    j.g_begin = 0;
    j.d1 = p.d1;
    j.sstride = staging_stride(p.d1);
    j.nkc = db.mfma.kp / KCH;
    j.L = p.nprimes;
    j.N = p.n;
    j.wm = wm;
    j.groups = p.nprimes * (p.n / 4);
    j.nblk_m = (j.mp + 32 * wm - 1) / (32 * wm);
    j.nblk_n = (p.d1 + 32 * (NWAVE / wm) - 1) / (32 * (NWAVE / wm));
    j.tile0 = tile0;
    j.tiles = j.groups * j.nblk_m * j.nblk_n;
    j.split = RECOMB_DIRECT;
    for (uint32_t l = 0; l < p.nprimes; ++l) {
        const ModQ &m = db.mod[l];
        const double c48 = (double)(uint32_t)((1ull << 48) % m.q);
        j.q[l] = EpiQ{m.qd, m.qinv, m.c32, m.c47, c48, m.q, 0};
        if (!combine_direct_ok(m.q)) j.split = std::max<uint32_t>(j.split, RECOMB_SPLIT);
    }
    if (db.wide) j.split = RECOMB_WIDE;
    return j;
}

// Tile shape: 128 x 64 when the batch fills 128 rows, else 64 x 128.
uint32_t pick_wm(uint32_t B) {
    if (const char *e = std::getenv("PIR_MFMA_WM")) {   // explicit choice (tuning runs)
        const int v = std::atoi(e);
        if (v == 2 || v == 4) return (uint32_t)v;
    }
    return 2 * B > 64 ? 4u : 2u;
}

// One persistent block per CU.  Either `one` (jobs_dev == NULL, njobs == 1)
// or a device array of njobs jobs.
void launch_mfma_jobs(const MfmaJob &one, const MfmaJob *jobs_dev, uint32_t njobs, uint32_t total_tiles,
                      hipStream_t st) {
    if (!total_tiles) return;
    const uint32_t grid = 8 * (uint32_t)std::max(1, cu_count() / 8);
    // every job of one launch shares the tile shape and the recombination
    // variant of `one`
    auto go = [&](auto bm, auto mode) {
        constexpr int BM = decltype(bm)::value;
        constexpr int MODE = decltype(mode)::value;
        if (jobs_dev)
            rowsel_mfma_persistent<false, BM, MODE><<<grid, 64 * NWAVE, 0, st>>>(one, jobs_dev, njobs, total_tiles);
        else
            rowsel_mfma_persistent<true, BM, MODE><<<grid, 64 * NWAVE, 0, st>>>(one, nullptr, 1, total_tiles);
    };
    auto go_mode = [&](auto bm) {
        switch (one.split) {
            case RECOMB_DIRECT: go(bm, std::integral_constant<int, RECOMB_DIRECT>{}); break;
            case RECOMB_SPLIT: go(bm, std::integral_constant<int, RECOMB_SPLIT>{}); break;
            default: go(bm, std::integral_constant<int, RECOMB_WIDE>{}); break;
        }
    };
    using B64 = std::integral_constant<int, 64>;
    using B128 = std::integral_constant<int, 128>;
    if (one.wm == 4) go_mode(B128{});
    else go_mode(B64{});
    PIR_LAUNCH_CHECK();
}

// Planes of rows m < 2B only (row stride Mp): rows 2B <= m < Mp are left as
// they are, since an output row of the GEMM depends on its own query row
// alone and rows m >= 2B never reach the output.  The k padding up to Kp is
// written as zero digits (it enters every valid row's sum).
void launch_query_digits(const pir_db &db, const uint32_t *q, uint32_t B, int8_t *qd, hipStream_t st) {
    const auto &p = db.p;
    const uint32_t P = p.n * p.nprimes;
    const uint32_t mp = (2 * B + 31) / 32 * 32;
    launch_digit_planes(db, q, (uint64_t)p.d0 * P, P, qd, 2 * B, 2 * B, P, db.mfma.kp, 0, p.d0, p.d0, st, mp);
}

void launch_query_digits_rows(const pir_db &db, const uint32_t *q, uint32_t rows, int8_t *qd,
                              uint32_t mstride, uint32_t row0, hipStream_t st) {
    const auto &p = db.p;
    const uint32_t P = p.n * p.nprimes;
    launch_digit_planes(db, q, (uint64_t)p.d0 * P, P, qd, rows, rows, P, db.mfma.kp, 0, p.d0, p.d0, st, mstride,
                        row0);
}

void launch_rowsel_mfma(const pir_db &db, const uint32_t *q, uint32_t B, uint32_t *out,
                        hipStream_t st, bool q_coeff) {
    // scratch: query digit planes [P][4][Kp/64][Mp][64], then the output
    // staging [P][Mp][sstride]
    const uint32_t mp = (2 * B + 31) / 32 * 32;
    const size_t qbytes = (mfma_query_scratch_bytes(db, B) + 255) / 256 * 256;
    const size_t sbytes = (size_t)db.slots() * mp * staging_stride(db.p.d1) * 4;
    StreamScratch buf(qbytes + sbytes, st);
    int8_t *scratch = buf.as<int8_t>();
    uint32_t *stage = reinterpret_cast<uint32_t *>(scratch + qbytes);
    if (q_coeff) {
        // coefficient-domain query: transform into an NTT-domain copy, then
        // the usual ingest (scratch freed when the call's work has passed)
        StreamScratch qn((size_t)B * 2 * db.p.d0 * db.slots() * 4, st);
        launch_query_ntt(db, q, B, qn.as<uint32_t>(), st);
        launch_query_digits(db, qn.as<uint32_t>(), B, scratch, st);
    } else {
        launch_query_digits(db, q, B, scratch, st);
    }
    const MfmaJob job = make_mfma_job(db, scratch, stage, B, 0, pick_wm(B));
    {
        KernelTimer::Scope timed(st);
        launch_mfma_jobs(job, nullptr, 1, job.tiles, st);
    }
    launch_out_transpose(stage, out, 2 * B, mp, db.p.d1, (uint32_t)db.slots(), st);
}

// ------------------------------------------------------------- grouped
// A grouped launch keeps, per distinct set of (DB, batch) items, a plan with
// the device job table and the scratch of every item (query digit planes and
// output staging).  The first call for a set allocates it; later calls only
// enqueue kernels (and may therefore be captured into a hipGraph).
struct GroupPlan {
    std::vector<std::pair<const pir_db *, uint32_t>> key;
    int device = 0;
    uint32_t wm = 4;
    int8_t *scratch = nullptr;
    MfmaJob *jobs_dev = nullptr;
    std::vector<MfmaJob> jobs;
    std::vector<size_t> item_job;   // item -> job index, or SIZE_MAX for B = 0
    uint32_t total_tiles = 0;
    ~GroupPlan() {
        if (scratch) {
            int prev = 0;
            const bool had = hipGetDevice(&prev) == hipSuccess;
            (void)hipSetDevice(device);
            (void)hipDeviceSynchronize();
            dev_free(scratch);
            if (had) (void)hipSetDevice(prev);
        }
    }
};

static std::mutex g_plan_mu;
static std::list<GroupPlan> g_plans;   // most recently used first
constexpr size_t MAX_PLANS = 8;

// Tile shape that pads fewer rows over the whole group (the choice when
// timing is switched off with PIR_AUTOTUNE=0).
static uint32_t pick_group_wm(const pir_rowsel_item *items, uint32_t count) {
    uint64_t waste4 = 0, waste2 = 0;
    for (uint32_t i = 0; i < count; ++i) {
        if (!items[i].B) continue;
        const uint64_t mp = (2ull * items[i].B + 31) / 32 * 32, d1 = items[i].db->p.d1;
        const uint64_t m4 = (mp + 127) / 128 * 128, n4 = (d1 + 63) / 64 * 64;
        const uint64_t m2 = (mp + 63) / 64 * 64, n2 = (d1 + 127) / 128 * 128;
        const uint64_t w = (uint64_t)items[i].db->mfma.kp * items[i].db->slots();
        waste4 += (m4 * n4 - mp * d1) * w;
        waste2 += (m2 * n2 - mp * d1) * w;
    }
    return waste4 <= waste2 ? 4u : 2u;
}

// PIR_MFMA_WM=4 or 2 forces the 128 x 64 or the 64 x 128 tile (0: not forced).
static uint32_t forced_wm() {
    if (const char *e = std::getenv("PIR_MFMA_WM")) {
        const int v = std::atoi(e);
        if (v == 2 || v == 4) return (uint32_t)v;
    }
    return 0;
}

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    EventPair() {
        PIR_HIP(hipEventCreate(&a));
        PIR_HIP(hipEventCreate(&b));
    }
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

static GroupPlan *find_plan(const std::vector<std::pair<const pir_db *, uint32_t>> &key, int dev, uint32_t forced) {
    for (auto it = g_plans.begin(); it != g_plans.end(); ++it)
        if (it->key == key && it->device == dev && (!forced || it->wm == forced)) {
            g_plans.splice(g_plans.begin(), g_plans, it);
            return &g_plans.front();
        }
    return nullptr;
}

// Builds the plan of a new item set.  Unless a shape is forced (or timing is
// off), both tile shapes run once on the call's own inputs, timed with events
// on the call's stream, and the faster one is kept for every later call.
static void build_plan(GroupPlan &pl, const pir_rowsel_item *items, uint32_t count, uint32_t forced,
                       hipStream_t st) {
    // layout of the scratch: per job [query digits][staging], then the job table
    std::vector<size_t> qoff, soff;
    size_t bytes = 0;
    for (uint32_t i = 0; i < count; ++i) {
        if (!items[i].B) {
            qoff.push_back(0);
            soff.push_back(0);
            continue;
        }
        const pir_db &db = *items[i].db;
        const uint64_t mp = (2ull * items[i].B + 31) / 32 * 32;
        qoff.push_back(bytes);
        bytes += (mfma_query_scratch_bytes(db, items[i].B) + 255) / 256 * 256;
        soff.push_back(bytes);
        bytes += ((size_t)db.slots() * mp * staging_stride(db.p.d1) * 4 + 255) / 256 * 256;
    }
    const size_t jobs_off = bytes;
    bytes += sizeof(MfmaJob) * count + 256;
    pl.scratch = static_cast<int8_t *>(dev_alloc(bytes));
    pl.jobs_dev = reinterpret_cast<MfmaJob *>(pl.scratch + jobs_off);

    auto set_shape = [&](uint32_t wm) {
        pl.wm = wm;
        pl.jobs.clear();
        pl.item_job.clear();
        uint32_t tile0 = 0;
        for (uint32_t i = 0; i < count; ++i) {
            if (!items[i].B) {
                pl.item_job.push_back(SIZE_MAX);
                continue;
            }
            pl.item_job.push_back(pl.jobs.size());
            MfmaJob j = make_mfma_job(*items[i].db, pl.scratch + qoff[i],
                                      reinterpret_cast<uint32_t *>(pl.scratch + soff[i]), items[i].B, tile0, wm);
            tile0 += j.tiles;
            pl.jobs.push_back(j);
        }
        pl.total_tiles = tile0;
        // one recombination variant per launch: the widest any job needs (each
        // variant is exact for the primes of the narrower ones)
        uint32_t split = RECOMB_DIRECT;
        for (const MfmaJob &j : pl.jobs) split = std::max(split, j.split);
        for (MfmaJob &j : pl.jobs) j.split = split;
        if (!pl.jobs.empty()) {
            PIR_HIP(hipMemcpyAsync(pl.jobs_dev, pl.jobs.data(), sizeof(MfmaJob) * pl.jobs.size(),
                                   hipMemcpyHostToDevice, st));
            PIR_HIP(hipStreamSynchronize(st));
        }
    };

    uint32_t wm = forced;
    if (!wm) {
        const char *tune = std::getenv("PIR_AUTOTUNE");
        if (tune && std::strcmp(tune, "0") == 0) wm = pick_group_wm(items, count);
    }
    if (!wm) {
        set_shape(4);
        if (pl.jobs.empty()) return;
        // the query digit planes do not depend on the tile shape
        for (uint32_t i = 0; i < count; ++i)
            if (pl.item_job[i] != SIZE_MAX)
                launch_query_digits(*items[i].db, items[i].q_dev, items[i].B,
                                    const_cast<int8_t *>(pl.jobs[pl.item_job[i]].qd), st);
        EventPair ev;
        float best = 0.0f;
        for (uint32_t cand : {4u, 2u}) {
            if (cand != pl.wm) set_shape(cand);
            for (int rep = 0; rep < 2; ++rep) {
                PIR_HIP(hipEventRecord(ev.a, st));
                launch_mfma_jobs(pl.jobs[0], pl.jobs_dev, (uint32_t)pl.jobs.size(), pl.total_tiles, st);
                PIR_HIP(hipEventRecord(ev.b, st));
                PIR_HIP(hipEventSynchronize(ev.b));
                float ms = 0.0f;
                PIR_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
                if (!wm || ms < best) {
                    best = ms;
                    wm = cand;
                }
            }
        }
    }
    if (wm != pl.wm || pl.jobs.empty()) set_shape(wm);
}

static GroupPlan &get_plan(const pir_rowsel_item *items, uint32_t count, hipStream_t st) {
    std::vector<std::pair<const pir_db *, uint32_t>> key(count);
    for (uint32_t i = 0; i < count; ++i) key[i] = {items[i].db, items[i].B};
    const uint32_t forced = forced_wm();
    int dev = 0;
    PIR_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_plan_mu);
    if (GroupPlan *pl = find_plan(key, dev, forced)) return *pl;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    PIR_HIP(hipStreamIsCapturing(st, &cap));
    PIR_REQUIRE(cap == hipStreamCaptureStatusNone,
                "pir_rowsel_grouped: the first call for a set of item shapes allocates and cannot be captured");
    g_plans.emplace_front();
    GroupPlan &pl = g_plans.front();
    pl.key = key;
    pl.device = dev;
    try {
        build_plan(pl, items, count, forced, st);
    } catch (...) {
        g_plans.pop_front();   // frees what was allocated
        throw;
    }
    while (g_plans.size() > MAX_PLANS) g_plans.pop_back();
    return g_plans.front();
}

bool group_plan_tile(const pir_rowsel_item *items, uint32_t count, uint32_t *bm, uint32_t *bn) {
    std::vector<std::pair<const pir_db *, uint32_t>> key(count);
    for (uint32_t i = 0; i < count; ++i) key[i] = {items[i].db, items[i].B};
    int dev = 0;
    PIR_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_plan_mu);
    GroupPlan *pl = find_plan(key, dev, 0);
    if (!pl) return false;
    *bm = 32 * pl->wm;
    *bn = 32 * (NWAVE / pl->wm);
    return true;
}

void launch_rowsel_mfma_grouped(const pir_rowsel_item *items, uint32_t count, hipStream_t st) {
    GroupPlan &pl = get_plan(items, count, st);
    if (pl.jobs.empty()) return;
    for (uint32_t i = 0; i < count; ++i)
        if (pl.item_job[i] != SIZE_MAX)
            launch_query_digits(*items[i].db, items[i].q_dev, items[i].B,
                                const_cast<int8_t *>(pl.jobs[pl.item_job[i]].qd), st);
    {
        KernelTimer::Scope timed(st);
        launch_mfma_jobs(pl.jobs[0], pl.jobs_dev, (uint32_t)pl.jobs.size(), pl.total_tiles, st);
    }
    for (uint32_t i = 0; i < count; ++i) {
        if (pl.item_job[i] == SIZE_MAX) continue;
        const MfmaJob &j = pl.jobs[pl.item_job[i]];
        launch_out_transpose(j.out, items[i].out_dev, j.m_rows, j.mp, j.d1, (uint32_t)items[i].db->slots(), st);
    }
}

void release_group_plans() {
    std::lock_guard<std::mutex> lock(g_plan_mu);
    g_plans.clear();
}

}  // namespace pir
