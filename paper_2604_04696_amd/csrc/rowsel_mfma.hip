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
#include <memory>
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
// A block (1024 threads) takes four rows r .. r+3, 64 k (aligned) and 128
// points.  A thread loads four consecutive points for eight consecutive k
// (16-byte loads when the source allows them, else four words), splits each
// residue into its four digit bytes and transposes bytes in registers
// (v_perm_b32), so that it holds, per point and digit, the eight bytes of
// its eight k: one 8-byte LDS store each.  The block then writes one
// 256-byte run (the four rows' 64-byte chunk rows, adjacent in dst) per
// point and digit, read from LDS in 16-byte pieces; its reads are 512-byte
// runs (128 points of one row and k).  LDS (128 KiB) holds
// [row][point][digit][64 k bytes] with the digit's 64-byte row and the
// 16-byte piece inside it XOR-swizzled by the point (conflict-free 8-byte
// stores and 16-byte reads) and row rr's part offset by 64 rr more bytes.
// (Measured on the 2 GiB query of 64 clients: 0.75-0.77 ms; 64 points per
// block 0.78-0.83 ms; two rows per block 0.82 ms; the form before it, a
// 4-byte load and 16 4-byte LDS reads per 16 bytes of output, 0.85-0.88
// ms.)  k outside [klo, khi) and rows
// r >= r_valid read as zero; rows r >= R are not written; 16-byte pieces
// that straddle [klo, khi) (only when loading a DB in row ranges) are
// written byte by byte so neighbouring ranges are not overwritten.  CENTER
// (DBs with a prime of 2^30 or more): a residue above 0x7F7F7F7F is taken
// as x - q_l, so that four balanced digits cover every prime below 2^32
// (point p belongs to prime p / N).
struct DigitCenter {
    uint32_t q[PIR_MAX_PRIMES];
    uint32_t n;
};

constexpr uint32_t DP_ROWS = 4;                         // rows per block
constexpr uint32_t DP_PTS = 128;                        // points per block
constexpr uint32_t DP_PQ = DP_PTS / 4;                  // four-point groups per block
constexpr uint32_t DP_THREADS = DP_PQ * 8 * DP_ROWS;    // a thread: four points x eight k of one row
constexpr uint32_t DP_ROW = DP_PTS * 256 + 64;          // LDS bytes per row of the block (+ offset)

// LDS byte offset of the 16-byte piece kq (k = 16 kq .. 16 kq + 15) of
// digit d of point pp in row rr.
__device__ __forceinline__ uint32_t dp_lds(uint32_t rr, uint32_t pp, uint32_t d, uint32_t kq) {
    return rr * DP_ROW + pp * 256 + ((d ^ ((pp >> 4) & 3)) * 64) + ((kq ^ ((pp >> 2) & 3)) * 16);
}

template <bool CENTER, bool VEC>
__global__ void __launch_bounds__(DP_THREADS)
digit_planes_kernel(const uint32_t *__restrict__ src, uint64_t s_r, uint64_t s_k,
                    int8_t *__restrict__ dst, uint32_t R, uint32_t r_valid, uint32_t P,
                    uint32_t kp, uint32_t klo, uint32_t khi, uint32_t kvalid, uint32_t kblk0,
                    uint32_t nkblk, uint32_t RS, uint32_t row0, DigitCenter dc) {
    __shared__ __attribute__((aligned(16))) uint8_t tile[DP_ROWS * DP_ROW];
    const uint32_t tid = threadIdx.x;
    uint64_t b = blockIdx.x;
    const uint32_t npb = (P + DP_PTS - 1) / DP_PTS;
    const uint32_t pb = (uint32_t)(b % npb);
    b /= npb;
    const uint32_t kb = kblk0 + (uint32_t)(b % nkblk);
    const uint32_t r0 = DP_ROWS * (uint32_t)(b / nkblk);
    const uint32_t k0 = kb * 64, p0 = pb * DP_PTS;

    // thread: points p0 + 4 pq .. + 3, k0 + 8 kg .. + 7, row r0 + rr; all
    // loads are issued before the first digit split
    const uint32_t pq = tid % DP_PQ, kg = (tid / DP_PQ) % 8, rr = tid / (DP_PQ * 8);
    const uint32_t r = r0 + rr, pb4 = p0 + 4 * pq;
    uint4 v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const uint32_t k = k0 + kg * 8 + i;
        const bool in = r < r_valid && k >= klo && k < khi;
        const uint32_t *at = src + (uint64_t)r * s_r + (uint64_t)(k - klo) * s_k + pb4;
        if (VEC) {   // P is a multiple of 4: the four points are all in or all out
            v[i] = in && pb4 < P ? ld_nt(reinterpret_cast<const uint4 *>(at)) : make_uint4(0, 0, 0, 0);
        } else {
            v[i].x = in && pb4 + 0 < P ? __builtin_nontemporal_load(at + 0) : 0u;
            v[i].y = in && pb4 + 1 < P ? __builtin_nontemporal_load(at + 1) : 0u;
            v[i].z = in && pb4 + 2 < P ? __builtin_nontemporal_load(at + 2) : 0u;
            v[i].w = in && pb4 + 3 < P ? __builtin_nontemporal_load(at + 3) : 0u;
        }
    }
    auto split = [&](uint32_t x, uint32_t pi) {
        if (CENTER) {
            // the prime of this point (a point past P holds 0, any prime serves)
            const uint32_t li = (pb4 + pi) / dc.n;
            return split_digits_window(x, dc.q[li < PIR_MAX_PRIMES ? li : 0]);
        }
        return split_digits(x);
    };
    // 4 x 4 byte transpose: o[d] byte j = byte d of w[j]
    auto transpose4 = [](uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3, uint32_t (&o)[4]) {
        const uint32_t a = __builtin_amdgcn_perm(w1, w0, 0x06020400u);   // w0.0 w1.0 w0.2 w1.2
        const uint32_t c = __builtin_amdgcn_perm(w1, w0, 0x07030501u);   // w0.1 w1.1 w0.3 w1.3
        const uint32_t e = __builtin_amdgcn_perm(w3, w2, 0x06020400u);
        const uint32_t f = __builtin_amdgcn_perm(w3, w2, 0x07030501u);
        o[0] = __builtin_amdgcn_perm(e, a, 0x05040100u);
        o[1] = __builtin_amdgcn_perm(f, c, 0x05040100u);
        o[2] = __builtin_amdgcn_perm(e, a, 0x07060302u);
        o[3] = __builtin_amdgcn_perm(f, c, 0x07060302u);
    };
#pragma unroll
    for (uint32_t pi = 0; pi < 4; ++pi) {
        uint32_t w[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const uint32_t x = pi == 0 ? v[i].x : pi == 1 ? v[i].y : pi == 2 ? v[i].z : v[i].w;
            w[i] = split(x, pi);
        }
        uint32_t lo[4], hi[4];
        transpose4(w[0], w[1], w[2], w[3], lo);
        transpose4(w[4], w[5], w[6], w[7], hi);
        const uint32_t pp = 4 * pq + pi;
#pragma unroll
        for (uint32_t d = 0; d < 4; ++d)
            *reinterpret_cast<uint2 *>(tile + dp_lds(rr, pp, d, kg / 2) + (kg % 2) * 8) = make_uint2(lo[d], hi[d]);
    }
    __syncthreads();

#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const uint32_t c = tid + DP_THREADS * j;
        const uint32_t kq = c % 4, orr = (c / 4) % DP_ROWS, d = (c / (4 * DP_ROWS)) % 4, pp = c / (16 * DP_ROWS);
        const uint32_t kc = k0 + kq * 16, orow = r0 + orr;
        if (orow >= R || kc >= kp || p0 + pp >= P) continue;
        const uint32_t hv = std::min(kc + 16, kvalid);   // k >= kvalid is padding
        const bool inside = kc >= klo && hv <= khi;
        const uint4 x = *reinterpret_cast<const uint4 *>(tile + dp_lds(orr, pp, d, kq));
        int8_t *o = dst + ((((uint64_t)(p0 + pp) * 4 + d) * (kp / 64) + kc / 64) * RS + row0 + orow) * 64 + kc % 64;
        if (inside) {
            st_nt(reinterpret_cast<uint4 *>(o), x);
        } else {
            const uint32_t w[4] = {x.x, x.y, x.z, x.w};
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
    const uint64_t blocks = (uint64_t)((P + DP_PTS - 1) / DP_PTS) * nkb * ((R + DP_ROWS - 1) / DP_ROWS);
    if (blocks >= (1ull << 31)) PIR_FAIL(PIR_EINVAL, "digit-plane launch too large");
    DigitCenter dc{};
    for (uint32_t l = 0; l < db.p.nprimes; ++l) dc.q[l] = db.p.q[l];
    dc.n = db.p.n;
    // 16-byte loads need an aligned source and whole four-point groups
    const bool vec = reinterpret_cast<uintptr_t>(src) % 16 == 0 && P % 4 == 0 && s_r % 4 == 0 && s_k % 4 == 0;
    auto go = [&](auto center, auto vec4) {
        digit_planes_kernel<decltype(center)::value, decltype(vec4)::value><<<(uint32_t)blocks, DP_THREADS, 0, st>>>(
            src, s_r, s_k, dst, R, r_valid, P, kp, klo, khi, kvalid, kb0, nkb, RS, row0, dc);
    };
    if (db.wide) {
        if (vec) go(std::true_type{}, std::true_type{});
        else go(std::true_type{}, std::false_type{});
    } else {
        if (vec) go(std::false_type{}, std::true_type{});
        else go(std::false_type{}, std::false_type{});
    }
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
// m < m_rows a P x d1 -> d1 x P transpose.  A block takes one row m, TP
// points and TC columns: it reads TP runs of 4 TC bytes (columns contiguous)
// and writes TC runs of 4 TP bytes (points contiguous), 16-byte vectors on
// both sides through a padded LDS tile (the paper's output transposition of
// sec. 5.2.2, here one coalesced pass).  P is a multiple of 4 (N >= 4).
template <int TP, int TC>
__global__ void __launch_bounds__(256)
out_transpose_kernel(const uint32_t *__restrict__ stage, uint32_t *__restrict__ out, uint32_t mp, uint32_t d1,
                     uint32_t ss, uint32_t P, uint32_t nblk_n, uint32_t nblk_p) {
    __shared__ __attribute__((aligned(16))) uint32_t tile[TC][TP + 4];   // [column][point]
    constexpr int NQ = TC / 4, PQ = TP / 4;                               // column and point quads
    constexpr int LOADS = TP * NQ / 256, STORES = TC * PQ / 256;
    static_assert(LOADS * 256 == TP * NQ && STORES * 256 == TC * PQ, "tile divides among the threads");
    const uint32_t tid = threadIdx.x;
    uint32_t b = blockIdx.x;
    const uint32_t pb = b % nblk_p;
    b /= nblk_p;
    const uint32_t nb = b % nblk_n;
    const uint32_t m = b / nblk_n;
    const uint32_t p0 = pb * TP, n0 = nb * TC;
    uint4 v[LOADS];
#pragma unroll
    for (int j = 0; j < LOADS; ++j) {
        const uint32_t e = tid + 256 * j, pi = e / NQ, nq = e % NQ;
        v[j] = p0 + pi < P && n0 + 4 * nq < d1
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
        if (n0 + ni < d1 && p0 + 4 * pq < P)
            st_nt(reinterpret_cast<uint4 *>(out + ((uint64_t)m * d1 + n0 + ni) * P + p0 + 4 * pq),
                  *reinterpret_cast<const uint4 *>(&tile[ni][4 * pq]));
    }
}

// Points and columns per transpose block: 512-byte write runs.  Measured on
// the 64-client output (2 GiB each way): 128 x 64 0.67 ms, 256 x 32 0.68 ms,
// 64 x 64 0.74-0.79 ms, 64 x 128 0.78 ms, 128 x 128 (68 KiB of LDS) 0.95 ms.
constexpr int OT_P = 128, OT_C = 64;

void launch_out_transpose(const uint32_t *stage, uint32_t *out, uint32_t m_rows, uint32_t mp, uint32_t d1,
                          uint32_t slots, hipStream_t st) {
    const uint32_t nblk_n = (d1 + OT_C - 1) / OT_C, nblk_p = (slots + OT_P - 1) / OT_P;
    const uint64_t blocks = (uint64_t)m_rows * nblk_n * nblk_p;
    if (!blocks) return;
    if (blocks >= (1ull << 31)) PIR_FAIL(PIR_EINVAL, "transpose launch too large");
    out_transpose_kernel<OT_P, OT_C><<<(uint32_t)blocks, 256, 0, st>>>(stage, out, mp, d1, staging_stride(d1),
                                                                       slots, nblk_n, nblk_p);
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

// ------------------------------------------------ grouped GEMM, a tile shape per job
// The tile of a grouped job is `pts` points side by side x BM rows x BN
// columns, BM = 32 wm, BN = 32 wn, with pts * wm * wn = 8: every wave owns
// one 32 x 32 sub-tile of one point, so a job whose output is narrow (few
// clients, few DB columns) still keeps all eight waves on useful sub-tiles
// (shapes: 1 x 128x64, 1 x 64x128, 1 x 32x256, 1 x 256x32, 2 x 64x64,
// 2 x 32x128, 2 x 128x32).  A pipeline stage holds the operand rows of all
// points of the tile, pts * (BM + BN) <= 320 rows of four digit planes
// (80 KiB), in two stages (the whole 160 KiB of LDS); stage layout per point:
// [4 digits][BM query rows][64] then [4 digits][BN DB rows][64], points one
// after the other, so 16-row load unit u of a stage sits at byte u * 1024.
// The rest (XCD-aware persistent tile order, seven class accumulators, exact
// recombination, staging stores) is as in rowsel_mfma_persistent.
//
// The ring is a template (stage count and rows); the build uses two stages
// of 320 rows.  With more than two stages every shape of the ring must load
// the same number of 16-row units per wave, the fixed wait count of a step.
// (A three-stage 192-row ring of this kernel, holding only the 128x64 and
// 64x128 shapes, ran 5-20% slower than rowsel_mfma_persistent with the same
// shapes -- its per-unit run-time guards and address selects are scalar
// instructions, which the eight waves of a CU share one unit for -- so the
// 192-row shapes run in that kernel instead, see launch_mfma_grouped.)
template <int NST, int ROWS>
struct GRing {
    static constexpr int NST_ = NST;
    static constexpr int STAGE_BYTES = 4 * ROWS * KCH;
    static constexpr int LPW = (4 * ROWS / 16) / NWAVE;   // 16-row load units per wave at most
    static_assert(LPW * NWAVE * 16 == 4 * ROWS, "load units must divide among the waves");
    static_assert(NST * STAGE_BYTES <= 160 * 1024, "ring exceeds the LDS");
};
using RingWide = GRing<2, 320>;

struct GTile {
    const int8_t *qd, *dbd;
    uint32_t *out;
    uint32_t mp, mstride, d1, sstride, nkc, N, pts, bm, bn, wn, l, g, m0, n0, job, gl;
};

__device__ __forceinline__ GTile decode_gtile(uint32_t T, const MfmaJob &J, uint32_t j) {
    const uint32_t loc = T - J.tile0;
    const uint32_t tiles = J.nblk_m * J.nblk_n;
    uint32_t gg = loc / tiles;
    const uint32_t tile = loc % tiles;
    GTile t;
    t.gl = gg;
    gg += J.g_begin;
    t.qd = J.qd;
    t.dbd = J.dbd;
    t.out = J.out;
    t.mp = J.mp;
    t.mstride = J.mstride;
    t.d1 = J.d1;
    t.sstride = J.sstride;
    t.nkc = J.nkc;
    t.N = J.N;
    t.pts = J.pts;
    t.bm = 32 * J.wm;
    t.wn = NWAVE / (J.pts * J.wm);
    t.bn = 32 * t.wn;
    const uint32_t G = J.N / 4;
    t.l = gg / G;
    t.g = gg % G;
    t.m0 = (tile / J.nblk_n) * t.bm;
    t.n0 = (tile % J.nblk_n) * t.bn;
    t.job = j;
    return t;
}

// Load side for one wave: unit u = wave + 8 i (i < n) of each stage, the
// per-step advance of each unit's address (one query or DB plane chunk), and
// the jump to the next set of pts points after the last k chunk.
template <int G_LPW>
struct GLoadCursor {
    const int8_t *src[G_LPW];
    uint64_t qadv, dadv;   // bytes of one query / DB plane chunk
    uint32_t qmask;        // bit i: unit i reads a query plane
    uint32_t n, kc, s, nkc, nsets, pts;

    __device__ __forceinline__ uint64_t adv(int i) const { return (qmask >> i) & 1u ? qadv : dadv; }

    __device__ __forceinline__ void start(const GTile &t, uint32_t wv, uint32_t lane) {
        const uint64_t p0 = (uint64_t)t.l * t.N + 4 * t.g;
        const uint64_t qplane = (uint64_t)t.mstride * KCH, dplane = (uint64_t)t.d1 * KCH;
        const uint32_t upp = (t.bm + t.bn) / 4;   // units per point
        n = t.pts * upp / NWAVE;
        kc = s = 0;
        nkc = t.nkc;
        pts = t.pts;
        nsets = 4 / t.pts;
        const uint32_t lrow = lane / 4, lchunk = lane % 4;
        qadv = qplane;
        dadv = dplane;
        qmask = 0;
#pragma unroll
        for (int i = 0; i < G_LPW; ++i) {
            const uint32_t u = wv + NWAVE * i;
            const uint32_t pt = u / upp;
            uint32_t v = u % upp;
            const bool q = v < t.bm / 4;
            if (!q) v -= t.bm / 4;
            const uint32_t rbn = q ? t.bm / 16 : t.bn / 16;
            const uint32_t d = v / rbn, r = (v % rbn) * 16 + lrow;
            const uint32_t row = q ? min(t.m0 + r, t.mp - 1) : min(t.n0 + r, t.d1 - 1);
            const uint64_t plane = q ? qplane : dplane;
            const int8_t *base = (q ? t.qd : t.dbd) + ((p0 + pt) * 4 + d) * t.nkc * plane;
            src[i] = base + (uint64_t)row * KCH + 16 * (lchunk ^ swz(r));
            qmask |= (q ? 1u : 0u) << i;
        }
    }

    // Issues this wave's loads of the current step into `stage` (LDS
    // addresses are wave-uniform: unit u lands at stage + u * 1024); returns
    // true when the tile's last step has been issued.
    __device__ __forceinline__ bool issue(int8_t *stage, uint32_t wv) {
#pragma unroll
        for (int i = 0; i < G_LPW; ++i) {
            if (i < (int)n) {
                const int8_t *from = src[i];
                __builtin_amdgcn_global_load_lds(
                    from, (__attribute__((address_space(3))) void *)(stage + (wv + NWAVE * i) * 1024), 16, 0, 0);
                src[i] += adv(i);
            }
        }
        if (++kc == nkc) {
            kc = 0;
            // the next set of points: pts points on, digit 0, k chunk 0
#pragma unroll
            for (int i = 0; i < G_LPW; ++i)
                if (i < (int)n) src[i] += (uint64_t)(4 * pts - 1) * nkc * adv(i);
            if (++s == nsets) return true;
        }
        return false;
    }
};

// A single job travels by value in `one` (ONE = true: serving steps, whose
// job changes every step); a grouped launch passes a device array of jobs
// sorted by tile0.
template <bool ONE, int MODE, class RING>
__global__ void __launch_bounds__(64 * NWAVE) __attribute__((amdgpu_waves_per_eu(2, 2)))
rowsel_mfma_grouped_kernel(const MfmaJob one, const MfmaJob *__restrict__ jobs, uint32_t njobs,
                           uint32_t total_tiles) {
    constexpr int G_NSTAGE = RING::NST_, G_STAGE_BYTES = RING::STAGE_BYTES, G_LPW = RING::LPW;
    __shared__ __attribute__((aligned(1024))) int8_t lds[G_NSTAGE * G_STAGE_BYTES];
    auto decode = [&](uint32_t T) {
        uint32_t j = 0;
        if (!ONE)
            while (j + 1 < njobs && T >= jobs[j + 1].tile0) ++j;
        return decode_gtile(T, ONE ? one : jobs[j], j);
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
    GTile lt{};
    GLoadCursor<G_LPW> lc;
    lc.n = 0;
    if (!l_done) {
        lt = decode(tile_index(0));
        lc.start(lt, wv, lane);
    }
    uint32_t lbuf = 0;
    auto issue_next = [&]() {
        const bool tile_end = lc.issue(lds + lbuf * G_STAGE_BYTES, wv);
        lbuf = lbuf + 1 == G_NSTAGE ? 0 : lbuf + 1;
        if (tile_end) {
            ++li;
            l_done = tile_index(li) >= total_tiles;
            if (!l_done) {
                lt = decode(tile_index(li));
                lc.start(lt, wv, lane);
            }
        }
    };

    // ---- compute cursor
    uint32_t ci = 0, s = 0, kc = 0, cbuf = 0;
    bool c_done = l_done;
    GTile ct = lt;
    uint32_t wmi = 0, wni = 0, ptw = 0, abase = 0, bbase = 0, a_stride = 0, b_stride = 0;
    bool active = false;
    uint32_t achunk[2], bchunk[2];
    auto start_compute = [&]() {
        const uint32_t wpp = NWAVE / ct.pts;   // waves per point
        ptw = wv / wpp;
        const uint32_t r = wv % wpp;
        wmi = r / ct.wn;
        wni = r % ct.wn;
        active = ct.m0 + wmi * 32 < ct.mp && ct.n0 + wni * 32 < ct.d1;
        a_stride = ct.bm * KCH;
        b_stride = ct.bn * KCH;
        const uint32_t pbase = ptw * (ct.bm + ct.bn) * 4 * KCH;
        abase = pbase + (wmi * 32 + lane % 32) * KCH;
        bbase = pbase + 4 * a_stride + (wni * 32 + lane % 32) * KCH;
        const uint32_t ar = wmi * 32 + lane % 32, br = wni * 32 + lane % 32;
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            achunk[ks] = 16 * ((2 * ks + half) ^ swz(ar));
            bchunk[ks] = 16 * ((2 * ks + half) ^ swz(br));
        }
    };
    if (!c_done) start_compute();

    i32x16 acc[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) acc[c] = (i32x16){};
    uint32_t res[16];

    uint32_t outstanding = 0;   // steps issued beyond the one being computed
    for (int k = 0; k < G_NSTAGE - 1 && !l_done; ++k) {
        issue_next();
        ++outstanding;
    }

    bool after_store = false;
    while (!c_done) {
        // this step's operands are in once at most the later steps' loads
        // are outstanding (every wave issues G_LPW units per step in a
        // three-stage ring; after output stores, or near the end, wait for
        // everything)
        --outstanding;
        if (G_NSTAGE > 2 && !after_store && outstanding == G_NSTAGE - 2) wait_vmcnt<(G_NSTAGE - 2) * G_LPW>();
        else wait_vmcnt<0>();
        after_store = false;
        block_barrier();

        const int8_t *abuf = lds + cbuf * G_STAGE_BYTES + abase, *bbuf = lds + cbuf * G_STAGE_BYTES + bbase;
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
        // the next step's loads go to the stage every wave finished reading
        // before this step's barrier
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
        cbuf = cbuf + 1 == G_NSTAGE ? 0 : cbuf + 1;
        const bool last = kc + 1 == ct.nkc;
        if (last || ((kc + 1) * KCH) % KSUPER == 0) {
            const EpiQ mq = ONE ? one.q[ct.l] : jobs[ct.job].q[ct.l];
            const bool first = kc + 1 <= KSUPER / KCH;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                int gr[7];
#pragma unroll
                for (int c = 0; c < 7; ++c) gr[c] = acc[c][r];
                const uint32_t part = combine_classes<MODE>(gr, mq);
                res[r] = first ? part : MODE == RECOMB_WIDE ? add_mod_w(res[r], part, mq.q)
                                                            : add_mod(res[r], part, mq.q);
            }
#pragma unroll
            for (int c = 0; c < 7; ++c) acc[c] = (i32x16){};
            if (last) {
                const uint32_t n = ct.n0 + wni * 32 + lane % 32;
                if (active && n < ct.d1) {
                    const uint32_t point = 4 * ct.gl + s * ct.pts + ptw;
                    uint32_t *pt = ct.out + (uint64_t)point * ct.mp * ct.sstride + n;
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
            if (++s == 4 / ct.pts) {
                s = 0;
                ++ci;
                c_done = tile_index(ci) >= total_tiles;
                if (!c_done) {
                    ct = decode(tile_index(ci));
                    start_compute();
                }
            }
        }
    }
}

// One persistent block per CU, over the tiles of a device job table
// (jobs_dev, njobs) or of the single job `one` (jobs_dev == NULL).
// deep: the jobs are 1 x 128x64 or 1 x 64x128 tiles (all the same) and run
// in rowsel_mfma_persistent (three-stage 192-row ring, compile-time shape).
void launch_mfma_grouped(const MfmaJob &one, const MfmaJob *jobs_dev, uint32_t njobs, uint32_t total_tiles,
                         uint32_t split, bool deep, hipStream_t st) {
    if (!total_tiles) return;
    if (deep) {
        MfmaJob j = one;
        j.split = split;
        launch_mfma_jobs(j, jobs_dev, njobs, total_tiles, st);
        return;
    }
    const uint32_t grid = 8 * (uint32_t)std::max(1, cu_count() / 8);
    auto go = [&](auto mode) {
        constexpr int MODE = decltype(mode)::value;
        if (jobs_dev)
            rowsel_mfma_grouped_kernel<false, MODE, RingWide><<<grid, 64 * NWAVE, 0, st>>>(one, jobs_dev, njobs,
                                                                                        total_tiles);
        else
            rowsel_mfma_grouped_kernel<true, MODE, RingWide><<<grid, 64 * NWAVE, 0, st>>>(one, nullptr, 1,
                                                                                       total_tiles);
    };
    switch (split) {
        case RECOMB_DIRECT: go(std::integral_constant<int, RECOMB_DIRECT>{}); break;
        case RECOMB_SPLIT: go(std::integral_constant<int, RECOMB_SPLIT>{}); break;
        default: go(std::integral_constant<int, RECOMB_WIDE>{}); break;
    }
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
    const bool qres = qres_preferred(mp, db.mfma.kp / 64);
    const uint32_t shape = qres_shape_for(mp), bm = qres_rows(shape);
    const uint32_t mstride = qres ? (mp + bm - 1) / bm * bm : mp;
    const size_t qbytes = ((size_t)db.slots() * 4 * mstride * db.mfma.kp + 255) / 256 * 256;
    const size_t sbytes = (size_t)db.slots() * mp * staging_stride(db.p.d1) * 4;
    StreamScratch buf(qbytes + sbytes, st);
    int8_t *scratch = buf.as<int8_t>();
    uint32_t *stage = reinterpret_cast<uint32_t *>(scratch + qbytes);
    if (q_coeff) {
        // coefficient-domain query: transform into an NTT-domain copy, then
        // the usual ingest (scratch freed when the call's work has passed)
        StreamScratch qn((size_t)B * 2 * db.p.d0 * db.slots() * 4, st);
        launch_query_ntt(db, q, B, qn.as<uint32_t>(), st);
        launch_query_digits_rows(db, qn.as<uint32_t>(), 2 * B, scratch, mstride, 0, st);
    } else {
        launch_query_digits_rows(db, q, 2 * B, scratch, mstride, 0, st);
    }
    if (qres) {
        const MfmaJob job = make_qres_job(db, scratch, mstride, stage, B, shape);
        KernelTimer::Scope timed(st);
        launch_mfma_qres(job, st);
    } else {
        const MfmaJob job = make_mfma_job(db, scratch, stage, B, 0, pick_wm(B));
        KernelTimer::Scope timed(st);
        launch_mfma_jobs(job, nullptr, 1, job.tiles, st);
    }
    launch_out_transpose(stage, out, 2 * B, mp, db.p.d1, (uint32_t)db.slots(), st);
}

// ------------------------------------------------------------- grouped
// A grouped launch keeps, per distinct set of (DB, batch) items, a plan with
// the device job table and the scratch of every item (query digit planes and
// output staging).  The first call for a set allocates it; later calls only
// enqueue kernels (and may therefore be captured into a hipGraph).  A plan
// that has been used under stream capture is pinned: a captured graph keeps
// pointers into its scratch and job table, so it is never evicted to make
// room for other plans and is released only with one of its DBs.
//
// Tile shapes of rowsel_mfma_grouped_kernel (points side by side, waves along
// m; the waves along n follow): every job of a plan gets its own.
struct GShape {
    uint32_t pts, wm;
    uint32_t wn() const { return NWAVE / (pts * wm); }
    uint32_t bm() const { return 32 * wm; }
    uint32_t bn() const { return 32 * wn(); }
    // a shape of rowsel_mfma_persistent (192 operand rows, three-stage ring)
    bool deep_ok() const { return pts * (bm() + bn()) == 192; }
};
static const GShape G_SHAPES[] = {{1, 4}, {1, 2}, {1, 1}, {1, 8}, {2, 2}, {2, 1}, {2, 4}};

// Output words a shape computes for an mp x d1 point product (padding included).
static uint64_t shape_work(const GShape &s, uint64_t mp, uint64_t d1) {
    return (mp + s.bm() - 1) / s.bm() * s.bm() * ((d1 + s.bn() - 1) / s.bn() * s.bn());
}

struct GroupPlan {
    std::vector<std::pair<const pir_db *, uint32_t>> key;
    int device = 0;
    bool pinned = false;
    uint32_t forced = 0;            // shape forced by PIR_GROUPED_SHAPE (index + 1), 0 = chosen
    uint32_t ring_forced = 0;       // PIR_GROUPED_RING: 1 deep, 2 wide, 0 = chosen
    uint32_t sched_forced = 0;      // PIR_GROUPED_SCHED: 1 shared launches, 2 one per job, 0 = timed
    int8_t *scratch = nullptr;
    MfmaJob *jobs_dev = nullptr;
    // jobs in launch order: 128x64 tiles of the fixed-shape kernel, then its
    // 64x128 tiles, then the shaped kernel's jobs, then the query-resident
    // kernel's; in the shared schedule launch g < 3 covers jobs
    // [first[g], first[g+1]) with tiles numbered from 0, and every
    // query-resident job [first[3], first[4]) has a launch of its own
    std::vector<MfmaJob> jobs;
    std::vector<uint8_t> kind;      // per job: G_DEEP, G_WIDE or G_QRES
    std::vector<size_t> item_job;   // item -> job index, or SIZE_MAX for B = 0
    uint32_t first[5] = {0, 0, 0, 0, 0}, tiles[3] = {0, 0, 0}, split = RECOMB_DIRECT;
    bool per_job = false;           // one GEMM launch per job instead of one per kernel
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
static std::list<std::shared_ptr<GroupPlan>> g_plans;   // most recently used first
constexpr size_t MAX_PLANS = 8;                           // unpinned plans kept

// Drops least recently used unpinned plans beyond MAX_PLANS (lock held).
static void evict_plans_locked() {
    size_t unpinned = 0;
    for (const auto &p : g_plans) unpinned += !p->pinned;
    for (auto it = g_plans.end(); unpinned > MAX_PLANS && it != g_plans.begin();) {
        --it;
        if ((*it)->pinned) continue;
        it = g_plans.erase(it);
        --unpinned;
    }
}

// Kernels of a grouped job: the fixed-shape kernel (three-stage 192-row
// ring), the shaped kernel (two-stage 320-row ring), the query-resident
// kernel (rowsel_mfma_qres.hip).
enum : uint8_t { G_DEEP = 0, G_WIDE = 1, G_QRES = 2 };

// PIR_GROUPED_RING=deep|wide|qres restricts the candidates to one kernel
// (1 deep, 2 wide, 3 query-resident where it fits; 0 = all).
static uint32_t forced_ring() {
    const char *e = std::getenv("PIR_GROUPED_RING");
    if (e && !std::strcmp(e, "deep")) return 1;
    if (e && !std::strcmp(e, "wide")) return 2;
    if (e && !std::strcmp(e, "qres")) return 3;
    return 0;
}

// PIR_GROUPED_SCHED=shared|split forces the GEMM launch schedule (1 one
// launch per kernel, 2 one launch per job; 0 = timed at plan build).
static uint32_t forced_sched() {
    const char *e = std::getenv("PIR_GROUPED_SCHED");
    if (e && !std::strcmp(e, "shared")) return 1;
    if (e && !std::strcmp(e, "split")) return 2;
    return 0;
}

// PIR_GROUPED_SHAPE="pts,rows,cols" forces one tile shape on every job
// (returned as index + 1 into G_SHAPES; 0 = not forced or not a shape).
static uint32_t forced_shape() {
    const char *e = std::getenv("PIR_GROUPED_SHAPE");
    if (!e || !*e) return 0;
    unsigned pts = 0, bm = 0, bn = 0;
    if (std::sscanf(e, "%u,%u,%u", &pts, &bm, &bn) != 3) return 0;
    for (uint32_t i = 0; i < sizeof(G_SHAPES) / sizeof(G_SHAPES[0]); ++i)
        if (G_SHAPES[i].pts == pts && G_SHAPES[i].bm() == bm && G_SHAPES[i].bn() == bn) return i + 1;
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

static std::shared_ptr<GroupPlan> find_plan(const std::vector<std::pair<const pir_db *, uint32_t>> &key, int dev,
                                            uint32_t forced, uint32_t ring, uint32_t sched) {
    for (auto it = g_plans.begin(); it != g_plans.end(); ++it)
        if ((*it)->key == key && (*it)->device == dev && (*it)->forced == forced && (*it)->ring_forced == ring &&
            (*it)->sched_forced == sched) {
            g_plans.splice(g_plans.begin(), g_plans, it);
            return g_plans.front();
        }
    return nullptr;
}

MfmaJob make_shaped_job(const pir_db &db, const int8_t *qd, uint32_t *stage, uint32_t B, uint32_t pts,
                        uint32_t wm) {
    const GShape s{pts, wm};
    MfmaJob j = make_mfma_job(db, qd, stage, B, 0, s.wm);
    j.pts = s.pts;
    j.nblk_m = (j.mp + s.bm() - 1) / s.bm();
    j.nblk_n = (j.d1 + s.bn() - 1) / s.bn();
    j.tiles = j.groups * j.nblk_m * j.nblk_n;
    return j;
}

// Tile shape of one job of mp rows and d1 columns (serving steps):
// PIR_GROUPED_SHAPE when set, else the fewest padded output words, the
// fixed-shape kernel's shapes first on a tie; deep: it runs in
// rowsel_mfma_persistent (a 192-row shape, unless PIR_GROUPED_RING=wide).
void pick_shape(uint32_t mp, uint32_t d1, uint32_t *pts, uint32_t *wm, bool *deep) {
    const size_t nshape = sizeof(G_SHAPES) / sizeof(G_SHAPES[0]);
    uint32_t best = 0;
    if (const uint32_t f = forced_shape()) {
        best = f - 1;
    } else {
        for (uint32_t s2 = 1; s2 < nshape; ++s2)
            if (shape_work(G_SHAPES[s2], mp, d1) < shape_work(G_SHAPES[best], mp, d1)) best = s2;
    }
    *pts = G_SHAPES[best].pts;
    *wm = G_SHAPES[best].wm;
    *deep = G_SHAPES[best].deep_ok() && forced_ring() != 2;
}

// A job of a grouped plan in tile shape `s`.
static MfmaJob grouped_job(const pir_db &db, const int8_t *qd, uint32_t *stage, uint32_t B, const GShape &s) {
    return make_shaped_job(db, qd, stage, B, s.pts, s.wm);
}

static void launch_plan_gemms(const GroupPlan &pl, hipStream_t st);

// Builds the plan of a new item set.  Candidates of a job: the two 192-row
// shapes in rowsel_mfma_persistent (the "deep" ring: three stages), the
// shapes within 25% of the fewest padded output words in the shaped kernel
// (the "wide" ring) and the query-resident kernel's unit shapes (32 x 128,
// 64 x 128, 96 x 64, 128 x 64; a job whose K fits it gets query planes with
// rows for the row blocks of each of those units; the rows past 2B are
// never written and only feed output rows that are dropped).
// Without timing (PIR_AUTOTUNE=0) the job takes the candidate with the
// fewest padded words (the fixed-shape kernel on a tie); otherwise every
// candidate runs three times, alone, on the job's own inputs (the query digit
// planes are built first), timed with events on the call's stream, and the
// fastest is kept for every later call.  The jobs of the two tiled kernels
// then run either in up to three shared persistent launches (fixed-shape
// 128x64, fixed-shape 64x128, shaped kernel, all taking the widest
// recombination form any job needs: each form is exact for the primes of
// the narrower ones) or in one launch per job; the query-resident jobs
// always run one launch each.  With timing both schedules run three times and the
// faster is kept (jobs that share a launch also share its persistent
// blocks, but their point groups then compete for the L2 of each XCD).
static void build_plan(GroupPlan &pl, const pir_rowsel_item *items, uint32_t count, hipStream_t st) {
    const uint32_t ring_forced = pl.ring_forced;
    // query-resident unit shapes a job of nkc chunks of k can take
    auto qres_shapes = [&](uint32_t nkc) {
        std::vector<uint32_t> v;
        if (pl.forced || ring_forced == 1 || ring_forced == 2) return v;
        for (uint32_t s2 = 0; s2 < qres_shape_count(); ++s2)
            if (nkc >= qres_min_chunks(s2)) v.push_back(s2);
        return v;
    };
    // scratch: per job [query digits][staging], then the job tables
    std::vector<size_t> qoff(count, 0), soff(count, 0);
    std::vector<uint32_t> mst(count, 0);
    size_t bytes = 0;
    for (uint32_t i = 0; i < count; ++i) {
        if (!items[i].B) continue;
        const pir_db &db = *items[i].db;
        const uint32_t mp = (2 * items[i].B + 31) / 32 * 32;
        mst[i] = mp;   // rows for every candidate's row blocks
        for (uint32_t s2 : qres_shapes(db.mfma.kp / KCH))
            mst[i] = std::max(mst[i], (mp + qres_rows(s2) - 1) / qres_rows(s2) * qres_rows(s2));
        qoff[i] = bytes;
        bytes += ((size_t)db.slots() * 4 * mst[i] * db.mfma.kp + 255) / 256 * 256;
        soff[i] = bytes;
        bytes += ((size_t)db.slots() * mp * staging_stride(db.p.d1) * 4 + 255) / 256 * 256;
    }
    const size_t jobs_off = bytes;
    bytes += (sizeof(MfmaJob) * count + 255) / 256 * 256;
    pl.scratch = static_cast<int8_t *>(dev_alloc(bytes));
    pl.jobs_dev = reinterpret_cast<MfmaJob *>(pl.scratch + jobs_off);

    // candidates of each job: (shape, kernel); shape indexes G_SHAPES, or
    // for G_QRES the query-resident unit shape
    const size_t nshape = sizeof(G_SHAPES) / sizeof(G_SHAPES[0]);
    struct Cand { uint32_t shape; uint8_t kind; uint64_t work; };
    std::vector<std::vector<Cand>> cands(count);
    auto make_job = [&](uint32_t i, const Cand &c) {
        const pir_db &db = *items[i].db;
        int8_t *qd = pl.scratch + qoff[i];
        uint32_t *stage = reinterpret_cast<uint32_t *>(pl.scratch + soff[i]);
        MfmaJob j = c.kind == G_QRES ? make_qres_job(db, qd, mst[i], stage, items[i].B, c.shape)
                                     : grouped_job(db, qd, stage, items[i].B, G_SHAPES[c.shape]);
        j.mstride = mst[i];
        return j;
    };
    std::vector<size_t> qj;   // item of each job
    std::vector<MfmaJob> jobs;
    std::vector<uint8_t> kind;
    for (uint32_t i = 0; i < count; ++i) {
        if (!items[i].B) continue;
        const pir_db &db = *items[i].db;
        const uint64_t mp = (2ull * items[i].B + 31) / 32 * 32, d1 = db.p.d1;
        std::vector<Cand> &cs = cands[i];
        const std::vector<uint32_t> qs = qres_shapes(db.mfma.kp / KCH);
        if (ring_forced == 3 && !qs.empty()) {
            for (uint32_t s2 : qs) {
                const uint64_t bm = qres_rows(s2), bn = qres_cols(s2);
                cs.push_back({s2, G_QRES, (mp + bm - 1) / bm * bm * ((d1 + bn - 1) / bn * bn)});
            }
        } else {
            std::vector<uint32_t> order(nshape);
            for (uint32_t s2 = 0; s2 < nshape; ++s2) order[s2] = s2;
            std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
                return shape_work(G_SHAPES[a], mp, d1) < shape_work(G_SHAPES[b], mp, d1);
            });
            const uint64_t best = shape_work(G_SHAPES[order[0]], mp, d1);
            std::vector<uint32_t> shapes;
            if (pl.forced) shapes.push_back(pl.forced - 1);
            else
                for (uint32_t s2 : order)
                    if (shape_work(G_SHAPES[s2], mp, d1) * 4 <= best * 5) shapes.push_back(s2);
            // (a ring forced to the query-resident kernel that the job's K
            // does not fit leaves every tiled candidate)
            if (!pl.forced && ring_forced != 2)   // the fixed-shape kernel's two shapes, always tried
                for (uint32_t s2 = 0; s2 < nshape; ++s2)
                    if (G_SHAPES[s2].deep_ok()) cs.push_back({s2, G_DEEP, shape_work(G_SHAPES[s2], mp, d1)});
            for (uint32_t s2 : shapes) {
                const uint64_t w = shape_work(G_SHAPES[s2], mp, d1);
                if (pl.forced && G_SHAPES[s2].deep_ok() && ring_forced != 2) cs.push_back({s2, G_DEEP, w});
                if (ring_forced != 1 || !G_SHAPES[s2].deep_ok()) cs.push_back({s2, G_WIDE, w});
            }
            for (uint32_t s2 : qs) {
                const uint64_t bm = qres_rows(s2), bn = qres_cols(s2);
                cs.push_back({s2, G_QRES, (mp + bm - 1) / bm * bm * ((d1 + bn - 1) / bn * bn)});
            }
        }
        if (!pl.forced)   // the geometric best first when not timing
            std::stable_sort(cs.begin(), cs.end(), [](const Cand &a, const Cand &b) { return a.work < b.work; });
        qj.push_back(i);
        jobs.push_back(make_job(i, cs[0]));
        kind.push_back(cs[0].kind);
    }
    pl.item_job.assign(count, SIZE_MAX);
    if (jobs.empty()) return;
    pl.split = RECOMB_DIRECT;
    for (const MfmaJob &j : jobs) pl.split = std::max(pl.split, j.split);

    // one job alone in its own launch
    auto launch_alone = [&](MfmaJob j, uint8_t k) {
        j.split = pl.split;
        if (k == G_QRES) {
            launch_mfma_qres(j, st);
        } else {
            j.tile0 = 0;
            launch_mfma_grouped(j, nullptr, 1, j.tiles, pl.split, k == G_DEEP, st);
        }
    };
    EventPair ev;
    auto time_ms = [&](auto &&enqueue) {
        float best = 0.0f;
        for (int rep = 0; rep < 3; ++rep) {
            PIR_HIP(hipEventRecord(ev.a, st));
            enqueue();
            PIR_HIP(hipEventRecord(ev.b, st));
            PIR_HIP(hipEventSynchronize(ev.b));
            float t = 0.0f;
            PIR_HIP(hipEventElapsedTime(&t, ev.a, ev.b));
            best = rep ? std::min(best, t) : t;
        }
        return best;
    };

    const char *tune = std::getenv("PIR_AUTOTUNE");
    const bool timing = !pl.forced && !(tune && std::strcmp(tune, "0") == 0);
    if (timing) {
        for (size_t k = 0; k < jobs.size(); ++k)
            launch_query_digits_rows(*items[qj[k]].db, items[qj[k]].q_dev, 2 * items[qj[k]].B,
                                     const_cast<int8_t *>(jobs[k].qd), jobs[k].mstride, 0, st);
        for (size_t k = 0; k < jobs.size(); ++k) {
            const uint32_t i = (uint32_t)qj[k];
            if (cands[i].size() < 2) continue;
            float best = 0.0f;
            bool first = true;
            for (const Cand &c : cands[i]) {
                MfmaJob probe = make_job(i, c);
                probe.split = pl.split;
                const float ms = time_ms([&] { launch_alone(probe, c.kind); });
                if (first || ms < best) {
                    best = ms;
                    jobs[k] = probe;
                    kind[k] = c.kind;
                    first = false;
                }
            }
        }
    }
    // launch order: fixed-shape 128x64, fixed-shape 64x128, shaped kernel,
    // query-resident kernel; tile numbers restart at 0 in each launch
    for (int g = 0; g < 4; ++g) {
        pl.first[g] = (uint32_t)pl.jobs.size();
        uint32_t tile0 = 0;
        for (size_t k = 0; k < jobs.size(); ++k) {
            const int gk = kind[k] == G_QRES ? 3 : kind[k] == G_WIDE ? 2 : jobs[k].wm == 4 ? 0 : 1;
            if (gk != g) continue;
            MfmaJob j = jobs[k];
            j.tile0 = g < 3 ? tile0 : 0;
            j.split = pl.split;
            tile0 += j.tiles;
            pl.item_job[qj[k]] = pl.jobs.size();
            pl.jobs.push_back(j);
            pl.kind.push_back(kind[k]);
        }
        if (g < 3) pl.tiles[g] = tile0;
    }
    pl.first[4] = (uint32_t)pl.jobs.size();
    PIR_HIP(hipMemcpyAsync(pl.jobs_dev, pl.jobs.data(), sizeof(MfmaJob) * pl.jobs.size(), hipMemcpyHostToDevice, st));
    PIR_HIP(hipStreamSynchronize(st));
    pl.per_job = pl.sched_forced == 2;
    if (timing && !pl.sched_forced) {
        pl.per_job = false;
        const float shared = time_ms([&] { launch_plan_gemms(pl, st); });
        pl.per_job = true;
        const float alone = time_ms([&] { launch_plan_gemms(pl, st); });
        pl.per_job = alone < shared;
    }
}

// The GEMM launches of a plan, in its schedule.
static void launch_plan_gemms(const GroupPlan &pl, hipStream_t st) {
    for (int g = 0; g < 3; ++g) {
        if (pl.first[g + 1] == pl.first[g]) continue;
        if (pl.per_job) {
            for (uint32_t k = pl.first[g]; k < pl.first[g + 1]; ++k) {
                MfmaJob j = pl.jobs[k];
                j.tile0 = 0;
                launch_mfma_grouped(j, nullptr, 1, j.tiles, pl.split, g < 2, st);
            }
        } else {
            launch_mfma_grouped(pl.jobs[pl.first[g]], pl.jobs_dev + pl.first[g], pl.first[g + 1] - pl.first[g],
                                pl.tiles[g], pl.split, g < 2, st);
        }
    }
    for (uint32_t k = pl.first[3]; k < pl.first[4]; ++k) launch_mfma_qres(pl.jobs[k], st);
}

// The plan of an item list (built on first use).  The caller holds a
// reference, so a concurrent eviction cannot free it while it is in use.
static std::shared_ptr<GroupPlan> get_plan(const pir_rowsel_item *items, uint32_t count, hipStream_t st) {
    std::vector<std::pair<const pir_db *, uint32_t>> key(count);
    for (uint32_t i = 0; i < count; ++i) key[i] = {items[i].db, items[i].B};
    const uint32_t forced = forced_shape(), ring = forced_ring(), sched = forced_sched();
    int dev = 0;
    PIR_HIP(hipGetDevice(&dev));
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    PIR_HIP(hipStreamIsCapturing(st, &cap));
    std::lock_guard<std::mutex> lock(g_plan_mu);
    if (auto pl = find_plan(key, dev, forced, ring, sched)) {
        if (cap != hipStreamCaptureStatusNone) pl->pinned = true;
        return pl;
    }
    PIR_REQUIRE(cap == hipStreamCaptureStatusNone,
                "pir_rowsel_grouped: the first call for a set of item shapes allocates and cannot be captured");
    auto pl = std::make_shared<GroupPlan>();
    pl->key = key;
    pl->device = dev;
    pl->forced = forced;
    pl->ring_forced = ring;
    pl->sched_forced = sched;
    build_plan(*pl, items, count, st);   // on failure the plan frees what it allocated
    g_plans.push_front(pl);
    evict_plans_locked();
    return pl;
}

bool group_plan_tiles(const pir_rowsel_item *items, uint32_t count, uint32_t *tiles) {
    std::vector<std::pair<const pir_db *, uint32_t>> key(count);
    for (uint32_t i = 0; i < count; ++i) key[i] = {items[i].db, items[i].B};
    int dev = 0;
    PIR_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_plan_mu);
    std::shared_ptr<GroupPlan> pl;
    for (const auto &p : g_plans)
        if (p->key == key && p->device == dev) {
            pl = p;
            break;
        }
    if (!pl) return false;
    for (uint32_t i = 0; i < count; ++i) {
        uint32_t *t = tiles + PIR_GROUPED_TILE_WORDS * i;
        for (int w = 0; w < PIR_GROUPED_TILE_WORDS; ++w) t[w] = 0;
        if (pl->item_job[i] == SIZE_MAX) continue;
        const size_t k = pl->item_job[i];
        const MfmaJob &j = pl->jobs[k];
        if (pl->kind[k] == G_QRES) {
            t[0] = 1;
            t[1] = qres_rows(j.wm);
            t[2] = qres_cols(j.wm);
        } else {
            t[0] = j.pts;
            t[1] = 32 * j.wm;
            t[2] = 32 * (NWAVE / (j.pts * j.wm));
        }
        t[3] = pl->kind[k];
        t[4] = pl->kind[k] == G_QRES || pl->per_job;
    }
    return true;
}

void launch_rowsel_mfma_grouped(const pir_rowsel_item *items, uint32_t count, hipStream_t st) {
    const std::shared_ptr<GroupPlan> plan = get_plan(items, count, st);
    GroupPlan &pl = *plan;
    if (pl.jobs.empty()) return;
    for (uint32_t i = 0; i < count; ++i)
        if (pl.item_job[i] != SIZE_MAX) {
            const MfmaJob &j = pl.jobs[pl.item_job[i]];
            launch_query_digits_rows(*items[i].db, items[i].q_dev, 2 * items[i].B, const_cast<int8_t *>(j.qd),
                                     j.mstride, 0, st);
        }
    {
        KernelTimer::Scope timed(st);
        launch_plan_gemms(pl, st);
    }
    for (uint32_t i = 0; i < count; ++i) {
        if (pl.item_job[i] == SIZE_MAX) continue;
        const MfmaJob &j = pl.jobs[pl.item_job[i]];
        launch_out_transpose(j.out, items[i].out_dev, j.m_rows, j.mp, j.d1, (uint32_t)items[i].db->slots(), st);
    }
}

void release_group_plans(const pir_db *db) {
    std::lock_guard<std::mutex> lock(g_plan_mu);
    g_plans.remove_if([db](const std::shared_ptr<GroupPlan> &p) {
        for (const auto &k : p->key)
            if (k.first == db) return true;
        return false;
    });
}

}  // namespace pir
