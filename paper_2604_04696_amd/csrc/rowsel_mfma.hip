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
// with Kp = D0 rounded up to 64 and Mp = 2B rounded up to 32, zero padded.
#include <algorithm>
#include <cstdio>
#include <cstdlib>

#include "common.h"
#include "modarith.h"

namespace pir {

typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x16 __attribute__((ext_vector_type(16)));

struct ModQ4m {
    ModQ m[PIR_MAX_PRIMES];
};

// ----------------------------------------------------------- digit planes
// Generic transpose + digit split:  element (r, k, p) of a uint32 source at
// src[r*s_r + (k - klo)*s_k + p] (points p contiguous) goes to byte k%64 of
// row r of chunk k/64 of plane [p][d]: dst[(((p*4 + d)*Kp/64 + k/64)*R + r)*64 + k%64].  A block takes one row r,
// 64 k (aligned) and 64 points: it reads 64 runs of 256 bytes, splits in
// LDS, and writes 64-byte runs.  k outside [klo, khi) and rows r >= r_valid
// read as zero; 16-byte chunks that straddle [klo, khi) (only when loading
// a DB in row ranges) are written byte by byte so neighbouring ranges are
// not overwritten.
__global__ void __launch_bounds__(256)
digit_planes_kernel(const uint32_t *__restrict__ src, uint64_t s_r, uint64_t s_k,
                    int8_t *__restrict__ dst, uint32_t R, uint32_t r_valid, uint32_t P,
                    uint32_t kp, uint32_t klo, uint32_t khi, uint32_t kvalid, uint32_t kblk0,
                    uint32_t nkblk) {
    __shared__ uint32_t tile[64][65];
    const uint32_t tid = threadIdx.x;
    uint64_t b = blockIdx.x;
    const uint32_t npb = (P + 63) / 64;
    const uint32_t pb = (uint32_t)(b % npb);
    b /= npb;
    const uint32_t kb = kblk0 + (uint32_t)(b % nkblk);
    const uint32_t r = (uint32_t)(b / nkblk);
    const uint32_t k0 = kb * 64, p0 = pb * 64;
    const bool rv = r < r_valid;

    for (uint32_t e = tid; e < 64 * 64; e += 256) {
        uint32_t kk = e / 64, pp = e % 64;
        uint32_t k = k0 + kk;
        uint32_t v = 0;
        if (rv && k >= klo && k < khi && p0 + pp < P)
            v = split_digits(src[(uint64_t)r * s_r + (uint64_t)(k - klo) * s_k + p0 + pp]);
        tile[kk][pp] = v;
    }
    __syncthreads();

    for (uint32_t c = tid; c < 1024; c += 256) {
        const uint32_t kq = c % 4, d = (c / 4) % 4, pp = c / 16;
        const uint32_t kc = k0 + kq * 16;
        if (kc >= kp || p0 + pp >= P) continue;
        const uint32_t hv = std::min(kc + 16, kvalid);   // k >= kvalid is padding
        const bool inside = kc >= klo && hv <= khi;
        uint32_t w[4];
#pragma unroll
        for (int i4 = 0; i4 < 4; ++i4) {
            uint32_t x = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                x |= ((tile[kq * 16 + i4 * 4 + i][pp] >> (8 * d)) & 0xFFu) << (8 * i);
            w[i4] = x;
        }
        int8_t *o = dst + ((((uint64_t)(p0 + pp) * 4 + d) * (kp / 64) + kc / 64) * R + r) * 64 + kc % 64;
        if (inside) {
            *reinterpret_cast<uint4 *>(o) = make_uint4(w[0], w[1], w[2], w[3]);
        } else {
            for (int i = 0; i < 16; ++i) {
                const uint32_t k = kc + i;
                if (k >= klo && k < khi && k < kvalid) o[i] = (int8_t)(w[i / 4] >> (8 * (i % 4)));
            }
        }
    }
}

static void launch_digit_planes(const uint32_t *src, uint64_t s_r, uint64_t s_k, int8_t *dst,
                                uint32_t R, uint32_t r_valid, uint32_t P, uint32_t kp,
                                uint32_t klo, uint32_t khi, uint32_t kvalid, hipStream_t st) {
    if (klo >= khi || R == 0) return;
    // blocks cover [klo, khi); when khi = D0 the last block also zero-fills
    // the padding up to Kp (Kp is D0 rounded up to 64)
    const uint32_t kb0 = klo / 64, kb1 = (khi + 63) / 64;
    const uint32_t nkb = kb1 - kb0;
    const uint64_t blocks = (uint64_t)((P + 63) / 64) * nkb * R;
    if (blocks >= (1ull << 31)) PIR_FAIL(PIR_EINVAL, "digit-plane launch too large");
    digit_planes_kernel<<<(uint32_t)blocks, 256, 0, st>>>(src, s_r, s_k, dst, R, r_valid, P, kp, klo,
                                                          khi, kvalid, kb0, nkb);
    PIR_LAUNCH_CHECK();
}

// DB rows [row0, row0+nrows) of an NTT-domain source [nrows][D1][L][N]:
// the GEMM's k is the DB row, r the DB column.
void launch_db_layout_mfma(const pir_db &db, const uint32_t *ntt_src, uint32_t row0,
                           uint32_t nrows, hipStream_t st) {
    const auto &p = db.p;
    const uint32_t P = p.n * p.nprimes;
    // src index = (k - row0)*D1*P + n*P + point
    launch_digit_planes(ntt_src, P, (uint64_t)p.d1 * P, db.mfma.data, p.d1, p.d1, P, db.mfma.kp,
                        row0, row0 + nrows, p.d0, st);
}

size_t mfma_query_scratch_bytes(const pir_db &db, uint32_t B) {
    const uint64_t mp = (2ull * B + 31) / 32 * 32;
    return (size_t)db.slots() * 4 * mp * db.mfma.kp;
}

// ------------------------------------------------------------- the GEMM
constexpr int KCH = 64;             // k bytes per pipeline step (two MFMA k-steps of 32)
constexpr uint32_t KSUPER = 2048;   // rows per int32 accumulation (bound above)

// LDS rows are 64 bytes (four 16-byte chunks).  Chunk c of row r is stored at
// position c ^ swz(r).  Reading one chunk index across consecutive rows then
// hits distinct 16-byte bank groups both for 8 rows in 128 bytes of banks and
// for 16 rows in 256 bytes of banks (rows r, r+4, r+8, r+12 get four
// different positions).
__device__ __forceinline__ uint32_t swz(uint32_t r) { return ((r >> 1) ^ (r >> 3)) & 3u; }

// Workgroup barrier without the memory fences of __syncthreads(): those make
// the compiler wait for every outstanding global load, which would drain the
// operand pipeline.  LDS visibility is handled explicitly: each wave waits
// for its own direct-to-LDS loads (wait_vmcnt) before the barrier, and its
// LDS reads of a buffer complete (their values are consumed) before it
// reaches the barrier after which that buffer is refilled.
__device__ __forceinline__ void block_barrier() { asm volatile("s_barrier" ::: "memory"); }

// Waits until at most N vector-memory loads of this wave are outstanding
// (loads complete in issue order for this count).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// One block = a group of four consecutive points of one prime and a BM x BN
// output tile; WM x WN waves, each owning a 32 x 32 sub-tile with seven int32
// class accumulators (sixteen digit products per k-step of 32).
//
// Operands move global -> LDS with global_load_lds_dwordx4 (no register
// staging) into STAGES buffers: while the waves run the MFMAs of step t, the
// loads of steps t+1 .. t+STAGES-1 are in flight.  Steps run over (point, k chunk) in one
// sequence, so the pipeline does not drain between the four points.  The
// four residues of each (m, n) stay in registers and leave as one 16-byte
// vector into the boundary layout [B][2][D1][L][N].
template <int WM, int WN, int STAGES>
__global__ void __launch_bounds__(64 * WM * WN) __attribute__((amdgpu_waves_per_eu(2, 2)))
rowsel_mfma_kernel(const int8_t *__restrict__ dbd, const int8_t *__restrict__ qd,
                   uint32_t *__restrict__ out, uint32_t m_rows, uint32_t mp, uint32_t d1,
                   uint32_t kp, uint32_t L, uint32_t N, uint32_t nblk_m, uint32_t nblk_n,
                   ModQ4m mods) {
    constexpr int BM = 32 * WM, BN = 32 * WN, NW = WM * WN;
    constexpr int A_BYTES = 4 * BM * KCH, B_BYTES = 4 * BN * KCH;
    constexpr int BUF = A_BYTES + B_BYTES;
    constexpr int A_INST = 4 * BM / 16, B_INST = 4 * BN / 16;   // 1 KiB = 16 rows per instruction
    constexpr int INST = A_INST + B_INST;
    static_assert(INST % NW == 0, "load instructions must divide among the waves");
    constexpr int LPW = INST / NW;   // load instructions per wave per step
    __shared__ __attribute__((aligned(1024))) int8_t lds[STAGES * BUF];

    const uint32_t tid = threadIdx.x;
    // Block order: eight consecutive point groups (32 points = one 128-byte
    // output line per (m, n)) run side by side for each output tile, so the
    // 16-byte stores of those groups meet in one XCD's L2 and leave as whole
    // lines; the tiles of one octet follow each other closely, so its query
    // planes are re-read from L2.
    const uint32_t groups = gridDim.x / (nblk_m * nblk_n);
    const uint32_t bid = xcd_remap(blockIdx.x, gridDim.x);
    const uint32_t tiles = nblk_m * nblk_n, per_oct = 8 * tiles, full = groups / 8;
    uint32_t gg, tile;
    if (bid < full * per_oct) {
        gg = (bid / per_oct) * 8 + bid % 8;
        tile = (bid % per_oct) / 8;
    } else {
        const uint32_t rem = bid - full * per_oct, w = groups - full * 8;
        gg = full * 8 + rem % w;
        tile = rem / w;
    }
    const uint32_t nb = tile % nblk_n, mb = tile / nblk_n;
    const uint32_t G = N / 4;
    const uint32_t l = gg / G, g = gg % G;
    const ModQ mq = mods.m[l];
    const uint32_t wave = tid / 64, lane = tid % 64;
    const uint32_t wm = wave / WN, wn = wave % WN;
    const uint32_t m0 = mb * BM, n0 = nb * BN;
    const bool wave_active = m0 + wm * 32 < mp && n0 + wn * 32 < d1;
    const uint32_t nkc = kp / KCH;
    const uint32_t T = 4 * nkc;              // pipeline steps: 4 points x k chunks

    // Per-lane byte offsets of this wave's load instructions inside their
    // operand plane (fixed for the whole block), and the wave-uniform parts
    // (plane, LDS destination) computed per step with scalar arithmetic.
    const uint32_t wv = __builtin_amdgcn_readfirstlane(wave);
    const uint32_t lrow = lane / 4, lchunk = lane % 4;
    uint32_t loff[LPW];
#pragma unroll
    for (int i = 0; i < LPW; ++i) {
        const uint32_t ii = wv + i * NW;
        if (ii < (uint32_t)A_INST) {
            const uint32_t r = (ii % (BM / 16)) * 16 + lrow;
            loff[i] = min(m0 + r, mp - 1) * KCH + 16 * (lchunk ^ swz(r));
        } else {
            const uint32_t jj = ii - A_INST;
            const uint32_t r = (jj % (BN / 16)) * 16 + lrow;
            loff[i] = min(n0 + r, d1 - 1) * KCH + 16 * (lchunk ^ swz(r));
        }
    }
    const uint64_t a_plane = (uint64_t)mp * KCH, b_plane = (uint64_t)d1 * KCH;   // bytes per (p, d, kc)

    auto issue = [&](uint32_t t) {
        const uint32_t s = t / nkc, kc = t % nkc;
        const uint64_t p = (uint64_t)l * N + 4 * g + s;
        int8_t *buf = lds + (t % STAGES) * BUF;
#pragma unroll
        for (int i = 0; i < LPW; ++i) {
            const uint32_t ii = wv + i * NW;
            const int8_t *plane;
            int8_t *dst;
            if (ii < (uint32_t)A_INST) {
                const uint32_t d = ii / (BM / 16);
                plane = qd + ((p * 4 + d) * nkc + kc) * a_plane;
                dst = buf + d * BM * KCH + (ii % (BM / 16)) * 1024;
            } else {
                const uint32_t jj = ii - A_INST;
                const uint32_t d = jj / (BN / 16);
                plane = dbd + ((p * 4 + d) * nkc + kc) * b_plane;
                dst = buf + A_BYTES + d * BN * KCH + (jj % (BN / 16)) * 1024;
            }
            // (a named pointer: an arithmetic expression as the builtin's
            // argument stops the host pass from emitting the kernel stub)
            const int8_t *src = plane + loff[i];
            __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)dst, 16, 0, 0);
        }
    };

    uint32_t res[4][16];
    i32x16 acc[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) acc[c] = (i32x16){};

    // fragment byte offsets inside a buffer, per k-step (digit planes follow
    // at fixed strides)
    const uint32_t ar = wm * 32 + lane % 32, br = wn * 32 + lane % 32;   // fragment rows
    const uint32_t half = lane / 32;
    uint32_t aoff[2], boff[2];
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
        aoff[ks] = ar * KCH + 16 * ((2 * ks + half) ^ swz(ar));
        boff[ks] = A_BYTES + br * KCH + 16 * ((2 * ks + half) ^ swz(br));
    }

    for (uint32_t t = 0; t + 1 < STAGES && t < T; ++t) issue(t);
    for (uint32_t t = 0; t < T; ++t) {
        // this wave's loads of step t are done once only the later steps'
        // (up to STAGES-2 of them) are outstanding; the barrier then makes
        // every wave's part visible and frees the buffer of step t-1
        if (t + STAGES - 2 < T) wait_vmcnt<(STAGES - 2) * LPW>();
        else wait_vmcnt<0>();
        block_barrier();
        if (t + STAGES - 1 < T) issue(t + STAGES - 1);
        const int8_t *buf = lds + (t % STAGES) * BUF;
        if (wave_active) {
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                i32x4 a[4];
#pragma unroll
                for (int d = 0; d < 4; ++d)
                    a[d] = *reinterpret_cast<const i32x4 *>(buf + aoff[ks] + d * BM * KCH);
                // one DB digit at a time: four MFMAs into four different classes
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const i32x4 b = *reinterpret_cast<const i32x4 *>(buf + boff[ks] + j * BN * KCH);
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        acc[i + j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[i], b, acc[i + j], 0, 0, 0);
                }
            }
        }
        const uint32_t s = t / nkc, kc = t % nkc;
        const bool last = kc + 1 == nkc;
        const bool flush = last || ((kc + 1) * KCH) % KSUPER == 0;
        if (flush) {
            // recombine the seven classes: sum_s G_s * 2^(8s) mod q
            uint32_t part[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                int gr[7];
#pragma unroll
                for (int c = 0; c < 7; ++c) gr[c] = acc[c][r];
                part[r] = combine_classes(gr, mq);
            }
            const bool first = kc + 1 <= KSUPER / KCH;
#pragma unroll
            for (int ss = 0; ss < 4; ++ss) {
                if ((uint32_t)ss != s) continue;
#pragma unroll
                for (int r = 0; r < 16; ++r) res[ss][r] = first ? part[r] : add_mod(res[ss][r], part[r], mq.q);
            }
#pragma unroll
            for (int c = 0; c < 7; ++c) acc[c] = (i32x16){};
        }
    }

    if (!wave_active) return;
    // accumulator element r of a lane: row 8*(r/4) + 4*(lane/32) + r%4, column lane%32
    const uint32_t n = n0 + wn * 32 + lane % 32;
    if (n >= d1) return;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const uint32_t m = m0 + wm * 32 + 8 * (r / 4) + 4 * half + (r % 4);
        if (m < m_rows)
            *reinterpret_cast<uint4 *>(out + (((uint64_t)m * d1 + n) * L + l) * N + 4 * g) =
                make_uint4(res[0][r], res[1][r], res[2][r], res[3][r]);
    }
}

template <int WM, int WN, int STAGES>
static void launch_mfma_tile(const pir_db &db, const int8_t *qd, uint32_t *out, uint32_t m_rows,
                             uint32_t mp, const ModQ4m &mods, hipStream_t st) {
    const auto &p = db.p;
    const uint64_t groups = (uint64_t)p.nprimes * (p.n / 4);
    const uint32_t nblk_m = (mp + 32 * WM - 1) / (32 * WM);
    const uint32_t nblk_n = (p.d1 + 32 * WN - 1) / (32 * WN);
    const uint64_t blocks = groups * nblk_m * nblk_n;
    if (blocks >= (1ull << 31)) PIR_FAIL(PIR_EINVAL, "grid too large");
    rowsel_mfma_kernel<WM, WN, STAGES><<<(uint32_t)blocks, 64 * WM * WN, 0, st>>>(
        db.mfma.data, qd, out, m_rows, mp, p.d1, db.mfma.kp, p.nprimes, p.n, nblk_m, nblk_n, mods);
    PIR_LAUNCH_CHECK();
}

// Tile variants: (waves along m, waves along n, pipeline stages).
struct MfmaTile {
    int wm, wn, stages;
};

static const MfmaTile kTiles[] = {
    {4, 2, 3}, {2, 4, 3}, {1, 8, 2}, {2, 2, 2}, {4, 1, 2}, {1, 4, 2}, {2, 2, 3},
};

static void launch_tile(const MfmaTile &t, const pir_db &db, const int8_t *qd, uint32_t *out,
                        uint32_t m_rows, uint32_t mp, const ModQ4m &mods, hipStream_t st) {
#define PIR_TILE(a, b, c)                                                      \
    if (t.wm == a && t.wn == b && t.stages == c)                               \
        return launch_mfma_tile<a, b, c>(db, qd, out, m_rows, mp, mods, st);
    PIR_TILE(4, 2, 3)
    PIR_TILE(2, 4, 3)
    PIR_TILE(1, 8, 2)
    PIR_TILE(2, 2, 2)
    PIR_TILE(4, 1, 2)
    PIR_TILE(1, 4, 2)
    PIR_TILE(2, 2, 3)
#undef PIR_TILE
    PIR_FAIL(PIR_EINVAL, "unknown MFMA tile %d,%d,%d", t.wm, t.wn, t.stages);
}

static MfmaTile pick_tile(uint32_t mp) {
    if (const char *e = std::getenv("PIR_MFMA_TILE")) {   // explicit choice (tuning runs)
        MfmaTile t{};
        if (std::sscanf(e, "%d,%d,%d", &t.wm, &t.wn, &t.stages) == 3) return t;
    }
    if (mp >= 128) return {4, 2, 3};
    if (mp >= 64) return {2, 4, 3};
    return {1, 8, 2};
}

void launch_rowsel_mfma(const pir_db &db, const uint32_t *q, uint32_t B, uint32_t *out,
                        hipStream_t st) {
    const auto &p = db.p;
    const uint32_t m_rows = 2 * B;
    const uint32_t mp = (m_rows + 31) / 32 * 32;
    const uint32_t P = p.n * p.nprimes;
    const uint32_t kp = db.mfma.kp;

    // query ingest: [B][2][D0][L][N] -> [P][4][Kp/64][Mp][64] digit planes
    int8_t *qd = nullptr;
    const size_t qbytes = mfma_query_scratch_bytes(db, B);
    PIR_HIP(hipMallocAsync((void **)&qd, qbytes, st));
    launch_digit_planes(q, (uint64_t)p.d0 * P, P, qd, mp, m_rows, P, kp, 0, p.d0, p.d0, st);

    ModQ4m mods{};
    for (uint32_t l = 0; l < p.nprimes; ++l) mods.m[l] = db.mod[l];
    launch_tile(pick_tile(mp), db, qd, out, m_rows, mp, mods, st);
    PIR_HIP(hipFreeAsync(qd, st));
}

}  // namespace pir
