// RowSel on the vector ALUs for larger batches (2B > 8): exact 32x32->64-bit
// multiply-adds (v_mad_u64_u32) with lazy 64-bit accumulation; one to four
// clients take the streaming kernel of rowsel_stream.hip.
//
// The operation (sec. 2.3): for each of the L*N points p and prime q_l,
//   out[m][n] = sum_k Q[m][k] * DB[k][n] mod q_l.
// The tiled kernel reads the DB from the VALU layout [L][N/4][S][D0][W][4]: a
// thread owns four consecutive points of one prime (one 16-byte vector), so
// the four independent per-point GEMMs of a group advance in lock step, and
// the D0 rows of a 256-column strip of a group are one contiguous run (the
// transposed, point-innermost layout of the paper's sec. 5.2.1).  The query
// is first copied into a group-major layout (valu_query_kernel); the output
// is written in the boundary layout directly (for fixed (m, n) the four
// points of a group are one 16-byte vector there).
//
// Accumulation: products of residues are < 2^60, so a 64-bit sum absorbs
// fifteen of them on top of a folded remainder (< 2^60 + 2^32); every
// fifteen rows the sum is folded (hi*2^32 + lo -> hi*(2^32 mod q) + lo) and
// one Barrett reduction at the end yields the canonical residue.
#include <algorithm>

#include "common.h"
#include "modarith.h"

namespace pir {

struct ModQ4 {
    ModQ m[PIR_MAX_PRIMES];
};

__device__ __forceinline__ void mad4(uint64_t (&acc)[4], const uint4 &a, const uint4 &b) {
    acc[0] += (uint64_t)a.x * b.x;
    acc[1] += (uint64_t)a.y * b.y;
    acc[2] += (uint64_t)a.z * b.z;
    acc[3] += (uint64_t)a.w * b.w;
}

// ---------------------------------------------------------- query ingest
// Larger batches read the query from a group-major copy
//   qv[G_all][D0][Mp][4] u32   (G_all = L*N/4 point groups, Mp = rows rounded
//                               up to the tile height, zero padded)
// so that a tile's query rows for one k are one contiguous 1 KiB run and a
// group's whole slice (D0 x Mp vectors) is contiguous and stays in L2 while
// the group's column tiles run.  A block moves 8 groups x 16 k x 16 rows:
// 128-byte reads (8 consecutive groups of one (row, k)) and 256-byte writes
// (16 consecutive rows of one (group, k)) through a padded LDS tile.
__global__ void __launch_bounds__(256)
valu_query_kernel(const uint4 *__restrict__ q, uint4 *__restrict__ qv, uint32_t m_rows, uint32_t mp,
                  uint32_t d0, uint32_t gall, uint32_t nkb, uint32_t ngb) {
    // [group][k][row], group stride 273 vectors (not a multiple of the bank
    // period) so the 8 groups a wave writes at once fall in distinct banks
    __shared__ uint4 tile[8 * 273];
    const uint32_t tid = threadIdx.x;
    uint32_t b = blockIdx.x;
    const uint32_t gb = b % ngb;
    b /= ngb;
    const uint32_t kb = b % nkb;
    const uint32_t mb = b / nkb;
    const uint32_t g0 = gb * 8, k0 = kb * 16, m0 = mb * 16;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const uint32_t e = tid + 256 * j, gi = e % 8, ki = (e / 8) % 16, mi = e / 128;
        const uint32_t g = g0 + gi, k = k0 + ki, m = m0 + mi;
        tile[gi * 273 + ki * 17 + mi] = g < gall && k < d0 && m < m_rows ? q[((uint64_t)m * d0 + k) * gall + g]
                                                                          : make_uint4(0, 0, 0, 0);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const uint32_t e = tid + 256 * j, mi = e % 16, ki = (e / 16) % 16, gi = e / 256;
        const uint32_t g = g0 + gi, k = k0 + ki;
        if (g < gall && k < d0) qv[((uint64_t)g * d0 + k) * mp + m0 + mi] = tile[gi * 273 + ki * 17 + mi];
    }
}

// ------------------------------------------------------------------ tiled
// Larger batches: a 256-thread block computes a BM x BN output tile of one
// point group (four points), thread tile TM x TN x 4 points, staging KC rows
// of query and DB vectors in LDS per step (the classic tiled GEMM of
// sec. 5.1.1 with an extra innermost point dimension of four).
constexpr int TILE_THREADS = 256;
constexpr int TM = 4, TN = 2;            // per-thread rows x columns
constexpr int BM = 16 * TM, BN = 16 * TN;
constexpr int TKC = 30;                   // rows per LDS step (two lazy groups)
static_assert(VALU_STRIP % BN == 0, "a tiled block's columns lie in one DB strip");

// WIDE (some prime >= 2^30): each sum counts its 64-bit wraps instead of
// being folded (mad_wide / reduce_wide in modarith.h).
template <bool WIDE>
__global__ void __launch_bounds__(TILE_THREADS)
rowsel_tiled_kernel(const uint4 *__restrict__ db, const uint4 *__restrict__ qv,
                    uint32_t *__restrict__ out, uint32_t m_rows, uint32_t mp, uint32_t d0, uint32_t d1,
                    uint32_t L, uint32_t N, uint32_t nblk_m, uint32_t nblk_n, ModQ4 mods) {
    __shared__ uint4 qs[TKC][BM];
    __shared__ uint4 ds[TKC][BN];

    const uint32_t tid = threadIdx.x;
    const uint32_t bid = xcd_remap(blockIdx.x, gridDim.x);
    const uint32_t nb = bid % nblk_n;
    const uint32_t mb = (bid / nblk_n) % nblk_m;
    const uint32_t gg = bid / (nblk_n * nblk_m);
    const uint32_t G = N / 4;
    const uint32_t l = gg / G, g = gg % G;
    const ModQ mq = mods.m[l];
    const uint32_t tm = tid / 16, tn = tid % 16;   // thread's rows tm + 16*i, cols tn + 16*j
    const uint32_t m0 = mb * BM, n0 = nb * BN;

    // the block's 32 columns lie in one strip (VALU_STRIP is a multiple of BN)
    const uint32_t strip = n0 / VALU_STRIP, sw = valu_strip_width(strip, d1), c0 = n0 % VALU_STRIP;
    const uint4 *dgrp = db + valu_strip_base(gg, strip, d0, d1) + c0;
    const uint4 *qgrp = qv + (uint64_t)gg * d0 * mp + m0;   // rows m0.. of this group, k-major
    uint64_t acc[TM][TN][4];
    uint32_t wraps[TM][TN][4];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                acc[i][j][s] = 0;
                wraps[i][j][s] = 0;
            }

    for (uint32_t k0 = 0; k0 < d0; k0 += TKC) {
        const uint32_t kc = min((uint32_t)TKC, d0 - k0);
        __syncthreads();
        for (uint32_t e = tid; e < TKC * BM; e += TILE_THREADS) {
            uint32_t kk = e / BM, mm = e % BM;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (kk < kc) v = qgrp[(uint64_t)(k0 + kk) * mp + mm];   // rows >= m_rows are zero
            qs[kk][mm] = v;
        }
        for (uint32_t e = tid; e < TKC * BN; e += TILE_THREADS) {
            uint32_t kk = e / BN, nn = e % BN;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (kk < kc && n0 + nn < d1) v = dgrp[(uint64_t)(k0 + kk) * sw + nn];
            ds[kk][nn] = v;
        }
        __syncthreads();
        // zero-padded rows contribute nothing, so full lazy groups are safe
#pragma unroll 1
        for (uint32_t kh = 0; kh < TKC; kh += 15) {
#pragma unroll 5
            for (uint32_t kk = kh; kk < kh + 15; ++kk) {
                uint4 a[TM], b[TN];
#pragma unroll
                for (int i = 0; i < TM; ++i) a[i] = qs[kk][tm + 16 * i];
#pragma unroll
                for (int j = 0; j < TN; ++j) b[j] = ds[kk][tn + 16 * j];
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j) {
                        if (WIDE) {
                            mad_wide(acc[i][j][0], wraps[i][j][0], a[i].x, b[j].x);
                            mad_wide(acc[i][j][1], wraps[i][j][1], a[i].y, b[j].y);
                            mad_wide(acc[i][j][2], wraps[i][j][2], a[i].z, b[j].z);
                            mad_wide(acc[i][j][3], wraps[i][j][3], a[i].w, b[j].w);
                        } else {
                            mad4(acc[i][j], a[i], b[j]);
                        }
                    }
            }
            if (!WIDE) {
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j)
#pragma unroll
                        for (int s = 0; s < 4; ++s) acc[i][j][s] = lazy_fold(acc[i][j][s], mq);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        const uint32_t m = m0 + tm + 16 * i;
        if (m >= m_rows) continue;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const uint32_t n = n0 + tn + 16 * j;
            if (n >= d1) continue;
            uint4 r;
            if (WIDE) {
                r.x = reduce_wide(acc[i][j][0], wraps[i][j][0], mq);
                r.y = reduce_wide(acc[i][j][1], wraps[i][j][1], mq);
                r.z = reduce_wide(acc[i][j][2], wraps[i][j][2], mq);
                r.w = reduce_wide(acc[i][j][3], wraps[i][j][3], mq);
            } else {
                r.x = reduce64(acc[i][j][0], mq);
                r.y = reduce64(acc[i][j][1], mq);
                r.z = reduce64(acc[i][j][2], mq);
                r.w = reduce64(acc[i][j][3], mq);
            }
            *reinterpret_cast<uint4 *>(out + (((uint64_t)m * d1 + n) * L + l) * N + 4 * g) = r;
        }
    }
}

static ModQ4 pack_mods(const pir_db &db) {
    ModQ4 m{};
    for (uint32_t l = 0; l < db.p.nprimes; ++l) m.m[l] = db.mod[l];
    return m;
}

void launch_rowsel_valu(const pir_db &db, const uint32_t *q, uint32_t B, uint32_t *out,
                        hipStream_t st) {
    const auto &p = db.p;
    const uint32_t m_rows = 2 * B;
    const uint64_t groups = (uint64_t)p.nprimes * (p.n / 4);
    const ModQ4 mods = pack_mods(db);
    const uint4 *dbv = reinterpret_cast<const uint4 *>(db.valu.data);
    if (m_rows <= 8) {
        launch_rowsel_stream(db, q, B, out, st);
        return;
    } else {
        const uint32_t nblk_m = (m_rows + BM - 1) / BM;
        const uint32_t nblk_n = (p.d1 + BN - 1) / BN;
        const uint32_t mp = nblk_m * BM;
        const uint64_t blocks = groups * nblk_m * nblk_n;
        const uint32_t nkb = (p.d0 + 15) / 16, ngb = (uint32_t)((groups + 7) / 8);
        const uint64_t iblocks = (uint64_t)(mp / 16) * nkb * ngb;
        if (blocks >= (1ull << 31) || iblocks >= (1ull << 31)) PIR_FAIL(PIR_EINVAL, "grid too large");
        // stream-ordered scratch for the group-major query copy
        StreamScratch buf(groups * p.d0 * mp * sizeof(uint4), st);
        uint4 *qv = buf.as<uint4>();
        valu_query_kernel<<<(uint32_t)iblocks, 256, 0, st>>>(reinterpret_cast<const uint4 *>(q), qv, m_rows, mp,
                                                             p.d0, (uint32_t)groups, nkb, ngb);
        PIR_LAUNCH_CHECK();
        KernelTimer::Scope timed(st);
        if (db.wide)
            rowsel_tiled_kernel<true><<<(uint32_t)blocks, TILE_THREADS, 0, st>>>(
                dbv, qv, out, m_rows, mp, p.d0, p.d1, p.nprimes, p.n, nblk_m, nblk_n, mods);
        else
            rowsel_tiled_kernel<false><<<(uint32_t)blocks, TILE_THREADS, 0, st>>>(
                dbv, qv, out, m_rows, mp, p.d0, p.d1, p.nprimes, p.n, nblk_m, nblk_n, mods);
        PIR_LAUNCH_CHECK();
        return;
    }
    PIR_LAUNCH_CHECK();
}

}  // namespace pir
