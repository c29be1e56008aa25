// RowSel for one to four clients on the vector ALUs: a pure HBM stream.
//
// The operation (sec. 2.3): for each of the L*N points p and prime q_l,
//   out[m][n] = sum_k Q[m][k] * DB[k][n] mod q_l,   m < 2B <= 8.
// The DB is read from the VALU layout [L][N/4][S][D0][W][4] (see
// DbLayoutValu): a thread owns four consecutive points of one prime (one
// 16-byte vector) and one column; a block owns one 256-column strip of one
// point group, whose D0 rows are one contiguous run that the block reads
// front to back with non-temporal 16-byte loads, eight rows per batch, the
// next batch in flight while the current one is multiplied.  The query is
// read in the boundary layout.  Products of residues are < 2^60; a 64-bit
// sum absorbs fifteen of them on top of a folded remainder, the sum is
// folded (hi*2^32 + lo -> hi*(2^32 mod q) + lo) after every batch and one
// Barrett reduction at the end yields the canonical residue.
//
// Results leave the kernel through a staging buffer [L*N/4][2B][D1] of
// 16-byte vectors: every wave stores one contiguous kilobyte with
// non-temporal stores, and a transpose kernel then writes the boundary
// layout.  Storing into the boundary layout directly scatters one 16-byte
// piece per lane over as many cache lines, and those partial-line writes,
// interleaved with the DB stream, cost about a tenth of the kernel's time.
#include <optional>
#include <type_traits>

#include "common.h"
#include "modarith.h"

namespace pir {

struct ModQ4s {
    ModQ m[PIR_MAX_PRIMES];
};

__device__ __forceinline__ void mad4s(uint64_t (&acc)[4], const uint4 &a, const uint4 &b) {
    acc[0] += (uint64_t)a.x * b.x;
    acc[1] += (uint64_t)a.y * b.y;
    acc[2] += (uint64_t)a.z * b.z;
    acc[3] += (uint64_t)a.w * b.w;
}

// --------------------------------------------------------------- streaming
// Small batches (m = 2B <= 8 rows): the whole m extent lives in registers;
// a block owns one point group and 256 consecutive columns and streams the
// group's DB rows once.  The query vector of (m, k) is the same for every
// lane, so it is read with scalar loads into SGPRs and feeds
// v_mad_u64_u32 as its scalar operand: no LDS staging, no VGPRs.  This is
// the HBM-bound regime of one client (sec. 3.1): two multiply-adds per
// 4-byte DB word.
constexpr int STREAM_THREADS = 256;
static_assert(STREAM_THREADS == VALU_STRIP, "a streaming block covers one DB strip");
constexpr int STREAM_ROWS = 8;   // rows per load batch and per fold
static_assert(STREAM_ROWS <= 15, "a 64-bit sum absorbs at most fifteen products between folds");

// WIDE (some prime >= 2^30): products reach 2^64, so each sum counts its
// wraps instead of being folded (mad_wide / reduce_wide in modarith.h).
template <int MB, bool WIDE>
__global__ void __launch_bounds__(STREAM_THREADS)
rowsel_stream_kernel(const uint4 *__restrict__ db, const uint32_t *__restrict__ qry,
                     uint4 *__restrict__ stage, uint32_t d0, uint32_t d1, uint32_t L, uint32_t N,
                     uint32_t nblk_n, ModQ4s mods) {
    const uint32_t tid = threadIdx.x;
    const uint32_t bid = xcd_remap(blockIdx.x, gridDim.x);
    const uint32_t nb = bid % nblk_n;
    const uint32_t gg = bid / nblk_n;          // point group over all primes
    const uint32_t G = N / 4;
    const uint32_t l = gg / G, g = gg % G;
    const ModQ mq = mods.m[l];
    const uint32_t n = nb * STREAM_THREADS + tid;
    if (n >= d1) return;

    // the block's columns are strip nb: its rows are one contiguous run
    const uint32_t w = valu_strip_width(nb, d1);
    const uint4 *dcol = db + valu_strip_base(gg, nb, d0, d1) + tid;
    // query vector (m, k) at qv + m*mstride + k*kstride (16-byte units)
    const uint4 *qv = reinterpret_cast<const uint4 *>(qry + (uint64_t)l * N + 4 * g);
    const uint64_t kstride = (uint64_t)L * N / 4, mstride = (uint64_t)d0 * kstride;
    uint64_t acc[MB][4];
    uint32_t wraps[MB][4];
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            acc[i][s] = 0;
            wraps[i][s] = 0;
        }
    auto mad = [&](int i, const uint4 &qq, const uint4 &d) {
        if (WIDE) {
            mad_wide(acc[i][0], wraps[i][0], qq.x, d.x);
            mad_wide(acc[i][1], wraps[i][1], qq.y, d.y);
            mad_wide(acc[i][2], wraps[i][2], qq.z, d.z);
            mad_wide(acc[i][3], wraps[i][3], qq.w, d.w);
        } else {
            mad4s(acc[i], qq, d);
        }
    };

    auto load = [&](uint4 (&v)[STREAM_ROWS], uint32_t k) {
#pragma unroll
        for (int u = 0; u < STREAM_ROWS; ++u) v[u] = ld_nt(dcol + (uint64_t)(k + u) * w);
    };
    auto fold_all = [&]() {
        if (WIDE) return;
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
            for (int s = 0; s < 4; ++s) acc[i][s] = lazy_fold(acc[i][s], mq);
    };
    auto mul = [&](const uint4 (&v)[STREAM_ROWS], uint32_t k) {
#pragma unroll
        for (int u = 0; u < STREAM_ROWS; ++u)
#pragma unroll
            for (int i = 0; i < MB; ++i) mad(i, qv[i * mstride + (k + u) * kstride], v[u]);
        fold_all();
    };

    // full batches, two buffers: batch j+1 is loaded while batch j is multiplied
    const uint32_t nfull = d0 / STREAM_ROWS;
    uint4 a[STREAM_ROWS], b[STREAM_ROWS];
    if (nfull > 0) load(a, 0);
    uint32_t j = 0;
    for (; j + 2 <= nfull; j += 2) {
        load(b, (j + 1) * STREAM_ROWS);
        mul(a, j * STREAM_ROWS);
        if (j + 2 < nfull) load(a, (j + 2) * STREAM_ROWS);
        mul(b, (j + 1) * STREAM_ROWS);
    }
    if (j < nfull) mul(a, j * STREAM_ROWS);   // odd batch count: `a` holds the last one
    // ragged tail: fewer than STREAM_ROWS rows
    const uint32_t k0 = nfull * STREAM_ROWS;
    if (k0 < d0) {
        for (uint32_t k = k0; k < d0; ++k) {
            const uint4 v = ld_nt(dcol + (uint64_t)k * w);
#pragma unroll
            for (int i = 0; i < MB; ++i) mad(i, qv[i * mstride + k * kstride], v);
        }
        fold_all();
    }
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        uint4 r;
        if (WIDE) {
            r.x = reduce_wide(acc[i][0], wraps[i][0], mq);
            r.y = reduce_wide(acc[i][1], wraps[i][1], mq);
            r.z = reduce_wide(acc[i][2], wraps[i][2], mq);
            r.w = reduce_wide(acc[i][3], wraps[i][3], mq);
        } else {
            r.x = reduce64(acc[i][0], mq);
            r.y = reduce64(acc[i][1], mq);
            r.z = reduce64(acc[i][2], mq);
            r.w = reduce64(acc[i][3], mq);
        }
        st_nt(stage + ((uint64_t)gg * MB + i) * d1 + n, r);
    }
}

// Staging [GG][C] -> boundary output [C][GG], in 16-byte vectors, GG = L*N/4
// point groups and C = 2B*D1 output rows: word ((m*D1 + n)*L + l)*N + 4g of
// the output is vector (m*D1 + n)*GG + gg.  Tiles of 32 groups x 64 rows pass
// through LDS, so both sides move runs of at least 512 bytes.
constexpr int TR_G = 32, TR_C = 64;

__global__ void __launch_bounds__(256)
stream_out_transpose_kernel(const uint4 *__restrict__ stage, uint4 *__restrict__ out, uint64_t GG,
                            uint64_t C, uint32_t nblk_c) {
    __shared__ uint4 tile[TR_G][TR_C + 1];
    const uint32_t tid = threadIdx.x;
    const uint64_t c0 = (uint64_t)(blockIdx.x % nblk_c) * TR_C;
    const uint64_t g0 = (uint64_t)(blockIdx.x / nblk_c) * TR_G;
#pragma unroll
    for (int r = 0; r < TR_G * TR_C / 256; ++r) {
        const uint32_t gi = r * 4 + tid / 64, ci = tid % 64;
        if (g0 + gi < GG && c0 + ci < C) tile[gi][ci] = ld_nt(stage + (g0 + gi) * C + c0 + ci);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < TR_G * TR_C / 256; ++r) {
        const uint32_t ci = r * 8 + tid / 32, gi = tid % 32;
        if (g0 + gi < GG && c0 + ci < C) out[(c0 + ci) * GG + g0 + gi] = tile[gi][ci];
    }
}

size_t stream_staging_bytes(const pir_db &db, uint32_t B) {
    const uint64_t rows_per_pass = db.wide ? 2u : 2ull * B;
    return (size_t)db.slots() * rows_per_pass * db.p.d1 * 4;
}

void launch_rowsel_stream(const pir_db &db, const uint32_t *q, uint32_t B, uint32_t *out, hipStream_t st,
                          void *stage_buf) {
    const auto &p = db.p;
    const uint64_t groups = (uint64_t)p.nprimes * (p.n / 4);
    ModQ4s mods{};
    for (uint32_t l = 0; l < p.nprimes; ++l) mods.m[l] = db.mod[l];
    const uint4 *dbv = reinterpret_cast<const uint4 *>(db.valu.data);
    const uint32_t nblk_n = (p.d1 + STREAM_THREADS - 1) / STREAM_THREADS;
    const uint64_t blocks = groups * nblk_n;
    // With 32-bit primes the kernel's registers grow with the rows it carries
    // (two 64-bit words per sum), and beyond one client it runs at low
    // occupancy: 4 clients in one pass took 15.6 ms on the 8 GiB DB, one pass
    // per client 1.5 ms each.  So wide DBs take one pass per client, each
    // re-reading the DB.
    const uint32_t rows_per_pass = db.wide ? 2u : 2 * B;
    const uint32_t passes = 2 * B / rows_per_pass;
    const uint64_t C = (uint64_t)rows_per_pass * p.d1;
    const uint64_t nblk_c = (C + TR_C - 1) / TR_C;
    const uint64_t tblocks = nblk_c * ((groups + TR_G - 1) / TR_G);
    if (blocks >= (1ull << 31) || tblocks >= (1ull << 31)) PIR_FAIL(PIR_EINVAL, "grid too large");

    // [groups][rows][D1] vectors, reused per pass: the caller's buffer, else stream-ordered scratch
    StreamScratch scratch(stage_buf ? 0 : groups * C * sizeof(uint4), st);
    uint4 *stage = stage_buf ? static_cast<uint4 *>(stage_buf) : scratch.as<uint4>();
    const uint64_t q_rows = (uint64_t)p.d0 * p.nprimes * p.n, o_rows = (uint64_t)p.d1 * p.nprimes * p.n;
    for (uint32_t pass = 0; pass < passes; ++pass) {
        const uint32_t *qp = q + pass * rows_per_pass * q_rows;
        uint32_t *op = out + pass * rows_per_pass * o_rows;
        {
            // (no timing events around a launch into a caller's buffer: that
            // form allocates nothing, events included)
            std::optional<KernelTimer::Scope> timed;
            if (!stage_buf) timed.emplace(st);
            dim3 grid((uint32_t)blocks), block(STREAM_THREADS);
            auto go = [&](auto wide) {
                constexpr bool W = decltype(wide)::value;
                switch (rows_per_pass) {
                    case 2: rowsel_stream_kernel<2, W><<<grid, block, 0, st>>>(dbv, qp, stage, p.d0, p.d1, p.nprimes, p.n, nblk_n, mods); break;
                    case 4: rowsel_stream_kernel<4, W><<<grid, block, 0, st>>>(dbv, qp, stage, p.d0, p.d1, p.nprimes, p.n, nblk_n, mods); break;
                    case 6: rowsel_stream_kernel<6, W><<<grid, block, 0, st>>>(dbv, qp, stage, p.d0, p.d1, p.nprimes, p.n, nblk_n, mods); break;
                    case 8: rowsel_stream_kernel<8, W><<<grid, block, 0, st>>>(dbv, qp, stage, p.d0, p.d1, p.nprimes, p.n, nblk_n, mods); break;
                    default: PIR_FAIL(PIR_EINVAL, "unexpected row count %u", rows_per_pass);
                }
            };
            if (db.wide) go(std::true_type{});
            else go(std::false_type{});
            PIR_LAUNCH_CHECK();
        }
        stream_out_transpose_kernel<<<(uint32_t)tblocks, 256, 0, st>>>(stage, reinterpret_cast<uint4 *>(op), groups,
                                                                     C, (uint32_t)nblk_c);
        PIR_LAUNCH_CHECK();
    }
}

}  // namespace pir
