// RowSel for one to four clients on the vector ALUs: a pure HBM stream.
//
// The operation (sec. 2.3): for each of the L*N points p and prime q_l,
//   out[m][n] = sum_k Q[m][k] * DB[k][n] mod q_l,   m < 2B <= 8.
// The DB is read from the VALU layout [L][N/4][S][D0][W][4] (see
// DbLayoutValu): a thread owns four consecutive points of one prime (one
// 16-byte vector) and one column; a block owns one 256-column strip of one
// point group, whose D0 rows are one contiguous run that the block reads
// front to back with non-temporal 16-byte loads.  The query and the output
// stay in the boundary layout.  Products of residues are < 2^60; a 64-bit
// sum absorbs fifteen of them on top of a folded remainder, every fifteen
// rows the sum is folded (hi*2^32 + lo -> hi*(2^32 mod q) + lo) and one
// Barrett reduction at the end yields the canonical residue.
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
constexpr int STREAM_UNROLL = 15;

template <int MB>
__global__ void __launch_bounds__(STREAM_THREADS)
rowsel_stream_kernel(const uint4 *__restrict__ db, const uint32_t *__restrict__ qry,
                     uint32_t *__restrict__ out, uint32_t d0, uint32_t d1, uint32_t L, uint32_t N,
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
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int s = 0; s < 4; ++s) acc[i][s] = 0;

    uint32_t k = 0;
    for (; k + STREAM_UNROLL <= d0; k += STREAM_UNROLL) {
        uint4 v[STREAM_UNROLL];
#pragma unroll
        for (int u = 0; u < STREAM_UNROLL; ++u) v[u] = ld_nt(dcol + (uint64_t)(k + u) * w);
#pragma unroll
        for (int u = 0; u < STREAM_UNROLL; ++u)
#pragma unroll
            for (int i = 0; i < MB; ++i) mad4s(acc[i], qv[i * mstride + (k + u) * kstride], v[u]);
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
            for (int s = 0; s < 4; ++s) acc[i][s] = lazy_fold(acc[i][s], mq);
    }
    if (k < d0) {   // ragged tail: fewer than fifteen rows
        for (; k < d0; ++k) {
            const uint4 v = ld_nt(dcol + (uint64_t)k * w);
#pragma unroll
            for (int i = 0; i < MB; ++i) mad4s(acc[i], qv[i * mstride + k * kstride], v);
        }
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
            for (int s = 0; s < 4; ++s) acc[i][s] = lazy_fold(acc[i][s], mq);
    }
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        uint4 r;
        r.x = reduce64(acc[i][0], mq);
        r.y = reduce64(acc[i][1], mq);
        r.z = reduce64(acc[i][2], mq);
        r.w = reduce64(acc[i][3], mq);
        *reinterpret_cast<uint4 *>(out + (((uint64_t)i * d1 + n) * L + l) * N + 4 * g) = r;
    }
}


void launch_rowsel_stream(const pir_db &db, const uint32_t *q, uint32_t B, uint32_t *out, hipStream_t st) {
    const auto &p = db.p;
    const uint32_t m_rows = 2 * B;
    const uint64_t groups = (uint64_t)p.nprimes * (p.n / 4);
    ModQ4s mods{};
    for (uint32_t l = 0; l < p.nprimes; ++l) mods.m[l] = db.mod[l];
    const uint4 *dbv = reinterpret_cast<const uint4 *>(db.valu.data);
    const uint32_t nblk_n = (p.d1 + STREAM_THREADS - 1) / STREAM_THREADS;
    const uint64_t blocks = groups * nblk_n;
    if (blocks >= (1ull << 31)) PIR_FAIL(PIR_EINVAL, "grid too large");
    dim3 grid((uint32_t)blocks), block(STREAM_THREADS);
    switch (m_rows) {
        case 2: rowsel_stream_kernel<2><<<grid, block, 0, st>>>(dbv, q, out, p.d0, p.d1, p.nprimes, p.n, nblk_n, mods); break;
        case 4: rowsel_stream_kernel<4><<<grid, block, 0, st>>>(dbv, q, out, p.d0, p.d1, p.nprimes, p.n, nblk_n, mods); break;
        case 6: rowsel_stream_kernel<6><<<grid, block, 0, st>>>(dbv, q, out, p.d0, p.d1, p.nprimes, p.n, nblk_n, mods); break;
        case 8: rowsel_stream_kernel<8><<<grid, block, 0, st>>>(dbv, q, out, p.d0, p.d1, p.nprimes, p.n, nblk_n, mods); break;
        default: PIR_FAIL(PIR_EINVAL, "unexpected row count %u", m_rows);
    }
    PIR_LAUNCH_CHECK();
}

}  // namespace pir
