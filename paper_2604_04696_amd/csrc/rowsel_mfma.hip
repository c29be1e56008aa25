// RowSel on the INT8 matrix cores, exact.
//
// Every residue x < 2^30 is written as four balanced signed 8-bit digits,
// x = sum_i d_i 2^(8i), d_i in [-128, 127].  A point's GEMM (sec. 2.3)
//   out[m][n] = sum_k Q[m][k] DB[k][n]  mod q
// then splits into sixteen digit products
//   P_ij[m][n] = sum_k dQ_i[m][k] dDB_j[k][n]
// computed by v_mfma_i32_32x32x32_i8 and summed per weight class s = i + j
// in int32: G_s = sum_{i+j=s} P_ij.  With |d| <= 128 and at most four pairs
// per class, |G_s| <= 4 * K * 2^14, so a K chunk of up to 8192 rows cannot
// overflow.  The result is recombined as sum_s G_s * (2^(8s) mod q) in
// signed 64-bit (|sum| < K * 2^48 < 2^62), shifted by a multiple of q into
// [0, 2^64) and Barrett-reduced: bit-identical to the 64-bit VALU path.
//
// Layouts (k contiguous, "k-major" in the paper's terms, sec. 5.2.1):
//   DB digits    [L*N][4][D1][Kp] int8   built once at load time
//   query digits [L*N][4][Mp][Kp] int8   built per call (ingest kernel)
// with Kp = D0 rounded up to 64 and Mp = 2B rounded up to 32, zero padded.
#include <algorithm>

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
// src[r*s_r + (k - klo)*s_k + p] (points p contiguous) goes to byte k of row r of
// plane [p][d] in dst[((p*4 + d)*R + r)*Kp + k].  A block takes one row r,
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
        int8_t *o = dst + (((uint64_t)(p0 + pp) * 4 + d) * R + r) * kp + kc;
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
constexpr int MFMA_K = 64;       // k bytes staged per LDS step (two MFMA k-steps)
constexpr int LDS_PITCH = 80;    // row pitch (bytes): 64 + 16 keeps 8-lane b128 reads conflict free
constexpr uint32_t KSUPER = 8192;   // rows per int32 accumulation (overflow bound above)

// One block = one group of four consecutive points of a prime, a BM x BN
// output tile; WM x WN waves, each owning a 32 x 32 sub-tile with seven
// int32 class accumulators.  The four points run one after another and
// their residues stay in registers, so the output leaves as one 16-byte
// vector (four points) per (m, n) -- written straight into the boundary
// layout [B][2][D1][L][N].
template <int WM, int WN>
__global__ void __launch_bounds__(64 * WM * WN)
rowsel_mfma_kernel(const int8_t *__restrict__ dbd, const int8_t *__restrict__ qd,
                   uint32_t *__restrict__ out, uint32_t m_rows, uint32_t mp, uint32_t d1,
                   uint32_t kp, uint32_t L, uint32_t N, uint32_t nblk_m, uint32_t nblk_n,
                   ModQ4m mods) {
    constexpr int BM = 32 * WM, BN = 32 * WN, NT = 64 * WM * WN;
    __shared__ __attribute__((aligned(16))) int8_t As[4][BM][LDS_PITCH];
    __shared__ __attribute__((aligned(16))) int8_t Bs[4][BN][LDS_PITCH];

    const uint32_t tid = threadIdx.x;
    const uint32_t bid = xcd_remap(blockIdx.x, gridDim.x);
    const uint32_t nb = bid % nblk_n;
    const uint32_t mb = (bid / nblk_n) % nblk_m;
    const uint32_t gg = bid / (nblk_n * nblk_m);
    const uint32_t G = N / 4;
    const uint32_t l = gg / G, g = gg % G;
    const ModQ mq = mods.m[l];
    const uint32_t wave = tid / 64, lane = tid % 64;
    const uint32_t wm = wave / WN, wn = wave % WN;
    const uint32_t m0 = mb * BM, n0 = nb * BN;
    const bool wave_active = m0 + wm * 32 < mp && n0 + wn * 32 < d1;
    const uint32_t fr = lane % 32, fk = 16 * (lane / 32);   // fragment row and k offset

    uint32_t res[4][16];

    for (int s = 0; s < 4; ++s) {
        const uint64_t p = (uint64_t)l * N + 4 * g + s;
        const int8_t *qa = qd + p * 4 * mp * kp;
        const int8_t *db = dbd + p * 4 * (uint64_t)d1 * kp;
#pragma unroll
        for (int r = 0; r < 16; ++r) res[s][r] = 0;

        for (uint32_t ks0 = 0; ks0 < kp; ks0 += KSUPER) {
            const uint32_t ks1 = std::min(kp, ks0 + KSUPER);
            i32x16 acc[7];
#pragma unroll
            for (int c = 0; c < 7; ++c) acc[c] = (i32x16){};

            for (uint32_t kc = ks0; kc < ks1; kc += MFMA_K) {
                __syncthreads();
                for (uint32_t e = tid; e < 4 * BM * 4; e += NT) {
                    const uint32_t d = e / (BM * 4), r = (e / 4) % BM, c = e % 4;
                    const uint32_t row = m0 + r;
                    uint4 v = make_uint4(0, 0, 0, 0);
                    if (row < mp)
                        v = *reinterpret_cast<const uint4 *>(qa + ((uint64_t)d * mp + row) * kp + kc + 16 * c);
                    *reinterpret_cast<uint4 *>(&As[d][r][16 * c]) = v;
                }
                for (uint32_t e = tid; e < 4 * BN * 4; e += NT) {
                    const uint32_t d = e / (BN * 4), r = (e / 4) % BN, c = e % 4;
                    const uint32_t col = n0 + r;
                    uint4 v = make_uint4(0, 0, 0, 0);
                    if (col < d1)
                        v = *reinterpret_cast<const uint4 *>(db + ((uint64_t)d * d1 + col) * kp + kc + 16 * c);
                    *reinterpret_cast<uint4 *>(&Bs[d][r][16 * c]) = v;
                }
                __syncthreads();
                if (wave_active) {
#pragma unroll
                    for (int kstep = 0; kstep < MFMA_K; kstep += 32) {
                        i32x4 a[4], b[4];
#pragma unroll
                        for (int d = 0; d < 4; ++d) {
                            a[d] = *reinterpret_cast<const i32x4 *>(&As[d][wm * 32 + fr][kstep + fk]);
                            b[d] = *reinterpret_cast<const i32x4 *>(&Bs[d][wn * 32 + fr][kstep + fk]);
                        }
#pragma unroll
                        for (int i = 0; i < 4; ++i)
#pragma unroll
                            for (int j = 0; j < 4; ++j)
                                acc[i + j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[i], b[j], acc[i + j], 0, 0, 0);
                    }
                }
            }
            // recombine the seven classes: sum_s G_s * 2^(8s) mod q
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                int64_t t = 0;
#pragma unroll
                for (int c = 0; c < 7; ++c) t += (int64_t)acc[c][r] * (int64_t)mq.w[c];
                const uint32_t part = reduce64((uint64_t)t + mq.moff, mq);
                res[s][r] = add_mod(res[s][r], part, mq.q);
            }
        }
    }

    if (!wave_active) return;
    // accumulator element r of lane: row 8*(r/4) + 4*(lane/32) + r%4, column lane%32
    const uint32_t n = n0 + wn * 32 + lane % 32;
    if (n >= d1) return;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const uint32_t m = m0 + wm * 32 + 8 * (r / 4) + 4 * (lane / 32) + (r % 4);
        if (m < m_rows)
            *reinterpret_cast<uint4 *>(out + (((uint64_t)m * d1 + n) * L + l) * N + 4 * g) =
                make_uint4(res[0][r], res[1][r], res[2][r], res[3][r]);
    }
}

void launch_rowsel_mfma(const pir_db &db, const uint32_t *q, uint32_t B, uint32_t *out,
                        hipStream_t st) {
    const auto &p = db.p;
    const uint32_t m_rows = 2 * B;
    const uint32_t mp = (m_rows + 31) / 32 * 32;
    const uint32_t P = p.n * p.nprimes;
    const uint32_t kp = db.mfma.kp;

    // query ingest: [B][2][D0][L][N] -> [P][4][Mp][Kp] digit planes
    int8_t *qd = nullptr;
    const size_t qbytes = mfma_query_scratch_bytes(db, B);
    PIR_HIP(hipMallocAsync((void **)&qd, qbytes, st));
    launch_digit_planes(q, (uint64_t)p.d0 * P, P, qd, mp, m_rows, P, kp, 0, p.d0, p.d0, st);

    ModQ4m mods{};
    for (uint32_t l = 0; l < p.nprimes; ++l) mods.m[l] = db.mod[l];
    const uint64_t groups = (uint64_t)p.nprimes * (p.n / 4);
    constexpr int WM = 4, WN = 1;
    const uint32_t nblk_m = (mp + 32 * WM - 1) / (32 * WM);
    const uint32_t nblk_n = (p.d1 + 32 * WN - 1) / (32 * WN);
    const uint64_t blocks = groups * nblk_m * nblk_n;
    if (blocks >= (1ull << 31)) PIR_FAIL(PIR_EINVAL, "grid too large");
    rowsel_mfma_kernel<WM, WN><<<(uint32_t)blocks, 64 * WM * WN, 0, st>>>(
        db.mfma.data, qd, out, m_rows, mp, p.d1, kp, p.nprimes, p.n, nblk_m, nblk_n, mods);
    PIR_LAUNCH_CHECK();
    PIR_HIP(hipFreeAsync(qd, st));
}

}  // namespace pir
