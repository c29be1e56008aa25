// Query front end: RowSel on selector ciphertexts given in the coefficient
// domain.
//
// RowSel multiplies NTT-domain polynomials point by point (sec. 2.3,
// sec. 2.4.1), so a query that arrives as coefficients (the form query
// expansion leaves it in, sec. 2.2) needs the forward negacyclic NTT of each
// of its 2B*D0*L polynomials first, with the convention of the DB load:
// ahat_i = a(psi^(2i+1)), natural order.
//
// INT8 MFMA path: one launch transforms the polynomials and writes the
// signed-digit query planes [L*N][4][Kp/64][Mp][64] that the persistent GEMM
// reads, so no NTT-domain copy of the query is ever stored.  A block takes
// KG polynomials of one row m and prime l with consecutive k (KG = 8 at
// N <= 4096), transforms them in LDS (Cooley-Tukey with psi powers in
// bit-reversed order, as the DB load's NTT) and, for every point, writes the
// KG digit bytes of each digit plane as one KG-byte piece of the plane's
// 64-byte row.  The 64/KG blocks that fill one row are consecutive in the
// launch order and run on one XCD, so the pieces meet in its L2 before the
// line goes to HBM.  Digits of k >= D0 (padding up to Kp) are written as
// zero; padding rows 2B <= m < Mp are not written at all: an output row of
// the GEMM depends on its own query row only, and rows m >= 2B never reach
// the output.
//
// VALU path: the polynomials are transformed into an NTT-domain copy of the
// query in stream-ordered scratch, which the VALU kernels then read.
#include "common.h"
#include "mfma.h"
#include "modarith.h"

namespace pir {

constexpr int QF_THREADS = 1024;
constexpr uint32_t QF_LDS_WORDS = 32768;   // 128 KiB of polynomials per block

struct QfPrimes {
    const uint32_t *tw[PIR_MAX_PRIMES];   // forward twiddles: [n] powers, [n] Shoup companions
    uint32_t q[PIR_MAX_PRIMES];
};

// Polynomials per block at ring dimension n (a power of two, 8 <= n <= 16384).
static uint32_t qf_group(uint32_t n) { return std::min<uint32_t>(8, QF_LDS_WORDS / n); }

template <int KG>
__global__ void __launch_bounds__(QF_THREADS)
query_ntt_digits_kernel(const uint32_t *__restrict__ q, int8_t *__restrict__ qd, uint32_t mp, uint32_t d0,
                        uint32_t L, uint32_t n, uint32_t logn, uint32_t nkc, QfPrimes pr) {
    extern __shared__ uint32_t s[];   // [KG][n]
    const uint32_t tid = threadIdx.x;
    const uint32_t kgroups = nkc * (64 / KG);
    uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
    const uint32_t kg = b % kgroups;
    b /= kgroups;
    const uint32_t l = b % L;
    const uint32_t m = b / L;
    const uint32_t k0 = kg * KG;
    const uint32_t qv = pr.q[l];

    // load: polynomial (m, k, l) is n contiguous words of the query
    for (uint32_t e = tid; e < KG * n; e += QF_THREADS) {
        const uint32_t kk = e >> logn, i = e & (n - 1), k = k0 + kk;
        uint32_t v = 0;
        if (k < d0) {
            v = q[((uint64_t)m * d0 + k) * L * n + (uint64_t)l * n + i];
            v = v >= qv ? v % qv : v;
        }
        s[e] = v;
    }
    __syncthreads();
    const uint32_t *tw = pr.tw[l], *tws = tw + n;
    const uint32_t half = n >> 1;
    for (uint32_t mm = 1, lt = logn - 1; mm < n; mm <<= 1, --lt) {
        for (uint32_t e = tid; e < KG * half; e += QF_THREADS) {
            const uint32_t kk = e >> (logn - 1), bb = e & (half - 1);
            const uint32_t i = bb >> lt;
            const uint32_t j = (i << (lt + 1)) + (bb & ((1u << lt) - 1));
            uint32_t *poly = s + kk * n;
            const uint32_t u = poly[j];
            const uint32_t v = mul_shoup(poly[j + (1u << lt)], tw[mm + i], tws[mm + i], qv);
            poly[j] = add_mod(u, v, qv);
            poly[j + (1u << lt)] = sub_mod(u, v, qv);
        }
        __syncthreads();
    }

    // LDS position i holds point j = bitrev(i) of every polynomial; each
    // point's four digit planes receive KG bytes (k0 .. k0+KG-1) of one row
    const uint64_t plane = (uint64_t)mp * 64;                 // bytes of one (point, digit, chunk) plane
    int8_t *base = qd + (uint64_t)(k0 / 64) * plane + (uint64_t)m * 64 + (k0 % 64);
    for (uint32_t i = tid; i < n; i += QF_THREADS) {
        const uint32_t j = __brev(i) >> (32 - logn);
        uint32_t dg[KG];
#pragma unroll
        for (int kk = 0; kk < KG; ++kk) dg[kk] = split_digits(s[kk * n + i]);
        const uint64_t p = (uint64_t)l * n + j;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            uint8_t bytes[KG];
#pragma unroll
            for (int kk = 0; kk < KG; ++kk) bytes[kk] = (uint8_t)(dg[kk] >> (8 * d));
            int8_t *dst = base + (p * 4 + d) * nkc * plane;
            if (KG == 8) {
                uint2 w;
                __builtin_memcpy(&w, bytes, 8);
                *reinterpret_cast<uint2 *>(dst) = w;
            } else if (KG == 4) {
                uint32_t w;
                __builtin_memcpy(&w, bytes, 4);
                *reinterpret_cast<uint32_t *>(dst) = w;
            } else {
                uint16_t w;
                __builtin_memcpy(&w, bytes, 2);
                *reinterpret_cast<uint16_t *>(dst) = w;
            }
        }
    }
}

// Dynamic LDS above 64 KiB has to be allowed per kernel.
static void qf_attr(const void *fn, size_t lds) {
    PIR_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
}

void launch_query_ntt_digits(const pir_db &db, const uint32_t *q_coeff, uint32_t B, int8_t *qd,
                             hipStream_t st) {
    const auto &p = db.p;
    const uint32_t mp = (2 * B + 31) / 32 * 32;
    const uint32_t nkc = db.mfma.kp / 64;
    const uint32_t kgs = qf_group(p.n);
    uint32_t logn = 0;
    while ((1u << logn) < p.n) ++logn;
    QfPrimes pr{};
    for (uint32_t l = 0; l < p.nprimes; ++l) {
        const NttTables &t = ntt_tables(p.q[l], p.n);
        pr.tw[l] = t.fwd;
        pr.q[l] = p.q[l];
    }
    const uint64_t blocks = 2ull * B * p.nprimes * nkc * (64 / kgs);   // rows m < 2B only
    if (blocks >= (1ull << 31)) PIR_FAIL(PIR_EINVAL, "query front-end launch too large");
    const size_t lds = (size_t)kgs * p.n * sizeof(uint32_t);
    switch (kgs) {
        case 8:
            qf_attr(reinterpret_cast<const void *>(&query_ntt_digits_kernel<8>), lds);
            query_ntt_digits_kernel<8><<<(uint32_t)blocks, QF_THREADS, lds, st>>>(
                q_coeff, qd, mp, p.d0, p.nprimes, p.n, logn, nkc, pr);
            break;
        case 4:
            qf_attr(reinterpret_cast<const void *>(&query_ntt_digits_kernel<4>), lds);
            query_ntt_digits_kernel<4><<<(uint32_t)blocks, QF_THREADS, lds, st>>>(
                q_coeff, qd, mp, p.d0, p.nprimes, p.n, logn, nkc, pr);
            break;
        case 2:
            qf_attr(reinterpret_cast<const void *>(&query_ntt_digits_kernel<2>), lds);
            query_ntt_digits_kernel<2><<<(uint32_t)blocks, QF_THREADS, lds, st>>>(
                q_coeff, qd, mp, p.d0, p.nprimes, p.n, logn, nkc, pr);
            break;
        default: PIR_FAIL(PIR_EINVAL, "unsupported ring dimension %u", p.n);
    }
    PIR_LAUNCH_CHECK();
}

void launch_query_ntt(const pir_db &db, const uint32_t *q_coeff, uint32_t B, uint32_t *q_ntt, hipStream_t st) {
    const auto &p = db.p;
    const uint64_t polys = 2ull * B * p.d0;   // per prime; polynomial (m, k) of prime l at ((m*D0 + k)*L + l)*N
    for (uint32_t l = 0; l < p.nprimes; ++l) {
        const NttTables &t = ntt_tables(p.q[l], p.n);
        launch_ntt(q_coeff + (uint64_t)l * p.n, q_ntt + (uint64_t)l * p.n, polys, (uint64_t)p.nprimes * p.n,
                   (uint64_t)p.nprimes * p.n, t, false, st);
    }
}

}  // namespace pir
