// Query front end: RowSel on selector ciphertexts given in the coefficient
// domain.
//
// RowSel multiplies NTT-domain polynomials point by point (sec. 2.3,
// sec. 2.4.1), so a query that arrives as coefficients (the form query
// expansion leaves it in, sec. 2.2) needs the forward negacyclic NTT of each
// of its 2B*D0*L polynomials first, with the convention of the DB load:
// ahat_i = a(psi^(2i+1)), natural order.  One launch transforms the whole
// query into an NTT-domain copy in the boundary layout, which the chosen
// path then consumes like any query (the MFMA path through its digit-plane
// ingest).
//
// For N >= 256 the transform is register-blocked (query_ntt_reg_kernel: 16
// values per thread, up to four butterfly stages per LDS exchange, three
// exchanges at N = 4096); smaller rings use one LDS stage per barrier with
// KG polynomials of consecutive k per block (query_ntt_kernel).  On the
// 2 GiB query of 64 clients (N = 4096, two primes, D0 = 512) the transform
// takes ~1.15 ms, against ~4.3 ms for the per-polynomial NTT of the DB load
// and ~7 ms for the one-stage-per-barrier form over 8 polynomials.
//
// Writing the MFMA path's digit planes straight from the transform (KG bytes
// of each 64-byte plane row per block) was measured and is not used: those
// scattered 8-byte stores ran at a few hundred GB/s (7.9 ms for the 2 GiB
// 64-client query), far slower than the NTT-domain copy plus the ingest.
// One pass cannot write whole plane rows: a row needs the same point of all
// the 64 k of a chunk, i.e. 64 full polynomials (1 MiB at N = 4096) in one
// block.
#include <type_traits>

#include "common.h"
#include "mfma.h"
#include "modarith.h"
#include "nttreg.h"

namespace pir {

constexpr int QF_THREADS = 1024;
constexpr uint32_t QF_LDS_WORDS = 32768;   // 128 KiB of polynomials per block

struct QfPrimes {
    const uint32_t *tw[PIR_MAX_PRIMES];   // forward twiddles: [n] powers, [n] Shoup companions
    uint32_t q[PIR_MAX_PRIMES];
    uint32_t r1[PIR_MAX_PRIMES];          // floor(2^32 / q): Shoup companion of 1
};

// Polynomials per block at ring dimension n (a power of two, 8 <= n <= 16384).
static uint32_t qf_group(uint32_t n) { return std::min<uint32_t>(8, QF_LDS_WORDS / n); }

template <int KG, bool WIDE>
__global__ void __launch_bounds__(QF_THREADS)
query_ntt_kernel(const uint32_t *__restrict__ q, uint32_t *__restrict__ qn, uint32_t d0, uint32_t L,
                 uint32_t n, uint32_t logn, QfPrimes pr) {
    extern __shared__ uint32_t s[];   // [KG][n]
    const uint32_t tid = threadIdx.x;
    const uint32_t kgroups = (d0 + KG - 1) / KG;
    uint32_t b = blockIdx.x;
    const uint32_t kg = b % kgroups;
    b /= kgroups;
    const uint32_t l = b % L;
    const uint32_t m = b / L;
    const uint32_t k0 = kg * KG;
    const uint32_t kn = min((uint32_t)KG, d0 - k0);   // polynomials of this block
    const uint32_t qv = pr.q[l];

    // polynomial (m, k, l) is n contiguous words of the query
    for (uint32_t e = tid; e < kn * n; e += QF_THREADS) {
        const uint32_t kk = e >> logn, i = e & (n - 1);
        uint32_t v = q[((uint64_t)m * d0 + k0 + kk) * L * n + (uint64_t)l * n + i];
        s[e] = v >= qv ? v % qv : v;
    }
    __syncthreads();
    const uint32_t *tw = pr.tw[l], *tws = tw + n;
    const uint32_t half = n >> 1;
    for (uint32_t mm = 1, lt = logn - 1; mm < n; mm <<= 1, --lt) {
        for (uint32_t e = tid; e < kn * half; e += QF_THREADS) {
            const uint32_t kk = e >> (logn - 1), bb = e & (half - 1);
            const uint32_t i = bb >> lt;
            const uint32_t j = (i << (lt + 1)) + (bb & ((1u << lt) - 1));
            uint32_t *poly = s + kk * n;
            const uint32_t u = poly[j];
            const uint32_t v = WIDE ? mul_shoup_w(poly[j + (1u << lt)], tw[mm + i], tws[mm + i], qv)
                                    : mul_shoup(poly[j + (1u << lt)], tw[mm + i], tws[mm + i], qv);
            poly[j] = WIDE ? add_mod_w(u, v, qv) : add_mod(u, v, qv);
            poly[j + (1u << lt)] = sub_mod(u, v, qv);
        }
        __syncthreads();
    }
    // LDS position i holds point bitrev(i): lanes read LDS in order (no bank
    // conflicts) and scatter within the polynomial's 16 KiB (whole lines are
    // completed by the same block)
    for (uint32_t e = tid; e < kn * n; e += QF_THREADS) {
        const uint32_t kk = e >> logn, i = e & (n - 1);
        const uint32_t j = __brev(i) >> (32 - logn);
        qn[((uint64_t)m * d0 + k0 + kk) * L * n + (uint64_t)l * n + j] = s[e];
    }
}

// Register-blocked transform for N >= 256 (the scheme and helpers are in
// nttreg.h).

template <int LOGN, bool WIDE>
__global__ void __launch_bounds__(QF_THREADS)
query_ntt_reg_kernel(const uint32_t *__restrict__ q, uint32_t *__restrict__ qn, uint32_t d0, uint32_t L,
                     uint32_t ppb, QfPrimes pr) {
    constexpr uint32_t n = 1u << LOGN, logn = LOGN;
    extern __shared__ uint32_t s[];                  // ppb polynomials of n + n/16 words
    constexpr uint32_t T = n / QR;
    const uint32_t tid = threadIdx.x;
    const uint32_t pi = tid / T, t = tid % T;       // polynomial of the block, thread within it
    const uint32_t kgroups = (d0 + ppb - 1) / ppb;
    uint32_t b = blockIdx.x;
    const uint32_t kg = b % kgroups;
    b /= kgroups;
    const uint32_t l = b % L;
    const uint32_t m = b / L;
    const uint32_t k = kg * ppb + pi;
    const bool live = pi < ppb && k < d0;            // uniform per polynomial's threads
    const uint32_t qv = pr.q[l];
    const uint32_t *tw = pr.tw[l], *tws = tw + n;
    uint32_t *poly = s + pi * (n + n / 16);
    const uint64_t off = ((uint64_t)m * d0 + k) * L * n + (uint64_t)l * n;

    uint32_t v[QR];
    uint32_t lo = logn - 4;                          // register bits of the first chunk
    if (live) {
        // any 32-bit coefficient: x - floor(x * floor(2^32/q) / 2^32) * q is
        // x mod q or x mod q + q, in [0, 2q) as the lazy butterflies allow.
        // The first stage pairs registers r and r + 8, and only its first
        // operands need the reduction: the second ones go into Shoup's
        // product, which takes any 32-bit value.
        const uint32_t r1 = pr.r1[l];
#pragma unroll
        for (int r = 0; r < QR; ++r) {
            const uint32_t x = q[off + qf_elem(t, 0, lo) + qf_rpart(r, lo)];
            if (WIDE) {   // q >= 2^30: [0, 2q) needs 64 bits; reduce fully (no lazy range)
                const uint64_t y = (uint64_t)x - (uint64_t)__umulhi(x, r1) * qv;
                v[r] = (uint32_t)(y >= qv ? y - qv : y);
            } else if (r & 8) {
                v[r] = x;
            } else {
                v[r] = x - __umulhi(x, r1) * qv;
            }
        }
    }
#pragma unroll
    for (int hi = (int)logn; hi > 0; hi -= 4) {
        const int clo = hi - 4 > 0 ? hi - 4 : 0;     // lowest stage of this chunk
        const uint32_t rlo = (uint32_t)clo;          // registers cover bits [rlo, rlo + 4)
        if (rlo != lo) {                              // redistribute through LDS
            __syncthreads();
            const uint32_t pw = qf_pad(qf_elem(t, 0, lo)), pr = qf_pad(qf_elem(t, 0, rlo));
            if (live) {
#pragma unroll
                for (int r = 0; r < QR; ++r) poly[pw + qf_pad(qf_rpart(r, lo))] = v[r];
            }
            __syncthreads();
            if (live) {
#pragma unroll
                for (int r = 0; r < QR; ++r) v[r] = poly[pr + qf_pad(qf_rpart(r, rlo))];
            }
            lo = rlo;
        }
        if (live) {
            const uint32_t eb = qf_elem(t, 0, lo);
#pragma unroll
            for (int x = hi - 1; x >= clo; --x) {
                const uint32_t bit = 1u << (x - (int)lo), mgroups = n >> (x + 1);
                const uint32_t gb = mgroups + (eb >> (x + 1));
#pragma unroll
                for (int r = 0; r < QR; ++r) {
                    if (r & bit) continue;
                    const uint32_t gi = gb + (qf_rpart(r, lo) >> (x + 1));
                    if (WIDE) {   // canonical butterflies with 64-bit intermediates
                        const uint32_t u = v[r], w = mul_shoup_w(v[r | bit], tw[gi], tws[gi], qv);
                        v[r] = add_mod_w(u, w, qv);
                        v[r | bit] = sub_mod(u, w, qv);
                    } else {
                        qf_bfly(v[r], v[r | bit], tw[gi], tws[gi], qv, 2 * qv);
                    }
                }
            }
        }
    }
    // element e holds point bitrev(e): place points in natural order, then
    // store coalesced
    __syncthreads();
    if (live) {
        const uint32_t pb = qf_pad(__brev(qf_elem(t, 0, lo)) >> (32 - logn));
#pragma unroll
        for (int r = 0; r < QR; ++r)
            poly[pb + qf_pad(__brev(qf_rpart(r, lo)) >> (32 - logn))] = WIDE ? v[r] : qf_reduce4(v[r], qv, 2 * qv);
    }
    __syncthreads();
    if (live) {
#pragma unroll
        for (int r = 0; r < QR; ++r) qn[off + t + r * T] = poly[qf_pad(t) + qf_pad(r * T)];   // t < T = 2^k
    }
}

// Dynamic LDS above 64 KiB has to be allowed per kernel.
static void qf_attr(const void *fn, size_t lds) {
    PIR_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
}

void launch_query_ntt(const pir_db &db, const uint32_t *q_coeff, uint32_t B, uint32_t *q_ntt, hipStream_t st) {
    const auto &p = db.p;
    const uint32_t kgs = qf_group(p.n);
    uint32_t logn = 0;
    while ((1u << logn) < p.n) ++logn;
    QfPrimes pr{};
    for (uint32_t l = 0; l < p.nprimes; ++l) {
        const NttTables &t = ntt_tables(p.q[l], p.n);
        pr.tw[l] = t.fwd;
        pr.q[l] = p.q[l];
        pr.r1[l] = (uint32_t)((1ull << 32) / p.q[l]);
    }
    if (p.n >= 256) {
        // register-blocked form: polynomials per block so that a block has
        // up to 1024 threads (N/16 per polynomial)
        const uint32_t ppb = std::max<uint32_t>(1, QF_THREADS / (p.n / QR));
        const uint64_t blocks = 2ull * B * p.nprimes * ((p.d0 + ppb - 1) / ppb);
        if (blocks >= (1ull << 31)) PIR_FAIL(PIR_EINVAL, "query front-end launch too large");
        const size_t lds = (size_t)ppb * (p.n + p.n / 16) * sizeof(uint32_t);
        const uint32_t threads = ppb * (p.n / QR);
        auto go = [&](auto kern) {
            qf_attr(reinterpret_cast<const void *>(kern), lds);
            kern<<<(uint32_t)blocks, threads, lds, st>>>(q_coeff, q_ntt, p.d0, p.nprimes, ppb, pr);
        };
        auto pick = [&](auto wide) {
            constexpr bool W = decltype(wide)::value;
            switch (logn) {
                case 8: go(&query_ntt_reg_kernel<8, W>); break;
                case 9: go(&query_ntt_reg_kernel<9, W>); break;
                case 10: go(&query_ntt_reg_kernel<10, W>); break;
                case 11: go(&query_ntt_reg_kernel<11, W>); break;
                case 12: go(&query_ntt_reg_kernel<12, W>); break;
                case 13: go(&query_ntt_reg_kernel<13, W>); break;
                case 14: go(&query_ntt_reg_kernel<14, W>); break;
                default: PIR_FAIL(PIR_EINVAL, "unsupported ring dimension %u", p.n);
            }
        };
        if (db.wide) pick(std::true_type{});
        else pick(std::false_type{});
        PIR_LAUNCH_CHECK();
        return;
    }
    const uint64_t blocks = 2ull * B * p.nprimes * ((p.d0 + kgs - 1) / kgs);
    if (blocks >= (1ull << 31)) PIR_FAIL(PIR_EINVAL, "query front-end launch too large");
    const size_t lds = (size_t)kgs * p.n * sizeof(uint32_t);
    // small rings (N < 256): at most 32 KiB of polynomials per block, KG = 8
    if (kgs != 8) PIR_FAIL(PIR_EINVAL, "unsupported ring dimension %u", p.n);
    auto small = [&](auto kern) {
        qf_attr(reinterpret_cast<const void *>(kern), lds);
        kern<<<(uint32_t)blocks, QF_THREADS, lds, st>>>(q_coeff, q_ntt, p.d0, p.nprimes, p.n, logn, pr);
    };
    if (db.wide) small(&query_ntt_kernel<8, true>);
    else small(&query_ntt_kernel<8, false>);
    PIR_LAUNCH_CHECK();
}

}  // namespace pir
