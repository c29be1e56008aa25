// First ColTor stage: the tournament step that follows RowSel (sec. 2.2).
//
// For every client b and every pair of RowSel output ciphertexts (columns 2t
// and 2t+1) the stage computes the selector
//     out[b][t] = ct0 + RGSW_b [x] (ct1 - ct0)
// where [x] is the external product (sec. 2.4.2): both polynomials of the
// difference go to the coefficient domain, each coefficient is rebuilt from
// its L residues as a value mod Q = prod q_l (RNS reconstruction), centred
// into (-Q/2, Q/2] and cut into ell digits of base z = 2^log2z (digits
// 0..ell-2 balanced in [-z/2, z/2), the last one the rest), and the 2*ell
// digit polynomials go back to the NTT domain limb by limb and
// multiply-accumulate against the RGSW rows into two polynomials.  An
// unpaired last column (odd count) passes through.
//
// Two kernels:
//   coltor_dcp_kernel  one block per (node, input polynomial): the
//                      difference of the two columns and its inverse NTT for
//                      all L limbs in LDS (L*N <= 16384 words), then the
//                      reconstruction and decomposition, coefficient by
//                      coefficient; digits go out as int32 [node][2][ell][N]
//                      (ell*N words per polynomial instead of L*N residues
//                      per digit: each limb reduces them on load);
//   coltor_mac_kernel  one block per (node, limb): for each of the 2*ell
//                      digit polynomials, the residues mod q_l, the forward
//                      NTT in LDS and the product with the two RGSW
//                      components of that row, accumulated in registers;
//                      then ct0 is added and both output polynomials stored.
// Every modular step uses the forms that hold for any prime below 2^32.
#include <type_traits>

#include "common.h"
#include "modarith.h"

namespace pir {

typedef unsigned __int128 u128;
typedef __int128 i128;

constexpr int CT_THREADS = 512;

struct ColtorPrimes {
    const uint32_t *fwd[PIR_MAX_PRIMES];   // forward twiddles [n] + Shoup companions [n]
    const uint32_t *inv[PIR_MAX_PRIMES];   // inverse twiddles [n] + companions [n]
    uint32_t q[PIR_MAX_PRIMES];
    uint32_t ninv[PIR_MAX_PRIMES], ninv_s[PIR_MAX_PRIMES];
    uint32_t crt_c[PIR_MAX_PRIMES], crt_cs[PIR_MAX_PRIMES];   // (Q/q_l)^-1 mod q_l and its companion
    uint64_t mu[PIR_MAX_PRIMES];                               // Barrett constants of reduce64
    uint32_t qhat[PIR_MAX_PRIMES][4];                          // Q/q_l, 32-bit limbs, low first
    uint32_t Q[4], Qhalf[4];                                   // Q and floor(Q/2)
};

__device__ __forceinline__ u128 u128_of(const uint32_t (&w)[4]) {
    return ((u128)(((uint64_t)w[3] << 32) | w[2]) << 64) | (((uint64_t)w[1] << 32) | w[0]);
}

__device__ __forceinline__ uint32_t mulmod_any(uint32_t a, uint32_t b, uint32_t q, uint64_t mu) {
    const uint64_t x = (uint64_t)a * b;
    const uint64_t r = x - __umul64hi(x, mu) * (uint64_t)q;
    return (uint32_t)(r >= q ? r - q : r);
}

// ----------------------------------------------------- kernel 1: INTT + Dcp
// grid: nodes * 2 blocks (node = b * nout + t, p = polynomial of the pair).
__global__ void __launch_bounds__(CT_THREADS)
coltor_dcp_kernel(const uint32_t *__restrict__ ct, uint32_t ncols, uint32_t nout, uint32_t L, uint32_t n,
                  uint32_t logn, uint32_t log2z, uint32_t ell, int32_t *__restrict__ digits,
                  ColtorPrimes pr) {
    extern __shared__ uint32_t s[];                  // [L][n]
    const uint32_t tid = threadIdx.x;
    const uint32_t p = blockIdx.x % 2, node = blockIdx.x / 2;
    const uint32_t b = node / nout, t = node % nout;
    if (2 * t + 1 >= ncols) return;                  // unpaired column: no product
    const uint32_t LN = L * n;
    const uint32_t *c0 = ct + ((uint64_t)(b * 2 + p) * ncols + 2 * t) * LN;
    const uint32_t *c1 = c0 + LN;

    // difference, stored at bit-reversed positions for the inverse transform
    for (uint32_t e = tid; e < LN; e += CT_THREADS) {
        const uint32_t l = e / n, i = e % n, q = pr.q[l];
        s[l * n + (__brev(i) >> (32 - logn))] = sub_mod(c1[e], c0[e], q);
    }
    __syncthreads();
    // Gentleman-Sande stages, all limbs at once
    const uint32_t half = n >> 1;
    for (uint32_t m = half, lt = 0; m >= 1; m >>= 1, ++lt) {
        for (uint32_t bb = tid; bb < L * half; bb += CT_THREADS) {
            const uint32_t l = bb / half, b2 = bb % half, q = pr.q[l];
            const uint32_t *tw = pr.inv[l], *tws = tw + n;
            const uint32_t i = b2 >> lt;
            const uint32_t j = l * n + (i << (lt + 1)) + (b2 & ((1u << lt) - 1));
            const uint32_t tt = 1u << lt;
            const uint32_t u = s[j], v = s[j + tt];
            s[j] = add_mod_w(u, v, q);
            s[j + tt] = mul_shoup_w(sub_mod(u, v, q), tw[m + i], tws[m + i], q);
        }
        __syncthreads();
    }
    // reconstruction and decomposition of each coefficient
    const u128 Q = u128_of(pr.Q), Qhalf = u128_of(pr.Qhalf);
    const i128 zhalf = (i128)1 << (log2z - 1);
    const i128 zmask = ((i128)1 << log2z) - 1;
    int32_t *dst = digits + ((uint64_t)node * 2 + p) * ell * n;
    for (uint32_t j = tid; j < n; j += CT_THREADS) {
        u128 acc = 0;
        for (uint32_t l = 0; l < L; ++l) {
            const uint32_t q = pr.q[l];
            const uint32_t r = mul_shoup_w(s[l * n + j], pr.ninv[l], pr.ninv_s[l], q);     // INTT scale
            const uint32_t y = mul_shoup_w(r, pr.crt_c[l], pr.crt_cs[l], q);
            const u128 term = (u128)y * u128_of(pr.qhat[l]);                              // < Q
            u128 sum = acc + term;
            if (sum < acc || sum >= Q) sum -= Q;     // a wrap past 2^128 is undone by the same subtraction
            acc = sum;
        }
        i128 v = acc > Qhalf ? -(i128)(Q - acc) : (i128)acc;
        for (uint32_t i = 0; i + 1 < ell; ++i) {
            const i128 d = ((v + zhalf) & zmask) - zhalf;
            dst[(uint64_t)i * n + j] = (int32_t)d;
            v = (v - d) >> log2z;
        }
        dst[(uint64_t)(ell - 1) * n + j] = (int32_t)v;
    }
}

// ------------------------------------------------- kernel 2: NTT + products
// grid: nodes * L blocks.  Thread tid owns points j = tid + k * CT_THREADS.
constexpr int CT_MAXK = 16384 / CT_THREADS;   // points per thread at n = 16384

template <int K>
__global__ void __launch_bounds__(CT_THREADS)
coltor_mac_kernel(const uint32_t *__restrict__ ct, const uint32_t *__restrict__ rgsw,
                  const int32_t *__restrict__ digits, uint32_t *__restrict__ out, uint32_t ncols,
                  uint32_t nout, uint32_t L, uint32_t n, uint32_t logn, uint32_t ell, ColtorPrimes pr) {
    extern __shared__ uint32_t s[];                  // [n]
    const uint32_t tid = threadIdx.x;
    const uint32_t l = blockIdx.x % L, node = blockIdx.x / L;
    const uint32_t b = node / nout, t = node % nout;
    const uint32_t q = pr.q[l];
    const uint64_t mu = pr.mu[l];
    const uint64_t LN = (uint64_t)L * n;
    const bool paired = 2 * t + 1 < ncols;

    uint32_t acc[2][K];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int k = 0; k < K; ++k) acc[c][k] = 0;

    if (paired) {
        const uint32_t *tw = pr.fwd[l], *tws = tw + n;
        const uint32_t half = n >> 1;
        for (uint32_t p = 0; p < 2; ++p) {
            for (uint32_t i = 0; i < ell; ++i) {
                const int32_t *dg = digits + (((uint64_t)node * 2 + p) * ell + i) * n;
                __syncthreads();                       // the previous transform's reads are done
                for (uint32_t j = tid; j < n; j += CT_THREADS) {
                    const int32_t d = dg[j];
                    s[j] = d < 0 ? (uint32_t)(d + (int64_t)q) : (uint32_t)d;
                }
                __syncthreads();
                // Cooley-Tukey stages; point j ends at position bitrev(j)
                for (uint32_t m = 1, lt = logn - 1; m < n; m <<= 1, --lt) {
                    for (uint32_t bb = tid; bb < half; bb += CT_THREADS) {
                        const uint32_t ii = bb >> lt;
                        const uint32_t j = (ii << (lt + 1)) + (bb & ((1u << lt) - 1));
                        const uint32_t tt = 1u << lt;
                        const uint32_t u = s[j];
                        const uint32_t v = mul_shoup_w(s[j + tt], tw[m + ii], tws[m + ii], q);
                        s[j] = add_mod_w(u, v, q);
                        s[j + tt] = sub_mod(u, v, q);
                    }
                    __syncthreads();
                }
                const uint32_t *row = rgsw + ((((uint64_t)b * 2 + p) * ell + i) * 2) * LN + (uint64_t)l * n;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const uint32_t j = tid + k * CT_THREADS;
                    if (j < n) {
                        const uint32_t dh = s[__brev(j) >> (32 - logn)];
                        acc[0][k] = add_mod_w(acc[0][k], mulmod_any(dh, row[j], q, mu), q);
                        acc[1][k] = add_mod_w(acc[1][k], mulmod_any(dh, row[LN + j], q, mu), q);
                    }
                }
            }
        }
    }
    // out[b][c][t] = ct0[b][c][2t] + acc[c]
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const uint32_t *c0 = ct + ((uint64_t)(b * 2 + c) * ncols + 2 * t) * LN + (uint64_t)l * n;
        uint32_t *o = out + ((uint64_t)(b * 2 + c) * nout + t) * LN + (uint64_t)l * n;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint32_t j = tid + k * CT_THREADS;
            if (j < n) o[j] = add_mod_w(c0[j], acc[c][k], q);
        }
    }
}

// ------------------------------------------------------------------ host
static void split128(u128 x, uint32_t (&w)[4]) {
    for (int i = 0; i < 4; ++i) w[i] = (uint32_t)(x >> (32 * i));
}

static uint32_t shoup32(uint32_t w, uint32_t q) { return (uint32_t)(((uint64_t)w << 32) / q); }

void coltor_check_gadget(const pir_params &ring, uint32_t log2z, uint32_t ell) {
    PIR_REQUIRE(ell >= 1 && ell <= 8, "ell must be 1..8 (got %u)", ell);
    PIR_REQUIRE(log2z >= 1 && log2z <= 30, "log2z must be 1..30 (got %u)", log2z);
    u128 Q = 1;
    uint32_t qmin = 0xFFFFFFFFu;
    for (uint32_t l = 0; l < ring.nprimes; ++l) {
        Q *= ring.q[l];
        qmin = std::min(qmin, ring.q[l]);
    }
    const uint32_t bits = log2z * ell;
    PIR_REQUIRE(bits >= 128 || ((u128)1 << bits) > Q, "z^ell = 2^%u must exceed Q", bits);
    PIR_REQUIRE((1u << (log2z - 1)) + 1u < qmin, "digits up to 2^%u + 1 must stay below every prime",
                log2z - 1);
    if (ring.n * ring.nprimes > 16384)
        PIR_FAIL(PIR_EUNSUPPORTED, "the stage keeps L*N = %u words in LDS; at most 16384",
                 ring.n * ring.nprimes);
}

void launch_coltor_stage(const pir_params &ring, const uint32_t *ct, uint32_t B, uint32_t ncols,
                         const uint32_t *rgsw, uint32_t log2z, uint32_t ell, uint32_t *out, hipStream_t st) {
    const uint32_t L = ring.nprimes, n = ring.n, nout = (ncols + 1) / 2;
    uint32_t logn = 0;
    while ((1u << logn) < n) ++logn;
    ColtorPrimes pr{};
    u128 Q = 1;
    for (uint32_t l = 0; l < L; ++l) Q *= ring.q[l];
    split128(Q, pr.Q);
    split128(Q >> 1, pr.Qhalf);
    for (uint32_t l = 0; l < L; ++l) {
        const uint32_t q = ring.q[l];
        const NttTables &t = ntt_tables(q, n);
        pr.fwd[l] = t.fwd;
        pr.inv[l] = t.inv;
        pr.q[l] = q;
        pr.ninv[l] = t.n_inv;
        pr.ninv_s[l] = t.n_inv_shoup;
        const u128 qh = Q / q;
        split128(qh, pr.qhat[l]);
        const uint32_t c = pow_mod((uint64_t)(qh % q), q - 2, q);
        pr.crt_c[l] = c;
        pr.crt_cs[l] = shoup32(c, q);
        pr.mu[l] = make_modq(q).mu;
    }
    const uint64_t nodes = (uint64_t)B * nout;
    if (nodes == 0) return;
    PIR_REQUIRE(nodes * 2 < (1ull << 31) && nodes * L < (1ull << 31), "ColTor launch too large");
    StreamScratch scratch((size_t)nodes * 2 * ell * n * sizeof(int32_t), st);
    int32_t *dg = scratch.as<int32_t>();

    const size_t lds1 = (size_t)L * n * sizeof(uint32_t);
    PIR_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&coltor_dcp_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds1));
    coltor_dcp_kernel<<<(uint32_t)(nodes * 2), CT_THREADS, lds1, st>>>(ct, ncols, nout, L, n, logn, log2z, ell,
                                                                       dg, pr);
    PIR_LAUNCH_CHECK();
    const size_t lds2 = (size_t)n * sizeof(uint32_t);
    auto go = [&](auto kern) {
        PIR_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds2));
        kern<<<(uint32_t)(nodes * L), CT_THREADS, lds2, st>>>(ct, rgsw, dg, out, ncols, nout, L, n, logn, ell, pr);
    };
    const uint32_t K = (n + CT_THREADS - 1) / CT_THREADS;
    if (K <= 1) go(&coltor_mac_kernel<1>);
    else if (K <= 2) go(&coltor_mac_kernel<2>);
    else if (K <= 4) go(&coltor_mac_kernel<4>);
    else if (K <= 8) go(&coltor_mac_kernel<8>);
    else go(&coltor_mac_kernel<CT_MAXK>);
    PIR_LAUNCH_CHECK();
}

}  // namespace pir
