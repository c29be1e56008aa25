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
// Two kernels, each in a register-blocked form for N >= 256 (16 values per
// thread, up to four butterfly stages per LDS exchange) and a
// one-stage-per-barrier form for smaller rings:
//   decomposition      one block per (node, input polynomial): the
//                      difference of the two columns and its inverse NTT for
//                      all L limbs (L*N <= 16384 words in LDS), then the
//                      reconstruction and decomposition, coefficient by
//                      coefficient; digits go out as int32 [node][2][ell][N]
//                      (ell*N words per polynomial instead of L*N residues
//                      per digit: each limb reduces them on load);
//   multiply-accumulate one block per (node, limb): for each of the 2*ell
//                      digit polynomials, the residues mod q_l, the forward
//                      NTT and the product with the two RGSW components of
//                      that row, summed in registers (up to N = 4096 the
//                      limb's twiddles are staged in LDS, and the next digit
//                      polynomial is loaded during the current transform);
//                      then ct0 is added and both output polynomials stored.
// The butterfly and sum forms are chosen per launch from the primes: wide
// (64-bit intermediates) for any prime of 2^30 or more, lazy below, and
// unreduced forward butterflies when (1 + 2 logN) q < 2^32; the small-ring
// forms use the wide arithmetic throughout.
#include <type_traits>

#include "common.h"
#include "modarith.h"
#include "nttreg.h"

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
    uint32_t crt_cn[PIR_MAX_PRIMES], crt_cns[PIR_MAX_PRIMES]; // the same times N^-1 (folds the INTT scale)
    uint64_t mu[PIR_MAX_PRIMES];                               // Barrett constants of reduce64
    ModQ mod[PIR_MAX_PRIMES];
    uint32_t qhat[PIR_MAX_PRIMES][4];                          // Q/q_l, 32-bit limbs, low first
    uint32_t Q[4], Qhalf[4];                                   // Q and floor(Q/2)
    // the short form (Q < 2^125 and log2z * ell <= 126): C = sum_{i < ell-1} (z/2) z^i
    // and C - Q mod 2^128, and 1/q_l in binary64
    uint32_t C[4], CmQ[4];
    double qinv[PIR_MAX_PRIMES];
    uint32_t fast;
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

// ------------------------------- kernel 1, register-blocked (N >= 256)
// L*N/16 threads: thread group l (N/16 threads) transforms limb l with 16
// values per thread, then all limbs of a coefficient meet in LDS for the
// reconstruction.  Shared by the decomposition: (Q/q_l)^-1 N^-1 mod q_l.
// The short form: y_l = x_l (Q/q_l)^-1 N^-1 mod q_l; S = sum_l y_l Q/q_l taken
// mod 2^128 and k = floor(sum_l y_l / q_l) in binary64 (S - k Q is the
// reconstruction up to one Q either way: the estimate's error is far below 1,
// and S - k Q lies in (-Q, 2Q), inside the signed 128-bit range for
// Q < 2^125).  The balanced digits of the centred value v are the plain
// base-z digits of v + C, each less z/2 (C = sum_{i < ell-1} (z/2) z^i: adding
// z/2 to each digit position is what the balanced recursion's rounding does),
// and the last one is what remains after ell-1 arithmetic shifts; the value
// stays below 2^126 since log2z * ell <= 126.  Digit i is then one mask of the
// low word and a 4-word funnel shift.
__device__ __forceinline__ void dcp_coefficient_short(const uint32_t *x, uint32_t L, uint32_t j, uint32_t log2z,
                                                      uint32_t ell, uint64_t n, int32_t *dst,
                                                      const ColtorPrimes &pr, bool wide) {
    const u128 Q = u128_of(pr.Q);
    u128 S = 0;
    double fk = 0.0;
    for (uint32_t l = 0; l < L; ++l) {
        const uint32_t q = pr.q[l];
        const uint32_t y = wide ? mul_shoup_w(x[l], pr.crt_cn[l], pr.crt_cns[l], q)
                                : mul_shoup(x[l], pr.crt_cn[l], pr.crt_cns[l], q);
        fk = fma((double)y, pr.qinv[l], fk);
        S += (u128)y * u128_of(pr.qhat[l]);
    }
    u128 v = S - (u128)(uint32_t)fk * Q;
    if ((i128)v < 0) v += Q;
    else if (v >= Q) v -= Q;
    v += v > u128_of(pr.Qhalf) ? u128_of(pr.CmQ) : u128_of(pr.C);
    uint32_t w0 = (uint32_t)v, w1 = (uint32_t)(v >> 32), w2 = (uint32_t)(v >> 64), w3 = (uint32_t)(v >> 96);
    const uint32_t zmask = (1u << log2z) - 1, zhalf = 1u << (log2z - 1);
    for (uint32_t i = 0; i + 1 < ell; ++i) {
        dst[i * n + j] = (int32_t)(w0 & zmask) - (int32_t)zhalf;
        w0 = __builtin_amdgcn_alignbit(w1, w0, log2z);
        w1 = __builtin_amdgcn_alignbit(w2, w1, log2z);
        w2 = __builtin_amdgcn_alignbit(w3, w2, log2z);
        w3 = (uint32_t)((int32_t)w3 >> log2z);
    }
    dst[(ell - 1) * n + j] = (int32_t)w0;
}

__device__ __forceinline__ void dcp_coefficient(const uint32_t *x, uint32_t L, uint32_t j, uint32_t log2z,
                                                uint32_t ell, uint64_t n, int32_t *dst, const ColtorPrimes &pr,
                                                bool wide) {
    if (pr.fast) {
        dcp_coefficient_short(x, L, j, log2z, ell, n, dst, pr, wide);
        return;
    }
    const u128 Q = u128_of(pr.Q), Qhalf = u128_of(pr.Qhalf);
    u128 acc = 0;
    for (uint32_t l = 0; l < L; ++l) {
        const uint32_t q = pr.q[l];
        const uint32_t y = wide ? mul_shoup_w(x[l], pr.crt_cn[l], pr.crt_cns[l], q)
                                : mul_shoup(x[l], pr.crt_cn[l], pr.crt_cns[l], q);
        const u128 term = (u128)y * u128_of(pr.qhat[l]);
        u128 sum = acc + term;
        if (sum < acc || sum >= Q) sum -= Q;
        acc = sum;
    }
    const i128 zhalf = (i128)1 << (log2z - 1);
    const i128 zmask = ((i128)1 << log2z) - 1;
    i128 v = acc > Qhalf ? -(i128)(Q - acc) : (i128)acc;
    for (uint32_t i = 0; i + 1 < ell; ++i) {
        const i128 d = ((v + zhalf) & zmask) - zhalf;
        dst[i * n + j] = (int32_t)d;
        v = (v - d) >> log2z;
    }
    dst[(ell - 1) * n + j] = (int32_t)v;
}

template <int LOGN, bool WIDE>
__global__ void __launch_bounds__(1024)
coltor_dcp_reg_kernel(const uint32_t *__restrict__ ct, uint32_t ncols, uint32_t nout, uint32_t L,
                      uint32_t log2z, uint32_t ell, int32_t *__restrict__ digits, ColtorPrimes pr) {
    constexpr uint32_t n = 1u << LOGN, T = n / QR, PW = n + n / 16;
    extern __shared__ uint32_t s[];                  // [L][PW]
    const uint32_t tid = threadIdx.x, l = tid / T, t = tid % T;
    const uint32_t p = blockIdx.x % 2, node = blockIdx.x / 2;
    const uint32_t b = node / nout, tn = node % nout;
    if (2 * tn + 1 >= ncols) return;                 // unpaired column: no product
    const uint64_t LN = (uint64_t)L * n;
    const uint32_t *c0 = ct + ((uint64_t)(b * 2 + p) * ncols + 2 * tn) * LN + (uint64_t)l * n;
    const uint32_t *c1 = c0 + LN;
    const uint32_t q = pr.q[l];
    uint32_t *poly = s + l * PW;

    // difference; point j goes to position bitrev(j)
#pragma unroll
    for (int r = 0; r < QR; ++r) {
        // t < T = 2^(LOGN-4): t and r T are disjoint bit fields (see qf_rpart)
        const uint32_t j = t + r * T;
        poly[qf_pad(__brev(t) >> (32 - LOGN)) + qf_pad(__brev((uint32_t)r * T) >> (32 - LOGN))] =
            sub_mod(c1[j], c0[j], q);
    }
    __syncthreads();
    uint32_t v[QR];
#pragma unroll
    for (int r = 0; r < QR; ++r) v[r] = poly[qf_pad(t * QR) + r];
    intt_reg_block<LOGN, WIDE>(v, t, poly, pr.inv[l], pr.inv[l] + n, q);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < QR; ++r) poly[qf_pad(qf_elem(t, 0, LOGN - 4)) + qf_pad(qf_rpart(r, LOGN - 4))] = v[r];
    __syncthreads();
    int32_t *dst = digits + ((uint64_t)node * 2 + p) * ell * n;
    for (uint32_t j = tid; j < n; j += L * T) {
        uint32_t x[PIR_MAX_PRIMES];
        for (uint32_t k = 0; k < L; ++k) x[k] = s[k * PW + qf_pad(j)];
        dcp_coefficient(x, L, j, log2z, ell, n, dst, pr, WIDE);
    }
}

// ------------------------------------------------- kernel 2: NTT + products
// One-stage-per-barrier form for small rings (N < 256).  grid: nodes * L
// blocks; thread tid owns points j = tid + k * CT_THREADS.

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

// ------------------------------- kernel 2, register-blocked (N >= 256)
// The RGSW rows are first permuted so that word 16t + r of a row holds point
// bitrev(16t + r) (rgsw_permute_kernel): after the register-blocked forward
// transform thread t holds exactly those points of a digit polynomial in
// registers 0..15, so each multiply reads 64 contiguous bytes per thread and
// no digit polynomial goes back through LDS to natural order.  Products are
// summed lazily in 64 bits (at most 16 below 2^60 each for q < 2^30;
// wrap-counting sums for wider primes) and reduced once; the two results
// then take one LDS exchange each to natural order, where ct0 is added.
// One block per row of n words: the row goes to LDS with coalesced loads
// (padded one word per 64, so that the bit-reversed reads of a wave fall on
// distinct banks two lanes at a time) and leaves with coalesced stores.  (The
// gather straight from global memory ran at ~1.6 TB/s.)
__global__ void __launch_bounds__(256)
rgsw_permute_kernel(const uint32_t *__restrict__ in, uint32_t *__restrict__ out, uint32_t logn) {
    extern __shared__ uint32_t s[];   // n + n/64 words
    const uint32_t n = 1u << logn;
    const uint64_t base = (uint64_t)blockIdx.x * n;
    for (uint32_t i = threadIdx.x; i < n; i += 256) s[i + (i >> 6)] = in[base + i];
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < n; j += 256) {
        const uint32_t k = __brev(j) >> (32 - logn);
        out[base + j] = s[k + (k >> 6)];
    }
}

template <int LOGN, int MODE>
__global__ void __launch_bounds__((1u << LOGN) / QR)
coltor_mac_reg_kernel(const uint32_t *__restrict__ ct, const uint32_t *__restrict__ rgsw_p,
                      const int32_t *__restrict__ digits, uint32_t *__restrict__ out, uint32_t ncols,
                      uint32_t nout, uint32_t L, uint32_t ell, ColtorPrimes pr) {
    constexpr uint32_t n = 1u << LOGN, T = n / QR;
    // up to N = 4096 the twiddles are staged in LDS: kept in registers across
    // the 2 ell transforms they took ~90 VGPRs (236 in all, two waves per
    // SIMD, 61% of the VALU issue slots used)
    constexpr bool TW_LDS = LOGN <= 12;
    extern __shared__ uint32_t s[];                  // n + n/16 words, then (TW_LDS) n twiddle pairs
    const uint32_t t = threadIdx.x;
    // the L limb blocks of a node, and consecutive nodes of a client, run on
    // one XCD: the node's digits and the client's RGSW rows stay in its L2
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const uint32_t l = lb % L, node = lb / L;
    const uint32_t b = node / nout, tn = node % nout;
    const uint32_t q = pr.q[l];
    const uint64_t LN = (uint64_t)L * n;
    const uint32_t *c0 = ct + ((uint64_t)(b * 2) * ncols + 2 * tn) * LN + (uint64_t)l * n;   // component 0
    uint32_t *o = out + ((uint64_t)(b * 2) * nout + tn) * LN + (uint64_t)l * n;
    const uint64_t c_in = (uint64_t)ncols * LN, c_out = (uint64_t)nout * LN;   // component strides

    if (2 * tn + 1 >= ncols) {                       // unpaired column passes through
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int r = 0; r < QR; ++r) o[c * c_out + t + r * T] = c0[c * c_in + t + r * T];
        return;
    }
    const ModQ &m = pr.mod[l];
    const uint32_t *tw = pr.fwd[l], *tws = tw + n;
    uint2 *stw = reinterpret_cast<uint2 *>(s + n + n / 16);
    if constexpr (TW_LDS) {
        tw_pairs_fill<LOGN>(stw, tw, tws, t);
        __syncthreads();
    }
    uint64_t acc[2][QR];
    uint32_t wraps[2][QR];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int r = 0; r < QR; ++r) acc[c][r] = 0, wraps[c][r] = 0;

    // the 2 ell digit polynomials of the node (p, i) in turn; the next one's
    // values are loaded while the current one is transformed (waiting for
    // them right before each transform left the SIMDs idle for a third of
    // the kernel)
    const uint32_t ne = 2 * ell;
    const int32_t *dg = digits + (uint64_t)node * ne * n + qf_elem(t, 0, LOGN - 4);
    int32_t dn[QR];
#pragma unroll
    for (int r = 0; r < QR; ++r) dn[r] = dg[qf_rpart(r, LOGN - 4)];
    for (uint32_t pi = 0; pi < ne; ++pi) {
        const uint32_t p = pi >= ell, i = pi - p * ell;
        uint32_t v[QR];
#pragma unroll
        for (int r = 0; r < QR; ++r) v[r] = dn[r] < 0 ? (uint32_t)(dn[r] + (int64_t)q) : (uint32_t)dn[r];
        if (pi + 1 < ne) {
            dg += n;
#pragma unroll
            for (int r = 0; r < QR; ++r) dn[r] = dg[qf_rpart(r, LOGN - 4)];
        }
        if constexpr (TW_LDS) ntt_reg_block<LOGN, MODE>(v, t, s, TwPairsLds<LOGN>{stw}, q);
        else ntt_reg_block<LOGN, MODE>(v, t, s, TwGlobal{tw, tws}, q);
        const uint4 *row = reinterpret_cast<const uint4 *>(
            rgsw_p + ((((uint64_t)b * 2 + p) * ell + i) * 2) * LN + (uint64_t)l * n + (uint64_t)t * QR);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const uint4 w4 = row[c * (LN / 4) + g];
                const uint32_t w[4] = {w4.x, w4.y, w4.z, w4.w};
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int r = 4 * g + k;
                    // NTT_GROW: the unreduced value (below (1 + 2 logN) q)
                    // goes into the 64-bit sum; the host checks 2 ell of
                    // these products fit
                    const uint32_t x = MODE == NTT_LAZY ? qf_reduce4(v[r], q, 2 * q) : v[r];
                    if (MODE == NTT_WIDE) mad_wide(acc[c][r], wraps[c][r], x, w[k]);
                    else acc[c][r] += (uint64_t)x * w[k];
                }
            }
        }
    }
    // register r of thread t holds point bitrev(16t + r): one exchange per
    // output polynomial to natural order, then out = ct0 + sum
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < QR; ++r) {
            const uint32_t res = MODE == NTT_WIDE ? reduce_wide(acc[c][r], wraps[c][r], m) : reduce64(acc[c][r], m);
            s[qf_pad(__brev(t * QR) >> (32 - LOGN)) + qf_pad(__brev((uint32_t)r) >> (32 - LOGN))] = res;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < QR; ++r) {
            const uint32_t j = t + r * T;
            o[c * c_out + j] = add_mod_w(c0[c * c_in + j], s[qf_pad(t) + qf_pad(r * T)], q);
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
    bool wide = false;
    u128 Q = 1;
    for (uint32_t l = 0; l < L; ++l) Q *= ring.q[l];
    split128(Q, pr.Q);
    split128(Q >> 1, pr.Qhalf);
    pr.fast = (Q >> 125) == 0 && log2z * ell <= 126;
    if (pr.fast) {
        u128 C = 0, zi = 1;
        for (uint32_t i = 0; i + 1 < ell; ++i, zi <<= log2z) C += zi << (log2z - 1);
        split128(C, pr.C);
        split128(C - Q, pr.CmQ);
    }
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
        pr.crt_cn[l] = (uint32_t)((uint64_t)c * t.n_inv % q);
        pr.crt_cns[l] = shoup32(pr.crt_cn[l], q);
        pr.mod[l] = make_modq(q);
        pr.qinv[l] = 1.0 / (double)q;
        pr.mu[l] = pr.mod[l].mu;
        wide = wide || q >= WIDE_Q;
    }
    const uint64_t nodes = (uint64_t)B * nout;
    if (nodes == 0) return;
    PIR_REQUIRE(nodes * 2 < (1ull << 31) && nodes * L < (1ull << 31), "ColTor launch too large");
    StreamScratch scratch((size_t)nodes * 2 * ell * n * sizeof(int32_t), st);
    int32_t *dg = scratch.as<int32_t>();

    if (n >= 256) {
        const size_t lds = (size_t)L * (n + n / 16) * sizeof(uint32_t);
        auto go1 = [&](auto kern) {
            PIR_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            kern<<<(uint32_t)(nodes * 2), L * (n / QR), lds, st>>>(ct, ncols, nout, L, log2z, ell, dg, pr);
        };
        auto pick1 = [&](auto w) {
            constexpr bool W = decltype(w)::value;
            switch (logn) {
                case 8: go1(&coltor_dcp_reg_kernel<8, W>); break;
                case 9: go1(&coltor_dcp_reg_kernel<9, W>); break;
                case 10: go1(&coltor_dcp_reg_kernel<10, W>); break;
                case 11: go1(&coltor_dcp_reg_kernel<11, W>); break;
                case 12: go1(&coltor_dcp_reg_kernel<12, W>); break;
                case 13: go1(&coltor_dcp_reg_kernel<13, W>); break;
                default: go1(&coltor_dcp_reg_kernel<14, W>); break;
            }
        };
        if (wide) pick1(std::true_type{});
        else pick1(std::false_type{});
    } else {
        const size_t lds1 = (size_t)L * n * sizeof(uint32_t);
        PIR_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&coltor_dcp_kernel),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds1));
        coltor_dcp_kernel<<<(uint32_t)(nodes * 2), CT_THREADS, lds1, st>>>(ct, ncols, nout, L, n, logn, log2z,
                                                                           ell, dg, pr);
    }
    PIR_LAUNCH_CHECK();
    if (n >= 256) {
        // RGSW rows in the transform's register order, then the blocked kernel
        const uint64_t rg_words = (uint64_t)B * 4 * ell * L * n;
        PIR_REQUIRE(rg_words / 256 < (1ull << 31), "ColTor launch too large");
        StreamScratch rgp(rg_words * sizeof(uint32_t), st);
        const size_t lds_p = (size_t)(n + n / 64) * sizeof(uint32_t);
        PIR_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&rgsw_permute_kernel),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_p));
        rgsw_permute_kernel<<<(uint32_t)(rg_words / n), 256, lds_p, st>>>(rgsw, rgp.as<uint32_t>(), logn);
        PIR_LAUNCH_CHECK();
        const size_t lds = (size_t)(n + n / 16) * sizeof(uint32_t) + (logn <= 12 ? (size_t)n * sizeof(uint2) : 0);
        auto go2 = [&](auto kern) {
            PIR_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            kern<<<(uint32_t)(nodes * L), n / QR, lds, st>>>(ct, rgp.as<uint32_t>(), dg, out, ncols, nout, L, ell,
                                                               pr);
        };
        // unreduced butterflies when every prime leaves room for logN stages of
        // growth and 2 ell products of the grown values fit a 64-bit sum
        bool grow = !wide;
        for (uint32_t l = 0; l < L && grow; ++l) {
            const u128 bound = (u128)(1 + 2 * logn) * ring.q[l];
            grow = bound < ((u128)1 << 32) && bound * ring.q[l] * (2 * ell) < ((u128)1 << 64);
        }
        auto pick = [&](auto mode) {
            constexpr int M = decltype(mode)::value;
            switch (logn) {
                case 8: go2(&coltor_mac_reg_kernel<8, M>); break;
                case 9: go2(&coltor_mac_reg_kernel<9, M>); break;
                case 10: go2(&coltor_mac_reg_kernel<10, M>); break;
                case 11: go2(&coltor_mac_reg_kernel<11, M>); break;
                case 12: go2(&coltor_mac_reg_kernel<12, M>); break;
                case 13: go2(&coltor_mac_reg_kernel<13, M>); break;
                default: go2(&coltor_mac_reg_kernel<14, M>); break;
            }
        };
        if (wide) pick(std::integral_constant<int, NTT_WIDE>{});
        else if (grow) pick(std::integral_constant<int, NTT_GROW>{});
        else pick(std::integral_constant<int, NTT_LAZY>{});
        PIR_LAUNCH_CHECK();
        return;
    }
    const size_t lds2 = (size_t)n * sizeof(uint32_t);
    auto go = [&](auto kern) {
        PIR_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds2));
        kern<<<(uint32_t)(nodes * L), CT_THREADS, lds2, st>>>(ct, rgsw, dg, out, ncols, nout, L, n, logn, ell, pr);
    };
    go(&coltor_mac_kernel<1>);   // n < 256: one point per thread
    PIR_LAUNCH_CHECK();
}

}  // namespace pir
