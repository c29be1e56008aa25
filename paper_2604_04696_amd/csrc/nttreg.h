// Register-blocked negacyclic NTT helpers shared by the query front end and
// the ColTor stage.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "modarith.h"

namespace pir {

// Register-blocked transform for N >= 256: a polynomial is handled by
// T = N/16 threads that each keep 16 of its values in registers.  The
// butterfly stages (bit x of the pair distance, from logN-1 down to 0) run in
// chunks of up to four: during a chunk the register index r of a thread
// covers four index bits [lo, lo+4) (for the last chunk, bits [0, 4)), so
// every pair of the chunk's stages is local to one thread; between chunks
// the values are redistributed through LDS (padded one word per 16).  The
// element index of (thread t, register r) with register bits starting at lo:
//   e = (t mod 2^lo) | r << lo | (t >> lo) << (lo + 4).
// The butterfly of stage x on pair (e, e + 2^x) uses the psi power of group
// e >> (x+1) among N >> (x+1) groups, exactly as the one-stage-per-barrier
// form; values stay in [0, 4q) between stages (lazy butterflies) and are
// reduced once before the store.  A last exchange writes point bitrev(e) so that global stores are in
// natural point order and coalesced.
constexpr int QR = 16;   // values per thread

__device__ __forceinline__ uint32_t qf_pad(uint32_t e) { return e + (e >> 4); }

// Lazy butterfly (Harvey): inputs and outputs in [0, 4q), which fits 32 bits
// for q < 2^30.  x is first brought into [0, 2q) (x - 2q wraps above x when
// x < 2q, so the minimum picks the reduced value); Shoup's product
// t = y w - floor(y w' / 2^32) q without its final correction lies in
// [0, 2q) for any 32-bit y.  It is formed negated, nt = -t mod 2^32, so that
// x + t = x - nt and x - t + 2q = x + 2q + nt, the latter one three-input
// add.
__device__ __forceinline__ void qf_bfly(uint32_t &x, uint32_t &y, uint32_t w, uint32_t ws, uint32_t q,
                                        uint32_t q2) {
    const uint32_t xr = min(x, x - q2);
    const uint32_t nt = __umulhi(y, ws) * q - y * w;
    x = xr - nt;
    y = xr + q2 + nt;
}

// [0, 4q) -> [0, q)
__device__ __forceinline__ uint32_t qf_reduce4(uint32_t x, uint32_t q, uint32_t q2) {
    x = min(x, x - q2);
    return min(x, x - q);
}
__device__ __forceinline__ uint32_t qf_elem(uint32_t t, uint32_t r, uint32_t lo) {
    return (t & ((1u << lo) - 1)) | (r << lo) | ((t >> lo) << (lo + 4));
}

// qf_elem(t, r, lo) is qf_elem(t, 0, lo) | r << lo with disjoint bit fields,
// so a shift, a bit reversal or the padding of it splits into a part of the
// thread and a part of the register index, which is a compile-time constant
// in the unrolled loops (qf_pad(a | b) = qf_pad(a) + qf_pad(b) for disjoint
// a and b): the LDS exchanges, twiddle reads and stores then take a per-
// thread base and immediate offsets instead of recomputing the index of
// every register (those index computations were a quarter of the
// transform's vector instructions).
__device__ __forceinline__ uint32_t qf_rpart(int r, uint32_t lo) { return (uint32_t)r << lo; }

// Butterfly forms of ntt_reg_block.
enum : int {
    NTT_LAZY = 0,   // q < 2^30: Harvey's butterfly, values in [0, 4q)
    NTT_WIDE = 1,   // q >= 2^30: canonical, 64-bit intermediates, values in [0, q)
    NTT_GROW = 2,   // (1 + 2 logN) q < 2^32: no correction at all, (x + t, x - t + 2q)
};

// Twiddle sources of ntt_reg_block: tw(x, gi) returns the psi power of group
// index gi (used by stage x) and its Shoup companion.
struct TwGlobal {   // two tables in global memory
    const uint32_t *w, *ws;
    __device__ __forceinline__ uint2 operator()(int, uint32_t gi) const { return make_uint2(w[gi], ws[gi]); }
};

// {w, w'} pairs staged in LDS (tw_pairs_fill).  Stage x uses the groups
// [N >> (x+1), N >> x); in the last chunk (register bits from 0, element
// r | 16t) thread t needs groups (N >> (x+1)) + t K + k, k < K = 2^(3-x), of
// stages x <= 3.  Those are stored at (N >> (x+1)) + k N/16 + t, so that the
// lanes of a wave read consecutive pairs instead of pairs K apart (K-way bank
// conflicts); the slot of a group depends on the group alone, so other
// chunks' reads of these stages stay correct.
template <int LOGN>
__device__ __forceinline__ uint32_t tw_pair_slot(int x, uint32_t gi) {
    constexpr uint32_t n = 1u << LOGN, T = n / QR;
    if (x > 3) return gi;
    const uint32_t base = n >> (x + 1), j = gi - base, sh = 3 - (uint32_t)x;
    return base + (j & ((1u << sh) - 1)) * T + (j >> sh);
}

template <int LOGN>
struct TwPairsLds {
    const uint2 *p;
    __device__ __forceinline__ uint2 operator()(int x, uint32_t gi) const { return p[tw_pair_slot<LOGN>(x, gi)]; }
};

// Fills the N pairs of TwPairsLds from the global tables w, ws (the N/16
// threads of the block, thread t); the caller synchronises before use.
template <int LOGN>
__device__ __forceinline__ void tw_pairs_fill(uint2 *p, const uint32_t *w, const uint32_t *ws, uint32_t t) {
    constexpr uint32_t n = 1u << LOGN, T = n / QR;
#pragma unroll
    for (uint32_t i = 0; i < QR; ++i) {
        const uint32_t gi = t + i * T;
        const int x = gi == 0 ? LOGN : LOGN - 1 - (31 - __clz(gi));   // gi in [N >> (x+1), N >> x)
        p[gi < T ? gi : tw_pair_slot<LOGN>(x, gi)] = make_uint2(w[gi], ws[gi]);
    }
}

// Forward transform of one polynomial held by all N/16 threads of a block
// (N = 2^LOGN >= 256).  On entry register r of thread t holds element
// qf_elem(t, r, LOGN - 4) of the natural coefficient order (a residue below
// q); on return it holds element 16t + r of the transform, which is point
// bitrev(16t + r), congruent mod q and bounded by the form: NTT_WIDE [0, q),
// NTT_LAZY [0, 4q), NTT_GROW [0, (1 + 2 logN) q) (each stage adds at most 2q,
// since Shoup's product without its correction lies in [0, 2q) for any
// 32-bit input).  poly is LDS of N + N/16 words; the first exchange begins
// with a barrier, so earlier reads of poly by the block are complete before
// it is overwritten.  tw: a twiddle source (TwGlobal, TwPairsLds).
template <int LOGN, int MODE, class TW>
__device__ __forceinline__ void ntt_reg_block(uint32_t (&v)[QR], uint32_t t, uint32_t *poly, const TW &tw,
                                              uint32_t q) {
    constexpr uint32_t n = 1u << LOGN;
    uint32_t lo = LOGN - 4;
#pragma unroll
    for (int hi = LOGN; hi > 0; hi -= 4) {
        const int clo = hi - 4 > 0 ? hi - 4 : 0;
        const uint32_t rlo = (uint32_t)clo;
        if (rlo != lo) {
            __syncthreads();
            const uint32_t pw = qf_pad(qf_elem(t, 0, lo)), pr = qf_pad(qf_elem(t, 0, rlo));
#pragma unroll
            for (int r = 0; r < QR; ++r) poly[pw + qf_pad(qf_rpart(r, lo))] = v[r];
            __syncthreads();
#pragma unroll
            for (int r = 0; r < QR; ++r) v[r] = poly[pr + qf_pad(qf_rpart(r, rlo))];
            lo = rlo;
        }
        // (the twiddle index stays in the per-register form: written as a
        // thread base plus a constant, the compiler proves the first chunk's
        // twiddles wave-uniform and, from global memory, reads them with
        // scalar loads, whose wait counter the LDS exchanges share)
#pragma unroll
        for (int x = hi - 1; x >= clo; --x) {
            const uint32_t bit = 1u << (x - (int)lo), mgroups = n >> (x + 1);
#pragma unroll
            for (int r = 0; r < QR; ++r) {
                if (r & bit) continue;
                const uint32_t gi = mgroups + (qf_elem(t, r, lo) >> (x + 1));
                const uint2 w2 = tw(x, gi);
                if (MODE == NTT_WIDE) {
                    const uint32_t u = v[r], w = mul_shoup_w(v[r | bit], w2.x, w2.y, q);
                    v[r] = add_mod_w(u, w, q);
                    v[r | bit] = sub_mod(u, w, q);
                } else if (MODE == NTT_GROW) {
                    // Shoup's product negated, as in qf_bfly
                    const uint32_t y = v[r | bit];
                    const uint32_t nt = __umulhi(y, w2.y) * q - y * w2.x;
                    v[r | bit] = v[r] + 2 * q + nt;
                    v[r] = v[r] - nt;
                } else {
                    qf_bfly(v[r], v[r | bit], w2.x, w2.y, q, 2 * q);
                }
            }
        }
    }
}

// Lazy Gentleman-Sande butterfly: (x, y) -> (x + y, (x - y) w), inputs and
// outputs in [0, 2q) for q < 2^30 (x - y + 2q < 4q fits 32 bits; Shoup's
// product without its correction lies in [0, 2q)).
__device__ __forceinline__ void qf_gs_bfly(uint32_t &x, uint32_t &y, uint32_t w, uint32_t ws, uint32_t q,
                                           uint32_t q2) {
    const uint32_t sum = x + y, d = x - y + q2;
    x = min(sum, sum - q2);
    y = d * w - __umulhi(d, ws) * q;
}

// Inverse transform (without the 1/N scale) of one polynomial held by N/16
// threads, stages ascending in chunks of four bits.  On entry register r of
// thread t holds position 16t + r of the bit-reversed arrangement (point
// bitrev(16t + r)); on return it holds N times coefficient
// qf_elem(t, r, LOGN - 4).  tw are the inverse twiddles (psi^-1 powers at
// bit-reversed indices) with companions at tws.  WIDE (q >= 2^30):
// canonical butterflies, outputs in [0, q); otherwise lazy, [0, 2q) from
// inputs in [0, 2q).  poly: LDS of N + N/16 words owned by these threads;
// exchanges begin with a block-wide barrier.
template <int LOGN, bool WIDE>
__device__ __forceinline__ void intt_reg_block(uint32_t (&v)[QR], uint32_t t, uint32_t *poly,
                                               const uint32_t *tw, const uint32_t *tws, uint32_t q) {
    constexpr uint32_t n = 1u << LOGN;
    uint32_t lo = 0;
#pragma unroll
    for (int clo = 0; clo < LOGN; clo += 4) {
        const int chi = clo + 4 < LOGN ? clo + 4 : LOGN;
        const uint32_t rlo = (uint32_t)(clo < LOGN - 4 ? clo : LOGN - 4);   // registers cover [rlo, rlo + 4)
        if (rlo != lo) {
            __syncthreads();
            const uint32_t pw = qf_pad(qf_elem(t, 0, lo)), pr = qf_pad(qf_elem(t, 0, rlo));
#pragma unroll
            for (int r = 0; r < QR; ++r) poly[pw + qf_pad(qf_rpart(r, lo))] = v[r];
            __syncthreads();
#pragma unroll
            for (int r = 0; r < QR; ++r) v[r] = poly[pr + qf_pad(qf_rpart(r, rlo))];
            lo = rlo;
        }
        const uint32_t eb = qf_elem(t, 0, lo);
#pragma unroll
        for (int x = clo; x < chi; ++x) {
            const uint32_t bit = 1u << (x - (int)lo), mgroups = n >> (x + 1);
            const uint32_t gb = mgroups + (eb >> (x + 1));
#pragma unroll
            for (int r = 0; r < QR; ++r) {
                if (r & bit) continue;
                const uint32_t gi = gb + (qf_rpart(r, lo) >> (x + 1));
                if (WIDE) {
                    const uint32_t u = v[r], w = v[r | bit];
                    v[r] = add_mod_w(u, w, q);
                    v[r | bit] = mul_shoup_w(sub_mod(u, w, q), tw[gi], tws[gi], q);
                } else {
                    qf_gs_bfly(v[r], v[r | bit], tw[gi], tws[gi], q, 2 * q);
                }
            }
        }
    }
}

}  // namespace pir
