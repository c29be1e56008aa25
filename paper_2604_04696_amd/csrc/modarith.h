// Device-side modular arithmetic for primes q < 2^32 (the lazy and MFMA forms
// need q < 2^30; the _w / wide forms cover 2^30 <= q < 2^32).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "common.h"

namespace pir {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// 16-byte load marked non-temporal: streamed data that is read once should
// not displace reused lines from the caches.
__device__ __forceinline__ uint4 ld_nt(const uint4 *p) {
    u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
}

// 16-byte store marked non-temporal (written once, read back only by a later
// kernel).
__device__ __forceinline__ void st_nt(uint4 *p, const uint4 &x) {
    const u32x4 v = {x.x, x.y, x.z, x.w};
    __builtin_nontemporal_store(v, reinterpret_cast<u32x4 *>(p));
}

// hi*2^32 + lo  ==  hi*r32 + lo  (mod q).  For x < 2^64 the result is below
// 2^32*r32 + 2^32; a single v_mad_u64_u32.
__device__ __forceinline__ uint64_t fold32(uint64_t x, uint32_t r32) {
    return (uint64_t)(uint32_t)(x >> 32) * r32 + (uint64_t)(uint32_t)x;
}

// Brings a lazy 64-bit sum back under 2^60 + 2^32, after which fifteen more
// products of residues (< (2^30-1)^2 each) still fit in 64 bits:
//   one fold suffices when r32 < 2^28 (2^32 * 2^28 + 2^32),
//   otherwise a second fold takes the first result (< 2^62 + 2^32) there.
__device__ __forceinline__ uint64_t lazy_fold(uint64_t x, const ModQ &m) {
    x = fold32(x, m.r32);
    if (m.fold2) x = fold32(x, m.r32);
    return x;
}

// Barrett reduction of any 64-bit value into [0, q) for any q < 2^32:
// qhat = floor(x * mu / 2^64) is floor(x/q) or one less, so one correction.
__device__ __forceinline__ uint32_t reduce64(uint64_t x, const ModQ &m) {
    uint64_t qh = __umul64hi(x, m.mu);
    uint64_t r = x - qh * (uint64_t)m.q;
    return (uint32_t)(r >= m.q ? r - m.q : r);
}

// (wraps * 2^64 + sum) mod q: wraps * (2^64 mod q) < 2^16 * 2^32 for up to
// 2^16 products, so one more Barrett step after adding it to sum mod q.
__device__ __forceinline__ uint32_t reduce_wide(uint64_t sum, uint32_t wraps, const ModQ &m) {
    return reduce64((uint64_t)reduce64(sum, m) + (uint64_t)wraps * m.r64, m);
}

// ------------------------------------------------- wide primes (q >= 2^30)
// For 2^30 <= q < 2^32 a product of residues reaches 2^64 and a sum of two
// residues 2^33, so these forms keep 64-bit intermediates.
__device__ __forceinline__ uint32_t add_mod_w(uint32_t a, uint32_t b, uint32_t q) {
    const uint64_t s = (uint64_t)a + b;
    return (uint32_t)(s >= q ? s - q : s);
}

// Shoup's product with its [0, 2q) intermediate held in 64 bits.
__device__ __forceinline__ uint32_t mul_shoup_w(uint32_t a, uint32_t w, uint32_t ws, uint32_t q) {
    const uint64_t r = (uint64_t)a * w - (uint64_t)__umulhi(a, ws) * q;
    return (uint32_t)(r >= q ? r - q : r);
}

// A multiply-add keeps a 64-bit sum and counts its wraps (at most one per
// product); the value is wraps * 2^64 + sum.
__device__ __forceinline__ void mad_wide(uint64_t &sum, uint32_t &wraps, uint32_t x, uint32_t y) {
    uint64_t t;
    wraps += __builtin_add_overflow(sum, (uint64_t)x * y, &t) ? 1u : 0u;
    sum = t;
}

// Shoup multiplication by a constant w < q with companion ws = floor(w*2^32/q):
// a*w - floor(a*ws/2^32)*q lies in [0, 2q) for a < 2^32; one correction.
__device__ __forceinline__ uint32_t mul_shoup(uint32_t a, uint32_t w, uint32_t ws, uint32_t q) {
    uint32_t qt = __umulhi(a, ws);
    uint32_t r = a * w - qt * q;
    return r >= q ? r - q : r;
}

__device__ __forceinline__ uint32_t add_mod(uint32_t a, uint32_t b, uint32_t q) {
    uint32_t s = a + b;
    return s >= q ? s - q : s;
}

__device__ __forceinline__ uint32_t sub_mod(uint32_t a, uint32_t b, uint32_t q) {
    return a >= b ? a - b : a + q - b;
}

// Nearest integer of x for |x| < 2^51: adding and removing 1.5 * 2^52 leaves
// no fraction bits (round to nearest even).  Written as an fma so the product
// x * s is not rounded before the shift.
__device__ __forceinline__ double round_mul(double x, double s) {
    constexpr double SHIFT = 6755399441055744.0;   // 1.5 * 2^52
    return fma(x, s, SHIFT) - SHIFT;
}

// Recombines the seven digit-product classes of one output,
//   sum_s G_s 2^(8s) mod q,   |G_s| <= 2^27,
// in exact binary64 arithmetic:
//   E = G_0 + 2^8 G_1 + 2^16 G_2 + 2^24 G_3        |E| < 2^51 + 2^44 (exact)
//   H = G_4 + 2^8 G_5 + 2^16 G_6                   |H| < 2^44 (exact)
//   h = H - round(H/q) q                           |h| < q (exact remainder)
// then, with c32 = 2^32 mod q,
//   SPLIT = false:  t = E + h c32, exact when q c32 < 3 * 2^51 - 2^45 (the
//                   host checks this; it holds for every q < 2^26 and for q
//                   just below 2^30, where c32 = 4 (2^30 - q) is small);
//   MODE = 1:       h = 2^15 h1 + h0 (0 <= h0 < 2^15, |h1| <= 2^15) and
//                   t = E + h0 c32 + h1 c47, c47 = 2^47 mod q, each product
//                   below 2^45 in magnitude;
//   MODE = 2 (any q < 2^32; taken when some prime is 2^30 or more;
//             |h| <= q/2 < 2^31):
//                   h = 2^16 h1 + h0 (0 <= h0 < 2^16, |h1| <= 2^15) and
//                   t = E + h0 c32 + h1 c48, c48 = 2^48 mod q, products below
//                   2^48, |t| < 2^52;
// finally r = t - round(t/q) q lies in (-q, q) and min(r, r + q) taken as
// unsigned 32-bit words is the canonical residue (for MODE 2, where q may
// exceed 2^31, r goes through a 64-bit integer).  MODE = 0 is the direct
// form above.  (M is any struct with qd, qinv, c32, c47, c48 and q.)
template <int MODE, class M>
__device__ __forceinline__ uint32_t combine_classes(const int (&g)[7], const M &m) {
    double e = (double)g[3];
    e = fma(e, 256.0, (double)g[2]);
    e = fma(e, 256.0, (double)g[1]);
    e = fma(e, 256.0, (double)g[0]);
    double hh = (double)g[6];
    hh = fma(hh, 256.0, (double)g[5]);
    hh = fma(hh, 256.0, (double)g[4]);
    const double h = fma(-round_mul(hh, m.qinv), m.qd, hh);
    double t;
    if (MODE == 2) {
        const double h1 = floor(h * (1.0 / 65536.0));
        const double h0 = fma(-h1, 65536.0, h);
        t = fma(h0, m.c32, e);
        t = fma(h1, m.c48, t);
        const int64_t r = (int64_t)fma(-round_mul(t, m.qinv), m.qd, t);
        return (uint32_t)(r < 0 ? r + (int64_t)m.q : r);
    }
    if (MODE == 1) {
        const double h1 = floor(h * (1.0 / 32768.0));
        const double h0 = fma(-h1, 32768.0, h);
        t = fma(h0, m.c32, e);
        t = fma(h1, m.c47, t);
    } else {
        t = fma(h, m.c32, e);
    }
    const uint32_t r = (uint32_t)(int32_t)fma(-round_mul(t, m.qinv), m.qd, t);
    return min(r, r + m.q);
}

// Whether the SPLIT = false recombination is exact for q (see above).
__host__ __device__ inline bool combine_direct_ok(uint32_t q) {
    const double c32 = (double)((1ull << 32) % q);
    return (double)q * c32 <= 3.0 * 2251799813685248.0 - 35184372088832.0;   // 3*2^51 - 2^45
}

// Balanced signed base-2^8 digits: x = sum_i d_i 2^(8i), d_i in [-128, 127],
// for -2155905152 <= x <= 2139062143 (-0x80808080 .. 0x7F7F7F7F, the whole
// reach of four such digits).  Returned packed as four int8 in one 32-bit
// word, digit i in byte i.  The top digit of 0 <= x < 2^30 stays in [0, 64].
__device__ __forceinline__ uint32_t split_digits(uint32_t x) {
    uint32_t packed = 0;
    int32_t v = (int32_t)x;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        int32_t d = ((v + 128) & 255) - 128;
        packed |= ((uint32_t)(uint8_t)(int8_t)d) << (8 * i);
        v = (v - d) >> 8;
    }
    return packed;
}

// The digits of a residue r of any prime q < 2^32.  The reach of four digits
// holds 2^32 - 1 consecutive integers, so every residue class has a
// representative in it: x = r for r <= 0x7F7F7F7F, x = r - q above, which is
// at least 0x7F7F7F80 - q >= -2155905151.  That x may lie below -2^31, so the
// split runs on 64-bit values.
__device__ __forceinline__ uint32_t split_digits_window(uint32_t r, uint32_t q) {
    int64_t v = r > 0x7F7F7F7Fu ? (int64_t)r - (int64_t)q : (int64_t)r;
    uint32_t packed = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t d = ((v + 128) & 255) - 128;
        packed |= ((uint32_t)(uint8_t)(int8_t)d) << (8 * i);
        v = (v - d) >> 8;
    }
    return packed;
}

// Maps blockIdx.x so that runs of consecutive logical block indices execute
// on the same XCD (the hardware deals workgroups to the 8 XCDs round-robin),
// keeping data that neighbouring blocks share inside one XCD's L2.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t bid, uint32_t nblocks) {
    constexpr uint32_t X = 8;
    uint32_t per = nblocks / X, rem = nblocks % X;
    uint32_t xcd = bid % X, r = bid / X;
    // XCDs [0, rem) own per+1 logical blocks, the rest own per
    uint32_t base = xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per;
    return base + r;
}

}  // namespace pir
