// Negacyclic NTT helper and the DB layout builders.
//
// The NTT is not on RowSel's hot path: it turns coefficient-domain DB records
// into the NTT domain at load time (sec. 2.2 / sec. 2.4.1: records are kept
// NTT'd so RowSel is point-wise) and serves tests as the client-side
// transform.  Convention: ahat_i = a(psi^(2i+1)), natural order.
//
// One workgroup transforms one polynomial in LDS: Cooley-Tukey butterflies
// with psi powers in bit-reversed order (forward, natural in -> bit-reversed
// positions) and Gentleman-Sande with inverse powers (inverse), the merged
// negacyclic formulation of Longa and Naehrig (CANS 2016); the bit reversal
// is folded into the global store (forward) or load (inverse).
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>
#include <vector>

#include "common.h"
#include "modarith.h"

namespace pir {

// ------------------------------------------------------------- host tables
uint32_t pow_mod(uint64_t a, uint64_t e, uint32_t q) {
    uint64_t r = 1 % q;
    a %= q;
    while (e) {
        if (e & 1) r = r * a % q;
        a = a * a % q;
        e >>= 1;
    }
    return (uint32_t)r;
}

static uint32_t smallest_generator(uint32_t q) {
    std::vector<uint32_t> f;
    uint32_t r = q - 1;
    for (uint32_t d = 2; (uint64_t)d * d <= r; ++d)
        if (r % d == 0) {
            f.push_back(d);
            while (r % d == 0) r /= d;
        }
    if (r > 1) f.push_back(r);
    for (uint32_t g = 2; g < q; ++g) {
        bool ok = true;
        for (uint32_t p : f)
            if (pow_mod(g, (q - 1) / p, q) == 1) { ok = false; break; }
        if (ok) return g;
    }
    PIR_FAIL(PIR_EINVAL, "no generator found for %u", q);
}

static uint32_t bitrev(uint32_t x, uint32_t logn) {
    uint32_t r = 0;
    for (uint32_t i = 0; i < logn; ++i) { r = (r << 1) | (x & 1); x >>= 1; }
    return r;
}

static uint32_t shoup(uint32_t w, uint32_t q) {
    return (uint32_t)(((uint64_t)w << 32) / q);
}

const NttTables &ntt_tables(uint32_t q, uint32_t n) {
    static std::mutex mu;
    static std::map<std::tuple<int, uint32_t, uint32_t>, NttTables> cache;
    int dev = 0;
    PIR_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    auto key = std::make_tuple(dev, q, n);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;

    uint32_t logn = 0;
    while ((1u << logn) < n) ++logn;
    uint32_t g = smallest_generator(q);
    uint32_t psi = pow_mod(g, (q - 1) / (2ull * n), q);
    uint32_t psi_inv = pow_mod(psi, q - 2, q);
    if (pow_mod(psi, n, q) != q - 1)
        PIR_FAIL(PIR_EINVAL, "psi is not a primitive 2N-th root mod %u", q);
    std::vector<uint32_t> fwd(2 * n), inv(2 * n);
    for (uint32_t k = 0; k < n; ++k) {
        uint32_t e = bitrev(k, logn);
        fwd[k] = pow_mod(psi, e, q);
        fwd[n + k] = shoup(fwd[k], q);
        inv[k] = pow_mod(psi_inv, e, q);
        inv[n + k] = shoup(inv[k], q);
    }
    NttTables t;
    t.q = q;
    t.n = n;
    t.fwd = static_cast<uint32_t *>(dev_alloc(sizeof(uint32_t) * 2 * n));
    t.inv = static_cast<uint32_t *>(dev_alloc(sizeof(uint32_t) * 2 * n));
    PIR_HIP(hipMemcpy(t.fwd, fwd.data(), sizeof(uint32_t) * 2 * n, hipMemcpyHostToDevice));
    PIR_HIP(hipMemcpy(t.inv, inv.data(), sizeof(uint32_t) * 2 * n, hipMemcpyHostToDevice));
    t.n_inv = pow_mod(n, q - 2, q);
    t.n_inv_shoup = shoup(t.n_inv, q);
    return cache.emplace(key, t).first->second;
}

// ------------------------------------------------------------------ kernels
constexpr int NTT_THREADS = 512;

// WIDE: q >= 2^30, sums and Shoup products kept in 64 bits (modarith.h).
template <bool INV, bool WIDE>
__global__ void __launch_bounds__(NTT_THREADS)
ntt_kernel(const uint32_t *in, uint32_t *out, uint64_t in_stride,   // in may equal out
           uint64_t out_stride, const uint32_t *__restrict__ tw, uint32_t q, uint32_t n,
           uint32_t logn, uint32_t ninv, uint32_t ninv_s) {
    extern __shared__ uint32_t s[];
    const uint32_t *src = in + (uint64_t)blockIdx.x * in_stride;
    uint32_t *dst = out + (uint64_t)blockIdx.x * out_stride;
    const uint32_t *tws = tw + n;
    const uint32_t tid = threadIdx.x;
    auto addm = [](uint32_t a, uint32_t b, uint32_t qq) { return WIDE ? add_mod_w(a, b, qq) : add_mod(a, b, qq); };
    auto mulm = [](uint32_t a, uint32_t w, uint32_t ws, uint32_t qq) {
        return WIDE ? mul_shoup_w(a, w, ws, qq) : mul_shoup(a, w, ws, qq);
    };

    for (uint32_t i = tid; i < n; i += NTT_THREADS) {
        uint32_t v = src[i];
        v = v >= q ? v % q : v;
        if (INV) s[__brev(i) >> (32 - logn)] = v;
        else     s[i] = v;
    }
    __syncthreads();

    const uint32_t half = n >> 1;
    if (!INV) {
        for (uint32_t m = 1, lt = logn - 1; m < n; m <<= 1, --lt) {
            for (uint32_t b = tid; b < half; b += NTT_THREADS) {
                uint32_t i = b >> lt;
                uint32_t j = (i << (lt + 1)) + (b & ((1u << lt) - 1));
                uint32_t t = 1u << lt;
                uint32_t u = s[j];
                uint32_t v = mulm(s[j + t], tw[m + i], tws[m + i], q);
                s[j] = addm(u, v, q);
                s[j + t] = sub_mod(u, v, q);
            }
            __syncthreads();
        }
        for (uint32_t i = tid; i < n; i += NTT_THREADS) dst[i] = s[__brev(i) >> (32 - logn)];
    } else {
        for (uint32_t m = half, lt = 0; m >= 1; m >>= 1, ++lt) {
            for (uint32_t b = tid; b < half; b += NTT_THREADS) {
                uint32_t i = b >> lt;
                uint32_t j = (i << (lt + 1)) + (b & ((1u << lt) - 1));
                uint32_t t = 1u << lt;
                uint32_t u = s[j], v = s[j + t];
                s[j] = addm(u, v, q);
                s[j + t] = mulm(sub_mod(u, v, q), tw[m + i], tws[m + i], q);
            }
            __syncthreads();
        }
        for (uint32_t i = tid; i < n; i += NTT_THREADS) dst[i] = mulm(s[i], ninv, ninv_s, q);
    }
}

void launch_ntt(const uint32_t *in, uint32_t *out, uint64_t count, uint64_t in_stride,
                uint64_t out_stride, const NttTables &t, bool inverse, hipStream_t st) {
    if (count == 0) return;
    uint32_t logn = 0;
    while ((1u << logn) < t.n) ++logn;
    const size_t lds = sizeof(uint32_t) * t.n;
    // gridDim.x is limited to 2^31-1; count stays far below in practice
    for (uint64_t c0 = 0; c0 < count; c0 += (1u << 30)) {
        uint32_t c = (uint32_t)std::min<uint64_t>(count - c0, 1u << 30);
        auto go = [&](auto inv, auto wide) {
            constexpr bool I = decltype(inv)::value, W = decltype(wide)::value;
            ntt_kernel<I, W><<<c, NTT_THREADS, lds, st>>>(in + c0 * in_stride, out + c0 * out_stride, in_stride,
                                                          out_stride, I ? t.inv : t.fwd, t.q, t.n, logn,
                                                          I ? t.n_inv : 0, I ? t.n_inv_shoup : 0);
        };
        const bool wide = t.q >= WIDE_Q;
        if (inverse) {
            if (wide) go(std::true_type{}, std::true_type{});
            else go(std::true_type{}, std::false_type{});
        } else {
            if (wide) go(std::false_type{}, std::true_type{});
            else go(std::false_type{}, std::false_type{});
        }
        PIR_LAUNCH_CHECK();
    }
}

// ------------------------------------------------------------ DB layouts
// NTT-domain source rows [nrows][D1][L][N] -> VALU layout [L][N/4][S][D0][W][4]
// (256-column strips, see DbLayoutValu).
// One thread moves one 16-byte vector (four consecutive points); consecutive
// threads take consecutive columns so every store wavefront is one
// contiguous 1 KiB run.
__global__ void db_layout_valu_kernel(const uint32_t *__restrict__ src, uint32_t *__restrict__ dst,
                                      uint32_t row0, uint32_t nrows, uint32_t d0, uint32_t d1,
                                      uint32_t L, uint32_t N) {
    const uint32_t G = N / 4;
    const uint64_t total = (uint64_t)nrows * L * G * d1;
    for (uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t n = (uint32_t)(idx % d1);
        uint64_t r1 = idx / d1;
        uint32_t g = (uint32_t)(r1 % G);
        uint64_t r2 = r1 / G;
        uint32_t l = (uint32_t)(r2 % L);
        uint32_t r = (uint32_t)(r2 / L);
        const uint4 v = *reinterpret_cast<const uint4 *>(src + (((uint64_t)r * d1 + n) * L + l) * N + 4 * g);
        const uint32_t strip = n / VALU_STRIP;
        const uint64_t o = valu_strip_base((uint64_t)l * G + g, strip, d0, d1) +
                           (uint64_t)(row0 + r) * valu_strip_width(strip, d1) + n % VALU_STRIP;
        *reinterpret_cast<uint4 *>(dst + 4 * o) = v;
    }
}

void launch_db_layout_valu(const pir_db &db, const uint32_t *ntt_src, uint32_t row0,
                           uint32_t nrows, hipStream_t st) {
    const auto &p = db.p;
    uint64_t total = (uint64_t)nrows * p.nprimes * (p.n / 4) * p.d1;
    if (!total) return;
    uint32_t blocks = (uint32_t)std::min<uint64_t>((total + 255) / 256, 1u << 20);
    db_layout_valu_kernel<<<blocks, 256, 0, st>>>(ntt_src, db.valu.data, row0, nrows, p.d0, p.d1,
                                                  p.nprimes, p.n);
    PIR_LAUNCH_CHECK();
}


}  // namespace pir
