/*
 * CPU oracle for RowSel -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the package's smoke check and the benchmark's CPU-baseline
 * leg may load this library.  It shares no code, header, table or constant
 * generator with the HIP library: everything here is written from the paper's
 * definitions, as plainly as possible, in exact integer arithmetic (products
 * in 64 bits, sums in unsigned 128 bits, one `%` per result).
 *
 * What each function follows:
 *   - RNS primes and the negacyclic NTT: paper section 2.4.1 (RNS and NTT
 *     representation): a polynomial of degree < N is stored as one length-N
 *     limb per prime q_l, and NTT turns negacyclic convolution into a
 *     point-wise product, NTT(a*b) = NTT(a) (.) NTT(b).
 *     Point order (a reading; the paper fixes none): natural order,
 *     ahat_i = a(psi^(2i+1)) = sum_j a_j psi^((2i+1) j), psi a primitive
 *     2N-th root of unity, psi = g^((q-1)/2N) with g the smallest generator.
 *   - RowSel: section 2.2 (RowSel) and section 2.3 (the point-wise GEMM
 *     M_out[p,m,n] = sum_k M_in0[p,m,k] * M_in1[p,k,n], p ranging over the
 *     L*N points, m over the 2*batch ciphertext polynomials, k over the D0
 *     rows and n over the D1 columns).  Boundary layouts:
 *       query [B][2][D0][L][N], DB [D0][D1][L][N], out [B][2][D1][L][N],
 *     with p = l*N + j and m = 2b + c.  Outputs are canonical residues in
 *     [0, q_l).
 *
 * Parity pins for every function live in the CPU test suite (direct O(N^2)
 * evaluation, Python big-integer products, closed forms, toy encryption).
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* ---------------------------------------------------------------- scalar */
static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q)
{
    return (uint64_t)(((u128)a * b) % q);
}

static uint64_t powmod(uint64_t a, uint64_t e, uint64_t q)
{
    uint64_t r = 1 % q;
    a %= q;
    while (e) {
        if (e & 1) r = mulmod(r, a, q);
        a = mulmod(a, a, q);
        e >>= 1;
    }
    return r;
}

/* Trial division; fine for the < 2^40 moduli this oracle is asked about. */
int oracle_is_prime(uint64_t n)
{
    if (n < 2) return 0;
    if (n % 2 == 0) return n == 2;
    for (uint64_t d = 3; d * d <= n; d += 2)
        if (n % d == 0) return 0;
    return 1;
}

/* The `count` largest primes q < 2^bits with q = 1 (mod 2n), descending.
 * Returns how many were found. */
uint32_t oracle_ntt_primes(uint32_t n, uint32_t bits, uint32_t count, uint64_t *out)
{
    uint64_t m = 2ull * n, top = (1ull << bits) - 1;
    uint64_t x = (top / m) * m + 1;
    if (x > top) x -= m;
    uint32_t found = 0;
    while (found < count && x > m) {
        if (oracle_is_prime(x)) out[found++] = x;
        x -= m;
    }
    return found;
}

/* Smallest generator of the multiplicative group mod prime q. */
uint64_t oracle_primitive_root(uint64_t q)
{
    uint64_t f[64];
    int nf = 0;
    uint64_t r = q - 1;
    for (uint64_t d = 2; d * d <= r; ++d) {
        if (r % d == 0) {
            f[nf++] = d;
            while (r % d == 0) r /= d;
        }
    }
    if (r > 1) f[nf++] = r;
    for (uint64_t g = 2; g < q; ++g) {
        int ok = 1;
        for (int i = 0; i < nf && ok; ++i)
            if (powmod(g, (q - 1) / f[i], q) == 1) ok = 0;
        if (ok) return g;
    }
    return 0;
}

/* psi = g^((q-1)/(2n)): a primitive 2n-th root of unity mod q. */
uint64_t oracle_psi(uint64_t q, uint32_t n)
{
    return powmod(oracle_primitive_root(q), (q - 1) / (2ull * n), q);
}

/* -------------------------------------------------------------- NTT / INTT */
static uint32_t bitrev(uint32_t x, int logn)
{
    uint32_t r = 0;
    for (int i = 0; i < logn; ++i) { r = (r << 1) | (x & 1); x >>= 1; }
    return r;
}

/* In-place cyclic DFT over Z_q of length n with root w (textbook iterative
 * radix-2 Cooley-Tukey: bit-reversal permutation, then log2(n) levels of
 * butterflies). Output in natural order: X_i = sum_j x_j w^(ij). */
static void cyclic_dft(uint64_t *x, uint32_t n, uint64_t w, uint64_t q)
{
    int logn = 0;
    while ((1u << logn) < n) ++logn;
    for (uint32_t i = 0; i < n; ++i) {
        uint32_t r = bitrev(i, logn);
        if (r > i) { uint64_t t = x[i]; x[i] = x[r]; x[r] = t; }
    }
    for (uint32_t len = 2; len <= n; len <<= 1) {
        uint64_t wl = powmod(w, n / len, q);
        for (uint32_t s = 0; s < n; s += len) {
            uint64_t wk = 1;
            for (uint32_t j = 0; j < len / 2; ++j) {
                uint64_t u = x[s + j];
                uint64_t v = mulmod(x[s + j + len / 2], wk, q);
                x[s + j] = (u + v) % q;
                x[s + j + len / 2] = (u + q - v) % q;
                wk = mulmod(wk, wl, q);
            }
        }
    }
}

/* Negacyclic forward NTT, natural order: out_i = sum_j a_j psi^((2i+1) j).
 * Written as b_j = a_j psi^j followed by a cyclic DFT with w = psi^2. */
void oracle_ntt_forward(uint64_t q, uint32_t n, uint64_t psi,
                        const uint32_t *a, uint32_t *out)
{
    uint64_t *x = (uint64_t *)malloc(sizeof(uint64_t) * n);
    uint64_t pj = 1;
    for (uint32_t j = 0; j < n; ++j) {
        x[j] = mulmod(a[j] % q, pj, q);
        pj = mulmod(pj, psi, q);
    }
    cyclic_dft(x, n, mulmod(psi, psi, q), q);
    for (uint32_t i = 0; i < n; ++i) out[i] = (uint32_t)x[i];
    free(x);
}

/* Inverse of oracle_ntt_forward: a_j = n^-1 psi^-j sum_i ahat_i w^(-ij). */
void oracle_ntt_inverse(uint64_t q, uint32_t n, uint64_t psi,
                        const uint32_t *ahat, uint32_t *out)
{
    uint64_t *x = (uint64_t *)malloc(sizeof(uint64_t) * n);
    for (uint32_t i = 0; i < n; ++i) x[i] = ahat[i] % q;
    uint64_t psi_inv = powmod(psi, q - 2, q);
    cyclic_dft(x, n, mulmod(psi_inv, psi_inv, q), q);
    uint64_t n_inv = powmod(n, q - 2, q);
    uint64_t pj = n_inv;
    for (uint32_t j = 0; j < n; ++j) {
        out[j] = (uint32_t)mulmod(x[j], pj, q);
        pj = mulmod(pj, psi_inv, q);
    }
    free(x);
}

/* Batched forward NTT over `count` contiguous length-n vectors (OpenMP). */
void oracle_ntt_forward_many(uint64_t q, uint32_t n, uint64_t psi, uint64_t count,
                             const uint32_t *a, uint32_t *out, uint64_t stride)
{
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < (int64_t)count; ++i)
        oracle_ntt_forward(q, n, psi, a + (uint64_t)i * stride, out + (uint64_t)i * stride);
}

/* Batched inverse NTT over `count` contiguous length-n vectors (OpenMP). */
void oracle_ntt_inverse_many(uint64_t q, uint32_t n, uint64_t psi, uint64_t count,
                             const uint32_t *ahat, uint32_t *out, uint64_t stride)
{
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < (int64_t)count; ++i)
        oracle_ntt_inverse(q, n, psi, ahat + (uint64_t)i * stride, out + (uint64_t)i * stride);
}

/* Schoolbook product in Z_q[X]/(X^n + 1): X^n = -1. */
void oracle_negacyclic_mul(uint64_t q, uint32_t n, const int64_t *a,
                           const int64_t *b, uint32_t *out)
{
    /* Signed inputs are reduced into [0, q) first. */
    uint64_t *acc = (uint64_t *)calloc(n, sizeof(uint64_t));
    for (uint32_t i = 0; i < n; ++i) {
        uint64_t ai = (uint64_t)(((a[i] % (int64_t)q) + (int64_t)q) % (int64_t)q);
        if (!ai) continue;
        for (uint32_t j = 0; j < n; ++j) {
            uint64_t bj = (uint64_t)(((b[j] % (int64_t)q) + (int64_t)q) % (int64_t)q);
            uint64_t p = mulmod(ai, bj, q);
            if (i + j < n) acc[i + j] = (acc[i + j] + p) % q;
            else           acc[i + j - n] = (acc[i + j - n] + q - p) % q;
        }
    }
    for (uint32_t i = 0; i < n; ++i) out[i] = (uint32_t)acc[i];
    free(acc);
}

/* ------------------------------------------------------------------ RowSel */
/* out[b][c][n][l][j] = ( sum_k query[b][c][k][l][j] * db[k][n][l][j] ) mod q_l
 * Exact: each product < 2^64, the sum is kept in 128 bits, one `%` at the end. */
void oracle_rowsel(uint32_t B, uint32_t D0, uint32_t D1, uint32_t L, uint32_t N,
                   const uint64_t *primes, const uint32_t *query,
                   const uint32_t *db, uint32_t *out)
{
    const uint64_t P = (uint64_t)L * N;
    #pragma omp parallel
    {
        u128 *acc = (u128 *)malloc(sizeof(u128) * P);
        #pragma omp for schedule(dynamic, 1) collapse(2)
        for (int64_t bc = 0; bc < (int64_t)B * 2; ++bc) {
            for (int64_t n = 0; n < (int64_t)D1; ++n) {
                memset(acc, 0, sizeof(u128) * P);
                for (uint64_t k = 0; k < D0; ++k) {
                    const uint32_t *qv = query + ((uint64_t)bc * D0 + k) * P;
                    const uint32_t *dv = db + ((uint64_t)k * D1 + (uint64_t)n) * P;
                    for (uint64_t p = 0; p < P; ++p)
                        acc[p] += (u128)((uint64_t)qv[p] * (uint64_t)dv[p]);
                }
                uint32_t *o = out + ((uint64_t)bc * D1 + (uint64_t)n) * P;
                for (uint64_t p = 0; p < P; ++p)
                    o[p] = (uint32_t)(acc[p] % primes[p / N]);
            }
        }
        free(acc);
    }
}

/* ------------------------------------------------------------ threading */
/* Threads the OpenMP loops above use (for timing the oracle on one core). */
void oracle_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int oracle_max_threads(void) { return omp_get_max_threads(); }
