/* Drives the CPU oracle (oracle/oracle.c, linked in) through each of its
 * functions on small inputs, for the AddressSanitizer / UndefinedBehavior-
 * Sanitizer build of the CPU test suite.  Exit status 0 when every result
 * checks (INTT(NTT(a)) = a, NTT(1) = all ones, RowSel of one-hot selectors
 * returns the selected row, the schoolbook product against X^i * X^j). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_is_prime(uint64_t n);
uint32_t oracle_ntt_primes(uint32_t n, uint32_t bits, uint32_t count, uint64_t *out);
uint64_t oracle_psi(uint64_t q, uint32_t n);
void oracle_ntt_forward_many(uint64_t q, uint32_t n, uint64_t psi, uint64_t count, const uint32_t *a,
                             uint32_t *out, uint64_t stride);
void oracle_ntt_inverse_many(uint64_t q, uint32_t n, uint64_t psi, uint64_t count, const uint32_t *a,
                             uint32_t *out, uint64_t stride);
void oracle_negacyclic_mul(uint64_t q, uint32_t n, const int64_t *a, const int64_t *b, uint32_t *out);
void oracle_rowsel(uint32_t B, uint32_t D0, uint32_t D1, uint32_t L, uint32_t N, const uint64_t *primes,
                   const uint32_t *query, const uint32_t *db, uint32_t *out);

#define CHECK(c, msg) do { if (!(c)) { fprintf(stderr, "FAIL: %s\n", msg); return 1; } } while (0)

int main(void)
{
    static const uint32_t ns[] = {8, 64, 1024};
    for (int t = 0; t < 3; ++t) {
        const uint32_t n = ns[t];
        uint64_t qs[2];
        CHECK(oracle_ntt_primes(n, 30, 2, qs) == 2, "two primes");
        for (int l = 0; l < 2; ++l) {
            CHECK(oracle_is_prime(qs[l]) && qs[l] % (2 * n) == 1, "prime = 1 mod 2n");
            const uint64_t psi = oracle_psi(qs[l], n);
            uint32_t *a = malloc(3 * n * sizeof(uint32_t)), *f = malloc(3 * n * sizeof(uint32_t)),
                     *b = malloc(3 * n * sizeof(uint32_t));
            for (uint32_t i = 0; i < 3 * n; ++i) a[i] = (uint32_t)((i * 2654435761u) % qs[l]);
            for (uint32_t i = 0; i < n; ++i) a[i] = i == 0;   /* the constant 1 */
            oracle_ntt_forward_many(qs[l], n, psi, 3, a, f, n);
            for (uint32_t i = 0; i < n; ++i) CHECK(f[i] == 1, "NTT(1) = all ones");
            oracle_ntt_inverse_many(qs[l], n, psi, 3, f, b, n);
            for (uint32_t i = 0; i < 3 * n; ++i) CHECK(a[i] == b[i], "INTT(NTT(a)) = a");
            free(a); free(f); free(b);
        }
        /* X^i * X^j = +-X^((i+j) mod n) */
        int64_t *x = calloc(n, sizeof(int64_t)), *y = calloc(n, sizeof(int64_t));
        uint32_t *o = malloc(n * sizeof(uint32_t));
        const uint32_t i = n - 3, j = 5;
        x[i] = 1;
        y[j] = 1;
        oracle_negacyclic_mul(qs[0], n, x, y, o);
        for (uint32_t k = 0; k < n; ++k)
            CHECK(o[k] == (k == (i + j) % n ? (uint32_t)(qs[0] - 1) : 0u), "negacyclic X^i X^j");
        free(x); free(y); free(o);
        /* RowSel with one-hot selectors (all ones in the NTT domain) picks row r */
        const uint32_t B = 2, D0 = 5, D1 = 3, L = 2, r = 3;
        const uint64_t P = (uint64_t)L * n;
        uint32_t *q = calloc((size_t)B * 2 * D0 * P, sizeof(uint32_t)), *db = malloc((size_t)D0 * D1 * P * 4),
                 *out = malloc((size_t)B * 2 * D1 * P * 4);
        for (uint64_t e = 0; e < (uint64_t)D0 * D1 * P; ++e) db[e] = (uint32_t)((e * 40503u) % qs[(e / n) % L]);
        for (uint32_t b2 = 0; b2 < B; ++b2)
            for (uint64_t p = 0; p < P; ++p) q[((uint64_t)(b2 * 2) * D0 + r) * P + p] = 1;
        oracle_rowsel(B, D0, D1, L, n, qs, q, db, out);
        for (uint32_t b2 = 0; b2 < B; ++b2)
            for (uint32_t c = 0; c < 2; ++c)
                for (uint32_t col = 0; col < D1; ++col)
                    for (uint64_t p = 0; p < P; ++p) {
                        const uint32_t got = out[(((uint64_t)b2 * 2 + c) * D1 + col) * P + p];
                        const uint32_t want = c ? 0u : db[((uint64_t)r * D1 + col) * P + p];
                        CHECK(got == want, "one-hot RowSel");
                    }
        free(q); free(db); free(out);
    }
    printf("oracle driver ok\n");
    return 0;
}
