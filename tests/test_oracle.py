"""Pins for the CPU oracle: each check compares it with something other than
itself -- a published generator vector, direct O(N^2) evaluation in Python
integers, exact integer convolution in numpy, Python big-integer matrix
products, closed forms and the selection semantics of RowSel (sec. 2.2)."""
import math
import os

import numpy as np
import pytest

import oracle
import oracle.rlwe as rlwe
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ generator
def test_splitmix64_published_vector():
    vals = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    assert [synth.draw_scalar(0, i) for i in range(3)] == vals
    assert [int(x) for x in synth.draw(0, [0, 1, 2])] == vals


def test_uniform_mod_is_exact_mulhi():
    key = synth.stream_key(9, synth.TAG_QUERY, 3)
    q = 1073692673
    got = synth.uniform_mod(key, np.arange(2000), q)
    want = [(synth.draw_scalar(key, i) * q) >> 64 for i in range(2000)]
    assert got.tolist() == want
    assert got.max() < q


# ---------------------------------------------------------------- primes / psi
def _trial_prime(n):
    if n < 2:
        return False
    d = 2
    while d * d <= n:
        if n % d == 0:
            return False
        d += 1
    return True


@pytest.mark.parametrize("n,bits,count,table", [(1024, 30, 1, synth.PRIME_N1024),
                                                (4096, 30, 2, synth.PRIMES_N4096),
                                                (4096, 27, 4, synth.PRIMES_Q108),
                                                (4096, 32, 2, synth.PRIMES_W32),
                                                (4096, 31, 2, synth.PRIMES_W31),
                                                (8, 32, 1, (synth.PRIME_W32_TOP_N8,))])
def test_primes_are_largest_ntt_friendly(n, bits, count, table):
    got = oracle.ntt_primes(n, bits, count)
    assert tuple(got) == tuple(table)
    # independent check: primality by trial division, q = 1 mod 2N, < 2^bits,
    # and no NTT-friendly prime skipped between them and 2^bits
    cands = [x for x in range((1 << bits) - 1, table[-1] - 1, -1) if x % (2 * n) == 1]
    primes = [x for x in cands if _trial_prime(x)]
    assert tuple(primes[:count]) == tuple(table)


def test_w32_sym_primes_are_largest_below_twice_digit_reach():
    # four balanced base-2^8 digits reach 127 * (1 + 2^8 + 2^16 + 2^24); the
    # table holds the two largest NTT-friendly primes at most twice that
    reach = 127 * (1 + 256 + 65536 + 16777216)
    top = 2 * reach
    table = synth.PRIMES_W32_SYM
    cands = [x for x in range(top, table[-1] - 1, -1) if x % 8192 == 1]
    primes = [x for x in cands if _trial_prime(x)]
    assert tuple(primes[:2]) == tuple(table)
    assert all((q - 1) // 2 <= reach for q in table)


def test_q108_primes_product():
    # the paper's modulus size: Q = q0 q1 q2 q3 of about 2^108 (sec. 2.4.1)
    Q = 1
    for q in synth.PRIMES_Q108:
        Q *= q
    assert 107.9 < math.log2(Q) < 108.1


@pytest.mark.parametrize("q,n", [(1073707009, 1024), (1073692673, 4096), (1073668097, 4096),
                                 (1073707009, 8), (1073707009, 64)])
def test_psi_primitive_2n_root(q, n):
    p = oracle.psi(q, n)
    assert pow(p, n, q) == q - 1           # psi^N = -1
    assert pow(p, 2 * n, q) == 1
    g = oracle.primitive_root(q)
    # g generates Z_q^*: g^((q-1)/f) != 1 for every prime factor f of q-1
    r, f, facs = q - 1, 2, []
    while f * f <= r:
        if r % f == 0:
            facs.append(f)
            while r % f == 0:
                r //= f
        f += 1
    if r > 1:
        facs.append(r)
    assert all(pow(g, (q - 1) // f, q) != 1 for f in facs)
    # and it is the smallest generator: every h in [2, g) fails for some factor
    assert all(any(pow(h, (q - 1) // f, q) == 1 for f in facs) for h in range(2, g))


def test_psi_values_table():
    # values derived in the hot-path scope analysis; re-derived here
    assert oracle.psi(1073707009, 1024) == 992735929
    assert oracle.psi(1073692673, 4096) == 510015274
    assert oracle.psi(1073668097, 4096) == 1047115509


# ----------------------------------------------------------------------- NTT
def _direct_ntt(a, q, psi, idx=None):
    n = len(a)
    idx = range(n) if idx is None else idx
    return [sum(int(a[j]) * pow(psi, (2 * i + 1) * j, q) for j in range(n)) % q for i in idx]


@pytest.mark.parametrize("n", [8, 64, 256])
def test_ntt_matches_direct_evaluation(n):
    q = 1073707009
    psi = oracle.psi(q, n)
    key = synth.stream_key(11, synth.TAG_QUERY, n)
    a = synth.uniform_mod(key, np.arange(n), q)
    assert oracle.ntt_forward(a, q, psi).tolist() == _direct_ntt(a, q, psi)


@pytest.mark.parametrize("q,n", [(1073707009, 1024), (1073692673, 4096), (133963777, 4096),
                                 (4294828033, 4096), (4294729729, 64)])
def test_ntt_matches_direct_evaluation_sampled(q, n):
    psi = oracle.psi(q, n)
    a = synth.uniform_mod(synth.stream_key(12, synth.TAG_QUERY), np.arange(n), q)
    got = oracle.ntt_forward(a, q, psi)
    idx = [0, 1, 2, n // 3, n // 2, n - 2, n - 1]
    assert [int(got[i]) for i in idx] == _direct_ntt(a, q, psi, idx)


@pytest.mark.parametrize("q,n", [(1073707009, 1024), (1073668097, 4096)])
def test_ntt_roundtrip_and_special_vectors(q, n):
    a = synth.uniform_mod(synth.stream_key(13, synth.TAG_QUERY), np.arange(n), q)
    assert np.array_equal(oracle.ntt_inverse(oracle.ntt_forward(a, q), q), a)
    one = np.zeros(n, dtype=np.uint32)
    one[0] = 1
    assert np.all(oracle.ntt_forward(one, q) == 1)          # NTT(1) = all ones
    x = np.zeros(n, dtype=np.uint32)
    x[1] = 1
    psi = oracle.psi(q, n)
    got = oracle.ntt_forward(x, q)                          # NTT(X)_i = psi^(2i+1)
    assert [int(got[i]) for i in (0, 1, n - 1)] == [pow(psi, 2 * i + 1, q) for i in (0, 1, n - 1)]


def _negacyclic_mod(a, b, q):
    n = len(a)
    full = np.convolve(np.asarray(a, dtype=object), np.asarray(b, dtype=object))
    res = list(full[:n])
    for i in range(n - 1):
        res[i] -= full[n + i]
    return [int(x) % q for x in res]


@pytest.mark.parametrize("n", [8, 64])
def test_convolution_theorem_against_schoolbook(n):
    q = 1073707009
    k = synth.stream_key(14, synth.TAG_QUERY, n)
    a = synth.uniform_mod(k, np.arange(n), q)
    b = synth.uniform_mod(k, np.arange(n, 2 * n), q)
    want = _negacyclic_mod(a, b, q)                     # Python big ints, no NTT
    assert oracle.negacyclic_mul(a.astype(np.int64), b.astype(np.int64), q).tolist() == want
    prod = (oracle.ntt_forward(a, q).astype(object) * oracle.ntt_forward(b, q).astype(object)) % q
    assert oracle.ntt_inverse(prod.astype(np.uint32), q).tolist() == want


# -------------------------------------------------------------------- RowSel
def _bigint_rowsel(Q, D, primes):
    B, _, D0, L, N = Q.shape
    D1 = D.shape[1]
    out = np.zeros((B, 2, D1, L, N), dtype=np.uint32)
    for l, q in enumerate(primes):
        for j in range(N):
            A = [[int(Q[b, c, k, l, j]) for k in range(D0)] for b in range(B) for c in range(2)]
            M = [[int(D[k, n, l, j]) for n in range(D1)] for k in range(D0)]
            for m, row in enumerate(A):
                for n in range(D1):
                    out[m // 2, m % 2, n, l, j] = sum(row[k] * M[k][n] for k in range(D0)) % q
    return out


def _rand(seed, shape, primes, tag=synth.TAG_QUERY):
    key = synth.stream_key(seed, tag)
    L = len(primes)
    x = np.empty(shape, dtype=np.uint32)
    idx = np.arange(int(np.prod(shape))).reshape(shape)
    for l, q in enumerate(primes):
        x[..., l, :] = synth.uniform_mod(key, idx[..., l, :], int(q))
    return x


P2 = synth.PRIMES_N4096


@pytest.mark.parametrize("primes", [P2, synth.PRIMES_W32], ids=["30bit", "32bit"])
def test_rowsel_matches_bigint_matmul(primes):
    Q = _rand(21, (3, 2, 5, 2, 8), primes)
    D = _rand(22, (5, 4, 2, 8), primes, synth.TAG_DB)
    assert np.array_equal(oracle.rowsel(Q, D, primes), _bigint_rowsel(Q, D, primes))


@pytest.mark.parametrize("primes", [P2, synth.PRIMES_W32], ids=["30bit", "32bit"])
def test_rowsel_all_q_minus_one_is_d0(primes):
    # (q-1)^2 = 1 mod q, so every output is D0 mod q (with 32-bit primes the
    # products are just below 2^64 and their sums far above)
    d0, d1, n = 37, 3, 16
    Q = np.empty((2, 2, d0, 2, n), dtype=np.uint32)
    D = np.empty((d0, d1, 2, n), dtype=np.uint32)
    for l, q in enumerate(primes):
        Q[..., l, :] = q - 1
        D[..., l, :] = q - 1
    out = oracle.rowsel(Q, D, primes)
    assert np.all(out == d0)


def test_rowsel_one_hot_selects_row():
    # noiseless selectors (delta_{k,i*} * NTT(1), 0): component 0 is row i*, component 1 is 0
    d0, d1, n, istar = 9, 5, 32, 6
    D = _rand(23, (d0, d1, 2, n), P2, synth.TAG_DB)
    Q = np.zeros((1, 2, d0, 2, n), dtype=np.uint32)
    Q[0, 0, istar] = 1
    out = oracle.rowsel(Q, D, P2)
    assert np.array_equal(out[0, 0], D[istar])
    assert np.all(out[0, 1] == 0)


def test_rowsel_linearity_split_independence_permutation():
    d0, d1, n = 12, 6, 16
    D = _rand(24, (d0, d1, 2, n), P2, synth.TAG_DB)
    Q1 = _rand(25, (2, 2, d0, 2, n), P2)
    Q2 = _rand(26, (2, 2, d0, 2, n), P2)
    alpha, beta = 12345, 987654321
    qv = np.array(P2, dtype=np.uint64)[None, None, None, :, None]
    comb = ((alpha * Q1.astype(np.uint64)) % qv + (beta * Q2.astype(np.uint64)) % qv) % qv
    lhs = oracle.rowsel(comb.astype(np.uint32), D, P2).astype(np.uint64)
    r1 = oracle.rowsel(Q1, D, P2).astype(np.uint64)
    r2 = oracle.rowsel(Q2, D, P2).astype(np.uint64)
    assert np.array_equal(lhs, ((alpha * r1) % qv + (beta * r2) % qv) % qv)
    # k-split additivity
    h = 5
    a = oracle.rowsel(np.ascontiguousarray(Q1[:, :, :h]), np.ascontiguousarray(D[:h]), P2)
    b = oracle.rowsel(np.ascontiguousarray(Q1[:, :, h:]), np.ascontiguousarray(D[h:]), P2)
    assert np.array_equal((a.astype(np.uint64) + b) % qv, r1)
    # client independence
    for bi in range(2):
        assert np.array_equal(oracle.rowsel(np.ascontiguousarray(Q1[bi:bi + 1]), D, P2)[0], r1[bi])
    # k-permutation invariance
    perm = np.random.RandomState(0).permutation(d0)
    assert np.array_equal(oracle.rowsel(np.ascontiguousarray(Q1[:, :, perm]),
                                        np.ascontiguousarray(D[perm]), P2), r1)
    # zero query -> zero output
    assert not oracle.rowsel(np.zeros_like(Q1), D, P2).any()


def test_rowsel_coefficient_domain_semantics():
    # INTT(out[b][c][n]) = sum_k ct_{b,c,k} * d_{k,n} in Z_q[X]/(X^N+1), brute force
    n, d0, d1 = 16, 3, 2
    q = 1073707009
    key = synth.stream_key(27, synth.TAG_DB)
    dco = synth.bits16(key, np.arange(d0 * d1 * n)).reshape(d0, d1, 1, n)
    ct = synth.uniform_mod(synth.stream_key(27, synth.TAG_QUERY), np.arange(2 * d0 * n), q) \
        .reshape(1, 2, d0, 1, n)
    Dhat = oracle.ntt_forward(dco, q)
    Qhat = oracle.ntt_forward(ct, q)
    out = oracle.rowsel(Qhat, Dhat, [q])
    for c in range(2):
        for col in range(d1):
            want = [0] * n
            for k in range(d0):
                term = _negacyclic_mod(ct[0, c, k, 0], dco[k, col, 0], q)
                want = [(x + y) % q for x, y in zip(want, term)]
            assert oracle.ntt_inverse(out[0, c, col, 0], q).tolist() == want


# ------------------------------------------------------------- toy RLWE
def test_toy_rlwe_tiny_config_recovers_row():
    w = synth.TINY
    d0, d1, n = w.d0, w.d1, w.n
    istar = synth.selected_row(w.seed, d0)
    coeffs = synth.db_coeffs(w.dbseed, d0, d1, 1, n)            # [D0][D1][1][N]
    Dhat = oracle.ntt_db(coeffs, w.primes)
    Q, s, e = rlwe.encrypt_selectors(w.seed, n, w.primes, d0, istar, t=1 << 16)
    out = oracle.rowsel(Q, Dhat, w.primes)
    rec = rlwe.decrypt_known_noise(out[0], s, e, coeffs[:, :, 0, :], w.primes, 1 << 16)
    assert np.array_equal(rec[:, 0, :], coeffs[istar, :, 0, :])


def test_toy_rlwe_rounding_decrypt_small_plaintext():
    # t = 2^8: the noise stays below Delta/2, so honest rounding decrypts
    n, d0, d1, t = 1024, 16, 3, 1 << 8
    primes = synth.PRIME_N1024
    coeffs = (synth.bits16(synth.stream_key(31, synth.TAG_DB), np.arange(d0 * d1 * n)) % t) \
        .reshape(d0, d1, 1, n).astype(np.uint32)
    istar = 11
    Dhat = oracle.ntt_db(coeffs, primes)
    Q, s, e = rlwe.encrypt_selectors(31, n, primes, d0, istar, t)
    out = oracle.rowsel(Q, Dhat, primes)
    assert np.array_equal(rlwe.decrypt_round(out[0], s, primes, t), coeffs[istar, :, 0, :])


@pytest.mark.slow
def test_toy_rlwe_two_prime_crt_decrypt():
    # N = 4096 with both primes: Delta = floor(q0 q1 / 2^16) ~ 2^44 >> noise
    n, d0, d1, t = 4096, 4, 2, 1 << 16
    primes = synth.PRIMES_N4096
    coeffs = synth.db_coeffs(32, d0, d1, 2, n)
    istar = 2
    Dhat = oracle.ntt_db(coeffs, primes)
    Q, s, e = rlwe.encrypt_selectors(32, n, primes, d0, istar, t)
    out = oracle.rowsel(Q, Dhat, primes)
    assert np.array_equal(rlwe.decrypt_round(out[0], s, primes, t), coeffs[istar, :, 0, :])
