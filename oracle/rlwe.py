"""Toy RLWE encryption of one-hot row selectors -- TEST INFRASTRUCTURE ONLY.

RowSel's selection semantics (paper sec. 2.2, RowSel): of the D0 selector
ciphertexts, all encrypt zero except the i*-th, which encrypts one; the
product with the DB then yields an encryption of row i*.  The paper names
BFV but prints no encryption formulas, so this module takes the usual
BFV-style reading, entirely in the NTT domain:

  * secret s: ternary coefficients; shat_l = NTT_l(s mod q_l)
  * selector k: ahat_k uniform mod q_l (drawn directly in the NTT domain),
    error e_k rounded Gaussian (sigma 3.2, cut at 6 sigma),
    component 0 = ahat_k,
    component 1 = -ahat_k (.) shat + NTT(e_k) + Delta * NTT(m_k),
    with m_k the constant polynomial delta_{k,i*}, whose NTT is the all-ones
    vector, and Delta = floor(Q / t) reduced mod each q_l (Q = prod q_l).
  * decryption of an output pair (A, B): phi = B + A (.) shat, then INTT:
    phi = sum_k e_k * d_k + Delta * d_{i*}  (mod Q, negacyclic products).

Two decryptions are offered:
  * ``decrypt_known_noise``: subtract the harness-known noise sum_k e_k * d_k
    (exact integer negacyclic convolution, numpy) and multiply by Delta^-1;
    exact whatever the noise size.
  * ``decrypt_round``: CRT-reconstruct phi and round phi * t / Q; exact only
    while the noise stays below Delta / 2.
"""
from __future__ import annotations

import numpy as np

import synth

from . import ntt_forward, ntt_inverse

SIGMA = 3.2
TAIL = 19


def secret(seed: int, n: int) -> np.ndarray:
    return synth.ternary(synth.stream_key(seed, synth.TAG_SECRET), np.arange(n))


def errors(seed: int, d0: int, n: int) -> np.ndarray:
    e = synth.gaussian_int(synth.stream_key(seed, synth.TAG_ERROR), np.arange(d0 * n),
                           SIGMA, TAIL)
    return e.reshape(d0, n)


def _mod(x: np.ndarray, q: int) -> np.ndarray:
    return np.mod(x, q).astype(np.uint32)


def delta(primes, t: int) -> int:
    Q = 1
    for q in primes:
        Q *= int(q)
    return Q // t


def encrypt_selectors(seed: int, n: int, primes, d0: int, i_star: int, t: int):
    """One client's D0 selector ciphertexts, layout [1][2][D0][L][N]."""
    L = len(primes)
    s = secret(seed, n)
    e = errors(seed, d0, n)
    dl = delta(primes, t)
    keyA = synth.stream_key(seed, synth.TAG_A)
    out = np.empty((1, 2, d0, L, n), dtype=np.uint32)
    for l, q in enumerate(primes):
        q = int(q)
        shat = ntt_forward(_mod(s, q), q).astype(np.uint64)
        ehat = ntt_forward(_mod(e, q), q).astype(np.uint64)          # [D0][N]
        idx = (np.arange(d0, dtype=np.uint64)[:, None] * np.uint64(L) + np.uint64(l)) \
            * np.uint64(n) + np.arange(n, dtype=np.uint64)[None, :]
        ahat = synth.uniform_mod(keyA, idx, q).astype(np.uint64)      # [D0][N]
        m = np.zeros((d0, 1), dtype=np.uint64)
        m[i_star, 0] = (dl % q)
        body = (q - (ahat * shat) % np.uint64(q)) % np.uint64(q)
        body = (body + ehat + m) % np.uint64(q)
        out[0, 0, :, l, :] = ahat.astype(np.uint32)
        out[0, 1, :, l, :] = body.astype(np.uint32)
    return out, s, e


def phase(out_ct: np.ndarray, s: np.ndarray, primes) -> np.ndarray:
    """phi = INTT(B + A (.) shat) per prime, for output ciphertexts [2][D1][L][N]."""
    _, d1, L, n = out_ct.shape
    phi = np.empty((d1, L, n), dtype=np.uint32)
    for l, q in enumerate(primes):
        q = int(q)
        shat = ntt_forward(_mod(s, q), q).astype(np.uint64)
        A = out_ct[0, :, l, :].astype(np.uint64)
        Bp = out_ct[1, :, l, :].astype(np.uint64)
        ph = (Bp + (A * shat) % np.uint64(q)) % np.uint64(q)
        phi[:, l, :] = ntt_inverse(ph.astype(np.uint32), q)
    return phi


def negacyclic_int(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Exact integer product in Z[X]/(X^N + 1) (int64, no modulus)."""
    n = a.shape[0]
    full = np.convolve(a.astype(np.int64), b.astype(np.int64))   # length 2N-1
    res = full[:n].copy()
    res[: n - 1] -= full[n:]
    return res


def decrypt_known_noise(out_ct, s, e, db_coeffs_cols, primes, t):
    """Recover row i* of the DB from RowSel output [2][D1][L][N].

    ``db_coeffs_cols`` is the coefficient-domain DB [D0][D1][N] (small, < t)."""
    phi = phase(out_ct, s, primes)
    d0, d1, n = db_coeffs_cols.shape
    dl = delta(primes, t)
    rec = np.empty((d1, len(primes), n), dtype=np.uint32)
    for c in range(d1):
        noise = np.zeros(n, dtype=np.int64)
        for k in range(d0):
            noise += negacyclic_int(e[k], db_coeffs_cols[k, c])
        for l, q in enumerate(primes):
            q = int(q)
            x = (phi[c, l].astype(np.int64) - noise) % q
            dinv = pow(dl % q, -1, q)
            rec[c, l] = ((x.astype(object) * dinv) % q).astype(np.uint32)
    return rec


def decrypt_round(out_ct, s, primes, t):
    """Honest BFV-style decryption by CRT reconstruction and rounding."""
    phi = phase(out_ct, s, primes)
    d1, L, n = phi.shape
    Q = 1
    for q in primes:
        Q *= int(q)
    res = np.empty((d1, n), dtype=np.int64)
    # CRT: x = sum_l phi_l * (Q/q_l) * ((Q/q_l)^-1 mod q_l)  mod Q  (Python ints)
    basis = []
    for q in primes:
        q = int(q)
        Ml = Q // q
        basis.append(Ml * pow(Ml % q, -1, q))
    for c in range(d1):
        for j in range(n):
            x = 0
            for l in range(L):
                x += int(phi[c, l, j]) * basis[l]
            x %= Q
            res[c, j] = ((x * t + Q // 2) // Q) % t
    return res
