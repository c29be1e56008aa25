"""CPU oracle for the first ColTor stage -- TEST INFRASTRUCTURE ONLY.

Plain and slow: Python integers for every value mod Q, the library NTT of
``oracle`` (its own C code) for the transforms, no blocking or fusion.

What it follows:
  * ColTor (sec. 2.2): a binary tournament over the D1 RowSel output
    ciphertexts; each node takes two ciphertexts and returns one by an
    external product with the stage's RGSW ciphertext.  A node is read as the
    usual selector, out = ct0 + RGSW(bit) [x] (ct1 - ct0), so a bit of 0 keeps
    column 2t and a bit of 1 takes column 2t + 1; an unpaired last column
    (odd count) passes through.
  * The external product (sec. 2.4.2, Dcp): both polynomials of the input
    ciphertext are brought to the coefficient domain (inverse NTT), each
    coefficient is rebuilt from its L residues (RNS reconstruction, a value in
    [0, Q)), decomposed into ell digits of base z = 2^log2z, each digit
    polynomial goes back to the NTT domain limb by limb, and the 2*ell digit
    polynomials multiply-accumulate against the RGSW rows into two
    polynomials.
  * Digits: the value is centred into (-Q/2, Q/2]; digits 0 .. ell-2 are
    balanced in [-z/2, z/2) and digit ell-1 takes the rest, which stays within
    [-z/2, z/2 + 1] when z^ell > Q (the range sec. 2.4.2 gives).

Layouts (NTT domain, residues < q_l, limb-major polynomials [L][N]):
  ciphertexts ``[B][2][ncols][L][N]`` (the RowSel output layout),
  RGSW        ``[B][2][ell][2][L][N]``: row (p, i) is the RLWE pair that
              multiplies digit i of input polynomial p,
  output      ``[B][2][(ncols + 1) // 2][L][N]``.
"""
from __future__ import annotations

import numpy as np

from . import ntt_forward, ntt_inverse


def modulus(primes) -> int:
    Q = 1
    for q in primes:
        Q *= int(q)
    return Q


def crt(res: np.ndarray, primes) -> np.ndarray:
    """RNS reconstruction: res[..., l] are residues mod q_l; returns the unique
    x in [0, Q) with x = res[..., l] (mod q_l), as Python ints (object array).
    The textbook sum x = sum_l (r_l * (Q/q_l)^-1 mod q_l) * (Q/q_l) mod Q."""
    primes = [int(q) for q in primes]
    Q = modulus(primes)
    out = np.zeros(res.shape[:-1], dtype=object)
    for l, q in enumerate(primes):
        m = Q // q
        c = pow(m, -1, q)
        out = out + (res[..., l].astype(object) * c % q) * m
    return out % Q


def decompose(x: np.ndarray, Q: int, log2z: int, ell: int) -> np.ndarray:
    """Digits of x in [0, Q) (object array): returns int64 digits [ell][...]
    with sum_i d_i z^i = x - Q if x > Q/2 else x."""
    z = 1 << log2z
    v = np.where(x > Q // 2, x - Q, x)
    digits = []
    for i in range(ell - 1):
        d = (v + z // 2) % z - z // 2          # Python ints: % is floor-mod
        digits.append(d)
        v = (v - d) // z
    digits.append(v)
    return np.array([np.asarray(d, dtype=object).astype(np.int64) for d in digits])


def gadget_check(primes, log2z: int, ell: int) -> None:
    Q = modulus(primes)
    if not (1 <= ell <= 8 and 1 <= log2z <= 30):
        raise ValueError("gadget out of range")
    if (1 << (log2z * ell)) <= Q:
        raise ValueError("z^ell must exceed Q")
    if (1 << (log2z - 1)) + 1 >= min(int(q) for q in primes):
        raise ValueError("digits must stay below every prime")


def external_product(ct: np.ndarray, rgsw: np.ndarray, primes, log2z: int, ell: int) -> np.ndarray:
    """ct [2][L][N] (NTT domain) and rgsw [2][ell][2][L][N] -> [2][L][N]."""
    primes = [int(q) for q in primes]
    L, n = ct.shape[1], ct.shape[2]
    Q = modulus(primes)
    coef = np.stack([np.stack([ntt_inverse(ct[p, l], primes[l]) for l in range(L)], axis=-1)
                     for p in range(2)])                                   # [2][N][L]
    digits = np.stack([decompose(crt(coef[p], primes), Q, log2z, ell) for p in range(2)])  # [2][ell][N]
    out = [[0] * L for _ in range(2)]
    for l, q in enumerate(primes):
        acc = [np.zeros(n, dtype=object) for _ in range(2)]
        for p in range(2):
            for i in range(ell):
                dhat = ntt_forward((digits[p, i] % q).astype(np.uint32), q).astype(object)
                for c in range(2):
                    acc[c] = acc[c] + dhat * rgsw[p, i, c, l].astype(object)
        for c in range(2):
            out[c][l] = (acc[c] % q).astype(np.uint32)
    return np.array([[out[c][l] for l in range(L)] for c in range(2)], dtype=np.uint32)


def cmux(ct0: np.ndarray, ct1: np.ndarray, rgsw: np.ndarray, primes, log2z: int, ell: int) -> np.ndarray:
    """ct0 + RGSW [x] (ct1 - ct0), residue by residue mod q_l."""
    qs = np.array([int(q) for q in primes], dtype=np.int64)[None, :, None]
    diff = ((ct1.astype(np.int64) - ct0.astype(np.int64)) % qs).astype(np.uint32)
    ext = external_product(diff, rgsw, primes, log2z, ell)
    return ((ct0.astype(np.int64) + ext.astype(np.int64)) % qs).astype(np.uint32)


def coltor_stage(cts: np.ndarray, rgsw: np.ndarray, primes, log2z: int, ell: int) -> np.ndarray:
    """One tournament stage: cts [B][2][ncols][L][N], rgsw [B][2][ell][2][L][N]
    -> [B][2][(ncols + 1) // 2][L][N]."""
    gadget_check(primes, log2z, ell)
    B, _, ncols, L, n = cts.shape
    nout = (ncols + 1) // 2
    out = np.empty((B, 2, nout, L, n), dtype=np.uint32)
    for b in range(B):
        for t in range(nout):
            ct0 = cts[b, :, 2 * t]
            if 2 * t + 1 < ncols:
                out[b, :, t] = cmux(ct0, cts[b, :, 2 * t + 1], rgsw[b], primes, log2z, ell)
            else:
                out[b, :, t] = ct0
    return out


def trivial_rgsw(m: int, primes, n: int, log2z: int, ell: int) -> np.ndarray:
    """The noiseless RGSW of the constant m: row (p, i) has m z^i in component
    p and 0 in the other (NTT of a constant is that constant in every slot)."""
    L = len(primes)
    g = np.zeros((2, ell, 2, L, n), dtype=np.uint32)
    for p in range(2):
        for i in range(ell):
            for l, q in enumerate(primes):
                g[p, i, p, l, :] = (m * pow(2, log2z * i, int(q))) % int(q)
    return g
