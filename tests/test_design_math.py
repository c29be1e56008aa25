"""CPU checks of the number theory the GPU kernels rely on, written out in
Python integers (no GPU, no library code): the INT8 digit window that lets the
MFMA path take every prime below 2^32, the short reconstruction form of the
ColTor decomposition (against the oracle's decomposition), and the growth
bound of the unreduced forward butterflies (against the oracle's NTT)."""
import random

import numpy as np
import pytest

import oracle
import synth
from oracle import coltor

LOW, HIGH = -0x80808080, 0x7F7F7F7F      # reach of four balanced signed 8-bit digits


def balanced_digits(x):
    d = []
    for _ in range(4):
        di = ((x + 128) & 255) - 128
        d.append(di)
        x = (x - di) >> 8
    assert x == 0
    return d


@pytest.mark.parametrize("q", [3, 1073692673, synth.PRIMES_W31[0], synth.PRIMES_W32_SYM[0],
                               synth.PRIMES_W32[0], synth.PRIME_W32_TOP_N8, 4294967291])
def test_digit_window_covers_every_residue(q):
    # r <= HIGH is taken as is, r > HIGH as r - q: the reach holds 2^32 - 1
    # consecutive integers, so every residue class of a q < 2^32 lands in it
    rng = random.Random(q)
    rs = {0, 1, q - 1, q // 2, (q + 1) // 2, min(HIGH, q - 1), min(HIGH + 1, q - 1)}
    rs |= {rng.randrange(q) for _ in range(3000)}
    for r in rs:
        x = r - q if r > HIGH else r
        assert LOW <= x <= HIGH and (x - r) % q == 0
        d = balanced_digits(x)
        assert all(-128 <= v <= 127 for v in d)
        assert sum(v << (8 * i) for i, v in enumerate(d)) == x


def short_form(xs, primes, log2z, ell):
    """The decomposition's short form on 32-bit words: y_l = x_l (Q/q_l)^-1 mod
    q_l; S = sum y_l Q/q_l mod 2^128; k = floor(sum y_l / q_l) in binary64;
    one correction either way; then the bit fields of v + C, C = sum over
    i < ell-1 of (z/2) z^i."""
    M = (1 << 128) - 1
    Q = coltor.modulus(primes)
    z = 1 << log2z
    C = sum((z // 2) * z ** i for i in range(ell - 1))
    S, fk = 0, 0.0
    for x, q in zip(xs, primes):
        y = x * pow(Q // q % q, -1, q) % q
        fk += float(y) * (1.0 / q)
        S = (S + y * (Q // q)) & M
    v = (S - int(fk) * Q) & M
    if v >> 127:
        v = (v + Q) & M
    elif v >= Q:
        v = (v - Q) & M
    v = (v + ((C - Q) if v > Q // 2 else C)) & M
    w = [(v >> (32 * i)) & 0xFFFFFFFF for i in range(4)]
    out = []
    for _ in range(ell - 1):
        out.append((w[0] & (z - 1)) - z // 2)
        top = w[3] - (1 << 32) if w[3] >> 31 else w[3]
        w = [((w[1] << 32 | w[0]) >> log2z) & 0xFFFFFFFF, ((w[2] << 32 | w[1]) >> log2z) & 0xFFFFFFFF,
             ((w[3] << 32 | w[2]) >> log2z) & 0xFFFFFFFF, (top >> log2z) & 0xFFFFFFFF]
    out.append(w[0] - (1 << 32) if w[0] >> 31 else w[0])
    return out


@pytest.mark.parametrize("primes,log2z,ell", [(synth.PRIMES_Q108, 22, 5), (synth.PRIMES_Q108, 25, 5),
                                              (synth.PRIMES_N4096, 20, 3), (synth.PRIMES_W32, 22, 3),
                                              ((synth.PRIME_W32_TOP_N8,), 17, 2)])
def test_short_reconstruction_equals_oracle_digits(primes, log2z, ell):
    Q = coltor.modulus(primes)
    assert Q < 2 ** 125 and log2z * ell <= 126          # where the kernels take the short form
    rng = random.Random(log2z * ell)
    z = 1 << log2z
    xs = [0, 1, Q - 1, Q // 2, Q // 2 + 1, z // 2, Q - z // 2] + [rng.randrange(Q) for _ in range(3000)]
    want = coltor.decompose(np.array(xs, dtype=object), Q, log2z, ell)
    for j, X in enumerate(xs):
        got = short_form([X % q for q in primes], primes, log2z, ell)
        assert got == [int(v) for v in want[:, j]], X


def test_unreduced_forward_butterflies_stay_bounded():
    # (x, y) -> (x + t, x - t + 2q) with t = Shoup's uncorrected product of y in
    # [0, 2q): after s stages every value is below q (1 + 2s), so logN stages
    # fit 32 bits when (1 + 2 logN) q < 2^32; the result is the NTT mod q
    q, n = synth.PRIMES_Q108[0], 256
    logn = n.bit_length() - 1
    assert (1 + 2 * logn) * q < 2 ** 32
    psi = oracle.psi(q, n)
    brev = lambda x: int(format(x, f"0{logn}b")[::-1], 2)
    tw = [pow(psi, brev(k), q) for k in range(n)]
    rng = random.Random(3)
    a = [rng.randrange(q) for _ in range(n)]
    v = list(a)
    m, t = 1, n // 2
    stage = 0
    while m < n:
        for i in range(m):
            w = tw[m + i]
            ws = (w << 32) // q
            for j in range(2 * i * t, 2 * i * t + t):
                x, y = v[j], v[j + t]
                tt = (y * w - ((y * ws) >> 32) * q) & 0xFFFFFFFF
                assert tt < 2 * q
                v[j], v[j + t] = x + tt, x - tt + 2 * q
        stage += 1
        assert max(v) < q * (1 + 2 * stage)
        m, t = 2 * m, t // 2
    out = [0] * n
    for e in range(n):
        out[brev(e)] = v[e] % q
    assert out == oracle.ntt_forward(np.array(a, dtype=np.uint32), q).tolist()
