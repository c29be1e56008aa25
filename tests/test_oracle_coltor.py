"""Pins of the ColTor oracle (oracle/coltor.py) against what the mathematics
fixes, independent of the oracle's own formulas:
  * RNS reconstruction: brute force over [0, Q) for tiny primes, and the
    defining congruences for the four-limb modulus;
  * Dcp: the digits sum back to the centred value, stay in range, and special
    values have known digits;
  * the external product with a noiseless RGSW of m multiplies the
    ciphertext by m (closed form), so the selector returns column 2t for a bit
    of 0 and 2t + 1 for a bit of 1;
  * the NTT-domain external product equals schoolbook negacyclic products of
    the digit polynomials with the RGSW rows in the coefficient domain;
  * with a real RGSW encryption of the bit under a ternary secret, the
    stage's output decrypts to the selected column's message (sec. 2.2).
"""
import itertools

import numpy as np
import pytest

import oracle
import synth
from oracle import coltor, rlwe

Q108 = synth.PRIMES_Q108


def _rand_res(seed, shape, primes):
    """Residues uniform mod q_l along a trailing limb axis."""
    out = np.empty(shape + (len(primes),), dtype=np.uint32)
    for l, q in enumerate(primes):
        key = synth.stream_key(seed, synth.TAG_QUERY, l)
        out[..., l] = synth.uniform_mod(key, np.arange(int(np.prod(shape))), q).reshape(shape)
    return out


def test_crt_brute_force_tiny_primes():
    primes = (17, 97, 113)
    Q = 17 * 97 * 113
    xs = np.arange(Q)
    res = np.stack([xs % q for q in primes], axis=-1).astype(np.uint32)
    got = coltor.crt(res, primes)
    assert [int(v) for v in got] == list(range(Q))


def test_crt_four_limbs_congruences():
    res = _rand_res(200, (3000,), Q108)
    x = coltor.crt(res, Q108)
    Q = coltor.modulus(Q108)
    for j in range(0, 3000, 7):
        v = int(x[j])
        assert 0 <= v < Q
        assert all(v % q == int(res[j, l]) for l, q in enumerate(Q108))


@pytest.mark.parametrize("log2z,ell", [(22, 5), (20, 6), (28, 4)])
def test_decompose_sums_back_and_stays_in_range(log2z, ell):
    Q = coltor.modulus(Q108)
    z = 1 << log2z
    rng = np.random.default_rng(5)
    xs = [0, 1, Q - 1, Q // 2, Q // 2 + 1, z // 2, z // 2 - 1, Q - z // 2]
    xs += [int.from_bytes(rng.bytes(14), "little") % Q for _ in range(4000)]
    x = np.array(xs, dtype=object)
    d = coltor.decompose(x, Q, log2z, ell)
    for j, v in enumerate(xs):
        centred = v - Q if v > Q // 2 else v
        assert sum(int(d[i, j]) << (log2z * i) for i in range(ell)) == centred
        assert all(-z // 2 <= int(d[i, j]) < z // 2 for i in range(ell - 1))
        assert -z // 2 <= int(d[ell - 1, j]) <= z // 2 + 1
    # Q - 1 is -1: digit 0 is -1 and the rest vanish
    assert [int(d[i, 2]) for i in range(ell)] == [-1] + [0] * (ell - 1)


def test_gadget_check_rejects():
    with pytest.raises(ValueError):
        coltor.gadget_check(Q108, 22, 4)          # 2^88 < Q
    with pytest.raises(ValueError):
        coltor.gadget_check(Q108, 30, 4)          # digits up to 2^29 + 1 exceed 27-bit primes
    coltor.gadget_check(Q108, 22, 5)
    coltor.gadget_check((1073692673,), 30, 2)


def _random_ct(seed, primes, n, count=1):
    L = len(primes)
    ct = _rand_res(seed, (count, 2, n), primes)          # [count][2][N][L]
    return np.ascontiguousarray(np.moveaxis(ct, -1, -2))  # [count][2][L][N]


@pytest.mark.parametrize("primes,log2z,ell,n", [(Q108, 22, 5, 16), (synth.PRIMES_N4096, 20, 3, 64),
                                                (synth.PRIMES_W32, 26, 3, 8)])
@pytest.mark.parametrize("m", [0, 1, 5])
def test_external_product_trivial_rgsw_scales(primes, log2z, ell, n, m):
    ct = _random_ct(210 + m, primes, n)[0]
    g = coltor.trivial_rgsw(m, primes, n, log2z, ell)
    got = coltor.external_product(ct, g, primes, log2z, ell)
    qs = np.array(primes, dtype=object)[None, :, None]
    want = (ct.astype(object) * m) % qs
    assert np.array_equal(got.astype(object), want)


def test_selector_with_trivial_rgsw_picks_columns():
    primes, log2z, ell, n = Q108, 22, 5, 16
    B, ncols = 2, 5
    cts = np.stack([np.moveaxis(_random_ct(220 + b, primes, n, ncols), 0, 1) for b in range(B)])  # [B][2][ncols][L][N]
    bits = [0, 1]
    rg = np.stack([coltor.trivial_rgsw(bits[b], primes, n, log2z, ell) for b in range(B)])
    out = coltor.coltor_stage(cts, rg, primes, log2z, ell)
    assert out.shape == (B, 2, 3, len(primes), n)
    for b in range(B):
        for t in range(2):
            assert np.array_equal(out[b, :, t], cts[b, :, 2 * t + bits[b]])
        assert np.array_equal(out[b, :, 2], cts[b, :, 4])   # unpaired column passes through


def test_external_product_equals_coefficient_domain_schoolbook():
    # ct and RGSW drawn in the coefficient domain; the expected value decomposes
    # the coefficients directly and multiplies in Z_q[X]/(X^N + 1) by schoolbook
    primes, log2z, ell, n = Q108, 22, 5, 8
    L = len(primes)
    Q = coltor.modulus(primes)
    c_coef = _rand_res(230, (2, n), primes)                        # [2][N][L]
    r_coef = _rand_res(231, (2, ell, 2, n), primes)                # [2][ell][2][N][L]
    want = np.zeros((2, L, n), dtype=np.uint32)
    digits = [coltor.decompose(coltor.crt(c_coef[p], primes), Q, log2z, ell) for p in range(2)]
    for c, l in itertools.product(range(2), range(L)):
        q = int(primes[l])
        acc = np.zeros(n, dtype=object)
        for p, i in itertools.product(range(2), range(ell)):
            a = [int(v) % q for v in digits[p][i]]
            b = [int(v) for v in r_coef[p, i, c, :, l]]
            for u in range(n):
                for v in range(n):
                    k = u + v
                    term = a[u] * b[v]
                    if k < n:
                        acc[k] += term
                    else:
                        acc[k - n] -= term
        want[c, l] = np.array([int(v) % q for v in acc], dtype=np.uint32)
    ct_hat = np.stack([np.stack([oracle.ntt_forward(c_coef[p, :, l], primes[l]) for l in range(L)])
                       for p in range(2)])
    rg_hat = np.empty((2, ell, 2, L, n), dtype=np.uint32)
    for p, i, c, l in itertools.product(range(2), range(ell), range(2), range(L)):
        rg_hat[p, i, c, l] = oracle.ntt_forward(r_coef[p, i, c, :, l], primes[l])
    got = coltor.external_product(ct_hat, rg_hat, primes, log2z, ell)
    want_hat = np.stack([np.stack([oracle.ntt_forward(want[c, l], primes[l]) for l in range(L)])
                         for c in range(2)])
    assert np.array_equal(got, want_hat)


def _enc_zero(seed, shat, primes, n):
    """RLWE encryption of 0 in the NTT domain: (a, -a s + e)."""
    L = len(primes)
    e = synth.gaussian_int(synth.stream_key(seed, synth.TAG_ERROR), np.arange(n), rlwe.SIGMA, rlwe.TAIL)
    a = _rand_res(seed, (n,), primes)                             # [N][L]
    out = np.empty((2, L, n), dtype=np.uint32)
    for l, q in enumerate(primes):
        q = int(q)
        ehat = oracle.ntt_forward(np.mod(e, q).astype(np.uint32), q).astype(object)
        out[0, l] = a[:, l]
        out[1, l] = ((-(a[:, l].astype(object) * shat[l]) + ehat) % q).astype(np.uint32)
    return out


def test_stage_decrypts_to_selected_column():
    # messages m_j (polynomials with coefficients below t, scaled by Delta = Q // t);
    # RGSW(bit) = encryptions of zero + bit * gadget rows; decryption of the
    # stage output rounds to m_{2t + bit}
    primes, log2z, ell, n, t_pt = Q108, 22, 5, 32, 1 << 16
    L = len(primes)
    Q = coltor.modulus(primes)
    s = rlwe.secret(240, n)
    shat = [oracle.ntt_forward(np.mod(s, int(q)).astype(np.uint32), int(q)).astype(object) for q in primes]
    dl = Q // t_pt
    ncols = 4
    msgs = [synth.draw_scalar(synth.stream_key(241, synth.TAG_DB), j) % t_pt for j in range(ncols * n)]
    msgs = np.array(msgs, dtype=object).reshape(ncols, n)
    cts = np.empty((1, 2, ncols, L, n), dtype=np.uint32)
    for j in range(ncols):
        z0 = _enc_zero(300 + j, shat, primes, n)
        for l, q in enumerate(primes):
            q = int(q)
            mhat = oracle.ntt_forward(np.array([(int(v) * dl) % q for v in msgs[j]], dtype=np.uint32), q)
            cts[0, 0, j, l] = z0[0, l]
            cts[0, 1, j, l] = ((z0[1, l].astype(object) + mhat.astype(object)) % q).astype(np.uint32)
    for bit in (0, 1):
        rg = np.empty((1, 2, ell, 2, L, n), dtype=np.uint32)
        gad = coltor.trivial_rgsw(bit, primes, n, log2z, ell)
        for p, i in itertools.product(range(2), range(ell)):
            z0 = _enc_zero(400 + 10 * p + i, shat, primes, n)
            for c, l in itertools.product(range(2), range(L)):
                q = int(primes[l])
                rg[0, p, i, c, l] = ((z0[c, l].astype(object) + gad[p, i, c, l].astype(object)) % q).astype(np.uint32)
        out = coltor.coltor_stage(cts, rg, primes, log2z, ell)
        phi = rlwe.phase(out[0], s, primes)                        # [ncols/2][L][N]
        for t in range(ncols // 2):
            x = coltor.crt(np.moveaxis(phi[t], 0, -1), primes)     # [N]
            dec = [((int(v) * t_pt + Q // 2) // Q) % t_pt for v in x]
            assert dec == [int(v) for v in msgs[2 * t + bit]], (bit, t)
