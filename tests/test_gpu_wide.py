"""GPU parity with primes of 2^30 or more (products of residues reach 2^64):
the VALU path keeps 64-bit sums that count their wraps, the NTTs keep 64-bit
intermediates, and the INT8 MFMA path splits each residue r as r or r - q,
whichever four signed 8-bit digits reach, and recombines in its wide form.
Against the CPU oracle word for word (tolerance 0)."""
import numpy as np
import pytest

import oracle
import synth
from helpers import empty_u32, np_u32, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

W32 = synth.PRIMES_W32


@pytest.fixture(scope="module")
def pir():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_04696_amd as pkg
    pkg.lib()
    return pkg


def say(*a):
    print(*a, flush=True)


SHAPES = [
    # (N, primes, D0, D1, B): streaming kernel (2B <= 8) and tiled kernel
    (64, W32, 37, 300, 1),
    (64, W32, 100, 70, 3),
    (64, (W32[0],), 20, 9, 4),
    (32, W32, 130, 33, 9),
    (4096, W32, 9, 5, 2),
    # a wide prime next to a 30-bit one
    (64, (W32[1], 1073692673), 45, 20, 5),
]


@pytest.mark.parametrize("shape", SHAPES, ids=[f"N{s[0]}L{len(s[1])}_{s[2]}x{s[3]}_B{s[4]}" for s in SHAPES])
def test_wide_rowsel_matches_oracle(pir, shape):
    n, primes, d0, d1, B = shape
    say("wide rowsel", shape)
    coeffs = synth.db_coeffs(80, d0, d1, len(primes), n)
    query = synth.query_uniform(81, B, d0, primes, n)
    want = oracle.rowsel(query, oracle.ntt_db(coeffs, primes), primes)
    db = pir.pir_db_create(pir.make_params(n, primes, d0, d1), pir.PIR_LAYOUT_VALU)
    pir.pir_db_load_ntt(db, to_dev(coeffs), domain=pir.PIR_DOMAIN_COEFF)
    out = empty_u32(want.size)
    out.fill_(-1)
    pir.pir_rowsel(db, to_dev(query), out, pir.PIR_PATH_AUTO)
    torch.cuda.synchronize()
    got = np_u32(out).reshape(want.shape)
    assert np.array_equal(got, want), f"{(got != want).sum()} of {want.size} words differ"


@pytest.mark.parametrize("B", [2, 5])
def test_wide_all_q_minus_one(pir, B):
    # (q-1)^2 = 1 mod q with (q-1)^2 just below 2^64: almost every product
    # wraps the 64-bit sum; every output must be D0 mod q
    n, primes, d0, d1 = 16, W32, 4100, 6
    say("wide q-1, B", B)
    dhat = np.empty((d0, d1, len(primes), n), dtype=np.uint32)
    qv = np.empty((B, 2, d0, len(primes), n), dtype=np.uint32)
    for l, q in enumerate(primes):
        dhat[..., l, :] = q - 1
        qv[..., l, :] = q - 1
    db = pir.pir_db_create(pir.make_params(n, primes, d0, d1), pir.PIR_LAYOUT_VALU)
    pir.pir_db_load_ntt(db, to_dev(dhat), domain=pir.PIR_DOMAIN_NTT)
    out = empty_u32(B * 2 * d1 * len(primes) * n)
    pir.pir_rowsel(db, to_dev(qv), out, pir.PIR_PATH_VALU)
    torch.cuda.synchronize()
    want = np.array([d0 % q for q in primes], dtype=np.uint32)
    assert np.all(np_u32(out).reshape(B, 2, d1, len(primes), n) == want[:, None])


@pytest.mark.parametrize("q,n", [(W32[0], 4096), (W32[1], 64)])
def test_wide_ntt_helper_matches_oracle(pir, q, n):
    say("wide ntt", q, n)
    a = synth.uniform_mod(synth.stream_key(82, synth.TAG_QUERY), np.arange(3 * n), q).reshape(3, n)
    want = oracle.ntt_forward(a, q)
    out = empty_u32(a.size)
    pir.pir_ntt_forward(to_dev(a), out, n, q)
    back = empty_u32(a.size)
    pir.pir_ntt_inverse(out, back, n, q)
    torch.cuda.synchronize()
    assert np.array_equal(np_u32(out).reshape(a.shape), want)
    assert np.array_equal(np_u32(back).reshape(a.shape), a)


@pytest.mark.parametrize("n", [64, 4096])
def test_wide_coeff_query_matches_oracle(pir, n):
    # the coefficient-domain front end: small-ring and register-blocked transforms
    primes, d0, d1, B = W32, 21, 7, 3
    say("wide rowsel_coeff N", n)
    coeffs = synth.db_coeffs(83, d0, d1, len(primes), n)
    w = synth.draw(synth.stream_key(84, synth.TAG_QUERY, 7), np.arange(B * 2 * d0 * len(primes) * n,
                                                                        dtype=np.uint64))
    qc = (w & np.uint64(0xFFFFFFFF)).astype(np.uint32).reshape(B, 2, d0, len(primes), n)
    want = oracle.rowsel(oracle.ntt_db(qc, primes), oracle.ntt_db(coeffs, primes), primes)
    db = pir.pir_db_create(pir.make_params(n, primes, d0, d1), pir.PIR_LAYOUT_VALU)
    pir.pir_db_load_ntt(db, to_dev(coeffs), domain=pir.PIR_DOMAIN_COEFF)
    out = empty_u32(want.size)
    pir.pir_rowsel_coeff(db, to_dev(qc), out, pir.PIR_PATH_AUTO)
    torch.cuda.synchronize()
    assert np.array_equal(np_u32(out).reshape(want.shape), want)


# ------------------------------------------------ INT8 MFMA path, centred digits
W31, W32S = synth.PRIMES_W31, synth.PRIMES_W32_SYM

MFMA_SHAPES = [
    # (N, primes, D0, D1, B): 64 x 128 tiles (2B <= 64) and 128 x 64 tiles
    (64, W32, 37, 40, 3),
    (64, W31, 130, 33, 17),
    (32, W32S, 100, 24, 40),
    (8, (synth.PRIME_W32_TOP_N8,), 30, 20, 4),
    # a wide prime beside a 30-bit one (one launch, the wide recombination)
    (16, (W32[0], 1073692673), 70, 20, 9),
    # D0 above the 2048-row int32 accumulation chunk
    (16, W32, 2100, 6, 2),
    (16, W32S, 2100, 6, 2),
]


@pytest.mark.parametrize("shape", MFMA_SHAPES, ids=[f"N{s[0]}L{len(s[1])}_{s[2]}x{s[3]}_B{s[4]}"
                                                     for s in MFMA_SHAPES])
def test_wide_mfma_matches_oracle(pir, shape):
    n, primes, d0, d1, B = shape
    say("wide mfma", shape)
    coeffs = synth.db_coeffs(85, d0, d1, len(primes), n)
    query = synth.query_uniform(86, B, d0, primes, n)
    want = oracle.rowsel(query, oracle.ntt_db(coeffs, primes), primes)
    db = pir.pir_db_create(pir.make_params(n, primes, d0, d1))          # both layouts
    pir.pir_db_load_ntt(db, to_dev(coeffs), domain=pir.PIR_DOMAIN_COEFF)
    for path in (pir.PIR_PATH_MFMA_I8, pir.PIR_PATH_VALU):
        out = empty_u32(want.size)
        out.fill_(-1)
        pir.pir_rowsel(db, to_dev(query), out, path)
        torch.cuda.synchronize()
        got = np_u32(out).reshape(want.shape)
        assert np.array_equal(got, want), f"path {path}: {(got != want).sum()} of {want.size} words differ"


EDGE = [(16, W32), (16, W32S), (8, (synth.PRIME_W32_TOP_N8,))]


@pytest.mark.parametrize("n,primes", EDGE, ids=[f"q{p[0]}" for _, p in EDGE])
def test_wide_mfma_digit_window_edges(pir, n, primes):
    # residues at both ends of the digit window: T = 0x7F7F7F7F is split as
    # +T (all digits 127) and T + 1 as T + 1 - q (near -0x80808080); DB rows
    # alternate T + 1 and T, component 0 of every query is T + 1 and
    # component 1 is T, so products of every sign pairing reach about 2^62;
    # D0 spans three int32 accumulation chunks
    d0, d1, B, T = 4100, 5, 2, 0x7F7F7F7F
    say("wide mfma window edges", primes)
    dhat = np.empty((d0, d1, len(primes), n), dtype=np.uint32)
    qv = np.empty((B, 2, d0, len(primes), n), dtype=np.uint32)
    dhat[0::2], dhat[1::2] = T + 1, T
    qv[:, 0], qv[:, 1] = T + 1, T
    want = oracle.rowsel(qv, dhat, primes)
    db = pir.pir_db_create(pir.make_params(n, primes, d0, d1), pir.PIR_LAYOUT_MFMA)
    pir.pir_db_load_ntt(db, to_dev(dhat), domain=pir.PIR_DOMAIN_NTT)
    out = empty_u32(want.size)
    pir.pir_rowsel(db, to_dev(qv), out, pir.PIR_PATH_MFMA_I8)
    torch.cuda.synchronize()
    assert np.array_equal(np_u32(out).reshape(want.shape), want)


@pytest.mark.parametrize("B", [2, 5])
def test_wide_mfma_all_q_minus_one(pir, B):
    # every residue q - 1 (split as -1): every output is D0 mod q
    n, primes, d0, d1 = 16, W32, 4100, 6
    say("wide mfma q-1, B", B)
    dhat = np.empty((d0, d1, len(primes), n), dtype=np.uint32)
    qv = np.empty((B, 2, d0, len(primes), n), dtype=np.uint32)
    for l, q in enumerate(primes):
        dhat[..., l, :] = q - 1
        qv[..., l, :] = q - 1
    db = pir.pir_db_create(pir.make_params(n, primes, d0, d1), pir.PIR_LAYOUT_MFMA)
    pir.pir_db_load_ntt(db, to_dev(dhat), domain=pir.PIR_DOMAIN_NTT)
    out = empty_u32(B * 2 * d1 * len(primes) * n)
    pir.pir_rowsel(db, to_dev(qv), out, pir.PIR_PATH_MFMA_I8)
    torch.cuda.synchronize()
    want = np.array([d0 % q for q in primes], dtype=np.uint32)
    assert np.all(np_u32(out).reshape(B, 2, d1, len(primes), n) == want[:, None])


def test_wide_mfma_grouped_with_narrow_instance(pir):
    # one grouped launch over a wide and a 30-bit instance: the widest
    # recombination serves both
    specs = [(64, W32, 40, 24, 5), (64, synth.PRIMES_N4096, 70, 16, 20), (64, W31, 33, 9, 2)]
    items, wants = [], []
    for i, (n, primes, d0, d1, B) in enumerate(specs):
        coeffs = synth.db_coeffs(87 + i, d0, d1, len(primes), n)
        query = synth.query_uniform(89 + i, B, d0, primes, n)
        wants.append(oracle.rowsel(query, oracle.ntt_db(coeffs, primes), primes))
        db = pir.pir_db_create(pir.make_params(n, primes, d0, d1), pir.PIR_LAYOUT_MFMA)
        pir.pir_db_load_ntt(db, to_dev(coeffs), domain=pir.PIR_DOMAIN_COEFF)
        items.append((db, to_dev(query), B, empty_u32(wants[-1].size)))
    say("wide grouped")
    pir.pir_rowsel_grouped(items, pir.PIR_PATH_MFMA_I8)
    torch.cuda.synchronize()
    for (db, q, B, out), want in zip(items, wants):
        assert np.array_equal(np_u32(out).reshape(want.shape), want)


def test_wide_serving_matches_oracle(pir):
    # the continuous-batching server on a DB of two full 32-bit primes: its
    # MFMA steps take the digit window and the wide recombination
    import time
    n, primes, d0, d1 = 64, W32, 40, 30
    say("wide serving")
    coeffs = synth.db_coeffs(93, d0, d1, len(primes), n)
    dhat = oracle.ntt_db(coeffs, primes)
    db = pir.pir_db_create(pir.make_params(n, primes, d0, d1), pir.PIR_LAYOUT_MFMA)
    pir.pir_db_load_ntt(db, to_dev(dhat), domain=pir.PIR_DOMAIN_NTT)
    queries = synth.query_uniform(94, 6, d0, primes, n)
    wants = oracle.rowsel(queries, dhat, primes)
    srv = pir.pir_server_create(db, max_clients=4, chunks=3)
    outs = [empty_u32(2 * d1 * len(primes) * n) for _ in range(6)]
    qs = [to_dev(queries[i]) for i in range(6)]
    schedule = {0: [(i, qs[i], outs[i]) for i in range(4)], 2: [(i, qs[i], outs[i]) for i in range(4, 6)]}
    got, turn, t0 = {}, 0, time.time()
    while len(got) < 6:
        for c in pir.pir_serve_step(srv, schedule.get(turn, ())):
            got[c.id] = c
        turn += 1
        assert time.time() - t0 < 60, f"only {len(got)} of 6 completions"
    torch.cuda.synchronize()
    for i in range(6):
        assert got[i].status == 0
        assert np.array_equal(np_u32(outs[i]).reshape(wants[i].shape), wants[i]), f"request {i}"
    pir.pir_server_destroy(srv)
