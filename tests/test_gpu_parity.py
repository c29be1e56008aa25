"""GPU parity: the HIP library, called through its C ABI, against the CPU
oracle, word for word (integer arithmetic: tolerance 0)."""
import numpy as np
import pytest

import oracle
import oracle.rlwe as rlwe
import synth
from helpers import assert_guards, device_db, device_query, empty_u32, guarded_u32, np_u32, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pir():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_04696_amd as pkg
    pkg.lib()
    return pkg


BOTH = pytest.mark.parametrize("path", [1, 2], ids=["valu", "mfma"])


def say(*a):
    print(*a, flush=True)


# ------------------------------------------------------------ generators
def test_device_generators_match_numpy(pir):
    key = synth.stream_key(5, synth.TAG_QUERY, 1)
    d = torch.empty(4096, dtype=torch.int64, device="cuda")
    pir.pir_synth_draw(d, key, 123)
    torch.cuda.synchronize()
    assert np.array_equal(d.cpu().numpy().view(np.uint64), synth.draw(key, np.arange(123, 123 + 4096)))

    primes, n, d0, B = synth.PRIMES_N4096, 64, 7, 3
    q = device_query(pir, B, d0, primes, n, seed=5, sub=1)
    torch.cuda.synchronize()
    want = synth.query_uniform(5, B, d0, primes, n, sub=1)
    assert np.array_equal(np_u32(q).reshape(want.shape), want)

    out = empty_u32(3 * 5 * 2 * n)
    pir.pir_synth_db_coeffs(out, synth.stream_key(6, synth.TAG_DB), 4, 3, 5, 2, n)
    torch.cuda.synchronize()
    want = synth.db_coeffs(6, 10, 5, 2, n, rows=[4, 5, 6])
    assert np.array_equal(np_u32(out).reshape(want.shape), want)


# ------------------------------------------------------------------- NTT
@pytest.mark.parametrize("q,n", [(1073707009, 1024), (1073692673, 4096), (1073668097, 4096),
                                 (1073707009, 8), (1073643521, 16384)])
def test_ntt_helper_matches_oracle(pir, q, n):
    say("ntt", q, n)
    count = 3
    a = synth.uniform_mod(synth.stream_key(40, synth.TAG_QUERY, n), np.arange(count * n), q) \
        .reshape(count, n)
    src = to_dev(a)
    fwd = empty_u32(count * n)
    pir.pir_ntt_forward(src, fwd, n, q)
    inv = empty_u32(count * n)
    pir.pir_ntt_inverse(fwd, inv, n, q)
    torch.cuda.synchronize()
    assert np.array_equal(np_u32(fwd).reshape(count, n), oracle.ntt_forward(a, q))
    assert np.array_equal(np_u32(inv).reshape(count, n), a)
    pir.pir_ntt_inverse(src, src, n, q)          # in place
    torch.cuda.synchronize()
    assert np.array_equal(np_u32(src).reshape(count, n), oracle.ntt_inverse(a, q))


# ------------------------------------------------------- small shapes
SHAPES = [
    # (N, primes, D0, D1, B)
    (8, (1073707009,), 5, 3, 1),
    (64, synth.PRIMES_N4096, 37, 300, 1),
    (64, synth.PRIMES_N4096, 37, 300, 2),
    (64, (1073692673,), 100, 70, 3),
    (64, synth.PRIMES_N4096, 15, 256, 4),
    (32, synth.PRIMES_N4096, 64, 64, 5),
    (64, synth.PRIMES_N4096, 130, 33, 17),
    (128, synth.PRIMES_N4096, 31, 40, 33),
    (64, synth.PRIMES_N4096, 1, 1, 1),
    (16, synth.PRIMES_N4096, 200, 5, 64),
    # D1 over three 256-column strips of the VALU layout (the last 8 wide),
    # on the streaming (B <= 4) and the tiled (B > 4) VALU kernels
    (16, synth.PRIMES_N4096, 33, 520, 2),
    (16, synth.PRIMES_N4096, 70, 520, 9),
    # streaming kernel: an even count of 8-row batches and no ragged tail,
    # fewer point groups than one output-transpose tile
    (32, synth.PRIMES_N4096, 48, 260, 1),
    # the paper's RNS setting: four 27-bit limbs (Q ~ 2^108)
    (64, synth.PRIMES_Q108, 45, 70, 1),
    (64, synth.PRIMES_Q108, 100, 40, 3),
    (32, synth.PRIMES_Q108, 130, 33, 9),
    (4096, synth.PRIMES_Q108, 9, 5, 2),
    # D0 above the 2048-row int32 accumulation chunk of the MFMA path
    (16, synth.PRIMES_N4096, 4200, 5, 2),
    # a prime with large 2^32 mod q (954376193: the recombination takes the
    # split form), alone and beside a prime that does not need it
    (64, (954376193,), 600, 24, 3),
    (64, (954376193, 1073692673), 130, 40, 17),
]


@pytest.mark.parametrize("shape", SHAPES, ids=[f"N{s[0]}L{len(s[1])}_{s[2]}x{s[3]}_B{s[4]}"
                                               for s in SHAPES])
@BOTH
def test_rowsel_matches_oracle(pir, shape, path):
    n, primes, d0, d1, B = shape
    say("rowsel", shape, "path", path)
    coeffs = synth.db_coeffs(50, d0, d1, len(primes), n)
    query = synth.query_uniform(51, B, d0, primes, n)
    want = oracle.rowsel(query, oracle.ntt_db(coeffs, primes), primes)
    db = pir.pir_db_create(pir.make_params(n, primes, d0, d1))
    pir.pir_db_load_ntt(db, to_dev(coeffs), domain=pir.PIR_DOMAIN_COEFF)
    guard, out = guarded_u32(want.size)
    pir.pir_rowsel(db, to_dev(query), out, path)
    torch.cuda.synchronize()
    got = np_u32(out).reshape(want.shape)
    assert np.array_equal(got, want), f"{(got != want).sum()} of {want.size} words differ"
    assert_guards(guard)


@BOTH
def test_rowsel_ntt_domain_load_and_row_chunks(pir, path):
    n, primes, d0, d1, B = 64, synth.PRIMES_N4096, 70, 20, 3
    say("chunks path", path)
    dhat = oracle.ntt_db(synth.db_coeffs(52, d0, d1, 2, n), primes)
    query = synth.query_uniform(53, B, d0, primes, n)
    want = oracle.rowsel(query, dhat, primes)
    db = pir.pir_db_create(pir.make_params(n, primes, d0, d1))
    for r0, r1 in [(40, 45), (0, 7), (45, 70), (7, 40)]:      # any order, ragged sizes
        pir.pir_db_load_ntt(db, to_dev(dhat[r0:r1]), r0, r1 - r0, pir.PIR_DOMAIN_NTT)
    out = empty_u32(want.size)
    pir.pir_rowsel(db, to_dev(query), out, path)
    torch.cuda.synchronize()
    assert np.array_equal(np_u32(out).reshape(want.shape), want)


@pytest.mark.parametrize("case", [(32, synth.PRIMES_N4096, 1000, 40), (16, (954376193,), 4100, 8),
                                  (16, synth.PRIMES_Q108, 2100, 6)],
                         ids=["two_primes_1000", "split_prime_4100", "four_limbs_2100"])
@BOTH
def test_rowsel_all_q_minus_one(pir, path, case):
    # (q-1)^2 = 1 mod q: every output is D0 mod q; stresses the lazy 64-bit
    # bound and the largest digit products
    n, primes, d0, d1 = case
    B = 2
    say("q-1 path", path, case)
    dhat = np.empty((d0, d1, len(primes), n), dtype=np.uint32)
    qv = np.empty((B, 2, d0, len(primes), n), dtype=np.uint32)
    for l, q in enumerate(primes):
        dhat[..., l, :] = q - 1
        qv[..., l, :] = q - 1
    db = pir.pir_db_create(pir.make_params(n, primes, d0, d1))
    pir.pir_db_load_ntt(db, to_dev(dhat), domain=pir.PIR_DOMAIN_NTT)
    out = empty_u32(B * 2 * d1 * len(primes) * n)
    pir.pir_rowsel(db, to_dev(qv), out, path)
    torch.cuda.synchronize()
    want = np.array([d0 % q for q in primes], dtype=np.uint32)
    assert np.all(np_u32(out).reshape(B, 2, d1, len(primes), n) == want[:, None])


# ------------------------------------------------------- toy encryption
@BOTH
def test_tiny_config_toy_rlwe(pir, path):
    """N = 1024, one prime, 16 x 16 DB of 16-bit coefficients, one client's
    16 toy encryptions of a one-hot selector: the GPU output equals the
    oracle's, and decrypting it returns DB row i* exactly."""
    w = synth.TINY
    say("tiny toy rlwe path", path)
    istar = synth.selected_row(w.seed, w.d0)
    coeffs = synth.db_coeffs(w.dbseed, w.d0, w.d1, 1, w.n)
    Q, s, e = rlwe.encrypt_selectors(w.seed, w.n, w.primes, w.d0, istar, t=1 << 16)
    want = oracle.rowsel(Q, oracle.ntt_db(coeffs, w.primes), w.primes)
    db = pir.pir_db_create(pir.make_params(w.n, w.primes, w.d0, w.d1))
    pir.pir_db_load_ntt(db, to_dev(coeffs), domain=pir.PIR_DOMAIN_COEFF)
    out = empty_u32(want.size)
    pir.pir_rowsel(db, to_dev(Q), out, path)
    torch.cuda.synchronize()
    got = np_u32(out).reshape(want.shape)
    assert np.array_equal(got, want)
    rec = rlwe.decrypt_known_noise(got[0], s, e, coeffs[:, :, 0, :], w.primes, 1 << 16)
    assert np.array_equal(rec[:, 0, :], coeffs[istar, :, 0, :])


# ------------------------------------------------------------ error paths
def test_error_paths_on_device(pir):
    n, primes, d0, d1 = 64, synth.PRIMES_N4096, 8, 8
    db = pir.pir_db_create(pir.make_params(n, primes, d0, d1), pir.PIR_LAYOUT_VALU)
    q = empty_u32(2 * d0 * 2 * n)
    out = empty_u32(2 * d1 * 2 * n)
    with pytest.raises(pir.PirError, match="no MFMA layout"):
        pir.pir_rowsel(db, q, out, pir.PIR_PATH_MFMA_I8)
    with pytest.raises(pir.PirError, match="overlaps"):
        pir.pir_rowsel(db, q, q, pir.PIR_PATH_VALU)
    with pytest.raises(pir.PirError, match="exceed"):
        pir.pir_db_load_ntt(db, empty_u32(2 * d1 * 2 * n), 7, 2, pir.PIR_DOMAIN_NTT)
    pir.pir_rowsel(db, q, out, pir.PIR_PATH_VALU, B=0)     # B = 0 is a no-op
    torch.cuda.synchronize()


def test_kernel_timing_counts_main_kernels(pir):
    # one timed launch per call: streaming (B <= 4), tiled (B > 4) and INT8 GEMM
    n, primes, d0, d1 = 64, synth.PRIMES_N4096, 40, 24
    db = pir.pir_db_create(pir.make_params(n, primes, d0, d1))
    pir.pir_db_load_ntt(db, to_dev(synth.db_coeffs(60, d0, d1, len(primes), n)),
                        domain=pir.PIR_DOMAIN_COEFF)
    calls = [(1, pir.PIR_PATH_VALU), (5, pir.PIR_PATH_VALU), (3, pir.PIR_PATH_MFMA_I8)]
    args = [(to_dev(synth.query_uniform(61, B, d0, primes, n)), empty_u32(B * 2 * d1 * len(primes) * n), path)
            for B, path in calls]
    pir.pir_kernel_timing(True)
    try:
        for q, out, path in args:
            pir.pir_rowsel(db, q, out, path)
        launches, ms = pir.pir_kernel_time_read()
        assert launches == len(calls) and ms > 0
        assert pir.pir_kernel_time_read() == (0, 0.0)
    finally:
        pir.pir_kernel_timing(False)
    q, out, path = args[0]
    pir.pir_rowsel(db, q, out, path)    # not recorded once disabled
    torch.cuda.synchronize()
    assert pir.pir_kernel_time_read() == (0, 0.0)


def test_rowsel_validate_rejects_non_residues(pir, monkeypatch):
    # PIR_VALIDATE=1: a query word >= its prime fails with PIR_EINVAL on both
    # paths; valid queries still run
    n, primes, d0, d1, B = 64, synth.PRIMES_N4096, 12, 5, 2
    monkeypatch.setenv("PIR_VALIDATE", "1")
    coeffs = synth.db_coeffs(95, d0, d1, len(primes), n)
    db = pir.pir_db_create(pir.make_params(n, primes, d0, d1))
    pir.pir_db_load_ntt(db, to_dev(coeffs), domain=pir.PIR_DOMAIN_COEFF)
    q = synth.query_uniform(96, B, d0, primes, n)
    out = empty_u32(B * 2 * d1 * len(primes) * n)
    bad = q.copy()
    bad[1, 0, 7, 1, 33] = primes[1]
    for path in (pir.PIR_PATH_VALU, pir.PIR_PATH_MFMA_I8):
        pir.pir_rowsel(db, to_dev(q), out, path)
        torch.cuda.synchronize()
        with pytest.raises(pir.PirError, match="PIR_VALIDATE"):
            pir.pir_rowsel(db, to_dev(bad), out, path)
