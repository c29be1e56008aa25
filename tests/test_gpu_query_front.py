"""GPU parity of the coefficient-domain query front end (pir_rowsel_coeff)
against the CPU oracle: the oracle transforms the query polynomials with its
own NTT and multiplies (tolerance 0), and the GPU result also equals
pir_rowsel on the query transformed by the library's NTT helper."""
import numpy as np
import pytest

import oracle
import synth
from helpers import empty_u32, np_u32, to_dev

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


def raw_coeffs(seed, shape):
    """Seeded full-range 32-bit words: limb l is read mod q_l."""
    count = int(np.prod(shape))
    w = synth.draw(synth.stream_key(seed, synth.TAG_QUERY, 7), np.arange(count, dtype=np.uint64))
    return (w & np.uint64(0xFFFFFFFF)).astype(np.uint32).reshape(shape)


SHAPES = [
    # (N, primes, D0, D1, B); the front end groups 8 polynomials of consecutive
    # k per block at N <= 4096, 4 at N = 8192 and 2 at N = 16384
    (8, (1073707009,), 5, 3, 1),
    (64, synth.PRIMES_N4096, 37, 300, 1),
    (64, (1073692673,), 100, 70, 3),
    (32, synth.PRIMES_N4096, 64, 64, 5),
    (64, synth.PRIMES_N4096, 130, 33, 17),
    (16, (954376193, 1073692673), 70, 40, 9),
    (1024, (1073707009,), 40, 24, 2),
    (4096, synth.PRIMES_N4096, 9, 5, 3),
    (8192, (1073692673,), 6, 3, 1),
    (16384, (1073643521,), 3, 2, 2),
    (256, synth.PRIMES_Q108, 20, 9, 3),
    # many clients (the N = 4096 register form and the four-limb setting)
    (4096, synth.PRIMES_N4096, 7, 5, 19),
    (512, synth.PRIMES_Q108, 33, 10, 16),
    (64, synth.PRIMES_N4096, 20, 12, 40),
]


@pytest.mark.parametrize("shape", SHAPES, ids=[f"N{s[0]}L{len(s[1])}_{s[2]}x{s[3]}_B{s[4]}" for s in SHAPES])
@BOTH
def test_coeff_query_matches_oracle(pir, shape, path):
    n, primes, d0, d1, B = shape
    say("rowsel_coeff", shape, "path", path)
    coeffs = synth.db_coeffs(70, d0, d1, len(primes), n)
    qc = raw_coeffs(71, (B, 2, d0, len(primes), n))
    want = oracle.rowsel(oracle.ntt_db(qc, primes), oracle.ntt_db(coeffs, primes), primes)
    db = pir.pir_db_create(pir.make_params(n, primes, d0, d1))
    pir.pir_db_load_ntt(db, to_dev(coeffs), domain=pir.PIR_DOMAIN_COEFF)
    out = empty_u32(want.size)
    out.fill_(-1)
    pir.pir_rowsel_coeff(db, to_dev(qc), out, path)
    torch.cuda.synchronize()
    got = np_u32(out).reshape(want.shape)
    assert np.array_equal(got, want), f"{(got != want).sum()} of {want.size} words differ"


@BOTH
def test_coeff_query_equals_transformed_query(pir, path):
    # the front end against the library's own NTT helper followed by RowSel
    n, primes, d0, d1, B = 256, synth.PRIMES_N4096, 200, 48, 6
    say("rowsel_coeff vs ntt helper, path", path)
    coeffs = synth.db_coeffs(72, d0, d1, len(primes), n)
    qc = raw_coeffs(73, (B, 2, d0, len(primes), n))
    db = pir.pir_db_create(pir.make_params(n, primes, d0, d1))
    pir.pir_db_load_ntt(db, to_dev(coeffs), domain=pir.PIR_DOMAIN_COEFF)
    qd = to_dev(qc)
    qn = torch.empty_like(qd)
    for l, q in enumerate(primes):
        src = qd.view(B * 2 * d0, len(primes), n)[:, l, :].contiguous()
        dst = torch.empty_like(src)
        pir.pir_ntt_forward(src, dst, n, q)
        qn.view(B * 2 * d0, len(primes), n)[:, l, :] = dst
    a, b = empty_u32(B * 2 * d1 * len(primes) * n), empty_u32(B * 2 * d1 * len(primes) * n)
    pir.pir_rowsel_coeff(db, qd, a, path)
    pir.pir_rowsel(db, qn, b, path)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_coeff_query_all_q_minus_one(pir):
    # every coefficient q-1 (= -1): the query polynomial is -(1 + X + ... + X^(N-1)),
    # whose NTT values are not all equal; compare with the oracle at D0 above
    # one K chunk of the MFMA path, both paths
    n, primes, d0, d1, B = 16, (954376193,), 2100, 4, 2
    q = primes[0]
    say("rowsel_coeff q-1")
    dhat = np.full((d0, d1, 1, n), q - 1, dtype=np.uint32)
    qc = np.full((B, 2, d0, 1, n), q - 1, dtype=np.uint32)
    want = oracle.rowsel(oracle.ntt_db(qc, primes), dhat, primes)
    db = pir.pir_db_create(pir.make_params(n, primes, d0, d1))
    pir.pir_db_load_ntt(db, to_dev(dhat), domain=pir.PIR_DOMAIN_NTT)
    for path in (1, 2):
        out = empty_u32(want.size)
        pir.pir_rowsel_coeff(db, to_dev(qc), out, path)
        torch.cuda.synchronize()
        assert np.array_equal(np_u32(out).reshape(want.shape), want), path


def test_coeff_query_errors(pir):
    n, primes, d0, d1 = 64, synth.PRIMES_N4096, 8, 8
    db = pir.pir_db_create(pir.make_params(n, primes, d0, d1), pir.PIR_LAYOUT_VALU)
    q = empty_u32(2 * d0 * 2 * n)
    out = empty_u32(2 * d1 * 2 * n)
    with pytest.raises(pir.PirError, match="no MFMA layout"):
        pir.pir_rowsel_coeff(db, q, out, pir.PIR_PATH_MFMA_I8)
    with pytest.raises(pir.PirError, match="overlaps"):
        pir.pir_rowsel_coeff(db, q, q, pir.PIR_PATH_VALU)
    pir.pir_rowsel_coeff(db, q, out, pir.PIR_PATH_VALU, B=0)   # no-op
    torch.cuda.synchronize()
