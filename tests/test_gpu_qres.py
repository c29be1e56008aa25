"""GPU parity of the query-resident INT8 MFMA kernel (16 x 16 x 64 MFMAs, a
per-wave DB ring and a block-shared query ring in LDS) against the CPU
oracle, word for word, and against the tiled MFMA kernel on the same inputs.

PIR_MFMA_KERNEL=qres forces single pir_rowsel calls on the MFMA path through
it (PIR_MFMA_KERNEL=tile through the tiled kernel).  The shapes cover its
four unit shapes (32 x 128 and 64 x 128 with a DB ring per wave, 96 x 64
and 128 x 64 with one per block; picked from the padded row count, or
forced taller) and more than 128 rows (units in several row blocks), D1 ragged
against every unit width, D0 at the fewest chunks of k the kernel takes, D0
above the 2048-row int32 accumulation (flushes that add to what an earlier
flush of the unit stored), the split and wide recombination forms, four
limbs, and more or fewer work units than persistent blocks."""
import numpy as np
import pytest

import oracle
import synth
from helpers import assert_guards, guarded_u32, np_u32, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pir():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_04696_amd as pkg
    pkg.lib()
    return pkg


def say(*a):
    print(*a, flush=True)


P2 = synth.PRIMES_N4096
SHAPES = [
    # (N, primes, D0, D1, B); the kernel needs at least 3 (32-row units) or 2
    # (64- and 128-row units) chunks of 64 rows of k
    (64, P2, 200, 300, 1),           # 32-row units, 4 chunks, D1 ragged
    (64, P2, 130, 33, 17),           # 64-row units, 3 chunks (the last ragged)
    (128, P2, 160, 40, 33),          # 66 rows in 96-row units
    (16, P2, 200, 5, 64),            # 128 rows, D1 = 5
    (64, P2, 300, 100, 80),          # 160 rows: two 128-row blocks
    (16, P2, 4200, 5, 2),            # 66 chunks: flushes at 32, 64, 66
    (16, P2, 2100, 20, 20),          # 64-row units, 33 chunks
    (16, P2, 4100, 8, 50),           # 128-row units, 65 chunks
    (16, P2, 4100, 70, 40),          # 96-row units, 65 chunks, D1 ragged
    (64, P2, 256, 200, 48),          # 96 rows, whole units, 4 chunks
    (64, (954376193,), 600, 24, 3),  # split recombination
    (64, (954376193, 1073692673), 130, 40, 17),
    (32, synth.PRIMES_Q108, 130, 33, 9),
    (16, P2, 150, 520, 9),
    (256, P2, 512, 130, 30),         # 1024 units (more than the blocks)
    (64, P2, 192, 256, 16),          # whole unit widths, 3 chunks
    (64, P2, 512, 128, 32),          # whole 64 x 128 units
    (8, P2, 128, 16, 40),            # 2 chunks, fewer units than blocks
]


def _case(pir, shape, layout=None):
    n, primes, d0, d1, B = shape
    coeffs = synth.db_coeffs(60, d0, d1, len(primes), n)
    query = synth.query_uniform(61, B, d0, primes, n)
    want = oracle.rowsel(query, oracle.ntt_db(coeffs, primes), primes)
    db = pir.pir_db_create(pir.make_params(n, primes, d0, d1), layout or pir.PIR_LAYOUT_MFMA)
    pir.pir_db_load_ntt(db, to_dev(coeffs), domain=pir.PIR_DOMAIN_COEFF)
    return db, to_dev(query), want


def _run(pir, db, q, size, kernel, monkeypatch):
    monkeypatch.setenv("PIR_MFMA_KERNEL", kernel)
    guard, out = guarded_u32(size)
    pir.pir_rowsel(db, q, out, pir.PIR_PATH_MFMA_I8)
    torch.cuda.synchronize()
    assert_guards(guard)
    return out


@pytest.mark.parametrize("shape", SHAPES, ids=[f"N{s[0]}L{len(s[1])}_{s[2]}x{s[3]}_B{s[4]}" for s in SHAPES])
def test_qres_matches_oracle(pir, shape, monkeypatch):
    say("qres rowsel", shape)
    db, q, want = _case(pir, shape)
    got = _run(pir, db, q, want.size, "qres", monkeypatch)
    g = np_u32(got).reshape(want.shape)
    assert np.array_equal(g, want), f"{(g != want).sum()} of {want.size} words differ"
    tiled = _run(pir, db, q, want.size, "tile", monkeypatch)
    assert torch.equal(got, tiled)
    pir.pir_db_free(db)


@pytest.mark.parametrize("B", [8, 30, 40, 64])
def test_qres_all_q_minus_one(pir, B, monkeypatch):
    # every product (q-1)^2 = 1 mod q with the largest digit sums: each output
    # is D0 mod q (D0 above the 2048-row accumulation chunk)
    n, primes, d0, d1 = 16, P2, 4100, 40
    say("qres q-1, B", B)
    dhat = np.empty((d0, d1, len(primes), n), dtype=np.uint32)
    qv = np.empty((B, 2, d0, len(primes), n), dtype=np.uint32)
    for l, qq in enumerate(primes):
        dhat[..., l, :] = qq - 1
        qv[..., l, :] = qq - 1
    db = pir.pir_db_create(pir.make_params(n, primes, d0, d1), pir.PIR_LAYOUT_MFMA)
    pir.pir_db_load_ntt(db, to_dev(dhat), domain=pir.PIR_DOMAIN_NTT)
    out = _run(pir, db, to_dev(qv), B * 2 * d1 * len(primes) * n, "qres", monkeypatch)
    want = np.array([d0 % qq for qq in primes], dtype=np.uint32)
    assert np.all(np_u32(out).reshape(B, 2, d1, len(primes), n) == want[:, None])
    pir.pir_db_free(db)


@pytest.mark.parametrize("shape", [(64, synth.PRIMES_W32, 200, 33, 9), (64, (synth.PRIMES_W32[1], 1073692673), 145, 20, 40)],
                         ids=["w32_B9", "w32mix_B40"])
def test_qres_wide_primes(pir, shape, monkeypatch):
    say("qres wide", shape)
    db, q, want = _case(pir, shape)
    got = _run(pir, db, q, want.size, "qres", monkeypatch)
    g = np_u32(got).reshape(want.shape)
    assert np.array_equal(g, want), f"{(g != want).sum()} of {want.size} words differ"
    pir.pir_db_free(db)


def test_qres_coefficient_domain_query(pir, monkeypatch):
    n, primes, d0, d1, B = 256, P2, 96, 70, 24
    say("qres coefficient-domain query")
    db, _, _ = _case(pir, (n, primes, d0, d1, B))
    qn = synth.query_uniform(62, B, d0, primes, n)
    want = oracle.rowsel(qn, oracle.ntt_db(synth.db_coeffs(60, d0, d1, len(primes), n), primes), primes)
    qc = np.empty_like(qn)
    for l, qq in enumerate(primes):
        qc[:, :, :, l, :] = oracle.ntt_inverse(np.ascontiguousarray(qn[:, :, :, l, :]), qq)
    monkeypatch.setenv("PIR_MFMA_KERNEL", "qres")
    guard, out = guarded_u32(want.size)
    pir.pir_rowsel_coeff(db, to_dev(qc), out, pir.PIR_PATH_MFMA_I8)
    torch.cuda.synchronize()
    assert_guards(guard)
    assert np.array_equal(np_u32(out).reshape(want.shape), want)
    pir.pir_db_free(db)


FORCED = [(s, 3) for s in SHAPES if 2 * s[4] <= 64] + [((16, P2, 200, 20, 30), 3)] + \
         [(s, 2) for s in SHAPES if 2 * s[4] <= 64] + [(s, 1) for s in SHAPES if 2 * s[4] <= 32]


@pytest.mark.parametrize("shape,variant", FORCED,
                         ids=[f"N{s[0]}L{len(s[1])}_{s[2]}x{s[3]}_B{s[4]}_u{v}" for s, v in FORCED])
def test_qres_larger_units(pir, shape, variant, monkeypatch):
    """Rows in units taller than they need (PIR_QRES_VARIANT picks the unit
    shape): 128-row units (four row groups of 2 x 2 sub-tiles per wave
    sharing one DB ring), 96-row units (two row groups, one ring) and 64-row
    units, with a third or more of their rows past the batch."""
    say("qres larger units", shape, variant)
    monkeypatch.setenv("PIR_QRES_VARIANT", str(variant))
    db, q, want = _case(pir, shape)
    got = _run(pir, db, q, want.size, "qres", monkeypatch)
    g = np_u32(got).reshape(want.shape)
    assert np.array_equal(g, want), f"{(g != want).sum()} of {want.size} words differ"
    pir.pir_db_free(db)
