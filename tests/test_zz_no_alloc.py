"""The allocation-free entry point pir_rowsel_noalloc, through the C ABI:
two calls in a row (the second smaller, on another DB) give the same words
as pir_rowsel on the same inputs, which the oracle checks too; sizes beyond
the fixed scratch fail before any device work."""
import numpy as np
import pytest

import oracle
import synth
from helpers import empty_u32, np_u32, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

PR = synth.PRIMES_N4096


@pytest.fixture(scope="module")
def pir():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_04696_amd as pkg
    pkg.lib()
    return pkg


def _case(pir, n, d0, d1, B, seed, primes=PR):
    coeffs = synth.db_coeffs(seed, d0, d1, len(primes), n)
    query = synth.query_uniform(seed + 1, B, d0, primes, n)
    db = pir.pir_db_create(pir.make_params(n, primes, d0, d1), pir.PIR_LAYOUT_VALU)
    pir.pir_db_load_ntt(db, to_dev(coeffs), domain=pir.PIR_DOMAIN_COEFF)
    want = oracle.rowsel(query, oracle.ntt_db(coeffs, primes), primes)
    return db, to_dev(query), want


@pytest.mark.parametrize("primes", [PR, synth.PRIMES_W32], ids=["q30", "w32"])
def test_noalloc_equals_rowsel_twice(pir, primes):
    big = _case(pir, 1024, 70, 300, 4 if primes == PR else 2, 91, primes)
    small = _case(pir, 256, 33, 45, 1, 93, primes)
    for db, q, want in (big, small):            # two calls in a row, the second smaller
        B = want.shape[0]
        ref = empty_u32(want.size)
        got = empty_u32(want.size)
        got.fill_(-1)
        print("noalloc case", db.n, db.d0, db.d1, B, flush=True)
        pir.pir_rowsel(db, q, ref, pir.PIR_PATH_VALU)
        pir.pir_rowsel_noalloc(db, q, got)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
        assert np.array_equal(np_u32(got).reshape(want.shape), want)
    for db, _, _ in (big, small):
        pir.pir_db_free(db)


def test_noalloc_rejects_beyond_scratch(pir):
    # N = 4096, L = 2, D1 = 512: two clients fill 64 MiB of staging, three do not fit
    db = pir.pir_db_create(pir.make_params(4096, PR, 4, 512), pir.PIR_LAYOUT_VALU)
    q = empty_u32(3 * 2 * 4 * 2 * 4096)
    out = empty_u32(3 * 2 * 512 * 2 * 4096)
    with pytest.raises(pir.PirError, match="maximum"):
        pir.pir_rowsel_noalloc(db, q, out, B=3)
    with pytest.raises(pir.PirError, match="1..4 clients"):
        pir.pir_rowsel_noalloc(db, empty_u32(5 * 2 * 4 * 2 * 4096), empty_u32(5 * 2 * 512 * 2 * 4096), B=5)
    pir.pir_db_free(db)
    mdb = pir.pir_db_create(pir.make_params(64, PR, 4, 8), pir.PIR_LAYOUT_MFMA)
    with pytest.raises(pir.PirError, match="VALU layout"):
        pir.pir_rowsel_noalloc(mdb, empty_u32(2 * 4 * 2 * 64), empty_u32(2 * 8 * 2 * 64))
    pir.pir_db_free(mdb)


def test_noalloc_under_graph_capture(pir):
    """The allocation-free call captured into a hipGraph (its first call on
    the device, outside capture, takes the scratch address): three replays
    with eager work between them, each equal to pir_rowsel."""
    db, q, want = _case(pir, 512, 40, 200, 2, 95)
    ref = empty_u32(want.size)
    pir.pir_rowsel(db, q, ref, pir.PIR_PATH_VALU)
    out = empty_u32(want.size)
    pir.pir_rowsel_noalloc(db, q, out)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        pir.pir_rowsel_noalloc(db, q, out, stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        out.fill_(rep + 7)                       # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"replay {rep}"
    assert np.array_equal(np_u32(out).reshape(want.shape), want)
    del g
    pir.pir_db_free(db)
