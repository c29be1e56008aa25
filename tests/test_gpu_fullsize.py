"""Parity at the full workload sizes, in the launch configuration the
benchmark times: N = 4096, two primes, a 512 x 512 DB of 16-bit
coefficients (8 GiB per layout), one client and 64 clients.  The oracle
checks sampled columns (every point, every component) from inputs it
regenerates by index; the two GPU paths are compared with each other on
every word."""
import numpy as np
import pytest

import oracle
import synth
from helpers import device_db, device_query, empty_u32, np_u32

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

W1, W64 = synth.HBM, synth.BATCHED


@pytest.fixture(scope="module")
def pir():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_04696_amd as pkg
    pkg.lib()
    return pkg


@pytest.fixture(scope="module")
def big_db(pir):
    print("building the 512 x 512 N=4096 two-prime DB (both layouts)", flush=True)
    db = device_db(pir, W1.n, W1.primes, W1.d0, W1.d1, W1.dbseed,
                   pir.PIR_LAYOUT_VALU | pir.PIR_LAYOUT_MFMA)
    yield db
    pir.pir_db_free(db)


def oracle_columns(w, cols, clients, query_seed, B):
    coeffs = synth.db_coeffs(w.dbseed, w.d0, w.d1, w.nprimes, w.n, cols=cols)
    dhat = oracle.ntt_db(coeffs, w.primes)                       # [D0][len(cols)][L][N]
    q = synth.query_uniform(query_seed, B, w.d0, w.primes, w.n, clients=clients)
    return oracle.rowsel(q, dhat, w.primes)                      # [len(clients)][2][len(cols)][L][N]


def test_one_client_sampled(pir, big_db):
    w = W1
    q = device_query(pir, 1, w.d0, w.primes, w.n, w.seed)
    out = empty_u32(2 * w.d1 * w.slots)
    print("rowsel B=1 VALU full size", flush=True)
    pir.pir_rowsel(big_db, q, out, pir.PIR_PATH_VALU)
    torch.cuda.synchronize()
    got = np_u32(out).reshape(1, 2, w.d1, w.nprimes, w.n)
    cols = [0, 257, 511]
    want = oracle_columns(w, cols, [0], w.seed, 1)
    assert np.array_equal(got[:, :, cols], want)
    assert np.all(got < np.array(w.primes, dtype=np.uint32)[None, None, None, :, None])


def test_batched_sampled_and_paths_identical(pir, big_db):
    w = W64
    q = device_query(pir, w.clients, w.d0, w.primes, w.n, w.seed)
    outs = {}
    for path, name in [(pir.PIR_PATH_MFMA_I8, "mfma"), (pir.PIR_PATH_VALU, "valu")]:
        out = empty_u32(w.clients * 2 * w.d1 * w.slots)
        print(f"rowsel B=64 {name} full size", flush=True)
        pir.pir_rowsel(big_db, q, out, path)
        torch.cuda.synchronize()
        outs[name] = out
    assert torch.equal(outs["mfma"], outs["valu"])
    got = np_u32(outs["mfma"]).reshape(w.clients, 2, w.d1, w.nprimes, w.n)
    clients, cols = [0, 37, 63], [5, 300]
    want = oracle_columns(w, cols, clients, w.seed, w.clients)
    assert np.array_equal(got[clients][:, :, cols], want)


def test_coeff_query_batched_full_size(pir, big_db):
    # coefficient-domain query at the 64-client size: the fused front end on
    # the MFMA path equals the NTT helper followed by pir_rowsel on every
    # word, and the oracle (its own NTT of the sampled clients' polynomials)
    # on sampled columns
    w = W64
    key = synth.stream_key(w.seed, synth.TAG_QUERY, 9)
    count = w.clients * 2 * w.d0 * w.slots
    qc = torch.empty(count, dtype=torch.int32, device="cuda")
    pir.pir_synth_query(qc, key, 0, w.clients, w.d0, w.primes, w.n)    # residues < q_l as coefficients
    qn = torch.empty_like(qc)
    rows = w.clients * 2 * w.d0
    for l, q in enumerate(w.primes):
        src = qc.view(rows, w.nprimes, w.n)[:, l, :].contiguous()
        dst = torch.empty_like(src)
        pir.pir_ntt_forward(src, dst, w.n, q)
        qn.view(rows, w.nprimes, w.n)[:, l, :] = dst
        del src, dst
    a = empty_u32(w.clients * 2 * w.d1 * w.slots)
    b = empty_u32(w.clients * 2 * w.d1 * w.slots)
    print("rowsel_coeff B=64 mfma full size", flush=True)
    pir.pir_rowsel_coeff(big_db, qc, a, pir.PIR_PATH_MFMA_I8)
    pir.pir_rowsel(big_db, qn, b, pir.PIR_PATH_MFMA_I8)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    clients, cols = [0, 41], [7, 400]
    qsel = np_u32(qc).reshape(w.clients, 2, w.d0, w.nprimes, w.n)[clients]
    coeffs = synth.db_coeffs(w.dbseed, w.d0, w.d1, w.nprimes, w.n, cols=cols)
    want = oracle.rowsel(oracle.ntt_db(qsel, w.primes), oracle.ntt_db(coeffs, w.primes), w.primes)
    got = np_u32(a).reshape(w.clients, 2, w.d1, w.nprimes, w.n)
    assert np.array_equal(got[clients][:, :, cols], want)
