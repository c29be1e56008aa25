"""Parity at the full sizes of the two RNS settings the benchmark times
beside the headline: the paper's four 27-bit limbs (N = 4096, 256 x 512,
8 GiB; one client and 32) and two full 32-bit primes (N = 4096, 512 x 512,
8 GiB; one client and 32, where the MFMA path splits residues inside the
digit window).  The oracle checks sampled columns (every point, every
component) from inputs it regenerates by index; the two GPU paths are
compared with each other on every word."""
import numpy as np
import pytest

import oracle
import synth
from helpers import device_db, device_query, empty_u32, np_u32

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pir():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_04696_amd as pkg
    pkg.lib()
    return pkg


def oracle_columns(w, cols, clients, B):
    coeffs = synth.db_coeffs(w.dbseed, w.d0, w.d1, w.nprimes, w.n, cols=cols)
    dhat = oracle.ntt_db(coeffs, w.primes)
    q = synth.query_uniform(w.seed, B, w.d0, w.primes, w.n, clients=clients)
    return oracle.rowsel(q, dhat, w.primes)


@pytest.mark.parametrize("w", [synth.PAPER_Q108, synth.WIDE32], ids=["q108", "w32"])
def test_rns_full_size_sampled(pir, w):
    print("building", w.name, "(both layouts)", flush=True)
    db = device_db(pir, w.n, w.primes, w.d0, w.d1, w.dbseed, pir.PIR_LAYOUT_VALU | pir.PIR_LAYOUT_MFMA)
    try:
        bound = np.array(w.primes, dtype=np.uint32)[None, None, None, :, None]
        # one client: the streaming kernel
        q1 = device_query(pir, 1, w.d0, w.primes, w.n, w.seed)
        out1 = empty_u32(2 * w.d1 * w.slots)
        print(w.name, "B=1 VALU", flush=True)
        pir.pir_rowsel(db, q1, out1, pir.PIR_PATH_VALU)
        torch.cuda.synchronize()
        got1 = np_u32(out1).reshape(1, 2, w.d1, w.nprimes, w.n)
        cols = [0, w.d1 - 1]
        assert np.array_equal(got1[:, :, cols], oracle_columns(w, cols, [0], 1))
        assert np.all(got1 < bound)
        del q1, out1
        # 32 clients on both paths
        B = 32
        q = device_query(pir, B, w.d0, w.primes, w.n, w.seed)
        outs = {}
        for path, name in [(pir.PIR_PATH_MFMA_I8, "mfma"), (pir.PIR_PATH_VALU, "valu")]:
            out = empty_u32(B * 2 * w.d1 * w.slots)
            print(w.name, f"B={B}", name, flush=True)
            pir.pir_rowsel(db, q, out, path)
            torch.cuda.synchronize()
            outs[name] = out
        assert torch.equal(outs["mfma"], outs["valu"])
        got = np_u32(outs["mfma"]).reshape(B, 2, w.d1, w.nprimes, w.n)
        clients, cols = [0, 31], [3, w.d1 // 2 + 7]
        assert np.array_equal(got[clients][:, :, cols], oracle_columns(w, cols, clients, B))
        assert np.all(got[clients] < bound)
    finally:
        pir.pir_db_free(db)
