"""Parity at the full sizes of the two RNS settings the benchmark times
beside the headline: the paper's four 27-bit limbs (N = 4096, 256 x 512,
8 GiB; one client and 32) and two full 32-bit primes (N = 4096, 512 x 512,
8 GiB; one client and 32, where the MFMA path splits residues inside the
digit window).  Every output word of both paths is compared with the oracle,
which regenerates the DB and queries from their seeds and runs its own NTT
and RowSel on the host cores."""
import time

import numpy as np
import pytest

import oracle
import synth
from helpers import assert_guards, device_db, device_query, guarded_u32, host_db_ntt, host_query, np_u32

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pir():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_04696_amd as pkg
    pkg.lib()
    return pkg


@pytest.mark.parametrize("w", [synth.PAPER_Q108, synth.WIDE32], ids=["q108", "w32"])
def test_rns_full_size_every_word(pir, w):
    print("building", w.name, "(both layouts)", flush=True)
    db = device_db(pir, w.n, w.primes, w.d0, w.d1, w.dbseed, pir.PIR_LAYOUT_VALU | pir.PIR_LAYOUT_MFMA)
    try:
        t = time.time()
        dhat = host_db_ntt(w.dbseed, w.d0, w.d1, w.primes, w.n)
        print(f"host: oracle DB in {time.time() - t:.1f} s", flush=True)
        bound = np.array(w.primes, dtype=np.uint32)[None, None, None, :, None]
        for B, paths in ((1, [(pir.PIR_PATH_VALU, "valu"), (pir.PIR_PATH_MFMA_I8, "mfma")]),
                         (32, [(pir.PIR_PATH_MFMA_I8, "mfma"), (pir.PIR_PATH_VALU, "valu")])):
            want = oracle.rowsel(host_query(w.seed, B, w.d0, w.primes, w.n), dhat, w.primes)
            q = device_query(pir, B, w.d0, w.primes, w.n, w.seed)
            for path, name in paths:
                guard, out = guarded_u32(B * 2 * w.d1 * w.slots)
                print(w.name, f"B={B}", name, flush=True)
                pir.pir_rowsel(db, q, out, path)
                torch.cuda.synchronize()
                assert_guards(guard)
                got = np_u32(out).reshape(want.shape)
                assert np.array_equal(got, want), f"{w.name} B={B} {name}: {(got != want).sum()} words differ"
                assert np.all(got < bound)
                del guard, out
            del q, want
    finally:
        pir.pir_db_free(db)
