"""Parity at the full workload sizes, in the launch configuration the
benchmark times: N = 4096, two primes, a 512 x 512 DB of 16-bit
coefficients (8 GiB per layout), one client and 64 clients, on both paths,
and the 64-client query given in the coefficient domain.

Every output word is compared with the oracle (sec. 2.3's point-wise
products mod q_l): the host regenerates the DB coefficients and the queries
from the same seeds (``synth``), transforms the DB with the oracle's own NTT
and runs the oracle's RowSel on the host cores."""
import time

import numpy as np
import pytest

import oracle
import synth
from helpers import assert_guards, device_db, device_query, guarded_u32, host_db_ntt, host_query, np_u32, to_dev

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]
torch = pytest.importorskip("torch")

W1, W64 = synth.HBM, synth.BATCHED
assert (W1.dbseed, W1.d0, W1.d1, W1.primes) == (W64.dbseed, W64.d0, W64.d1, W64.primes)


def log(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def pir():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_04696_amd as pkg
    pkg.lib()
    return pkg


@pytest.fixture(scope="module")
def big_db(pir):
    log("building the 512 x 512 N=4096 two-prime DB on the device (both layouts)")
    db = device_db(pir, W1.n, W1.primes, W1.d0, W1.d1, W1.dbseed,
                   pir.PIR_LAYOUT_VALU | pir.PIR_LAYOUT_MFMA)
    yield db
    pir.pir_db_free(db)


@pytest.fixture(scope="module")
def dhat():
    t = time.time()
    log("host: seeded DB coefficients and the oracle's NTT (8 GiB)")
    d = host_db_ntt(W1.dbseed, W1.d0, W1.d1, W1.primes, W1.n, log=log)
    log(f"host: oracle DB ready in {time.time() - t:.1f} s")
    return d


@pytest.fixture(scope="module")
def batched_want(dhat):
    t = time.time()
    qh = host_query(W64.seed, W64.clients, W64.d0, W64.primes, W64.n)
    log("host: oracle RowSel, 64 clients (2.7e11 products)")
    want = oracle.rowsel(qh, dhat, W64.primes)
    log(f"host: oracle 64-client output ready in {time.time() - t:.1f} s")
    return qh, want


def _run(pir, db, q, B, path, w, fn=None):
    guard, out = guarded_u32(B * 2 * w.d1 * w.slots)
    (fn or pir.pir_rowsel)(db, q, out, path)
    torch.cuda.synchronize()
    assert_guards(guard)
    return np_u32(out).reshape(B, 2, w.d1, w.nprimes, w.n)


def _assert_equal(got, want, what):
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        raise AssertionError(f"{what}: {len(bad)} words differ from the oracle, first at {bad[0].tolist()}")


@pytest.mark.parametrize("path", [1, 2], ids=["valu", "mfma"])
def test_one_client_every_word(pir, big_db, dhat, path):
    w = W1
    want = oracle.rowsel(host_query(w.seed, 1, w.d0, w.primes, w.n), dhat, w.primes)
    q = device_query(pir, 1, w.d0, w.primes, w.n, w.seed)
    log(f"rowsel B=1 path {path} full size")
    _assert_equal(_run(pir, big_db, q, 1, path, w), want, f"B=1 path {path}")


@pytest.mark.parametrize("path", [2, 1], ids=["mfma", "valu"])
def test_batched_every_word(pir, big_db, batched_want, path):
    w = W64
    _, want = batched_want
    q = device_query(pir, w.clients, w.d0, w.primes, w.n, w.seed)
    log(f"rowsel B=64 path {path} full size")
    _assert_equal(_run(pir, big_db, q, w.clients, path, w), want, f"B=64 path {path}")


@pytest.mark.parametrize("path", [2, 1], ids=["mfma", "valu"])
def test_coeff_query_batched_every_word(pir, big_db, batched_want, path):
    """The 64-client query in the coefficient domain: the oracle's inverse NTT
    of the uniform query, so its transform is that query again and the
    expected output is the 64-client oracle output."""
    w = W64
    qh, want = batched_want
    qc = np.empty_like(qh)
    for l, q in enumerate(w.primes):
        qc[:, :, :, l, :] = oracle.ntt_inverse(np.ascontiguousarray(qh[:, :, :, l, :]), q)
    qd = to_dev(qc)
    del qc
    log(f"rowsel_coeff B=64 path {path} full size")
    got = _run(pir, big_db, qd, w.clients, path, w, fn=pir.pir_rowsel_coeff)
    _assert_equal(got, want, f"coefficient-domain B=64 path {path}")
