"""GPU parity of pir_rowsel_grouped: uneven instances (own DB, own batch) in
one call, against the oracle word for word, against separate pir_rowsel calls,
and replayed from a captured hipGraph."""
import numpy as np
import pytest

import oracle
import synth
from helpers import device_db, device_query, empty_u32, np_u32, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pir():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_04696_amd as pkg
    pkg.lib()
    return pkg


# (N, D0, D1, B): ragged sizes, a B = 0 item, one- and many-client items
SMALL = [(64, 37, 300, 3), (32, 64, 16, 1), (64, 130, 33, 17), (16, 5, 70, 0),
         (64, 96, 128, 40), (32, 200, 9, 2)]


def _small_items(pir):
    primes = synth.PRIMES_N4096
    items, wants = [], []
    for i, (n, d0, d1, B) in enumerate(SMALL):
        coeffs = synth.db_coeffs(60 + i, d0, d1, 2, n)
        query = synth.query_uniform(70 + i, B, d0, primes, n)
        db = pir.pir_db_create(pir.make_params(n, primes, d0, d1))
        pir.pir_db_load_ntt(db, to_dev(coeffs), domain=pir.PIR_DOMAIN_COEFF)
        out = empty_u32(max(1, B * 2 * d1 * 2 * n))
        out.fill_(-1)
        q = to_dev(query) if B else empty_u32(1)
        items.append((db, q, B, out))
        wants.append(oracle.rowsel(query, oracle.ntt_db(coeffs, primes), primes) if B else None)
    return items, wants


@pytest.mark.parametrize("path", [1, 2], ids=["valu", "mfma"])
def test_grouped_matches_oracle(pir, path):
    print("grouped small path", path, flush=True)
    items, wants = _small_items(pir)
    pir.pir_rowsel_grouped(items, path)
    torch.cuda.synchronize()
    for (db, q, B, out), want in zip(items, wants):
        if B:
            got = np_u32(out)[: want.size].reshape(want.shape)
            assert np.array_equal(got, want)
        else:
            assert np.all(np_u32(out) == 0xFFFFFFFF)      # untouched


def test_grouped_graph_replay(pir):
    print("grouped graph capture", flush=True)
    items, wants = _small_items(pir)
    pir.pir_rowsel_grouped(items, pir.PIR_PATH_MFMA_I8)      # builds the plan outside capture
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        pir.pir_rowsel_grouped(items, pir.PIR_PATH_MFMA_I8)
    torch.cuda.synchronize()
    for rep in range(3):
        for _, _, B, out in items:
            if B:
                out.fill_(0)                                # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for (db, q, B, out), want in zip(items, wants):
            if B:
                got = np_u32(out)[: want.size].reshape(want.shape)
                assert np.array_equal(got, want), f"replay {rep} differs"


def test_grouped_tile_choice(pir, monkeypatch):
    """The plan keeps a tile shape, timed or forced, and any shape gives the
    same bits."""
    items, wants = _small_items(pir)
    with pytest.raises(pir.PirError, match="no grouped plan"):
        pir.pir_rowsel_grouped_tile(items[:3])
    outs = {}
    for forced in ("", "4", "2"):
        monkeypatch.setenv("PIR_MFMA_WM", forced)
        for _, _, B, out in items:
            out.fill_(0)
        pir.pir_rowsel_grouped(items[:3], pir.PIR_PATH_MFMA_I8)
        torch.cuda.synchronize()
        tm, tn = pir.pir_rowsel_grouped_tile(items[:3])
        assert (tm, tn) in ((128, 64), (64, 128))
        if forced:
            assert tm == 32 * int(forced)
        for (db, q, B, out), want in zip(items[:3], wants[:3]):
            if B:
                assert np.array_equal(np_u32(out)[: want.size].reshape(want.shape), want), forced
    monkeypatch.delenv("PIR_MFMA_WM")


def test_grouped_first_call_refuses_capture(pir):
    items, _ = _small_items(pir)
    items = items[:2]
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with pytest.raises(pir.PirError, match="cannot be captured"):
        with torch.cuda.graph(g, stream=s):
            pir.pir_rowsel_grouped(items, pir.PIR_PATH_MFMA_I8)
    torch.cuda.synchronize()


def test_grouped_rejects_overlapping_outputs(pir):
    items, _ = _small_items(pir)
    db, q, B, out = items[0]
    with pytest.raises(pir.PirError, match="overlap"):
        pir.pir_rowsel_grouped([(db, q, B, out), (db, q, B, out)])


def test_grouped_full_size_sampled(pir):
    """The 24 uneven instances (N = 4096, two primes) in one call; each
    instance is checked against the oracle on two sampled columns of its
    first and last client, and the whole call equals separate calls."""
    insts = synth.grouped_instances()
    items = []
    for it in insts:
        print("building instance", it.index, it.d0, it.d1, it.clients, flush=True)
        db = device_db(pir, it.n, it.primes, it.d0, it.d1, it.seed, pir.PIR_LAYOUT_MFMA, sub=it.index)
        q = device_query(pir, it.clients, it.d0, it.primes, it.n, it.seed, sub=it.index)
        out = empty_u32(it.clients * 2 * it.d1 * 2 * it.n)
        items.append((db, q, it.clients, out))
    print("grouped call", flush=True)
    pir.pir_rowsel_grouped(items, pir.PIR_PATH_MFMA_I8)
    torch.cuda.synchronize()
    for it, (db, q, B, out) in zip(insts, items):
        sep = empty_u32(out.numel())
        pir.pir_rowsel(db, q, sep, pir.PIR_PATH_MFMA_I8)
        torch.cuda.synchronize()
        assert torch.equal(sep, out), f"instance {it.index}: grouped != separate"
        cols = [0, it.d1 - 1]
        clients = sorted({0, B - 1})
        coeffs = synth.db_coeffs(it.seed, it.d0, it.d1, 2, it.n, sub=it.index, cols=cols)
        qv = synth.query_uniform(it.seed, B, it.d0, it.primes, it.n, sub=it.index, clients=clients)
        want = oracle.rowsel(qv, oracle.ntt_db(coeffs, it.primes), it.primes)
        got = np_u32(out).reshape(B, 2, it.d1, 2, it.n)[clients][:, :, cols]
        assert np.array_equal(got, want), f"instance {it.index} differs from the oracle"
        del sep
    for db, q, B, out in items:
        pir.pir_db_free(db)
