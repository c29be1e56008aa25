"""GPU parity of pir_rowsel_grouped: uneven instances (own DB, own batch) in
one call, against the oracle word for word, against separate pir_rowsel calls,
and replayed from a captured hipGraph."""
import numpy as np
import pytest

import oracle
import synth
from helpers import assert_guards, empty_u32, guarded_u32, np_u32, to_dev

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


SHAPES = [(1, 128, 64), (1, 64, 128), (1, 32, 256), (1, 256, 32), (2, 64, 64), (2, 32, 128), (2, 128, 32)]
QRES_UNITS = [(1, 32, 128), (1, 64, 128), (1, 96, 64), (1, 128, 64)]


def test_grouped_tile_choice(pir, monkeypatch):
    """Every item of a plan gets a tile shape, timed, geometric or forced, and
    every shape gives the oracle's bits."""
    items, wants = _small_items(pir)
    with pytest.raises(pir.PirError, match="no grouped plan"):
        pir.pir_rowsel_grouped_tiles(items)
    settings = [("", "")] + [("", "0")] + [(",".join(map(str, s)), "") for s in SHAPES]
    for forced, tune in settings:
        monkeypatch.setenv("PIR_GROUPED_SHAPE", forced)
        monkeypatch.setenv("PIR_AUTOTUNE", tune)
        for _, _, B, out in items:
            out.fill_(-1)
        pir.pir_rowsel_grouped(items, pir.PIR_PATH_MFMA_I8)
        torch.cuda.synchronize()
        tiles = pir.pir_rowsel_grouped_tiles(items)
        for (db, q, B, out), want, t in zip(items, wants, tiles):
            if not B:
                assert t == (0, 0, 0, 0, 0) and np.all(np_u32(out) == 0xFFFFFFFF)
                continue
            assert (t[3] < 2 and t[:3] in SHAPES) or (t[3] == 2 and t[:3] in QRES_UNITS and t[4] == 1)
            if forced:
                assert ",".join(map(str, t[:3])) == forced and t[3] < 2
            assert np.array_equal(np_u32(out)[: want.size].reshape(want.shape), want), (forced, tune, t)
    monkeypatch.delenv("PIR_GROUPED_SHAPE")
    monkeypatch.delenv("PIR_AUTOTUNE")


RINGS = [(s, "wide") for s in SHAPES] + [(s, "deep") for s in SHAPES if s[0] * (s[1] + s[2]) == 192]


@pytest.mark.parametrize("shape,ring", RINGS, ids=["x".join(map(str, s)) + "-" + r for s, r in RINGS])
def test_grouped_shape_long_k_and_extremes(pir, monkeypatch, shape, ring):
    """Each tile shape, in each pipeline ring it fits, on a K of 2100 rows
    (two int32 accumulation chunks), all-(q-1) residues (every output equals
    D0 mod q, since (q-1)^2 = 1) and uniform residues, ragged D1 and batch."""
    monkeypatch.setenv("PIR_GROUPED_SHAPE", ",".join(map(str, shape)))
    monkeypatch.setenv("PIR_GROUPED_RING", ring)
    primes = synth.PRIMES_N4096
    n, d0 = 16, 2100
    cases = [(d0, 37, 5, "ones"), (d0, 70, 19, "uniform"), (100, 200, 3, "uniform")]
    items, wants, guards = [], [], []
    for i, (k, d1, B, kind) in enumerate(cases):
        if kind == "ones":
            dhat = np.broadcast_to(np.array(primes, np.uint32)[None, None, :, None] - 1, (k, d1, 2, n)).copy()
            query = np.broadcast_to(np.array(primes, np.uint32)[None, None, None, :, None] - 1,
                                    (B, 2, k, 2, n)).copy()
        else:
            dhat = oracle.ntt_db(synth.db_coeffs(40 + i, k, d1, 2, n), primes)
            query = synth.query_uniform(50 + i, B, k, primes, n)
        db = pir.pir_db_create(pir.make_params(n, primes, k, d1), pir.PIR_LAYOUT_MFMA)
        pir.pir_db_load_ntt(db, to_dev(dhat), domain=pir.PIR_DOMAIN_NTT)
        guard, out = guarded_u32(B * 2 * d1 * 2 * n)
        guards.append(guard)
        items.append((db, to_dev(query), B, out))
        want = oracle.rowsel(query, dhat, primes)
        if kind == "ones":
            assert np.all(want == np.array([k % q for q in primes], np.uint32)[None, None, None, :, None])
        wants.append(want)
    pir.pir_rowsel_grouped(items, pir.PIR_PATH_MFMA_I8)
    torch.cuda.synchronize()
    assert all(t[:3] == shape and t[3] == (0 if ring == "deep" else 1) for t in pir.pir_rowsel_grouped_tiles(items))
    for (db, q, B, out), want, guard in zip(items, wants, guards):
        assert np.array_equal(np_u32(out).reshape(want.shape), want), (shape, ring)
        assert_guards(guard)
    monkeypatch.delenv("PIR_GROUPED_SHAPE")
    monkeypatch.delenv("PIR_GROUPED_RING")


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


def test_grouped_graph_survives_other_plans_and_frees(pir):
    """A plan used under capture stays alive: freeing an unrelated DB and
    building more than the cache's worth of other plans leaves the graph's
    replays equal to the oracle."""
    items, wants = _small_items(pir)
    items, wants = items[:3], wants[:3]
    pir.pir_rowsel_grouped(items, pir.PIR_PATH_MFMA_I8)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        pir.pir_rowsel_grouped(items, pir.PIR_PATH_MFMA_I8)
    torch.cuda.synchronize()
    # an unrelated DB created and freed
    other = pir.pir_db_create(pir.make_params(16, synth.PRIMES_N4096, 8, 8))
    pir.pir_db_free(other)
    # ten other plans (one-item lists of distinct batch sizes) evict every
    # unpinned plan
    db0 = items[0][0]
    extra = empty_u32(10 * 2 * db0.d1 * 2 * db0.n)
    qz = to_dev(np.zeros((10, 2, db0.d0, 2, db0.n), np.uint32))
    for b in range(1, 11):
        pir.pir_rowsel_grouped([(db0, qz[: b * 2 * db0.d0 * 2 * db0.n], b, extra[: b * 2 * db0.d1 * 2 * db0.n])],
                               pir.PIR_PATH_MFMA_I8)
    assert np.all(np_u32(extra) == 0)
    torch.cuda.synchronize()
    for rep in range(2):
        for _, _, B, out in items:
            out.fill_(0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for (db, q, B, out), want in zip(items, wants):
            if B:
                got = np_u32(out)[: want.size].reshape(want.shape)
                assert np.array_equal(got, want), f"replay {rep} differs"


@pytest.mark.parametrize("sched", ["shared", "split"])
@pytest.mark.parametrize("ring,tune", [("qres", ""), ("qres", "0"), ("", "")], ids=["qres", "qres-untimed", "any"])
def test_grouped_kernels_and_schedules(pir, monkeypatch, ring, tune, sched):
    """The query-resident kernel in grouped plans (forced on every item whose
    D0 spans enough 64-row chunks: the others keep a tiled kernel) and both
    GEMM schedules (shared persistent launches, one launch per item), against
    the oracle word for word, then replayed from a captured graph."""
    monkeypatch.setenv("PIR_GROUPED_RING", ring)
    monkeypatch.setenv("PIR_AUTOTUNE", tune)
    monkeypatch.setenv("PIR_GROUPED_SCHED", sched)
    print("grouped kernels", ring, tune, sched, flush=True)
    items, wants = _small_items(pir)
    pir.pir_rowsel_grouped(items, pir.PIR_PATH_MFMA_I8)
    torch.cuda.synchronize()
    plan = pir.pir_rowsel_grouped_tiles(items)
    for (db, q, B, out), want, t, (n, d0, d1, _) in zip(items, wants, plan, SMALL):
        if not B:
            assert t == (0, 0, 0, 0, 0)
            continue
        if ring == "qres":
            assert (t[3] == 2) == (d0 > 64), (d0, t)
        assert t[4] == (1 if t[3] == 2 or sched == "split" else 0), t
        assert np.array_equal(np_u32(out)[: want.size].reshape(want.shape), want), (ring, tune, sched, t)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        pir.pir_rowsel_grouped(items, pir.PIR_PATH_MFMA_I8)
    torch.cuda.synchronize()
    for rep in range(2):
        for _, _, B, out in items:
            if B:
                out.fill_(0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for (db, q, B, out), want in zip(items, wants):
            if B:
                assert np.array_equal(np_u32(out)[: want.size].reshape(want.shape), want), f"replay {rep}"
    del g
    for db, *_ in items:
        pir.pir_db_free(db)


@pytest.mark.parametrize("sched", ["shared", "split"])
def test_grouped_qres_long_k_and_extremes(pir, monkeypatch, sched):
    """The query-resident kernel in a grouped plan on a K of 4100 rows (flushes
    that add to what an earlier flush stored), all-(q-1) residues (every
    output D0 mod q), more than 128 rows (two row blocks) and ragged D1."""
    monkeypatch.setenv("PIR_GROUPED_RING", "qres")
    monkeypatch.setenv("PIR_GROUPED_SCHED", sched)
    primes = synth.PRIMES_N4096
    n = 16
    cases = [(4100, 37, 5, "ones"), (4100, 70, 70, "uniform"), (300, 200, 9, "uniform"), (130, 33, 17, "ones")]
    items, wants, guards = [], [], []
    for i, (k, d1, B, kind) in enumerate(cases):
        if kind == "ones":
            dhat = np.broadcast_to(np.array(primes, np.uint32)[None, None, :, None] - 1, (k, d1, 2, n)).copy()
            query = np.broadcast_to(np.array(primes, np.uint32)[None, None, None, :, None] - 1,
                                    (B, 2, k, 2, n)).copy()
        else:
            dhat = oracle.ntt_db(synth.db_coeffs(80 + i, k, d1, 2, n), primes)
            query = synth.query_uniform(90 + i, B, k, primes, n)
        db = pir.pir_db_create(pir.make_params(n, primes, k, d1), pir.PIR_LAYOUT_MFMA)
        pir.pir_db_load_ntt(db, to_dev(dhat), domain=pir.PIR_DOMAIN_NTT)
        guard, out = guarded_u32(B * 2 * d1 * 2 * n)
        guards.append(guard)
        items.append((db, to_dev(query), B, out))
        want = oracle.rowsel(query, dhat, primes)
        if kind == "ones":
            assert np.all(want == np.array([k % q for q in primes], np.uint32)[None, None, None, :, None])
        wants.append(want)
    print("grouped qres long k", sched, flush=True)
    pir.pir_rowsel_grouped(items, pir.PIR_PATH_MFMA_I8)
    torch.cuda.synchronize()
    assert all(t[3] == 2 and t[4] == 1 for t in pir.pir_rowsel_grouped_tiles(items))
    for (db, q, B, out), want, guard in zip(items, wants, guards):
        assert np.array_equal(np_u32(out).reshape(want.shape), want), sched
        assert_guards(guard)
    for db, *_ in items:
        pir.pir_db_free(db)
