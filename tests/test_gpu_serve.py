"""GPU tests of the continuous-batching server: every completed request's
output equals the oracle's RowSel of its query (also with steps whose
active rows reach every step kernel, up to 80 clients at once), a request
gives the same bits alone and in a mix, requests arriving while others run
are admitted, malformed requests fail alone, and the HBM budget bounds the
capacity."""
import time

import numpy as np
import pytest

import oracle
import synth
from helpers import empty_u32, np_u32, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N, PR, D0, D1 = 64, synth.PRIMES_N4096, 40, 50


@pytest.fixture(scope="module")
def pir():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_04696_amd as pkg
    pkg.lib()
    return pkg


@pytest.fixture(scope="module")
def served(pir):
    coeffs = synth.db_coeffs(80, D0, D1, 2, N)
    dhat = oracle.ntt_db(coeffs, PR)
    db = pir.pir_db_create(pir.make_params(N, PR, D0, D1), pir.PIR_LAYOUT_MFMA)
    pir.pir_db_load_ntt(db, to_dev(dhat), domain=pir.PIR_DOMAIN_NTT)
    torch.cuda.synchronize()
    queries = synth.query_uniform(81, 12, D0, PR, N)          # 12 distinct clients
    wants = oracle.rowsel(queries, dhat, PR)
    return db, queries, wants


def run_until(pir, srv, schedule, expect, timeout=60.0):
    """schedule: {turn: [(id, q, out), ...]}; loops serve_step until `expect`
    completions arrived."""
    got, turn, t0 = {}, 0, time.time()
    while len(got) < expect:
        for c in pir.pir_serve_step(srv, schedule.get(turn, ())):
            got[c.id] = c
        turn += 1
        if time.time() - t0 > timeout:
            raise TimeoutError(f"only {len(got)} of {expect} completions")
    return got


def test_serve_matches_oracle_with_staggered_arrivals(pir, served):
    db, queries, wants = served
    srv = pir.pir_server_create(db, max_clients=4, chunks=4, pipeline=2)
    outs = [empty_u32(2 * D1 * 2 * N) for _ in range(12)]
    qs = [to_dev(queries[i]) for i in range(12)]
    # requests arrive over several turns, while earlier ones are on the GPU
    schedule = {0: [(i, qs[i], outs[i]) for i in range(5)],
                1: [(i, qs[i], outs[i]) for i in range(5, 8)],
                3: [(i, qs[i], outs[i]) for i in range(8, 12)]}
    got = run_until(pir, srv, schedule, 12)
    torch.cuda.synchronize()
    st = pir.pir_server_get_stats(srv)
    assert st.capacity == 4 and st.admitted == 12 and st.completed == 12
    for i in range(12):
        c = got[i]
        assert c.status == 0
        assert c.t_submit <= c.t_admit <= c.t_done
        assert np.array_equal(np_u32(outs[i]).reshape(wants[i].shape), wants[i]), f"request {i}"
    pir.pir_server_destroy(srv)


def test_serve_alone_equals_in_mix(pir, served):
    db, queries, wants = served
    q7 = to_dev(queries[7])
    alone = empty_u32(2 * D1 * 2 * N)
    srv = pir.pir_server_create(db, max_clients=8, chunks=3)
    run_until(pir, srv, {0: [(7, q7, alone)]}, 1)
    pir.pir_server_destroy(srv)
    srv = pir.pir_server_create(db, max_clients=8, chunks=3)
    outs = {i: empty_u32(2 * D1 * 2 * N) for i in range(12)}
    schedule = {0: [(i, to_dev(queries[i]), outs[i]) for i in (0, 3, 9)],
                2: [(7, q7, outs[7])] + [(i, to_dev(queries[i]), outs[i]) for i in (1, 11, 4)]}
    run_until(pir, srv, schedule, 7)
    torch.cuda.synchronize()
    assert torch.equal(alone, outs[7])
    assert np.array_equal(np_u32(alone).reshape(wants[7].shape), wants[7])
    pir.pir_server_destroy(srv)


def test_serve_bad_request_fails_alone(pir, served):
    db, queries, wants = served
    srv = pir.pir_server_create(db, max_clients=2, chunks=2)
    good = empty_u32(2 * D1 * 2 * N)
    bad = empty_u32(2 * max(D0, D1) * 2 * N)      # query and output are the same buffer
    got = run_until(pir, srv, {0: [(1, bad, bad), (2, to_dev(queries[2]), good)]}, 2)
    assert got[1].status == pir.PIR_EINVAL
    assert got[2].status == 0
    torch.cuda.synchronize()
    assert np.array_equal(np_u32(good).reshape(wants[2].shape), wants[2])
    pir.pir_server_destroy(srv)


def test_serve_budget_bounds_capacity(pir, served):
    db, queries, wants = served
    big = pir.pir_server_create(db, max_clients=256)
    per_all = pir.pir_server_get_stats(big).device_bytes
    assert pir.pir_server_get_stats(big).capacity == 256
    pir.pir_server_destroy(big)
    small = pir.pir_server_create(db, max_clients=256, hbm_budget=per_all // 3)
    st = pir.pir_server_get_stats(small)
    assert 0 < st.capacity < 256 and st.device_bytes <= per_all // 3
    outs = [empty_u32(2 * D1 * 2 * N) for _ in range(6)]
    got = run_until(pir, small, {0: [(i, to_dev(queries[i]), outs[i]) for i in range(6)]}, 6)
    torch.cuda.synchronize()
    for i in range(6):
        assert got[i].status == 0
        assert np.array_equal(np_u32(outs[i]).reshape(wants[i].shape), wants[i])
    pir.pir_server_destroy(small)
    with pytest.raises(pir.PirError, match="holds no client"):
        pir.pir_server_create(db, max_clients=4, hbm_budget=1024)


def test_serve_many_clients_every_kernel(pir):
    """Steps whose active rows span the step kernels: up to 16 clients (tiled
    32-row shape), 17-32 (64-row query-resident units), 33-48 (96-row),
    49-64 (128-row) and more than 64 (query-resident row blocks), on a DB
    whose K spans four 64-row chunks; 150 requests arrive in waves and every
    output word is compared with the oracle."""
    n, primes, d0, d1 = 16, PR, 200, 40
    coeffs = synth.db_coeffs(82, d0, d1, 2, n)
    dhat = oracle.ntt_db(coeffs, primes)
    db = pir.pir_db_create(pir.make_params(n, primes, d0, d1), pir.PIR_LAYOUT_MFMA)
    pir.pir_db_load_ntt(db, to_dev(dhat), domain=pir.PIR_DOMAIN_NTT)
    count = 150
    queries = synth.query_uniform(83, count, d0, primes, n)
    wants = oracle.rowsel(queries, dhat, primes)
    qs = [to_dev(queries[i]) for i in range(count)]
    outs = [empty_u32(2 * d1 * 2 * n) for _ in range(count)]
    srv = pir.pir_server_create(db, max_clients=160, chunks=2)
    waves = [(0, 10), (10, 30), (30, 70), (70, 150)]   # the last 80 arrive at once
    schedule = {2 * t: [(i, qs[i], outs[i]) for i in range(a, b)] for t, (a, b) in enumerate(waves)}
    got = run_until(pir, srv, schedule, count)
    torch.cuda.synchronize()
    assert all(got[i].status == 0 for i in range(count))
    for i in range(count):
        g = np_u32(outs[i]).reshape(wants[i].shape)
        assert np.array_equal(g, wants[i]), f"request {i}: {(g != wants[i]).sum()} words differ"
    pir.pir_server_destroy(srv)
    pir.pir_db_free(db)


@pytest.mark.timeout(900)
def test_serve_full_size_every_word(pir):
    """The serving workload's DB (N = 4096, two primes, 1024 x 1024, 32 GiB)
    and its whole 32-query pool, served through pir_serve_step with 8 client
    slots (requests arrive over several turns, so most are admitted while
    others run); every output word of every request is compared with the
    oracle, which regenerates the DB and the pool from their seeds and runs
    its own NTT and RowSel on the host cores."""
    import time
    from helpers import device_db, host_db_ntt, host_query
    w = synth.SERVE_DB
    print("device: building the 32 GiB serving DB", flush=True)
    db = device_db(pir, w.n, w.primes, w.d0, w.d1, w.seed, pir.PIR_LAYOUT_MFMA)
    pool = []
    for i in range(32):
        q = empty_u32(2 * w.d0 * w.slots)
        pir.pir_synth_query(q, synth.stream_key(w.seed, synth.TAG_POOL, i), 0, 1, w.d0, w.primes, w.n)
        pool.append(q)
    outs = [empty_u32(2 * w.d1 * w.slots) for _ in range(32)]
    srv = pir.pir_server_create(db, max_clients=8, chunks=16)
    schedule = {t: [(i, pool[i], outs[i]) for i in range(4 * t, 4 * t + 4)] for t in range(8)}
    print("serving the 32 pool queries", flush=True)
    got = run_until(pir, srv, schedule, 32, timeout=300.0)
    torch.cuda.synchronize()
    st = pir.pir_server_get_stats(srv)
    pir.pir_server_destroy(srv)
    pir.pir_db_free(db)
    del pool
    assert all(got[i].status == 0 for i in range(32)) and st.completed == 32
    t = time.time()
    print("host: the oracle's NTT of the 32 GiB DB", flush=True)
    dhat = host_db_ntt(w.seed, w.d0, w.d1, w.primes, w.n)
    print(f"host: DB ready in {time.time() - t:.1f} s", flush=True)
    for c0 in range(0, 32, 8):
        # pool query i, regenerated on the host from its own seeded stream
        qh = np.concatenate([host_query(w.seed, 1, w.d0, w.primes, w.n, sub=i, tag=synth.TAG_POOL)
                             for i in range(c0, c0 + 8)])
        want = oracle.rowsel(qh, dhat, w.primes)
        for i in range(c0, c0 + 8):
            got_i = np_u32(outs[i]).reshape(1, 2, w.d1, 2, w.n)
            assert np.array_equal(got_i, want[i - c0: i - c0 + 1]), f"request {i}"
        print(f"requests {c0}..{c0 + 7}: every word equals the oracle ({time.time() - t:.1f} s)", flush=True)


def test_serve_duplicate_ids_rejected(pir, served):
    db, queries, wants = served
    srv = pir.pir_server_create(db, max_clients=2, chunks=2)
    q, out, out2 = to_dev(queries[0]), empty_u32(2 * D1 * 2 * N), empty_u32(2 * D1 * 2 * N)
    with pytest.raises(ValueError, match="already live"):
        pir.pir_serve_step(srv, [(5, q, out), (5, q, out2)])
    # the C call itself refuses a live id and queues nothing
    import ctypes
    arr = (pir.pir_request * 2)()
    for i, o in enumerate((out, out2)):
        arr[i].id, arr[i].q_dev, arr[i].out_dev, arr[i].ready_event = 9, q.data_ptr(), o.data_ptr(), None
    nd = ctypes.c_uint32()
    st = pir.lib().pir_serve_step(srv.handle, ctypes.cast(arr, ctypes.c_void_p), 2, None, 0, ctypes.byref(nd))
    assert st == pir.PIR_EINVAL and "already live" in pir.pir_last_error()
    assert pir.pir_server_get_stats(srv).waiting == 0 and pir.pir_server_get_stats(srv).admitted == 0
    got = run_until(pir, srv, {0: [(5, q, out)]}, 1)
    with pytest.raises(ValueError, match="already live"):
        pir.pir_serve_step(srv, [(6, q, out2), (6, q, out2)])
    torch.cuda.synchronize()
    assert got[5].status == 0
    assert np.array_equal(np_u32(out).reshape(wants[0].shape), wants[0])
    pir.pir_server_destroy(srv)


def test_serve_max_waiting_busy(pir, served):
    """With one slot and room for two waiting requests, a burst of five
    admits one, queues two and completes two at once with PIR_EBUSY."""
    db, queries, wants = served
    srv = pir.pir_server_create(db, max_clients=1, chunks=2, max_waiting=2)
    outs = [empty_u32(2 * D1 * 2 * N) for _ in range(5)]
    burst = [(i, to_dev(queries[i]), outs[i]) for i in range(5)]
    got = run_until(pir, srv, {0: burst}, 5)
    torch.cuda.synchronize()
    busy = sorted(i for i in range(5) if got[i].status == pir.PIR_EBUSY)
    ok = sorted(i for i in range(5) if got[i].status == 0)
    assert busy == [2, 3, 4] and ok == [0, 1]
    for i in ok:
        assert np.array_equal(np_u32(outs[i]).reshape(wants[i].shape), wants[i]), f"request {i}"
    pir.pir_server_destroy(srv)


def test_serve_reads_query_after_its_producer(pir, served):
    """The query is written by work still queued on torch's stream (a copy
    behind a GPU sleep) when it is submitted: the server waits for it."""
    db, queries, wants = served
    srv = pir.pir_server_create(db, max_clients=2, chunks=2)
    src = to_dev(queries[3])
    qbuf = torch.zeros_like(src)
    out = empty_u32(2 * D1 * 2 * N)
    torch.cuda.synchronize()
    torch.cuda._sleep(200_000_000)          # ~0.1 s of device time before the copy
    qbuf.copy_(src)
    got = run_until(pir, srv, {0: [(3, qbuf, out)]}, 1)
    torch.cuda.synchronize()
    assert got[3].status == 0
    assert np.array_equal(np_u32(out).reshape(wants[3].shape), wants[3])
    pir.pir_server_destroy(srv)
