"""The grouped workload at full size: 24 uneven RowSel instances (N = 4096,
two primes, own DBs of 33 GiB in total, D0 in {32..512}, D1 in {16..256},
1..96 clients) in one pir_rowsel_grouped call on the MFMA path, eager and
replayed from a captured hipGraph (the launch the benchmark times).

Every output word of every instance is compared with the oracle (sec. 2.3),
which regenerates each instance's DB coefficients and queries from the same
seeds, transforms the DB with its own NTT and runs its RowSel on the host
cores.  The graph replays (two, with eager work between them) and separate
pir_rowsel calls must equal the eager outputs word for word."""
import time

import numpy as np
import pytest

import oracle
import synth
from helpers import assert_guards, device_db, device_query, empty_u32, guarded_u32, host_db_ntt, host_query, np_u32

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]
torch = pytest.importorskip("torch")

INSTS = synth.grouped_instances()
PARTS = 4


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
def grouped(pir):
    items, outs, guards = [], [], []
    for it in INSTS:
        log(f"device: instance {it.index} D0={it.d0} D1={it.d1} B={it.clients}")
        db = device_db(pir, it.n, it.primes, it.d0, it.d1, it.seed, pir.PIR_LAYOUT_MFMA, sub=it.index)
        q = device_query(pir, it.clients, it.d0, it.primes, it.n, it.seed, sub=it.index)
        guard, out = guarded_u32(it.clients * 2 * it.d1 * 2 * it.n)
        items.append((db, q, it.clients, out))
        outs.append(out)
        guards.append(guard)
    log("grouped call (eager; builds the plan)")
    pir.pir_rowsel_grouped(items, pir.PIR_PATH_MFMA_I8)
    torch.cuda.synchronize()
    for g in guards:
        assert_guards(g)

    # capture the same call into a graph writing to other buffers, replay it
    # twice with eager work in between, compare each replay with eager
    log("graph capture and two replays")
    rep_outs = [empty_u32(o.numel()) for o in outs]
    rep_items = [(db, q, B, ro) for (db, q, B, _), ro in zip(items, rep_outs)]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        pir.pir_rowsel_grouped(rep_items, pir.PIR_PATH_MFMA_I8)
    torch.cuda.synchronize()
    replay_equal = []
    for rep in range(2):
        for ro in rep_outs:
            ro.fill_(rep + 1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        replay_equal.append([torch.equal(ro, o) for ro, o in zip(rep_outs, outs)])
    del g, rep_outs, rep_items

    log("separate pir_rowsel calls")
    separate_equal = []
    for (db, q, B, out) in items:
        sep = empty_u32(out.numel())
        pir.pir_rowsel(db, q, sep, pir.PIR_PATH_MFMA_I8)
        torch.cuda.synchronize()
        separate_equal.append(torch.equal(sep, out))
        del sep
    yield dict(items=items, replay_equal=replay_equal, separate_equal=separate_equal)
    for db, q, B, out in items:
        pir.pir_db_free(db)


@pytest.mark.parametrize("part", range(PARTS))
def test_grouped_every_word(pir, grouped, part):
    for it in INSTS[part::PARTS]:
        t = time.time()
        i = it.index
        dhat = host_db_ntt(it.seed, it.d0, it.d1, it.primes, it.n, sub=i)
        qh = host_query(it.seed, it.clients, it.d0, it.primes, it.n, sub=i)
        want = oracle.rowsel(qh, dhat, it.primes)
        del dhat, qh
        got = np_u32(grouped["items"][i][3]).reshape(want.shape)
        if not np.array_equal(got, want):
            bad = np.argwhere(got != want)
            raise AssertionError(f"instance {i}: {len(bad)} words differ from the oracle, first at {bad[0].tolist()}")
        log(f"instance {i} (D0={it.d0} D1={it.d1} B={it.clients}): "
            f"{want.size} words equal the oracle ({time.time() - t:.1f} s on the host)")
        assert grouped["replay_equal"][0][i] and grouped["replay_equal"][1][i], f"instance {i}: graph replay differs"
        assert grouped["separate_equal"][i], f"instance {i}: separate pir_rowsel differs"
