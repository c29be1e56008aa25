"""Helpers shared by the GPU tests (inputs from ``synth``, expectations from
``oracle``; nothing here computes RowSel)."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle
import synth


def np_u32(t):
    return t.detach().cpu().numpy().view(np.uint32)


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


def empty_u32(count):
    import torch
    return torch.empty(int(count), dtype=torch.int32, device="cuda")


def device_db(pir, n, primes, d0, d1, seed, layouts, chunk_rows=None, sub=0):
    """DB built on the device: seeded coefficients (pir_synth_db_coeffs, the
    device twin of synth.db_coeffs) loaded in the coefficient domain, so the
    library's own NTT produces the NTT-domain records."""
    import torch
    db = pir.pir_db_create(pir.make_params(n, primes, d0, d1), layouts)
    key = synth.stream_key(seed, synth.TAG_DB, sub)
    per_row = d1 * len(primes) * n
    chunk = chunk_rows or max(1, min(d0, (256 << 20) // (per_row * 4)))
    buf = empty_u32(chunk * per_row)
    for r0 in range(0, d0, chunk):
        nr = min(chunk, d0 - r0)
        view = buf[: nr * per_row]
        pir.pir_synth_db_coeffs(view, key, r0, nr, d1, len(primes), n)
        pir.pir_db_load_ntt(db, view, r0, nr, pir.PIR_DOMAIN_COEFF)
    torch.cuda.synchronize()
    return db


def device_query(pir, B, d0, primes, n, seed, sub=0):
    q = empty_u32(B * 2 * d0 * len(primes) * n)
    pir.pir_synth_query(q, synth.stream_key(seed, synth.TAG_QUERY, sub), 0, B, d0, primes, n)
    return q


# ---------------------------------------------------------------------------
# full-size host inputs for the oracle (thread-parallel generation; numpy
# releases the GIL inside its array operations)
def _workers():
    return max(1, min(16, os.cpu_count() or 4))


def host_db_ntt(seed, d0, d1, primes, n, sub=0, log=None):
    """The oracle's NTT-domain DB [D0][D1][L][N] for the seeded coefficients
    that pir_synth_db_coeffs produces on the device: coefficients from
    ``synth.db_coeffs`` in row blocks on a thread pool, then the oracle's own
    NTT of every limb."""
    L = len(primes)
    coeffs = np.empty((d0, d1, L, n), dtype=np.uint32)
    step = max(1, -(-d0 // (4 * _workers())))

    def fill(r0):
        r1 = min(d0, r0 + step)
        coeffs[r0:r1] = synth.db_coeffs(seed, d0, d1, L, n, sub=sub, rows=np.arange(r0, r1))

    with ThreadPoolExecutor(_workers()) as ex:
        list(ex.map(fill, range(0, d0, step)))
    if log:
        log(f"oracle NTT of {d0} x {d1} x {L} polynomials (N = {n})")
    return oracle.ntt_db(coeffs, primes)


def host_query(seed, B, d0, primes, n, sub=0, tag=synth.TAG_QUERY):
    """synth.query_uniform for all B clients, clients generated in parallel."""
    out = np.empty((B, 2, d0, len(primes), n), dtype=np.uint32)

    def fill(b):
        out[b] = synth.query_uniform(seed, B, d0, primes, n, sub=sub, clients=[b], tag=tag)[0]

    with ThreadPoolExecutor(_workers()) as ex:
        list(ex.map(fill, range(B)))
    return out


# ---------------------------------------------------------------------------
# guard bands: an output view with canary words on both sides, to show that a
# kernel writes inside its output and nowhere next to it
GUARD_WORDS = 256                      # 1 KiB each side (keeps 16-byte alignment)
CANARY = 0x5EC0DE42


def guarded_u32(count):
    """(buffer, view): `view` is `count` words in the middle of `buffer`,
    which has GUARD_WORDS canary words before and after it."""
    import torch
    buf = torch.full((int(count) + 2 * GUARD_WORDS,), CANARY, dtype=torch.int32, device="cuda")
    return buf, buf[GUARD_WORDS: GUARD_WORDS + int(count)]


def assert_guards(buf):
    import torch
    canary = torch.tensor(CANARY, dtype=torch.int32, device=buf.device)
    head, tail = buf[:GUARD_WORDS], buf[-GUARD_WORDS:]
    assert bool(torch.all(head == canary)) and bool(torch.all(tail == canary)), \
        "a kernel wrote into the guard band around its output"
