"""Helpers shared by the GPU tests (inputs from ``synth``, expectations from
``oracle``; nothing here computes RowSel)."""
import numpy as np

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
