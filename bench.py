"""RowSel benchmark on one MI355X.

Headline workload (one JSON line on stdout): RowSel of one client against an
N = 4096, two-prime, 512 x 512 NTT-domain database of 16-bit coefficients
(8 GiB), through the C ABI, VALU streaming path.  A step is one pir_rowsel
call (query in HBM -> output in HBM).  value = DB bytes streamed per second.

Further figures in the same line:
  batched_b64  64 clients on the same DB, VALU and INT8-MFMA paths;
  grouped      24 uneven instances (own DBs) in one pir_rowsel_grouped call,
               eager and replayed from a captured hipGraph;
  serving      a 1024 x 1024 (32 GiB) DB behind pir_serve_step, Poisson
               arrivals, queries/s and p50/p99 latency;
  cpu_baseline the CPU oracle on a bounded sample of the headline workload;
  roofline     of the headline kernel (traffic from the committed counter
               summary when the kernel source is unchanged since it was taken).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, datasheet
I8_PEAK_TOPS = 5000.0          # dense INT8 MFMA, TOP/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_db(pir, w, layouts):
    import torch
    import synth
    db = pir.pir_db_create(pir.make_params(w.n, w.primes, w.d0, w.d1), layouts)
    key = synth.stream_key(w.dbseed, synth.TAG_DB)
    per_row = w.d1 * w.nprimes * w.n
    chunk = max(1, (512 << 20) // (per_row * 4))
    buf = torch.empty(chunk * per_row, dtype=torch.int32, device="cuda")
    for r0 in range(0, w.d0, chunk):
        nr = min(chunk, w.d0 - r0)
        v = buf[: nr * per_row]
        pir.pir_synth_db_coeffs(v, key, r0, nr, w.d1, w.nprimes, w.n)
        pir.pir_db_load_ntt(db, v, r0, nr, pir.PIR_DOMAIN_COEFF)
    torch.cuda.synchronize()
    del buf
    return db


def make_query(pir, w, B, seed):
    import torch
    import synth
    q = torch.empty(B * 2 * w.d0 * w.slots, dtype=torch.int32, device="cuda")
    pir.pir_synth_query(q, synth.stream_key(seed, synth.TAG_QUERY), 0, B, w.d0, w.primes, w.n)
    return q


def timed_calls(fn, reps):
    """Per-call device time (ms) from events on the current stream."""
    import torch
    st = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for a, b in ev:
        a.record(st)
        fn()
        b.record(st)
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in ev]


PROFILE = os.path.join(ROOT, "profiles", "rowsel_stream_kernel_n4096_l2_512x512_b1.md")
# the headline kernel and the headers it is compiled with
STREAM_SRCS = [os.path.join(ROOT, "paper_2604_04696_amd", "csrc", f)
               for f in ("rowsel_stream.hip", "modarith.h", "common.h")]


def stream_source_sha256():
    h = hashlib.sha256()
    for f in STREAM_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the headline kernel from the committed counter
    summary, or None when the kernel's sources changed since it was measured."""
    try:
        text = open(PROFILE).read()
        rec = json.loads(text.split("<!-- traffic ")[1].split(" -->")[0])
        return rec["traffic_bytes"] if rec["source_sha256"] == stream_source_sha256() else None
    except (OSError, IndexError, KeyError, ValueError):
        return None


def grouped_section(pir, reps: int):
    """24 uneven instances in one pir_rowsel_grouped call (MFMA path)."""
    import torch
    import synth
    insts = synth.grouped_instances()
    items, macs, dbb = [], 0, 0
    for it in insts:
        w = synth.Workload(f"g{it.index}", it.seed, it.n, it.primes, it.d0, it.d1, it.clients, "uniform")
        db = pir.pir_db_create(pir.make_params(it.n, it.primes, it.d0, it.d1), pir.PIR_LAYOUT_MFMA)
        key = synth.stream_key(it.seed, synth.TAG_DB, it.index)
        per_row = it.d1 * 2 * it.n
        buf = torch.empty(it.d0 * per_row, dtype=torch.int32, device="cuda")
        pir.pir_synth_db_coeffs(buf, key, 0, it.d0, it.d1, 2, it.n)
        pir.pir_db_load_ntt(db, buf, 0, it.d0, pir.PIR_DOMAIN_COEFF)
        del buf
        q = torch.empty(it.clients * 2 * it.d0 * w.slots, dtype=torch.int32, device="cuda")
        pir.pir_synth_query(q, synth.stream_key(it.seed, synth.TAG_QUERY, it.index), 0, it.clients, it.d0,
                            it.primes, it.n)
        out = torch.empty(it.clients * 2 * it.d1 * w.slots, dtype=torch.int32, device="cuda")
        items.append((db, q, it.clients, out))
        macs += w.macs
        dbb += w.db_bytes
    fn = lambda: pir.pir_rowsel_grouped(items, pir.PIR_PATH_MFMA_I8)
    fn()
    torch.cuda.synchronize()
    eager = statistics.median(timed_calls(fn, reps))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        fn()
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    graph = statistics.median(timed_calls(g.replay, reps))
    res = {"instances": len(insts), "mod_macs": macs, "db_gib": round(dbb / 2**30, 2),
           "eager_ms": round(eager, 3), "graph_ms": round(graph, 3),
           "mac_per_s": macs / (graph * 1e-3), "db_gbs": round(dbb / (graph * 1e-3) / 1e9, 1)}
    plan = pir.pir_rowsel_grouped_tiles(items)
    # points x rows x columns per instance, its kernel, "+" when its GEMM has a launch of its own
    res["tiles"] = [f"{pir.GROUPED_KERNELS[k]}:{p}x{m}x{n}{'+' if alone else ''}" for p, m, n, k, alone in plan]
    shared = {(k, m) for p, m, n, k, alone in plan if not alone and k == 0} | \
             {k for p, m, n, k, alone in plan if not alone and k == 1}
    res["launches"] = 2 * len(insts) + len(shared) + sum(alone for *_, alone in plan)
    res["tile_note"] = ("per instance, timed at plan build: fixed-shape and shaped tiled kernels (shapes within "
                        "25% of the fewest padded words) and the query-resident kernel; shared launches or one "
                        "per instance, timed")
    # output words the GEMM computes (tile padding included) against the
    # 2B x D1 it needs, per point and K row (query rows are padded to 32)
    useful = computed = 0
    for it, (p, m, n, _, _) in zip(insts, plan):
        mp = (2 * it.clients + 31) // 32 * 32
        useful += 2 * it.clients * it.d1 * it.d0
        computed += (mp + m - 1) // m * m * ((it.d1 + n - 1) // n * n) * it.d0
    res["useful_over_computed"] = round(useful / computed, 3)
    del g
    for db, q, B, out in items:
        pir.pir_db_free(db)
    return res


def serving_section(pir, n_requests: int, rates):
    """pir_serve_step over the 1024 x 1024 DB: saturated throughput with the
    admission cap full, then seeded Poisson streams at each of the frozen
    `rates` (queries/s; 0.7x and 0.9x the saturated rate as calibrated once,
    synth.SERVE_RATES_QPS)."""
    import numpy as np
    import torch
    import synth
    w = synth.SERVE_DB
    db = build_db(pir, w, pir.PIR_LAYOUT_MFMA)
    pool = [make_query_sub(pir, w, i) for i in range(32)]
    nring = 512
    outs = [torch.empty(2 * w.d1 * w.slots, dtype=torch.int32, device="cuda") for _ in range(nring)]
    chunks = 16
    srv = pir.pir_server_create(db, max_clients=256, chunks=chunks, pipeline=1)
    cap = pir.pir_server_get_stats(srv).capacity

    def drive(arrival_times, choice):
        """Feeds each request at its scheduled arrival time (host clock of
        the library); returns completions, the start time, the span and the
        number of active clients after every step."""
        t0 = pir.pir_clock()
        nxt, got, active = 0, [], []
        while len(got) < len(arrival_times):
            now = pir.pir_clock() - t0
            batch = []
            while nxt < len(arrival_times) and arrival_times[nxt] <= now:
                batch.append((nxt, pool[choice[nxt]], outs[nxt % nring]))
                nxt += 1
            got += pir.pir_serve_step(srv, batch)
            active.append(pir.pir_server_get_stats(srv).active)
        return got, t0, pir.pir_clock() - t0, active

    # untimed warm-up (first launches of the step kernels), then saturated:
    # twice the admission cap arrives at once
    drive(np.zeros(cap), np.arange(cap) % 32)
    sat_n = 2 * cap
    got, _, dt, _ = drive(np.zeros(sat_n), np.arange(sat_n) % 32)
    qps_sat = sat_n / dt
    runs = []
    same = True
    for lam in rates:
        arr = synth.poisson_arrivals(w.seed, lam, n_requests)
        choice = synth.pool_choice(w.seed, n_requests)
        got, t0, dt, active = drive(arr, choice)
        # latency from the scheduled arrival (includes the wait for the next step)
        lat = np.array([c.t_done - (t0 + arr[c.id]) for c in got])
        edges = [0, 1, 2, 4, 8, 16, 32, 64, 128, 256, 4097]
        hist = np.histogram(np.array(active), bins=edges)[0]
        runs.append({"offered_qps": round(lam, 1), "load_vs_this_run_saturated": round(lam / qps_sat, 3),
                     "requests": n_requests,
                     "qps": round(n_requests / dt, 1),
                     "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
                     "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
                     "all_ok": all(c.status == 0 for c in got),
                     "active_per_step_hist": {f"{a}-{b - 1}": int(h) for a, b, h in zip(edges, edges[1:], hist) if h}})
        # the last requests' outputs against the same query served alone
        torch.cuda.synchronize()
        for c in sorted(got, key=lambda c: c.id)[-4:]:
            ref = torch.empty_like(outs[0])
            pir.pir_rowsel(db, pool[choice[c.id]], ref, pir.PIR_PATH_MFMA_I8)
            torch.cuda.synchronize()
            same = same and torch.equal(ref, outs[c.id % nring])
    st = pir.pir_server_get_stats(srv)
    pir.pir_server_destroy(srv)
    pir.pir_db_free(db)
    return {"workload": w.name, "capacity": cap, "chunks": chunks, "saturated_qps": round(qps_sat, 1),
            "frozen_rates_qps": list(rates), "frozen_from_saturated_qps": synth.SERVE_SATURATED_QPS,
            "runs": runs, "in_mix_equals_alone": same, "steps": st.steps}


def peaks_section(pir):
    """Measured ceilings on this GPU (include/pir_peak.h): INT8 MFMA issue
    rate on zero and on changing operands (with the shader clock it ran at),
    the v_mad_u64_u32 rate, and a streaming read of 4 GiB.  Second of two
    runs each."""
    import torch
    res = {}
    for name, rnd in (("mfma_i8_zero", False), ("mfma_i8_random", True)):
        for _ in range(2):
            tops, mhz = pir.pir_peak_mfma_i8(200_000, rnd)
        res[name] = {"tops": round(tops, 1), "mhz": round(mhz)}
    for _ in range(2):
        gops, mhz = pir.pir_peak_valu_mad64(200_000)
    res["valu_mad64"] = {"gops": round(gops, 1), "mhz": round(mhz)}
    buf = torch.zeros(1 << 30, dtype=torch.int32, device="cuda")
    for _ in range(2):
        gbs = pir.pir_peak_hbm_read(buf)
    res["hbm_read_gbs"] = round(gbs, 1)
    del buf
    return res


def query_front_section(pir, db, w, q_ntt, out, ntt_domain_ms):
    """64 clients with the query in the coefficient domain (the same words as
    the NTT-domain query, read as coefficients): the fused front end
    (pir_rowsel_coeff, MFMA path) against the library's NTT helper on the
    query followed by pir_rowsel, and against pir_rowsel on an NTT-domain
    query (no transform)."""
    import torch
    rows = w.clients * 2 * w.d0
    # the helper transforms contiguous polynomials: each prime's limbs, gathered
    # once outside the timed calls (the same bytes as the interleaved query)
    srcs = [q_ntt.view(rows, w.nprimes, w.n)[:, l, :].contiguous() for l in range(w.nprimes)]
    dsts = [torch.empty_like(x) for x in srcs]

    def two_pass():   # transform, then RowSel (on q_ntt: the same work as on the transformed words)
        for l, q in enumerate(w.primes):
            pir.pir_ntt_forward(srcs[l], dsts[l], w.n, q)
        pir.pir_rowsel(db, q_ntt, out, pir.PIR_PATH_MFMA_I8)

    def fused():
        pir.pir_rowsel_coeff(db, q_ntt, out, pir.PIR_PATH_MFMA_I8)

    res = {}
    for name, fn in (("fused_ms", fused), ("ntt_then_rowsel_ms", two_pass)):
        fn()
        torch.cuda.synchronize()
        res[name] = round(statistics.median(timed_calls(fn, 7)), 3)
    res["ntt_domain_rowsel_ms"] = round(ntt_domain_ms, 3)
    res["query_gib"] = round(rows * w.slots * 4 / 2**30, 2)
    del srcs, dsts
    return res


def q108_section(pir):
    """The paper's RNS setting: four 27-bit limbs (Q ~ 2^108), D0 = 256,
    D1 = 512 (8 GiB DB); one client (streaming kernel) and a batch of 32 on
    both paths, median of event-timed calls."""
    import torch
    import synth
    w = synth.PAPER_Q108
    db = build_db(pir, w, pir.PIR_LAYOUT_VALU | pir.PIR_LAYOUT_MFMA)
    time.sleep(2.0)   # let the DB build's frees settle (see the headline)
    res = {"workload": w.name, "primes": list(w.primes), "d0": w.d0, "d1": w.d1, "db_gib": w.db_bytes / 2**30}
    for B, path, name in ((1, pir.PIR_PATH_VALU, "b1_valu"), (w.clients, pir.PIR_PATH_MFMA_I8, "b32_mfma_i8"),
                          (w.clients, pir.PIR_PATH_VALU, "b32_valu")):
        q = make_query(pir, w, B, w.seed)
        out = torch.empty(B * 2 * w.d1 * w.slots, dtype=torch.int32, device="cuda")
        fn = lambda: pir.pir_rowsel(db, q, out, path)
        fn()
        torch.cuda.synchronize()
        ms = statistics.median(timed_calls(fn, 10 if B == 1 else 5))
        macs = w.slots * 2 * B * w.d0 * w.d1
        res[name] = {"ms": round(ms, 3), "db_gbs": round(w.db_bytes / (ms * 1e-3) / 1e9, 1),
                     "mac_per_s": macs / (ms * 1e-3)}
        del q, out
    # the path at the paper's parameters end to end: 32 clients' selector
    # ciphertexts in the coefficient domain -> NTT + RowSel (MFMA) -> the first
    # ColTor stage on its 512 output columns (gadget z = 2^22, ell = 5)
    B, log2z, ell = w.clients, 22, 5
    qc = torch.empty(B * 2 * w.d0 * w.slots, dtype=torch.int32, device="cuda")
    pir.pir_synth_query(qc, synth.stream_key(w.seed, synth.TAG_QUERY, 3), 0, B, w.d0, w.primes, w.n)
    rs = torch.empty(B * 2 * w.d1 * w.slots, dtype=torch.int32, device="cuda")
    rg = torch.empty(B * 2 * ell * 2 * w.slots, dtype=torch.int32, device="cuda")
    pir.pir_synth_query(rg, synth.stream_key(w.seed, synth.TAG_QUERY, 4), 0, B * ell * 2, 1, w.primes, w.n)
    ct1 = torch.empty(B * 2 * (w.d1 // 2) * w.slots, dtype=torch.int32, device="cuda")

    def pipeline():
        pir.pir_rowsel_coeff(db, qc, rs, pir.PIR_PATH_MFMA_I8)
        pir.pir_coltor_stage(w.n, w.primes, rs, B, w.d1, rg, log2z, ell, ct1)

    pipeline()
    torch.cuda.synchronize()
    res["b32_coeff_rowsel_coltor1_ms"] = round(statistics.median(timed_calls(pipeline, 5)), 3)
    del qc, rs, rg, ct1
    pir.pir_db_free(db)
    return res


def w32_section(pir):
    """Two full 32-bit primes (products of residues up to 2^64) on the
    headline shape (N = 4096, 512 x 512, 8 GiB, both layouts): 1, 2 and 4
    clients on the streaming kernel, 32 on the tiled kernel and on the INT8
    MFMA path.  Median of event-timed calls."""
    import torch
    import synth
    w = synth.WIDE32
    db = build_db(pir, w, pir.PIR_LAYOUT_VALU | pir.PIR_LAYOUT_MFMA)
    time.sleep(2.0)
    res = {"workload": w.name, "primes": list(w.primes), "db_gib": w.db_bytes / 2**30}
    for B, reps, path, name in ((1, 10, pir.PIR_PATH_VALU, "b1_valu"), (2, 5, pir.PIR_PATH_VALU, "b2_valu"),
                                (4, 5, pir.PIR_PATH_VALU, "b4_valu"), (2, 5, pir.PIR_PATH_MFMA_I8, "b2_mfma_i8"),
                                (4, 5, pir.PIR_PATH_MFMA_I8, "b4_mfma_i8"), (32, 3, pir.PIR_PATH_VALU, "b32_valu"),
                                (32, 3, pir.PIR_PATH_MFMA_I8, "b32_mfma_i8")):
        q = make_query(pir, w, B, w.seed)
        out = torch.empty(B * 2 * w.d1 * w.slots, dtype=torch.int32, device="cuda")
        fn = lambda: pir.pir_rowsel(db, q, out, path)
        fn()
        torch.cuda.synchronize()
        ms = statistics.median(timed_calls(fn, reps))
        res[name] = {"ms": round(ms, 3), "db_gbs": round(w.db_bytes / (ms * 1e-3) / 1e9, 1),
                     "mac_per_s": w.slots * 2 * B * w.d0 * w.d1 / (ms * 1e-3)}
        del q, out
    pir.pir_db_free(db)
    return res


def coltor_section(pir, reps=5):
    """First ColTor stage at the paper's setting: 32 clients, the 512 RowSel
    output ciphertexts of each (N = 4096, four 27-bit limbs), gadget z = 2^22,
    ell = 5; random NTT-domain ciphertexts and RGSW rows.  Median of
    event-timed calls."""
    import torch
    import synth
    n, primes, log2z, ell, B, ncols = 4096, synth.PRIMES_Q108, 22, 5, 32, 512
    L = len(primes)
    ct = torch.empty(B * 2 * ncols * L * n, dtype=torch.int32, device="cuda")
    pir.pir_synth_query(ct, synth.stream_key(9, synth.TAG_QUERY), 0, B, ncols, primes, n)
    rg = torch.empty(B * 2 * ell * 2 * L * n, dtype=torch.int32, device="cuda")
    pir.pir_synth_query(rg, synth.stream_key(9, synth.TAG_QUERY, 1), 0, B * ell * 2, 1, primes, n)
    out = torch.empty(B * 2 * (ncols // 2) * L * n, dtype=torch.int32, device="cuda")
    fn = lambda: pir.pir_coltor_stage(n, primes, ct, B, ncols, rg, log2z, ell, out)
    fn()
    torch.cuda.synchronize()
    time.sleep(1.0)
    ms = statistics.median(timed_calls(fn, reps))
    nodes = B * ncols // 2
    io = (ct.numel() + rg.numel() + out.numel()) * 4
    # transforms per node: 2 polynomials x L limbs inverse, 2 x ell x L forward
    ntts = nodes * (2 * L + 2 * ell * L)
    res = {"workload": f"coltor_stage1_n{n}_l4q108_z{log2z}l{ell}_b{B}_{ncols}cols", "ms": round(ms, 3),
           "nodes": nodes, "nodes_per_s": nodes / (ms * 1e-3), "io_gib": round(io / 2**30, 3),
           "io_gbs": round(io / (ms * 1e-3) / 1e9, 1), "ntt_per_s": ntts / (ms * 1e-3),
           "butterflies_per_s": ntts * (n // 2) * (n.bit_length() - 1) / (ms * 1e-3)}
    # the whole tournament: log2(512) = 9 stages down to one ciphertext per
    # client (the same RGSW rows serve every stage here; the arithmetic is that
    # of distinct ones)
    bufs = [torch.empty(B * 2 * (ncols >> s) * L * n, dtype=torch.int32, device="cuda") for s in range(1, 10)]

    def tournament():
        cur, cols = ct, ncols
        for buf in bufs:
            pir.pir_coltor_stage(n, primes, cur, B, cols, rg, log2z, ell, buf)
            cur, cols = buf, cols // 2

    tournament()
    torch.cuda.synchronize()
    res["tournament_ms"] = round(statistics.median(timed_calls(tournament, 3)), 3)
    res["tournament_stages"] = len(bufs)
    del ct, rg, out, bufs
    return res


def make_query_sub(pir, w, sub):
    import torch
    import synth
    q = torch.empty(2 * w.d0 * w.slots, dtype=torch.int32, device="cuda")
    pir.pir_synth_query(q, synth.stream_key(w.seed, synth.TAG_POOL, sub), 0, 1, w.d0, w.primes, w.n)
    return q


def cpu_baseline(w, target_s: float):
    """The oracle (unmodified) on a bounded sample of the headline workload:
    all 512 rows and all 8192 points of a subset of DB columns, one client,
    repeated until about `target_s` seconds of oracle RowSel time on all host
    threads; then the same sample on one thread, and the whole tiny workload
    (N = 1024, 16 x 16, one client) on one thread."""
    import oracle
    import synth

    def timed(fn, budget):
        reps, t = 0, 0.0
        while t < budget and reps < 1000:
            t0 = time.perf_counter()
            fn()
            t += time.perf_counter() - t0
            reps += 1
        return reps, t

    cols = list(range(32))
    coeffs = synth.db_coeffs(w.dbseed, w.d0, w.d1, w.nprimes, w.n, cols=cols)
    dhat = oracle.ntt_db(coeffs, w.primes)
    q = synth.query_uniform(w.seed, 1, w.d0, w.primes, w.n)
    threads = oracle.max_threads()
    reps, t = timed(lambda: oracle.rowsel(q, dhat, w.primes), target_s)
    col_bytes = w.slots * w.d0 * len(cols) * 4
    col_macs = w.slots * 2 * w.d0 * len(cols)
    res = {"value": col_bytes * reps / t / 1e9, "unit": "GB/s", "cores": threads, "kind": "oracle",
           "sample": f"RowSel of DB columns 0-{len(cols) - 1} (all {w.d0} rows, {w.slots} points, "
                     f"1 client), repeated {reps}x, {t:.1f} s of oracle time",
           "mac_per_s": col_macs * reps / t}
    oracle.set_threads(1)
    try:
        reps1, t1 = timed(lambda: oracle.rowsel(q, dhat, w.primes), target_s / 2)
        res["one_core"] = {"gbs": round(col_bytes * reps1 / t1 / 1e9, 3), "mac_per_s": col_macs * reps1 / t1,
                           "sample": f"the same sample on one thread, {reps1}x, {t1:.1f} s"}
        tw = synth.TINY
        tq = synth.query_uniform(tw.seed, 1, tw.d0, tw.primes, tw.n)
        tdb = oracle.ntt_db(synth.db_coeffs(tw.seed, tw.d0, tw.d1, tw.nprimes, tw.n), tw.primes)
        repst, tt = timed(lambda: oracle.rowsel(tq, tdb, tw.primes), 1.0)
        res["tiny_one_core"] = {"ms_per_call": round(tt / repst * 1e3, 4), "mac_per_s": tw.macs * repst / tt,
                                "workload": tw.name}
    finally:
        oracle.set_threads(threads)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-client figures")
    ap.add_argument("--no-grouped", action="store_true", help="skip the grouped-instances figures")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving figures")
    ap.add_argument("--no-coltor", action="store_true", help="skip the ColTor-stage figures")
    ap.add_argument("--serve-requests", type=int, default=1024)
    ap.add_argument("--serve-rates", default=None,
                    help="offered Poisson rates in queries/s (default: the frozen 0.7x and 0.9x of the "
                         "calibrated saturated rate, synth.SERVE_RATES_QPS)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 1 GiB read + 1 GiB write elementwise kernel (bitwise_not) "
                         "so HBM byte counters can be scaled against a kernel of known traffic")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2604_04696_amd as pir
    import synth

    pir.lib()
    torch.cuda.set_device(0)
    if args.copy_calib:
        src = torch.zeros(1 << 28, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.bitwise_not(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    w, wb = synth.HBM, synth.BATCHED
    log("building DB", w.name)
    t0 = time.time()
    db = build_db(pir, w, pir.PIR_LAYOUT_VALU | pir.PIR_LAYOUT_MFMA)
    log(f"DB built in {time.time() - t0:.1f} s")

    # ---------------------------------------------------------- headline
    q1 = make_query(pir, w, 1, w.seed)
    out1 = torch.empty(2 * w.d1 * w.slots, dtype=torch.int32, device="cuda")

    def step():
        pir.pir_rowsel(db, q1, out1, pir.PIR_PATH_VALU)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # the DB load released its temporaries; HBM-bound kernels run ~4% slower
    # for a second or two after device memory is released, so let that pass
    # (setup, not part of a step: every timed call still allocates and frees
    # its own stream-ordered scratch)
    time.sleep(2.0)
    pir.pir_kernel_timing(True)      # HIP events around the streaming kernel, on its stream
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launches, ktotal = pir.pir_kernel_time_read()
    pir.pir_kernel_timing(False)
    if launches != args.steps:
        raise RuntimeError(f"timed {launches} kernel launches for {args.steps} steps")
    kmean = ktotal / launches
    # whole calls (kernel, output transpose, scratch), event-timed after the steps
    call_ms = statistics.mean(timed_calls(step, min(args.steps, 10)))
    log(f"B=1 VALU: wall {wall / args.steps * 1e3:.3f} ms/step, call {call_ms:.3f} ms, kernel {kmean:.3f} ms")

    # ------------------------------------------- measured HBM reference
    # a STREAM-style pass on the same GPU: 2 GiB read + 2 GiB written.  Taken
    # after the headline: releasing device memory slows HBM-bound kernels on
    # this GPU for up to a few seconds afterwards (about 4% on the streaming
    # kernel after a 4 GiB free), so nothing is freed before the timed steps.
    ref_src = torch.zeros(1 << 29, dtype=torch.int32, device="cuda")
    ref_dst = torch.empty_like(ref_src)
    for _ in range(2):
        torch.bitwise_not(ref_src, out=ref_dst)
    torch.cuda.synchronize()
    ref_ms = statistics.median(timed_calls(lambda: torch.bitwise_not(ref_src, out=ref_dst), 10))
    copy_gbs = 2 * ref_src.numel() * 4 / (ref_ms * 1e-3) / 1e9
    del ref_src, ref_dst
    torch.cuda.empty_cache()

    peaks = peaks_section(pir)
    log(f"measured peaks: {peaks}")

    ms_step = wall / args.steps * 1e3
    db_gbs = w.db_bytes / (ms_step * 1e-3) / 1e9
    alg_bytes = w.db_bytes + w.io_bytes
    achieved = alg_bytes / (kmean * 1e-3) / 1e9

    line = {
        "metric": "RowSel mod-q MAC/s + DB GB/s streamed at B=1/64; served-query p50/p99 latency",
        "value": round(db_gbs, 1),
        "unit": "GB/s (DB streamed, B=1)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32 residues, u64 accumulation",
        "data": "synthetic (seeded)",
        "config": {"workload": w.name, "n": w.n, "primes": list(w.primes), "d0": w.d0, "d1": w.d1,
                   "clients": 1, "path": "VALU", "db_gib": w.db_bytes / 2**30},
        "mac_per_s": w.macs / (ms_step * 1e-3),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
                     "kernel": "rowsel_stream_kernel<2, false>", "kernel_ms": round(kmean, 4),
                     "call_ms": round(call_ms, 4),
                     "alg_bytes_per_launch": alg_bytes,
                     "measured_copy_gbs": round(copy_gbs, 1),
                     "frac_of_measured_copy": round(achieved / copy_gbs, 4),
                     "measured_read_gbs": peaks["hbm_read_gbs"],
                     "frac_of_measured": round(achieved / peaks["hbm_read_gbs"], 4)},
        "measured_peaks": peaks,
    }

    # ------------------------------------------------------------ batched
    if not args.no_batched:
        qb = make_query(pir, wb, wb.clients, wb.seed)
        ob = torch.empty(wb.clients * 2 * wb.d1 * wb.slots, dtype=torch.int32, device="cuda")
        res = {}
        for name, path, reps in [("mfma_i8", pir.PIR_PATH_MFMA_I8, 10), ("valu", pir.PIR_PATH_VALU, 3)]:
            fn = lambda: pir.pir_rowsel(db, qb, ob, path)
            fn()
            torch.cuda.synchronize()
            ms = statistics.median(timed_calls(fn, reps))
            res[name] = {"ms": round(ms, 3), "mac_per_s": wb.macs / (ms * 1e-3),
                         "db_gbs": round(wb.db_bytes / (ms * 1e-3) / 1e9, 1)}
            log(f"B=64 {name}: {ms:.3f} ms")
        m = res["mfma_i8"]
        m["i8_tops"] = round(wb.macs * 16 * 2 / (m["ms"] * 1e-3) / 1e12, 1)
        m["mfma_frac"] = round(m["i8_tops"] / I8_PEAK_TOPS, 4)
        # against the measured MFMA loop on changing operands (the chip's
        # attainable INT8 rate under load), and the VALU path against the
        # measured v_mad_u64_u32 rate (one multiply-add per mod-MAC at least)
        m["frac_of_measured"] = round(m["i8_tops"] / peaks["mfma_i8_random"]["tops"], 4)
        v = res["valu"]
        v["frac_of_measured_mad64"] = round(v["mac_per_s"] / (peaks["valu_mad64"]["gops"] * 1e9), 4)
        res["mfma_over_valu"] = round(res["valu"]["ms"] / m["ms"], 2)
        line["batched_b64"] = res
        line["query_front_b64"] = query_front_section(pir, db, wb, qb, ob, m["ms"])
        log(f"query front end: {line['query_front_b64']}")
        del qb, ob

    pir.pir_db_free(db)
    del q1, out1
    torch.cuda.empty_cache()

    if not args.no_batched:
        line["q108"] = q108_section(pir)
        torch.cuda.empty_cache()
        log(f"four-limb setting: {line['q108']}")
        line["w32"] = w32_section(pir)
        torch.cuda.empty_cache()
        log(f"32-bit primes: {line['w32']}")

    if not args.no_coltor:
        line["coltor"] = coltor_section(pir)
        torch.cuda.empty_cache()
        log(f"ColTor stage: {line['coltor']}")

    if not args.no_grouped:
        log("grouped instances")
        line["grouped"] = grouped_section(pir, reps=5)
        torch.cuda.empty_cache()
        log(f"grouped: {line['grouped']}")

    if not args.no_serve:
        log("serving")
        line["serving"] = serving_section(pir, args.serve_requests,
                                          [float(x) for x in args.serve_rates.split(",")] if args.serve_rates
                                          else list(synth.SERVE_RATES_QPS))
        torch.cuda.empty_cache()
        log(f"serving: {line['serving']}")

    if not args.no_cpu:
        log("CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)

    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
