"""RowSel benchmark on one MI355X.

Headline workload (one JSON line on stdout): RowSel of one client against an
N = 4096, two-prime, 512 x 512 NTT-domain database of 16-bit coefficients
(8 GiB), through the C ABI, VALU streaming path.  A step is one pir_rowsel
call (query in HBM -> output in HBM).  value = DB bytes streamed per second.

Extra figures on the same DB: 64 clients on the VALU and the INT8-MFMA
paths.  Beside them: the CPU oracle timed on a bounded sample of the
headline workload, and the roofline of the dominant kernel.
"""
from __future__ import annotations

import argparse
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


def cpu_baseline(w, target_s: float):
    """The oracle (unmodified) on a bounded sample of the headline workload:
    all 512 rows and all 8192 points of a subset of DB columns, one client,
    repeated until about `target_s` seconds of oracle RowSel time."""
    import numpy as np
    import oracle
    import synth
    cols = list(range(32))
    coeffs = synth.db_coeffs(w.dbseed, w.d0, w.d1, w.nprimes, w.n, cols=cols)
    dhat = oracle.ntt_db(coeffs, w.primes)
    q = synth.query_uniform(w.seed, 1, w.d0, w.primes, w.n)
    reps, t = 0, 0.0
    while t < target_s and reps < 1000:
        t0 = time.perf_counter()
        oracle.rowsel(q, dhat, w.primes)
        t += time.perf_counter() - t0
        reps += 1
    db_bytes = w.slots * w.d0 * len(cols) * 4 * reps
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": db_bytes / t / 1e9, "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": f"RowSel of DB columns 0-{len(cols) - 1} (all {w.d0} rows, {w.slots} points, "
                      f"1 client), repeated {reps}x, {t:.1f} s of oracle time",
            "mac_per_s": w.slots * 2 * w.d0 * len(cols) * reps / t}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-client figures")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 1 GiB read + 1 GiB write elementwise kernel (bitwise_not) "
                         "so HBM byte counters can be scaled against a kernel of known traffic")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
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
    st = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(st)
        step()
        b.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms = [a.elapsed_time(b) for a, b in evs]
    log(f"B=1 VALU: wall {wall / args.steps * 1e3:.3f} ms/step, kernel mean {statistics.mean(kms):.3f} ms")

    ms_step = wall / args.steps * 1e3
    db_gbs = w.db_bytes / (ms_step * 1e-3) / 1e9
    kmean = statistics.mean(kms)
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
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "rowsel_stream_kernel<2>", "kernel_ms": round(kmean, 4),
                     "alg_bytes_per_launch": alg_bytes},
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
        res["mfma_over_valu"] = round(res["valu"]["ms"] / m["ms"], 2)
        line["batched_b64"] = res
        del qb, ob

    if not args.no_cpu:
        log("CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)

    pir.pir_db_free(db)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
