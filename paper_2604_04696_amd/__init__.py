"""Python binding of libpir.so (include/pir.h, include/pir_synth.h, include/pir_peak.h).

Argument marshalling only: every step of RowSel runs in the HIP library.
Tensors are torch device tensors (int32 or uint32, contiguous) whose data
pointers are handed to the C ABI; the HIP stream defaults to torch's current
stream.  The library must be built (``paper_2604_04696_amd.build.build()``);
every call raises if it is missing -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpir.so")

PIR_OK = 0
PIR_EINVAL = -1
PIR_ENOMEM = -2
PIR_EDEVICE = -3
PIR_EBUSY = -4
PIR_EUNSUPPORTED = -5
_STATUS = {0: "PIR_OK", -1: "PIR_EINVAL", -2: "PIR_ENOMEM", -3: "PIR_EDEVICE", -4: "PIR_EBUSY",
           -5: "PIR_EUNSUPPORTED"}

PIR_MAX_PRIMES = 4
PIR_DOMAIN_COEFF = 0
PIR_DOMAIN_NTT = 1
PIR_PATH_AUTO = 0
PIR_PATH_VALU = 1
PIR_PATH_MFMA_I8 = 2
PIR_LAYOUT_VALU = 1
PIR_LAYOUT_MFMA = 2


class PirError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {_STATUS.get(status, status)}: {msg}")
        self.status = status


class pir_params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("nprimes", ctypes.c_uint32),
                ("q", ctypes.c_uint32 * PIR_MAX_PRIMES), ("d0", ctypes.c_uint32),
                ("d1", ctypes.c_uint32)]


_u32, _u64, _vp, _i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int

# name -> (restype, argtypes); the list mirrors the public headers and is what
# the CPU symbol test checks against them
SIGNATURES = {
    "pir_db_create": (_i32, [ctypes.POINTER(pir_params), _u32, ctypes.POINTER(_vp)]),
    "pir_db_load_ntt": (_i32, [_vp, _vp, _u32, _u32, _i32, _vp]),
    "pir_db_params": (_i32, [_vp, ctypes.POINTER(pir_params)]),
    "pir_db_layouts": (_u32, [_vp]),
    "pir_db_free": (None, [_vp]),
    "pir_rowsel": (_i32, [_vp, _vp, _u32, _vp, _i32, _vp]),
    "pir_rowsel_coeff": (_i32, [_vp, _vp, _u32, _vp, _i32, _vp]),
    "pir_rowsel_noalloc": (_i32, [_vp, _vp, _u32, _vp, _vp]),
    "pir_rowsel_grouped": (_i32, [_vp, _u32, _i32, _vp]),
    "pir_coltor_stage": (_i32, [ctypes.POINTER(pir_params), _vp, _u32, _u32, _vp, _u32, _u32, _vp, _vp]),
    "pir_rowsel_grouped_tiles": (_i32, [_vp, _u32, ctypes.POINTER(_u32)]),
    "pir_clock": (ctypes.c_double, []),
    "pir_server_create": (_i32, [_vp, _vp, ctypes.POINTER(_vp)]),
    "pir_serve_step": (_i32, [_vp, _vp, _u32, _vp, _u32, ctypes.POINTER(_u32)]),
    "pir_server_get_stats": (_i32, [_vp, _vp]),
    "pir_server_destroy": (None, [_vp]),
    "pir_ntt_forward": (_i32, [_vp, _vp, _u32, _u32, _u32, _vp]),
    "pir_ntt_inverse": (_i32, [_vp, _vp, _u32, _u32, _u32, _vp]),
    "pir_kernel_timing": (_i32, [_i32]),
    "pir_kernel_time_read": (_i32, [ctypes.POINTER(_u32), ctypes.POINTER(ctypes.c_double)]),
    "pir_last_error": (ctypes.c_char_p, []),
    "pir_version": (ctypes.c_char_p, []),
    "pir_peak_mfma_i8": (_i32, [_u32, _i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                _vp]),
    "pir_peak_valu_mad64": (_i32, [_u32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), _vp]),
    "pir_peak_hbm_read": (_i32, [_vp, _u64, ctypes.POINTER(ctypes.c_double), _vp]),
    "pir_synth_query": (_i32, [_vp, _u64, _u32, _u32, _u32, _u32, _u32,
                               ctypes.POINTER(_u32), _vp]),
    "pir_synth_db_coeffs": (_i32, [_vp, _u64, _u32, _u32, _u32, _u32, _u32, _vp]),
    "pir_synth_draw": (_i32, [_vp, _u64, _u64, _u64, _vp]),
}

_lib = None


def lib():
    """Load libpir.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "paper_2604_04696_amd.build.build() (there is no fallback)")
        # torch's HIP runtime is loaded first so that libpir.so binds to it:
        # the library takes torch's device memory and streams, and loading it
        # ahead of torch left torch without a visible GPU
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(st: int, where: str):
    if st != PIR_OK:
        raise PirError(st, where, lib().pir_last_error().decode())


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def _ptr(t, what: str):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{what} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return t.data_ptr()


def _need_u32(t, what: str):
    import torch
    if t.dtype not in (torch.int32, torch.uint32):
        raise TypeError(f"{what} must be int32/uint32 (got {t.dtype})")


# ------------------------------------------------------------------ pir.h
def make_params(n: int, primes, d0: int, d1: int) -> pir_params:
    p = pir_params()
    p.n, p.nprimes, p.d0, p.d1 = n, len(primes), d0, d1
    for i, q in enumerate(primes):
        p.q[i] = int(q)
    return p


class Db:
    """Owning handle of a pir_db (freed by ``pir_db_free`` or on collection)."""

    def __init__(self, handle: int, params: pir_params):
        self.handle = handle
        self.params = params

    @property
    def n(self):
        return self.params.n

    @property
    def nprimes(self):
        return self.params.nprimes

    @property
    def d0(self):
        return self.params.d0

    @property
    def d1(self):
        return self.params.d1

    @property
    def primes(self):
        return [self.params.q[i] for i in range(self.params.nprimes)]

    def __del__(self):
        h, self.handle = getattr(self, "handle", None), None
        if h and _lib is not None:
            _lib.pir_db_free(h)


def pir_db_create(params: pir_params, layouts: int = PIR_LAYOUT_VALU | PIR_LAYOUT_MFMA) -> Db:
    h = _vp()
    _check(lib().pir_db_create(ctypes.byref(params), layouts, ctypes.byref(h)), "pir_db_create")
    return Db(h.value, params)


def pir_db_load_ntt(db: Db, src, row0: int = 0, nrows: int | None = None,
                    domain: int = PIR_DOMAIN_COEFF, stream=None):
    _need_u32(src, "src")
    nrows = db.d0 - row0 if nrows is None else nrows
    per_row = db.d1 * db.nprimes * db.n
    if src.numel() != nrows * per_row:
        raise ValueError(f"src has {src.numel()} words, expected {nrows} x {per_row}")
    _check(lib().pir_db_load_ntt(db.handle, _ptr(src, "src"), row0, nrows, domain, _stream(stream)),
           "pir_db_load_ntt")


def pir_db_params(db: Db) -> pir_params:
    p = pir_params()
    _check(lib().pir_db_params(db.handle, ctypes.byref(p)), "pir_db_params")
    return p


def pir_db_layouts(db: Db) -> int:
    return lib().pir_db_layouts(db.handle)


def pir_db_free(db: Db):
    h, db.handle = db.handle, None
    if h:
        lib().pir_db_free(h)


def _rowsel_args(db: Db, query, out, B):
    _need_u32(query, "query")
    _need_u32(out, "out")
    per_q = 2 * db.d0 * db.nprimes * db.n
    per_o = 2 * db.d1 * db.nprimes * db.n
    B = query.numel() // per_q if B is None else B
    if query.numel() < B * per_q or out.numel() < B * per_o:
        raise ValueError("query/out smaller than B clients")
    return (_ptr(query, "query") if B else 0), B, (_ptr(out, "out") if B else 0)


def pir_rowsel(db: Db, query, out, path: int = PIR_PATH_AUTO, stream=None, B: int | None = None):
    qp, B, op = _rowsel_args(db, query, out, B)
    _check(lib().pir_rowsel(db.handle, qp, B, op, path, _stream(stream)), "pir_rowsel")


def pir_rowsel_noalloc(db: Db, query, out, stream=None, B: int | None = None):
    """Allocation-free RowSel (streaming VALU path, 1..4 clients, staging in
    the library's fixed per-GPU array of PIR_NOALLOC_SCRATCH_BYTES)."""
    qp, B, op = _rowsel_args(db, query, out, B)
    _check(lib().pir_rowsel_noalloc(db.handle, qp, B, op, _stream(stream)), "pir_rowsel_noalloc")


PIR_NOALLOC_SCRATCH_BYTES = 64 << 20


def pir_rowsel_coeff(db: Db, query_coeff, out, path: int = PIR_PATH_AUTO, stream=None, B: int | None = None):
    """RowSel on a coefficient-domain query (transformed to the NTT domain by the library)."""
    qp, B, op = _rowsel_args(db, query_coeff, out, B)
    _check(lib().pir_rowsel_coeff(db.handle, qp, B, op, path, _stream(stream)), "pir_rowsel_coeff")


def pir_coltor_stage(n: int, primes, ct, B: int, ncols: int, rgsw, log2z: int, ell: int, out, stream=None):
    """First ColTor stage: ct [B][2][ncols][L][N], rgsw [B][2][ell][2][L][N]
    -> out [B][2][(ncols+1)//2][L][N] (device tensors of 32-bit words)."""
    ring = make_params(n, primes, 1, 1)
    cp = _ptr(ct, "ct") if B else 0
    rp = _ptr(rgsw, "rgsw") if B else 0
    op = _ptr(out, "out") if B else 0
    _check(lib().pir_coltor_stage(ctypes.byref(ring), cp, B, ncols, rp, log2z, ell, op, _stream(stream)),
           "pir_coltor_stage")


class pir_rowsel_item(ctypes.Structure):
    _fields_ = [("db", ctypes.c_void_p), ("q_dev", ctypes.c_void_p), ("B", ctypes.c_uint32),
                ("out_dev", ctypes.c_void_p)]


def pir_rowsel_grouped(items, path: int = PIR_PATH_AUTO, stream=None):
    """items: list of (Db, query tensor, B, out tensor)."""
    arr = (pir_rowsel_item * max(1, len(items)))()
    for i, (db, q, B, out) in enumerate(items):
        _need_u32(q, "query")
        _need_u32(out, "out")
        per_q = 2 * db.d0 * db.nprimes * db.n
        per_o = 2 * db.d1 * db.nprimes * db.n
        if q.numel() < B * per_q or out.numel() < B * per_o:
            raise ValueError(f"item {i}: query/out smaller than B clients")
        arr[i].db = db.handle
        arr[i].q_dev = _ptr(q, "query") if B else None
        arr[i].B = B
        arr[i].out_dev = _ptr(out, "out") if B else None
    _check(lib().pir_rowsel_grouped(ctypes.cast(arr, ctypes.c_void_p), len(items), path,
                                    _stream(stream)), "pir_rowsel_grouped")


PIR_GROUPED_TILE_WORDS = 5
GROUPED_KERNELS = ("fixed", "shaped", "qres")   # kernel ids of pir_rowsel_grouped_tiles


def pir_rowsel_grouped_tiles(items):
    """[(points, rows, cols, kernel, alone)] of the plan of this item list:
    the tile or work unit kept for each item, its kernel (0 fixed-shape
    tiled, 1 shaped tiled, 2 query-resident) and whether its GEMM has a
    launch of its own ((0, 0, 0, 0, 0) for B = 0 items)."""
    w = PIR_GROUPED_TILE_WORDS
    arr = (pir_rowsel_item * max(1, len(items)))()
    for i, (db, q, B, out) in enumerate(items):
        arr[i].db, arr[i].B = db.handle, B
    t = (_u32 * max(w, w * len(items)))()
    _check(lib().pir_rowsel_grouped_tiles(ctypes.cast(arr, ctypes.c_void_p), len(items), t),
           "pir_rowsel_grouped_tiles")
    return [tuple(t[w * i + j] for j in range(w)) for i in range(len(items))]


# ---------------------------------------------------------------- serving
class pir_server_opts(ctypes.Structure):
    _fields_ = [("max_clients", _u32), ("chunks", _u32), ("pipeline", _u32), ("max_waiting", _u32),
                ("hbm_budget", _u64)]


class pir_request(ctypes.Structure):
    _fields_ = [("id", _u64), ("q_dev", _vp), ("out_dev", _vp), ("ready_event", _vp)]


class pir_completion(ctypes.Structure):
    _fields_ = [("id", _u64), ("status", ctypes.c_int32), ("reserved", _u32), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


class pir_server_stats(ctypes.Structure):
    _fields_ = [("capacity", _u32), ("active", _u32), ("waiting", _u32), ("inflight", _u32),
                ("steps", _u64), ("admitted", _u64), ("completed", _u64), ("device_bytes", _u64)]


def pir_clock() -> float:
    return lib().pir_clock()


class Server:
    """Owning handle of a pir_server; keeps the DB and every live request's
    tensors referenced until their completion is returned."""

    def __init__(self, handle, db):
        self.handle, self.db = handle, db
        self.live = {}

    def __del__(self):
        h, self.handle = getattr(self, "handle", None), None
        if h and _lib is not None:
            _lib.pir_server_destroy(h)


def pir_server_create(db: Db, max_clients: int = 0, chunks: int = 0, pipeline: int = 0,
                      hbm_budget: int = 0, max_waiting: int = 0) -> Server:
    o = pir_server_opts(max_clients, chunks, pipeline, max_waiting, hbm_budget)
    h = _vp()
    _check(lib().pir_server_create(db.handle, ctypes.byref(o), ctypes.byref(h)), "pir_server_create")
    return Server(h.value, db)


def pir_serve_step(srv: Server, arrivals=(), cap: int = 1024):
    """arrivals: iterable of (id, query tensor [2][D0][L][N], out tensor [2][D1][L][N]).
    The server's reads of each query are ordered after the work enqueued so
    far on torch's current stream (an event recorded there).  Request ids
    must be unique among live requests (ValueError otherwise).
    Returns the list of finished pir_completion records."""
    import torch
    arrivals = list(arrivals)
    ids = [rid for rid, _, _ in arrivals]
    if len(set(ids)) != len(ids) or any(rid in srv.live for rid in ids):
        raise ValueError("pir_serve_step: a request id is already live")
    ready = None
    if arrivals:
        ready = torch.cuda.Event()
        ready.record(torch.cuda.current_stream())
    arr = (pir_request * max(1, len(arrivals)))()
    for i, (rid, q, out) in enumerate(arrivals):
        _need_u32(q, "query")
        _need_u32(out, "out")
        arr[i].id, arr[i].q_dev, arr[i].out_dev = rid, _ptr(q, "query"), _ptr(out, "out")
        arr[i].ready_event = ready.cuda_event
    done = (pir_completion * max(1, cap))()
    nd = _u32()
    _check(lib().pir_serve_step(srv.handle, ctypes.cast(arr, _vp), len(arrivals), ctypes.cast(done, _vp), cap,
                                ctypes.byref(nd)), "pir_serve_step")
    for rid, q, out in arrivals:
        srv.live[rid] = (q, out)
    res = [done[i] for i in range(nd.value)]
    for c in res:
        srv.live.pop(c.id, None)
    return res


def pir_server_get_stats(srv: Server) -> pir_server_stats:
    s = pir_server_stats()
    _check(lib().pir_server_get_stats(srv.handle, ctypes.byref(s)), "pir_server_get_stats")
    return s


def pir_server_destroy(srv: Server):
    h, srv.handle = srv.handle, None
    if h:
        lib().pir_server_destroy(h)
    srv.live.clear()


def pir_ntt_forward(src, out, n: int, q: int, stream=None):
    _need_u32(src, "src")
    _need_u32(out, "out")
    count = src.numel() // n
    _check(lib().pir_ntt_forward(_ptr(src, "src"), _ptr(out, "out"), count, n, q,
                                 _stream(stream)), "pir_ntt_forward")


def pir_ntt_inverse(src, out, n: int, q: int, stream=None):
    _need_u32(src, "src")
    _need_u32(out, "out")
    count = src.numel() // n
    _check(lib().pir_ntt_inverse(_ptr(src, "src"), _ptr(out, "out"), count, n, q,
                                 _stream(stream)), "pir_ntt_inverse")


def pir_kernel_timing(enable: bool):
    """Start (True) or stop (False) event timing of each call's main kernel."""
    _check(lib().pir_kernel_timing(1 if enable else 0), "pir_kernel_timing")


def pir_kernel_time_read():
    """(launches, total_ms) of the main-kernel launches timed since the last read."""
    n, ms = _u32(), ctypes.c_double()
    _check(lib().pir_kernel_time_read(ctypes.byref(n), ctypes.byref(ms)), "pir_kernel_time_read")
    return n.value, ms.value


def pir_last_error() -> str:
    return lib().pir_last_error().decode()


def pir_version() -> str:
    return lib().pir_version().decode()


# ------------------------------------------------------------ pir_synth.h
def pir_synth_query(out, key: int, b0: int, nb: int, d0: int, primes, n: int, stream=None):
    _need_u32(out, "out")
    if out.numel() != nb * 2 * d0 * len(primes) * n:
        raise ValueError("out has the wrong size")
    qa = (_u32 * len(primes))(*[int(q) for q in primes])
    _check(lib().pir_synth_query(_ptr(out, "out"), key, b0, nb, d0, len(primes), n, qa,
                                 _stream(stream)), "pir_synth_query")


def pir_synth_db_coeffs(out, key: int, row0: int, nrows: int, d1: int, nprimes: int, n: int,
                        stream=None):
    _need_u32(out, "out")
    if out.numel() != nrows * d1 * nprimes * n:
        raise ValueError("out has the wrong size")
    _check(lib().pir_synth_db_coeffs(_ptr(out, "out"), key, row0, nrows, d1, nprimes, n,
                                     _stream(stream)), "pir_synth_db_coeffs")


def pir_synth_draw(out, key: int, i0: int, stream=None):
    import torch
    if out.dtype not in (torch.int64, torch.uint64):
        raise TypeError("out must be int64/uint64")
    _check(lib().pir_synth_draw(_ptr(out, "out"), key, i0, out.numel(), _stream(stream)),
           "pir_synth_draw")


# ------------------------------------------------------------- pir_peak.h
def pir_peak_mfma_i8(iters: int, random_operands: bool, stream=None):
    """(TOP/s, MHz) of a register-only v_mfma_i32_32x32x32_i8 loop."""
    t, m = ctypes.c_double(), ctypes.c_double()
    _check(lib().pir_peak_mfma_i8(iters, 1 if random_operands else 0, ctypes.byref(t), ctypes.byref(m),
                                  _stream(stream)), "pir_peak_mfma_i8")
    return t.value, m.value


def pir_peak_valu_mad64(iters: int, stream=None):
    """(G multiply-adds/s, MHz) of a v_mad_u64_u32 loop."""
    g, m = ctypes.c_double(), ctypes.c_double()
    _check(lib().pir_peak_valu_mad64(iters, ctypes.byref(g), ctypes.byref(m), _stream(stream)),
           "pir_peak_valu_mad64")
    return g.value, m.value


def pir_peak_hbm_read(src, stream=None):
    """GB/s of a streaming read of the device tensor `src`."""
    g = ctypes.c_double()
    nbytes = src.numel() * src.element_size()
    _check(lib().pir_peak_hbm_read(_ptr(src, "src"), nbytes, ctypes.byref(g), _stream(stream)),
           "pir_peak_hbm_read")
    return g.value
