"""Python binding of libpir.so (include/pir.h, include/pir_synth.h).

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
    "pir_ntt_forward": (_i32, [_vp, _vp, _u32, _u32, _u32, _vp]),
    "pir_ntt_inverse": (_i32, [_vp, _vp, _u32, _u32, _u32, _vp]),
    "pir_last_error": (ctypes.c_char_p, []),
    "pir_version": (ctypes.c_char_p, []),
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


def pir_rowsel(db: Db, query, out, path: int = PIR_PATH_AUTO, stream=None, B: int | None = None):
    _need_u32(query, "query")
    _need_u32(out, "out")
    per_q = 2 * db.d0 * db.nprimes * db.n
    per_o = 2 * db.d1 * db.nprimes * db.n
    B = query.numel() // per_q if B is None else B
    if query.numel() < B * per_q or out.numel() < B * per_o:
        raise ValueError("query/out smaller than B clients")
    qp = _ptr(query, "query") if B else 0
    op = _ptr(out, "out") if B else 0
    _check(lib().pir_rowsel(db.handle, qp, B, op, path, _stream(stream)), "pir_rowsel")


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
