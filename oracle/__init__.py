"""CPU oracle for RowSel -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the package smoke check and the benchmark's CPU-baseline leg
may import this package.  It is independent of the HIP library: the
arithmetic lives in ``oracle.c`` (plain C, exact 64/128-bit integers), built
into ``liboracle.so`` with gcc, and these are thin numpy wrappers around it.

Functions and the passage each follows:
  * ``ntt_primes``, ``psi``         -- RNS primes q = 1 (mod 2N) and the 2N-th
                                       root used by the negacyclic NTT (sec. 2.4.1).
  * ``ntt_forward``/``ntt_inverse`` -- negacyclic NTT, natural point order
                                       ahat_i = a(psi^(2i+1)) (sec. 2.4.1).
  * ``negacyclic_mul``              -- schoolbook product mod (X^N + 1, q).
  * ``rowsel``                      -- the point-wise GEMM of sec. 2.2 / 2.3:
       out[b][c][n][l][j] = sum_k Q[b][c][k][l][j] * DB[k][n][l][j]  mod q_l.
  * ``coltor`` (module)             -- the first ColTor stage: RNS
       reconstruction, digit decomposition and the external product
       (sec. 2.2, 2.4.2), in Python integers.
  * ``rlwe`` (module)               -- toy RLWE encryption and decryption.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "oracle.c")


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (-O2, OpenMP, no intrinsics)."""
    if not force and os.path.exists(LIB_PATH) and \
            os.path.getmtime(LIB_PATH) >= os.path.getmtime(SRC_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-Wall", "-Wextra", "-o", tmp, SRC_PATH]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or \
                os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        i64p = ctypes.POINTER(ctypes.c_int64)
        u64, u32 = ctypes.c_uint64, ctypes.c_uint32
        L.oracle_is_prime.argtypes = [u64]
        L.oracle_is_prime.restype = ctypes.c_int
        L.oracle_ntt_primes.argtypes = [u32, u32, u32, u64p]
        L.oracle_ntt_primes.restype = u32
        L.oracle_primitive_root.argtypes = [u64]
        L.oracle_primitive_root.restype = u64
        L.oracle_psi.argtypes = [u64, u32]
        L.oracle_psi.restype = u64
        L.oracle_ntt_forward.argtypes = [u64, u32, u64, u32p, u32p]
        L.oracle_ntt_forward.restype = None
        L.oracle_ntt_inverse.argtypes = [u64, u32, u64, u32p, u32p]
        L.oracle_ntt_inverse.restype = None
        L.oracle_ntt_forward_many.argtypes = [u64, u32, u64, u64, u32p, u32p, u64]
        L.oracle_ntt_forward_many.restype = None
        L.oracle_ntt_inverse_many.argtypes = [u64, u32, u64, u64, u32p, u32p, u64]
        L.oracle_ntt_inverse_many.restype = None
        L.oracle_negacyclic_mul.argtypes = [u64, u32, i64p, i64p, u32p]
        L.oracle_negacyclic_mul.restype = None
        L.oracle_rowsel.argtypes = [u32, u32, u32, u32, u32, u64p, u32p, u32p, u32p]
        L.oracle_rowsel.restype = None
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_set_threads.restype = None
        L.oracle_max_threads.argtypes = []
        L.oracle_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def is_prime(n: int) -> bool:
    return bool(lib().oracle_is_prime(int(n)))


def ntt_primes(n: int, bits: int, count: int) -> list:
    out = np.zeros(count, dtype=np.uint64)
    got = lib().oracle_ntt_primes(n, bits, count, _p(out, ctypes.c_uint64))
    return [int(x) for x in out[:got]]


def primitive_root(q: int) -> int:
    return int(lib().oracle_primitive_root(int(q)))


def psi(q: int, n: int) -> int:
    return int(lib().oracle_psi(int(q), int(n)))


def ntt_forward(a: np.ndarray, q: int, psi_: int | None = None) -> np.ndarray:
    """Forward negacyclic NTT along the last axis (length N)."""
    a = np.ascontiguousarray(a, dtype=np.uint32)
    n = a.shape[-1]
    psi_ = psi(q, n) if psi_ is None else psi_
    out = np.empty_like(a)
    count = a.size // n
    lib().oracle_ntt_forward_many(int(q), n, int(psi_), count, _p(a, ctypes.c_uint32),
                                  _p(out, ctypes.c_uint32), n)
    return out


def ntt_inverse(ahat: np.ndarray, q: int, psi_: int | None = None) -> np.ndarray:
    """Inverse of ntt_forward along the last axis (length N)."""
    ahat = np.ascontiguousarray(ahat, dtype=np.uint32)
    n = ahat.shape[-1]
    psi_ = psi(q, n) if psi_ is None else psi_
    out = np.empty_like(ahat)
    count = ahat.size // n
    lib().oracle_ntt_inverse_many(int(q), n, int(psi_), count, _p(ahat, ctypes.c_uint32),
                                  _p(out, ctypes.c_uint32), n)
    return out


def negacyclic_mul(a, b, q: int) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.int64)
    b = np.ascontiguousarray(b, dtype=np.int64)
    assert a.shape == b.shape and a.ndim == 1
    out = np.empty(a.shape[0], dtype=np.uint32)
    lib().oracle_negacyclic_mul(int(q), a.shape[0], _p(a, ctypes.c_int64),
                                _p(b, ctypes.c_int64), _p(out, ctypes.c_uint32))
    return out


def ntt_db(coeffs: np.ndarray, primes) -> np.ndarray:
    """NTT every limb of a [..][L][N] coefficient array (limb l mod q_l)."""
    coeffs = np.ascontiguousarray(coeffs, dtype=np.uint32)
    out = np.empty_like(coeffs)
    for l, q in enumerate(primes):
        out[..., l, :] = ntt_forward(np.ascontiguousarray(coeffs[..., l, :]), int(q))
    return out


def rowsel(query: np.ndarray, db: np.ndarray, primes) -> np.ndarray:
    """query [B][2][D0][L][N], db [D0][D1][L][N] (NTT domain) -> [B][2][D1][L][N]."""
    query = np.ascontiguousarray(query, dtype=np.uint32)
    db = np.ascontiguousarray(db, dtype=np.uint32)
    B, two, D0, L, N = query.shape
    assert two == 2 and db.shape[0] == D0 and db.shape[2:] == (L, N), (query.shape, db.shape)
    D1 = db.shape[1]
    pr = np.asarray(primes, dtype=np.uint64)
    assert pr.shape == (L,)
    out = np.empty((B, 2, D1, L, N), dtype=np.uint32)
    lib().oracle_rowsel(B, D0, D1, L, N, _p(pr, ctypes.c_uint64), _p(query, ctypes.c_uint32),
                        _p(db, ctypes.c_uint32), _p(out, ctypes.c_uint32))
    return out


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops from now on."""
    lib().oracle_set_threads(int(n))


def max_threads() -> int:
    return int(lib().oracle_max_threads())
