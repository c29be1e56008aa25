"""Seeded synthetic inputs for RowSel workloads.

This module is the one piece shared by the CPU oracle, the tests and the
benchmark.  It holds no RowSel arithmetic: only a counter-based random
generator, the draws built on it, and the table of workload shapes.

Generator (SplitMix64, Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014; finaliser constants as in Vigna's public
splitmix64.c):

    mix64(z)      = z ^= z >> 30; z *= 0xBF58476D1CE4E5B9;
                    z ^= z >> 27; z *= 0x94D049BB133111EB; z ^ (z >> 31)
    key(s, t, u)  = mix64((s << 40) | (t << 32) | u)   (s < 2^24, t < 2^8, u < 2^32)
    draw(key, i)  = mix64(key + (i + 1) * 0x9E3779B97F4A7C15)        (mod 2^64)

Derived draws (all by index, so any element can be regenerated alone):

    uniform_mod(key, i, q) = (draw(key, i) * q) >> 64        in [0, q)
    bits16(key, i)         = draw(key, i) & 0xFFFF           in [0, 2^16)
    ternary(key, i)        = ((draw(key, i) * 3) >> 64) - 1  in {-1, 0, 1}

The HIP library carries its own implementation of draw/uniform_mod/bits16
(written from the same definition) so that multi-GiB inputs can be produced
on the device; a GPU test checks the two bit for bit.

Stream tags (the ``t`` field of the key): DB=1, QUERY=2, SECRET=3, ERROR=4,
A=5 (the uniform ``a`` part of a toy encryption), ARRIVAL=6, SHAPES=7,
POOL=8, SELECT=9.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB
MASK64 = (1 << 64) - 1

TAG_DB = 1
TAG_QUERY = 2
TAG_SECRET = 3
TAG_ERROR = 4
TAG_A = 5
TAG_ARRIVAL = 6
TAG_SHAPES = 7
TAG_POOL = 8
TAG_SELECT = 9


# ----------------------------------------------------------------------------
# scalar reference (Python ints; used for keys and for tiny checks)
# ----------------------------------------------------------------------------
def mix64(z: int) -> int:
    z &= MASK64
    z ^= z >> 30
    z = (z * M1) & MASK64
    z ^= z >> 27
    z = (z * M2) & MASK64
    return z ^ (z >> 31)


def stream_key(seed: int, tag: int, sub: int = 0) -> int:
    if not (0 <= seed < (1 << 24) and 0 <= tag < 256 and 0 <= sub < (1 << 32)):
        raise ValueError("seed < 2^24, tag < 256, sub < 2^32 required")
    return mix64((seed << 40) | (tag << 32) | sub)


def draw_scalar(key: int, i: int) -> int:
    return mix64((key + (i + 1) * GAMMA) & MASK64)


# ----------------------------------------------------------------------------
# vectorised draws (numpy uint64 arithmetic wraps mod 2^64)
# ----------------------------------------------------------------------------
def _mix64_np(z: np.ndarray) -> np.ndarray:
    z = z ^ (z >> np.uint64(30))
    z = z * np.uint64(M1)
    z = z ^ (z >> np.uint64(27))
    z = z * np.uint64(M2)
    return z ^ (z >> np.uint64(31))


def draw(key: int, idx) -> np.ndarray:
    """draw(key, i) for every i in ``idx`` (array-like of non-negative ints)."""
    i = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(key) + (i + np.uint64(1)) * np.uint64(GAMMA)
        return _mix64_np(z)


def _mulhi64_small(x: np.ndarray, m: int) -> np.ndarray:
    """floor(x * m / 2^64) for uint64 x and 0 < m < 2^32, exactly."""
    if not (0 < m < (1 << 32)):
        raise ValueError("multiplier must be in (0, 2^32)")
    mm = np.uint64(m)
    hi = x >> np.uint64(32)
    lo = x & np.uint64(0xFFFFFFFF)
    with np.errstate(over="ignore"):
        return (hi * mm + ((lo * mm) >> np.uint64(32))) >> np.uint64(32)


def uniform_mod(key: int, idx, q: int) -> np.ndarray:
    return _mulhi64_small(draw(key, idx), q).astype(np.uint32)


def bits16(key: int, idx) -> np.ndarray:
    return (draw(key, idx) & np.uint64(0xFFFF)).astype(np.uint32)


def ternary(key: int, idx) -> np.ndarray:
    return _mulhi64_small(draw(key, idx), 3).astype(np.int64) - 1


def gaussian_int(key: int, idx, sigma: float, tail: int) -> np.ndarray:
    """Rounded normal N(0, sigma^2) samples cut at |e| <= tail.

    Sample i uses draws (i*64 + 2a, i*64 + 2a + 1) for attempt a (Box-Muller on
    53-bit uniforms); the first attempt inside the cut is kept.  At a 6-sigma
    cut more than a handful of attempts never happens in practice; 32 are
    available and exhaustion raises.
    """
    i = np.asarray(idx, dtype=np.uint64)
    out = np.zeros(i.shape, dtype=np.int64)
    todo = np.ones(i.shape, dtype=bool)
    scale = 1.0 / float(1 << 53)
    for a in range(32):
        if not todo.any():
            break
        base = i * np.uint64(64) + np.uint64(2 * a)
        u1 = (draw(key, base) >> np.uint64(11)).astype(np.float64) * scale
        u2 = (draw(key, base + np.uint64(1)) >> np.uint64(11)).astype(np.float64) * scale
        r = np.sqrt(-2.0 * np.log1p(-u1))          # 1 - u1 in (0, 1]
        z = np.rint(sigma * r * np.cos(2.0 * math.pi * u2)).astype(np.int64)
        ok = todo & (np.abs(z) <= tail)
        out[ok] = z[ok]
        todo &= ~ok
    if todo.any():
        raise RuntimeError("gaussian_int: tail cut not met after 32 attempts")
    return out


# ----------------------------------------------------------------------------
# array builders in the boundary's layouts
# ----------------------------------------------------------------------------
# Query:  [B][2][D0][L][N] uint32 residues      (element index is the flat index)
# DB:     [D0][D1][L][N] uint32 coefficients    (element index is the flat index)
def db_coeffs(seed: int, d0: int, d1: int, nprimes: int, n: int, sub: int = 0,
              rows=None, cols=None) -> np.ndarray:
    """DB coefficients in [0, 2^16), layout [D0][D1][L][N].

    Every limb of a record carries the same small coefficient vector (a
    coefficient < 2^16 < q reduces to itself mod every prime), so the draw
    index is (k*D1 + n)*N + t and ignores the limb.  ``rows``/``cols`` select a
    sub-grid (default: all); the result keeps the [rows][cols][L][N] order.
    """
    key = stream_key(seed, TAG_DB, sub)
    rows = np.arange(d0) if rows is None else np.asarray(rows)
    cols = np.arange(d1) if cols is None else np.asarray(cols)
    rec = (rows[:, None].astype(np.uint64) * np.uint64(d1) + cols[None, :].astype(np.uint64))
    idx = rec[:, :, None] * np.uint64(n) + np.arange(n, dtype=np.uint64)[None, None, :]
    c = bits16(key, idx)                                   # [rows][cols][N]
    return np.ascontiguousarray(np.broadcast_to(c[:, :, None, :],
                                                (len(rows), len(cols), nprimes, n)))


def query_uniform(seed: int, b_count: int, d0: int, primes, n: int, sub: int = 0,
                  clients=None, tag: int = TAG_QUERY) -> np.ndarray:
    """Uniform residues, layout [B][2][D0][L][N]; draw index is the flat index
    in the full [B][2][D0][L][N] array; limb l uses uniform_mod(., q_l).
    ``clients`` selects client indices (default all); the result keeps their order.
    ``tag`` names the stream (TAG_POOL for the serving workload's query pool)."""
    key = stream_key(seed, tag, sub)
    L = len(primes)
    clients = np.arange(b_count) if clients is None else np.asarray(clients)
    per_client = 2 * d0 * L * n
    out = np.empty((len(clients), 2, d0, L, n), dtype=np.uint32)
    t = np.arange(2 * d0 * n, dtype=np.uint64)
    cc = t // np.uint64(d0 * n)
    kk = (t // np.uint64(n)) % np.uint64(d0)
    jj = t % np.uint64(n)
    for bi, b in enumerate(clients):
        for l, q in enumerate(primes):
            idx = (np.uint64(int(b) * per_client)
                   + ((cc * np.uint64(d0) + kk) * np.uint64(L) + np.uint64(l)) * np.uint64(n) + jj)
            out[bi, :, :, l, :] = uniform_mod(key, idx, int(q)).reshape(2, d0, n)
    return out


# ----------------------------------------------------------------------------
# workload table
# ----------------------------------------------------------------------------
# Primes: the largest primes below 2^30 with q = 1 (mod 2N).  The oracle
# re-derives them and a test checks this table against it; the library checks
# primality and q = 1 (mod 2N) on its own.
PRIME_N1024 = (1073707009,)
PRIMES_N4096 = (1073692673, 1073668097)
# The paper's RNS setting: four primes in 32-bit words whose product is about
# 2^108 -- here the four largest 27-bit primes with q = 1 (mod 8192), product
# 2^107.99 (checked the same way as the table above).
PRIMES_Q108 = (134176769, 134111233, 134012929, 133963777)
# Full 32-bit primes (products of residues reach 2^64): the two largest with
# q = 1 (mod 8192).
PRIMES_W32 = (4294828033, 4294729729)
# Further wide primes (parity cases of the 64-bit paths and of the INT8 digit
# window): the two largest 31-bit ones, and the two largest 32-bit ones not
# above 4278124286 = 2 * 2139062143 (whose residues would also fit as
# (-q/2, q/2]), all with q = 1 (mod 8192).
PRIMES_W31 = (2147377153, 2147352577)
PRIMES_W32_SYM = (4278108161, 4277690369)
# The largest prime below 2^32 with q = 1 (mod 16) (N = 8): its residues come
# within 527 of the low end of the INT8 digit reach.
PRIME_W32_TOP_N8 = 4294966769


@dataclass(frozen=True)
class Workload:
    name: str
    seed: int
    n: int
    primes: tuple
    d0: int
    d1: int
    clients: int
    query: str            # "toy_rlwe" | "uniform"
    db_seed: int = 0      # seed of the DB stream (defaults to ``seed``)
    note: str = ""

    @property
    def nprimes(self) -> int:
        return len(self.primes)

    @property
    def slots(self) -> int:
        return self.n * len(self.primes)

    @property
    def macs(self) -> int:
        return self.slots * 2 * self.clients * self.d0 * self.d1

    @property
    def db_bytes(self) -> int:
        return self.slots * self.d0 * self.d1 * 4

    @property
    def io_bytes(self) -> int:
        return self.slots * 2 * self.clients * (self.d0 + self.d1) * 4

    @property
    def dbseed(self) -> int:
        return self.db_seed or self.seed


TINY = Workload("rowsel_tiny_n1024_16x16_b1", 1, 1024, PRIME_N1024, 16, 16, 1,
                "toy_rlwe", note="toy RLWE encryptions of a one-hot row selector")
HBM = Workload("rowsel_n4096_l2_512x512_b1", 2, 4096, PRIMES_N4096, 512, 512, 1,
               "uniform", note="8 GiB NTT-domain DB, one client")
BATCHED = Workload("rowsel_n4096_l2_512x512_b64", 3, 4096, PRIMES_N4096, 512, 512, 64,
                   "uniform", db_seed=2, note="same DB as the one-client case")
SERVE_DB = Workload("serve_n4096_l2_1024x1024", 5, 4096, PRIMES_N4096, 1024, 1024, 1,
                    "uniform", note="32 GiB resident DB; requests drawn from a 32-query pool")
WIDE32 = Workload("rowsel_n4096_l2w32_512x512_b1", 7, 4096, PRIMES_W32, 512, 512, 1, "uniform",
                  note="two full 32-bit primes (products up to 2^64), 8 GiB DB")
PAPER_Q108 = Workload("rowsel_n4096_l4q108_256x512_b32", 6, 4096, PRIMES_Q108, 256, 512, 32,
                      "uniform", note="four 27-bit limbs (Q ~ 2^108) and D0 = 256 as in the paper's "
                      "setting; 8 GiB DB; one client and a batch of 32")

# Offered loads of the serving workload, frozen: Poisson rates of 0.7x and
# 0.9x the saturated rate (twice the 256-client admission cap arriving at
# once, after an untimed warm-up burst) measured on one MI355X with this
# library, 3490 queries/s (3482-3503 in four runs).  Earlier calibrations:
# 2480 queries/s without the warm-up (the saturated run paid the step
# kernels' first launches), then 3100 queries/s before steps with more than
# 64 clients moved to the query-resident kernel.
SERVE_SATURATED_QPS = 3490.0
SERVE_LOADS = (0.7, 0.9)
SERVE_RATES_QPS = tuple(round(f * SERVE_SATURATED_QPS, 1) for f in SERVE_LOADS)

GROUPED_SEED = 4
GROUPED_COUNT = 24


@dataclass(frozen=True)
class GroupedInstance:
    index: int
    d0: int
    d1: int
    clients: int
    n: int = 4096
    primes: tuple = PRIMES_N4096

    @property
    def seed(self) -> int:
        return GROUPED_SEED

    @property
    def macs(self) -> int:
        return self.n * len(self.primes) * 2 * self.clients * self.d0 * self.d1


def grouped_instances(seed: int = GROUPED_SEED, count: int = GROUPED_COUNT,
                      n: int = 4096, primes=PRIMES_N4096):
    """Uneven instance shapes: D0 in {32,...,512}, D1 in {16,...,256},
    clients in 1..96, each drawn uniformly from the SHAPES stream."""
    key = stream_key(seed, TAG_SHAPES)
    out = []
    for i in range(count):
        d = draw(key, [3 * i, 3 * i + 1, 3 * i + 2])
        d0 = 32 * (1 + int(_mulhi64_small(d[0:1], 16)[0]))
        d1 = 16 * (1 + int(_mulhi64_small(d[1:2], 16)[0]))
        b = 1 + int(_mulhi64_small(d[2:3], 96)[0])
        out.append(GroupedInstance(i, d0, d1, b, n, tuple(primes)))
    return out


def selected_row(seed: int, d0: int) -> int:
    """Seed-chosen selected row index i* for the toy-encryption workload."""
    return int(_mulhi64_small(draw(stream_key(seed, TAG_SELECT), [0]), d0)[0])


def poisson_arrivals(seed: int, rate_per_s: float, count: int) -> np.ndarray:
    """Arrival times (s) of a Poisson stream: exponential gaps from the
    ARRIVAL stream, gap_i = -ln(1 - u_i) / rate with u_i a 53-bit uniform."""
    key = stream_key(seed, TAG_ARRIVAL)
    u = (draw(key, np.arange(count)) >> np.uint64(11)).astype(np.float64) / float(1 << 53)
    return np.cumsum(-np.log1p(-u) / rate_per_s)


def pool_choice(seed: int, count: int, pool: int = 32) -> np.ndarray:
    key = stream_key(seed, TAG_POOL)
    return _mulhi64_small(draw(key, np.arange(count)), pool).astype(np.int64)
