"""Seeded synthetic inputs for the MWHC build (shared by tests, bench and the oracle's callers).

This module produces *inputs only*: key sets, key lengths, bucket sizes and request arrival
times.  It holds none of the method's arithmetic (no hashing of keys into edges, no peeling,
no assignment, no ranking).  Its pseudo-random numbers come from the SplitMix64 generator
(Steele, Lea & Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014), used
here purely as a counter-based stream: output ``t`` of the stream seeded at state ``s`` is
``fin(s + t * GAMMA)`` for ``t = 1, 2, ...``.

Key sets stand in for the paper's URL and n-gram collections (Section 5: after hashing, the
nature of the data is irrelevant and random data gave the same results):

* u64 keys: ``key_i`` = output ``i + 1`` of the stream seeded at ``gen_seed``.  SplitMix64 is
  a bijection of its counter, so the keys are distinct.
* byte-string keys: key ``i`` draws from the stream seeded at ``key_i`` (the u64 key above).
  Output 1 picks the length through a 65,536-entry quantile table of a log-normal
  distribution (mean 60 bytes, sigma 0.5, clamped to [8, 512]).  Bytes 0..4 are the base-95
  digits of ``i`` (least significant first) plus 0x20, which makes the keys distinct by
  construction.  Byte ``j >= 5`` is byte ``(j - 5) % 8`` (little-endian) of output
  ``2 + (j - 5) // 8``, mapped to printable ASCII as ``0x20 + ((b * 95) >> 8)``.
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

STR_PREFIX = 5          # base-95 digits of the key index at the start of every string key
STR_MIN_LEN = 8
STR_MAX_LEN = 512
STR_MEAN = 60.0
STR_SIGMA = 0.5
QTABLE_BITS = 16


def _fin(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function (Stafford's 'Mix13' finalizer), vectorised over uint64."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream(state, t) -> np.ndarray:
    """Output ``t`` (1-based) of the SplitMix64 stream seeded at ``state`` (broadcasting)."""
    state = np.asarray(state, dtype=np.uint64)
    t = np.asarray(t, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _fin(state + t * GAMMA)


def u64_keys(n: int, gen_seed: int = 0, start: int = 0) -> np.ndarray:
    """Keys ``start .. start+n-1`` of the u64 key set seeded at ``gen_seed``."""
    idx = np.arange(start, start + n, dtype=np.uint64)
    return stream(np.uint64(gen_seed), idx + np.uint64(1))


def quantile_table(mean: float = STR_MEAN) -> np.ndarray:
    """Length table: entry u is the clamped log-normal quantile at (u + 0.5) / 65536.

    mu = ln(mean) - sigma^2 / 2 makes the unclamped mean exactly ``mean`` bytes (60 by
    default; the host-memory string split also uses 23, the n-gram keys' average length).
    """
    from scipy.special import ndtri

    size = 1 << QTABLE_BITS
    mu = math.log(mean) - STR_SIGMA * STR_SIGMA / 2.0
    u = (np.arange(size, dtype=np.float64) + 0.5) / size
    q = np.floor(np.exp(mu + STR_SIGMA * ndtri(u)) + 0.5)
    return np.clip(q, STR_MIN_LEN, STR_MAX_LEN).astype(np.uint16)


_QT = None


def _qtable() -> np.ndarray:
    global _QT
    if _QT is None:
        _QT = quantile_table()
    return _QT


def str_lengths(n: int, gen_seed: int = 0, start: int = 0) -> np.ndarray:
    base = u64_keys(n, gen_seed, start)
    r0 = stream(base, 1)
    return _qtable()[(r0 >> np.uint64(64 - QTABLE_BITS)).astype(np.int64)].astype(np.int64)


_STR_CHUNK = 1 << 19  # keys per vectorised pass: bounds the per-byte index arrays


def str_keys(n: int, gen_seed: int = 0, start: int = 0):
    """Byte-string keys ``start .. start+n-1``.

    Returns ``(data, offs)``: ``data`` is a uint8 array with all keys back to back and
    ``offs`` a uint64 array of n + 1 offsets (key i is ``data[offs[i]:offs[i+1]]``).
    """
    if n <= _STR_CHUNK:
        return _str_keys_chunk(n, gen_seed, start)
    lens = str_lengths(n, gen_seed, start)
    offs = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(lens, out=offs[1:])
    data = np.empty(int(offs[-1]), dtype=np.uint8)
    for c0 in range(0, n, _STR_CHUNK):
        c1 = min(c0 + _STR_CHUNK, n)
        d, _ = _str_keys_chunk(c1 - c0, gen_seed, start + c0)
        data[int(offs[c0]):int(offs[c1])] = d
    return data, offs


def _str_keys_chunk(n: int, gen_seed: int, start: int):
    base = u64_keys(n, gen_seed, start)
    lens = str_lengths(n, gen_seed, start)
    offs = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(lens, out=offs[1:])
    if n == 0:
        return np.empty(0, dtype=np.uint8), offs
    # Each key laid out in a row of the longest key's width: the prefix, then the mapped bytes
    # of its stream words; the keys are the rows' first len bytes, read in row order.
    body = lens - STR_PREFIX
    nwords = (body + 7) // 8
    wmax = int(nwords.max())
    have = np.arange(wmax, dtype=np.int64)[None, :] < nwords[:, None]
    key_of_word = np.repeat(np.arange(n, dtype=np.int64), nwords)
    wstart = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(nwords, out=wstart[1:])
    t = np.arange(wstart[-1], dtype=np.int64) - wstart[key_of_word]
    raw = stream(base[key_of_word], (t + 2).astype(np.uint64)).astype("<u8")
    printable = (0x20 + ((np.arange(256, dtype=np.uint32) * 95) >> 8)).astype(np.uint8)
    words = np.zeros((n, wmax), dtype="<u8")
    words[have] = printable[raw.view(np.uint8)].view("<u8")
    rows = np.empty((n, STR_PREFIX + 8 * wmax), dtype=np.uint8)
    gidx = np.arange(start, start + n, dtype=np.int64)
    digits = np.empty((n, STR_PREFIX), dtype=np.uint8)
    for d in range(STR_PREFIX):  # base-95 digits of the global index
        digits[:, d] = 0x20 + (gidx // (95 ** d)) % 95
    rows[:, :STR_PREFIX] = digits
    rows[:, STR_PREFIX:] = words.view(np.uint8).reshape(n, 8 * wmax)
    keep = np.arange(rows.shape[1], dtype=np.int64)[None, :] < lens[:, None]
    return rows[keep], offs


def str_key(i: int, gen_seed: int = 0) -> bytes:
    """One string key, built byte by byte from the definition above (for sampled checks)."""
    base = int(u64_keys(1, gen_seed, i)[0])
    ln = int(_qtable()[int(stream(np.uint64(base), 1)) >> (64 - QTABLE_BITS)])
    out = bytearray()
    for d in range(STR_PREFIX):
        out.append(0x20 + (i // (95 ** d)) % 95)
    t = 2
    while len(out) < ln:
        w = int(stream(np.uint64(base), t))
        for lane in range(8):
            if len(out) == ln:
                break
            b = (w >> (8 * lane)) & 0xFF
            out.append(0x20 + ((b * 95) >> 8))
        t += 1
    return bytes(out)


def uniform01(state, t) -> np.ndarray:
    """53-bit uniform doubles in [0, 1) from stream outputs (host-side workload shaping only)."""
    return (stream(state, t) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


def bucket_sizes(num_buckets: int, lo: int = 100, hi: int = 1_000_000, seed: int = 0) -> np.ndarray:
    """Log-uniform bucket sizes floor(lo * (hi/lo)^u), u uniform in [0,1) from the stream at seed."""
    u = uniform01(np.uint64(seed), np.arange(1, num_buckets + 1, dtype=np.uint64))
    s = np.floor(lo * np.power(hi / lo, u)).astype(np.int64)
    return np.clip(s, lo, hi)


def bucket_gen_seed(b: int) -> int:
    """Generator seed of bucket b's keys: output b + 1 of the stream at state 0."""
    return int(stream(np.uint64(0), np.uint64(b + 1)))


def poisson_arrivals(num: int, rate_per_s: float, seed: int = 0) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process: cumulative exponential gaps."""
    u = uniform01(np.uint64(seed), np.arange(1, num + 1, dtype=np.uint64))
    gaps = -np.log1p(-u) / rate_per_s
    return np.cumsum(gaps)


def request_sizes(num: int, lo: int = 1000, hi: int = 100_000_000, seed: int = 1) -> np.ndarray:
    return bucket_sizes(num, lo, hi, seed)
