"""CPU oracle for the MWHC build path -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline`` leg may
import this package.  The product library never does: it has no CPU fallback.

The arithmetic lives in ``mphx_oracle.c`` (plain single-threaded C).  This module compiles it
with gcc into ``liboracle.so`` when needed and wraps it with numpy arrays via ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mphx_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

OK, EINVAL, ERANGE, ENOMEM, ECORE, EDUP = 0, -1, -2, -3, 1, 2
NONE = 0xFFFFFFFF

_u64p = C.POINTER(C.c_uint64)
_u32p = C.POINTER(C.c_uint32)
_u8p = C.POINTER(C.c_uint8)


def compile_oracle(src: str = SRC, out: str = LIB, extra=()) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC", *extra, "-o", out, src]
    subprocess.check_call(cmd)
    return out


def _bind(lib):
    sig = {
        "orc_splitmix": (C.c_uint64, [C.c_uint64, C.c_uint64]),
        "orc_set_progress": (None, [C.c_int]),
        "orc_part_size": (C.c_uint64, [C.c_uint64, C.c_uint32, C.c_uint32]),
        "orc_hash_u64": (None, [_u64p, C.c_uint64, C.c_uint64, C.c_uint64, _u32p]),
        "orc_digest_str": (None, [_u8p, C.c_uint64, C.c_uint64, _u64p, _u64p]),
        "orc_hash_str": (None, [_u8p, _u64p, C.c_uint64, C.c_uint64, C.c_uint64, _u32p]),
        "orc_peel": (C.c_int, [_u32p, C.c_uint64, C.c_uint64, C.c_uint64, _u32p, _u32p, _u8p, _u8p, _u64p]),
        "orc_peel_r": (C.c_int, [_u32p, C.c_uint64, C.c_uint64, C.c_uint32, _u32p, _u32p, _u8p, _u8p, _u64p]),
        "orc_assign": (C.c_int, [_u32p, C.c_uint64, C.c_uint64, _u32p, _u32p, _u8p, _u8p]),
        "orc_pack_rank": (None, [_u8p, C.c_uint64, _u64p, _u64p]),
        "orc_lookup_u64": (None, [_u64p, _u64p, C.c_uint64, C.c_uint64, _u64p, C.c_uint64, _u64p]),
        "orc_lookup_str": (None, [_u64p, _u64p, C.c_uint64, C.c_uint64, _u8p, _u64p, C.c_uint64, _u64p]),
        "orc_mphf_build_u64": (C.c_int, [_u64p, C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32,
                                         C.c_uint32, _u64p, _u64p, _u64p]),
        "orc_mphf_build_str": (C.c_int, [_u8p, _u64p, C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32,
                                         C.c_uint32, _u64p, _u64p, _u64p]),
        "orc_hem_signature_u64": (C.c_uint64, [C.c_uint64, C.c_uint64]),
        "orc_hem_signature_str": (None, [_u8p, C.c_uint64, C.c_uint64, _u64p, _u64p]),
        "orc_hem_signatures_u64": (None, [_u64p, C.c_uint64, C.c_uint64, _u64p]),
        "orc_hem_signatures_str": (None, [_u8p, _u64p, C.c_uint64, C.c_uint64, _u64p, _u64p]),
        "orc_hem_build": (C.c_int, [_u64p, _u64p, C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                    _u64p, _u64p, _u64p, _u64p, _u64p, _u64p]),
        "orc_hem_lookup": (None, [_u64p, _u64p, C.c_uint64, C.c_uint32, _u64p, _u64p, _u64p, _u64p, _u64p, _u64p,
                                  C.c_uint32, C.c_uint32, _u64p]),
        "orc_sf_bits": (C.c_uint32, [C.c_uint64]),
        "orc_sf_assign": (C.c_int, [_u32p, C.c_uint64, C.c_uint64, _u32p, _u32p, _u8p, _u32p, C.c_uint64, _u32p]),
        "orc_sf_pack": (None, [_u32p, C.c_uint64, C.c_uint32, _u64p]),
        "orc_sf_build_u64": (C.c_int, [_u64p, _u32p, C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32,
                                       C.c_uint32, _u64p, _u64p]),
        "orc_sf_build_str": (C.c_int, [_u8p, _u64p, _u32p, C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint32,
                                       C.c_uint32, C.c_uint32, _u64p, _u64p]),
        "orc_sf_lookup_u64": (None, [_u64p, C.c_uint64, C.c_uint64, C.c_uint64, _u64p, C.c_uint64, _u64p]),
        "orc_sf_lookup_str": (None, [_u64p, C.c_uint64, C.c_uint64, C.c_uint64, _u8p, _u64p, C.c_uint64, _u64p]),
        "orc_sfr_rank_words": (C.c_uint64, [C.c_uint64]),
        "orc_sf_rank_layout": (C.c_uint64, [_u64p, C.c_uint64, C.c_uint32, _u64p, _u64p, _u64p]),
        "orc_sfr_lookup_u64": (None, [_u64p, _u64p, _u64p, C.c_uint64, C.c_uint64, C.c_uint64, _u64p, C.c_uint64,
                                      _u64p]),
        "orc_sfr_lookup_str": (None, [_u64p, _u64p, _u64p, C.c_uint64, C.c_uint64, C.c_uint64, _u8p, _u64p,
                                      C.c_uint64, _u64p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_LIB = None


def load(path: str | None = None):
    """Load the oracle library (compiling it first if it is missing or stale)."""
    global _LIB
    if path is not None:
        return _bind(C.CDLL(path))
    if _LIB is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            compile_oracle()
        _LIB = _bind(C.CDLL(LIB))
    return _LIB


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(t)


class Oracle:
    """numpy-facing wrapper; ``Oracle(lib)`` binds an alternative build (e.g. a planted mutant)."""

    def __init__(self, lib=None):
        self.lib = lib if lib is not None else load()

    # --- hashing --------------------------------------------------------------------------
    def splitmix(self, state: int, t: int) -> int:
        return int(self.lib.orc_splitmix(state, t))

    def part_size(self, n: int, gnum: int = 123, gden: int = 100) -> int:
        return int(self.lib.orc_part_size(n, gnum, gden))

    def hash_u64(self, keys: np.ndarray, seed: int, P: int) -> np.ndarray:
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        out = np.empty((len(keys), 3), dtype=np.uint32)
        self.lib.orc_hash_u64(_p(keys, _u64p), len(keys), seed, P, _p(out, _u32p))
        return out

    def digest_str(self, key: bytes, seed: int):
        buf = np.frombuffer(key, dtype=np.uint8).copy() if key else np.zeros(1, np.uint8)
        a = C.c_uint64()
        b = C.c_uint64()
        self.lib.orc_digest_str(_p(buf, _u8p), len(key), seed, C.byref(a), C.byref(b))
        return int(a.value), int(b.value)

    def hash_str(self, data: np.ndarray, offs: np.ndarray, seed: int, P: int) -> np.ndarray:
        data = np.ascontiguousarray(data, dtype=np.uint8)
        if data.size == 0:
            data = np.zeros(1, np.uint8)
        offs = np.ascontiguousarray(offs, dtype=np.uint64)
        n = len(offs) - 1
        out = np.empty((n, 3), dtype=np.uint32)
        self.lib.orc_hash_str(_p(data, _u8p), _p(offs, _u64p), n, seed, P, _p(out, _u32p))
        return out

    # --- peeling ------------------------------------------------------------------------------
    def peel(self, edges: np.ndarray, m: int, part_size: int = 0):
        """Returns (status, dict(order, round, core_mask, hinge, n_peeled, n_rounds, max_degree))."""
        edges = np.ascontiguousarray(edges, dtype=np.uint32).reshape(-1, 3)
        n = edges.shape[0]
        order = np.empty(n, np.uint32)
        rnd = np.empty(n, np.uint32)
        core = np.empty(n, np.uint8)
        hinge = np.empty(n, np.uint8)
        info = np.zeros(3, np.uint64)
        e = edges if n else np.zeros((1, 3), np.uint32)
        rc = self.lib.orc_peel(_p(e, _u32p), n, m, part_size, _p(order, _u32p), _p(rnd, _u32p),
                               _p(core, _u8p), _p(hinge, _u8p), _p(info, _u64p))
        return int(rc), dict(order=order, round=rnd, core_mask=core, hinge=hinge,
                             n_peeled=int(info[0]), n_rounds=int(info[1]), max_degree=int(info[2]))

    def peel_r(self, edges: np.ndarray, m: int, r: int):
        """r-hypergraph peel (2 <= r <= 8): (status, dict as peel)."""
        edges = np.ascontiguousarray(edges, dtype=np.uint32).reshape(-1, r)
        n = edges.shape[0]
        order = np.empty(n, np.uint32)
        rnd = np.empty(n, np.uint32)
        core = np.empty(n, np.uint8)
        hinge = np.empty(n, np.uint8)
        info = np.zeros(3, np.uint64)
        e = edges if n else np.zeros((1, r), np.uint32)
        rc = self.lib.orc_peel_r(_p(e, _u32p), n, m, r, _p(order, _u32p), _p(rnd, _u32p), _p(core, _u8p),
                                 _p(hinge, _u8p), _p(info, _u64p))
        return int(rc), dict(order=order, round=rnd, core_mask=core, hinge=hinge,
                             n_peeled=int(info[0]), n_rounds=int(info[1]), max_degree=int(info[2]))

    def assign(self, edges, m, order, rnd, hinge):
        edges = np.ascontiguousarray(edges, dtype=np.uint32).reshape(-1, 3)
        codes = np.zeros(max(m, 1), np.uint8)
        rc = self.lib.orc_assign(_p(edges, _u32p), edges.shape[0], m, _p(np.ascontiguousarray(order), _u32p),
                                 _p(np.ascontiguousarray(rnd), _u32p), _p(np.ascontiguousarray(hinge), _u8p),
                                 _p(codes, _u8p))
        return int(rc), codes[:m]

    def pack_rank(self, codes8: np.ndarray):
        m = len(codes8)
        words = np.zeros(max((m + 31) // 32, 1), np.uint64)
        rank = np.zeros(max((m + 511) // 512, 1), np.uint64)
        c = np.ascontiguousarray(codes8, dtype=np.uint8) if m else np.zeros(1, np.uint8)
        self.lib.orc_pack_rank(_p(c, _u8p), m, _p(words, _u64p), _p(rank, _u64p))
        return words[: (m + 31) // 32], rank[: (m + 511) // 512]

    # --- whole build and lookup -------------------------------------------------------------
    def mphf_build_u64(self, keys, seed=0, gnum=123, gden=100, max_tries=64):
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        n = len(keys)
        P = self.part_size(n, gnum, gden)
        m = 3 * P
        words = np.zeros(max((m + 31) // 32, 1), np.uint64)
        rank = np.zeros(max((m + 511) // 512, 1), np.uint64)
        info = np.zeros(6, np.uint64)
        k = keys if n else np.zeros(1, np.uint64)
        rc = self.lib.orc_mphf_build_u64(_p(k, _u64p), n, seed, gnum, gden, max_tries,
                                         _p(words, _u64p), _p(rank, _u64p), _p(info, _u64p))
        return int(rc), self._build_result(words, rank, info, m)

    def mphf_build_str(self, data, offs, seed=0, gnum=123, gden=100, max_tries=64):
        data = np.ascontiguousarray(data, dtype=np.uint8)
        if data.size == 0:
            data = np.zeros(1, np.uint8)
        offs = np.ascontiguousarray(offs, dtype=np.uint64)
        n = len(offs) - 1
        P = self.part_size(n, gnum, gden)
        m = 3 * P
        words = np.zeros(max((m + 31) // 32, 1), np.uint64)
        rank = np.zeros(max((m + 511) // 512, 1), np.uint64)
        info = np.zeros(6, np.uint64)
        rc = self.lib.orc_mphf_build_str(_p(data, _u8p), _p(offs, _u64p), n, seed, gnum, gden, max_tries,
                                         _p(words, _u64p), _p(rank, _u64p), _p(info, _u64p))
        return int(rc), self._build_result(words, rank, info, m)

    @staticmethod
    def _build_result(words, rank, info, m):
        return dict(words=words[: (m + 31) // 32], rank=rank[: (m + 511) // 512], P=int(info[0]),
                    m=int(info[1]), seed_used=int(info[2]), tries=int(info[3]), n_rounds=int(info[4]),
                    n_core=int(info[5]))

    def lookup_u64(self, words, rank, P, seed, keys):
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        out = np.empty(len(keys), np.uint64)
        w = np.ascontiguousarray(words, dtype=np.uint64) if len(words) else np.zeros(1, np.uint64)
        r = np.ascontiguousarray(rank, dtype=np.uint64) if len(rank) else np.zeros(1, np.uint64)
        self.lib.orc_lookup_u64(_p(w, _u64p), _p(r, _u64p), P, seed, _p(keys, _u64p), len(keys),
                                _p(out, _u64p))
        return out

    def lookup_str(self, words, rank, P, seed, data, offs):
        data = np.ascontiguousarray(data, dtype=np.uint8)
        if data.size == 0:
            data = np.zeros(1, np.uint8)
        offs = np.ascontiguousarray(offs, dtype=np.uint64)
        n = len(offs) - 1
        out = np.empty(n, np.uint64)
        w = np.ascontiguousarray(words, dtype=np.uint64) if len(words) else np.zeros(1, np.uint64)
        r = np.ascontiguousarray(rank, dtype=np.uint64) if len(rank) else np.zeros(1, np.uint64)
        self.lib.orc_lookup_str(_p(w, _u64p), _p(r, _u64p), P, seed, _p(data, _u8p), _p(offs, _u64p), n,
                                _p(out, _u64p))
        return out


    # --- static functions (Section 3: f(x) = u[h0] + u[h1] + u[h2] mod sigma) -------------------
    def sf_bits(self, sigma: int) -> int:
        return int(self.lib.orc_sf_bits(sigma))

    def sf_words(self, m: int, sigma: int) -> int:
        return (m * self.sf_bits(sigma) + 63) // 64

    def sf_assign(self, edges, m, order, rnd, hinge, values, sigma):
        """u (uint32, one per vertex) from a complete peel (orc_peel's outputs)."""
        n = len(order)
        u = np.zeros(max(m, 1), np.uint32)
        e = np.ascontiguousarray(edges, dtype=np.uint32).reshape(-1) if n else np.zeros(3, np.uint32)
        o = np.ascontiguousarray(order, dtype=np.uint32) if n else np.zeros(1, np.uint32)
        r = np.ascontiguousarray(rnd, dtype=np.uint32) if n else np.zeros(1, np.uint32)
        h = np.ascontiguousarray(hinge, dtype=np.uint8) if n else np.zeros(1, np.uint8)
        v = np.ascontiguousarray(values, dtype=np.uint32) if n else np.zeros(1, np.uint32)
        rc = self.lib.orc_sf_assign(_p(e, _u32p), n, m, _p(o, _u32p), _p(r, _u32p), _p(h, _u8p), _p(v, _u32p),
                                    sigma, _p(u, _u32p))
        return int(rc), u[:m]

    def sf_pack(self, u, sigma):
        m = len(u)
        b = self.sf_bits(sigma)
        words = np.zeros(max((m * b + 63) // 64, 1), np.uint64)
        uu = np.ascontiguousarray(u, dtype=np.uint32) if m else np.zeros(1, np.uint32)
        self.lib.orc_sf_pack(_p(uu, _u32p), m, b, _p(words, _u64p))
        return words[: (m * b + 63) // 64]

    def sf_build_u64(self, keys, values, sigma, seed=0, gnum=123, gden=100, max_tries=64):
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        values = np.ascontiguousarray(values, dtype=np.uint32)
        n = len(keys)
        P = self.part_size(n, gnum, gden)
        nw = self.sf_words(3 * P, sigma) if sigma else 0
        words = np.zeros(max(nw, 1), np.uint64)
        info = np.zeros(6, np.uint64)
        k = keys if n else np.zeros(1, np.uint64)
        v = values if n else np.zeros(1, np.uint32)
        rc = self.lib.orc_sf_build_u64(_p(k, _u64p), _p(v, _u32p), n, sigma, seed, gnum, gden, max_tries,
                                       _p(words, _u64p), _p(info, _u64p))
        return int(rc), self._sf_result(words[:nw], info)

    def sf_build_str(self, data, offs, values, sigma, seed=0, gnum=123, gden=100, max_tries=64):
        data = np.ascontiguousarray(data, dtype=np.uint8)
        if data.size == 0:
            data = np.zeros(1, np.uint8)
        offs = np.ascontiguousarray(offs, dtype=np.uint64)
        values = np.ascontiguousarray(values, dtype=np.uint32)
        n = len(offs) - 1
        P = self.part_size(n, gnum, gden)
        nw = self.sf_words(3 * P, sigma) if sigma else 0
        words = np.zeros(max(nw, 1), np.uint64)
        info = np.zeros(6, np.uint64)
        v = values if n else np.zeros(1, np.uint32)
        rc = self.lib.orc_sf_build_str(_p(data, _u8p), _p(offs, _u64p), _p(v, _u32p), n, sigma, seed, gnum, gden,
                                       max_tries, _p(words, _u64p), _p(info, _u64p))
        return int(rc), self._sf_result(words[:nw], info)

    @staticmethod
    def _sf_result(words, info):
        return dict(words=words, P=int(info[0]), m=int(info[1]), seed_used=int(info[2]), tries=int(info[3]),
                    n_rounds=int(info[4]), n_core=int(info[5]))

    def sf_lookup_u64(self, words, sigma, P, seed, keys):
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        out = np.empty(len(keys), np.uint64)
        w = np.ascontiguousarray(words, dtype=np.uint64) if len(words) else np.zeros(1, np.uint64)
        self.lib.orc_sf_lookup_u64(_p(w, _u64p), sigma, P, seed, _p(keys, _u64p), len(keys), _p(out, _u64p))
        return out

    def sf_lookup_str(self, words, sigma, P, seed, data, offs):
        data = np.ascontiguousarray(data, dtype=np.uint8)
        if data.size == 0:
            data = np.zeros(1, np.uint8)
        offs = np.ascontiguousarray(offs, dtype=np.uint64)
        n = len(offs) - 1
        out = np.empty(n, np.uint64)
        w = np.ascontiguousarray(words, dtype=np.uint64) if len(words) else np.zeros(1, np.uint64)
        self.lib.orc_sf_lookup_str(_p(w, _u64p), sigma, P, seed, _p(data, _u8p), _p(offs, _u64p), n,
                                   _p(out, _u64p))
        return out

    # --- ranked static-function layout (Section 3: ceil(log sigma) n + gamma n + o(n) bits) -----
    def sf_rank_layout(self, words, m, sigma):
        """The ranked layout of a static function given in the plain packed layout (m fields):
        marks (m bits), rank samples (one per 1024 vertices plus the total), the non-zero fields
        in vertex order, and their number."""
        b = self.sf_bits(sigma)
        marks = np.zeros(max((m + 63) // 64, 1), np.uint64)
        rank = np.zeros(int(self.lib.orc_sfr_rank_words(m)), np.uint64)
        vals = np.zeros(max((m * b + 63) // 64, 1), np.uint64)
        w = np.ascontiguousarray(words, dtype=np.uint64) if len(words) else np.zeros(1, np.uint64)
        count = int(self.lib.orc_sf_rank_layout(_p(w, _u64p), m, b, _p(marks, _u64p), _p(rank, _u64p),
                                                _p(vals, _u64p)))
        return dict(marks=marks[: (m + 63) // 64], rank=rank, vals=vals[: (count * b + 63) // 64], count=count)

    def sfr_lookup_u64(self, marks, rank, vals, sigma, P, seed, keys):
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        out = np.empty(len(keys), np.uint64)
        mk, rk, vl = (np.ascontiguousarray(x, dtype=np.uint64) if len(x) else np.zeros(1, np.uint64)
                      for x in (marks, rank, vals))
        self.lib.orc_sfr_lookup_u64(_p(mk, _u64p), _p(rk, _u64p), _p(vl, _u64p), sigma, P, seed, _p(keys, _u64p),
                                    len(keys), _p(out, _u64p))
        return out

    def sfr_lookup_str(self, marks, rank, vals, sigma, P, seed, data, offs):
        data = np.ascontiguousarray(data, dtype=np.uint8)
        if data.size == 0:
            data = np.zeros(1, np.uint8)
        offs = np.ascontiguousarray(offs, dtype=np.uint64)
        n = len(offs) - 1
        out = np.empty(n, np.uint64)
        mk, rk, vl = (np.ascontiguousarray(x, dtype=np.uint64) if len(x) else np.zeros(1, np.uint64)
                      for x in (marks, rank, vals))
        self.lib.orc_sfr_lookup_str(_p(mk, _u64p), _p(rk, _u64p), _p(vl, _u64p), sigma, P, seed, _p(data, _u8p),
                                    _p(offs, _u64p), n, _p(out, _u64p))
        return out

    # --- HEM split (Section 3: signatures, 2^k buckets, one MPHF per bucket) ---------------------
    def hem_signatures_u64(self, keys, seed):
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        out = np.empty(len(keys), np.uint64)
        if len(keys):
            self.lib.orc_hem_signatures_u64(_p(keys, _u64p), len(keys), seed, _p(out, _u64p))
        return out

    def hem_signatures_str(self, data, offs, seed):
        """(n, 2) array: each string's 128-bit signature (a, b)."""
        data = np.ascontiguousarray(data, dtype=np.uint8)
        if data.size == 0:
            data = np.zeros(1, np.uint8)
        offs = np.ascontiguousarray(offs, dtype=np.uint64)
        n = len(offs) - 1
        a, b = np.empty(max(n, 1), np.uint64), np.empty(max(n, 1), np.uint64)
        if n:
            self.lib.orc_hem_signatures_str(_p(data, _u8p), _p(offs, _u64p), n, seed, _p(a, _u64p), _p(b, _u64p))
        return np.stack([a[:n], b[:n]], axis=1)

    @staticmethod
    def _sig_words(sigs):
        """First and second signature words: a 1-D array holds 64-bit (u64-key) signatures, an
        (n, 2) array 128-bit (string) ones."""
        sigs = np.asarray(sigs, dtype=np.uint64)
        if sigs.ndim == 2:
            first = np.ascontiguousarray(sigs[:, 0])
            second = np.ascontiguousarray(sigs[:, 1])
            return first, (second if len(second) else np.zeros(1, np.uint64)), len(first)
        return np.ascontiguousarray(sigs), None, len(sigs)

    def hem_build(self, sigs, k, seed=0, gnum=123, gden=100, max_tries=64):
        sigs, sigs2, n = self._sig_words(sigs)
        s2 = _p(sigs2, _u64p) if sigs2 is not None else C.cast(None, _u64p)
        B = 1 << k
        bo = np.zeros(B + 1, np.uint64)
        co = np.zeros(B + 1, np.uint64)
        ro = np.zeros(B + 1, np.uint64)
        seeds = np.zeros(B, np.uint64)
        sg = sigs if n else np.zeros(1, np.uint64)
        none = C.cast(None, _u64p)
        rc = self.lib.orc_hem_build(_p(sg, _u64p), s2, n, k, seed, gnum, gden, max_tries, _p(bo, _u64p),
                                    _p(co, _u64p), _p(ro, _u64p), _p(seeds, _u64p), none, none)
        if rc != 0:
            return int(rc), None
        codes = np.zeros(max(int(co[-1]), 1), np.uint64)
        rank = np.zeros(max(int(ro[-1]), 1), np.uint64)
        rc = self.lib.orc_hem_build(_p(sg, _u64p), s2, n, k, seed, gnum, gden, max_tries, _p(bo, _u64p),
                                    _p(co, _u64p), _p(ro, _u64p), _p(seeds, _u64p), _p(codes, _u64p), _p(rank, _u64p))
        return int(rc), dict(bucket_off=bo, code_off=co, rank_off=ro, seeds=seeds, codes=codes[: int(co[-1])],
                             rank=rank[: int(ro[-1])], k=k)

    def hem_lookup(self, r, sigs, gnum=123, gden=100):
        sigs, sigs2, n = self._sig_words(sigs)
        s2 = _p(sigs2, _u64p) if sigs2 is not None else C.cast(None, _u64p)
        out = np.empty(n, np.uint64)
        codes = r["codes"] if len(r["codes"]) else np.zeros(1, np.uint64)
        rank = r["rank"] if len(r["rank"]) else np.zeros(1, np.uint64)
        self.lib.orc_hem_lookup(_p(sigs if n else np.zeros(1, np.uint64), _u64p), s2, n, r["k"], _p(r["bucket_off"], _u64p),
                                _p(r["code_off"], _u64p), _p(r["rank_off"], _u64p), _p(r["seeds"], _u64p),
                                _p(codes, _u64p), _p(rank, _u64p), gnum, gden, _p(out, _u64p))
        return out


if __name__ == "__main__":  # pragma: no cover
    compile_oracle()
    print("built", LIB, file=sys.stderr)
