#!/usr/bin/env python3
"""Golden digests of the oracle's MPHFs at the full workload sizes.

The full-size parity tests compare the GPU's tables with these digests instead of running the
oracle inside the test.  Only ``oracle/`` (the plain single-threaded C reference) and
``workloads/`` (the seeded generators) are used here; nothing comes from the GPU path.

* ``c4``: the 65,536 log-uniform buckets of 100..10^6 u64 keys (bucket b's keys from generator
  seed ``bucket_gen_seed(b)``, hash seed 0, up to 64 tries), one unchanged oracle build per
  bucket, buckets spread over worker processes.  Writes ``c4_buckets_65536.txt.gz``: per bucket
  its tries, rounds and a 48-bit digest of (codes, rank).
* ``c5``: the 60 requests of the served workload (sizes log-uniform 10^3..10^8; u64 keys are
  prefixes of the set at generator seed 7, strings of the set at seed 8; request i hashed with
  seed i).  Writes ``c5_served_60.txt``.
* ``c3``: 2^31 byte-string keys (generator seed 0), one MWHC build at hash seed 0.  The keys
  are generated and hashed chunk by chunk in worker processes (the oracle's hash is per key),
  then the oracle's peel, assignment and packing run once over all edges, retrying with the
  next seed while a 2-core remains.  Needs about 80 GB of host memory and a long
  single-threaded peel.  Writes ``c3_str_2e31.txt``.

The digest of a build is SHA-256 over its code words then its rank words, both as
little-endian u64 bytes (Section 5 layout: 2-bit codes, one rank sample per 512 vertices).

Usage: python tests/golden/make_fullsize.py {c3,c4,c5} [--procs N]
"""
from __future__ import annotations

import argparse
import gzip
import hashlib
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

C4_FILE = os.path.join(HERE, "c4_buckets_65536.txt.gz")
C5_FILE = os.path.join(HERE, "c5_served_60.txt")
C3_FILE = os.path.join(HERE, "c3_str_2e31.txt")
MAX_TRIES = 64


def digest(words: np.ndarray, rank: np.ndarray) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(words, dtype=np.uint64).tobytes())
    h.update(np.ascontiguousarray(rank, dtype=np.uint64).tobytes())
    return h.hexdigest()


def log(*a):
    print(*a, flush=True)


# ---- config 4 ---------------------------------------------------------------------------------
def _c4_work(bs):
    o = oracle.Oracle()
    sizes = workloads.bucket_sizes(65536, 100, 1_000_000, seed=0)
    out = []
    for b in bs:
        keys = workloads.u64_keys(int(sizes[b]), gen_seed=workloads.bucket_gen_seed(b))
        rc, ref = o.mphf_build_u64(keys, seed=0, max_tries=MAX_TRIES)
        if rc != 0:
            raise RuntimeError(f"bucket {b}: oracle status {rc}")
        out.append((b, ref["tries"], ref["n_rounds"], digest(ref["words"], ref["rank"])[:12]))
    return out


def make_c4(procs: int) -> None:
    sizes = workloads.bucket_sizes(65536, 100, 1_000_000, seed=0)
    order = np.argsort(-sizes, kind="stable")  # largest first, dealt round-robin
    jobs = [order[i::procs * 16].tolist() for i in range(procs * 16)]
    t0 = time.time()
    rows, done = [], 0
    with mp.get_context("fork").Pool(procs) as pool:
        for part in pool.imap_unordered(_c4_work, jobs):
            rows += part
            done += len(part)
            log(f"[c4] {done}/65536 buckets, {time.time() - t0:.0f} s")
    wall = time.time() - t0
    rows.sort()
    with gzip.open(C4_FILE, "wt") as fh:
        fh.write("# Oracle MPHFs of the 65,536 buckets of config 4 (log-uniform 100..10^6 u64 keys, bucket b from\n"
                 "# generator seed bucket_gen_seed(b), hash seed 0, gamma 123/100, up to 64 tries).\n"
                 "# Written by tests/golden/make_fullsize.py c4; digest = the first 12 hex digits of SHA-256 over the\n"
                 "# code words then the rank words (little-endian u64).\n"
                 f"# {procs} oracle processes on {os.cpu_count()} host CPUs, {wall:.0f} s wall, "
                 f"{int(sizes.sum())} keys\n"
                 "# bucket tries rounds digest\n")
        for b, tries, rounds, d in rows:
            fh.write(f"{b} {tries} {rounds} {d}\n")
    log(f"[c4] wrote {C4_FILE}: {len(rows)} buckets in {wall:.0f} s on {procs} processes")


def read_c4():
    rows = {}
    with gzip.open(C4_FILE, "rt") as fh:
        for line in fh:
            if line.startswith("#"):
                continue
            b, tries, rounds, d = line.split()
            rows[int(b)] = (int(tries), int(rounds), d)
    return rows


# ---- config 5 ---------------------------------------------------------------------------------
C5_REQUESTS = 60
C5_MAX = 100_000_000


def c5_plan():
    sizes = workloads.request_sizes(C5_REQUESTS, 1000, C5_MAX, seed=1)
    kinds = (workloads.stream(np.uint64(2), np.arange(1, C5_REQUESTS + 1, dtype=np.uint64)) & np.uint64(1)).astype(int)
    return sizes, kinds


def _c5_work(i):
    o = oracle.Oracle()
    sizes, kinds = c5_plan()
    n = int(sizes[i])
    if kinds[i] == 0:
        keys = workloads.u64_keys(n, gen_seed=7)
        t0 = time.time()
        rc, ref = o.mphf_build_u64(keys, seed=i, max_tries=MAX_TRIES)
    else:
        data, offs = workloads.str_keys(n, gen_seed=8)
        t0 = time.time()
        rc, ref = o.mphf_build_str(data, offs, seed=i, max_tries=MAX_TRIES)
    if rc != 0:
        raise RuntimeError(f"request {i}: oracle status {rc}")
    return i, int(kinds[i]), n, ref["seed_used"], ref["tries"], ref["n_rounds"], digest(ref["words"], ref["rank"]), \
        time.time() - t0


def make_c5(procs: int) -> None:
    sizes, kinds = c5_plan()
    order = np.argsort(-sizes, kind="stable").tolist()
    rows = []
    t0 = time.time()
    with mp.get_context("fork").Pool(procs) as pool:
        for r in pool.imap_unordered(_c5_work, order):
            rows.append(r)
            log(f"[c5] request {r[0]} ({r[2]} {'u64' if r[1] == 0 else 'string'} keys) in {r[7]:.1f} s")
    rows.sort()
    with open(C5_FILE, "w") as fh:
        fh.write("# Oracle MPHFs of the 60 requests of the served workload (sizes log-uniform 10^3..10^8 from seed 1;\n"
                 "# u64 keys: prefixes of the set at generator seed 7; strings: prefixes of the set at seed 8;\n"
                 "# request i at hash seed i, gamma 123/100, up to 64 tries).  Written by\n"
                 "# tests/golden/make_fullsize.py c5; digest = SHA-256 over the code words then the rank words.\n"
                 f"# {procs} oracle processes on {os.cpu_count()} host CPUs, {time.time() - t0:.0f} s wall; oracle_s = that\n"
                 "# request's oracle build time (key generation excluded), single-threaded\n"
                 "# request kind n seed_used tries rounds digest oracle_s\n")
        for i, kind, n, seed, tries, rounds, d, secs in rows:
            fh.write(f"{i} {kind} {n} {seed} {tries} {rounds} {d} {secs:.2f}\n")
    log(f"[c5] wrote {C5_FILE}")


def read_c5():
    rows = {}
    with open(C5_FILE) as fh:
        for line in fh:
            if line.startswith("#"):
                continue
            i, kind, n, seed, tries, rounds, d, secs = line.split()
            rows[int(i)] = dict(kind=int(kind), n=int(n), seed_used=int(seed), tries=int(tries), n_rounds=int(rounds),
                                digest=d, oracle_s=float(secs))
    return rows


# ---- config 3 ---------------------------------------------------------------------------------
C3_N = 1 << 31
C3_CHUNK = 1 << 24


_C3_EDGES = None  # the edge array, in a shared mapping the forked workers write into


def _c3_hash(args):
    c0, c1, seed, P = args
    data, offs = workloads.str_keys(c1 - c0, gen_seed=0, start=c0)
    _C3_EDGES[c0:c1] = oracle.Oracle().hash_str(data, offs, seed, P)
    return c1 - c0


def make_c3(procs: int) -> None:
    import mmap

    global _C3_EDGES
    o = oracle.Oracle()
    o.lib.orc_set_progress(1)
    n = C3_N
    P = o.part_size(n)
    m = 3 * P
    buf = mmap.mmap(-1, n * 12)  # anonymous and shared: the pool's forked workers see the same pages
    try:
        edges = np.frombuffer(buf, dtype=np.uint32).reshape(n, 3)
        _C3_EDGES = edges
        t_all = time.time()
        for t in range(MAX_TRIES):
            seed = t
            t0 = time.time()
            jobs = [(c0, min(n, c0 + C3_CHUNK), seed, P) for c0 in range(0, n, C3_CHUNK)]
            done = 0
            with mp.get_context("fork").Pool(procs) as pool:
                for k in pool.imap_unordered(_c3_hash, jobs):
                    done += k
                    if done % (1 << 28) < C3_CHUNK:
                        log(f"[c3] try {t}: {done}/{n} keys generated and hashed, {time.time() - t0:.0f} s")
            t_hash = time.time() - t0
            t0 = time.time()
            log("[c3] peeling (single-threaded oracle)")
            rc, pe = o.peel(edges, m, P)
            t_peel = time.time() - t0
            log(f"[c3] try {t}: status {rc}, {pe['n_peeled']} of {n} edges peeled in {pe['n_rounds']} rounds, "
                f"{t_peel:.0f} s")
            if rc != 0:
                raise RuntimeError(f"oracle peel status {rc}")
            if pe["n_peeled"] == n:
                break
            del pe
        else:
            raise RuntimeError("2-core on every try")
        t0 = time.time()
        codes8 = o.assign(edges, m, pe["order"], pe["round"], pe["hinge"])
        if isinstance(codes8, tuple):
            rc, codes8 = codes8
            if rc != 0:
                raise RuntimeError(f"oracle assign status {rc}")
        rounds = pe["n_rounds"]
        del pe
        words, rank = o.pack_rank(codes8)
        t_assign = time.time() - t0
        log(f"[c3] assignment and packing {t_assign:.0f} s")
        _C3_EDGES = None
        del edges
    finally:
        buf.close()
    hw = hashlib.sha256(words.tobytes()).hexdigest()
    hr = hashlib.sha256(rank.tobytes()).hexdigest()
    with open(C3_FILE, "w") as fh:
        fh.write("# Oracle MWHC MPHF of 2^31 byte-string keys (generator seed 0: log-normal lengths, mean 60 B, clamped\n"
                 "# 8..512 B), hash seed 0, gamma 123/100.  Written by tests/golden/make_fullsize.py c3 (keys generated\n"
                 "# and hashed per chunk in worker processes; the oracle's peel, assignment and packing run once).\n"
                 f"# hash {t_hash:.0f} s on {procs} processes, peel {t_peel:.0f} s, assign + pack {t_assign:.0f} s "
                 f"(single-threaded), total {time.time() - t_all:.0f} s\n")
        fh.write(f"n {n}\nP {P}\nseed_used {seed}\ntries {seed + 1}\nn_rounds {rounds}\n"
                 f"code_words {len(words)}\nrank_words {len(rank)}\ncodes_sha256 {hw}\nrank_sha256 {hr}\n")
    log(f"[c3] wrote {C3_FILE}")


def read_c3():
    out = {}
    with open(C3_FILE) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.split()
            out[k] = v if k.endswith("sha256") else int(v)
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("config", choices=["c3", "c4", "c5"])
    ap.add_argument("--procs", type=int, default=min(16, os.cpu_count() or 1))
    a = ap.parse_args()
    oracle.compile_oracle()
    {"c3": make_c3, "c4": make_c4, "c5": make_c5}[a.config](a.procs)
    return 0


if __name__ == "__main__":
    sys.exit(main())
