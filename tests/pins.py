"""Checks that pin the oracle to facts outside itself.

Each ``pin_*`` function takes an ``oracle.Oracle`` and returns a list of failure messages
(empty = pinned).  The same battery runs against the real oracle (must pass) and against
copies with planted mistakes (each must fail at least one pin).

Sources of truth used here, none of which is the oracle's own code:
  * published SplitMix64 outputs for state 0 (Steele, Lea & Flood 2014; the same values as
    Java's ``new SplittableRandom(0).nextLong()``), plus the closed form of the range
    reduction when P is a power of two;
  * hand-derived worked examples (tests/golden/worked_examples.json);
  * a definition-direct synchronous peel that recomputes every degree from scratch each
    round (brute force, O(n * rounds));
  * an exhaustive search of the maximum 2-core over all edge subsets (tiny inputs);
  * invariants of the definitions: a peeling order leaves every edge's hinge in no later
    edge; the 2-core has minimum degree 2; f(x) = g0+g1+g2 mod 3 equals the hinge; the MPHF
    is a bijection onto [0, n); rank equals a prefix count;
  * the paper's printed numbers: 2.61 bits/key for MWHC (Table 1) and the 2-core fraction
    p^3 of a random 3-hypergraph below the threshold (p = 1 - exp(-(3/gamma) p^2)), whose
    threshold is c_3 ~ 1.221 (Section 1).
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

import workloads

NONE = 0xFFFFFFFF
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "worked_examples.json")

# SplitMix64, state 0: outputs 1..3 (published known answers).
SPLITMIX0 = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def golden():
    with open(GOLDEN) as f:
        return json.load(f)


# --------------------------------------------------------------------------------------------
# independent helpers (brute force, written from the definitions)
# --------------------------------------------------------------------------------------------
def bf_sync_peel(edges: np.ndarray, m: int):
    """Synchronous layered peel by definition: every round recompute degrees over the edges
    still present; an edge leaves in this round iff one of its vertices has degree 1; its
    hinge is the lowest position holding such a vertex."""
    edges = _as_tuples(edges)
    n = len(edges)
    alive = np.ones(n, bool)
    rnd = np.full(n, NONE, np.uint32)
    hinge = np.full(n, 0xFF, np.uint8)
    r = 0
    while True:
        deg = np.bincount(edges[alive].ravel(), minlength=m) if alive.any() else np.zeros(m, np.int64)
        d1 = deg[edges] == 1
        go = alive & d1.any(axis=1)
        if not go.any():
            break
        rnd[go] = r
        hinge[go] = np.argmax(d1[go], axis=1)
        alive &= ~go
        r += 1
    key = np.where(rnd == NONE, r, rnd).astype(np.int64)
    order = np.lexsort((np.arange(n), key)).astype(np.uint32)
    return dict(round=rnd, hinge=hinge, core_mask=alive.astype(np.uint8), order=order, n_rounds=r)


def _as_tuples(edges) -> np.ndarray:
    """Edges as an (n, r) int64 array: a 2-D input keeps its width, a flat one is read as r = 3."""
    a = np.asarray(edges, dtype=np.int64)
    return a if a.ndim == 2 else a.reshape(-1, 3)


def bf_max_core(edges) -> set:
    """Largest edge subset in which every vertex that appears has degree >= 2, by trying every
    subset.  Such subsets are closed under union, so the largest is their union."""
    edges = [tuple(int(v) for v in e) for e in edges]
    n = len(edges)
    union = 0
    for mask in range(1, 1 << n):
        deg = {}
        for i in range(n):
            if mask >> i & 1:
                for v in edges[i]:
                    deg[v] = deg.get(v, 0) + 1
        if min(deg.values()) >= 2:
            union |= mask
    return {i for i in range(n) if union >> i & 1}


def random_tripartite(n, P, rng):
    e = rng.integers(0, P, size=(n, 3), dtype=np.int64)
    e[:, 1] += P
    e[:, 2] += 2 * P
    return e.astype(np.uint32)


def random_generic(n, m, rng):
    out = np.empty((n, 3), np.uint32)
    for i in range(n):
        out[i] = rng.choice(m, size=3, replace=False)
    return out


def peeling_order_ok(edges, order, hinge, n_peeled) -> bool:
    """Definition of a peeling order (Section 1): when an edge is removed, its hinge vertex has
    degree 1, i.e. it occurs in no edge placed later (core edges sit after every peeled one)."""
    edges = _as_tuples(edges)
    n, r = edges.shape
    if n == 0:
        return True
    pos = np.empty(n, np.int64)
    pos[np.asarray(order, dtype=np.int64)] = np.arange(n)
    m = int(edges.max()) + 1
    last = np.full(m, -1, np.int64)
    np.maximum.at(last, edges.ravel(), np.repeat(pos, r))
    peeled = np.asarray(order[:n_peeled], dtype=np.int64)
    h = edges[peeled, np.asarray(hinge, dtype=np.int64)[peeled]]
    return bool(np.all(last[h] == pos[peeled]))


def core_min_degree_ok(edges, core_mask) -> bool:
    edges = _as_tuples(edges)
    c = edges[np.asarray(core_mask, bool)]
    if len(c) == 0:
        return True
    deg = np.bincount(c.ravel())
    return bool(np.all(deg[c.ravel()] >= 2))


def unpack_codes(words, m):
    w = np.asarray(words, dtype=np.uint64)
    sh = (2 * np.arange(32, dtype=np.uint64))
    c = ((w[:, None] >> sh[None, :]) & np.uint64(3)).astype(np.uint8).ravel()
    return c[:m]


def core_fraction_closed_form(gamma: float, r: int = 3) -> float:
    """Fraction of the edges in the 2-core of a random r-hypergraph with gamma vertices per edge:
    p^r, p the largest root of p = 1 - exp(-(r/gamma) p^(r-1)) (Molloy's CORE analysis)."""
    lam = r / gamma
    p = 1.0
    for _ in range(100000):
        p = 1.0 - math.exp(-lam * p ** (r - 1))
    return p ** r


def random_uniform_r(n, m, r, rng):
    """n edges of r distinct vertices below m (rows with a repeat are drawn again)."""
    e = rng.integers(0, m, size=(n, r), dtype=np.int64)
    while True:
        s = np.sort(e, axis=1)
        bad = (s[:, 1:] == s[:, :-1]).any(axis=1)
        if not bad.any():
            return e.astype(np.uint32)
        e[bad] = rng.integers(0, m, size=(int(bad.sum()), r), dtype=np.int64)


# --------------------------------------------------------------------------------------------
# pins
# --------------------------------------------------------------------------------------------
def pin_splitmix(o) -> list:
    bad = []
    for t, want in enumerate(SPLITMIX0, start=1):
        got = o.splitmix(0, t)
        if got != want:
            bad.append(f"splitmix(0,{t}) = {got:#x}, published {want:#x}")
    return bad


def pin_hash_closed_form(o) -> list:
    """With P = 2^30 the range reduction floor(z*P/2^64) is z >> 34, so key 0 under seed 0
    (state 0) lands on the published stream outputs shifted by 34, offset into parts 0/1/2.
    key XOR seed is the stream state, so (key=K, seed=K) lands there too."""
    bad = []
    P = 1 << 30
    want = [SPLITMIX0[0] >> 34, P + (SPLITMIX0[1] >> 34), 2 * P + (SPLITMIX0[2] >> 34)]
    for key, seed in [(0, 0), (0xDEADBEEF12345678, 0xDEADBEEF12345678)]:
        got = o.hash_u64(np.array([key], np.uint64), seed, P)[0].tolist()
        if got != want:
            bad.append(f"hash(key={key:#x}, seed={seed:#x}, P=2^30) = {got}, expected {want}")
    # P = 1: everything collapses onto vertices 0, 1, 2.
    got = o.hash_u64(np.array([12345], np.uint64), 7, 1)[0].tolist()
    if got != [0, 1, 2]:
        bad.append(f"hash with P=1 = {got}")
    return bad


def pin_part_size(o) -> list:
    bad = []
    for n, gnum, gden, want in [(1_000_000, 123, 100, 410_000), (1 << 27, 123, 100, 55_029_269),
                                (1 << 31, 123, 100, 880_468_296), (1 << 27, 120, 100, 53_687_092),
                                (1, 123, 100, 1), (0, 123, 100, 0), (3, 1, 1, 1), (4, 1, 1, 2)]:
        got = o.part_size(n, gnum, gden)
        if got != want:
            bad.append(f"P(n={n}, {gnum}/{gden}) = {got}, expected {want}")
    return bad


def pin_worked_examples(o) -> list:
    bad = []
    g = golden()
    m = g["m"]
    for name in ("E1", "E2"):
        ex = g[name]
        edges = np.array(ex["edges"], np.uint32)
        for part in (g["P"], 0):
            rc, r = o.peel(edges, m, part)
            if rc != 0:
                bad.append(f"{name}: peel status {rc}")
                continue
            for key in ("round", "hinge", "order", "core_mask"):
                got = r[key].tolist()
                want = ex[key]
                if key == "hinge":  # hinge is unspecified for core edges
                    got = [h if c == 0 else 255 for h, c in zip(got, ex["core_mask"])]
                if got != want:
                    bad.append(f"{name} (part={part}): {key} {got} != {want}")
            if r["n_rounds"] != ex["n_rounds"]:
                bad.append(f"{name}: n_rounds {r['n_rounds']} != {ex['n_rounds']}")
        if "codes" in ex:
            rc, r = o.peel(edges, m, g["P"])
            rc, codes = o.assign(edges, m, r["order"], r["round"], r["hinge"])
            if rc != 0 or codes.tolist() != ex["codes"]:
                bad.append(f"{name}: codes {codes.tolist()} != {ex['codes']}")
                continue
            words, rank = o.pack_rank(codes)
            c = unpack_codes(words, m)
            gv = c % 3
            prefix = np.concatenate([[0], np.cumsum(c != 0)])
            vals = []
            for e in edges:
                i = int(gv[e].sum() % 3)
                vals.append(int(prefix[e[i]]))
            if vals != ex["mphf"]:
                bad.append(f"{name}: mphf {vals} != {ex['mphf']}")
            if gv.tolist() != ex["g"]:
                bad.append(f"{name}: g {gv.tolist()} != {ex['g']}")
    return bad


def pin_bruteforce_tripartite(o, trials=(200, 1000, 3000), seed=1) -> list:
    bad = []
    rng = np.random.default_rng(seed)
    for n in trials:
        for gamma in (1.05, 1.23, 1.4):
            P = max(1, math.ceil(gamma * n / 3))
            edges = random_tripartite(n, P, rng)
            rc, r = o.peel(edges, 3 * P, P)
            b = bf_sync_peel(edges, 3 * P)
            if rc != 0:
                bad.append(f"tripartite n={n} gamma={gamma}: status {rc}")
                continue
            peeled = b["core_mask"] == 0
            for key in ("round", "core_mask", "order"):
                if not np.array_equal(r[key], b[key]):
                    bad.append(f"tripartite n={n} gamma={gamma}: {key} differs from brute force")
            if not np.array_equal(r["hinge"][peeled], b["hinge"][peeled]):
                bad.append(f"tripartite n={n} gamma={gamma}: hinge differs from brute force")
            if r["n_rounds"] != b["n_rounds"]:
                bad.append(f"tripartite n={n} gamma={gamma}: rounds {r['n_rounds']} != {b['n_rounds']}")
    return bad


def pin_bruteforce_generic(o, seed=2) -> list:
    bad = []
    rng = np.random.default_rng(seed)
    for trial in range(40):
        n = int(rng.integers(1, 11))
        m = int(rng.integers(3, 9))
        edges = random_generic(n, m, rng)
        rc, r = o.peel(edges, m, 0)
        if rc != 0:
            bad.append(f"generic trial {trial}: status {rc}")
            continue
        core = set(np.nonzero(r["core_mask"])[0].tolist())
        if core != bf_max_core(edges):
            bad.append(f"generic trial {trial}: core {sorted(core)} != max 2-core")
        b = bf_sync_peel(edges, m)
        peeled = b["core_mask"] == 0
        if not (np.array_equal(r["round"], b["round"]) and np.array_equal(r["order"], b["order"])
                and np.array_equal(r["hinge"][peeled], b["hinge"][peeled])):
            bad.append(f"generic trial {trial}: differs from brute-force synchronous peel")
    return bad


def pin_invariants(o, n=20000, seed=3) -> list:
    bad = []
    keys = workloads.u64_keys(n, gen_seed=seed)
    for gnum in (123, 118):
        P = o.part_size(n, gnum, 100)
        edges = o.hash_u64(keys, 0, P)
        rc, r = o.peel(edges, 3 * P, P)
        if rc != 0:
            return [f"invariants: status {rc}"]
        if not peeling_order_ok(edges, r["order"], r["hinge"], r["n_peeled"]):
            bad.append(f"invariants gamma={gnum}/100: order is not a peeling order")
        if not core_min_degree_ok(edges, r["core_mask"]):
            bad.append(f"invariants gamma={gnum}/100: core has a vertex of degree 1")
        if int(np.sum(r["core_mask"])) != n - r["n_peeled"]:
            bad.append("invariants: core count mismatch")
        if gnum == 123:
            if r["n_peeled"] != n:
                bad.append("invariants: gamma=1.23 did not peel completely")
                continue
            rc, codes = o.assign(edges, 3 * P, r["order"], r["round"], r["hinge"])
            gv = codes.astype(np.int64) % 3
            s = gv[edges.astype(np.int64)].sum(axis=1) % 3
            if not np.array_equal(s, r["hinge"].astype(np.int64)):
                bad.append("invariants: g0+g1+g2 mod 3 != hinge for some key")
            hv = edges[np.arange(n), r["hinge"].astype(np.int64)]
            if not np.all(codes[hv] != 0) or int(np.sum(codes != 0)) != n:
                bad.append("invariants: hinge vertices are not exactly the used vertices")
            words, rank = o.pack_rank(codes)
            if not np.array_equal(unpack_codes(words, 3 * P), codes):
                bad.append("invariants: packed codes do not unpack to the code vector")
            prefix = np.concatenate([[0], np.cumsum(codes != 0)])
            if not np.array_equal(rank, prefix[np.arange(len(rank)) * 512]):
                bad.append("invariants: rank sample != prefix count")
            # permuting edges inside each layer leaves g unchanged (Section 4.2)
            rng = np.random.default_rng(seed)
            order2 = r["order"].copy()
            rr = r["round"][order2]
            for lay in range(r["n_rounds"]):
                idx = np.nonzero(rr == lay)[0]
                order2[idx] = order2[idx][rng.permutation(len(idx))]
            rc2, codes2 = o.assign(edges, 3 * P, order2, r["round"], r["hinge"])
            if rc2 != 0 or not np.array_equal(codes, codes2):
                bad.append("invariants: within-layer order changed the assignment")
    return bad


def pin_mphf(o, n=30000, seed=4) -> list:
    bad = []
    keys = workloads.u64_keys(n, gen_seed=seed)
    rc, r = o.mphf_build_u64(keys, seed=9)
    if rc != 0:
        return [f"mphf u64: status {rc}"]
    f = o.lookup_u64(r["words"], r["rank"], r["P"], r["seed_used"], keys)
    if not np.array_equal(np.sort(f), np.arange(n, dtype=np.uint64)):
        bad.append("mphf u64: lookup is not a bijection onto [0, n)")
    bits = (2 * r["m"] + 64 * len(r["rank"])) / n
    if abs(bits - 2.61) > 0.01:
        bad.append(f"mphf u64: {bits:.4f} bits/key, Table 1 prints 2.61")
    data, offs = workloads.str_keys(n // 3, gen_seed=seed)
    rc, r = o.mphf_build_str(data, offs, seed=5)
    if rc != 0:
        return bad + [f"mphf str: status {rc}"]
    f = o.lookup_str(r["words"], r["rank"], r["P"], r["seed_used"], data, offs)
    if not np.array_equal(np.sort(f), np.arange(n // 3, dtype=np.uint64)):
        bad.append("mphf str: lookup is not a bijection onto [0, n)")
    return bad


def pin_errors(o) -> list:
    bad = []
    keys = workloads.u64_keys(1000)
    dup = np.concatenate([keys, keys[:3]])
    rc, r = o.mphf_build_u64(dup, max_tries=3)
    if rc != 2:
        bad.append(f"duplicate keys: status {rc}, expected EDUP")
    rc, r = o.mphf_build_u64(workloads.u64_keys(20000), gnum=120, max_tries=1)
    if rc != 1:
        bad.append(f"gamma below threshold, one try: status {rc}, expected ECORE")
    star = np.array([[0, 1 + i, 300 + i] for i in range(256)], np.uint32)
    rc, r = o.peel(star, 600, 0)
    if rc != -2:
        bad.append(f"degree 256: status {rc}, expected ERANGE")
    rc, r = o.peel(star[:255], 600, 0)
    if rc != 0:
        bad.append(f"degree 255: status {rc}, expected OK")
    for e, m in (([[0, 1, 5]], 5), ([[0, 1, 1]], 5)):
        rc, r = o.peel(np.array(e, np.uint32), m, 0)
        if rc != -1:
            bad.append(f"edge {e} with m={m}: status {rc}, expected EINVAL")
    return bad


def pin_general_r(o, seed=9) -> list:
    """r-hypergraphs, 2 <= r <= 8: tiny inputs against the exhaustive maximum 2-core and the
    definition-direct synchronous peel; r = 3 against the tripartite-free r = 3 peel; the
    peeling-order invariants at r = 5; the 2-core fraction at r = 4 against its closed form on
    both sides of the threshold (c*_4 = 0.772 edges per vertex, gamma* = 1.295); the errors."""
    bad = []
    rng = np.random.default_rng(seed)
    for r in (2, 4, 5, 8):
        for trial in range(25):
            n = int(rng.integers(1, 11))
            m = int(rng.integers(r, r + 7))
            edges = random_uniform_r(n, m, r, rng)
            rc, got = o.peel_r(edges, m, r)
            if rc != 0:
                bad.append(f"r={r} trial {trial}: status {rc}")
                continue
            if set(np.nonzero(got["core_mask"])[0].tolist()) != bf_max_core(edges):
                bad.append(f"r={r} trial {trial}: core differs from the maximum 2-core")
            b = bf_sync_peel(edges, m)
            peeled = b["core_mask"] == 0
            if not (np.array_equal(got["round"], b["round"]) and np.array_equal(got["order"], b["order"])
                    and np.array_equal(got["hinge"][peeled], b["hinge"][peeled])):
                bad.append(f"r={r} trial {trial}: differs from the synchronous peel by definition")
    edges = random_uniform_r(3000, 3600, 3, rng)
    rc3, a = o.peel(edges, 3600, 0)
    rcr, b = o.peel_r(edges, 3600, 3)
    if rc3 != rcr or any(not np.array_equal(a[k], b[k]) for k in ("order", "round", "core_mask", "hinge")):
        bad.append("r = 3 differs from the three-vertex peel")
    edges = random_uniform_r(20_000, 30_000, 5, rng)
    rc, got = o.peel_r(edges, 30_000, 5)
    if rc != 0 or not peeling_order_ok(edges, got["order"], got["hinge"], got["n_peeled"]):
        bad.append("r = 5: not a peeling order")
    if not core_min_degree_ok(edges, got["core_mask"]):
        bad.append("r = 5: a core vertex of degree below 2")
    n = 200_000
    for gamma in (1.20, 1.40):
        m = int(gamma * n)
        rc, got = o.peel_r(random_uniform_r(n, m, 4, rng), m, 4)
        frac = 1.0 - got["n_peeled"] / n
        want = core_fraction_closed_form(gamma, 4)
        if rc != 0 or abs(frac - want) > 0.01:
            bad.append(f"r = 4, gamma = {gamma}: core fraction {frac:.4f}, closed form {want:.4f}")
    star = np.array([[0, 1 + i] for i in range(256)], np.uint32)
    if o.peel_r(star, 257, 2)[0] != -2 or o.peel_r(star[:255], 256, 2)[0] != 0:
        bad.append("r = 2: degree 256 must give ERANGE and 255 not")
    if o.peel_r(np.array([[0, 1, 1, 2]], np.uint32), 3, 4)[0] != -1:
        bad.append("r = 4: a repeated vertex must give EINVAL")
    if o.peel_r(np.array([[0, 5]], np.uint32), 5, 2)[0] != -1:
        bad.append("r = 2: a vertex id >= m must give EINVAL")
    for r in (1, 9):
        if o.peel_r(np.zeros((1, r), np.uint32), 10, r)[0] != -1:
            bad.append(f"r = {r} must give EINVAL")
    return bad


def pin_threshold(o, n=200_000) -> list:
    """Section 1: above c_3 ~ 1.221 the 2-core is empty w.h.p.; below it the core holds the
    fraction p^3 of the edges (p the largest root of p = 1 - exp(-(3/gamma) p^2))."""
    bad = []
    keys = workloads.u64_keys(n)
    for gnum, want in ((123, 0.0), (120, core_fraction_closed_form(1.20)), (110, core_fraction_closed_form(1.10))):
        P = o.part_size(n, gnum, 100)
        rc, r = o.peel(o.hash_u64(keys, 0, P), 3 * P, P)
        frac = 1.0 - r["n_peeled"] / n
        if abs(frac - want) > 0.01:
            bad.append(f"gamma={gnum}/100: core fraction {frac:.4f}, closed form {want:.4f}")
    return bad


def pin_string_digest(o) -> list:
    """Properties of the byte-string digest that a dropped term, a wrong index or a missing
    zero-padding would break."""
    bad = []
    d = o.digest_str

    def differ(x, y):  # both lanes must change
        return x[0] != y[0] and x[1] != y[1]

    a, b = d(b"abcdefgh12345678", 0)
    if a == b:
        bad.append("digest lanes are not independent")
    if not differ(d(b"abcdefgh12345678", 0), d(b"12345678abcdefgh", 0)):
        bad.append("digest ignores word positions")
    if not (differ(d(b"abc", 0), d(b"abc\x00", 0)) and differ(d(b"", 0), d(b"\x00", 0))):
        bad.append("digest ignores the key length")
    if not differ(d(b"abc", 0), d(b"abc", 1)):
        bad.append("digest ignores the seed")
    if not (differ(d(b"abcdefghi", 0), d(b"abcdefghj", 0)) and differ(d(b"xbcdefgh", 0), d(b"abcdefgh", 0))):
        bad.append("digest ignores some byte")
    # keys embedded with different trailing garbage hash the same (no read past the end)
    data1 = np.frombuffer(b"hello world!XXXXXXXX", np.uint8)
    data2 = np.frombuffer(b"hello world!YYYYYYYY", np.uint8)
    offs = np.array([0, 12], np.uint64)
    if not np.array_equal(o.hash_str(data1, offs, 3, 1000), o.hash_str(data2, offs, 3, 1000)):
        bad.append("string hash reads past the key")
    # vertices spread evenly over each part (chi-square, 64 bins per part)
    data, offs = workloads.str_keys(40000)
    P = 1 << 20
    e = o.hash_str(data, offs, 0, P).astype(np.int64)
    for k in range(3):
        loc = e[:, k] - k * P
        if loc.min() < 0 or loc.max() >= P:
            bad.append(f"string hash part {k} out of range")
            continue
        h = np.bincount(loc >> 14, minlength=64)
        chi2 = float(((h - len(loc) / 64) ** 2 / (len(loc) / 64)).sum())
        if chi2 > 130:  # 63 degrees of freedom; p < 1e-6 above this
            bad.append(f"string hash part {k}: chi2 {chi2:.1f}")
    return bad


def pin_static_function(o, seed=6) -> list:
    """Static functions (Section 3): the lookup returns every key's value for several sigma;
    u is zero off the hinges; with sigma = 3 and the hinge positions as values, u is the MPHF's
    g (two separate assignments); the packed layout equals the closed form sum of u[v] << b*v."""
    bad = []
    rng = np.random.default_rng(seed)
    n = 20000
    keys = workloads.u64_keys(n, gen_seed=seed)
    for sigma in (1, 2, 3, 7, 256, 1_000_003, 1 << 32):
        values = (rng.integers(0, sigma, n, dtype=np.uint64)).astype(np.uint32)
        rc, r = o.sf_build_u64(keys, values, sigma, seed=1)
        if rc != 0:
            bad.append(f"sf u64 sigma={sigma}: status {rc}")
            continue
        b = o.sf_bits(sigma)
        if b != (sigma - 1).bit_length() or len(r["words"]) != (r["m"] * b + 63) // 64:
            bad.append(f"sf sigma={sigma}: {b} bits, {len(r['words'])} words")
        f = o.sf_lookup_u64(r["words"], sigma, r["P"], r["seed_used"], keys)
        if not np.array_equal(f, values.astype(np.uint64)):
            bad.append(f"sf u64 sigma={sigma}: lookup differs from the values at {int((f != values).sum())} keys")
    data, offs = workloads.str_keys(7000, gen_seed=seed)
    values = rng.integers(0, 1000, 7000).astype(np.uint32)
    rc, r = o.sf_build_str(data, offs, values, 1000, seed=2)
    f = o.sf_lookup_str(r["words"], 1000, r["P"], r["seed_used"], data, offs) if rc == 0 else None
    if rc != 0 or not np.array_equal(f, values.astype(np.uint64)):
        bad.append(f"sf str: status {rc} or lookup differs from the values")
    # zero off the hinges; the MPHF is the case sigma = 3, f = hinge position
    P = o.part_size(5000)
    for hseed in range(20):  # the first hash seed whose graph peels completely
        edges = o.hash_u64(workloads.u64_keys(5000, gen_seed=seed + 1), hseed, P)
        rc, pr = o.peel(edges, 3 * P, P)
        if rc == 0 and pr["n_peeled"] == 5000:
            break
    if rc == 0 and pr["n_peeled"] == 5000:
        vals = rng.integers(0, 97, 5000).astype(np.uint32)
        rc1, u = o.sf_assign(edges, 3 * P, pr["order"], pr["round"], pr["hinge"], vals, 97)
        hinges = np.zeros(3 * P, bool)
        hinges[edges[np.arange(5000), pr["hinge"].astype(np.int64)]] = True
        if rc1 != 0 or (u[~hinges] != 0).any() or (u >= 97).any():
            bad.append("sf: u not zero off the hinges or not below sigma")
        rc2, u3 = o.sf_assign(edges, 3 * P, pr["order"], pr["round"], pr["hinge"], pr["hinge"].astype(np.uint32), 3)
        rc3, codes8 = o.assign(edges, 3 * P, pr["order"], pr["round"], pr["hinge"])
        if rc2 != 0 or rc3 != 0 or not np.array_equal(u3, (codes8 % 3).astype(np.uint32)):
            bad.append("sf: sigma = 3 with the hinge positions does not give the MPHF's g")
    else:
        bad.append("sf: the 5000-edge test graph did not peel")
    # packing: v's b bits at bit b*v of the little-endian bit string (straddling word ends)
    for b_sigma, count in ((32, 5), (128, 10), (1 << 20, 7), (1 << 32, 3)):
        u = rng.integers(0, b_sigma, count, dtype=np.uint64).astype(np.uint32)
        b = (b_sigma - 1).bit_length()
        big = sum(int(x) << (b * v) for v, x in enumerate(u))
        nw = (count * b + 63) // 64
        want = np.array([(big >> (64 * w)) & ((1 << 64) - 1) for w in range(nw)], np.uint64)
        if not np.array_equal(o.sf_pack(u, b_sigma), want):
            bad.append(f"sf pack b={b}: differs from the closed form")
    # values outside [0, sigma) and sigma = 0 are rejected
    rc, _ = o.sf_build_u64(keys[:100], np.full(100, 7, np.uint32), 7)
    rc0, _ = o.sf_build_u64(keys[:100], np.zeros(100, np.uint32), 0)
    if rc != -1 or rc0 != -1:
        bad.append(f"sf: value >= sigma gave {rc}, sigma = 0 gave {rc0} (EINVAL expected)")
    return bad


def pin_hem(o) -> list:
    """HEM split (Section 3): the u64 signature is SplitMix64 output 4 at state key XOR seed
    (published outputs: state -(4-t)*GAMMA gives output t of state 0); each bucket holds
    exactly the keys whose signatures carry its top bits; with one bucket the structure is the
    MWHC MPHF of the half-swapped signatures; the function is a bijection onto [0, n) for u64
    and string keys and several bucket counts."""
    bad = []
    G = 0x9E3779B97F4A7C15
    for t, want in enumerate(SPLITMIX0, start=1):
        key = (-(4 - t) * G) % (1 << 64)
        if int(o.hem_signatures_u64(np.array([key], np.uint64), 0)[0]) != want:
            bad.append(f"hem signature of state -{4 - t}*GAMMA is not published output {t}")
        if int(o.hem_signatures_u64(np.array([key ^ 0x1234], np.uint64), 0x1234)[0]) != want:
            bad.append("hem signature does not depend on key XOR seed alone")
    n = 40_000
    keys = workloads.u64_keys(n, gen_seed=11)
    sigs = o.hem_signatures_u64(keys, 5)
    for k in (0, 1, 6, 10):
        rc, r = o.hem_build(sigs, k, seed=5)
        if rc != 0:
            bad.append(f"hem k={k}: status {rc}")
            continue
        bo = r["bucket_off"].astype(np.int64)
        top = (sigs >> np.uint64(64 - k)).astype(np.int64) if k else np.zeros(n, np.int64)
        if bo[-1] != n or not np.array_equal(np.diff(bo), np.bincount(top, minlength=1 << k)):
            bad.append(f"hem k={k}: bucket sizes differ from the signatures' top bits")
        f = o.hem_lookup(r, sigs)
        if not np.array_equal(np.sort(f), np.arange(n, dtype=np.uint64)):
            bad.append(f"hem k={k}: lookup is not a bijection onto [0, n)")
        if k == 0:
            swapped = (sigs << np.uint64(32)) | (sigs >> np.uint64(32))
            rc1, one = o.mphf_build_u64(swapped, seed=5)
            if rc1 != 0 or not np.array_equal(one["words"], r["codes"]) or not np.array_equal(one["rank"], r["rank"]):
                bad.append("hem k=0: not the MWHC MPHF of the half-swapped signatures")
        if k == 6:
            for b in (0, 17, 63):
                inb = np.sort(f[top == b])
                if not np.array_equal(inb, np.arange(bo[b], bo[b + 1], dtype=np.uint64)):
                    bad.append(f"hem k=6: bucket {b}'s keys do not map onto its own range")
    # string keys: the signature is the whole 128-bit digest, the bucket the top bits of its
    # first word
    data, offs = workloads.str_keys(9000, gen_seed=12)
    sg = o.hem_signatures_str(data, offs, 2)
    for i in (0, 4321, 8999):
        a_, b_ = o.digest_str(bytes(data[offs[i]:offs[i + 1]]), 2)
        if (int(sg[i, 0]), int(sg[i, 1])) != (a_, b_):
            bad.append("hem string signature is not the key's 128-bit digest")
    rc, r = o.hem_build(sg, 3, seed=2)
    f = o.hem_lookup(r, sg) if rc == 0 else None
    if rc != 0 or not np.array_equal(np.sort(f), np.arange(9000, dtype=np.uint64)):
        bad.append(f"hem strings: status {rc} or not a bijection")
    elif not np.array_equal(np.diff(r["bucket_off"].astype(np.int64)),
                            np.bincount((sg[:, 0] >> np.uint64(61)).astype(np.int64), minlength=8)):
        bad.append("hem strings: buckets are not the top bits of the signature's first word")
    # a 128-bit signature whose second word is the first with its halves swapped stands for the
    # same bucket key as the 64-bit signature: both splits are the same structure
    sw = (sigs << np.uint64(32)) | (sigs >> np.uint64(32))
    for k in (0, 6):
        rc1, r1 = o.hem_build(sigs, k, seed=5)
        rc2, r2 = o.hem_build(np.stack([sigs, sw], axis=1), k, seed=5)
        if rc1 != 0 or rc2 != 0 or any(not np.array_equal(r1[x], r2[x]) for x in
                                      ("bucket_off", "seeds", "codes", "rank")):
            bad.append(f"hem k={k}: a 128-bit signature (s, swap(s)) differs from the 64-bit signature s")
    # signatures that agree in their first word and differ in the second are distinct keys:
    # no collision, the split is a bijection
    rng = np.random.default_rng(3)
    pairs = rng.integers(0, 1 << 63, size=(3000, 2), dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    pairs[2970:, 0] = pairs[:30, 0]
    rc, r = o.hem_build(pairs, 2, seed=9)
    f = o.hem_lookup(r, pairs) if rc == 0 else None
    if rc != 0 or not np.array_equal(np.sort(f), np.arange(3000, dtype=np.uint64)):
        bad.append(f"hem: signatures sharing their first word collide (status {rc})")
    return bad


def pin_sf_ranked(o, seed=11) -> list:
    """Ranked static-function layout (Section 3: ceil(log sigma) n + gamma n + o(n) bits with
    a ranking structure). A hand-worked layout; on built functions every key's lookup through
    the ranking structure returns its value, at most n fields are kept (u is zero off the
    hinges) and the space stays within b n + m + the rank samples."""
    bad = []
    # Worked example: m = 2100 vertices (blocks of 1024: two whole, one of 52), sigma = 8 (3
    # bits), non-zero values u[0] = 5, u[63] = 1, u[64] = 7, u[1023] = 2, u[1024] = 3,
    # u[2099] = 4.  Marks: word 0 bits 0 and 63, word 1 bit 0, word 15 bit 63, word 16 bit 0,
    # word 32 bit 51 (2099 = 32 * 64 + 51).  Rank samples: 0 below vertex 0, 4 below 1024,
    # 5 below 2048, 6 in all.  Fields 5, 1, 7, 2, 3, 4 at bits 0, 3, 6, 9, 12, 15 form the
    # word 5 + 8 + 448 + 1024 + 12288 + 131072 = 144845.
    u = np.zeros(2100, np.uint32)
    for v, x in ((0, 5), (63, 1), (64, 7), (1023, 2), (1024, 3), (2099, 4)):
        u[v] = x
    lay = o.sf_rank_layout(o.sf_pack(u, 8), 2100, 8)
    want_marks = np.zeros(33, np.uint64)
    want_marks[0] = 0x8000000000000001
    want_marks[1] = 1
    want_marks[15] = 0x8000000000000000
    want_marks[16] = 1
    want_marks[32] = 0x0008000000000000
    if (lay["count"] != 6 or not np.array_equal(lay["marks"], want_marks)
            or lay["rank"].tolist() != [0, 4, 5, 6] or lay["vals"].tolist() != [144845]):
        bad.append(f"sf ranked: worked example gave count {lay['count']}, rank {lay['rank'].tolist()}, "
                   f"vals {lay['vals'].tolist()}")
    # built functions: lookups through the ranking structure, the field count, the space
    rng = np.random.default_rng(seed)
    n = 20000
    keys = workloads.u64_keys(n, gen_seed=seed)
    for sigma in (1, 2, 256, 1_000_003, 1 << 32):
        values = rng.integers(0, sigma, n, dtype=np.uint64).astype(np.uint32)
        rc, r = o.sf_build_u64(keys, values, sigma, seed=3)
        if rc != 0:
            bad.append(f"sf ranked sigma={sigma}: status {rc}")
            continue
        b, m = o.sf_bits(sigma), r["m"]
        lay = o.sf_rank_layout(r["words"], m, sigma)
        f = o.sfr_lookup_u64(lay["marks"], lay["rank"], lay["vals"], sigma, r["P"], r["seed_used"], keys)
        if not np.array_equal(f, values.astype(np.uint64)):
            bad.append(f"sf ranked sigma={sigma}: lookup differs from the values at {int((f != values).sum())} keys")
        nonzero = int((values != 0).sum())
        bits = m + 64 * len(lay["rank"]) + lay["count"] * b
        # every key with a non-zero value needs a non-zero field on its edge, and no two keys
        # share a hinge: between that many and n fields
        if not (min(nonzero, 1) <= lay["count"] <= n) or bits > b * n + m + 64 * (m // 1024 + 2):
            bad.append(f"sf ranked sigma={sigma}: {lay['count']} fields, {bits} bits")
    data, offs = workloads.str_keys(5000, gen_seed=seed)
    values = rng.integers(0, 1000, 5000).astype(np.uint32)
    rc, r = o.sf_build_str(data, offs, values, 1000, seed=4)
    if rc == 0:
        lay = o.sf_rank_layout(r["words"], r["m"], 1000)
        f = o.sfr_lookup_str(lay["marks"], lay["rank"], lay["vals"], 1000, r["P"], r["seed_used"], data, offs)
    if rc != 0 or not np.array_equal(f, values.astype(np.uint64)):
        bad.append(f"sf ranked str: status {rc} or lookup differs from the values")
    return bad


ALL_PINS = [pin_splitmix, pin_hash_closed_form, pin_part_size, pin_worked_examples,
            pin_bruteforce_tripartite, pin_bruteforce_generic, pin_invariants, pin_mphf, pin_errors,
            pin_string_digest, pin_static_function, pin_sf_ranked, pin_hem, pin_general_r]


def run_all(o, pins=None) -> list:
    bad = []
    for p in pins or ALL_PINS:
        try:
            bad += [f"{p.__name__}: {msg}" for msg in p(o)]
        except Exception as exc:  # a crash inside a check is a failed pin too
            bad.append(f"{p.__name__}: raised {type(exc).__name__}: {exc}")
    return bad
