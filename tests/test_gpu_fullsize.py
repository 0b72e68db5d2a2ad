"""Parity at the full workload sizes (GPU only; minutes of CPU for the oracle).

The oracle's results at the sizes it cannot build inside a test run are stored as digests in
tests/golden/ by tests/golden/make_fullsize.py (which runs only the oracle): config 3's 2^31-key
MPHF, each of config 4's 65,536 buckets and each of config 5's 60 requests.

* 2^27 u64 keys: the whole MPHF (codes + rank) equals the oracle's, with atomic claims and
  with claim and update lists; at gamma = 120/100 (below
  the threshold c_3 ~ 1.221, Section 1) the peel returns exactly the oracle's 2-core, rounds,
  hinges and order, and a one-try build reports the same 2-core size.
* 2^31 byte-string keys generated on the device (the configuration the benchmark times): the
  codes and rank equal the oracle's bit for bit (SHA-256 of both against the golden digest;
  P, seed, tries and rounds equal); besides, the device keys equal the generator's definition
  at sampled indices, the device hash equals the oracle's hash for those keys, the MPHF is a
  bijection onto [0, n) over all keys, the rank samples equal the prefix counts of the codes,
  and the oracle's evaluation of the GPU tables agrees with the GPU lookup at sampled keys.
* 65,536 u64 buckets of 100 to 10^6 keys in one captured batched launch: every bucket equals
  the oracle's single build (tries, rounds and a digest of its codes and rank), and the two
  largest are compared word for word with a fresh oracle build.
* The served workload at full size (requests of 10^3 to 10^8 keys): every result equals the
  oracle's (tries, seed, rounds, digest of codes and rank) and the request built alone, and the
  largest ones are bijections.
"""
import hashlib
import os
import sys

import numpy as np
import pytest

import oracle
import workloads

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_fullsize as golden  # noqa: E402

pytestmark = pytest.mark.gpu


def _digest(codes_h, rank_h):
    return golden.digest(codes_h, rank_h)


@pytest.fixture(scope="module")
def mx():
    import torch

    import paper_1312_0526_amd as mx

    assert torch.cuda.is_available()
    mx.lib()
    return mx


def host(t, dt):
    return t.cpu().numpy().view(dt)


@pytest.mark.timeout(1200)
def test_config2_full_parity(mx):
    import torch

    n = 1 << 27
    o = oracle.Oracle()
    keys_h = workloads.u64_keys(n)
    keys = mx.gen_keys_u64(n)
    assert np.array_equal(host(keys[:1000], np.uint64), keys_h[:1000])
    assert np.array_equal(host(keys[-1000:], np.uint64), keys_h[-1000:])
    r = mx.mphf_build_u64(keys, seed=0)
    assert r["update_deletes"] > 0  # the default here: claim lists, dense rounds by update lists
    rc, ref = o.mphf_build_u64(keys_h, seed=0)
    assert rc == 0 and r["tries"] == ref["tries"] == 1 and r["n_rounds"] == ref["n_rounds"]
    assert np.array_equal(host(r["codes"], np.uint64), ref["words"])
    assert np.array_equal(host(r["rank"], np.uint64), ref["rank"])
    del r
    # below the threshold: the exact 2-core through the peel entry point
    P = o.part_size(n, 120, 100)
    edges = o.hash_u64(keys_h, 0, P)
    rc, pref = o.peel(edges, 3 * P, P)
    assert rc == 0 and abs((n - pref["n_peeled"]) / n - 0.4921) < 0.003
    got = mx.peel(torch.from_numpy(edges.view(np.int32)).cuda(), 3 * P)
    assert got["n_peeled"] == pref["n_peeled"] and got["n_rounds"] == pref["n_rounds"]
    for key, dt in (("order", np.uint32), ("round", np.uint32), ("core_mask", np.uint8), ("hinge", np.uint8)):
        assert np.array_equal(host(got[key], dt), pref[key]), key
    del got
    with pytest.raises(mx.MphxError) as ei:
        mx.mphf_build_u64(keys, gamma=(120, 100), max_tries=1)
    assert ei.value.status == mx.ECORE and ei.value.info["n_core"] == n - pref["n_peeled"]


@pytest.mark.timeout(1200)
def test_config2_full_parity_atomic_claims(mx):
    """2^27 keys through the path smaller builds take by default (2^27 keys take claim lists
    from round 1 and sorted update lists for the dense rounds): one device atomic per claim."""
    n = 1 << 27
    o = oracle.Oracle()
    keys_h = workloads.u64_keys(n)
    keys = mx.gen_keys_u64(n)
    old = mx.get_option("claim_lists")
    mx.set_option("claim_lists", 0)
    try:
        r = mx.mphf_build_u64(keys, seed=0)
    finally:
        mx.set_option("claim_lists", old)
    assert r["update_deletes"] == 0
    rc, ref = o.mphf_build_u64(keys_h, seed=0)
    assert rc == 0 and r["tries"] == ref["tries"] == 1 and r["n_rounds"] == ref["n_rounds"]
    assert np.array_equal(host(r["codes"], np.uint64), ref["words"])
    assert np.array_equal(host(r["rank"], np.uint64), ref["rank"])


_POP8 = np.array([bin(i).count("1") for i in range(256)], np.uint8)


def _nz_pairs(words):
    """Non-zero 2-bit pairs per word, counted bit by bit through a byte table."""
    x = (words | (words >> np.uint64(1))) & np.uint64(0x5555555555555555)
    return _POP8[x.view(np.uint8)].reshape(-1, 8).sum(axis=1, dtype=np.int64)


@pytest.mark.timeout(1200)
def test_config3_full_parity(mx):
    import torch

    n = 1 << 31
    o = oracle.Oracle()
    q = torch.from_numpy(workloads.quantile_table().view(np.int16)).cuda()
    data, offs = mx.gen_str_keys(n, q, gen_seed=0)
    rng = np.random.default_rng(7)
    sample = np.unique(np.concatenate([[0, 1, n - 1], rng.integers(0, n, size=2000)])).astype(np.int64)
    offs_h = host(offs, np.uint64)
    # device keys equal the generator's definition at sampled indices
    for i in sample[:300]:
        lo, hi = int(offs_h[i]), int(offs_h[i + 1])
        assert bytes(data[lo:hi].cpu().numpy()) == workloads.str_key(int(i)), i
    r = mx.mphf_build_str(data, offs, seed=0)
    assert r["tries"] == 1 and r["n_core"] == 0
    P, seed = r["P"], r["seed_used"]
    # device hash of the sampled keys equals the oracle's
    skeys = [workloads.str_key(int(i)) for i in sample]
    sd = np.frombuffer(b"".join(skeys), np.uint8).copy()
    so = np.zeros(len(skeys) + 1, np.uint64)
    so[1:] = np.cumsum([len(k) for k in skeys])
    ge = host(mx.hash_str(torch.from_numpy(sd).cuda(), torch.from_numpy(so.view(np.int64)).cuda(), seed, P),
              np.uint32).reshape(-1, 3)
    assert np.array_equal(ge, o.hash_str(sd, so, seed, P))
    # bijection over all 2^31 keys
    f = mx.lookup_str(r["codes"], r["rank"], P, seed, data, offs)
    assert mx.check_bijection(f) == 0
    f_s = host(f[torch.from_numpy(sample).cuda()], np.uint64)
    del f
    codes = host(r["codes"], np.uint64)
    rank = host(r["rank"], np.uint64)
    # the oracle's evaluation of the GPU tables at the sampled keys
    assert np.array_equal(o.lookup_str(codes, rank, P, seed, sd, so), f_s)
    # rank samples are the prefix counts of non-zero codes; exactly n hinge vertices
    nz = _nz_pairs(codes)
    per_block = np.add.reduceat(nz, np.arange(0, len(nz), 16))
    prefix = np.concatenate([[0], np.cumsum(per_block)[:-1]])
    assert np.array_equal(rank.astype(np.int64), prefix)
    assert int(nz.sum()) == n
    # bit for bit the oracle's MPHF of all 2^31 keys
    g = golden.read_c3()
    assert (g["n"], g["P"], g["seed_used"], g["tries"], g["n_rounds"]) == (n, P, seed, r["tries"], r["n_rounds"])
    assert (g["code_words"], g["rank_words"]) == (len(codes), len(rank))
    assert hashlib.sha256(codes.tobytes()).hexdigest() == g["codes_sha256"]
    assert hashlib.sha256(rank.tobytes()).hexdigest() == g["rank_sha256"]


@pytest.mark.timeout(600)
def test_config4_full_batch_parity(mx):
    # 65,536 buckets of 100 to 10^6 u64 keys (log-uniform, 7.09e9 keys) in one captured
    # persistent launch at 1024 threads x one workgroup per compute unit, as the benchmark runs
    # it: every bucket equals the oracle's build of it (tries, rounds, digest of codes and rank,
    # from the golden file), and the two largest equal a fresh oracle build word for word
    import torch

    torch.cuda.empty_cache()
    o = oracle.Oracle()
    sizes = workloads.bucket_sizes(65536, 100, 1_000_000, seed=0)
    off = np.zeros(len(sizes) + 1, np.uint64)
    off[1:] = np.cumsum(sizes)
    keys = mx.gen_buckets_u64(torch.from_numpy(off.view(np.int64)).cuda())
    bb = mx.BatchBuild(off, block=1024, grid=0)
    bb.capture(keys)
    bb.launch()
    bb.launch()  # a replay rebuilds the same tables
    torch.cuda.synchronize()
    res = bb.bucket_results()
    assert (res["status"] == 0).all() and (res["tries"] >= 1).all()
    assert int(bb.code_off_h[-1]) == bb.codes.numel() and int(bb.rank_off_h[-1]) == bb.rank.numel()
    gold = golden.read_c4()
    assert len(gold) == len(sizes)
    codes_h = host(bb.codes, np.uint64)
    rank_h = host(bb.rank, np.uint64)
    co, ro = bb.code_off_h.astype(np.int64), bb.rank_off_h.astype(np.int64)
    bad = []
    for b in range(len(sizes)):
        tries, rounds, d = gold[b]
        got = _digest(codes_h[co[b]:co[b + 1]], rank_h[ro[b]:ro[b + 1]])[:12]
        if (int(res[b]["tries"]), int(res[b]["n_rounds"]), got) != (tries, rounds, d):
            bad.append(b)
    assert not bad, f"{len(bad)} buckets differ from the oracle, first {bad[:10]}"
    del codes_h, rank_h
    which = np.argsort(-sizes, kind="stable")[:2].tolist()
    for b in which:
        kb = host(keys[int(off[b]):int(off[b + 1])], np.uint64)
        assert np.array_equal(kb, workloads.u64_keys(int(sizes[b]), gen_seed=workloads.bucket_gen_seed(b))), b
        rc, ref = o.mphf_build_u64(kb, seed=0, max_tries=bb.max_tries)
        assert rc == 0 and res[b]["tries"] == ref["tries"] and res[b]["seed_used"] == ref["seed_used"], b
        assert res[b]["n_rounds"] == ref["n_rounds"], b
        assert np.array_equal(host(bb.bucket_codes(b), np.uint64), ref["words"]), b
        assert np.array_equal(host(bb.bucket_rank(b), np.uint64), ref["rank"]), b
    bb.destroy_graph()


@pytest.mark.timeout(600)
def test_config5_served_full_sizes(mx):
    # 60 requests of the served workload (sizes log-uniform 1e3..1e8, u64 or string keys, each
    # a prefix of one device-generated key set per kind, as the benchmark builds them), all
    # submitted at once to a server with the benchmark's budget and slots: every result equals
    # the same request built alone, the largest of each kind is a bijection, and the small
    # requests equal the oracle's builds
    import torch

    # the server allocates its pool itself: give back what earlier tests left in torch's cache
    torch.cuda.empty_cache()
    max_n = 100_000_000
    keys = mx.gen_keys_u64(max_n, gen_seed=7)
    q = torch.from_numpy(workloads.quantile_table().view(np.int16)).cuda()
    data, offs = mx.gen_str_keys(max_n, q, gen_seed=8)
    nreq = 60
    sizes = workloads.request_sizes(nreq, 1000, max_n, seed=1)
    kinds = (workloads.stream(np.uint64(2), np.arange(1, nreq + 1, dtype=np.uint64)) & np.uint64(1)).astype(int)
    assert sizes.max() > 3 * 10**7 and set(kinds) == {0, 1}

    def req(i):
        n = int(sizes[i])
        return (keys[:n],) if kinds[i] == 0 else (data, offs[: n + 1])

    srv = mx.Server(hbm_budget=64 << 30, slots=4)
    tickets = [srv.submit_u64(*req(i), seed=i) if kinds[i] == 0 else srv.submit_str(*req(i), seed=i)
               for i in range(nreq)]
    res = [srv.wait(t) for t in tickets]
    torch.cuda.synchronize()
    gold = golden.read_c5()
    for i, r in enumerate(res):
        assert r["status"] == 0, i
        g = gold[i]
        assert (g["kind"], g["n"]) == (int(kinds[i]), int(sizes[i])), i
        assert (r["seed_used"], r["tries"], r["n_rounds"]) == (g["seed_used"], g["tries"], g["n_rounds"]), i
        assert _digest(host(r["codes"], np.uint64), host(r["rank"], np.uint64)) == g["digest"], i
        a = mx.mphf_build_u64(*req(i), seed=i) if kinds[i] == 0 else mx.mphf_build_str(*req(i), seed=i)
        assert (r["tries"], r["seed_used"], r["P"]) == (a["tries"], a["seed_used"], a["P"]), i
        assert torch.equal(r["codes"], a["codes"]) and torch.equal(r["rank"], a["rank"]), i
    for kind in (0, 1):
        i = int(np.argmax(np.where(kinds == kind, sizes, 0)))
        r = res[i]
        if kind == 0:
            f = mx.lookup_u64(r["codes"], r["rank"], r["P"], r["seed_used"], keys[: int(sizes[i])])
        else:
            f = mx.lookup_str(r["codes"], r["rank"], r["P"], r["seed_used"], data, offs[: int(sizes[i]) + 1])
        assert mx.check_bijection(f) == 0, i
    # the device key sets are the generator's (the golden digests were built from it)
    assert np.array_equal(host(keys[-1000:], np.uint64), workloads.u64_keys(max_n, gen_seed=7)[-1000:])
    oh = host(offs[:1001], np.uint64)
    d_h, o_h = workloads.str_keys(1000, gen_seed=8)
    assert np.array_equal(oh, o_h) and np.array_equal(data[: int(oh[-1])].cpu().numpy(), d_h[: int(oh[-1])])
    srv.close()


@pytest.mark.timeout(1200)
def test_stream_beyond_2e32_vertices(mx):
    """The streamed build past the in-HBM build's limit: 3.6e9 u64 keys in host memory, so
    m = 3P = 4.43e9 vertex positions pass 2^32 (the oracle's 32-bit vertex ids cannot express
    this; checked by what holds at any size).  The MPHF is a bijection onto [0, n) over all
    keys, its rank samples are the prefix counts of its codes, and the build with every layer
    spilled to host memory gives the same codes and rank as the build with the layers in HBM."""
    import torch

    torch.cuda.empty_cache()
    n = 3_600_000_000
    P = mx.part_size(n)
    assert 3 * P > (1 << 32)
    hk = torch.empty(n, dtype=torch.int64)
    chunk = 1 << 27
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        hk[c0:c1].copy_(mx.gen_keys_u64(c1 - c0, gen_seed=36, start=c0))
    assert np.array_equal(hk[-1000:].numpy().view(np.uint64), workloads.u64_keys(1000, gen_seed=36, start=n - 1000))
    a = mx.mphf_build_stream_u64(hk, seed=0, chunk_keys=chunk)
    assert a["n_core"] == 0 and a["P"] == P
    assert mx.check_stream_u64(a["codes"], a["rank"], a["P"], a["seed_used"], hk, chunk_keys=chunk) == 0
    codes = host(a["codes"], np.uint64)
    rank = host(a["rank"], np.uint64)
    nz = _nz_pairs(codes)
    per_block = np.add.reduceat(nz, np.arange(0, len(nz), 16))
    assert np.array_equal(rank.astype(np.int64), np.concatenate([[0], np.cumsum(per_block)[:-1]]))
    assert int(nz.sum()) == n
    del a, nz, per_block
    torch.cuda.empty_cache()
    b = mx.mphf_build_stream_u64(hk, seed=0, chunk_keys=chunk, layer_slots=(3 * n) // 10)
    assert (b["tries"], b["n_rounds"]) == (1, b["n_rounds"])
    assert np.array_equal(host(b["codes"], np.uint64), codes) and np.array_equal(host(b["rank"], np.uint64), rank)
