"""Parity at the full workload sizes (GPU only; minutes of CPU for the oracle).

* 2^27 u64 keys: the whole MPHF (codes + rank) equals the oracle's, with atomic claims and
  with claim and update lists; at gamma = 120/100 (below
  the threshold c_3 ~ 1.221, Section 1) the peel returns exactly the oracle's 2-core, rounds,
  hinges and order, and a one-try build reports the same 2-core size.
* 2^31 byte-string keys generated on the device (the configuration the benchmark times): the
  oracle cannot build it, so the test checks what holds at any size -- the device keys equal
  the generator's definition at sampled indices, the device hash equals the oracle's hash for
  those keys, the MPHF is a bijection onto [0, n) over all keys, the rank samples equal the
  prefix counts of the codes, and the oracle's evaluation of the GPU tables agrees with the
  GPU lookup at sampled keys.
* 65,536 u64 buckets of 100 to 10^6 keys in one captured batched launch: every bucket builds,
  and the largest buckets and a random sample equal the oracle's single builds.
* The served workload at full size (requests of 10^3 to 10^8 keys): every result equals the
  request built alone, the largest ones are bijections, small ones equal the oracle.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


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
def test_config2_full_parity_claim_and_update_lists(mx):
    """2^27 keys through the path the largest builds take by default: claim lists from round 1,
    the dense rounds' deletes through sorted update lists."""
    n = 1 << 27
    o = oracle.Oracle()
    keys_h = workloads.u64_keys(n)
    keys = mx.gen_keys_u64(n)
    mx.set_option("claim_lists", 27)
    try:
        assert mx.get_option("update_lists") == 16
        r = mx.mphf_build_u64(keys, seed=0)
    finally:
        mx.set_option("claim_lists", 28)
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
def test_config3_sampled_parity(mx):
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


@pytest.mark.timeout(600)
def test_config4_full_batch_sampled_parity(mx):
    # 65,536 buckets of 100 to 10^6 u64 keys (log-uniform, 7.09e9 keys) in one captured
    # persistent launch at 1024 threads x one workgroup per compute unit, as the benchmark runs
    # it: every bucket builds, the sum of the per-bucket code and rank lengths is the layout's,
    # and the largest buckets and a random sample equal the oracle's single builds
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
    rng = np.random.default_rng(11)
    which = np.argsort(-sizes, kind="stable")[:2].tolist() + rng.choice(len(sizes), 24, replace=False).tolist()
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
    for i, r in enumerate(res):
        assert r["status"] == 0, i
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
    o = oracle.Oracle()
    small = [i for i in range(nreq) if sizes[i] <= 200_000][:8]
    assert len(small) >= 4
    for i in small:
        n = int(sizes[i])
        if kinds[i] == 0:
            rc, ref = o.mphf_build_u64(host(keys[:n], np.uint64), seed=i)
        else:
            oh = host(offs[: n + 1], np.uint64)
            rc, ref = o.mphf_build_str(data[: int(oh[-1])].cpu().numpy(), oh, seed=i)
        assert rc == 0 and np.array_equal(host(res[i]["codes"], np.uint64), ref["words"]), i
        assert np.array_equal(host(res[i]["rank"], np.uint64), ref["rank"]), i
    srv.close()
