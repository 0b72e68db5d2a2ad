"""HIP path against the oracle, element by element, through the C ABI (GPU only).

Sizes span several tiles and ragged tails; the configuration-1 workload (10^6 u64 keys,
gamma = 123/100) runs in full.  Integer work: the bar is bit-exact equality.
"""
import numpy as np
import pytest

import oracle
import pins
import workloads

pytestmark = pytest.mark.gpu

NONE = 0xFFFFFFFF


@pytest.fixture(scope="module")
def mx():
    import torch

    import paper_1312_0526_amd as mx

    assert torch.cuda.is_available()
    mx.lib()
    return mx


@pytest.fixture(scope="module")
def o():
    return oracle.Oracle()


@pytest.fixture(params=[(0, None), (96, 1)], ids=["auto-grid", "small-grid-one-round-batches"])
def record(request, mx):
    """Launch shapes: automatic grids with the default round batches, and a small fixed grid
    with a check after the first round."""
    old = mx.get_option("grid"), mx.get_option("round_batch")
    mx.set_option("grid", request.param[0])
    if request.param[1] is not None:
        mx.set_option("round_batch", request.param[1])
    yield request.param
    mx.set_option("grid", old[0])
    mx.set_option("round_batch", old[1])


def dev(a):
    import torch

    a = np.ascontiguousarray(a)
    view = {np.dtype(np.uint64): np.int64, np.dtype(np.uint32): np.int32}.get(a.dtype)
    if view is not None:
        a = a.view(view)
    return torch.from_numpy(a).to("cuda")


def host(t, dtype):
    return t.cpu().numpy().view(dtype)


# ------------------------------------------------------------------------------------------
# hashing and generators
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("n,seed,P", [(1, 0, 1), (1000, 0, 1 << 30), (1_000_000, 0, 410_000),
                                      (300_001, 0xDEADBEEF, 123_457), (4099, (1 << 64) - 1, 7)])
def test_hash_u64(mx, o, n, seed, P):
    keys = workloads.u64_keys(n, gen_seed=11)
    got = host(mx.hash_u64(dev(keys), seed, P), np.uint32).reshape(-1, 3)
    assert np.array_equal(got, o.hash_u64(keys, seed, P))


def test_hash_u64_known_answer(mx):
    P = 1 << 30
    got = host(mx.hash_u64(dev(np.zeros(1, np.uint64)), 0, P), np.uint32).reshape(-1).tolist()
    want = [pins.SPLITMIX0[0] >> 34, P + (pins.SPLITMIX0[1] >> 34), 2 * P + (pins.SPLITMIX0[2] >> 34)]
    assert got == want


def _str_cases():
    rng = np.random.default_rng(5)
    keys = [b"", b"a", b"ab", b"abc", b"abcd", b"abcdefg", b"abcdefgh", b"abcdefghi", bytes(range(256)),
            b"\x00" * 9, b"x" * 512]
    keys += [bytes(rng.integers(0, 256, size=int(l), dtype=np.uint8)) for l in rng.integers(0, 40, size=300)]
    # longer than 512 bytes (digested by their own thread), between short keys of the same block
    for pos, l in ((20, 513), (150, 1000), (400, 4099), (401, 520)):
        keys.insert(pos, bytes(rng.integers(0, 256, size=l, dtype=np.uint8)))
    data = np.frombuffer(b"".join(keys), np.uint8).copy()
    offs = np.zeros(len(keys) + 1, np.uint64)
    offs[1:] = np.cumsum([len(k) for k in keys])
    return data, offs


@pytest.mark.parametrize("seed", [0, 1, 0x123456789ABCDEF])
def test_hash_str_edge_cases(mx, o, seed):
    data, offs = _str_cases()  # every alignment of start and end, empty keys, 512-byte and longer keys
    P = 1000003
    got = host(mx.hash_str(dev(data), dev(offs), seed, P), np.uint32).reshape(-1, 3)
    assert np.array_equal(got, o.hash_str(data, offs, seed, P))


def test_hash_str_generated(mx, o):
    data, offs = workloads.str_keys(100_003, gen_seed=2)
    P = mx.part_size(100_003)
    got = host(mx.hash_str(dev(data), dev(offs), 9, P), np.uint32).reshape(-1, 3)
    assert np.array_equal(got, o.hash_str(data, offs, 9, P))


def test_device_generators_match_host(mx):
    import torch

    k = host(mx.gen_keys_u64(70_001, gen_seed=3, start=5), np.uint64)
    assert np.array_equal(k, workloads.u64_keys(70_001, gen_seed=3, start=5))
    q = dev(workloads.quantile_table().view(np.int16))
    for n, start in ((50_001, 0), (3, 123_456_789_012)):
        data, offs = mx.gen_str_keys(n, q, gen_seed=4, start=start)
        hd, ho = workloads.str_keys(n, gen_seed=4, start=start)
        assert np.array_equal(host(offs, np.uint64), ho)
        assert np.array_equal(data.cpu().numpy()[: int(ho[-1])], hd)
    torch.cuda.synchronize()


# ------------------------------------------------------------------------------------------
# peeling
# ------------------------------------------------------------------------------------------
def _peel_both(mx, o, edges, m):
    rc, ref = o.peel(edges, m, 0)
    assert rc == 0
    got = mx.peel(dev(edges.astype(np.uint32)), m)
    return got, ref


def _assert_peel_equal(got, ref):
    assert got["n_peeled"] == ref["n_peeled"]
    assert got["n_rounds"] == ref["n_rounds"]
    for key, dt in (("order", np.uint32), ("round", np.uint32), ("core_mask", np.uint8), ("hinge", np.uint8)):
        g = host(got[key], dt)
        assert np.array_equal(g, ref[key]), f"{key} differs"


def test_peel_worked_examples(mx, o, record):
    g = pins.golden()
    for name in ("E1", "E2"):
        ex = g[name]
        edges = np.array(ex["edges"], np.uint32)
        got = mx.peel(dev(edges), g["m"])
        assert host(got["round"], np.uint32).tolist() == ex["round"]
        assert host(got["order"], np.uint32).tolist() == ex["order"]
        assert host(got["core_mask"], np.uint8).tolist() == ex["core_mask"]
        h = host(got["hinge"], np.uint8).tolist()
        assert h == ex["hinge"]
        assert got["n_rounds"] == ex["n_rounds"]


@pytest.mark.parametrize("n,gamma", [(1, 1.23), (2, 1.0), (5000, 1.23), (65_537, 1.23), (65_537, 1.18),
                                     (200_000, 1.05), (1_000_000, 1.23), (1_000_000, 1.20)])
def test_peel_tripartite(mx, o, record, n, gamma):
    rng = np.random.default_rng(n)
    P = max(1, int(np.ceil(gamma * n / 3)))
    edges = pins.random_tripartite(n, P, rng)
    got, ref = _peel_both(mx, o, edges, 3 * P)
    _assert_peel_equal(got, ref)


@pytest.mark.parametrize("trial", range(6))
def test_peel_generic(mx, o, record, trial):
    rng = np.random.default_rng(100 + trial)
    n = int(rng.integers(1, 3000))
    m = int(rng.integers(3, max(4, n)))
    edges = pins.random_generic(n, m, rng)
    if trial % 2:
        edges = np.concatenate([edges, edges[: n // 10]])  # duplicates stay in the core
    got, ref = _peel_both(mx, o, edges, m)
    _assert_peel_equal(got, ref)


def test_peel_long_chain(mx, o):
    """Overlapping triples (i, i+1, i+2): only the two ends have a degree-1 vertex, so the
    chain peels one edge per round from each end, about n/2 rounds."""
    n = 3001
    edges = np.array([[i, i + 1, i + 2] for i in range(n)], np.uint32)
    got, ref = _peel_both(mx, o, edges, n + 2)
    assert ref["n_rounds"] > 1000
    _assert_peel_equal(got, ref)


def test_peel_empty(mx):
    got = mx.peel(dev(np.zeros((0, 3), np.uint32)), 10)
    assert got["n_peeled"] == 0 and got["n_rounds"] == 0


def test_peel_errors(mx):
    with pytest.raises(mx.MphxError) as ei:
        mx.peel(dev(np.array([[0, 1, 5]], np.uint32)), 5)
    assert ei.value.status == mx.EINVAL
    with pytest.raises(mx.MphxError) as ei:
        mx.peel(dev(np.array([[0, 1, 1]], np.uint32)), 5)
    assert ei.value.status == mx.EINVAL
    star = np.array([[0, 1 + i, 300 + i] for i in range(256)], np.uint32)
    with pytest.raises(mx.MphxError) as ei:
        mx.peel(dev(star), 600)
    assert ei.value.status == mx.ERANGE
    got = mx.peel(dev(star[:255]), 600)
    assert got["n_peeled"] == 255
    # a vertex in 2^24 + 1 edges wraps a 24-bit degree field: still caught (total != 3n)
    big = 1 << 24
    wrap = np.stack([np.zeros(big + 1, np.uint32), np.arange(1, big + 2, dtype=np.uint32),
                     np.arange(big + 2, 2 * big + 3, dtype=np.uint32)], axis=1)
    with pytest.raises(mx.MphxError) as ei:
        mx.peel(dev(wrap), 2 * big + 3)
    assert ei.value.status == mx.ERANGE


# ------------------------------------------------------------------------------------------
# whole MPHF build
# ------------------------------------------------------------------------------------------
def _assert_mphf_equal(got, ref):
    for key in ("P", "m", "seed_used", "tries", "n_rounds"):
        assert got[key] == ref[key], key
    assert np.array_equal(host(got["codes"], np.uint64), ref["words"])
    assert np.array_equal(host(got["rank"], np.uint64), ref["rank"])


def test_mphf_two_keys_one_vertex_per_part(mx, o):
    """n = 2 gives P = 1: both edges are (0, 1, 2) and can never peel (distinct keys: ECORE)."""
    keys = workloads.u64_keys(2)
    rc, ref = o.mphf_build_u64(keys, max_tries=5)
    assert rc == oracle.ECORE
    with pytest.raises(mx.MphxError) as ei:
        mx.mphf_build_u64(dev(keys), max_tries=5)
    assert ei.value.status == mx.ECORE and ei.value.info["n_core"] == ref["n_core"] == 2


@pytest.mark.parametrize("n,seed", [(1_000_000, 0), (12_345, 77), (1, 0), (7, 5)])
def test_mphf_u64(mx, o, record, n, seed):
    keys = workloads.u64_keys(n)
    got = mx.mphf_build_u64(dev(keys), seed=seed)
    rc, ref = o.mphf_build_u64(keys, seed=seed)
    assert rc == 0
    _assert_mphf_equal(got, ref)
    f = mx.lookup_u64(got["codes"], got["rank"], got["P"], got["seed_used"], dev(keys))
    assert np.array_equal(host(f, np.uint64), o.lookup_u64(ref["words"], ref["rank"], ref["P"], ref["seed_used"], keys))
    assert mx.check_bijection(f) == 0


def test_mphf_small_buckets_retry(mx, o):
    """n = 100 fails often at gamma 1.23: tries and seeds must follow the oracle."""
    retried = 0
    for b in range(30):
        keys = workloads.u64_keys(100, gen_seed=workloads.bucket_gen_seed(b))
        got = mx.mphf_build_u64(dev(keys), seed=0)
        rc, ref = o.mphf_build_u64(keys, seed=0)
        assert rc == 0
        _assert_mphf_equal(got, ref)
        retried += got["tries"] > 1
    assert retried > 5


def test_mphf_str(mx, o, record):
    data, offs = workloads.str_keys(200_000, gen_seed=1)
    got = mx.mphf_build_str(dev(data), dev(offs), seed=4)
    rc, ref = o.mphf_build_str(data, offs, seed=4)
    assert rc == 0
    _assert_mphf_equal(got, ref)
    f = mx.lookup_str(got["codes"], got["rank"], got["P"], got["seed_used"], dev(data), dev(offs))
    assert np.array_equal(host(f, np.uint64),
                          o.lookup_str(ref["words"], ref["rank"], ref["P"], ref["seed_used"], data, offs))


def test_lookup_in_batches_of_2_16(mx, o):
    """The lookup experiment's shape (Section 5, Table 2): keys evaluated in batches of 2^16,
    each batch one call on a slice of the offsets (absolute in the byte array) writing a slice
    of a preallocated output; the batches, with a ragged last one, equal the oracle's values."""
    import torch

    n = 3 * (1 << 16) + 4321
    data, offs = workloads.str_keys(n, gen_seed=9)
    got = mx.mphf_build_str(dev(data), dev(offs), seed=2)
    rc, ref = o.mphf_build_str(data, offs, seed=2)
    assert rc == 0
    d_data, d_offs = dev(data), dev(offs)
    out = torch.full((n,), -1, dtype=torch.int64, device="cuda")
    for b0 in range(0, n, 1 << 16):
        b1 = min(b0 + (1 << 16), n)
        mx.lookup_str(got["codes"], got["rank"], got["P"], got["seed_used"], d_data, d_offs[b0:b1 + 1], out=out[b0:b1])
    want = o.lookup_str(ref["words"], ref["rank"], ref["P"], ref["seed_used"], data, offs)
    assert np.array_equal(host(out, np.uint64), want)
    keys = workloads.u64_keys(n, gen_seed=10)
    got = mx.mphf_build_u64(dev(keys), seed=3)
    rc, ref = o.mphf_build_u64(keys, seed=3)
    assert rc == 0
    d_keys = dev(keys)
    out.fill_(-1)
    for b0 in range(0, n, 1 << 16):
        b1 = min(b0 + (1 << 16), n)
        mx.lookup_u64(got["codes"], got["rank"], got["P"], got["seed_used"], d_keys[b0:b1], out=out[b0:b1])
    assert np.array_equal(host(out, np.uint64), o.lookup_u64(ref["words"], ref["rank"], ref["P"], ref["seed_used"], keys))


def test_mphf_core_and_duplicates(mx, o):
    keys = workloads.u64_keys(50_000)
    with pytest.raises(mx.MphxError) as ei:
        mx.mphf_build_u64(dev(keys), gamma=(120, 100), max_tries=1)
    assert ei.value.status == mx.ECORE
    rc, ref = o.mphf_build_u64(keys, gnum=120, max_tries=1)
    assert rc == oracle.ECORE and ei.value.info["n_core"] == ref["n_core"]
    dup = np.concatenate([keys[:1000], keys[:2]])
    with pytest.raises(mx.MphxError) as ei:
        mx.mphf_build_u64(dev(dup), max_tries=2)
    assert ei.value.status == mx.EDUP
    assert o.mphf_build_u64(dup, max_tries=2)[0] == oracle.EDUP


def test_mphf_duplicates_inside_large_cores(mx, o):
    """Duplicate detection after the last try runs on the device (core edges, then pairs of
    them with equal vertex triples): a large core without duplicates stays ECORE; duplicates
    inside a large core, more duplicate pairs than the 1024 read back, and duplicate strings
    give EDUP, as in the oracle."""
    keys = workloads.u64_keys(200_000, gen_seed=21)
    with pytest.raises(mx.MphxError) as ei:
        mx.mphf_build_u64(dev(keys), gamma=(100, 100), max_tries=1)
    rc, ref = o.mphf_build_u64(keys, gnum=100, max_tries=1)
    assert ei.value.status == mx.ECORE and rc == oracle.ECORE
    assert ei.value.info["n_core"] == ref["n_core"] > 100_000
    for dup in (np.concatenate([keys, keys[7:9]]), np.concatenate([keys[:20_000], keys[:3000]])):
        gamma = (100, 100) if len(dup) > 100_000 else (123, 100)
        with pytest.raises(mx.MphxError) as ei:
            mx.mphf_build_u64(dev(dup), gamma=gamma, max_tries=1)
        assert ei.value.status == mx.EDUP
        assert o.mphf_build_u64(dup, gnum=gamma[0], max_tries=1)[0] == oracle.EDUP
    data, offs = workloads.str_keys(5000, gen_seed=22)
    lens = np.diff(offs)
    d2 = np.concatenate([data, data[offs[10]:offs[11]]])
    o2 = np.concatenate([offs, [offs[-1] + lens[10]]]).astype(np.uint64)
    with pytest.raises(mx.MphxError) as ei:
        mx.mphf_build_str(dev(d2), dev(o2), max_tries=2)
    assert ei.value.status == mx.EDUP
    assert o.mphf_build_str(d2, o2, max_tries=2)[0] == oracle.EDUP


def test_mphf_deterministic_across_launch_shapes(mx):
    keys = dev(workloads.u64_keys(300_000, gen_seed=9))
    outs = []
    old = mx.get_option("grid"), mx.get_option("round_batch")
    for grid, batch in ((0, 8), (64, 1), (1000, 64), (0, 3), (0, 200)):
        mx.set_option("grid", grid)
        mx.set_option("round_batch", batch)
        r = mx.mphf_build_u64(keys)
        outs.append((host(r["codes"], np.uint64), host(r["rank"], np.uint64)))
    mx.set_option("grid", old[0])
    mx.set_option("round_batch", old[1])
    for c, r in outs[1:]:
        assert np.array_equal(c, outs[0][0]) and np.array_equal(r, outs[0][1])


@pytest.fixture(params=[1, 0], ids=["partitioned-build", "atomic-build"])
def build_mode(request, mx):
    """The two record builds: radix-partitioned with LDS accumulation, and device atomics."""
    old = mx.get_option("part_build")
    mx.set_option("part_build", request.param)  # 1: partitioned at every size, 0: atomics
    yield request.param
    mx.set_option("part_build", old)


@pytest.mark.parametrize("n", [12_000_000, 333_333])
def test_mphf_record_builds_match_oracle(mx, o, build_mode, n):
    """12e6 keys give P = 4.92e6 vertices per part: two partition groups (2^22 vertices each)
    and 301 buckets of 2^14 vertices; 333,333 keys give one group and a ragged last bucket."""
    keys = workloads.u64_keys(n, gen_seed=21)
    got = mx.mphf_build_u64(dev(keys), seed=3)
    rc, ref = o.mphf_build_u64(keys, seed=3)
    assert rc == 0
    _assert_mphf_equal(got, ref)


def test_mphf_record_builds_agree_on_strings(mx):
    data, offs = workloads.str_keys(700_000, gen_seed=2)
    outs = []
    old = mx.get_option("part_build")
    for mode in (1, 0):
        mx.set_option("part_build", mode)
        r = mx.mphf_build_str(dev(data), dev(offs), seed=1)
        outs.append((host(r["codes"], np.uint64), host(r["rank"], np.uint64), r["n_rounds"]))
    mx.set_option("part_build", old)
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    assert outs[0][2] == outs[1][2]


@pytest.mark.parametrize("copies", [300, (1 << 24) + 1])
def test_mphf_degree_overflow(mx, o, build_mode, copies):
    """Equal keys give equal edges: their three vertices reach degree `copies`.  300 exceeds
    the 255 limit directly; 2^24 + 1 wraps the 24-bit degree field to 1 (and the label sum
    carries into it), which the total-degree check still catches."""
    keys = np.full(copies, 0x1234_5678_9ABC_DEF0, dtype=np.uint64)
    with pytest.raises(mx.MphxError) as ei:
        mx.mphf_build_u64(dev(keys), max_tries=2)
    assert ei.value.status == mx.ERANGE
    if copies < 1000:
        assert o.mphf_build_u64(keys, max_tries=2)[0] == oracle.ERANGE


@pytest.fixture(params=[(1, 0), (1, 1), (1, 16), (0, 0)],
                ids=["claim-lists", "update-lists-most-rounds", "update-lists-dense-rounds", "atomic-claims"])
def claim_mode(request, mx):
    """Next-layer claims: partitioned lists resolved in LDS (forced on at every size), with the
    deletes of rounds whose claim count c has 200 c >= p m going through sorted update lists
    (p = 1: nearly every round, p = 16: the dense ones, which the default picks), or one
    device atomic per claim."""
    lists, upd = request.param
    old = mx.get_option("claim_lists"), mx.get_option("update_lists")
    mx.set_option("claim_lists", lists)
    mx.set_option("update_lists", upd)
    yield request.param
    mx.set_option("claim_lists", old[0])
    mx.set_option("update_lists", old[1])


@pytest.mark.parametrize("n,seed", [(1_000_000, 0), (12_000_000, 4), (1, 0), (7, 5)])
def test_mphf_claim_modes_match_oracle(mx, o, claim_mode, n, seed):
    """12e6 keys span one claim group of 2^24 edges and 184 buckets of 2^16, and 2^14-vertex
    update buckets in three first-pass groups."""
    keys = workloads.u64_keys(n, gen_seed=41)
    got = mx.mphf_build_u64(dev(keys), seed=seed)
    rc, ref = o.mphf_build_u64(keys, seed=seed)
    assert rc == 0
    _assert_mphf_equal(got, ref)


@pytest.mark.parametrize("upd", [0, 1], ids=["claims", "update-lists"])
def test_mphf_claim_lists_strings_retries_and_failures(mx, o, upd):
    old = mx.get_option("claim_lists"), mx.get_option("update_lists")
    mx.set_option("claim_lists", 1)
    mx.set_option("update_lists", upd)
    try:
        data, offs = workloads.str_keys(300_000, gen_seed=43)
        got = mx.mphf_build_str(dev(data), dev(offs), seed=6)
        rc, ref = o.mphf_build_str(data, offs, seed=6)
        assert rc == 0
        _assert_mphf_equal(got, ref)
        retried = 0
        for b in range(20):
            keys = workloads.u64_keys(100, gen_seed=workloads.bucket_gen_seed(b))
            got = mx.mphf_build_u64(dev(keys), seed=0)
            rc, ref = o.mphf_build_u64(keys, seed=0)
            assert rc == 0
            _assert_mphf_equal(got, ref)
            retried += got["tries"] > 1
        assert retried > 3
        keys = workloads.u64_keys(50_000)
        with pytest.raises(mx.MphxError) as ei:
            mx.mphf_build_u64(dev(keys), gamma=(120, 100), max_tries=1)
        rc, ref = o.mphf_build_u64(keys, gnum=120, max_tries=1)
        assert ei.value.status == mx.ECORE and rc == oracle.ECORE
        assert ei.value.info["n_core"] == ref["n_core"] and ei.value.info["n_rounds"] == ref["n_rounds"]
        dup = np.concatenate([keys[:1000], keys[:2]])
        with pytest.raises(mx.MphxError) as ei:
            mx.mphf_build_u64(dev(dup), max_tries=2)
        assert ei.value.status == mx.EDUP
    finally:
        mx.set_option("claim_lists", old[0])
        mx.set_option("update_lists", old[1])


@pytest.mark.parametrize("upd,cap", [(16, 1000), (0, 5000), (16, 0)],
                         ids=["round0-deletes-overflow", "round1-claims-overflow", "no-overflow"])
def test_claim_list_overflow_redoes_the_try_with_atomic_claims(mx, o, upd, cap):
    """A claim-list round whose records exceed the list (forced here with a small list_cap)
    makes the try start again with atomic claims; the MPHF and a static function built that
    way equal the oracle's, and the fallback counter shows the redo happened."""
    old = mx.get_option("claim_lists"), mx.get_option("update_lists")
    mx.set_option("claim_lists", 10)
    mx.set_option("update_lists", upd)
    mx.set_option("list_cap", cap)
    mx.set_option("list_fallbacks", 0)
    try:
        keys = workloads.u64_keys(100_000, gen_seed=47)
        got = mx.mphf_build_u64(dev(keys), seed=3)
        rc, ref = o.mphf_build_u64(keys, seed=3)
        assert rc == 0
        _assert_mphf_equal(got, ref)
        vals = (workloads.u64_keys(100_000, gen_seed=48) % 1000).astype(np.uint32)
        sf = mx.sf_build_u64(dev(keys), dev(vals), 1000, seed=3)
        rc, sref = o.sf_build_u64(keys, vals, 1000, seed=3)
        assert rc == 0 and sf["seed_used"] == sref["seed_used"]
        assert np.array_equal(host(sf["words"], np.uint64), sref["words"])
        assert mx.get_option("list_fallbacks") == (2 if cap else 0)
    finally:
        mx.set_option("claim_lists", old[0])
        mx.set_option("update_lists", old[1])
        mx.set_option("list_cap", 0)
        mx.set_option("list_fallbacks", 0)
