"""Batched builds (one persistent launch for many buckets) against the oracle, bucket by
bucket, through the C ABI (GPU only).  Each bucket must equal the oracle's single build of
the same keys with the same seed, including the retry count and the seed used."""
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


@pytest.fixture(scope="module")
def o():
    return oracle.Oracle()


def _offsets(sizes):
    off = np.zeros(len(sizes) + 1, np.uint64)
    off[1:] = np.cumsum(sizes)
    return off


def _host_keys(sizes):
    return np.concatenate([workloads.u64_keys(int(s), gen_seed=workloads.bucket_gen_seed(b))
                           for b, s in enumerate(sizes)]) if len(sizes) else np.zeros(0, np.uint64)


def _check_buckets(mx, o, bb, keys_h, sizes, which=None):
    res = bb.bucket_results()
    off = _offsets(sizes)
    which = range(len(sizes)) if which is None else which
    for b in which:
        kb = keys_h[int(off[b]):int(off[b + 1])]
        rc, ref = o.mphf_build_u64(kb, seed=bb.seed, max_tries=bb.max_tries)
        assert res[b]["status"] == rc, (b, sizes[b])
        assert res[b]["tries"] == ref["tries"] and res[b]["seed_used"] == ref["seed_used"], b
        if rc == 0:
            assert res[b]["n_rounds"] == ref["n_rounds"], b
            assert np.array_equal(bb.bucket_codes(b).cpu().numpy().view(np.uint64), ref["words"]), b
            assert np.array_equal(bb.bucket_rank(b).cpu().numpy().view(np.uint64), ref["rank"]), b


SIZES = np.concatenate([[1, 3, 7, 100, 101, 4096], workloads.bucket_sizes(250, 100, 30_000, seed=5)])


@pytest.mark.parametrize("block,grid,scope", [(256, 0, 0), (512, 7, 0), (1024, 3, 1), (256, 1, 0), (1024, 0, 1)])
def test_batch_matches_oracle(mx, o, block, grid, scope):
    import torch

    off = _offsets(SIZES)
    keys = mx.gen_buckets_u64(torch.from_numpy(off.view(np.int64)).cuda())
    keys_h = _host_keys(SIZES)
    assert np.array_equal(keys.cpu().numpy().view(np.uint64)[: len(keys_h)], keys_h)
    bb = mx.BatchBuild(off, block=block, grid=grid, scope=scope)
    bb.run(keys)
    torch.cuda.synchronize()
    _check_buckets(mx, o, bb, keys_h, SIZES)
    res = bb.bucket_results()
    assert (res["tries"] > 1).sum() > 20  # small buckets retry often at gamma 1.23


_BATCH_OPTS = ("batch_lds", "batch_sort_deletes", "batch_claim_lists")


@pytest.mark.parametrize("lds,sort_div,cl", [(0, 0, 0), (0, 0, 1), (0, 8, 0), (0, 8, 1), (1, 8, 1)])
def test_batch_lds_path_on_and_off(mx, o, lds, sort_div, cl):
    # buckets up to about 18,000 keys run in LDS with 1024-thread workgroups, larger ones (and
    # every bucket with the option off) through device memory, whose dense layers delete
    # through sorted lists unless that is off too, and whose other layers claim through lists
    # resolved in LDS unless that is off: the same codes every way
    import torch

    old = [mx.get_option(k) for k in _BATCH_OPTS]
    for k, v in zip(_BATCH_OPTS, (lds, sort_div, cl)):
        mx.set_option(k, v)
    try:
        off = _offsets(SIZES)
        keys = mx.gen_buckets_u64(torch.from_numpy(off.view(np.int64)).cuda())
        bb = mx.BatchBuild(off, block=1024, grid=0, scope=0)
        bb.run(keys)
        torch.cuda.synchronize()
        _check_buckets(mx, o, bb, _host_keys(SIZES), SIZES)
    finally:
        for k, v in zip(_BATCH_OPTS, old):
            mx.set_option(k, v)


@pytest.mark.parametrize("block", [256, 1024])
def test_batch_claim_lists_over_several_edge_tiles(mx, o, block):
    """Buckets of 40,000 to 300,000 keys through device memory: their claim lists span several
    tiles of edges (32,768 per tile at 256 threads, 65,536 at 1024), each resolved in LDS."""
    import torch

    sizes = np.array([40_000, 70_001, 131_072, 299_999, 65_536, 100_003], np.uint64)
    old = [mx.get_option(k) for k in _BATCH_OPTS]
    for k, v in zip(_BATCH_OPTS, (0, 8, 1)):
        mx.set_option(k, v)
    try:
        off = _offsets(sizes)
        keys = mx.gen_buckets_u64(torch.from_numpy(off.view(np.int64)).cuda())
        bb = mx.BatchBuild(off, block=block, grid=0, scope=0)
        bb.run(keys)
        torch.cuda.synchronize()
        _check_buckets(mx, o, bb, _host_keys(sizes), sizes)
    finally:
        for k, v in zip(_BATCH_OPTS, old):
            mx.set_option(k, v)


@pytest.mark.parametrize("block", [512, 1024])
def test_batch_record_build_packed_boundary(mx, o, block):
    """Buckets on both sides of the one-pass record partition's limit: up to 2^20 keys given by
    key words pack each (vertex in tile, key) pair in one word; above it the parts are
    partitioned one by one with 8-byte pairs.  Both against the oracle."""
    import torch

    sizes = np.array([(1 << 20) - 1, 1 << 20, (1 << 20) + 1, 1_500_000], np.uint64)
    off = _offsets(sizes)
    keys = mx.gen_buckets_u64(torch.from_numpy(off.view(np.int64)).cuda())
    bb = mx.BatchBuild(off, block=block, grid=0, scope=0)
    bb.run(keys)
    torch.cuda.synchronize()
    _check_buckets(mx, o, bb, keys.cpu().numpy().view(np.uint64), sizes)


@pytest.mark.parametrize("cl", [1, 0])
def test_batch_sorted_deletes_on_nearly_every_layer(mx, o, cl):
    """batch_sort_deletes = 1024 sends every layer of at least m/2048 edges through the sorted
    deletes (their skips of degree-1 vertices, the marks and the state scan), between claim-list
    rounds (cl = 1) or atomicMin rounds (cl = 0); every bucket against the oracle."""
    import torch

    sizes = np.array([5_000, 20_000, 40_000, 131_072, 299_999], np.uint64)
    old = [mx.get_option(k) for k in _BATCH_OPTS]
    for k, v in zip(_BATCH_OPTS, (0, 1024, cl)):
        mx.set_option(k, v)
    try:
        off = _offsets(sizes)
        keys = mx.gen_buckets_u64(torch.from_numpy(off.view(np.int64)).cuda())
        for block in (512, 1024):
            bb = mx.BatchBuild(off, block=block, grid=0, scope=0)
            bb.run(keys)
            torch.cuda.synchronize()
            _check_buckets(mx, o, bb, _host_keys(sizes), sizes)
    finally:
        for k, v in zip(_BATCH_OPTS, old):
            mx.set_option(k, v)


def test_batch_large_buckets_sampled(mx, o):
    import torch

    sizes = workloads.bucket_sizes(64, 100, 1_000_000, seed=0)
    off = _offsets(sizes)
    keys = mx.gen_buckets_u64(torch.from_numpy(off.view(np.int64)).cuda())
    bb = mx.BatchBuild(off)
    bb.run(keys)
    torch.cuda.synchronize()
    res = bb.bucket_results()
    assert (res["status"] == 0).all()
    keys_h = keys.cpu().numpy().view(np.uint64)
    big = np.argsort(-sizes)[:2].tolist()
    _check_buckets(mx, o, bb, keys_h, sizes, which=big + [5, 17, 40])


def test_batch_graph_replays(mx, o):
    """Capture once, replay several times with eager work and synchronisations between the
    replays; every replay must reproduce the eager result."""
    import torch

    sizes = SIZES[:80]
    off = _offsets(sizes)
    keys = mx.gen_buckets_u64(torch.from_numpy(off.view(np.int64)).cuda())
    bb = mx.BatchBuild(off)
    bb.run(keys)
    torch.cuda.synchronize()
    ref_codes, ref_rank, ref_res = bb.codes.clone(), bb.rank.clone(), bb.results.clone()
    bb.capture(keys)
    for rep in range(4):
        bb.codes.zero_()
        bb.rank.zero_()
        bb.results.zero_()
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
        bb.launch()
        torch.cuda.synchronize()
        assert torch.equal(bb.codes, ref_codes), rep
        assert torch.equal(bb.rank, ref_rank), rep
        assert torch.equal(bb.results, ref_res), rep
    bb.destroy_graph()
    _check_buckets(mx, o, bb, _host_keys(sizes), sizes, which=range(0, 80, 7))


def test_batch_rejects_oversize_bucket(mx):
    import torch

    sizes = np.array([50, 500, 60], np.int64)
    off = _offsets(sizes)
    keys = mx.gen_buckets_u64(torch.from_numpy(off.view(np.int64)).cuda())
    bb = mx.BatchBuild(off)
    bb.results.fill_(0xAB)
    bb.run(keys, max_bucket=100)  # slots sized for 500; the declared bound says 100
    torch.cuda.synchronize()
    res = bb.bucket_results()
    assert res[1]["status"] == mx.EINVAL
    assert res[0]["status"] in (0, 1) and res[2]["status"] in (0, 1)


@pytest.mark.parametrize("block", [512, 1024])
def test_batch_clock_counts_the_work_and_changes_nothing(mx, o, block):
    """The clocked kernel (option batch_clock) builds the same outputs as the plain one, and its
    counters add up: every bucket and key counted once, by the LDS path or the device path, and
    the phases within the workgroups' lifetimes."""
    import torch

    sizes = np.concatenate([[1, 7, 3000], workloads.bucket_sizes(40, 100, 200_000, seed=11)]).astype(np.uint64)
    off = _offsets(sizes)
    keys = mx.gen_buckets_u64(torch.from_numpy(off.view(np.int64)).cuda())
    bb = mx.BatchBuild(off, block=block, grid=0, scope=0)
    bb.run(keys)
    torch.cuda.synchronize()
    ref_codes = [bb.bucket_codes(b).cpu().numpy().copy() for b in range(len(sizes))]
    ref_res = bb.bucket_results().copy()
    old = mx.get_option("batch_clock")
    try:
        mx.batch_clock(reset=True)
        mx.set_option("batch_clock", 1)
        bb.run(keys)
        torch.cuda.synchronize()
        c = mx.batch_clock(reset=True)
    finally:
        mx.set_option("batch_clock", old)
    res = bb.bucket_results()
    assert np.array_equal(res, ref_res)
    for b in range(len(sizes)):
        assert np.array_equal(bb.bucket_codes(b).cpu().numpy(), ref_codes[b]), b
    assert c["tick_hz"] > 0
    assert c["device_buckets"] + c["lds_bucket_count"] == len(sizes)
    assert c["device_keys"] + c["lds_keys"] == int(sizes.sum())
    big = sizes > 20_000  # too large for the LDS path at either workgroup size
    assert c["device_buckets"] >= int(big.sum()) and c["device_keys"] >= int(sizes[big].sum())
    assert c["tries"] >= c["device_buckets"] and c["rounds"] > 0 and c["list_records"] > 0
    # two deletes per edge of the device-path buckets' list rounds at most
    assert 0 < c["deletes_issued"] <= 2 * c["device_keys"]
    phases = ("records", "deletes", "claim_grouping", "resolve", "other_rounds", "assign", "pack", "lds_buckets", "queue")
    assert all(c[p] >= 0 for p in phases) and c["records"] > 0 and c["deletes"] > 0 and c["assign"] > 0
    assert sum(c[p] for p in phases) <= c["workgroup"]
    assert mx.batch_clock()["workgroup"] == 0  # the read above reset it


def test_build_batch_descriptors_mixed_kinds(mx, o):
    """The general entry point: unrelated u64 and string key sets, each with its own seed and
    outputs, built in one launch; each equals the oracle's single build."""
    import torch

    def dev(a):
        a = np.ascontiguousarray(a)
        return torch.from_numpy(a.view(np.int64) if a.dtype == np.uint64 else a).cuda()

    buckets, refs = [], []
    for i, n in enumerate([1, 5, 100, 999, 5000, 30000, 70001]):
        keys = workloads.u64_keys(n, gen_seed=300 + i)
        buckets.append(("u64", dev(keys), 7 + i))
        refs.append(o.mphf_build_u64(keys, seed=7 + i))
        d, of = workloads.str_keys(n, gen_seed=400 + i)
        buckets.append(("str", dev(d), dev(of), 9 + i))
        refs.append(o.mphf_build_str(d, of, seed=9 + i))
    for block, scope in ((1024, 0), (256, 1)):
        out = mx.build_batch(buckets, block=block, grid=5, scope=scope)
        for b, (got, (rc, ref)) in enumerate(zip(out, refs)):
            assert got["status"] == rc, b
            assert got["tries"] == ref["tries"] and got["seed_used"] == ref["seed_used"], b
            if rc == 0:
                assert got["n_rounds"] == ref["n_rounds"], b
                assert np.array_equal(got["codes"].cpu().numpy().view(np.uint64), ref["words"]), b
                assert np.array_equal(got["rank"].cpu().numpy().view(np.uint64), ref["rank"]), b


def test_autotune_picks_a_candidate_and_every_tuning_builds_the_same(mx, o):
    # the autotuner times the library's candidate tunings on this batch, keeps the fastest, and
    # leaves the batch built; a later run with the chosen tuning equals the oracle bucket by bucket
    import torch

    off = _offsets(SIZES)
    keys = mx.gen_buckets_u64(torch.from_numpy(off.view(np.int64)).cuda())
    keys_h = _host_keys(SIZES)
    bb = mx.BatchBuild(off, block=1024)
    ws_before = bb.ws.numel()
    bb.capture(keys)
    t = bb.autotune(keys, reps=1)
    assert bb.graph is None  # the graph held the old workspace: dropped
    assert len(t["candidates"]) == 5 and 0 <= t["best"] < 5
    assert all(ms > 0 for ms in t["ms"]) and t["ms"][t["best"]] == min(t["ms"])
    assert (bb.tuning.block, bb.tuning.grid) == tuple(t["candidates"][t["best"]])
    assert bb.ws.numel() >= ws_before
    torch.cuda.synchronize()
    _check_buckets(mx, o, bb, keys_h, SIZES)  # the outputs of the last timed build
    bb.codes.zero_()
    bb.rank.zero_()
    bb.run(keys)
    torch.cuda.synchronize()
    _check_buckets(mx, o, bb, keys_h, SIZES)
    bb.codes.zero_()
    bb.rank.zero_()
    bb.capture(keys)  # captured again with the chosen tuning and the new workspace
    bb.launch()
    torch.cuda.synchronize()
    _check_buckets(mx, o, bb, keys_h, SIZES)
    bb.destroy_graph()
    # a workspace cap below every candidate but the 1024-thread one skips the others
    bb2 = mx.BatchBuild(off, block=1024)
    t2 = bb2.autotune(keys, candidates=[(1024, 0, 0), (256, 4096, 0)], reps=1, max_ws_bytes=bb2.ws.numel())
    assert t2["best"] == 0 and t2["ms"][0] > 0 and t2["ms"][1] == -1
