"""Static functions (Section 3: f(x) = u[h0] + u[h1] + u[h2] mod sigma) through the C ABI,
against the oracle: the packed fields bit for bit, the lookups equal to the stored values."""
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


def dev(a):
    import torch

    a = np.ascontiguousarray(a)
    view = {np.dtype(np.uint64): np.int64, np.dtype(np.uint32): np.int32}.get(a.dtype)
    return torch.from_numpy(a.view(view) if view else a).cuda()


def host(t, dtype):
    return t.cpu().numpy().view(dtype)


def values_for(n, sigma, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, sigma, n, dtype=np.uint64).astype(np.uint32)


@pytest.fixture(params=[(None, None), (1, 0), (1, 1), (1, 16), (0, 0)],
                ids=["default", "claim-lists", "update-lists-most-rounds", "update-lists-dense-rounds", "atomic-claims"])
def mode(request, mx):
    lists, upd = request.param
    old = mx.get_option("claim_lists"), mx.get_option("update_lists")
    if lists is not None:
        mx.set_option("claim_lists", lists)
        mx.set_option("update_lists", upd)
    yield request.param
    mx.set_option("claim_lists", old[0])
    mx.set_option("update_lists", old[1])


@pytest.mark.parametrize("n,sigma", [(1_000_000, 256), (12_345, 3), (54_321, 1_000_003), (33_333, 65_521), (7, 2), (1, 1 << 32)])
def test_sf_u64_matches_oracle(mx, o, mode, n, sigma):
    keys = workloads.u64_keys(n, gen_seed=n)
    vals = values_for(n, sigma, n)
    got = mx.sf_build_u64(dev(keys), dev(vals), sigma, seed=5)
    rc, ref = o.sf_build_u64(keys, vals, sigma, seed=5)
    assert rc == 0
    assert got["P"] == ref["P"] and got["seed_used"] == ref["seed_used"] and got["tries"] == ref["tries"]
    assert np.array_equal(host(got["words"], np.uint64), ref["words"])
    f = mx.sf_lookup_u64(got["words"], sigma, got["P"], got["seed_used"], dev(keys))
    assert np.array_equal(host(f, np.uint64), vals.astype(np.uint64))


def test_sf_str_matches_oracle(mx, o, mode):
    data, offs = workloads.str_keys(150_000, gen_seed=31)
    vals = values_for(150_000, 1000, 3)
    got = mx.sf_build_str(dev(data), dev(offs), dev(vals), 1000, seed=1)
    rc, ref = o.sf_build_str(data, offs, vals, 1000, seed=1)
    assert rc == 0
    assert np.array_equal(host(got["words"], np.uint64), ref["words"])
    f = mx.sf_lookup_str(got["words"], 1000, got["P"], got["seed_used"], dev(data), dev(offs))
    assert np.array_equal(host(f, np.uint64), vals.astype(np.uint64))


def test_sf_sigma_one_small_buckets_and_errors(mx, o):
    keys = workloads.u64_keys(5000, gen_seed=77)
    got = mx.sf_build_u64(dev(keys), dev(np.zeros(5000, np.uint32)), 1)
    assert got["words"].numel() == 0
    f = mx.sf_lookup_u64(got["words"], 1, got["P"], got["seed_used"], dev(keys))
    assert int(f.abs().sum()) == 0
    retried = 0
    for b in range(20):  # n = 100 retries often: tries and seeds follow the oracle
        keys = workloads.u64_keys(100, gen_seed=workloads.bucket_gen_seed(b))
        vals = values_for(100, 97, b)
        got = mx.sf_build_u64(dev(keys), dev(vals), 97)
        rc, ref = o.sf_build_u64(keys, vals, 97)
        assert rc == 0 and got["tries"] == ref["tries"]
        assert np.array_equal(host(got["words"], np.uint64), ref["words"])
        retried += got["tries"] > 1
    assert retried > 3
    keys = workloads.u64_keys(1000)
    with pytest.raises(mx.MphxError) as ei:
        mx.sf_build_u64(dev(keys), dev(np.full(1000, 7, np.uint32)), 7)
    assert ei.value.status == mx.EINVAL
    with pytest.raises(mx.MphxError) as ei:
        mx.sf_build_u64(dev(keys), dev(np.zeros(1000, np.uint32)), 0)
    assert ei.value.status == mx.EINVAL
    with pytest.raises(mx.MphxError) as ei:
        mx.sf_build_u64(dev(keys), dev(np.zeros(1000, np.uint32)), 5, gamma=(120, 100), max_tries=1)
    assert ei.value.status == mx.ECORE


# ---- the ranked layout (Section 3: a ranking structure over the non-zero values) ------------
def _same_ranked(got, lay):
    assert np.array_equal(host(got["marks"], np.uint64), lay["marks"])
    assert np.array_equal(host(got["rank"], np.uint64), lay["rank"])
    gv = host(got["vals"], np.uint64)
    nv = len(lay["vals"])
    assert np.array_equal(gv[:nv], lay["vals"]) and not gv[nv:].any()


@pytest.mark.parametrize("n,sigma", [(1_000_000, 256), (12_345, 3), (54_321, 1_000_003), (33_333, 65_521), (7, 2),
                                     (1, 1 << 32), (300_001, 1 << 32), (5000, 1), (2_000_003, 2)])
def test_sfr_u64_matches_oracle(mx, o, n, sigma):
    """Marks, rank samples and fields bit for bit against the oracle's ranked layout of its own
    function; every key's lookup returns its value; the oracle's ranked lookup reads the GPU's
    tables the same way."""
    keys = workloads.u64_keys(n, gen_seed=n + 1)
    vals = values_for(n, sigma, n + 1)
    got = mx.sfr_build_u64(dev(keys), dev(vals), sigma, seed=5)
    rc, ref = o.sf_build_u64(keys, vals, sigma, seed=5)
    assert rc == 0
    assert got["P"] == ref["P"] and got["seed_used"] == ref["seed_used"] and got["tries"] == ref["tries"]
    lay = o.sf_rank_layout(ref["words"], ref["m"], sigma)
    _same_ranked(got, lay)
    assert int(host(got["rank"], np.uint64)[-1]) == lay["count"] <= n
    f = mx.sfr_lookup_u64(got, sigma, dev(keys))
    assert np.array_equal(host(f, np.uint64), vals.astype(np.uint64))
    pick = keys[:: max(1, n // 2000)]
    fo = o.sfr_lookup_u64(host(got["marks"], np.uint64), host(got["rank"], np.uint64), host(got["vals"], np.uint64),
                          sigma, got["P"], got["seed_used"], pick)
    assert np.array_equal(fo, vals[:: max(1, n // 2000)].astype(np.uint64))
    if sigma == 256:  # b n + m + rank samples, against b m for the plain layout
        m, b = ref["m"], 8
        assert m + 64 * len(lay["rank"]) + lay["count"] * b < 0.96 * b * m


def test_sfr_str_matches_oracle_and_reused_buffers(mx, o):
    """Strings; then the same output buffers reused by a smaller build, whose fields must not
    keep the larger build's words."""
    data, offs = workloads.str_keys(150_000, gen_seed=32)
    vals = values_for(150_000, 1000, 4)
    got = mx.sfr_build_str(dev(data), dev(offs), dev(vals), 1000, seed=1)
    rc, ref = o.sf_build_str(data, offs, vals, 1000, seed=1)
    assert rc == 0
    _same_ranked(got, o.sf_rank_layout(ref["words"], ref["m"], 1000))
    f = mx.sfr_lookup_str(got, 1000, dev(data), dev(offs))
    assert np.array_equal(host(f, np.uint64), vals.astype(np.uint64))
    import torch

    sizes = mx.sfr_sizes(150_000, 1000)
    bufs = tuple(torch.full((max(w, 1),), -1, dtype=torch.int64, device="cuda") for w in sizes)
    keys = workloads.u64_keys(40_000, gen_seed=8)
    vals = values_for(40_000, 1000, 8)
    got = mx.sfr_build_u64(dev(keys), dev(vals), 1000, seed=2, out=bufs)
    rc, ref = o.sf_build_u64(keys, vals, 1000, seed=2)
    assert rc == 0
    _same_ranked(got, o.sf_rank_layout(ref["words"], ref["m"], 1000))
    f = mx.sfr_lookup_u64(got, 1000, dev(keys))
    assert np.array_equal(host(f, np.uint64), vals.astype(np.uint64))


def test_sfr_errors(mx):
    keys = workloads.u64_keys(1000)
    with pytest.raises(mx.MphxError) as ei:
        mx.sfr_build_u64(dev(keys), dev(np.full(1000, 7, np.uint32)), 7)
    assert ei.value.status == mx.EINVAL
    lib = mx.lib()
    import ctypes as C

    import torch

    ws = torch.empty(mx.sf_workspace_bytes(1000), dtype=torch.uint8, device="cuda")
    info = mx._lib.MphfInfo()
    # null marks: refused before any work
    rc = lib.mphx_sfr_build_u64(dev(keys).data_ptr(), dev(np.zeros(1000, np.uint32)).data_ptr(), 1000, 5, 0, 123, 100,
                                4, None, ws.data_ptr(), ws.data_ptr(), ws.data_ptr(), ws.numel(), None, C.byref(info))
    assert rc == mx.EINVAL
