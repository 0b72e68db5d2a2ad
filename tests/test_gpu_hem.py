"""HEM split (Section 3) through the C ABI against the oracle: bucket offsets, per-bucket
seeds, codes and rank samples bit for bit, and the lookups."""
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


def host(t):
    return t.cpu().numpy().view(np.uint64)


def _assert_same(got, ref):
    for key in ("bucket_off", "code_off", "rank_off", "seeds", "codes", "rank"):
        assert np.array_equal(host(got[key]), ref[key]), key


@pytest.mark.parametrize("n,k,seed", [(1_000_000, 10, 3), (200_000, 9, 0), (20_000, 9, 5), (300_000, 14, 1)])
def test_hem_u64_matches_oracle(mx, o, n, k, seed):
    keys = workloads.u64_keys(n, gen_seed=k)
    got = mx.hem_build(keys=dev(keys), k=k, seed=seed)
    rc, ref = o.hem_build(o.hem_signatures_u64(keys, seed), k, seed=seed)
    assert rc == 0
    _assert_same(got, ref)
    f = mx.hem_lookup(got, keys=dev(keys))
    assert np.array_equal(host(f), o.hem_lookup(ref, o.hem_signatures_u64(keys, seed)))
    assert np.array_equal(np.sort(host(f)), np.arange(n, dtype=np.uint64))


def test_hem_str_matches_oracle(mx, o):
    data, offs = workloads.str_keys(120_000, gen_seed=21)
    got = mx.hem_build(data=dev(data), offs=dev(offs), k=11, seed=4)
    sigs = o.hem_signatures_str(data, offs, 4)
    rc, ref = o.hem_build(sigs, 11, seed=4)
    assert rc == 0
    _assert_same(got, ref)
    f = mx.hem_lookup(got, data=dev(data), offs=dev(offs))
    assert np.array_equal(host(f), o.hem_lookup(ref, sigs))


def test_hem_empty_and_errors(mx):
    import torch

    got = mx.hem_build(keys=torch.empty(0, dtype=torch.int64, device="cuda"), k=9)
    assert int(got["bucket_off"].abs().sum()) == 0 and got["codes"].numel() == 0
    keys = dev(workloads.u64_keys(1000))
    for bad_k in (8, 21):  # k = 8 would need a 32-bit group shift
        with pytest.raises((mx.MphxError, ValueError)):
            mx.hem_build(keys=keys, k=bad_k)


def test_hem_two_key_buckets_never_build(mx, o):
    # About two keys per bucket: a bucket of exactly two keys has parts of one vertex at
    # gamma = 1.23, so both edges are (0, 1, 2) and form a 2-core under every seed.  Both sides
    # must report the failure; the GPU counts at least those buckets as failed.
    k, seed = 9, 5
    keys = workloads.u64_keys(1000, gen_seed=k)
    sigs = o.hem_signatures_u64(keys, seed)
    sizes = np.bincount((sigs >> np.uint64(64 - k)).astype(np.int64), minlength=1 << k)
    assert (sizes == 2).sum() > 0
    rc, _ = o.hem_build(sigs, k, seed=seed)
    assert rc == 1  # the oracle's 2-core status
    with pytest.raises(mx.MphxError) as e:
        mx.hem_build(keys=dev(keys), k=k, seed=seed)
    assert e.value.status == mx.ECORE
    assert e.value.info["n_core"] >= int((sizes == 2).sum())


# ---- keys in host memory, streamed in chunks (key sets beyond device memory) ----------------
def _same_tables(a, b):
    for key in ("bucket_off", "code_off", "rank_off", "seeds", "codes", "rank"):
        assert np.array_equal(host(a[key]), host(b[key])), key


def _host_u64(keys, pinned=False):
    import torch

    t = torch.from_numpy(np.ascontiguousarray(keys).view(np.int64))
    return t.pin_memory() if pinned else t


@pytest.mark.parametrize("n,k,seed,chunk,batch,pinned", [
    (300_000, 12, 1, 40_000, 60_000, False),      # 8 chunks, 5 batches of 3-4 groups
    (1_000_000, 10, 3, 1 << 20, 1 << 20, True),   # one chunk, one batch, pinned
    (200_000, 9, 0, 65_537, 150_000, False),      # ragged chunks, one group per batch
    (120_000, 12, 2, 7_777, 10_000, True),        # 16 chunks, one group per batch
])
def test_hem_host_u64_matches_oracle_and_device_build(mx, o, n, k, seed, chunk, batch, pinned):
    keys = workloads.u64_keys(n, gen_seed=100 + k)
    got = mx.hem_build_host(keys=_host_u64(keys, pinned), k=k, seed=seed, chunk_keys=chunk, batch_keys=batch)
    rc, ref = o.hem_build(o.hem_signatures_u64(keys, seed), k, seed=seed)
    assert rc == 0
    _assert_same(got, ref)
    _same_tables(got, mx.hem_build(keys=dev(keys), k=k, seed=seed))
    f = mx.hem_lookup(got, keys=dev(keys))
    assert np.array_equal(host(f), o.hem_lookup(ref, o.hem_signatures_u64(keys, seed)))


def test_hem_host_str_matches_oracle(mx, o):
    import torch

    data, offs = workloads.str_keys(100_000, gen_seed=31)
    got = mx.hem_build_host(data=torch.from_numpy(data), offs=torch.from_numpy(offs.view(np.int64)), k=11, seed=6,
                            chunk_keys=20_000, chunk_bytes=1 << 19, batch_keys=30_000)
    sigs = o.hem_signatures_str(data, offs, 6)
    rc, ref = o.hem_build(sigs, 11, seed=6)
    assert rc == 0
    _assert_same(got, ref)
    f = mx.hem_lookup(got, data=dev(data), offs=dev(offs))
    assert np.array_equal(host(f), o.hem_lookup(ref, sigs))


def test_hem_host_empty_and_errors(mx):
    import torch

    empty = mx.hem_build_host(keys=torch.empty(0, dtype=torch.int64), k=9, chunk_keys=1000, batch_keys=1000)
    _same_tables(empty, mx.hem_build(keys=torch.empty(0, dtype=torch.int64, device="cuda"), k=9))
    keys = _host_u64(workloads.u64_keys(50_000))
    with pytest.raises(mx.MphxError) as e:  # groups of about 25,000 keys
        mx.hem_build_host(keys=keys, k=9, chunk_keys=10_000, batch_keys=20_000)
    assert e.value.status == mx.ENOMEM
    # a key longer than a chunk's bytes
    lens = np.array([10, 600, 10], dtype=np.int64)
    offs = np.zeros(4, dtype=np.int64)
    offs[1:] = np.cumsum(lens)
    data = torch.from_numpy(np.arange(offs[-1], dtype=np.int64).astype(np.uint8))
    with pytest.raises(mx.MphxError) as e:
        mx.hem_build_host(data=data, offs=torch.from_numpy(offs), k=9, chunk_keys=10, chunk_bytes=512, batch_keys=100)
    assert e.value.status == mx.EINVAL
    with pytest.raises(ValueError):
        mx.hem_build_host(keys=keys, k=9, chunk_keys=0, batch_keys=100)
    with pytest.raises(TypeError):
        mx.hem_build_host(keys=keys.cuda(), k=9)


# ---- more than 2^18 buckets: each bucket of the top 18 bits split by the next k - 18 bits ----
# gamma = 2 keeps buckets of a few dozen keys buildable within the retry budget on both sides
# (at 1.23 they hit a 2-core on most tries); the split itself does not depend on gamma.
def test_hem_k19_matches_oracle(mx, o):
    keys = workloads.u64_keys(12_000_000, gen_seed=219)
    got = mx.hem_build(keys=dev(keys), k=19, seed=7, gamma=(2, 1))
    sigs = o.hem_signatures_u64(keys, 7)
    rc, ref = o.hem_build(sigs, 19, seed=7, gnum=2, gden=1)
    assert rc == 0
    _assert_same(got, ref)
    sample = keys[:: 97]
    f = mx.hem_lookup(got, keys=dev(sample))
    assert np.array_equal(host(f), o.hem_lookup(ref, o.hem_signatures_u64(sample, 7), gnum=2, gden=1))


def _str_subset(data, offs, idx):
    """The keys idx of a string set, as a new (bytes, offsets) pair with 4-byte aligned data."""
    lens = (offs[idx + 1] - offs[idx]).astype(np.int64)
    so = np.zeros(len(idx) + 1, np.int64)
    so[1:] = np.cumsum(lens)
    sd = np.zeros(((int(so[-1]) + 3) // 4) * 4 or 4, np.uint8)
    for j, i in enumerate(idx):
        sd[so[j]:so[j + 1]] = data[offs[i]:offs[i + 1]]
    return sd, so.view(np.uint64)


def test_hem_str_k19_matches_oracle_in_hbm_and_from_host(mx, o):
    """String keys at 2^19 buckets: the 128-bit signature records through the two-pass
    partition and the refinement by the next bit, in HBM and streamed from host memory."""
    import torch

    data, offs = workloads.str_keys(6_000_000, gen_seed=319)
    got = mx.hem_build(data=dev(data), offs=dev(offs), k=19, seed=8, gamma=(2, 1))
    sigs = o.hem_signatures_str(data, offs, 8)
    rc, ref = o.hem_build(sigs, 19, seed=8, gnum=2, gden=1)
    assert rc == 0
    _assert_same(got, ref)
    sample = np.arange(0, 6_000_000, 89)
    sd, so = _str_subset(data, offs, sample)
    f = mx.hem_lookup(got, data=dev(sd), offs=dev(so))
    assert np.array_equal(host(f), o.hem_lookup(ref, sigs[sample], gnum=2, gden=1))
    got_h = mx.hem_build_host(data=torch.from_numpy(data), offs=torch.from_numpy(offs.view(np.int64)), k=19, seed=8,
                              gamma=(2, 1), chunk_keys=1_500_000, chunk_bytes=1 << 27, batch_keys=2_500_000)
    _assert_same(got_h, ref)


def test_hem_host_k20_matches_oracle_and_device_build(mx, o):
    keys = workloads.u64_keys(24_000_000, gen_seed=220)
    got = mx.hem_build_host(keys=_host_u64(keys), k=20, seed=7, gamma=(2, 1), chunk_keys=5_000_000,
                            batch_keys=8_000_000)
    rc, ref = o.hem_build(o.hem_signatures_u64(keys, 7), 20, seed=7, gnum=2, gden=1)
    assert rc == 0
    _assert_same(got, ref)
    _same_tables(got, mx.hem_build(keys=dev(keys), k=20, seed=7, gamma=(2, 1)))
