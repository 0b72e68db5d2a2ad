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
    for bad_k in (8, 19):  # k = 8 would need a 32-bit group shift
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
