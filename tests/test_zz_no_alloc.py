"""The allocation-free MPHF build (mphx_mphf_build_u64_static) through the C ABI: its outputs
equal those of mphx_mphf_build_u64 with a caller workspace, on two calls in a row (the second
on fewer keys, over the first call's leftovers in the shared static workspace), and sizes
beyond its 128 MiB workspace are refused with ENOMEM."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

STATIC_BYTES = 128 << 20


@pytest.fixture(scope="module")
def mx():
    import torch

    import paper_1312_0526_amd as mx

    assert torch.cuda.is_available()
    mx.lib()
    return mx


def _dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()


def _outs(mx, n):
    import torch

    m = 3 * mx.part_size(n, (123, 100))
    return (torch.full(((m + 31) // 32,), -1, dtype=torch.int64, device="cuda"),
            torch.full(((m + 511) // 512,), -1, dtype=torch.int64, device="cuda"))


def _max_keys(mx):
    a, b = 1, 1 << 26
    while a < b:
        mid = (a + b + 1) // 2
        if mx.mphf_workspace_bytes(mid) <= STATIC_BYTES:
            a = mid
        else:
            b = mid - 1
    return a


def test_static_build_equals_the_workspace_build_on_two_calls(mx):
    import torch

    nmax = _max_keys(mx)
    for n, gs, seed in [(nmax, 3, 11), (1_000, 4, 12)]:  # the largest accepted size, then a small one
        keys = _dev(workloads.u64_keys(n, gen_seed=gs))
        ref = mx.mphf_build_u64(keys, seed=seed)
        got = mx.mphf_build_u64_static(keys, _outs(mx, n), seed=seed)
        torch.cuda.synchronize()
        for k in ("P", "m", "seed_used", "tries", "n_rounds", "n_core", "layer0"):
            assert got[k] == ref[k], k
        assert torch.equal(got["codes"], ref["codes"]) and torch.equal(got["rank"], ref["rank"])
    # the small build also equals the oracle
    o = oracle.Oracle()
    rc, oref = o.mphf_build_u64(workloads.u64_keys(1_000, gen_seed=4), seed=12)
    assert rc == 0
    assert np.array_equal(got["codes"].cpu().numpy().view(np.uint64), oref["words"])
    assert np.array_equal(got["rank"].cpu().numpy().view(np.uint64), oref["rank"])


def test_static_build_refuses_sizes_beyond_its_workspace(mx):
    n = _max_keys(mx) + 1
    keys = _dev(workloads.u64_keys(n, gen_seed=5))
    with pytest.raises(mx.MphxError) as ei:
        mx.mphf_build_u64_static(keys, _outs(mx, n))
    assert ei.value.status == mx.ENOMEM
    # the next call on the device still works
    keys = _dev(workloads.u64_keys(5_000, gen_seed=6))
    got = mx.mphf_build_u64_static(keys, _outs(mx, 5_000), seed=2)
    ref = mx.mphf_build_u64(keys, seed=2)
    assert got["seed_used"] == ref["seed_used"]
    assert np.array_equal(got["codes"].cpu().numpy(), ref["codes"].cpu().numpy())
