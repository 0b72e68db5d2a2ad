"""The streamed MWHC build (keys in host memory; vertex records of Section 4.1 with the XOR of
the other two endpoints, no edge ids; layers optionally spilled to host memory) through the C
ABI, against the oracle: codes, rank, seed, tries and rounds bit for bit (GPU only)."""
import ctypes as C

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


def _host(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64))


def _same(got, ref):
    for key in ("P", "m", "seed_used", "tries", "n_rounds"):
        assert got[key] == ref[key], key
    assert np.array_equal(got["codes"].cpu().numpy().view(np.uint64), ref["words"])
    assert np.array_equal(got["rank"].cpu().numpy().view(np.uint64), ref["rank"])


@pytest.mark.parametrize("spill", [False, True], ids=["layers-in-hbm", "layers-spilled-to-host"])
def test_stream_build_2e24_matches_oracle(mx, o, spill):
    """2^24 keys in 8 chunks; with spilling, a layer area of 0.3 n slots (round 0's layer is
    about 0.24 n) and every layer through host memory."""
    import torch

    n = 1 << 24
    keys = workloads.u64_keys(n, gen_seed=24)
    rc, ref = o.mphf_build_u64(keys, seed=5)
    assert rc == 0
    got = mx.mphf_build_stream_u64(_host(keys), seed=5, chunk_keys=1 << 21,
                                   layer_slots=(3 * n) // 10 if spill else 0)
    _same(got, ref)
    assert got["n_core"] == 0 and 0.2 * n < got["layer0"] < 0.3 * n
    # the wide lookup of the device keys equals the oracle's evaluation
    dk = torch.from_numpy(keys[:: 1001].view(np.int64)).cuda()
    f = mx.lookup_wide_u64(got["codes"], got["rank"], got["P"], got["seed_used"], dk)
    assert np.array_equal(f.cpu().numpy().view(np.uint64),
                          o.lookup_u64(ref["words"], ref["rank"], ref["P"], ref["seed_used"], keys[:: 1001]))
    # all keys streamed through the evaluation: a bijection onto [0, n)
    assert mx.check_stream_u64(got["codes"], got["rank"], got["P"], got["seed_used"], _host(keys),
                               chunk_keys=3_000_000) == 0


def test_stream_build_pinned_keys_and_small_sets(mx, o):
    """Pinned host keys and layer buffer; small key sets whose first tries leave a 2-core (retries with seed + 1
    on both sides); one key; a set of two keys, which can never peel."""
    import torch

    keys = workloads.u64_keys(1_000_003, gen_seed=3)
    pinned = torch.empty(len(keys), dtype=torch.int64).pin_memory()
    pinned.copy_(_host(keys))
    layers = torch.empty(12 * len(keys), dtype=torch.uint8).pin_memory()  # spilled layers pinned too
    got = mx.mphf_build_stream_u64(pinned, seed=2, chunk_keys=300_000, layer_slots=400_000, host_layers=layers)
    rc, ref = o.mphf_build_u64(keys, seed=2)
    assert rc == 0
    _same(got, ref)
    retried = 0
    for b in range(12):
        kb = workloads.u64_keys(150, gen_seed=workloads.bucket_gen_seed(b))
        got = mx.mphf_build_stream_u64(_host(kb), seed=0, chunk_keys=64)
        rc, ref = o.mphf_build_u64(kb, seed=0)
        assert rc == 0
        _same(got, ref)
        retried += got["tries"] > 1
    assert retried >= 2
    one = workloads.u64_keys(1, gen_seed=9)
    got = mx.mphf_build_stream_u64(_host(one), seed=1)
    rc, ref = o.mphf_build_u64(one, seed=1)
    _same(got, ref)
    with pytest.raises(mx.MphxError) as ei:
        mx.mphf_build_stream_u64(_host(workloads.u64_keys(2)), max_tries=3)
    assert ei.value.status == mx.ECORE and o.mphf_build_u64(workloads.u64_keys(2), max_tries=3)[0] == oracle.ECORE


def test_stream_build_errors(mx):
    import torch

    keys = _host(workloads.u64_keys(100_000, gen_seed=4))
    # a layer area smaller than round 0's layer
    with pytest.raises(mx.MphxError) as ei:
        mx.mphf_build_stream_u64(keys, layer_slots=1000)
    assert ei.value.status == mx.ENOMEM
    # spilling without a big enough host buffer
    with pytest.raises(mx.MphxError) as ei:
        mx.mphf_build_stream_u64(keys, layer_slots=50_000, host_layers=torch.empty(1000, dtype=torch.uint8))
    assert ei.value.status == mx.EINVAL
    # below gamma 1 the 2-core is large: no seed peels it
    with pytest.raises(mx.MphxError) as ei:
        mx.mphf_build_stream_u64(keys, gamma=(100, 100), max_tries=2)
    assert ei.value.status == mx.ECORE and ei.value.info["n_core"] > 0
    # duplicate-heavy keys reach degree 256
    dup = _host(np.repeat(workloads.u64_keys(10, gen_seed=5), 300))
    with pytest.raises(mx.MphxError) as ei:
        mx.mphf_build_stream_u64(dup)
    assert ei.value.status == mx.ERANGE
    # P above 2^32 is refused before any key is read (n of 1.1e10 at gamma 1.23)
    lib = mx.lib()
    info = mx._lib.MphfInfo()
    ws = torch.empty(256, dtype=torch.uint8, device="cuda")
    rc = lib.mphx_mphf_build_stream_u64(keys.data_ptr(), 11_000_000_000, 0, 123, 100, 1, 1 << 20, 1 << 20, None, 0,
                                        ws.data_ptr(), ws.data_ptr(), ws.data_ptr(), 256, None, C.byref(info))
    assert rc == mx.EINVAL
    assert mx.stream_workspace_bytes(11_000_000_000) == 0
