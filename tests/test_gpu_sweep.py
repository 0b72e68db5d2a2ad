"""A seeded sweep of many small and ragged cases against the oracle (GPU only): sizes
log-uniform from 1 to 3*10^5 keys, gamma from 1.20 to 1.60, random seeds, u64 and string keys,
every claim mode, through the MPHF, static-function (plain and ranked) and batched entry
points.  Every case is bit-exact or fails with the same status on both sides."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

_OPTS = ("claim_lists", "update_lists")


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


def host(t, dt):
    return t.cpu().numpy().view(dt)


def _cases(count, seed):
    rng = np.random.default_rng(seed)
    for i in range(count):
        n = int(np.floor(10 ** rng.uniform(0, np.log10(3e5))))
        gnum = int(rng.integers(120, 161))
        yield i, n, (gnum, 100), int(rng.integers(0, 1 << 40)), bool(rng.integers(0, 2)), int(rng.integers(0, 3))


@pytest.mark.parametrize("chunk", range(4))
def test_mphf_sweep(mx, o, chunk):
    """60 cases per chunk: the claim mode cycles through atomic claims, claim lists and claim
    lists with update lists for nearly every round."""
    old = [mx.get_option(k) for k in _OPTS]
    try:
        for i, n, gamma, seed, strings, mode in _cases(60, 1000 + chunk):
            mx.set_option("claim_lists", (0, 1, 1)[mode])
            mx.set_option("update_lists", (16, 0, 1)[mode])
            case = f"case {i}: n={n} gamma={gamma} seed={seed} strings={strings} mode={mode}"
            if strings:
                data, offs = workloads.str_keys(n, gen_seed=seed & 0xFFFF)
                rc, ref = o.mphf_build_str(data, offs, seed=seed, gnum=gamma[0], gden=gamma[1], max_tries=8)
                call = lambda: mx.mphf_build_str(dev(data), dev(offs), seed=seed, gamma=gamma, max_tries=8)
            else:
                keys = workloads.u64_keys(n, gen_seed=seed & 0xFFFF)
                rc, ref = o.mphf_build_u64(keys, seed=seed, gnum=gamma[0], gden=gamma[1], max_tries=8)
                call = lambda: mx.mphf_build_u64(dev(keys), seed=seed, gamma=gamma, max_tries=8)
            if rc != 0:
                with pytest.raises(mx.MphxError) as ei:
                    call()
                assert ei.value.status == rc, case
                continue
            got = call()
            assert got["tries"] == ref["tries"] and got["seed_used"] == ref["seed_used"], case
            assert got["n_rounds"] == ref["n_rounds"], case
            assert np.array_equal(host(got["codes"], np.uint64), ref["words"]), case
            assert np.array_equal(host(got["rank"], np.uint64), ref["rank"]), case
    finally:
        for k, v in zip(_OPTS, old):
            mx.set_option(k, v)


def test_static_function_sweep(mx, o):
    """40 cases: sigma log-uniform from 1 to 2^32, plain and ranked layouts against the
    oracle's, and lookups equal to the values."""
    rng = np.random.default_rng(77)
    for i, n, gamma, seed, _, _ in _cases(40, 2000):
        sigma = int(min(1 << 32, max(1, np.floor(2 ** rng.uniform(0, 32)))))
        keys = workloads.u64_keys(n, gen_seed=seed & 0xFFFF)
        vals = rng.integers(0, sigma, n, dtype=np.uint64).astype(np.uint32)
        case = f"case {i}: n={n} gamma={gamma} seed={seed} sigma={sigma}"
        rc, ref = o.sf_build_u64(keys, vals, sigma, seed=seed, gnum=gamma[0], gden=gamma[1], max_tries=8)
        if rc != 0:
            with pytest.raises(mx.MphxError) as ei:
                mx.sf_build_u64(dev(keys), dev(vals), sigma, seed=seed, gamma=gamma, max_tries=8)
            assert ei.value.status == rc, case
            continue
        got = mx.sf_build_u64(dev(keys), dev(vals), sigma, seed=seed, gamma=gamma, max_tries=8)
        assert got["seed_used"] == ref["seed_used"], case
        assert np.array_equal(host(got["words"], np.uint64), ref["words"]), case
        lay = o.sf_rank_layout(ref["words"], ref["m"], sigma)
        gr = mx.sfr_build_u64(dev(keys), dev(vals), sigma, seed=seed, gamma=gamma, max_tries=8)
        assert np.array_equal(host(gr["marks"], np.uint64), lay["marks"]), case
        assert np.array_equal(host(gr["rank"], np.uint64), lay["rank"]), case
        gv = host(gr["vals"], np.uint64)
        assert np.array_equal(gv[: len(lay["vals"])], lay["vals"]) and not gv[len(lay["vals"]):].any(), case
        f = mx.sfr_lookup_u64(gr, sigma, dev(keys))
        assert np.array_equal(host(f, np.uint64), vals.astype(np.uint64)), case


@pytest.mark.parametrize("block", [256, 512, 1024])
def test_batch_sweep(mx, o, block):
    """300 buckets of log-uniform sizes 1 to 3*10^5 in one launch, every bucket against the
    oracle's single build (tries, seed, rounds, codes, rank)."""
    import torch

    rng = np.random.default_rng(block)
    sizes = np.floor(10 ** rng.uniform(0, np.log10(3e5), 300)).astype(np.uint64)
    off = np.zeros(len(sizes) + 1, np.uint64)
    off[1:] = np.cumsum(sizes)
    keys = mx.gen_buckets_u64(torch.from_numpy(off.view(np.int64)).cuda())
    bb = mx.BatchBuild(off, block=block, grid=0, scope=0, seed=block, max_tries=16)
    bb.run(keys)
    torch.cuda.synchronize()
    res = bb.bucket_results()
    kh = keys.cpu().numpy().view(np.uint64)
    for b in range(len(sizes)):
        kb = kh[int(off[b]):int(off[b + 1])]
        rc, ref = o.mphf_build_u64(kb, seed=block, max_tries=16)
        case = f"bucket {b}: n={int(sizes[b])}"
        assert res[b]["status"] == rc, case
        assert res[b]["tries"] == ref["tries"] and res[b]["seed_used"] == ref["seed_used"], case
        if rc == 0:
            assert res[b]["n_rounds"] == ref["n_rounds"], case
            assert np.array_equal(bb.bucket_codes(b).cpu().numpy().view(np.uint64), ref["words"]), case
            assert np.array_equal(bb.bucket_rank(b).cpu().numpy().view(np.uint64), ref["rank"]), case
