"""The golden digests of the full-size configurations (CPU only): well formed, and spot
recomputations with the oracle give the stored values (buckets of config 4 across the size
range, small requests of config 5)."""
import os
import sys

import numpy as np

import oracle
import workloads

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_fullsize as golden  # noqa: E402


def test_config4_digests_recompute():
    rows = golden.read_c4()
    assert sorted(rows) == list(range(65536))
    assert all(t >= 1 and r >= 1 and len(d) == 12 for t, r, d in rows.values())
    sizes = workloads.bucket_sizes(65536, 100, 1_000_000, seed=0)
    # retries are frequent only for small buckets (Section 3: one trial suffices at scale)
    small, large = sizes < 1000, sizes >= 100_000
    tries = np.array([rows[b][0] for b in range(65536)])
    assert tries[small].mean() > 1.5 and tries[large].mean() < 1.05
    o = oracle.Oracle()
    for b in (0, 1, int(np.argmin(sizes)), int(np.argsort(sizes)[len(sizes) // 2]), 65535):
        keys = workloads.u64_keys(int(sizes[b]), gen_seed=workloads.bucket_gen_seed(b))
        rc, ref = o.mphf_build_u64(keys, seed=0, max_tries=golden.MAX_TRIES)
        assert rc == 0
        assert rows[b] == (ref["tries"], ref["n_rounds"], golden.digest(ref["words"], ref["rank"])[:12]), b


def test_config5_digests_recompute():
    rows = golden.read_c5()
    sizes, kinds = golden.c5_plan()
    assert sorted(rows) == list(range(golden.C5_REQUESTS))
    assert [rows[i]["n"] for i in range(60)] == [int(x) for x in sizes]
    assert [rows[i]["kind"] for i in range(60)] == [int(x) for x in kinds]
    o = oracle.Oracle()
    small = [i for i in range(60) if sizes[i] <= 30_000][:4]
    assert small
    for i in small:
        n = int(sizes[i])
        if kinds[i] == 0:
            rc, ref = o.mphf_build_u64(workloads.u64_keys(n, gen_seed=7), seed=i)
        else:
            rc, ref = o.mphf_build_str(*workloads.str_keys(n, gen_seed=8), seed=i)
        assert rc == 0
        assert rows[i]["digest"] == golden.digest(ref["words"], ref["rank"]), i
        assert (rows[i]["seed_used"], rows[i]["tries"], rows[i]["n_rounds"]) == (ref["seed_used"], ref["tries"],
                                                                                  ref["n_rounds"]), i


def test_config3_digest_is_complete():
    g = golden.read_c3()
    n = 1 << 31
    P = oracle.Oracle().part_size(n)
    assert g["n"] == n and g["P"] == P
    assert g["code_words"] == (3 * P + 31) // 32 and g["rank_words"] == (3 * P + 511) // 512
    assert g["tries"] == g["seed_used"] + 1 >= 1 and 50 < g["n_rounds"] < 80
    assert len(g["codes_sha256"]) == 64 and len(g["rank_sha256"]) == 64
