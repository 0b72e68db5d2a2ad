"""The oracle against facts outside itself (CPU only)."""
import numpy as np
import pytest

import oracle
import pins
import workloads


@pytest.fixture(scope="module")
def o():
    return oracle.Oracle()


@pytest.mark.parametrize("pin", pins.ALL_PINS + [pins.pin_threshold], ids=lambda p: p.__name__)
def test_pin(o, pin):
    assert pin(o) == []


def test_config1_oracle_build(o):
    """1,000,000 u64 keys from seed 0, gamma = 123/100: one try, full peel, bijection."""
    keys = workloads.u64_keys(1_000_000)
    rc, r = o.mphf_build_u64(keys, seed=0)
    assert rc == 0 and r["tries"] == 1 and r["P"] == 410_000
    f = o.lookup_u64(r["words"], r["rank"], r["P"], r["seed_used"], keys)
    assert np.array_equal(np.sort(f), np.arange(len(keys), dtype=np.uint64))
    edge0 = o.hash_u64(keys[:1], 0, r["P"])[0].tolist()
    assert keys[0] == pins.SPLITMIX0[0]
    assert all(k * r["P"] <= v < (k + 1) * r["P"] for k, v in enumerate(edge0))


def test_generator_definition():
    """The vectorised string generator equals the byte-by-byte definition."""
    data, offs = workloads.str_keys(2000, start=123)
    for j in (0, 1, 500, 1999):
        assert bytes(data[offs[j]:offs[j + 1]]) == workloads.str_key(123 + j)
    lens = np.diff(offs.astype(np.int64))
    assert lens.min() >= 8 and lens.max() <= 512
    assert len({bytes(data[offs[j]:offs[j + 1]]) for j in range(2000)}) == 2000
    q = workloads.quantile_table()
    assert abs(float(q.mean()) - 60.0) < 0.2
