"""The C-ABI library loads and exports every symbol include/mphx.h declares (CPU only; no
compute calls).  Argument errors are reported before any device work."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mphx.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"MPHX_API\s+[\w\s\*]+?\b(mphx_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def mx():
    import paper_1312_0526_amd as mx

    mx.lib()
    return mx


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("mphx_peel", "mphx_peel_workspace_bytes", "mphx_mphf_build_u64", "mphx_mphf_build_str",
                     "mphx_mphf_workspace_bytes", "mphx_mphf_lookup_u64", "mphx_last_error"):
        assert required in names


def test_every_declared_symbol_is_exported(mx):
    lib = C.CDLL(mx.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert missing == []


def test_binding_constants_match_the_header(mx):
    text = open(HEADER).read()
    defs = dict(re.findall(r"#define MPHX_((?:PROBE|KEYS)_\w+)\s+(\d+)", text))
    assert len(defs) >= 9
    for name, value in defs.items():
        assert getattr(mx, name) == int(value), name


def test_part_size_matches_oracle(mx):
    import oracle

    o = oracle.Oracle()
    for n in (0, 1, 2, 3, 1000, 10**6, 1 << 27, 1 << 31, (1 << 32) - 2):
        for g in ((123, 100), (120, 100), (1, 1), (7, 3)):
            assert mx.part_size(n, g) == o.part_size(n, *g)


def test_options_roundtrip(mx):
    old = mx.get_option("round_batch")
    mx.set_option("round_batch", 3)
    assert mx.get_option("round_batch") == 3
    mx.set_option("round_batch", old)
    with pytest.raises(mx.MphxError):
        mx.set_option("timing", 7)
    with pytest.raises(mx.MphxError):
        mx.set_option("no_such_option", 1)


@pytest.mark.parametrize("key,default,good,bad", [
    ("batch_lds", 1, 0, 2),
    ("part_build", 21, 1, 33),
    ("batch_sort_deletes", 4, 8, 1025),
    ("batch_claim_lists", 1, 0, 2),
    ("batch_clock", 0, 1, 2),
    ("hem_block", 1024, 256, 300),
    ("hem_grid", 0, 512, 1 << 17),
])
def test_batch_and_hem_options(mx, key, default, good, bad):
    assert mx.get_option(key) == default
    mx.set_option(key, good)
    try:
        assert mx.get_option(key) == good
        with pytest.raises(mx.MphxError):
            mx.set_option(key, bad)
        assert mx.get_option(key) == good  # a refused value changes nothing
    finally:
        mx.set_option(key, default)


def test_hem_workspaces_follow_k_range_and_shape(mx):
    # k outside [9, 20] has no workspace; the grid option sizes the batched scratch
    assert mx.hem_workspace_bytes(1 << 20, 8) == 0 and mx.hem_workspace_bytes(1 << 20, 21) == 0
    assert mx.hem_host_workspace_bytes(1 << 20, 21, mx.KEYS_U64, 1 << 16, 0, 1 << 18) == 0
    base = mx.hem_workspace_bytes(1 << 20, 12)
    assert base > 16 * (1 << 20)  # signatures and the partition's second buffer at least
    mx.set_option("hem_grid", 4096)
    try:
        assert mx.hem_workspace_bytes(1 << 20, 12) > base
    finally:
        mx.set_option("hem_grid", 0)
    # beyond 2^18 buckets the coarse offsets of the refinement come on top
    assert mx.hem_workspace_bytes(1 << 22, 19) > mx.hem_workspace_bytes(1 << 22, 18)
    # string keys' signature records are 16 bytes (the whole digest), u64 keys' 8: two arrays
    # of n records each
    n = 1 << 20
    diff = mx.hem_workspace_bytes(n, 12, kind=mx.KEYS_STR) - mx.hem_workspace_bytes(n, 12, kind=mx.KEYS_U64)
    assert diff == 2 * 8 * n
    assert mx.hem_workspace_bytes(n, 12, kind=7) == 0
    host_diff = (mx.hem_host_workspace_bytes(n, 12, mx.KEYS_STR, 1 << 16, 1 << 20, 1 << 18)
                 - mx.hem_host_workspace_bytes(n, 12, mx.KEYS_U64, 1 << 16, 0, 1 << 18))
    assert host_diff >= 8 * (n + (1 << 16) + 2 * (1 << 18))


def test_info_struct_mirrors_match_the_header(mx):
    # the C side asserts the same sizes (88 and 40 bytes)
    assert C.sizeof(mx._lib.MphfInfo) == 88 and C.sizeof(mx._lib.PeelInfo) == 40
    names = [f for f, _ in mx._lib.MphfInfo._fields_]
    assert names[-3:] == ["update_deletes", "update_records", "layer0"]


def test_list_cap_option(mx):
    assert mx.get_option("list_cap") == 0 and mx.get_option("list_fallbacks") == 0
    for bad in (("list_cap", -1), ("list_fallbacks", 1)):
        with pytest.raises(mx.MphxError):
            mx.set_option(*bad)
    mx.set_option("list_cap", 1000)
    try:
        assert mx.get_option("list_cap") == 1000
    finally:
        mx.set_option("list_cap", 0)


def test_static_function_sizes(mx):
    import oracle

    o = oracle.Oracle()
    for sigma in (1, 2, 3, 4, 255, 256, 257, 65_535, 65_536, 65_537, 1_000_003, (1 << 32) - 1, 1 << 32):
        assert mx.sf_bits(sigma) == o.sf_bits(sigma) == (sigma - 1).bit_length()
        assert mx.sf_words(12_345, sigma) == o.sf_words(3 * o.part_size(12_345), sigma)
        # ranked layout: m mark bits, one rank sample per 1024 vertices plus the total, n fields
        m = 3 * o.part_size(12_345)
        assert mx.sfr_sizes(12_345, sigma) == ((m + 63) // 64, int(o.lib.orc_sfr_rank_words(m)),
                                               (12_345 * mx.sf_bits(sigma) + 63) // 64)
    # without claim lists the values in layer order take n more u32; with them, the edge states
    assert mx.sf_workspace_bytes(1 << 20) - mx.mphf_workspace_bytes(1 << 20) >= 4 << 20
    old = mx.get_option("claim_lists")
    mx.set_option("claim_lists", 20)
    try:
        assert mx.sf_workspace_bytes(1 << 20) == mx.mphf_workspace_bytes(1 << 20)
    finally:
        mx.set_option("claim_lists", old)


def test_update_lists_option_range(mx):
    assert mx.get_option("update_lists") == 16
    for bad in (-1, 101):
        with pytest.raises(mx.MphxError):
            mx.set_option("update_lists", bad)
    mx.set_option("update_lists", 0)
    assert mx.get_option("update_lists") == 0
    mx.set_option("update_lists", 16)


def test_argument_errors_need_no_device(mx):
    lib = mx.lib()
    info = mx._lib.PeelInfo()
    # null workspace
    assert lib.mphx_peel(None, 10, 30, None, None, None, None, None, 0, None, C.byref(info)) == mx.EINVAL
    # n too large
    assert lib.mphx_peel(None, 1 << 32, 30, None, None, None, None, None, 0, None, C.byref(info)) == mx.EINVAL
    # workspace too small (a fake aligned pointer: rejected before use)
    assert lib.mphx_peel(C.c_void_p(4096), 10, 30, C.c_void_p(4096), C.c_void_p(4096), C.c_void_p(4096), None,
                         C.c_void_p(4096), 16, None, C.byref(info)) == mx.ENOMEM
    minfo = mx._lib.MphfInfo()
    assert lib.mphx_mphf_build_u64(None, 10, 0, 0, 100, 1, None, None, None, 0, None, C.byref(minfo)) == mx.EINVAL
    assert lib.mphx_mphf_build_u64(None, 10, 0, 123, 100, 0, None, None, None, 0, None, C.byref(minfo)) == mx.EINVAL
    msg = lib.mphx_last_error().decode()
    assert "max_tries" in msg


def test_workspace_sizes_scale_linearly(mx):
    # above 2^22 keys the per-round arrays stop growing; the slope is the per-key state:
    # edges 12n + records 8m + layer slots 12n + edge states 4n, m = 1.23n
    a = mx.mphf_workspace_bytes(1 << 23)
    b = mx.mphf_workspace_bytes(1 << 24)
    slope = (b - a) / (1 << 23)
    assert 37.5 < slope < 38.2


def test_batch_autotune_arguments_need_no_device(mx):
    lib = mx.lib()
    n = lib.mphx_batch_tuning_candidates(None, 0)
    arr = (mx.BatchTuning * n)()
    assert lib.mphx_batch_tuning_candidates(arr, n) == n == 5
    assert {a.block for a in arr} == {256, 512, 1024} and all(a.grid > 0 for a in arr)
    best, ms = C.c_uint32(7), (C.c_float * n)()

    def call(B=1, cands=arr, ncand=n, reps=1, keys=None, gnum=123):
        return lib.mphx_batch_autotune_u64(keys, None, None, B, 10, 0, gnum, 100, 8, None, None, None, None, None,
                                           None, 0, cands, ncand, reps, ms, C.byref(best), None)

    assert call(ncand=0) == mx.EINVAL
    assert call(cands=None) == mx.EINVAL
    assert call(reps=0) == mx.EINVAL and call(reps=101) == mx.EINVAL
    assert call(gnum=0) == mx.EINVAL
    bad = (mx.BatchTuning * 1)(mx.BatchTuning(300, 1, 0, 0))
    assert call(cands=bad, ncand=1) == mx.EINVAL
    assert call() == mx.EINVAL  # null keys and outputs for a non-empty batch
    assert call(B=0) == 0 and best.value == 0 and list(ms) == [0.0] * n


def test_stream_workspace_sizes(mx):
    n = 1 << 24
    base = mx.stream_workspace_bytes(n, chunk_keys=1 << 20, layer_slots=n)
    # 12 bytes per layer slot; records of 9 bytes per vertex
    assert mx.stream_workspace_bytes(n, chunk_keys=1 << 20, layer_slots=n // 2) == base - 12 * (n - n // 2) or \
        abs(mx.stream_workspace_bytes(n, chunk_keys=1 << 20, layer_slots=n // 2) - (base - 6 * n)) < 512
    m = 3 * mx.part_size(n)
    assert base > 9 * m + 12 * n
    # P above 2^32, zero keys or zero sizes: no workspace
    assert mx.stream_workspace_bytes(11_000_000_000) == 0
    assert mx.lib().mphx_stream_workspace_bytes(0, 123, 100, 1, 1) == 0
    assert mx.lib().mphx_stream_workspace_bytes(1000, 123, 100, 0, 1) == 0
    assert mx.lib().mphx_stream_workspace_bytes(10_000_000_000, 123, 100, 1 << 20, 1 << 20) > 0
