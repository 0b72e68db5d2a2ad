"""MI355X (gfx950) MWHC build: hypergraph peeling and minimal perfect hashing.

After Belazzougui, Boldi, Ottaviano, Venturini, Vigna, "Cache-Oblivious Peeling of Random
Hypergraphs" (arXiv 1312.0526).  The work runs in the HIP kernels of libmphx.so behind the C
ABI of include/mphx.h; this package only marshals torch tensors and streams into that ABI.
"""
from ._lib import (  # noqa: F401
    BatchBuild, BatchTuning, Server, batch_clock, build_batch, gen_buckets_u64, ECANCELED, ECORE, EDEVICE, EDUP, EINVAL, ENOMEM, ERANGE, KEYS_STR, KEYS_U64, OK, ROUND_CORE, LIB_PATH, MphxError,
    check_bijection, gen_keys_u64, gen_str_keys, get_option, hash_str, hash_u64, lib, lookup_str, lookup_u64,
    mphf_build_str, mphf_build_u64, mphf_build_u64_static, mphf_workspace_bytes,
    mphf_build_stream_u64, stream_workspace_bytes, lookup_wide_u64, check_stream_u64, part_size, peel, peel_r, phase_times, set_option,
    PROBE_ATOMIC_ADD, PROBE_ATOMIC_ADD32, PROBE_ATOMIC_ADD_RET, PROBE_ATOMIC_ADD_WG, PROBE_LDS_ATOMIC_ADD, PROBE_LOAD8,
    PROBE_STORE1, probe_copy, probe_random,
    sf_bits, sf_build_str, sf_build_u64, sf_lookup_str, sf_lookup_u64, sf_words, sf_workspace_bytes,
    sfr_build_str, sfr_build_u64, sfr_lookup_str, sfr_lookup_u64, sfr_sizes,
    hem_build, hem_build_host, hem_capacity, hem_host_workspace_bytes, hem_lookup, hem_workspace_bytes,
)
