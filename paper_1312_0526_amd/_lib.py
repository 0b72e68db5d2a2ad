"""ctypes binding of libmphx.so (include/mphx.h): argument marshalling only.

torch provides device memory and the current stream; every step of the path runs in the
library's HIP kernels.  There is no CPU fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # loads the HIP runtime first, so the library binds to the same one

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmphx.so")

OK, EINVAL, ERANGE, ENOMEM, EDEVICE, ECANCELED, ECORE, EDUP = 0, -1, -2, -3, -4, -5, 1, 2
ROUND_CORE = 0xFFFFFFFF
KEYS_U64, KEYS_STR = 0, 1
_NAMES = {EINVAL: "EINVAL", ERANGE: "ERANGE", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE", ECANCELED: "ECANCELED",
          ECORE: "ECORE", EDUP: "EDUP"}


class MphxError(RuntimeError):
    def __init__(self, status: int, message: str, info=None):
        super().__init__(f"{_NAMES.get(status, status)}: {message}")
        self.status = status
        self.info = info


class PeelInfo(C.Structure):
    _fields_ = [("n_peeled", C.c_uint64), ("n_rounds", C.c_uint32), ("reserved", C.c_uint32),
                ("frontier_total", C.c_uint64), ("claims", C.c_uint64), ("frontier0", C.c_uint64)]


class MphfInfo(C.Structure):
    _fields_ = [("P", C.c_uint64), ("m", C.c_uint64), ("seed_used", C.c_uint64), ("tries", C.c_uint32),
                ("n_rounds", C.c_uint32), ("n_core", C.c_uint64), ("frontier_total", C.c_uint64),
                ("claims", C.c_uint64), ("frontier0", C.c_uint64), ("update_deletes", C.c_uint64),
                ("update_records", C.c_uint64), ("layer0", C.c_uint64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_vp, _u64, _u32, _i32, _sz = C.c_void_p, C.c_uint64, C.c_uint32, C.c_int, C.c_size_t
_SIGS = {
    "mphx_last_error": (C.c_char_p, []),
    "mphx_part_size": (_u64, [_u64, _u32, _u32]),
    "mphx_peel_workspace_bytes": (_sz, [_u64, _u64]),
    "mphx_peel": (_i32, [_vp, _u64, _u64, _vp, _vp, _vp, _vp, _vp, _sz, _vp, C.POINTER(PeelInfo)]),
    "mphx_peel_r_workspace_bytes": (_sz, [_u64, _u64, _u32]),
    "mphx_peel_r": (_i32, [_vp, _u64, _u64, _u32, _vp, _vp, _vp, _vp, _vp, _sz, _vp, C.POINTER(PeelInfo)]),
    "mphx_mphf_workspace_bytes": (_sz, [_u64, _u32, _u32, _i32]),
    "mphx_mphf_build_u64": (_i32, [_vp, _u64, _u64, _u32, _u32, _u32, _vp, _vp, _vp, _sz, _vp, C.POINTER(MphfInfo)]),
    "mphx_mphf_build_str": (_i32, [_vp, _vp, _u64, _u64, _u32, _u32, _u32, _vp, _vp, _vp, _sz, _vp,
                                   C.POINTER(MphfInfo)]),
    "mphx_mphf_build_u64_static": (_i32, [_vp, _u64, _u64, _u32, _u32, _u32, _vp, _vp, _vp, C.POINTER(MphfInfo)]),
    "mphx_stream_workspace_bytes": (_sz, [_u64, _u32, _u32, _u64, _u64]),
    "mphx_mphf_build_stream_u64": (_i32, [_vp, _u64, _u64, _u32, _u32, _u32, _u64, _u64, _vp, _sz, _vp, _vp, _vp,
                                          _sz, _vp, C.POINTER(MphfInfo)]),
    "mphx_mphf_lookup_wide_u64": (_i32, [_vp, _vp, _u64, _u64, _vp, _u64, _vp, _vp]),
    "mphx_check_stream_workspace_bytes": (_sz, [_u64, _u64]),
    "mphx_check_stream_u64": (_i32, [_vp, _vp, _u64, _u64, _vp, _u64, _u64, _vp, _sz, _vp, C.POINTER(_u64)]),
    "mphx_sf_bits": (_u32, [_u64]),
    "mphx_sf_words": (_u64, [_u64, _u32, _u32, _u64]),
    "mphx_sf_workspace_bytes": (_sz, [_u64, _u32, _u32, _i32]),
    "mphx_sf_build_u64": (_i32, [_vp, _vp, _u64, _u64, _u64, _u32, _u32, _u32, _vp, _vp, _sz, _vp, C.POINTER(MphfInfo)]),
    "mphx_sf_build_str": (_i32, [_vp, _vp, _vp, _u64, _u64, _u64, _u32, _u32, _u32, _vp, _vp, _sz, _vp,
                                 C.POINTER(MphfInfo)]),
    "mphx_sf_lookup_u64": (_i32, [_vp, _u64, _u64, _u64, _vp, _u64, _vp, _vp]),
    "mphx_sf_lookup_str": (_i32, [_vp, _u64, _u64, _u64, _vp, _vp, _u64, _vp, _vp]),
    "mphx_sfr_mark_words": (_u64, [_u64, _u32, _u32]),
    "mphx_sfr_rank_words": (_u64, [_u64, _u32, _u32]),
    "mphx_sfr_val_words": (_u64, [_u64, _u64]),
    "mphx_sfr_build_u64": (_i32, [_vp, _vp, _u64, _u64, _u64, _u32, _u32, _u32, _vp, _vp, _vp, _vp, _sz, _vp,
                                  C.POINTER(MphfInfo)]),
    "mphx_sfr_build_str": (_i32, [_vp, _vp, _vp, _u64, _u64, _u64, _u32, _u32, _u32, _vp, _vp, _vp, _vp, _sz, _vp,
                                  C.POINTER(MphfInfo)]),
    "mphx_sfr_lookup_u64": (_i32, [_vp, _vp, _vp, _u64, _u64, _u64, _vp, _u64, _vp, _vp]),
    "mphx_sfr_lookup_str": (_i32, [_vp, _vp, _vp, _u64, _u64, _u64, _vp, _vp, _u64, _vp, _vp]),
    "mphx_hem_workspace_bytes": (_sz, [_u64, _u32, _u32, _u32, _i32]),
    "mphx_hem_capacity": (_i32, [_u64, _u32, _u32, _u32, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    "mphx_hem_build_u64": (_i32, [_vp, _u64, _u32, _u64, _u32, _u32, _u32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp,
                                  C.POINTER(MphfInfo)]),
    "mphx_hem_build_str": (_i32, [_vp, _vp, _u64, _u32, _u64, _u32, _u32, _u32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz,
                                  _vp, C.POINTER(MphfInfo)]),
    "mphx_hem_host_workspace_bytes": (_sz, [_u64, _u32, _u32, _u32, _i32, _u64, _u64, _u64]),
    "mphx_hem_build_host_u64": (_i32, [_vp, _u64, _u32, _u64, _u32, _u32, _u32, _u64, _u64, _vp, _vp, _vp, _vp, _vp,
                                       _vp, _vp, _sz, _vp, C.POINTER(MphfInfo)]),
    "mphx_hem_build_host_str": (_i32, [_vp, _vp, _u64, _u32, _u64, _u32, _u32, _u32, _u64, _u64, _u64, _vp, _vp, _vp,
                                       _vp, _vp, _vp, _vp, _sz, _vp, C.POINTER(MphfInfo)]),
    "mphx_hem_lookup_u64": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _u32, _u32, _u32, _u64, _vp, _u64, _vp, _vp]),
    "mphx_hem_lookup_str": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _u32, _u32, _u32, _u64, _vp, _vp, _u64, _vp, _vp]),
    "mphx_mphf_lookup_u64": (_i32, [_vp, _vp, _u64, _u64, _vp, _u64, _vp, _vp]),
    "mphx_mphf_lookup_str": (_i32, [_vp, _vp, _u64, _u64, _vp, _vp, _u64, _vp, _vp]),
    "mphx_hash_u64": (_i32, [_vp, _u64, _u64, _u64, _vp, _vp]),
    "mphx_hash_str": (_i32, [_vp, _vp, _u64, _u64, _u64, _vp, _vp]),
    "mphx_bijection_scratch_bytes": (_sz, [_u64]),
    "mphx_check_bijection": (_i32, [_vp, _u64, _vp, C.POINTER(C.c_uint64), _vp]),
    "mphx_gen_keys_u64": (_i32, [_vp, _u64, _u64, _u64, _vp]),
    "mphx_gen_str_lengths": (_i32, [_vp, _u64, _u64, _u64, _vp, _vp]),
    "mphx_scan_scratch_bytes": (_sz, [_u64]),
    "mphx_gen_str_offsets": (_i32, [_vp, _u64, _vp, _vp, _sz, _vp]),
    "mphx_gen_str_bytes": (_i32, [_vp, _vp, _u64, _u64, _u64, _vp]),
    "mphx_set_option": (_i32, [C.c_char_p, C.c_int64]),
    "mphx_get_option": (C.c_int64, [C.c_char_p]),
    "mphx_gen_buckets_u64": (_i32, [_vp, _vp, _u32, _vp]),
    "mphx_batch_layout": (_i32, [_vp, _u32, _u32, _u32, _vp, _vp, _vp, C.POINTER(C.c_uint64)]),
    "mphx_batch_workspace_bytes": (_sz, [_u32, _u64, _u32, _u32, _vp]),
    "mphx_build_batch_u64": (_i32, [_vp, _vp, _vp, _u32, _u64, _u64, _u32, _u32, _u32, _vp, _vp, _vp, _vp, _vp,
                                    _vp, _sz, _vp, _vp]),
    "mphx_graph_capture_batch_u64": (_i32, [_vp, _vp, _vp, _u32, _u64, _u64, _u32, _u32, _u32, _vp, _vp, _vp, _vp,
                                            _vp, _vp, _sz, _vp, C.POINTER(C.c_void_p)]),
    "mphx_batch_tuning_candidates": (_u32, [_vp, _u32]),
    "mphx_batch_autotune_u64": (_i32, [_vp, _vp, _vp, _u32, _u64, _u64, _u32, _u32, _u32, _vp, _vp, _vp, _vp, _vp,
                                       _vp, _sz, _vp, _u32, _u32, _vp, C.POINTER(C.c_uint32), _vp]),
    "mphx_batch_desc_workspace_bytes": (_sz, [_u64, _u32, _u32, _vp]),
    "mphx_build_batch": (_i32, [_vp, _u32, _vp, _u64, _u32, _u32, _u32, _vp, _sz, _vp, _vp]),
    "mphx_graph_launch": (_i32, [_vp, _vp]),
    "mphx_graph_destroy": (_i32, [_vp]),
    "mphx_server_create": (_i32, [_i32, _sz, _u32, _u64, C.POINTER(C.c_void_p)]),
    "mphx_server_submit": (_i32, [_vp, _vp, C.POINTER(C.c_uint64)]),
    "mphx_server_poll": (_i32, [_vp, _u64, _vp]),
    "mphx_server_wait": (_i32, [_vp, _u64, _vp]),
    "mphx_server_stats": (_i32, [_vp, _vp]),
    "mphx_server_clock": (C.c_double, []),
    "mphx_server_destroy": (_i32, [_vp]),
    "mphx_phase_times": (_i32, [C.POINTER(C.c_double), C.POINTER(C.c_uint64), _i32, _i32]),
    "mphx_phase_name": (C.c_char_p, [_i32]),
    "mphx_batch_clock": (_i32, [C.POINTER(C.c_uint64), _i32, _i32]),
    "mphx_batch_clock_name": (C.c_char_p, [_i32]),
    "mphx_probe_copy": (_i32, [_vp, _vp, _u64, _u32, _vp]),
    "mphx_probe_random": (_i32, [_i32, _vp, _u64, _u64, _u64, _u32, _u32, _vp]),
}

_lib = None


def lib():
    """The loaded library; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1312_0526_amd.build`")
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


def _err(status, info=None):
    msg = lib().mphx_last_error().decode(errors="replace")
    raise MphxError(status, msg, info)


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _check(t, dtype, name, numel=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")


def _workspace(nbytes: int, device) -> torch.Tensor:
    # torch's caching allocator returns 512-byte aligned blocks
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


# ------------------------------------------------------------------------------------------
def set_option(key: str, value: int) -> None:
    rc = lib().mphx_set_option(key.encode(), int(value))
    if rc:
        _err(rc)


def get_option(key: str) -> int:
    return int(lib().mphx_get_option(key.encode()))


def phase_times(reset: bool = False) -> dict:
    """Accumulated per-phase kernel time (ms) and launch counts (needs option timing=1)."""
    ms = (C.c_double * 16)()
    cnt = (C.c_uint64 * 16)()
    k = lib().mphx_phase_times(ms, cnt, 16, int(reset))
    return {lib().mphx_phase_name(i).decode(): (float(ms[i]), int(cnt[i])) for i in range(k)}


def batch_clock(reset: bool = False) -> dict:
    """The current device's batch clock (launches made with option batch_clock=1): entry name ->
    value; "tick_hz" is the tick rate, phase entries are ticks summed over workgroups."""
    out = (C.c_uint64 * 64)()
    k = lib().mphx_batch_clock(out, 64, int(reset))
    if k < 0:
        _err(k)
    return {lib().mphx_batch_clock_name(i).decode(): int(out[i]) for i in range(min(k, 64))}


def part_size(n: int, gamma=(123, 100)) -> int:
    return int(lib().mphx_part_size(n, gamma[0], gamma[1]))


def peel(edges: torch.Tensor, m: int, with_hinge: bool = True) -> dict:
    """Layered peel of an n x 3 uint32 edge list (device).  Returns device tensors
    order/round (int32 views of uint32 data), core_mask/hinge (uint8) and host counts."""
    if edges.dim() != 2 or edges.shape[1] != 3:
        raise ValueError("edges must be n x 3")
    _check(edges, torch.int32, "edges")
    n = edges.shape[0]
    dev = edges.device
    order = torch.empty(n, dtype=torch.int32, device=dev)
    rnd = torch.empty(n, dtype=torch.int32, device=dev)
    core = torch.empty(n, dtype=torch.uint8, device=dev)
    hinge = torch.empty(n, dtype=torch.uint8, device=dev) if with_hinge else None
    ws = _workspace(lib().mphx_peel_workspace_bytes(n, m), dev)
    info = PeelInfo()
    rc = lib().mphx_peel(_ptr(edges), n, m, _ptr(order), _ptr(rnd), _ptr(core), _ptr(hinge), _ptr(ws), ws.numel(),
                         _stream(dev), C.byref(info))
    if rc:
        _err(rc)
    return dict(order=order, round=rnd, core_mask=core, hinge=hinge, n_peeled=int(info.n_peeled),
                n_rounds=int(info.n_rounds), frontier_total=int(info.frontier_total), claims=int(info.claims),
                frontier0=int(info.frontier0))


def peel_r(edges: torch.Tensor, m: int, with_hinge: bool = True) -> dict:
    """Layered peel of an n x r uint32 edge list (device), 2 <= r <= 8; outputs as peel."""
    if edges.dim() != 2 or not 2 <= edges.shape[1] <= 8:
        raise ValueError("edges must be n x r with 2 <= r <= 8")
    _check(edges, torch.int32, "edges")
    n, r = edges.shape
    dev = edges.device
    order = torch.empty(n, dtype=torch.int32, device=dev)
    rnd = torch.empty(n, dtype=torch.int32, device=dev)
    core = torch.empty(n, dtype=torch.uint8, device=dev)
    hinge = torch.empty(n, dtype=torch.uint8, device=dev) if with_hinge else None
    ws = _workspace(lib().mphx_peel_r_workspace_bytes(n, m, r), dev)
    info = PeelInfo()
    rc = lib().mphx_peel_r(_ptr(edges), n, m, r, _ptr(order), _ptr(rnd), _ptr(core), _ptr(hinge), _ptr(ws),
                           ws.numel(), _stream(dev), C.byref(info))
    if rc:
        _err(rc)
    return dict(order=order, round=rnd, core_mask=core, hinge=hinge, n_peeled=int(info.n_peeled),
                n_rounds=int(info.n_rounds), frontier_total=int(info.frontier_total), claims=int(info.claims),
                frontier0=int(info.frontier0))


def _mphf_outputs(n, gamma, kind, dev, ws, out):
    P = part_size(n, gamma)
    m = 3 * P
    if out is None:
        codes = torch.empty(max((m + 31) // 32, 1), dtype=torch.int64, device=dev)
        rank = torch.empty(max((m + 511) // 512, 1), dtype=torch.int64, device=dev)
    else:
        codes, rank = out
        _check(codes, torch.int64, "codes")
        _check(rank, torch.int64, "rank")
        if codes.numel() < (m + 31) // 32 or rank.numel() < (m + 511) // 512:
            raise ValueError("output buffers too small")
    if ws is None:
        ws = _workspace(lib().mphx_mphf_workspace_bytes(n, gamma[0], gamma[1], kind), dev)
    return P, m, codes, rank, ws


def _result(codes, rank, info, m):
    d = info.as_dict()
    d["codes"] = codes[: (m + 31) // 32]
    d["rank"] = rank[: (m + 511) // 512]
    return d


def mphf_build_u64(keys: torch.Tensor, seed: int = 0, gamma=(123, 100), max_tries: int = 64, ws=None,
                   out=None) -> dict:
    """Build an MPHF of u64 keys (int64 view).  ws / out=(codes, rank) may be preallocated."""
    _check(keys, torch.int64, "keys")
    n = keys.numel()
    P, m, codes, rank, ws = _mphf_outputs(n, gamma, KEYS_U64, keys.device, ws, out)
    info = MphfInfo()
    rc = lib().mphx_mphf_build_u64(_ptr(keys), n, seed, gamma[0], gamma[1], max_tries, _ptr(codes), _ptr(rank),
                                   _ptr(ws), ws.numel(), _stream(keys.device), C.byref(info))
    if rc:
        _err(rc, info.as_dict())
    return _result(codes, rank, info, m)


def mphf_build_u64_static(keys: torch.Tensor, out, seed: int = 0, gamma=(123, 100), max_tries: int = 64) -> dict:
    """mphf_build_u64 through the allocation-free entry point: the library's own static device
    workspace (128 MiB per device), outputs out=(codes, rank) passed by the caller; nothing is
    allocated on the call."""
    _check(keys, torch.int64, "keys")
    n = keys.numel()
    m = 3 * part_size(n, gamma)
    codes, rank = out
    _check(codes, torch.int64, "codes")
    _check(rank, torch.int64, "rank")
    if codes.numel() < (m + 31) // 32 or rank.numel() < (m + 511) // 512:
        raise ValueError("output buffers too small")
    info = MphfInfo()
    rc = lib().mphx_mphf_build_u64_static(_ptr(keys), n, seed, gamma[0], gamma[1], max_tries, _ptr(codes), _ptr(rank),
                                          _stream(keys.device), C.byref(info))
    if rc:
        _err(rc, info.as_dict())
    return _result(codes, rank, info, m)


def stream_workspace_bytes(n: int, gamma=(123, 100), chunk_keys: int = 1 << 26, layer_slots: int = 0) -> int:
    return int(lib().mphx_stream_workspace_bytes(n, gamma[0], gamma[1], chunk_keys, layer_slots or n))


def mphf_build_stream_u64(keys: torch.Tensor, seed: int = 0, gamma=(123, 100), max_tries: int = 64,
                          chunk_keys: int = 1 << 26, layer_slots: int = 0, host_layers=None, ws=None, out=None,
                          device="cuda") -> dict:
    """MWHC MPHF of u64 keys held in host memory (a CPU int64 tensor), built by the streamed
    path: the device holds the vertex records and layer_slots layer slots (0 = n: every layer
    on the device); with fewer, the layers go to host_layers (a CPU uint8 tensor of 12 n bytes,
    allocated here when not given).  Outputs equal mphf_build_u64's."""
    _check_host(keys, torch.int64, "keys")
    dev = torch.device(device)
    n = keys.numel()
    layer_slots = layer_slots or n
    P = part_size(n, gamma)
    m = 3 * P
    if out is None:
        codes = torch.empty(max((m + 31) // 32, 1), dtype=torch.int64, device=dev)
        rank = torch.empty(max((m + 511) // 512, 1), dtype=torch.int64, device=dev)
    else:
        codes, rank = out
    if layer_slots < n and host_layers is None:
        host_layers = torch.empty(12 * n, dtype=torch.uint8)
    if host_layers is not None:
        _check_host(host_layers, torch.uint8, "host_layers")
    need = stream_workspace_bytes(n, gamma, chunk_keys, layer_slots)
    if need == 0:
        raise ValueError("bad n, gamma, chunk_keys or layer_slots")
    ws = ws if ws is not None else _workspace(need, dev)
    info = MphfInfo()
    rc = lib().mphx_mphf_build_stream_u64(_ptr(keys), n, seed, gamma[0], gamma[1], max_tries, chunk_keys, layer_slots,
                                          _ptr(host_layers) if host_layers is not None else None,
                                          host_layers.numel() if host_layers is not None else 0, _ptr(codes),
                                          _ptr(rank), _ptr(ws), ws.numel(), _stream(dev), C.byref(info))
    if rc:
        _err(rc, info.as_dict())
    return _result(codes, rank, info, m)


def lookup_wide_u64(codes, rank, P: int, seed: int, keys: torch.Tensor, out=None) -> torch.Tensor:
    """MPHF values of device keys for any P <= 2^32 (vertex positions beyond 2^32)."""
    _check(keys, torch.int64, "keys")
    if out is None:
        out = torch.empty(keys.numel(), dtype=torch.int64, device=keys.device)
    rc = lib().mphx_mphf_lookup_wide_u64(_ptr(codes), _ptr(rank), P, seed, _ptr(keys), keys.numel(), _ptr(out),
                                         _stream(keys.device))
    if rc:
        _err(rc)
    return out


def check_stream_u64(codes, rank, P: int, seed: int, keys: torch.Tensor, chunk_keys: int = 1 << 26) -> int:
    """Values of host keys (CPU int64 tensor) that are >= n or repeated: 0 for a bijection."""
    _check_host(keys, torch.int64, "keys")
    n = keys.numel()
    ws = _workspace(int(lib().mphx_check_stream_workspace_bytes(n, chunk_keys)), codes.device)
    bad = C.c_uint64(0)
    rc = lib().mphx_check_stream_u64(_ptr(codes), _ptr(rank), P, seed, _ptr(keys), n, chunk_keys, _ptr(ws), ws.numel(),
                                     _stream(codes.device), C.byref(bad))
    if rc:
        _err(rc)
    return int(bad.value)


def mphf_build_str(data: torch.Tensor, offs: torch.Tensor, seed: int = 0, gamma=(123, 100), max_tries: int = 64,
                   ws=None, out=None) -> dict:
    """Build an MPHF of byte-string keys (data + n+1 offsets).  ws / out may be preallocated."""
    _check(data, torch.uint8, "data")
    _check(offs, torch.int64, "offs")
    n = offs.numel() - 1
    P, m, codes, rank, ws = _mphf_outputs(n, gamma, KEYS_STR, data.device, ws, out)
    info = MphfInfo()
    rc = lib().mphx_mphf_build_str(_ptr(data), _ptr(offs), n, seed, gamma[0], gamma[1], max_tries, _ptr(codes),
                                   _ptr(rank), _ptr(ws), ws.numel(), _stream(data.device), C.byref(info))
    if rc:
        _err(rc, info.as_dict())
    return _result(codes, rank, info, m)


def mphf_workspace_bytes(n: int, gamma=(123, 100), kind: int = KEYS_U64) -> int:
    return int(lib().mphx_mphf_workspace_bytes(n, gamma[0], gamma[1], kind))


def lookup_u64(codes, rank, P: int, seed: int, keys: torch.Tensor, out=None) -> torch.Tensor:
    """MPHF values of keys; out (int64, one per key) may be preallocated."""
    _check(keys, torch.int64, "keys")
    if out is None:
        out = torch.empty(keys.numel(), dtype=torch.int64, device=keys.device)
    _check(out, torch.int64, "out", keys.numel())
    rc = lib().mphx_mphf_lookup_u64(_ptr(codes), _ptr(rank), P, seed, _ptr(keys), keys.numel(), _ptr(out),
                                    _stream(keys.device))
    if rc:
        _err(rc)
    return out


def lookup_str(codes, rank, P: int, seed: int, data: torch.Tensor, offs: torch.Tensor, out=None) -> torch.Tensor:
    """MPHF values of the string keys data[offs[i]:offs[i+1]] (offs may be a slice of a larger
    offset array: offsets are absolute in data); out may be preallocated."""
    _check(data, torch.uint8, "data")
    _check(offs, torch.int64, "offs")
    n = offs.numel() - 1
    if out is None:
        out = torch.empty(n, dtype=torch.int64, device=data.device)
    _check(out, torch.int64, "out", n)
    rc = lib().mphx_mphf_lookup_str(_ptr(codes), _ptr(rank), P, seed, _ptr(data), _ptr(offs), n, _ptr(out),
                                    _stream(data.device))
    if rc:
        _err(rc)
    return out


# ---- HEM split (Section 3: signatures, 2^k buckets, an MPHF per bucket) -------------------------
def hem_workspace_bytes(n: int, k: int, gamma=(123, 100), kind: int = KEYS_U64) -> int:
    return int(lib().mphx_hem_workspace_bytes(n, k, gamma[0], gamma[1], kind))


def hem_capacity(n: int, k: int, gamma=(123, 100)):
    cw, rw = C.c_uint64(), C.c_uint64()
    rc = lib().mphx_hem_capacity(n, k, gamma[0], gamma[1], C.byref(cw), C.byref(rw))
    if rc:
        _err(rc)
    return int(cw.value), int(rw.value)


def hem_build(keys=None, data=None, offs=None, k: int = 15, seed: int = 0, gamma=(123, 100), max_tries: int = 64,
              ws=None) -> dict:
    """HEM split of u64 keys (keys) or string keys (data + offs).  Returns device tables
    (bucket_off, code_off, rank_off, seeds, codes, rank) and the build info."""
    if keys is not None:
        _check(keys, torch.int64, "keys")
        n, dev = keys.numel(), keys.device
    else:
        _check(data, torch.uint8, "data")
        _check(offs, torch.int64, "offs")
        n, dev = offs.numel() - 1, data.device
    B = 1 << k
    cw, rw = hem_capacity(n, k, gamma)
    t = {name: torch.empty(B + 1, dtype=torch.int64, device=dev) for name in ("bucket_off", "code_off", "rank_off")}
    t["seeds"] = torch.empty(B, dtype=torch.int64, device=dev)
    codes = torch.empty(max(cw, 1), dtype=torch.int64, device=dev)
    rank = torch.empty(max(rw, 1), dtype=torch.int64, device=dev)
    kind = KEYS_U64 if keys is not None else KEYS_STR
    ws = ws if ws is not None else _workspace(hem_workspace_bytes(n, k, gamma, kind), dev)
    info = MphfInfo()
    common = (_ptr(t["bucket_off"]), _ptr(t["code_off"]), _ptr(t["rank_off"]), _ptr(t["seeds"]), _ptr(codes),
              _ptr(rank), _ptr(ws), ws.numel(), _stream(dev), C.byref(info))
    if keys is not None:
        rc = lib().mphx_hem_build_u64(_ptr(keys), n, k, seed, gamma[0], gamma[1], max_tries, *common)
    else:
        rc = lib().mphx_hem_build_str(_ptr(data), _ptr(offs), n, k, seed, gamma[0], gamma[1], max_tries, *common)
    if rc:
        _err(rc, info.as_dict())
    d = info.as_dict()
    nc = int(t["code_off"][-1].item())
    nr = int(t["rank_off"][-1].item())
    d.update(t, codes=codes[:nc], rank=rank[:nr], k=k, seed=seed, gamma=gamma, n=n)
    return d


def _check_host(t, dtype, name):
    if not isinstance(t, torch.Tensor) or t.is_cuda:
        raise TypeError(f"{name} must be a host (CPU) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def hem_host_workspace_bytes(n: int, k: int, kind: int, chunk_keys: int, chunk_bytes: int = 0, batch_keys: int = 0,
                             gamma=(123, 100)) -> int:
    return int(lib().mphx_hem_host_workspace_bytes(n, k, gamma[0], gamma[1], kind, chunk_keys, chunk_bytes,
                                                   batch_keys))


def hem_build_host(keys=None, data=None, offs=None, k: int = 15, seed: int = 0, gamma=(123, 100), max_tries: int = 64,
                   chunk_keys: int = 1 << 26, chunk_bytes: int = 1 << 30, batch_keys: int = 1 << 28, ws=None,
                   device="cuda") -> dict:
    """HEM split of keys held in host memory (CPU tensors, pinned for the full PCIe rate): u64
    keys (keys) or string keys (data + offs).  The device tables equal hem_build's."""
    dev = torch.device(device)
    if keys is not None:
        _check_host(keys, torch.int64, "keys")
        n, kind = keys.numel(), KEYS_U64
    else:
        _check_host(data, torch.uint8, "data")
        _check_host(offs, torch.int64, "offs")
        n, kind = offs.numel() - 1, KEYS_STR
    B = 1 << k
    cw, rw = hem_capacity(n, k, gamma)
    t = {name: torch.empty(B + 1, dtype=torch.int64, device=dev) for name in ("bucket_off", "code_off", "rank_off")}
    t["seeds"] = torch.empty(B, dtype=torch.int64, device=dev)
    codes = torch.empty(max(cw, 1), dtype=torch.int64, device=dev)
    rank = torch.empty(max(rw, 1), dtype=torch.int64, device=dev)
    need = hem_host_workspace_bytes(n, k, kind, chunk_keys, chunk_bytes, batch_keys, gamma)
    if need == 0:
        raise ValueError("bad k, gamma, chunk or batch size")
    ws = ws if ws is not None else _workspace(need, dev)
    info = MphfInfo()
    common = (_ptr(t["bucket_off"]), _ptr(t["code_off"]), _ptr(t["rank_off"]), _ptr(t["seeds"]), _ptr(codes),
              _ptr(rank), _ptr(ws), ws.numel(), _stream(dev), C.byref(info))
    if keys is not None:
        rc = lib().mphx_hem_build_host_u64(_ptr(keys), n, k, seed, gamma[0], gamma[1], max_tries, chunk_keys,
                                           batch_keys, *common)
    else:
        rc = lib().mphx_hem_build_host_str(_ptr(data), _ptr(offs), n, k, seed, gamma[0], gamma[1], max_tries,
                                           chunk_keys, chunk_bytes, batch_keys, *common)
    if rc:
        _err(rc, info.as_dict())
    d = info.as_dict()
    nc = int(t["code_off"][-1].item())
    nr = int(t["rank_off"][-1].item())
    d.update(t, codes=codes[:nc], rank=rank[:nr], k=k, seed=seed, gamma=gamma, n=n)
    return d


def hem_lookup(h: dict, keys=None, data=None, offs=None, out=None) -> torch.Tensor:
    if keys is not None:
        _check(keys, torch.int64, "keys")
        n, dev = keys.numel(), keys.device
    else:
        _check(data, torch.uint8, "data")
        _check(offs, torch.int64, "offs")
        n, dev = offs.numel() - 1, data.device
    if out is None:
        out = torch.empty(n, dtype=torch.int64, device=dev)
    _check(out, torch.int64, "out", n)
    codes = h["codes"] if h["codes"].numel() else h["bucket_off"]
    rank = h["rank"] if h["rank"].numel() else h["bucket_off"]
    tables = (_ptr(h["bucket_off"]), _ptr(h["code_off"]), _ptr(h["rank_off"]), _ptr(h["seeds"]), _ptr(codes),
              _ptr(rank), h["k"], h["gamma"][0], h["gamma"][1], h["seed"])
    if keys is not None:
        rc = lib().mphx_hem_lookup_u64(*tables, _ptr(keys), n, _ptr(out), _stream(dev))
    else:
        rc = lib().mphx_hem_lookup_str(*tables, _ptr(data), _ptr(offs), n, _ptr(out), _stream(dev))
    if rc:
        _err(rc)
    return out


# ---- static functions (Section 3: f(x) = u[v0] + u[v1] + u[v2] mod sigma) ----------------------
def sf_bits(sigma: int) -> int:
    return int(lib().mphx_sf_bits(sigma))


def sf_words(n: int, sigma: int, gamma=(123, 100)) -> int:
    return int(lib().mphx_sf_words(n, gamma[0], gamma[1], sigma))


def sf_workspace_bytes(n: int, gamma=(123, 100), kind: int = KEYS_U64) -> int:
    return int(lib().mphx_sf_workspace_bytes(n, gamma[0], gamma[1], kind))


def _sf_finish(rc, info, words):
    if rc:
        _err(rc, info.as_dict())
    d = info.as_dict()
    d["words"] = words
    return d


def sf_build_u64(keys: torch.Tensor, values: torch.Tensor, sigma: int, seed: int = 0, gamma=(123, 100),
                 max_tries: int = 64, ws=None, words=None) -> dict:
    """Static function of u64 keys: values (int32 tensor holding uint32 values, one per key,
    each below sigma).  Returns info and the packed fields (int64 tensor of uint64 words)."""
    _check(keys, torch.int64, "keys")
    n = keys.numel()
    _check(values, torch.int32, "values", n)
    nw = sf_words(n, sigma, gamma)
    if words is None:
        words = torch.empty(max(nw, 1), dtype=torch.int64, device=keys.device)
    ws = ws if ws is not None else _workspace(sf_workspace_bytes(n, gamma, KEYS_U64), keys.device)
    info = MphfInfo()
    rc = lib().mphx_sf_build_u64(_ptr(keys), _ptr(values), n, sigma, seed, gamma[0], gamma[1], max_tries,
                                 _ptr(words), _ptr(ws), ws.numel(), _stream(keys.device), C.byref(info))
    return _sf_finish(rc, info, words[:nw])


def sf_build_str(data: torch.Tensor, offs: torch.Tensor, values: torch.Tensor, sigma: int, seed: int = 0,
                 gamma=(123, 100), max_tries: int = 64, ws=None, words=None) -> dict:
    _check(data, torch.uint8, "data")
    _check(offs, torch.int64, "offs")
    n = offs.numel() - 1
    _check(values, torch.int32, "values", n)
    nw = sf_words(n, sigma, gamma)
    if words is None:
        words = torch.empty(max(nw, 1), dtype=torch.int64, device=data.device)
    ws = ws if ws is not None else _workspace(sf_workspace_bytes(n, gamma, KEYS_STR), data.device)
    info = MphfInfo()
    rc = lib().mphx_sf_build_str(_ptr(data), _ptr(offs), _ptr(values), n, sigma, seed, gamma[0], gamma[1],
                                 max_tries, _ptr(words), _ptr(ws), ws.numel(), _stream(data.device), C.byref(info))
    return _sf_finish(rc, info, words[:nw])


def sf_lookup_u64(words, sigma: int, P: int, seed: int, keys: torch.Tensor, out=None) -> torch.Tensor:
    _check(keys, torch.int64, "keys")
    if out is None:
        out = torch.empty(keys.numel(), dtype=torch.int64, device=keys.device)
    _check(out, torch.int64, "out", keys.numel())
    rc = lib().mphx_sf_lookup_u64(_ptr(words) if words.numel() else None, sigma, P, seed, _ptr(keys), keys.numel(),
                                  _ptr(out), _stream(keys.device))
    if rc:
        _err(rc)
    return out


def sf_lookup_str(words, sigma: int, P: int, seed: int, data: torch.Tensor, offs: torch.Tensor, out=None) -> torch.Tensor:
    _check(data, torch.uint8, "data")
    _check(offs, torch.int64, "offs")
    n = offs.numel() - 1
    if out is None:
        out = torch.empty(n, dtype=torch.int64, device=data.device)
    _check(out, torch.int64, "out", n)
    rc = lib().mphx_sf_lookup_str(_ptr(words) if words.numel() else None, sigma, P, seed, _ptr(data), _ptr(offs), n,
                                  _ptr(out), _stream(data.device))
    if rc:
        _err(rc)
    return out


# ---- static functions in the ranked layout (Section 3: a ranking structure over the values) -----
def sfr_sizes(n: int, sigma: int, gamma=(123, 100)) -> tuple:
    """Words of the marks, the rank samples and the fields (capacity for n fields)."""
    L = lib()
    return (int(L.mphx_sfr_mark_words(n, gamma[0], gamma[1])), int(L.mphx_sfr_rank_words(n, gamma[0], gamma[1])),
            int(L.mphx_sfr_val_words(n, sigma)))


def _sfr_outputs(n, sigma, gamma, device, out):
    if out is not None:
        return out
    return tuple(torch.empty(max(w, 1), dtype=torch.int64, device=device) for w in sfr_sizes(n, sigma, gamma))


def _sfr_finish(rc, info, n, sigma, gamma, outs):
    if rc:
        _err(rc, info.as_dict())
    d = info.as_dict()
    nm, nr, nv = sfr_sizes(n, sigma, gamma)
    d["marks"], d["rank"], d["vals"] = outs[0][:nm], outs[1][:nr], outs[2][:nv]
    return d


def sfr_build_u64(keys: torch.Tensor, values: torch.Tensor, sigma: int, seed: int = 0, gamma=(123, 100),
                  max_tries: int = 64, ws=None, out=None) -> dict:
    """Static function of u64 keys in the ranked layout.  Returns info and the marks, the rank
    samples (the last one is the number of fields) and the fields (int64 tensors of uint64
    words); out = (marks, rank, vals) to reuse buffers."""
    _check(keys, torch.int64, "keys")
    n = keys.numel()
    _check(values, torch.int32, "values", n)
    outs = _sfr_outputs(n, sigma, gamma, keys.device, out)
    ws = ws if ws is not None else _workspace(sf_workspace_bytes(n, gamma, KEYS_U64), keys.device)
    info = MphfInfo()
    rc = lib().mphx_sfr_build_u64(_ptr(keys), _ptr(values), n, sigma, seed, gamma[0], gamma[1], max_tries,
                                  *(_ptr(t) for t in outs), _ptr(ws), ws.numel(), _stream(keys.device), C.byref(info))
    return _sfr_finish(rc, info, n, sigma, gamma, outs)


def sfr_build_str(data: torch.Tensor, offs: torch.Tensor, values: torch.Tensor, sigma: int, seed: int = 0,
                  gamma=(123, 100), max_tries: int = 64, ws=None, out=None) -> dict:
    _check(data, torch.uint8, "data")
    _check(offs, torch.int64, "offs")
    n = offs.numel() - 1
    _check(values, torch.int32, "values", n)
    outs = _sfr_outputs(n, sigma, gamma, data.device, out)
    ws = ws if ws is not None else _workspace(sf_workspace_bytes(n, gamma, KEYS_STR), data.device)
    info = MphfInfo()
    rc = lib().mphx_sfr_build_str(_ptr(data), _ptr(offs), _ptr(values), n, sigma, seed, gamma[0], gamma[1],
                                  max_tries, *(_ptr(t) for t in outs), _ptr(ws), ws.numel(), _stream(data.device),
                                  C.byref(info))
    return _sfr_finish(rc, info, n, sigma, gamma, outs)


def sfr_lookup_u64(r: dict, sigma: int, keys: torch.Tensor, out=None) -> torch.Tensor:
    """f(key) for every key through the ranked layout r (a dict from sfr_build_*)."""
    _check(keys, torch.int64, "keys")
    if out is None:
        out = torch.empty(keys.numel(), dtype=torch.int64, device=keys.device)
    _check(out, torch.int64, "out", keys.numel())
    vals = r["vals"]
    rc = lib().mphx_sfr_lookup_u64(_ptr(r["marks"]), _ptr(r["rank"]), _ptr(vals) if vals.numel() else None, sigma,
                                   r["P"], r["seed_used"], _ptr(keys), keys.numel(), _ptr(out), _stream(keys.device))
    if rc:
        _err(rc)
    return out


def sfr_lookup_str(r: dict, sigma: int, data: torch.Tensor, offs: torch.Tensor, out=None) -> torch.Tensor:
    _check(data, torch.uint8, "data")
    _check(offs, torch.int64, "offs")
    n = offs.numel() - 1
    if out is None:
        out = torch.empty(n, dtype=torch.int64, device=data.device)
    _check(out, torch.int64, "out", n)
    vals = r["vals"]
    rc = lib().mphx_sfr_lookup_str(_ptr(r["marks"]), _ptr(r["rank"]), _ptr(vals) if vals.numel() else None, sigma,
                                   r["P"], r["seed_used"], _ptr(data), _ptr(offs), n, _ptr(out), _stream(data.device))
    if rc:
        _err(rc)
    return out


def hash_u64(keys: torch.Tensor, seed: int, P: int) -> torch.Tensor:
    _check(keys, torch.int64, "keys")
    edges = torch.empty((keys.numel(), 3), dtype=torch.int32, device=keys.device)
    rc = lib().mphx_hash_u64(_ptr(keys), keys.numel(), seed, P, _ptr(edges), _stream(keys.device))
    if rc:
        _err(rc)
    return edges


def hash_str(data: torch.Tensor, offs: torch.Tensor, seed: int, P: int) -> torch.Tensor:
    _check(data, torch.uint8, "data")
    _check(offs, torch.int64, "offs")
    n = offs.numel() - 1
    edges = torch.empty((n, 3), dtype=torch.int32, device=data.device)
    rc = lib().mphx_hash_str(_ptr(data), _ptr(offs), n, seed, P, _ptr(edges), _stream(data.device))
    if rc:
        _err(rc)
    return edges


def check_bijection(vals: torch.Tensor) -> int:
    _check(vals, torch.int64, "vals")
    n = vals.numel()
    scratch = _workspace(lib().mphx_bijection_scratch_bytes(n), vals.device)
    bad = C.c_uint64(0)
    rc = lib().mphx_check_bijection(_ptr(vals), n, _ptr(scratch), C.byref(bad), _stream(vals.device))
    if rc:
        _err(rc)
    return int(bad.value)


PROBE_ATOMIC_ADD, PROBE_ATOMIC_ADD_RET, PROBE_LOAD8, PROBE_STORE1, PROBE_LDS_ATOMIC_ADD = 1, 2, 3, 4, 5
PROBE_ATOMIC_ADD32, PROBE_ATOMIC_ADD_WG = 6, 7


def probe_copy(src: torch.Tensor, dst: torch.Tensor, grid: int = 0):
    """Streaming copy of src's bytes into dst (the practical HBM ceiling)."""
    nbytes = src.numel() * src.element_size()
    if not (src.is_cuda and dst.is_cuda) or dst.numel() * dst.element_size() < nbytes:
        raise ValueError("probe_copy needs two device tensors, dst at least as large as src")
    rc = lib().mphx_probe_copy(_ptr(src), _ptr(dst), nbytes, grid, _stream(src.device))
    if rc:
        _err(rc)


def probe_random(op: int, table: torch.Tensor, slots: int, count: int, seed: int = 0, grid: int = 0,
                 block: int = 256):
    """`count` random operations of kind `op` over `slots` entries of `table` (see mphx.h)."""
    if not table.is_cuda:
        raise TypeError("table must be a device tensor")
    rc = lib().mphx_probe_random(op, _ptr(table), slots, count, seed, grid, block, _stream(table.device))
    if rc:
        _err(rc)


def gen_keys_u64(n: int, gen_seed: int = 0, start: int = 0, device="cuda") -> torch.Tensor:
    keys = torch.empty(n, dtype=torch.int64, device=device)
    rc = lib().mphx_gen_keys_u64(_ptr(keys), n, gen_seed, start, _stream(keys.device))
    if rc:
        _err(rc)
    return keys


def gen_str_keys(n: int, qtable: torch.Tensor, gen_seed: int = 0, start: int = 0, device="cuda"):
    """Device-generated string keys; qtable is the 65536-entry uint16 length table (as int16)."""
    _check(qtable, torch.int16, "qtable", 1 << 16)
    lens = torch.empty(max(n, 1), dtype=torch.int32, device=device)
    dev = lens.device
    rc = lib().mphx_gen_str_lengths(_ptr(lens), n, gen_seed, start, _ptr(qtable), _stream(dev))
    if rc:
        _err(rc)
    offs = torch.empty(n + 1, dtype=torch.int64, device=dev)
    scratch = _workspace(lib().mphx_scan_scratch_bytes(n + 1), dev)
    rc = lib().mphx_gen_str_offsets(_ptr(lens), n, _ptr(offs), _ptr(scratch), scratch.numel(), _stream(dev))
    if rc:
        _err(rc)
    del lens
    total = int(offs[-1].item())
    data = torch.empty(max(total, 4), dtype=torch.uint8, device=dev)
    rc = lib().mphx_gen_str_bytes(_ptr(data), _ptr(offs), n, gen_seed, start, _stream(dev))
    if rc:
        _err(rc)
    return data, offs


# ------------------------------------------------------------------------------------------
# batched builds
# ------------------------------------------------------------------------------------------
class BatchTuning(C.Structure):
    _fields_ = [("block", C.c_uint32), ("grid", C.c_uint32), ("scope", C.c_uint32), ("reserved", C.c_uint32)]


BUCKET_RESULT = None


def _bucket_dtype():
    import numpy as np

    return np.dtype([("seed_used", "<u8"), ("tries", "<u4"), ("status", "<i4"), ("n_rounds", "<u4"),
                     ("reserved", "<u4")])


def gen_buckets_u64(bucket_off: torch.Tensor) -> torch.Tensor:
    """Device keys of every bucket (bucket b: generator seed S(0, b + 1))."""
    _check(bucket_off, torch.int64, "bucket_off")
    B = bucket_off.numel() - 1
    total = int(bucket_off[-1].item())
    keys = torch.empty(max(total, 1), dtype=torch.int64, device=bucket_off.device)
    rc = lib().mphx_gen_buckets_u64(_ptr(keys), _ptr(bucket_off), B, _stream(bucket_off.device))
    if rc:
        _err(rc)
    return keys


class BatchBuild:
    """A batched build plan: B buckets of u64 keys with host offsets `bucket_off` (B+1)."""

    def __init__(self, bucket_off, device="cuda", gamma=(123, 100), max_tries=64, seed=0, block=0, grid=0, scope=0):
        import numpy as np

        off = np.ascontiguousarray(bucket_off, dtype=np.uint64)
        self.B = len(off) - 1
        self.gamma, self.max_tries, self.seed = gamma, max_tries, seed
        self.device = torch.device(device)
        code_off = np.zeros(self.B + 1, np.uint64)
        rank_off = np.zeros(self.B + 1, np.uint64)
        order = np.zeros(max(self.B, 1), np.uint32)
        mx = C.c_uint64(0)
        rc = lib().mphx_batch_layout(off.ctypes.data, self.B, gamma[0], gamma[1], code_off.ctypes.data,
                                     rank_off.ctypes.data, order.ctypes.data, C.byref(mx))
        if rc:
            _err(rc)
        self.max_bucket = int(mx.value)
        self.host_off, self.code_off_h, self.rank_off_h = off, code_off, rank_off
        self.tuning = BatchTuning(block, grid, scope, 0)
        dev = self.device
        self.bucket_off = torch.from_numpy(off.view(np.int64)).to(dev)
        self.order = torch.from_numpy(order.view(np.int32)).to(dev)
        self.code_off = torch.from_numpy(code_off.view(np.int64)).to(dev)
        self.rank_off = torch.from_numpy(rank_off.view(np.int64)).to(dev)
        self.codes = torch.zeros(max(int(code_off[-1]), 1), dtype=torch.int64, device=dev)
        self.rank = torch.zeros(max(int(rank_off[-1]), 1), dtype=torch.int64, device=dev)
        self.results = torch.zeros(max(self.B, 1) * 24, dtype=torch.uint8, device=dev)
        ws_bytes = lib().mphx_batch_workspace_bytes(self.B, self.max_bucket, gamma[0], gamma[1],
                                                    C.byref(self.tuning))
        if ws_bytes == 0:
            _err(EINVAL)
        self.ws = _workspace(ws_bytes, dev)
        self.graph = None

    def _args(self, keys):
        _check(keys, torch.int64, "keys")
        return (_ptr(keys), _ptr(self.bucket_off), _ptr(self.order), self.B, self.max_bucket, self.seed,
                self.gamma[0], self.gamma[1], self.max_tries, _ptr(self.code_off), _ptr(self.rank_off),
                _ptr(self.codes), _ptr(self.rank), _ptr(self.results), _ptr(self.ws), self.ws.numel(),
                C.byref(self.tuning))

    def autotune(self, keys, candidates=None, reps=2, max_ws_bytes=64 << 30):
        """Times each candidate tuning (default: the library's list) on this plan's buckets and
        keeps the fastest for later run() / capture() calls.  The workspace grows to the largest
        candidate's, up to max_ws_bytes (candidates beyond it are skipped).  A graph captured
        before is destroyed (it holds the old tuning and may hold the old workspace): capture
        again afterwards.  Returns dict(best, candidates [(block, grid)], ms [best time per
        candidate, -1 if skipped])."""
        self.destroy_graph()
        if candidates is None:
            cnt = lib().mphx_batch_tuning_candidates(None, 0)
            arr = (BatchTuning * cnt)()
            lib().mphx_batch_tuning_candidates(arr, cnt)
        else:
            arr = (BatchTuning * len(candidates))(*[BatchTuning(b, g, sc, 0) for b, g, sc in candidates])
        n = len(arr)
        need = max(lib().mphx_batch_workspace_bytes(self.B, self.max_bucket, self.gamma[0], self.gamma[1],
                                                    C.byref(arr[i])) for i in range(n))
        want = min(need, max_ws_bytes)
        if want > self.ws.numel():
            self.ws = None
            torch.cuda.empty_cache()
            self.ws = _workspace(want, self.device)
        args = list(self._args(keys))[:-1]  # everything but the tuning
        ms = (C.c_float * n)()
        best = C.c_uint32(0)
        rc = lib().mphx_batch_autotune_u64(*args, arr, n, reps, ms, C.byref(best), _stream(self.device))
        if rc:
            _err(rc)
        self.tuning = BatchTuning(arr[best.value].block, arr[best.value].grid, arr[best.value].scope, 0)
        return dict(best=int(best.value), candidates=[(int(a.block), int(a.grid)) for a in arr],
                    ms=[round(float(x), 3) for x in ms])

    def run(self, keys, max_bucket=None):
        """Enqueue the whole batch on the current stream (no synchronisation)."""
        args = list(self._args(keys))
        if max_bucket is not None:
            args[4] = max_bucket
        rc = lib().mphx_build_batch_u64(*args, _stream(self.device))
        if rc:
            _err(rc)

    def capture(self, keys):
        """Record the batch into a HIP graph (replayed by launch())."""
        self.destroy_graph()
        g = C.c_void_p()
        rc = lib().mphx_graph_capture_batch_u64(*self._args(keys), C.byref(g))
        if rc:
            _err(rc)
        self.graph = g

    def launch(self):
        rc = lib().mphx_graph_launch(self.graph, _stream(self.device))
        if rc:
            _err(rc)

    def destroy_graph(self):
        if self.graph is not None and self.graph.value:
            lib().mphx_graph_destroy(self.graph)
        self.graph = None

    def __del__(self):
        try:
            self.destroy_graph()
        except Exception:
            pass

    def bucket_results(self):
        return self.results.cpu().numpy()[: self.B * 24].view(_bucket_dtype())

    def bucket_codes(self, b):
        return self.codes[int(self.code_off_h[b]):int(self.code_off_h[b + 1])]

    def bucket_rank(self, b):
        return self.rank[int(self.rank_off_h[b]):int(self.rank_off_h[b + 1])]


# ------------------------------------------------------------------------------------------
# build server
# ------------------------------------------------------------------------------------------
class Request(C.Structure):
    _fields_ = [("key_kind", C.c_int32), ("max_tries", C.c_uint32), ("keys", C.c_void_p), ("bytes", C.c_void_p),
                ("offs", C.c_void_p), ("n", C.c_uint64), ("seed", C.c_uint64), ("gamma_num", C.c_uint32),
                ("gamma_den", C.c_uint32), ("codes", C.c_void_p), ("rank", C.c_void_p)]


class RequestResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("tries", C.c_uint32), ("n_rounds", C.c_uint32), ("reserved", C.c_uint32),
                ("seed_used", C.c_uint64), ("P", C.c_uint64), ("m", C.c_uint64), ("t_submit", C.c_double),
                ("t_start", C.c_double), ("t_done", C.c_double)]

    def as_dict(self):
        return {k: (float(getattr(self, k)) if k.startswith("t_") else int(getattr(self, k)))
                for k, _ in self._fields_}


class ServerStats(C.Structure):
    _fields_ = [("pending", C.c_uint32), ("running", C.c_uint32), ("completed", C.c_uint64), ("budget", C.c_size_t),
                ("in_use", C.c_size_t), ("peak_in_use", C.c_size_t)]


class Server:
    """Continuous-admission build server (see mphx_server_* in include/mphx.h).

    submit_*() returns a ticket at once; the caller keeps the key tensors alive until the
    ticket completes (the server holds references for it).  Outputs are allocated here."""

    def __init__(self, hbm_budget: int, slots: int = 4, batch_max_keys: int = 1 << 17, device="cuda"):
        self.device = torch.device(device)
        idx = self.device.index if self.device.index is not None else torch.cuda.current_device()
        h = C.c_void_p()
        rc = lib().mphx_server_create(idx, int(hbm_budget), int(slots), int(batch_max_keys), C.byref(h))
        if rc == ENOMEM:
            # the server allocates its pool itself; memory torch has cached but not in use
            # cannot serve that until it is given back
            torch.cuda.empty_cache()
            rc = lib().mphx_server_create(idx, int(hbm_budget), int(slots), int(batch_max_keys), C.byref(h))
        if rc:
            raise MphxError(rc, "server create failed")
        self.h = h
        self._live = {}

    @staticmethod
    def clock() -> float:
        return float(lib().mphx_server_clock())

    def _submit(self, req, hold, n, gamma):
        P = part_size(n, gamma)
        m = 3 * P
        codes = torch.empty(max((m + 31) // 32, 1), dtype=torch.int64, device=self.device)
        rank = torch.empty(max((m + 511) // 512, 1), dtype=torch.int64, device=self.device)
        req.codes, req.rank = _ptr(codes), _ptr(rank)
        torch.cuda.current_stream(self.device).synchronize()  # inputs/outputs exist before workers run
        t = C.c_uint64(0)
        rc = lib().mphx_server_submit(self.h, C.byref(req), C.byref(t))
        if rc:
            raise MphxError(rc, "submit failed")
        self._live[t.value] = (hold, codes, rank)
        return t.value

    def submit_u64(self, keys: torch.Tensor, seed: int = 0, gamma=(123, 100), max_tries: int = 64) -> int:
        _check(keys, torch.int64, "keys")
        req = Request(KEYS_U64, max_tries, _ptr(keys), None, None, keys.numel(), seed, gamma[0], gamma[1])
        return self._submit(req, (keys,), keys.numel(), gamma)

    def submit_str(self, data: torch.Tensor, offs: torch.Tensor, seed: int = 0, gamma=(123, 100),
                   max_tries: int = 64) -> int:
        _check(data, torch.uint8, "data")
        _check(offs, torch.int64, "offs")
        n = offs.numel() - 1
        req = Request(KEYS_STR, max_tries, None, _ptr(data), _ptr(offs), n, seed, gamma[0], gamma[1])
        return self._submit(req, (data, offs), n, gamma)

    def poll(self, ticket: int):
        r = RequestResult()
        rc = lib().mphx_server_poll(self.h, ticket, C.byref(r))
        if rc < 0:
            raise MphxError(rc, "poll failed")
        return None if rc == 1 else self._finish(ticket, r)

    def wait(self, ticket: int) -> dict:
        r = RequestResult()
        rc = lib().mphx_server_wait(self.h, ticket, C.byref(r))
        if rc:
            raise MphxError(rc, "wait failed")
        return self._finish(ticket, r)

    def _finish(self, ticket, r):
        d = r.as_dict()
        hold, codes, rank = self._live.get(ticket, (None, None, None))
        d["codes"], d["rank"] = codes, rank
        if codes is not None and d["m"]:
            d["codes"] = codes[: (d["m"] + 31) // 32]
            d["rank"] = rank[: (d["m"] + 511) // 512]
        return d

    def release(self, ticket: int):
        self._live.pop(ticket, None)

    def stats(self) -> dict:
        st = ServerStats()
        lib().mphx_server_stats(self.h, C.byref(st))
        return {k: int(getattr(st, k)) for k, _ in st._fields_}

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().mphx_server_destroy(self.h)
            self.h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_batch(buckets, gamma=(123, 100), max_tries=64, block=0, grid=0, scope=0, device="cuda"):
    """Batched builds of independent key sets given one by one.

    buckets: list of ("u64", keys) or ("str", data, offs) device tensors with a seed, as
    (kind, *tensors, seed).  Returns one dict per bucket (status, tries, seed_used, n_rounds,
    codes, rank), built in one persistent launch."""
    import numpy as np

    dev = torch.device(device)
    B = len(buckets)
    descs = np.zeros(max(B, 1), dtype=np.dtype([("keys", "<u8"), ("bytes", "<u8"), ("offs", "<u8"), ("n", "<u8"),
                                                 ("seed", "<u8"), ("codes", "<u8"), ("rank", "<u8"),
                                                 ("result", "<u8")]))
    results = torch.zeros(max(B, 1) * 24, dtype=torch.uint8, device=dev)
    outs, sizes = [], []
    for b, bk in enumerate(buckets):
        kind, seed = bk[0], bk[-1]
        if kind == "u64":
            _check(bk[1], torch.int64, "keys")
            n = bk[1].numel()
            descs[b]["keys"] = _ptr(bk[1])
        else:
            _check(bk[1], torch.uint8, "data")
            _check(bk[2], torch.int64, "offs")
            n = bk[2].numel() - 1
            descs[b]["bytes"], descs[b]["offs"] = _ptr(bk[1]), _ptr(bk[2])
        m = 3 * part_size(n, gamma)
        codes = torch.zeros(max((m + 31) // 32, 1), dtype=torch.int64, device=dev)
        rank = torch.zeros(max((m + 511) // 512, 1), dtype=torch.int64, device=dev)
        descs[b]["n"], descs[b]["seed"] = n, seed
        descs[b]["codes"], descs[b]["rank"] = _ptr(codes), _ptr(rank)
        descs[b]["result"] = _ptr(results) + 24 * b
        outs.append((codes, rank, m))
        sizes.append(n)
    d_descs = torch.from_numpy(descs.view(np.uint8).copy()).to(dev)
    order = np.argsort(-np.asarray(sizes, dtype=np.int64), kind="stable").astype(np.int32) if B else \
        np.zeros(1, np.int32)
    d_order = torch.from_numpy(order).to(dev)
    tuning = BatchTuning(block, grid, scope, 0)
    max_bucket = max(sizes) if sizes else 0
    ws = _workspace(lib().mphx_batch_desc_workspace_bytes(max_bucket, gamma[0], gamma[1], C.byref(tuning)), dev)
    rc = lib().mphx_build_batch(_ptr(d_descs), B, _ptr(d_order), max_bucket, gamma[0], gamma[1], max_tries, _ptr(ws),
                                ws.numel(), C.byref(tuning), _stream(dev))
    if rc:
        _err(rc)
    res = results.cpu().numpy()[: B * 24].view(_bucket_dtype())
    out = []
    for b in range(B):
        codes, rank, m = outs[b]
        out.append(dict(status=int(res[b]["status"]), tries=int(res[b]["tries"]), seed_used=int(res[b]["seed_used"]),
                        n_rounds=int(res[b]["n_rounds"]), codes=codes[: (m + 31) // 32], rank=rank[: (m + 511) // 512]))
    return out
