// Machine-ceiling probes: the streaming and random-access rates that bound the build's kernels.
// A streaming copy gives the practical HBM ceiling; random 8-byte atomics, loads and 1-byte
// stores over a table of a chosen footprint give the ceilings of the degree build, the peeling
// rounds and the assignment as a function of how much of the table the caches can hold.
#include "common.h"
#include "../../include/mphx.h"

namespace mphx {
namespace {

__global__ void k_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, uint64_t n16)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        dst[i] = src[i];
}

// Address i of a probe: uniform in [0, slots) from the SplitMix64 output of seed + (i+1)G.
__device__ __forceinline__ uint64_t probe_slot(uint64_t seed, uint64_t i, uint64_t slots)
{
    return range_reduce(fin(seed + (i + 1) * kGamma), slots);
}

template <int kOp>
__global__ void k_random(unsigned long long* __restrict__ table, uint64_t slots, uint64_t count, uint64_t seed)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t acc = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        const uint64_t j = probe_slot(seed, i, slots);
        if constexpr (kOp == MPHX_PROBE_ATOMIC_ADD) {
            __hip_atomic_fetch_add(&table[j], (unsigned long long)i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else if constexpr (kOp == MPHX_PROBE_ATOMIC_ADD_RET) {
            acc ^= atomicAdd(&table[j], (unsigned long long)i);
        } else if constexpr (kOp == MPHX_PROBE_LOAD8) {
            acc ^= table[j];
        } else if constexpr (kOp == MPHX_PROBE_STORE1) {
            reinterpret_cast<uint8_t*>(table)[j] = (uint8_t)i;
        } else if constexpr (kOp == MPHX_PROBE_ATOMIC_ADD32) {
            __hip_atomic_fetch_add(reinterpret_cast<uint32_t*>(table) + j, (uint32_t)i, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        } else if constexpr (kOp == MPHX_PROBE_ATOMIC_ADD_WG) {
            __hip_atomic_fetch_add(&table[j], (unsigned long long)i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    // keeps the returned values live; the table holds no such value unless the probe computed it
    if (acc == 0x0123456789ABCDEFull) table[0] = acc;
}

// Random 8-byte atomics into an LDS table of `slots` entries (at most kLdsSlots) per workgroup;
// the table is written out once so the work cannot be dropped.
constexpr uint32_t kLdsSlots = 8192;

__global__ void __launch_bounds__(1024) k_random_lds(unsigned long long* __restrict__ out, uint32_t slots,
                                                     uint64_t count, uint64_t seed)
{
    __shared__ unsigned long long t[kLdsSlots];
    for (uint32_t j = threadIdx.x; j < slots; j += blockDim.x) t[j] = 0;
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        atomicAdd(&t[probe_slot(seed, i, slots)], (unsigned long long)i);
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < slots; j += blockDim.x)
        out[(uint64_t)blockIdx.x * slots + j] = t[j];
}

}  // namespace
}  // namespace mphx

using namespace mphx;

extern "C" {

MPHX_API int mphx_probe_copy(const void* src, void* dst, uint64_t bytes, uint32_t grid, void* stream)
{
    if (!src || !dst || (bytes & 15) || (((uintptr_t)src | (uintptr_t)dst) & 15)) return MPHX_EINVAL;
    if (bytes == 0) return MPHX_OK;
    const uint32_t g = grid ? grid : 256u * 32u;
    hipLaunchKernelGGL(k_copy, dim3(g), dim3(256), 0, (hipStream_t)stream, (const uint4*)src, (uint4*)dst,
                       bytes / 16);
    return hipGetLastError() == hipSuccess ? MPHX_OK : MPHX_EDEVICE;
}

MPHX_API int mphx_probe_random(int op, void* table, uint64_t slots, uint64_t count, uint64_t seed, uint32_t grid,
                               uint32_t block, void* stream)
{
    if (!table || slots == 0 || block == 0 || block > 1024 || (block & 63)) return MPHX_EINVAL;
    if (count == 0) return MPHX_OK;
    hipStream_t s = (hipStream_t)stream;
    const uint32_t g = grid ? grid : 256u * 32u;
    auto* t = (unsigned long long*)table;
    switch (op) {
    case MPHX_PROBE_ATOMIC_ADD:
        hipLaunchKernelGGL(k_random<MPHX_PROBE_ATOMIC_ADD>, dim3(g), dim3(block), 0, s, t, slots, count, seed);
        break;
    case MPHX_PROBE_ATOMIC_ADD_RET:
        hipLaunchKernelGGL(k_random<MPHX_PROBE_ATOMIC_ADD_RET>, dim3(g), dim3(block), 0, s, t, slots, count, seed);
        break;
    case MPHX_PROBE_LOAD8:
        hipLaunchKernelGGL(k_random<MPHX_PROBE_LOAD8>, dim3(g), dim3(block), 0, s, t, slots, count, seed);
        break;
    case MPHX_PROBE_STORE1:
        hipLaunchKernelGGL(k_random<MPHX_PROBE_STORE1>, dim3(g), dim3(block), 0, s, t, slots, count, seed);
        break;
    case MPHX_PROBE_ATOMIC_ADD32:
        hipLaunchKernelGGL(k_random<MPHX_PROBE_ATOMIC_ADD32>, dim3(g), dim3(block), 0, s, t, slots, count, seed);
        break;
    case MPHX_PROBE_ATOMIC_ADD_WG:
        hipLaunchKernelGGL(k_random<MPHX_PROBE_ATOMIC_ADD_WG>, dim3(g), dim3(block), 0, s, t, slots, count, seed);
        break;
    case MPHX_PROBE_LDS_ATOMIC_ADD:
        // the table must hold grid * slots entries of 8 bytes
        if (slots > kLdsSlots) return MPHX_EINVAL;
        hipLaunchKernelGGL(k_random_lds, dim3(g), dim3(block), 0, s, t, (uint32_t)slots, count, seed);
        break;
    default:
        return MPHX_EINVAL;
    }
    return hipGetLastError() == hipSuccess ? MPHX_OK : MPHX_EDEVICE;
}

}  // extern "C"
