// Fill and exclusive-scan utilities (device kernels only; no hipMemset, so every step can sit
// inside a captured graph).
#include "common.h"
#include "launch.h"

namespace mphx {

constexpr uint32_t kScanItems = 16;
constexpr uint32_t kScanBlock = 256;
constexpr uint32_t kScanTile = kScanItems * kScanBlock;

__global__ __launch_bounds__(256) void k_zero16(uint4* p, uint64_t n16)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        p[i] = make_uint4(0, 0, 0, 0);
}

__global__ void k_zero_tail(uint8_t* p, uint64_t n)
{
    for (uint64_t i = threadIdx.x; i < n; i += blockDim.x)
        p[i] = 0;
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* p, uint64_t count, uint32_t value)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        p[i] = value;
}

__global__ void k_ctrl_init(Ctrl* ctrl, uint64_t* lstart)
{
    if (threadIdx.x == 0) {
        ctrl->ftail = 0;
        ctrl->ltail = 0;
        ctrl->nrounds = 0xFFFFFFFFu;
        ctrl->err = 0;
        ctrl->aux = 0;
        ctrl->claims = 0;
        ctrl->degsum = 0;
        ctrl->updates = 0;
        ctrl->touched = 0;
        ctrl->dups = 0;
        lstart[0] = 0;
    }
}

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T x)
{
    const uint32_t lane = threadIdx.x & (kWave - 1);
    for (uint32_t d = 1; d < kWave; d <<= 1) {
        T y = __shfl_up(x, d, kWave);
        if (lane >= d)
            x += y;
    }
    return x;
}

// Exclusive scan of one 4096-item tile per block; block totals go to sums[].
template <typename TIn, typename TOut>
__global__ __launch_bounds__(256) void k_scan_local(const TIn* in, uint64_t count_in, TOut* out, uint64_t count_out,
                                                    TOut* sums)
{
    __shared__ TOut wsum[kScanBlock / kWave];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    TOut v[kScanItems];
    TOut acc = 0;
#pragma unroll
    for (uint32_t t = 0; t < kScanItems; t++) {
        uint64_t idx = base + t;
        TOut x = idx < count_in ? (TOut)in[idx] : (TOut)0;
        v[t] = acc;
        acc += x;
    }
    TOut incl = wave_inclusive_scan(acc);
    const uint32_t w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == kWave - 1)
        wsum[w] = incl;
    __syncthreads();
    TOut wpre = 0;
    for (uint32_t q = 0; q < w; q++)
        wpre += wsum[q];
    TOut excl = wpre + incl - acc;
#pragma unroll
    for (uint32_t t = 0; t < kScanItems; t++) {
        uint64_t idx = base + t;
        if (idx < count_out)
            out[idx] = v[t] + excl;
    }
    if (threadIdx.x == kScanBlock - 1)
        sums[blockIdx.x] = wpre + incl;
}

// Exclusive scan of the block totals by one block, chunk by chunk.
template <typename T>
__global__ __launch_bounds__(256) void k_scan_sums(T* sums, uint64_t count)
{
    __shared__ T wsum[kScanBlock / kWave];
    __shared__ T carry_s;
    if (threadIdx.x == 0)
        carry_s = 0;
    __syncthreads();
    for (uint64_t chunk = 0; chunk < count; chunk += kScanTile) {
        const uint64_t base = chunk + (uint64_t)threadIdx.x * kScanItems;
        T v[kScanItems];
        T acc = 0;
#pragma unroll
        for (uint32_t t = 0; t < kScanItems; t++) {
            uint64_t idx = base + t;
            T x = idx < count ? sums[idx] : (T)0;
            v[t] = acc;
            acc += x;
        }
        T incl = wave_inclusive_scan(acc);
        const uint32_t w = threadIdx.x / kWave;
        if ((threadIdx.x & (kWave - 1)) == kWave - 1)
            wsum[w] = incl;
        __syncthreads();
        T wpre = 0;
        for (uint32_t q = 0; q < w; q++)
            wpre += wsum[q];
        T carry = carry_s;
        T excl = carry + wpre + incl - acc;
#pragma unroll
        for (uint32_t t = 0; t < kScanItems; t++) {
            uint64_t idx = base + t;
            if (idx < count)
                sums[idx] = v[t] + excl;
        }
        __syncthreads();
        if (threadIdx.x == kScanBlock - 1)
            carry_s = carry + wpre + incl;
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_scan_add(T* out, uint64_t count_out, const T* sums)
{
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    const T add = sums[blockIdx.x];
    for (uint32_t t = threadIdx.x; t < kScanTile; t += kScanBlock) {
        uint64_t idx = base + t;
        if (idx < count_out)
            out[idx] += add;
    }
}

static inline unsigned cap_grid(uint64_t count, unsigned cap)
{
    uint64_t g = (count + 255) / 256;
    return (unsigned)(g < 1 ? 1 : (g > cap ? cap : g));
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s)
{
    if (bytes == 0) return hipSuccess;
    uint64_t n16 = bytes / 16;
    if (n16)
        k_zero16<<<cap_grid(n16, 8192), 256, 0, s>>>(reinterpret_cast<uint4*>(p), n16);
    uint64_t tail = bytes - n16 * 16;
    if (tail)
        k_zero_tail<<<1, 64, 0, s>>>(reinterpret_cast<uint8_t*>(p) + n16 * 16, tail);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint64_t count, uint32_t value, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    k_fill_u32<<<cap_grid(count, 8192), 256, 0, s>>>(p, count, value);
    return hipGetLastError();
}

hipError_t launch_ctrl_init(Ctrl* ctrl, uint64_t* lstart, hipStream_t s)
{
    k_ctrl_init<<<1, 64, 0, s>>>(ctrl, lstart);
    return hipGetLastError();
}

size_t scan_scratch_bytes(uint64_t count)
{
    uint64_t tiles = (count + kScanTile - 1) / kScanTile;
    return (size_t)(tiles * 8 + 256);
}

template <typename TIn, typename TOut>
static hipError_t scan_impl(const TIn* in, uint64_t count_in, TOut* out, uint64_t count_out, void* scratch,
                            size_t scratch_bytes, hipStream_t s)
{
    if (count_out == 0) return hipSuccess;
    uint64_t tiles = (count_out + kScanTile - 1) / kScanTile;
    if (scratch_bytes < tiles * sizeof(TOut) || tiles > 0x7FFFFFFFull)
        return hipErrorInvalidValue;
    TOut* sums = reinterpret_cast<TOut*>(scratch);
    k_scan_local<TIn, TOut><<<(unsigned)tiles, kScanBlock, 0, s>>>(in, count_in, out, count_out, sums);
    if (tiles > 1) {
        k_scan_sums<TOut><<<1, kScanBlock, 0, s>>>(sums, tiles);
        k_scan_add<TOut><<<(unsigned)tiles, kScanBlock, 0, s>>>(out, count_out, sums);
    }
    return hipGetLastError();
}

hipError_t launch_scan_u32(const uint32_t* in, uint64_t count, uint32_t* out, void* scratch, size_t scratch_bytes,
                           hipStream_t s)
{
    return scan_impl<uint32_t, uint32_t>(in, count, out, count, scratch, scratch_bytes, s);
}

hipError_t launch_scan_u32_to_u64(const uint32_t* in, uint64_t count_in, uint64_t* out, uint64_t count_out,
                                  void* scratch, size_t scratch_bytes, hipStream_t s)
{
    return scan_impl<uint32_t, uint64_t>(in, count_in, out, count_out, scratch, scratch_bytes, s);
}

}  // namespace mphx
