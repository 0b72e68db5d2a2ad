// Key hashing (Section 3; tripartite layout of Section 4.3) fused with the packed-record build
// (Section 4.1 AddEdge, non-returning atomics; degree overflow is checked by the frontier
// scan), and the device-side synthetic key generators.
#include "common.h"
#include "launch.h"

namespace mphx {

// ---- u64 keys: one thread per key, state a = b = key XOR seed -------------------------------
template <bool kBuild>
__global__ __launch_bounds__(256) void k_hash_u64(const uint64_t* __restrict__ keys, uint64_t n, uint64_t seed,
                                                  uint64_t P, uint32_t* __restrict__ edges, uint64_t* __restrict__ rec)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint64_t s = keys[i] ^ seed;
        uint32_t v0, v1, v2;
        edge_of_digest(s, s, P, v0, v1, v2);
        edges[3 * i] = v0;
        edges[3 * i + 1] = v1;
        edges[3 * i + 2] = v2;
        if constexpr (kBuild) {
            Rec::add(rec, v0, (uint32_t)i);
            Rec::add(rec, v1, (uint32_t)i);
            Rec::add(rec, v2, (uint32_t)i);
        }
    }
}

template <bool kBuild>
__global__ __launch_bounds__(256) void k_hash_str(const uint8_t* __restrict__ bytes, const uint64_t* __restrict__ offs,
                                                  uint64_t n, uint64_t seed, uint64_t P, uint32_t* __restrict__ edges,
                                                  uint64_t* __restrict__ rec)
{
    const uint64_t total = offs[n];
    const uint64_t sa = fin(seed + kGamma);
    const uint64_t sb = fin(seed + 2 * kGamma);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint64_t o0 = offs[i], o1 = offs[i + 1];
        uint64_t a, b;
        digest_str(bytes, o0, o1 - o0, total, sa, sb, a, b);
        uint32_t v0, v1, v2;
        edge_of_digest(a, b, P, v0, v1, v2);
        edges[3 * i] = v0;
        edges[3 * i + 1] = v1;
        edges[3 * i + 2] = v2;
        if constexpr (kBuild) {
            Rec::add(rec, v0, (uint32_t)i);
            Rec::add(rec, v1, (uint32_t)i);
            Rec::add(rec, v2, (uint32_t)i);
        }
    }
}

// ---- synthetic key generators ------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gen_u64(uint64_t* __restrict__ keys, uint64_t n, uint64_t gen_seed,
                                                 uint64_t start)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        keys[i] = fin(gen_seed + (start + i + 1) * kGamma);
}

// Bucketed u64 key sets: bucket b uses generator seed S(0, b + 1); one block per bucket.
__global__ __launch_bounds__(256) void k_gen_buckets_u64(uint64_t* __restrict__ keys, const uint64_t* __restrict__ off,
                                                         uint32_t B)
{
    for (uint32_t b = blockIdx.x; b < B; b += gridDim.x) {
        const uint64_t lo = off[b], n = off[b + 1] - lo;
        const uint64_t gs = fin((uint64_t)(b + 1) * kGamma);
        for (uint64_t j = threadIdx.x; j < n; j += blockDim.x)
            keys[lo + j] = fin(gs + (j + 1) * kGamma);
    }
}

__global__ __launch_bounds__(256) void k_gen_str_len(uint32_t* __restrict__ lens, uint64_t n, uint64_t gen_seed,
                                                     uint64_t start, const uint16_t* __restrict__ qtable)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint64_t x = fin(gen_seed + (start + i + 1) * kGamma);
        lens[i] = qtable[fin(x + kGamma) >> 48];
    }
}

// Byte j of string key gi whose u64 key is x (see the header for the definition).
struct StrKeyBytes {
    uint64_t x, gi;
    uint64_t cur_t = 0, cur_w = 0;
    __device__ uint8_t at(uint64_t j)
    {
        if (j < 5) {
            uint64_t q = gi;
            for (uint64_t d = 0; d < j; d++)
                q /= 95;
            return (uint8_t)(0x20 + q % 95);
        }
        uint64_t t = 2 + (j - 5) / 8;
        if (t != cur_t) {
            cur_t = t;
            cur_w = fin(x + t * kGamma);
        }
        uint32_t b = (uint32_t)(cur_w >> (8 * ((j - 5) & 7))) & 0xFFu;
        return (uint8_t)(0x20 + ((b * 95u) >> 8));
    }
};

__global__ __launch_bounds__(256) void k_gen_str_bytes(uint8_t* __restrict__ bytes, const uint64_t* __restrict__ offs,
                                                       uint64_t n, uint64_t gen_seed, uint64_t start)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        StrKeyBytes kb;
        kb.gi = start + i;
        kb.x = fin(gen_seed + (kb.gi + 1) * kGamma);
        const uint64_t o0 = offs[i], o1 = offs[i + 1];
        if (o1 <= o0)
            continue;
        const uint64_t q0 = o0 >> 2, q1 = (o1 - 1) >> 2;
        for (uint64_t q = q0; q <= q1; q++) {
            uint64_t b0 = q * 4;
            if (b0 >= o0 && b0 + 4 <= o1) {
                uint32_t v = 0;
                for (uint32_t t = 0; t < 4; t++)
                    v |= (uint32_t)kb.at(b0 + t - o0) << (8 * t);
                *reinterpret_cast<uint32_t*>(bytes + b0) = v;
            } else {
                for (uint32_t t = 0; t < 4; t++) {
                    uint64_t p = b0 + t;
                    if (p >= o0 && p < o1)
                        bytes[p] = kb.at(p - o0);
                }
            }
        }
    }
}

static inline unsigned grid_cap(uint64_t count, unsigned cap)
{
    uint64_t g = (count + 255) / 256;
    return (unsigned)(g < 1 ? 1 : (g > cap ? cap : g));
}

hipError_t launch_hash_u64(const uint64_t* keys, uint64_t n, uint64_t seed, uint64_t P, uint32_t* edges,
                           uint64_t* rec, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    unsigned g = grid_cap(n, 16384);
    if (!rec)
        k_hash_u64<false><<<g, 256, 0, s>>>(keys, n, seed, P, edges, rec);
    else
        k_hash_u64<true><<<g, 256, 0, s>>>(keys, n, seed, P, edges, rec);
    return hipGetLastError();
}

hipError_t launch_hash_str(const uint8_t* bytes, const uint64_t* offs, uint64_t n, uint64_t seed, uint64_t P,
                           uint32_t* edges, uint64_t* rec, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    unsigned g = grid_cap(n, 16384);
    if (!rec)
        k_hash_str<false><<<g, 256, 0, s>>>(bytes, offs, n, seed, P, edges, rec);
    else
        k_hash_str<true><<<g, 256, 0, s>>>(bytes, offs, n, seed, P, edges, rec);
    return hipGetLastError();
}

hipError_t launch_gen_u64(uint64_t* keys, uint64_t n, uint64_t gen_seed, uint64_t start, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_gen_u64<<<grid_cap(n, 16384), 256, 0, s>>>(keys, n, gen_seed, start);
    return hipGetLastError();
}

hipError_t launch_gen_buckets_u64(uint64_t* keys, const uint64_t* off, uint32_t B, hipStream_t s)
{
    if (B == 0) return hipSuccess;
    k_gen_buckets_u64<<<(B < 65536u ? B : 65536u), 256, 0, s>>>(keys, off, B);
    return hipGetLastError();
}

hipError_t launch_gen_str_lengths(uint32_t* lens, uint64_t n, uint64_t gen_seed, uint64_t start,
                                  const uint16_t* qtable, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_gen_str_len<<<grid_cap(n, 16384), 256, 0, s>>>(lens, n, gen_seed, start, qtable);
    return hipGetLastError();
}

hipError_t launch_gen_str_bytes(uint8_t* bytes, const uint64_t* offs, uint64_t n, uint64_t gen_seed, uint64_t start,
                                hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_gen_str_bytes<<<grid_cap(n, 16384), 256, 0, s>>>(bytes, offs, n, gen_seed, start);
    return hipGetLastError();
}

}  // namespace mphx
