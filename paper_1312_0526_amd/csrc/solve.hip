// Assignment (Section 3, along the layers in reverse round order as in Section 4.3), code
// packing + rank counts, MPHF evaluation (Section 5 broadword ranking) and the bijection check.
#include "common.h"
#include "launch.h"

namespace mphx {

// code8[v]: 0 = not a hinge, 1/2 = hinge with g = 1/2, 3 = hinge with g = 0.
__device__ __forceinline__ uint32_t g_of_code(uint32_t c) { return c == 3 ? 0u : c; }

// One layer: every edge solves g[v_k] = k - g[v_k+1] - g[v_k+2] (mod 3) for its hinge k.
// Inside a layer no edge touches another edge's hinge (its only edge at round start), so the
// edges of a layer are independent.  Each layer slot holds the edge's vertices hinge first; the
// hinge position is the hinge vertex's part.
__global__ __launch_bounds__(256) void k_assign_round(const uint3* __restrict__ slots,
                                                      const uint64_t* __restrict__ lstart, uint32_t r, uint64_t P,
                                                      uint8_t* __restrict__ code8)
{
    const uint64_t lo = lstart[r], hi = lstart[r + 1];
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = lo + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hi; i += stride) {
        uint3 t = slots[i];
        uint32_t k = part_of(t.x, P);
        // the two code reads land on random lines that are rarely read again soon: marked
        // non-temporal (measured faster; the same hint on the write was slower)
        const uint32_t ga = __builtin_nontemporal_load(&code8[t.y]);
        const uint32_t gb = __builtin_nontemporal_load(&code8[t.z]);
        uint32_t g = (k + 6 - g_of_code(ga) - g_of_code(gb)) % 3;
        code8[t.x] = (uint8_t)(g ? g : 3);
    }
}

// Static-function layer: the hinge takes f(x) - u[v_a] - u[v_b] (mod sigma); the value of slot
// i's key travels in vals[i].  Every term is below sigma <= 2^32, so two conditional
// subtractions replace the division.  u is kept in the narrowest of u8 / u16 / u32 that holds
// b bits, which keeps its random accesses' footprint small.
template <typename T>
__global__ __launch_bounds__(256) void k_sf_assign_round(const uint3* __restrict__ slots,
                                                         const uint32_t* __restrict__ vals, uint64_t count,
                                                         uint64_t sigma, T* __restrict__ u)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        const uint3 t = slots[i];
        uint64_t x = (uint64_t)vals[i] + 2 * sigma - __builtin_nontemporal_load(&u[t.y]) -
                     __builtin_nontemporal_load(&u[t.z]);
        x = x >= sigma ? x - sigma : x;
        x = x >= sigma ? x - sigma : x;
        u[t.x] = (T)x;
    }
}

// One thread per output word w: the fields overlapping bits [64w, 64w + 64).
template <typename T>
__global__ __launch_bounds__(256) void k_sf_pack(const T* __restrict__ u, uint64_t m, uint32_t b,
                                                 uint64_t nwords, uint64_t* __restrict__ words)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nwords; w += stride) {
        const uint64_t lo = 64 * w, hi = lo + 64;
        uint64_t x = 0;
        for (uint64_t v = lo / b; v * b < hi && v < m; v++) {
            const uint64_t f = u[v];
            const int64_t sh = (int64_t)(v * b) - (int64_t)lo;  // in (-b, 64)
            x |= sh >= 0 ? f << sh : f >> (-sh);
        }
        words[w] = x;
    }
}

__global__ __launch_bounds__(256) void k_sf_lookup_u64(const uint64_t* __restrict__ words, uint64_t sigma, uint32_t b,
                                                       uint64_t P, uint64_t seed, const uint64_t* __restrict__ keys,
                                                       uint64_t n, uint64_t* __restrict__ out)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint64_t s = keys[i] ^ seed;
        uint32_t v0, v1, v2;
        edge_of_digest(s, s, P, v0, v1, v2);
        out[i] = sf_eval_edge(words, sigma, b, v0, v1, v2);
    }
}

// Ranked layout, pass 1: one thread per mark word (64 vertices): bit t set iff u[64w + t] != 0;
// the 16 words of a rank block sum their counts into bcount[block].
template <typename T>
__global__ __launch_bounds__(256) void k_sfr_marks(const T* __restrict__ u, uint64_t m, uint64_t nwords,
                                                   uint64_t* __restrict__ marks, uint32_t* __restrict__ bcount)
{
    constexpr uint32_t kVec = 16 / sizeof(T);  // elements per 16-byte load
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < nwords; base += stride) {
        const uint64_t w = base + threadIdx.x;
        uint64_t x = 0;
        if (w < nwords) {
            const uint64_t v0 = 64 * w;
            if (v0 + 64 <= m) {
                const uint4* p = reinterpret_cast<const uint4*>(u + v0);
#pragma unroll
                for (uint32_t q = 0; q < 64 / kVec; q++) {
                    union {
                        uint4 v;
                        T e[kVec];
                    } c;
                    c.v = p[q];
#pragma unroll
                    for (uint32_t t = 0; t < kVec; t++)
                        x |= (uint64_t)(c.e[t] != 0) << (q * kVec + t);
                }
            } else {
                for (uint64_t t = 0; v0 + t < m; t++)
                    x |= (uint64_t)(u[v0 + t] != 0) << t;
            }
            marks[w] = x;
        }
        uint32_t c = __popcll(x);
        c += __shfl_xor(c, 1, 16);
        c += __shfl_xor(c, 2, 16);
        c += __shfl_xor(c, 4, 16);
        c += __shfl_xor(c, 8, 16);
        if (w < nwords && (w & 15) == 0)
            bcount[w >> 4] = c;
    }
}

// Ranked layout, pass 2: one workgroup per rank block of 1024 vertices, 4 per thread.  The
// block's fields occupy bits [rank[j] b, rank[j + 1] b) of vals; they are assembled in LDS
// (word 0 = the word holding bit rank[j] b) and written out: words wholly inside the range with
// plain stores, the first and last -- which neighbouring blocks may share -- with atomicOr into
// zeroed memory.  Words from cap_words on are never written (there are at most n fields, one per
// hinge, and cap_words holds n of them).
template <typename T>
__global__ __launch_bounds__(256) void k_sfr_compact(const T* __restrict__ u, uint64_t m, uint32_t b,
                                                     const uint64_t* __restrict__ rank, uint64_t* __restrict__ vals,
                                                     uint64_t cap_words)
{
    constexpr uint32_t kWords = kSfrBlock * 32 / 64 + 2;  // b <= 32, plus the start offset
    __shared__ unsigned long long s_out[kWords];
    __shared__ uint32_t s_wave[256 / kWave];
    const uint64_t nblocks = (m + kSfrBlock - 1) / kSfrBlock;
    const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    for (uint64_t j = blockIdx.x; j < nblocks; j += gridDim.x) {
        const uint64_t v0 = j * kSfrBlock + 4 * tid;
        uint32_t x[4];
#pragma unroll
        for (uint32_t t = 0; t < 4; t++)
            x[t] = v0 + t < m ? (uint32_t)u[v0 + t] : 0u;
        const uint32_t c = (x[0] != 0) + (x[1] != 0) + (x[2] != 0) + (x[3] != 0);
        // exclusive prefix of c over the workgroup
        uint32_t incl = c;
#pragma unroll
        for (uint32_t d = 1; d < kWave; d <<= 1) {
            const uint32_t y = __shfl_up(incl, d, kWave);
            incl += lane >= d ? y : 0u;
        }
        if (lane == kWave - 1)
            s_wave[wave] = incl;
        for (uint32_t i = tid; i < kWords; i += blockDim.x)
            s_out[i] = 0;
        __syncthreads();
        uint32_t pre = incl - c;
        for (uint32_t q = 0; q < wave; q++)
            pre += s_wave[q];
        const uint64_t bit0 = rank[j] * b;
        const uint32_t off0 = (uint32_t)(bit0 & 63);
#pragma unroll
        for (uint32_t t = 0; t < 4; t++) {
            if (x[t] == 0)
                continue;
            const uint32_t lb = off0 + pre * b;
            const uint32_t lw = lb >> 6, sh = lb & 63;
            atomicOr(&s_out[lw], (unsigned long long)x[t] << sh);
            if (sh + b > 64)
                atomicOr(&s_out[lw + 1], (unsigned long long)x[t] >> (64 - sh));
            pre++;
        }
        __syncthreads();
        const uint32_t total = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
        if (total) {
            const uint32_t nw = (off0 + total * b + 63) / 64;
            unsigned long long* dst = reinterpret_cast<unsigned long long*>(vals) + (bit0 >> 6);
            for (uint32_t i = tid; i < nw && (bit0 >> 6) + i < cap_words; i += blockDim.x) {
                if (i == 0 || i == nw - 1)
                    atomicOr(&dst[i], s_out[i]);
                else
                    dst[i] = s_out[i];
            }
        }
        __syncthreads();  // s_out and s_wave are reused by the next block
    }
}

__global__ __launch_bounds__(256) void k_sfr_lookup_u64(const uint64_t* __restrict__ marks,
                                                        const uint64_t* __restrict__ rank,
                                                        const uint64_t* __restrict__ vals, uint64_t sigma, uint32_t b,
                                                        uint64_t P, uint64_t seed, const uint64_t* __restrict__ keys,
                                                        uint64_t n, uint64_t* __restrict__ out)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint64_t s = keys[i] ^ seed;
        uint32_t v0, v1, v2;
        edge_of_digest(s, s, P, v0, v1, v2);
        out[i] = sfr_eval_edge(marks, rank, vals, sigma, b, v0, v1, v2);
    }
}

// Flags a value outside [0, sigma) in ctrl->err.
__global__ __launch_bounds__(256) void k_sf_check(const uint32_t* __restrict__ vals, uint64_t n, uint64_t sigma,
                                                  Ctrl* ctrl)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        bad |= vals[i] >= sigma;
    if (__ballot(bad) && (threadIdx.x & (kWave - 1)) == 0)
        atomicOr(&ctrl->err, kErrValue);
}

__global__ __launch_bounds__(256) void k_pack_count(const uint8_t* __restrict__ code8, uint64_t m,
                                                    uint64_t* __restrict__ codes, uint32_t* __restrict__ bcount,
                                                    uint64_t nwords)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < nwords; base += stride) {
        uint64_t w = base + threadIdx.x;
        uint64_t x = 0;
        if (w < nwords) {
            uint64_t v0 = w * 32;
            if (v0 + 32 <= m) {
                const uint4* p = reinterpret_cast<const uint4*>(code8 + v0);
                uint4 a = p[0], b = p[1];
                uint32_t d[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
                for (int q = 0; q < 8; q++) {
#pragma unroll
                    for (int t = 0; t < 4; t++)
                        x |= (uint64_t)((d[q] >> (8 * t)) & 3u) << (2 * (4 * q + t));
                }
            } else {
                for (uint64_t t = 0; v0 + t < m && t < 32; t++)
                    x |= (uint64_t)(code8[v0 + t] & 3u) << (2 * t);
            }
            codes[w] = x;
        }
        uint32_t c = nz_pairs(x);
        c += __shfl_xor(c, 1, 16);
        c += __shfl_xor(c, 2, 16);
        c += __shfl_xor(c, 4, 16);
        c += __shfl_xor(c, 8, 16);
        if (w < nwords && (w & 15) == 0)
            bcount[w >> 4] = c;
    }
}

__global__ __launch_bounds__(256) void k_lookup_u64(const uint64_t* __restrict__ codes, const uint64_t* __restrict__ rank,
                                                    uint64_t P, uint64_t seed, const uint64_t* __restrict__ keys,
                                                    uint64_t n, uint64_t* __restrict__ out)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint64_t s = keys[i] ^ seed;
        uint32_t v0, v1, v2;
        edge_of_digest(s, s, P, v0, v1, v2);
        out[i] = eval_edge(codes, rank, v0, v1, v2);
    }
}

__global__ __launch_bounds__(256) void k_bijection(const uint64_t* __restrict__ vals, uint64_t n,
                                                   uint32_t* __restrict__ bitmap, Ctrl* ctrl)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    unsigned long long bad = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint64_t v = vals[i];
        if (v >= n) {
            bad++;
            continue;
        }
        uint32_t bit = 1u << (v & 31);
        uint32_t old = atomicOr(&bitmap[v >> 5], bit);
        if (old & bit)
            bad++;
    }
    if (bad)
        atomicAdd(&ctrl->aux, bad);
}

static inline unsigned grid_cap(uint64_t count, unsigned cap)
{
    uint64_t g = (count + 255) / 256;
    return (unsigned)(g < 1 ? 1 : (g > cap ? cap : g));
}

hipError_t launch_assign_round(const uint3* slots, const uint64_t* lstart, uint32_t r, uint64_t n_bound, uint64_t P,
                               uint8_t* code8, unsigned grid_cap_blocks, hipStream_t s)
{
    k_assign_round<<<grid_cap(n_bound, grid_cap_blocks), 256, 0, s>>>(slots, lstart, r, P, code8);
    return hipGetLastError();
}

uint32_t sf_elem_bytes(uint32_t b) { return b <= 8 ? 1u : (b <= 16 ? 2u : 4u); }

hipError_t launch_sf_assign_round(const uint3* slots, const uint32_t* vals, uint64_t count, uint64_t sigma,
                                  uint32_t b, void* u, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    const unsigned g = grid_cap(count, 16384);
    switch (sf_elem_bytes(b)) {
    case 1: k_sf_assign_round<uint8_t><<<g, 256, 0, s>>>(slots, vals, count, sigma, (uint8_t*)u); break;
    case 2: k_sf_assign_round<uint16_t><<<g, 256, 0, s>>>(slots, vals, count, sigma, (uint16_t*)u); break;
    default: k_sf_assign_round<uint32_t><<<g, 256, 0, s>>>(slots, vals, count, sigma, (uint32_t*)u);
    }
    return hipGetLastError();
}

hipError_t launch_sf_pack(const void* u, uint64_t m, uint32_t b, uint64_t* words, hipStream_t s)
{
    const uint64_t nwords = (m * b + 63) / 64;
    if (nwords == 0) return hipSuccess;
    const unsigned g = grid_cap(nwords, 16384);
    switch (sf_elem_bytes(b)) {
    case 1: k_sf_pack<uint8_t><<<g, 256, 0, s>>>((const uint8_t*)u, m, b, nwords, words); break;
    case 2: k_sf_pack<uint16_t><<<g, 256, 0, s>>>((const uint16_t*)u, m, b, nwords, words); break;
    default: k_sf_pack<uint32_t><<<g, 256, 0, s>>>((const uint32_t*)u, m, b, nwords, words);
    }
    return hipGetLastError();
}

hipError_t launch_sfr_marks(const void* u, uint64_t m, uint32_t b, uint64_t* marks, uint32_t* bcount, hipStream_t s)
{
    const uint64_t nwords = (m + 63) / 64;
    if (nwords == 0) return hipSuccess;
    const unsigned g = grid_cap(nwords, 16384);
    switch (sf_elem_bytes(b)) {
    case 1: k_sfr_marks<uint8_t><<<g, 256, 0, s>>>((const uint8_t*)u, m, nwords, marks, bcount); break;
    case 2: k_sfr_marks<uint16_t><<<g, 256, 0, s>>>((const uint16_t*)u, m, nwords, marks, bcount); break;
    default: k_sfr_marks<uint32_t><<<g, 256, 0, s>>>((const uint32_t*)u, m, nwords, marks, bcount);
    }
    return hipGetLastError();
}

hipError_t launch_sfr_compact(const void* u, uint64_t m, uint32_t b, const uint64_t* rank, uint64_t* vals,
                              uint64_t cap_words, hipStream_t s)
{
    const uint64_t nblocks = (m + kSfrBlock - 1) / kSfrBlock;
    if (nblocks == 0 || b == 0) return hipSuccess;
    const unsigned g = (unsigned)std::min<uint64_t>(nblocks, 8192);
    switch (sf_elem_bytes(b)) {
    case 1: k_sfr_compact<uint8_t><<<g, 256, 0, s>>>((const uint8_t*)u, m, b, rank, vals, cap_words); break;
    case 2: k_sfr_compact<uint16_t><<<g, 256, 0, s>>>((const uint16_t*)u, m, b, rank, vals, cap_words); break;
    default: k_sfr_compact<uint32_t><<<g, 256, 0, s>>>((const uint32_t*)u, m, b, rank, vals, cap_words);
    }
    return hipGetLastError();
}

hipError_t launch_sfr_lookup_u64(const uint64_t* marks, const uint64_t* rank, const uint64_t* vals, uint64_t sigma,
                                 uint32_t b, uint64_t P, uint64_t seed, const uint64_t* keys, uint64_t n,
                                 uint64_t* out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_sfr_lookup_u64<<<grid_cap(n, 16384), 256, 0, s>>>(marks, rank, vals, sigma, b, P, seed, keys, n, out);
    return hipGetLastError();
}

hipError_t launch_sf_lookup_u64(const uint64_t* words, uint64_t sigma, uint32_t b, uint64_t P, uint64_t seed,
                                const uint64_t* keys, uint64_t n, uint64_t* out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_sf_lookup_u64<<<grid_cap(n, 16384), 256, 0, s>>>(words, sigma, b, P, seed, keys, n, out);
    return hipGetLastError();
}

hipError_t launch_sf_check(const uint32_t* vals, uint64_t n, uint64_t sigma, Ctrl* ctrl, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_sf_check<<<grid_cap(n, 4096), 256, 0, s>>>(vals, n, sigma, ctrl);
    return hipGetLastError();
}

hipError_t launch_pack_count(const uint8_t* code8, uint64_t m, uint64_t* codes, uint32_t* bcount, hipStream_t s)
{
    uint64_t nwords = (m + 31) / 32;
    if (nwords == 0) return hipSuccess;
    k_pack_count<<<grid_cap(nwords, 16384), 256, 0, s>>>(code8, m, codes, bcount, nwords);
    return hipGetLastError();
}

hipError_t launch_lookup_u64(const uint64_t* codes, const uint64_t* rank, uint64_t P, uint64_t seed,
                             const uint64_t* keys, uint64_t n, uint64_t* out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_lookup_u64<<<grid_cap(n, 16384), 256, 0, s>>>(codes, rank, P, seed, keys, n, out);
    return hipGetLastError();
}

hipError_t launch_bijection(const uint64_t* vals, uint64_t n, uint32_t* bitmap, Ctrl* ctrl, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_bijection<<<grid_cap(n, 8192), 256, 0, s>>>(vals, n, bitmap, ctrl);
    return hipGetLastError();
}

}  // namespace mphx
