// Streamed MWHC build: keys in host memory, one hypergraph of up to 3 * 2^32 vertices.
//
// The vertex record is the paper's packed incidence list (Section 4.1) in its r = 3 form with
// the tripartition of Section 4.3: a vertex of part k keeps its degree and the XOR of
// pack(id in part k+1, id in part k+2) over its incident edges, ids being part-local (below
// P <= 2^32).  A vertex of degree 1 thus reads its only edge off its record, so the peel needs
// neither an edge array nor edge ids, and n can exceed 2^32.  Degrees are bytes (four to a
// 32-bit word, updated by shifted word atomics: a degree never drops below zero, so no borrow
// crosses a byte; a build that would pass 255 is reported).
//
// Rounds are synchronous (Section 4.2): at the start of round r, a scan of each part k finds
// the vertices of degree 1, and such a vertex appends its edge, hinge first, when no vertex of
// a lower part of that edge also has degree 1 -- the lowest position among the edge's degree-1
// vertices is the hinge, and each edge of the layer is appended exactly once, by its hinge.
// The scans of parts 0, 1, 2 append one after another, so a layer is three runs of slots,
// one per hinge part, and a slot (vh, va, vb) needs no stored part.  Then the deletes of the
// layer: the hinge's degree is cleared, the other two vertices lose one degree and the edge's
// pack.  Assignment walks the layers in reverse round order (Section 4.3).
#include "common.h"
#include "launch.h"

#include <algorithm>

namespace mphx {

namespace {

constexpr uint32_t kStBlock = 256;

__device__ __forceinline__ void st_locals(uint64_t key, uint64_t seed, uint64_t P, uint32_t l[3])
{
    const uint64_t s = key ^ seed;
    l[0] = (uint32_t)range_reduce(fin(s + kGamma), P);
    l[1] = (uint32_t)range_reduce(fin(s + 2 * kGamma), P);
    l[2] = (uint32_t)range_reduce(fin(s + 3 * kGamma), P);
}

// the two other endpoints of a part-k vertex: the ids in parts k+1 and k+2 (mod 3)
__device__ __forceinline__ uint64_t st_pack(uint32_t next, uint32_t next2) { return ((uint64_t)next2 << 32) | next; }

__device__ __forceinline__ uint32_t* deg_word(uint8_t* deg, uint64_t v)
{
    return reinterpret_cast<uint32_t*>(deg + (v & ~3ull));
}
__device__ __forceinline__ uint32_t deg_shift(uint64_t v) { return 8u * (uint32_t)(v & 3u); }

unsigned grid_for_st(uint64_t count, unsigned cap)
{
    const uint64_t g = (count + kStBlock - 1) / kStBlock;
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(g, cap));
}

// AddEdge of every key of a chunk at its three vertices (Section 4.1).
__global__ __launch_bounds__(kStBlock) void k_st_build(const uint64_t* __restrict__ keys, uint64_t cn, uint64_t seed,
                                                       uint64_t P, uint8_t* __restrict__ deg, uint64_t* __restrict__ X,
                                                       Ctrl* ctrl)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    bool over = false;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cn; i += stride) {
        uint32_t l[3];
        st_locals(keys[i], seed, P, l);
#pragma unroll
        for (uint32_t k = 0; k < 3; k++) {
            const uint64_t v = k * P + l[k];
            const uint32_t sh = deg_shift(v);
            const uint32_t old = atomicAdd(deg_word(deg, v), 1u << sh);
            over |= ((old >> sh) & 255u) == 255u;
            atomicXor(reinterpret_cast<unsigned long long*>(X + v),
                      (unsigned long long)st_pack(l[k == 2 ? 0 : k + 1], l[k == 0 ? 2 : k - 1]));
        }
    }
    if (over)
        atomicOr(&ctrl->err, kErrDegree);
}

// Round start, part k: every vertex of degree 1 whose edge has no degree-1 vertex in a lower
// part appends the edge hinge first.  Each thread looks at four consecutive vertices (one
// 32-bit word of degrees) per pass; the appends gather in an LDS buffer and go out with one
// cursor atomic per buffer (all hinges of a round append to one cursor, whose atomics
// serialise: one per wave would cost far more than the scan).
using StAppender = BlockAppender<uint3, kStBlock, 8 * kStBlock>;

__global__ __launch_bounds__(kStBlock) void k_st_claim(const uint8_t* __restrict__ deg, const uint64_t* __restrict__ X,
                                                       uint64_t P, uint32_t k, uint3* __restrict__ slots, uint64_t cap,
                                                       unsigned long long* cursor)
{
    __shared__ StAppender app;
    app.init();
    const uint64_t base = (uint64_t)k * P;
    const uint64_t words = (P + 3) / 4 + 1;  // the part may start inside a word
    const uint64_t w_first = base / 4;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    auto out = [slots, cap](uint64_t i, uint3 sl) {
        if (i < cap) slots[i] = sl;
    };
    for (uint64_t wb = (uint64_t)blockIdx.x * blockDim.x; wb < words; wb += stride) {  // uniform per block
        const uint64_t w = w_first + wb + threadIdx.x;
        uint32_t dw = 0;
        if (wb + threadIdx.x < words && 4 * w < base + P)
            dw = reinterpret_cast<const uint32_t*>(deg)[w];
        bool hinge[4] = {false, false, false, false};
        uint3 sl[4];
#pragma unroll
        for (uint32_t j = 0; j < 4; j++) {
            const uint64_t v = 4 * w + j;
            sl[j] = make_uint3(0u, 0u, 0u);
            if (((dw >> (8 * j)) & 255u) == 1u && v >= base && v < base + P) {
                const uint64_t x = X[v];
                const uint32_t a = (uint32_t)x, b = (uint32_t)(x >> 32);  // ids in parts k+1, k+2
                bool h = true;
                if (k >= 1)  // part 0's vertex: b when k = 1, a when k = 2
                    h = deg[k == 1 ? b : a] != 1;
                if (k == 2 && h)  // part 1's vertex
                    h = deg[P + b] != 1;
                hinge[j] = h;
                sl[j] = make_uint3((uint32_t)(v - base), a, b);
            }
        }
        if (__syncthreads_or(hinge[0] | hinge[1] | hinge[2] | hinge[3])) {
            app.push(hinge[0], sl[0], hinge[1], sl[1], cursor, out);
            app.push(hinge[2], sl[2], hinge[3], sl[3], cursor, out);
        }
    }
    app.flush(cursor, out);  // slots past cap are counted, not stored: the host checks the cursor
}

// DeleteEdge of every edge of a layer (runs [lo, b1), [b1, b2), [b2, hi) of hinge parts 0, 1, 2).
__global__ __launch_bounds__(kStBlock) void k_st_apply(const uint3* __restrict__ slots, uint64_t lo, uint64_t b1,
                                                       uint64_t b2, uint64_t hi, uint64_t P, uint8_t* __restrict__ deg,
                                                       uint64_t* __restrict__ X)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = lo + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hi; i += stride) {
        const uint32_t h = i < b1 ? 0u : (i < b2 ? 1u : 2u);
        const uint3 sl = slots[i];
        const uint32_t ha = h == 2 ? 0u : h + 1, hb = h == 0 ? 2u : h - 1;
        const uint64_t vh = (uint64_t)h * P + sl.x, va = (uint64_t)ha * P + sl.y, vb = (uint64_t)hb * P + sl.z;
        // the hinge keeps only this edge: its degree drops to zero, its pack is never read again
        atomicSub(deg_word(deg, vh), 1u << deg_shift(vh));
        atomicSub(deg_word(deg, va), 1u << deg_shift(va));
        atomicSub(deg_word(deg, vb), 1u << deg_shift(vb));
        atomicXor(reinterpret_cast<unsigned long long*>(X + va), (unsigned long long)st_pack(sl.z, sl.x));
        atomicXor(reinterpret_cast<unsigned long long*>(X + vb), (unsigned long long)st_pack(sl.x, sl.y));
    }
}

// Assignment of one layer: g(vh) = (h - g(va) - g(vb)) mod 3, code 3 standing for g = 0.
__global__ __launch_bounds__(kStBlock) void k_st_assign(const uint3* __restrict__ slots, uint64_t lo, uint64_t b1,
                                                        uint64_t b2, uint64_t hi, uint64_t P, uint8_t* __restrict__ code8)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = lo + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hi; i += stride) {
        const uint32_t h = i < b1 ? 0u : (i < b2 ? 1u : 2u);
        const uint3 sl = slots[i];
        const uint32_t ha = h == 2 ? 0u : h + 1, hb = h == 0 ? 2u : h - 1;
        const uint32_t ga = __builtin_nontemporal_load(code8 + (uint64_t)ha * P + sl.y) % 3u;
        const uint32_t gb = __builtin_nontemporal_load(code8 + (uint64_t)hb * P + sl.z) % 3u;
        const uint32_t g = (h + 6u - ga - gb) % 3u;
        code8[(uint64_t)h * P + sl.x] = (uint8_t)(g ? g : 3u);
    }
}

__device__ __forceinline__ uint32_t code_at64(const uint64_t* codes, uint64_t v)
{
    return (uint32_t)(codes[v >> 5] >> (2 * (v & 31))) & 3u;
}

__device__ __forceinline__ uint64_t nz_pairs(uint64_t w)
{
    return (uint64_t)__popcll((w | (w >> 1)) & 0x5555555555555555ull);
}

// rank of vertex h (64-bit positions): its block's sample plus the non-zero codes before it
__device__ __forceinline__ uint64_t rank_of64(const uint64_t* codes, const uint64_t* rank, uint64_t h)
{
    uint64_t r = rank[h >> 9];
    const uint64_t w0 = (h >> 9) * 16, w1 = h >> 5;
    for (uint64_t w = w0; w < w1; w++)
        r += nz_pairs(codes[w]);
    const uint32_t below = 2 * (uint32_t)(h & 31);
    return r + nz_pairs(codes[w1] & (below ? ((1ull << below) - 1) : 0ull));
}

// f(key): i = (g0 + g1 + g2) mod 3, the rank of vertex i.  With a bitmap, also marks f(key)
// and counts values out of range or seen twice (the bijection check, Section 1).
__global__ __launch_bounds__(kStBlock) void k_st_lookup(const uint64_t* __restrict__ codes,
                                                        const uint64_t* __restrict__ rank, uint64_t P, uint64_t seed,
                                                        const uint64_t* __restrict__ keys, uint64_t cn,
                                                        uint64_t* __restrict__ out, uint32_t* __restrict__ bitmap,
                                                        uint64_t n_total, Ctrl* ctrl)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    unsigned long long bad = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cn; i += stride) {
        uint32_t l[3];
        st_locals(keys[i], seed, P, l);
        const uint64_t v0 = l[0], v1 = P + l[1], v2 = 2 * P + l[2];
        const uint32_t s = (code_at64(codes, v0) % 3 + code_at64(codes, v1) % 3 + code_at64(codes, v2) % 3) % 3;
        const uint64_t f = rank_of64(codes, rank, s == 0 ? v0 : (s == 1 ? v1 : v2));
        if (out)
            out[i] = f;
        if (bitmap) {
            if (f >= n_total) {
                bad++;
            } else {
                const uint32_t bit = 1u << (f & 31);
                if (atomicOr(bitmap + (f >> 5), bit) & bit)
                    bad++;
            }
        }
    }
    if (bad)
        atomicAdd(&ctrl->aux, bad);
}

}  // namespace

hipError_t launch_st_build(const uint64_t* keys, uint64_t cn, uint64_t seed, uint64_t P, uint8_t* deg, uint64_t* X,
                           Ctrl* ctrl, hipStream_t s)
{
    if (cn == 0) return hipSuccess;
    k_st_build<<<grid_for_st(cn, 16384), kStBlock, 0, s>>>(keys, cn, seed, P, deg, X, ctrl);
    return hipGetLastError();
}

hipError_t launch_st_claim(const uint8_t* deg, const uint64_t* X, uint64_t P, uint32_t k, uint3* slots, uint64_t cap,
                           unsigned long long* cursor, Ctrl* ctrl, hipStream_t s)
{
    if (P == 0 || k > 2) return hipSuccess;
    (void)ctrl;
    k_st_claim<<<grid_for_st((P + 3) / 4 + 1, 16384), kStBlock, 0, s>>>(deg, X, P, k, slots, cap, cursor);
    return hipGetLastError();
}

hipError_t launch_st_apply(const uint3* slots, uint64_t lo, uint64_t b1, uint64_t b2, uint64_t hi, uint64_t P,
                           uint8_t* deg, uint64_t* X, hipStream_t s)
{
    if (hi <= lo) return hipSuccess;
    k_st_apply<<<grid_for_st(hi - lo, 16384), kStBlock, 0, s>>>(slots, lo, b1, b2, hi, P, deg, X);
    return hipGetLastError();
}

hipError_t launch_st_assign(const uint3* slots, uint64_t lo, uint64_t b1, uint64_t b2, uint64_t hi, uint64_t P,
                            uint8_t* code8, hipStream_t s)
{
    if (hi <= lo) return hipSuccess;
    k_st_assign<<<grid_for_st(hi - lo, 16384), kStBlock, 0, s>>>(slots, lo, b1, b2, hi, P, code8);
    return hipGetLastError();
}

hipError_t launch_st_lookup(const uint64_t* codes, const uint64_t* rank, uint64_t P, uint64_t seed,
                            const uint64_t* keys, uint64_t cn, uint64_t* out, uint32_t* bitmap, uint64_t n_total,
                            Ctrl* ctrl, hipStream_t s)
{
    if (cn == 0) return hipSuccess;
    k_st_lookup<<<grid_for_st(cn, 16384), kStBlock, 0, s>>>(codes, rank, P, seed, keys, cn, out, bitmap, n_total,
                                                            ctrl);
    return hipGetLastError();
}

}  // namespace mphx
