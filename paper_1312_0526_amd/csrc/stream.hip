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
// part appends the edge hinge first.  The degree bytes are scanned 64 per thread per pass (four
// coalesced 16-byte groups), bytes equal to 1 found with word arithmetic, and only those
// vertices read their pack; a thread keeps a 64-bit mask of its hinges, one block-wide scan of
// the masks' bit counts gives every hinge its place, and the slots are staged in LDS and go out with one cursor
// atomic per full buffer (a pass with more hinges than the buffer reserves its range at once).
// All hinges of a round append to one cursor, whose atomics serialise, so they stay rare.
constexpr uint32_t kStScanU = 4;      // 16-byte groups per thread per pass
constexpr uint32_t kStStage = 2048;   // staged slots per block (24 KB)

// bit 8j + 7 set iff byte j of w equals 1 (exact per byte: no borrow between bytes)
__device__ __forceinline__ uint32_t bytes_eq1(uint32_t w)
{
    const uint32_t y = w ^ 0x01010101u;
    return ~(((y & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | y) & 0x80808080u;
}
// those four flags as bits 0..3
__device__ __forceinline__ uint32_t flags4(uint32_t f)
{
    return ((f >> 7) & 1u) | ((f >> 14) & 2u) | ((f >> 21) & 4u) | ((f >> 28) & 8u);
}

__global__ __launch_bounds__(kStBlock) void k_st_claim(const uint8_t* __restrict__ deg, const uint64_t* __restrict__ X,
                                                       uint64_t P, uint32_t k, uint3* __restrict__ slots, uint64_t cap,
                                                       unsigned long long* cursor)
{
    __shared__ uint3 s_buf[kStStage];
    __shared__ uint32_t s_wsum[kStBlock / kWave];
    __shared__ uint32_t s_count;
    __shared__ unsigned long long s_base;
    const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    if (tid == 0)
        s_count = 0;
    const uint64_t base = (uint64_t)k * P, end = base + P;  // the part's vertices
    const uint64_t g0 = base / 16, g1 = (end + 15) / 16;      // 16-byte groups covering them
    const uint4* d4 = reinterpret_cast<const uint4*>(deg);
    auto out = [slots, cap](uint64_t i, uint3 sl) {
        if (i < cap) slots[i] = sl;  // slots past the area are counted, not stored
    };
    auto flush = [&]() {
        __syncthreads();
        const uint32_t c = s_count;
        if (tid == 0 && c)
            s_base = atomicAdd(cursor, (unsigned long long)c);
        __syncthreads();
        for (uint32_t i = tid; i < c; i += kStBlock)
            out(s_base + i, s_buf[i]);
        __syncthreads();
        if (tid == 0)
            s_count = 0;
        __syncthreads();
    };
    // the pack of vertex v as a slot: (id in part k, ids in parts k+1, k+2)
    auto slot_of = [&](uint64_t v) {
        const uint64_t x = X[v];
        return make_uint3((uint32_t)(v - base), (uint32_t)x, (uint32_t)(x >> 32));
    };
    constexpr uint64_t kPass = (uint64_t)kStScanU * kStBlock;  // groups per block per pass
    for (uint64_t gb = g0 + (uint64_t)blockIdx.x * kPass; gb < g1; gb += (uint64_t)gridDim.x * kPass) {  // uniform
        uint4 w[kStScanU];
#pragma unroll
        for (uint32_t u = 0; u < kStScanU; u++) {
            const uint64_t g = gb + u * kStBlock + tid;
            w[u] = g < g1 ? d4[g] : make_uint4(0u, 0u, 0u, 0u);
        }
        uint64_t hm = 0;  // bit 16u + j: byte j of group u is a hinge
#pragma unroll
        for (uint32_t u = 0; u < kStScanU; u++) {
            const uint64_t g = gb + u * kStBlock + tid;
            uint32_t mk = flags4(bytes_eq1(w[u].x)) | flags4(bytes_eq1(w[u].y)) << 4 |
                          flags4(bytes_eq1(w[u].z)) << 8 | flags4(bytes_eq1(w[u].w)) << 12;
            const uint64_t b0 = 16 * g;
            if (b0 < base)
                mk &= 0xFFFFu << (uint32_t)(base - b0);
            if (b0 + 16 > end)
                mk &= end > b0 ? 0xFFFFu >> (uint32_t)(b0 + 16 - end) : 0u;
            while (mk) {
                const uint32_t j = __builtin_ctz(mk);
                mk &= mk - 1;
                const uint3 sl = slot_of(b0 + j);
                bool h = true;
                if (k >= 1)  // part 0's vertex: b when k = 1, a when k = 2
                    h = deg[k == 1 ? sl.z : sl.y] != 1;
                if (k == 2 && h)  // part 1's vertex
                    h = deg[P + sl.z] != 1;
                if (h)
                    hm |= 1ull << (16 * u + j);
            }
        }
        // exclusive prefix of the hinge counts over the block, and their total
        const uint32_t c = __popcll(hm);
        uint32_t incl = c;
#pragma unroll
        for (uint32_t dd = 1; dd < kWave; dd <<= 1) {
            const uint32_t y = __shfl_up(incl, dd, kWave);
            incl += lane >= dd ? y : 0u;
        }
        if (lane == kWave - 1)
            s_wsum[wv] = incl;
        __syncthreads();
        uint32_t pre = incl - c, total = 0;
#pragma unroll
        for (uint32_t q = 0; q < kStBlock / kWave; q++) {
            pre += q < wv ? s_wsum[q] : 0u;
            total += s_wsum[q];
        }
        if (total) {  // uniform
            if (total > kStStage) {  // more than the buffer: reserve the range directly
                if (tid == 0)
                    s_base = atomicAdd(cursor, (unsigned long long)total);
                __syncthreads();
                uint64_t at = s_base + pre;
                for (uint64_t mm = hm; mm; mm &= mm - 1) {
                    const uint32_t bit = __builtin_ctzll(mm);
                    out(at++, slot_of(16 * (gb + (bit >> 4) * kStBlock + tid) + (bit & 15)));
                }
            } else {
                if (s_count + total > kStStage)
                    flush();
                uint32_t at = s_count + pre;
                for (uint64_t mm = hm; mm; mm &= mm - 1) {
                    const uint32_t bit = __builtin_ctzll(mm);
                    s_buf[at++] = slot_of(16 * (gb + (bit >> 4) * kStBlock + tid) + (bit & 15));
                }
                __syncthreads();
                if (tid == 0)
                    s_count += total;
            }
        }
        __syncthreads();  // s_wsum, s_base and s_count are reused by the next pass
    }
    flush();
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
    const uint64_t groups = (k * P + P + 15) / 16 - k * P / 16;
    const uint64_t passes = (groups + kStScanU * kStBlock - 1) / (kStScanU * kStBlock);
    k_st_claim<<<(unsigned)std::max<uint64_t>(1, std::min<uint64_t>(passes, 2048)), kStBlock, 0, s>>>(deg, X, P, k,
                                                                                                   slots, cap, cursor);
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
