// Key hashing (Section 3; tripartite layout of Section 4.3) fused with the packed-record build
// (Section 4.1 AddEdge, non-returning atomics; degree overflow is checked by the frontier
// scan), and the device-side synthetic key generators.
#include "common.h"
#include "launch.h"

#include <algorithm>

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

// ---- first-pass partition histograms, counted while hashing ----------------------------------
// A block that hashes exactly one partition tile counts each part's group digits in LDS and
// writes its column of the [3][NH][nt1] histogram at the end.
struct TileHist {
    uint32_t c[3 * kPartMaxGroups];
    __device__ void clear()
    {
        for (uint32_t j = threadIdx.x; j < 3 * kPartMaxGroups; j += blockDim.x)
            c[j] = 0;
    }
    __device__ void count(uint32_t v0, uint32_t v1, uint32_t v2, uint64_t P)
    {
        atomicAdd(&c[v0 >> kPartGrpShift], 1u);
        atomicAdd(&c[kPartMaxGroups + ((uint32_t)(v1 - P) >> kPartGrpShift)], 1u);
        atomicAdd(&c[2 * kPartMaxGroups + ((uint32_t)(v2 - 2 * P) >> kPartGrpShift)], 1u);
    }
    __device__ void store(const PartHist1& h, uint32_t tile)
    {
        for (uint32_t j = threadIdx.x; j < 3 * h.NH; j += blockDim.x) {
            const uint32_t k = j / h.NH, g = j - k * h.NH;
            h.hist[((uint64_t)k * h.NH + g) * h.nt1 + tile] = c[k * kPartMaxGroups + g];
        }
    }
};

// ---- u64 keys with the histograms: one block per partition tile ----------------------------
constexpr uint32_t kHuBlock = 256;

__global__ __launch_bounds__(kHuBlock) void k_hash_u64_tiles(const uint64_t* __restrict__ keys, uint64_t n,
                                                             uint64_t seed, uint64_t P, uint32_t* __restrict__ edges,
                                                             PartHist1 h1)
{
    __shared__ TileHist th;
    th.clear();
    __syncthreads();
    const uint64_t t0 = (uint64_t)blockIdx.x * kPartTile;
    const uint64_t t1 = min<uint64_t>(t0 + kPartTile, n);
    for (uint64_t i = t0 + threadIdx.x; i < t1; i += kHuBlock) {
        uint64_t s = keys[i] ^ seed;
        uint32_t v0, v1, v2;
        edge_of_digest(s, s, P, v0, v1, v2);
        edges[3 * i] = v0;
        edges[3 * i + 1] = v1;
        edges[3 * i + 2] = v2;
        th.count(v0, v1, v2, P);
    }
    __syncthreads();
    th.store(h1, blockIdx.x);
}

// ---- byte-string keys, word-parallel: the edge list alone ------------------------------------
// Key lengths vary (the generated ones from 8 to 512 bytes, mean 60), so one thread per key
// leaves most lanes of a wave idle while its longest key finishes.  Here a block takes 256
// consecutive keys and spreads their 8-byte words over its lanes: word f of the block's flat
// word list belongs to key owner[f] at word index j, adds its two mixed terms into that key's
// LDS sums, and the key's thread finishes the digest.  The owner table covers a window of
// kHsWindow words at a time (the block walks as many windows as its keys need, so a key of
// any length is spread too); it is filled by one mark per key and a block-wide running
// maximum, so no thread loops over a long key's words.  The loads of consecutive words are
// consecutive in memory; each lane has two words' loads in flight.
// With histograms requested, block b hashes exactly partition tile b.
constexpr uint32_t kHsBlock = 256;
constexpr uint32_t kHsWindow = 2048;
constexpr uint32_t kHsUnroll = 2;
constexpr uint32_t kHsSub = 2;
static_assert(kPartTile % kHsBlock == 0, "a partition tile is whole chunks");
static_assert(kHsWindow == 8 * kHsBlock, "each thread scans eight owner entries");

__device__ __forceinline__ uint64_t key_word(const uint8_t* bytes, uint64_t p, uint64_t total)
{
    const uint64_t q = p >> 2;
    const uint32_t sh = (uint32_t)(p & 3) * 8;
    const uint64_t lo = (uint64_t)load_dword(bytes, q, total) | ((uint64_t)load_dword(bytes, q + 1, total) << 32);
    if (sh == 0)
        return lo;
    return (lo >> sh) | ((uint64_t)load_dword(bytes, q + 2, total) << (64 - sh));
}

// With kMode = kHsEvalMphf / kHsEvalSf the kernel evaluates a built function instead (Section 3
// lookups): each key's edge gives out[i] = f(key i), from the MPHF's codes and rank samples or
// from a static function's packed values, and nothing else is written.
struct EvalTables {
    const uint64_t* codes;  // MPHF codes, or a static function's packed fields
    const uint64_t* rank;
    uint64_t* out;
    uint64_t sigma;
    uint32_t bits;
    HemTables hem;
    const uint64_t* marks;  // ranked static function: marks (codes then holds its fields)
};
// kHsHemSig writes each key's HEM signature record, its whole digest (out as uint4: high and
// low half of a, then low and high half of b); kHsEvalHem evaluates a HEM split
// (kHsEvalSfr: a static function in the ranked layout)
constexpr int kHsEdges = 0, kHsEvalMphf = 1, kHsEvalSf = 2, kHsHemSig = 3, kHsEvalHem = 4, kHsEvalSfr = 5;

template <int kMode>
__global__ __launch_bounds__(kHsBlock) void k_hash_str_words(const uint8_t* __restrict__ bytes,
                                                             const uint64_t* __restrict__ offs, uint64_t n,
                                                             uint64_t seed, uint64_t P, uint32_t* __restrict__ edges,
                                                             PartHist1 h1, EvalTables mt)
{
    // Per key t of the chunk, with pre its first word in the chunk's flat word list: word f of
    // the key (index j = f - pre) starts at byte base[t] + 8f and its lane-A salt is
    // salt[t] + f * GAMMA (lane B adds sb - sa), so both follow from f by additions; end[t]
    // is the key's end byte.
    __shared__ uint64_t s_base[kHsBlock], s_end[kHsBlock], s_salt[kHsBlock], s_wtot[kHsBlock / kWave];
    // each key's two sums are split over kHsSub partial sums (lane & (kHsSub - 1)), so that
    // the neighbouring lanes that add words of one key hit different LDS addresses
    __shared__ unsigned long long s_A[kHsBlock * kHsSub], s_B[kHsBlock * kHsSub];
    __shared__ uint4 s_owner4[kHsWindow / 8];  // kHsWindow u16 entries: owner + 1 of each word
    __shared__ uint32_t s_wmax[kHsBlock / kWave];
    __shared__ TileHist th;
    uint16_t* const s_owner = reinterpret_cast<uint16_t*>(s_owner4);
    const uint64_t total = offs[n];
    const uint64_t sa = fin(seed + kGamma);
    const uint64_t sb = fin(seed + 2 * kGamma);
    const uint64_t dba = sb - sa;
    constexpr uint64_t kStep = (uint64_t)kHsUnroll * kHsBlock;
    const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const uint64_t nchunks = (n + kHsBlock - 1) / kHsBlock;
    uint64_t c0 = blockIdx.x, c1 = nchunks, cstep = gridDim.x;
    if (h1.hist) {
        c0 = (uint64_t)blockIdx.x * (kPartTile / kHsBlock);
        c1 = min<uint64_t>(c0 + kPartTile / kHsBlock, nchunks);
        cstep = 1;
        th.clear();
    }
    for (uint64_t c = c0; c < c1; c += cstep) {
        const uint64_t i = c * kHsBlock + tid;
        uint64_t o0 = 0, len = 0;
        if (i < n) {
            o0 = offs[i];
            len = offs[i + 1] - o0;
        }
        const uint64_t nw = (len + 7) >> 3;
#pragma unroll
        for (uint32_t k = 0; k < kHsSub; k++) {
            s_A[tid * kHsSub + k] = 0;
            s_B[tid * kHsSub + k] = 0;
        }
        // exclusive prefix of the word counts over the block
        uint64_t incl = nw;
        for (uint32_t d = 1; d < kWave; d <<= 1) {
            uint64_t y = __shfl_up(incl, d, kWave);
            if (lane >= d)
                incl += y;
        }
        if (lane == kWave - 1)
            s_wtot[wv] = incl;
        __syncthreads();
        uint64_t pre = 0, W = 0;
        for (uint32_t q = 0; q < kHsBlock / kWave; q++) {
            pre += q < wv ? s_wtot[q] : 0ull;
            W += s_wtot[q];
        }
        pre += incl - nw;
        s_base[tid] = o0 - 8 * pre;
        s_end[tid] = o0 + len;
        s_salt[tid] = sa - pre * kGamma;
        for (uint64_t w0 = 0; w0 < W; w0 += kHsWindow) {
            const uint64_t w1 = min<uint64_t>(w0 + kHsWindow, W);
            // Owners of the window's words: every key with words in [w0, w1) marks its first
            // one there with its index + 1, and a running maximum over the window carries
            // each mark to the key's later words (keys own consecutive, increasing ranges).
            s_owner4[tid] = make_uint4(0u, 0u, 0u, 0u);
            __syncthreads();
            if (nw && pre < w1 && pre + nw > w0)
                s_owner[max<uint64_t>(pre, w0) - w0] = (uint16_t)(tid + 1);
            __syncthreads();
            {
                const uint4 m4 = s_owner4[tid];
                uint32_t e[8] = {m4.x & 0xFFFFu, m4.x >> 16, m4.y & 0xFFFFu, m4.y >> 16,
                                 m4.z & 0xFFFFu, m4.z >> 16, m4.w & 0xFFFFu, m4.w >> 16};
#pragma unroll
                for (uint32_t k = 1; k < 8; k++)
                    e[k] = max(e[k], e[k - 1]);
                uint32_t run = e[7];
                for (uint32_t d = 1; d < kWave; d <<= 1) {
                    const uint32_t y = __shfl_up(run, d, kWave);
                    if (lane >= d)
                        run = max(run, y);
                }
                if (lane == kWave - 1)
                    s_wmax[wv] = run;
                uint32_t carry = __shfl_up(run, 1, kWave);
                if (lane == 0)
                    carry = 0;
                __syncthreads();
                for (uint32_t q = 0; q < wv; q++)
                    carry = max(carry, s_wmax[q]);
#pragma unroll
                for (uint32_t k = 0; k < 8; k++)
                    e[k] = max(e[k], carry);
                s_owner4[tid] = make_uint4(e[0] | e[1] << 16, e[2] | e[3] << 16, e[4] | e[5] << 16, e[6] | e[7] << 16);
            }
            __syncthreads();
            uint64_t fg = (w0 + tid) * kGamma;  // f0 * GAMMA
            for (uint64_t f0 = w0 + tid; f0 < w1; f0 += kStep, fg += kStep * kGamma) {
                uint32_t t[kHsUnroll];
                uint64_t p[kHsUnroll], w[kHsUnroll];
                bool fast = true;
#pragma unroll
                for (uint32_t u = 0; u < kHsUnroll; u++) {
                    const uint64_t f = f0 + u * kHsBlock;
                    t[u] = 0;
                    p[u] = 0;
                    if (f < w1) {
                        t[u] = s_owner[f - w0] - 1u;
                        p[u] = s_base[t[u]] + 8 * f;
                    }
                    fast = fast && ((p[u] >> 2) + 3) * 4 <= total;
                }
                if (fast) {  // all three dwords of every word inside the array: plain loads
                    const uint32_t* d = reinterpret_cast<const uint32_t*>(bytes);
                    uint32_t x0[kHsUnroll], x1[kHsUnroll], x2[kHsUnroll];
#pragma unroll
                    for (uint32_t u = 0; u < kHsUnroll; u++) {
                        const uint64_t q = p[u] >> 2;
                        x0[u] = d[q];
                        x1[u] = d[q + 1];
                        x2[u] = d[q + 2];
                    }
                    // the 8 bytes from p: alignbyte shifts a dword pair right by (p & 3) bytes
#pragma unroll
                    for (uint32_t u = 0; u < kHsUnroll; u++) {
                        const uint32_t sh = (uint32_t)p[u];
                        const uint32_t lo = __builtin_amdgcn_alignbyte(x1[u], x0[u], sh);
                        const uint32_t hi = __builtin_amdgcn_alignbyte(x2[u], x1[u], sh);
                        w[u] = (uint64_t)lo | ((uint64_t)hi << 32);
                    }
                } else {
#pragma unroll
                    for (uint32_t u = 0; u < kHsUnroll; u++)
                        w[u] = f0 + u * kHsBlock < w1 ? key_word(bytes, p[u], total) : 0ull;
                }
#pragma unroll
                for (uint32_t u = 0; u < kHsUnroll; u++) {
                    if (f0 + u * kHsBlock < w1) {
                        // bytes past the key's end count as zero: shift them out and back
                        const uint64_t rem = s_end[t[u]] - p[u];
                        const uint32_t sh = rem < 8 ? 64u - 8u * (uint32_t)rem : 0u;
                        const uint64_t x = (w[u] << sh) >> sh;
                        const uint64_t salt = s_salt[t[u]] + fg + (uint64_t)u * kHsBlock * kGamma;
                        const uint32_t slot = t[u] * kHsSub + (lane & (kHsSub - 1));
                        atomicAdd(&s_A[slot], (unsigned long long)fin(x ^ salt));
                        atomicAdd(&s_B[slot], (unsigned long long)fin(x ^ (salt + dba)));
                    }
                }
            }
            __syncthreads();  // the owner window is rewritten next
        }
        if (i < n) {
            uint64_t A = 0, B = 0;
#pragma unroll
            for (uint32_t k = 0; k < kHsSub; k++) {
                A += s_A[tid * kHsSub + k];
                B += s_B[tid * kHsSub + k];
            }
            const uint64_t a = fin(A ^ sa ^ len);
            const uint64_t b = fin(B ^ sb ^ len);
            uint32_t v0, v1, v2;
            edge_of_digest(a, b, P, v0, v1, v2);
            if constexpr (kMode == kHsHemSig) {
                reinterpret_cast<uint4*>(mt.out)[i] =
                    make_uint4((uint32_t)(a >> 32), (uint32_t)a, (uint32_t)b, (uint32_t)(b >> 32));
            } else if constexpr (kMode == kHsEvalHem) {
                mt.out[i] = hem_eval_digest(mt.hem, a, b);
            } else if constexpr (kMode == kHsEvalMphf) {
                mt.out[i] = eval_edge(mt.codes, mt.rank, v0, v1, v2);
            } else if constexpr (kMode == kHsEvalSf) {
                mt.out[i] = sf_eval_edge(mt.codes, mt.sigma, mt.bits, v0, v1, v2);
            } else if constexpr (kMode == kHsEvalSfr) {
                mt.out[i] = sfr_eval_edge(mt.marks, mt.rank, mt.codes, mt.sigma, mt.bits, v0, v1, v2);
            } else {
                edges[3 * i] = v0;
                edges[3 * i + 1] = v1;
                edges[3 * i + 2] = v2;
                if (h1.hist)
                    th.count(v0, v1, v2, P);
            }
        }
        __syncthreads();  // the per-key LDS arrays are reused by the next chunk
    }
    if (h1.hist)
        th.store(h1, blockIdx.x);
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
                           uint64_t* rec, PartHist1 h1, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    if (!rec && h1.hist) {
        k_hash_u64_tiles<<<(unsigned)h1.nt1, kHuBlock, 0, s>>>(keys, n, seed, P, edges, h1);
        return hipGetLastError();
    }
    unsigned g = grid_cap(n, 16384);
    if (!rec)
        k_hash_u64<false><<<g, 256, 0, s>>>(keys, n, seed, P, edges, rec);
    else
        k_hash_u64<true><<<g, 256, 0, s>>>(keys, n, seed, P, edges, rec);
    return hipGetLastError();
}

hipError_t launch_hash_str(const uint8_t* bytes, const uint64_t* offs, uint64_t n, uint64_t seed, uint64_t P,
                           uint32_t* edges, uint64_t* rec, PartHist1 h1, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    if (!rec) {
        const uint64_t chunks = (n + kHsBlock - 1) / kHsBlock;
        const unsigned g = h1.hist ? (unsigned)h1.nt1 : (unsigned)std::min<uint64_t>(chunks, 65536);
        k_hash_str_words<kHsEdges><<<g, kHsBlock, 0, s>>>(bytes, offs, n, seed, P, edges, h1, EvalTables{});
        return hipGetLastError();
    }
    unsigned g = grid_cap(n, 16384);
    k_hash_str<true><<<g, 256, 0, s>>>(bytes, offs, n, seed, P, edges, rec);
    return hipGetLastError();
}

hipError_t launch_lookup_str_words(const uint64_t* codes, const uint64_t* rank, uint64_t P, uint64_t seed,
                                   const uint8_t* bytes, const uint64_t* offs, uint64_t n, uint64_t* out,
                                   hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const uint64_t chunks = (n + kHsBlock - 1) / kHsBlock;
    const unsigned g = (unsigned)std::min<uint64_t>(chunks, 65536);
    k_hash_str_words<kHsEvalMphf><<<g, kHsBlock, 0, s>>>(bytes, offs, n, seed, P, nullptr, PartHist1{nullptr, 0, 0},
                                                         EvalTables{codes, rank, out, 0, 0, HemTables{}});
    return hipGetLastError();
}

hipError_t launch_sf_lookup_str_words(const uint64_t* words, uint64_t sigma, uint32_t b, uint64_t P, uint64_t seed,
                                      const uint8_t* bytes, const uint64_t* offs, uint64_t n, uint64_t* out,
                                      hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const uint64_t chunks = (n + kHsBlock - 1) / kHsBlock;
    const unsigned g = (unsigned)std::min<uint64_t>(chunks, 65536);
    k_hash_str_words<kHsEvalSf><<<g, kHsBlock, 0, s>>>(bytes, offs, n, seed, P, nullptr, PartHist1{nullptr, 0, 0},
                                                       EvalTables{words, nullptr, out, sigma, b, HemTables{}});
    return hipGetLastError();
}

hipError_t launch_sfr_lookup_str_words(const uint64_t* marks, const uint64_t* rank, const uint64_t* vals,
                                       uint64_t sigma, uint32_t b, uint64_t P, uint64_t seed, const uint8_t* bytes,
                                       const uint64_t* offs, uint64_t n, uint64_t* out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const uint64_t chunks = (n + kHsBlock - 1) / kHsBlock;
    const unsigned g = (unsigned)std::min<uint64_t>(chunks, 65536);
    k_hash_str_words<kHsEvalSfr><<<g, kHsBlock, 0, s>>>(bytes, offs, n, seed, P, nullptr, PartHist1{nullptr, 0, 0},
                                                        EvalTables{vals, rank, out, sigma, b, HemTables{}, marks});
    return hipGetLastError();
}

// HEM signature records of u64 keys: (signature >> 32, signature & 0xFFFFFFFF), which read as
// a u64 are the half-swapped signature (the key inside its bucket).
__global__ __launch_bounds__(256) void k_hem_sig_u64(const uint64_t* __restrict__ keys, uint64_t n, uint64_t seed,
                                                     uint2* __restrict__ rec)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t sig = hem_signature_u64(keys[i], seed);
        rec[i] = make_uint2((uint32_t)(sig >> 32), (uint32_t)sig);
    }
}

__global__ __launch_bounds__(256) void k_hem_lookup_u64(HemTables t, uint64_t seed, const uint64_t* __restrict__ keys,
                                                        uint64_t n, uint64_t* __restrict__ out)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = hem_eval(t, hem_signature_u64(keys[i], seed));
}

hipError_t launch_hem_sig_u64(const uint64_t* keys, uint64_t n, uint64_t seed, uint2* rec, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_hem_sig_u64<<<grid_cap(n, 16384), 256, 0, s>>>(keys, n, seed, rec);
    return hipGetLastError();
}

hipError_t launch_hem_sig_str(const uint8_t* bytes, const uint64_t* offs, uint64_t n, uint64_t seed, uint4* rec,
                              hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const uint64_t chunks = (n + kHsBlock - 1) / kHsBlock;
    const unsigned g = (unsigned)std::min<uint64_t>(chunks, 65536);
    EvalTables t{};
    t.out = reinterpret_cast<uint64_t*>(rec);
    // P only shapes the (unused) edge: any valid value
    k_hash_str_words<kHsHemSig><<<g, kHsBlock, 0, s>>>(bytes, offs, n, seed, 1, nullptr, PartHist1{nullptr, 0, 0}, t);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_offs_rebase(uint64_t* __restrict__ offs, uint64_t count, uint64_t base)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        offs[i] -= base;
}

hipError_t launch_offs_rebase(uint64_t* offs, uint64_t count, uint64_t base, hipStream_t s)
{
    if (count == 0 || base == 0) return hipSuccess;
    k_offs_rebase<<<grid_cap(count, 16384), 256, 0, s>>>(offs, count, base);
    return hipGetLastError();
}

hipError_t launch_hem_lookup_u64(const HemTables& t, uint64_t seed, const uint64_t* keys, uint64_t n, uint64_t* out,
                                 hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_hem_lookup_u64<<<grid_cap(n, 16384), 256, 0, s>>>(t, seed, keys, n, out);
    return hipGetLastError();
}

hipError_t launch_hem_lookup_str(const HemTables& ht, uint64_t seed, const uint8_t* bytes, const uint64_t* offs,
                                 uint64_t n, uint64_t* out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const uint64_t chunks = (n + kHsBlock - 1) / kHsBlock;
    const unsigned g = (unsigned)std::min<uint64_t>(chunks, 65536);
    EvalTables t{};
    t.out = out;
    t.hem = ht;
    k_hash_str_words<kHsEvalHem><<<g, kHsBlock, 0, s>>>(bytes, offs, n, seed, 1, nullptr, PartHist1{nullptr, 0, 0}, t);
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
