// Internal device helpers of the gfx950 MWHC build library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace mphx {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
constexpr uint32_t kRoundCore = 0xFFFFFFFFu;
constexpr uint32_t kMaxDegree = 255u;
constexpr int kWave = 64;

// Error bits raised by kernels into Ctrl::err.
constexpr uint32_t kErrBadEdge = 1u;  // vertex id >= m or a repeated vertex in an edge
constexpr uint32_t kErrDegree = 2u;   // a vertex reached degree 256
constexpr uint32_t kErrValue = 4u;    // a static-function value outside [0, sigma)

// Device-side control block of one peeling run (lives in the workspace).
struct Ctrl {
    unsigned long long ftail;  // append cursor of the frontier array (all rounds back to back)
    unsigned long long ltail;  // append cursor of the layer array (all rounds back to back)
    uint32_t nrounds;          // first round whose layer was empty (UINT32_MAX while running)
    uint32_t err;              // kErr* bits
    unsigned long long aux;    // scratch counter (bijection check)
    unsigned long long claims; // (vertex, edge) claims made over all rounds
    unsigned long long degsum; // sum of all degree fields (overflow check: must be 3n)
    unsigned long long updates;  // deletes applied through update lists
    unsigned long long touched;  // records those deletes changed
    unsigned long long dups;     // pairs of 2-core edges with equal vertex triples (failure path)
    uint64_t pad[23];
};
static_assert(sizeof(Ctrl) == 256, "Ctrl is one 256-byte slot");

// Per-bucket outcome of a batched build (same layout as mphx_bucket_result).
struct BucketResult {
    uint64_t seed_used;
    uint32_t tries;
    int32_t status;  // 0 ok, 1 a 2-core remained after every try, -2 degree above 255
    uint32_t n_rounds;
    uint32_t reserved;
};
static_assert(sizeof(BucketResult) == 24, "BucketResult is 24 bytes");

// SplitMix64 output function (Steele, Lea & Flood 2014; Stafford's Mix13 constants).
__device__ __forceinline__ uint64_t fin(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// floor(z * p / 2^64), a uniform 64-bit value mapped into [0, p).
__device__ __forceinline__ uint64_t range_reduce(uint64_t z, uint64_t p) { return __umul64hi(z, p); }

// Tripartite edge of a key with digest (a, b): vertex k in part k.
__device__ __forceinline__ void edge_of_digest(uint64_t a, uint64_t b, uint64_t P, uint32_t& v0,
                                               uint32_t& v1, uint32_t& v2)
{
    v0 = (uint32_t)range_reduce(fin(a + kGamma), P);
    v1 = (uint32_t)(P + range_reduce(fin(a + 2 * kGamma), P));
    v2 = (uint32_t)(2 * P + range_reduce(fin(b + 3 * kGamma), P));
}

// ----- wave64 helpers ---------------------------------------------------------------------
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t wave_bcast64(uint64_t x, int lane)
{
    uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)x, lane);
    uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

// Reserve slots in an append-only array for the active lanes of a wave: lane j asks for
// c_j in {0, 1, 2} slots (bit0 = first slot, bit1 = second).  One atomic per wave.
// Returns the first slot of this lane (meaningless if it asked for none).
__device__ __forceinline__ uint64_t wave_append(unsigned long long* tail, bool want1, bool want2)
{
    uint64_t b1 = __ballot(want1);
    uint64_t b2 = __ballot(want2);
    uint32_t total = (uint32_t)(__popcll(b1) + __popcll(b2));
    uint64_t base = 0;
    if (total) {
        uint64_t active = __ballot(1);
        int leader = __ffsll((long long)active) - 1;
        if ((int)__lane_id() == leader)
            base = atomicAdd(tail, (unsigned long long)total);
        base = wave_bcast64(base, leader);
    }
    return base + lanes_below(b1) + lanes_below(b2);
}

// Block-wide append-only output with LDS staging.  Each call, every thread of the block offers
// up to two values; they are packed into an LDS buffer (wave ballot + lane prefix, then a
// prefix over the block's waves) and the buffer is copied out with a single atomicAdd on the
// global cursor whenever the next call could overflow it, and once at the end.  Every thread
// of the block must make the same sequence of calls (uniform loops only).  `out(i, v)` stores
// value v at global position i.
template <typename T, int kBlock, int kCap>
struct BlockAppender {
    // a push adds at most 2 * kBlock entries and flushes beyond kCap - 2 * kBlock
    static_assert(kCap >= 3 * kBlock, "buffer must hold several calls");
    T buf[kCap];
    uint32_t wtot[kBlock / kWave];
    uint32_t count;
    unsigned long long base;

    __device__ void init()
    {
        if (threadIdx.x == 0)
            count = 0;
        __syncthreads();
    }

    template <class Out>
    __device__ void flush(unsigned long long* tail, Out out)
    {
        if (threadIdx.x == 0 && count)
            base = atomicAdd(tail, (unsigned long long)count);
        __syncthreads();
        const uint32_t c = count;
        for (uint32_t i = threadIdx.x; i < c; i += kBlock)
            out(base + i, buf[i]);
        __syncthreads();
        if (threadIdx.x == 0)
            count = 0;
        __syncthreads();
    }

    template <class Out>
    __device__ void push(bool want1, T v1, bool want2, T v2, unsigned long long* tail, Out out)
    {
        const uint32_t w = threadIdx.x / kWave;
        uint64_t b1 = __ballot(want1);
        uint64_t b2 = __ballot(want2);
        if ((threadIdx.x & (kWave - 1)) == 0)
            wtot[w] = (uint32_t)(__popcll(b1) + __popcll(b2));
        __syncthreads();
        uint32_t off = count;
        for (uint32_t q = 0; q < w; q++)
            off += wtot[q];
        off += lanes_below(b1) + lanes_below(b2);
        if (want1)
            buf[off++] = v1;
        if (want2)
            buf[off] = v2;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t t = 0;
            for (uint32_t q = 0; q < kBlock / kWave; q++)
                t += wtot[q];
            count += t;
        }
        __syncthreads();
        if (count > kCap - 2 * kBlock)
            flush(tail, out);
    }
};

// ----- per-vertex packed incidence record (Section 4.1) ----------------------------------
// Each vertex keeps its degree and a combination of the ids of its incident edges from which
// the single remaining edge is read off when the degree is 1.  The paper combines the ids
// with XOR; here they are summed, the same structure over the group Z/2^40 instead of
// (Z/2)^32, so that AddEdge / DeleteEdge of edge e is ONE 64-bit atomic add of +-(2^40 + e)
// that updates degree and label together and returns a consistent (degree, label) snapshot.
// Layout: bits [40, 64) degree, bits [0, 40) sum of incident edge ids.  While the degree is
// <= 255 the sum stays below 2^40 and never carries into the degree.
struct Rec {
    static constexpr uint64_t kOne = 1ull << 40;
    __device__ static __forceinline__ uint32_t deg(uint64_t r) { return (uint32_t)(r >> 40); }
    __device__ static __forceinline__ uint32_t edge(uint64_t r) { return (uint32_t)(r & (kOne - 1)); }
    __device__ static __forceinline__ void add(uint64_t* rec, uint32_t v, uint32_t e)
    {
        atomicAdd(reinterpret_cast<unsigned long long*>(rec + v), (unsigned long long)(kOne + e));
    }
    // returns the record before the deletion
    __device__ static __forceinline__ uint64_t del(uint64_t* rec, uint32_t v, uint32_t e)
    {
        return atomicAdd(reinterpret_cast<unsigned long long*>(rec + v), (unsigned long long)(0ull - (kOne + e)));
    }
};

// Frontier entry: the only remaining edge of a vertex that reached degree 1, and that vertex's
// position in the edge (its part, for tripartite edges).
__device__ __forceinline__ uint64_t fentry(uint32_t e, uint32_t k) { return ((uint64_t)k << 32) | e; }
__device__ __forceinline__ uint32_t fentry_edge(uint64_t f) { return (uint32_t)f; }
__device__ __forceinline__ uint32_t fentry_pos(uint64_t f) { return (uint32_t)(f >> 32); }

// Per-edge peel state: 0xFFFFFFFF until claimed, then (round << 2) | hinge position.  Claims
// use atomicMin, so the lowest position among the edge's degree-1 vertices of that round wins.
constexpr uint32_t kUnclaimed = 0xFFFFFFFFu;

// Part of a vertex in the tripartite layout.
__device__ __forceinline__ uint32_t part_of(uint32_t v, uint64_t P)
{
    return (uint32_t)((uint64_t)v >= 2 * P ? 2 : ((uint64_t)v >= P ? 1 : 0));
}

// ---- byte-string keys --------------------------------------------------------------------
// Aligned 32-bit read of dword q of the byte array; the dword holding the array's last byte
// is assembled byte by byte so nothing past `total` is touched.
__device__ __forceinline__ uint32_t load_dword(const uint8_t* bytes, uint64_t q, uint64_t total)
{
    uint64_t b = q * 4;
    if (b + 4 <= total)
        return *reinterpret_cast<const uint32_t*>(bytes + b);
    uint32_t x = 0;
    for (uint32_t t = 0; t < 4; t++)
        if (b + t < total)
            x |= (uint32_t)bytes[b + t] << (8 * t);
    return x;
}

// 128-bit digest (a, b): per lane, sum of fin(w_j XOR (s_lane + j*GAMMA)) over the key's
// little-endian 8-byte words (zero padded), then fin(sum XOR s_lane XOR len).  The key's words
// are rebuilt from aligned dwords with a funnel shift.
__device__ __forceinline__ void digest_str(const uint8_t* bytes, uint64_t off, uint64_t len, uint64_t total,
                                           uint64_t sa, uint64_t sb, uint64_t& a, uint64_t& b)
{
    uint64_t A = 0, B = 0;
    const uint64_t nw = (len + 7) >> 3;
    const uint64_t q0 = off >> 2;
    const uint32_t sh = (uint32_t)(off & 3) * 8;
    // four words per step, their nine dwords loaded before any is used (one round trip)
    constexpr uint32_t kStep = 4;
    for (uint64_t j0 = 0; j0 < nw; j0 += kStep) {
        uint32_t c[2 * kStep + 1];
#pragma unroll
        for (uint32_t k = 0; k < 2 * kStep + 1; k++)
            c[k] = 2 * j0 + k <= 2 * nw ? load_dword(bytes, q0 + 2 * j0 + k, total) : 0u;
#pragma unroll
        for (uint32_t u = 0; u < kStep; u++) {
            const uint64_t j = j0 + u;
            if (j < nw) {
                const uint64_t lo = (uint64_t)c[2 * u] | ((uint64_t)c[2 * u + 1] << 32);
                uint64_t w = sh ? ((lo >> sh) | ((uint64_t)c[2 * u + 2] << (64 - sh))) : lo;
                const uint64_t rem = len - 8 * j;
                if (rem < 8)
                    w &= (1ull << (8 * rem)) - 1;
                A += fin(w ^ (sa + j * kGamma));
                B += fin(w ^ (sb + j * kGamma));
            }
        }
    }
    a = fin(A ^ sa ^ len);
    b = fin(B ^ sb ^ len);
}

// ----- MPHF evaluation (Section 3 definition, Section 5 broadword ranking) -----------------
__device__ __forceinline__ uint32_t nz_pairs(uint64_t w)
{
    return (uint32_t)__popcll((w | (w >> 1)) & 0x5555555555555555ull);
}

// One thread per output word: pack 32 codes, count the non-zero ones; 16 words (512
// vertices) per rank block are summed across 16 lanes.
__device__ __forceinline__ uint32_t code_at(const uint64_t* codes, uint32_t v)
{
    return (uint32_t)(codes[v >> 5] >> (2 * (v & 31))) & 3u;
}

__device__ __forceinline__ uint64_t rank_of(const uint64_t* codes, const uint64_t* rank, uint32_t h)
{
    // the rank sample and the block's words up to h's own, all loads issued together (the
    // words past h's are not read: they may lie past the end of the code array)
    const uint64_t r = rank[h >> 9];
    const uint32_t w0 = (h >> 9) * 16, w1 = h >> 5;
    const uint32_t below = 2 * (h & 31);
    const uint64_t mask = below ? ((1ull << below) - 1) : 0ull;
    uint32_t acc = 0;
#pragma unroll
    for (uint32_t k = 0; k < 16; k++) {
        const uint32_t w = w0 + k;
        uint64_t x = w <= w1 ? codes[w] : 0ull;
        if (w == w1)
            x &= mask;
        acc += nz_pairs(x);
    }
    return r + acc;
}

// ----- static functions (Section 3): f(x) = u[v0] + u[v1] + u[v2] mod sigma ---------------
// u[v] is a field of b bits at bit v*b of the little-endian bit string of the u64 words.
__device__ __forceinline__ uint64_t sf_field(const uint64_t* words, uint32_t b, uint32_t v)
{
    if (b == 0)
        return 0;
    const uint64_t bit = (uint64_t)v * b;
    const uint64_t w = bit >> 6;
    const uint32_t off = (uint32_t)(bit & 63);
    uint64_t x = words[w] >> off;
    if (off + b > 64)  // the field runs into the next word
        x |= words[w + 1] << (64 - off);
    return x & ((1ull << b) - 1);
}

__device__ __forceinline__ uint64_t sf_eval_edge(const uint64_t* words, uint64_t sigma, uint32_t b, uint32_t v0,
                                                 uint32_t v1, uint32_t v2)
{
    const uint64_t s = sf_field(words, b, v0) + sf_field(words, b, v1) + sf_field(words, b, v2);
    return s % sigma;
}

// ----- ranked static-function layout (Section 3: ceil(log sigma) n + gamma n + o(n) bits) ----
// Only vertices with u != 0 keep a field: bit v % 64 of marks[v / 64] says whether v has one;
// rank[j] counts the marked vertices below vertex kSfrBlock * j; the fields of the marked
// vertices follow in vertex order, b bits each, in vals.
constexpr uint32_t kSfrBlock = 1024;  // vertices per rank sample: 16 mark words, two 64-byte lines

__device__ __forceinline__ uint64_t sfr_value(const uint64_t* marks, const uint64_t* rank, const uint64_t* vals,
                                              uint32_t b, uint32_t v)
{
    const uint32_t w = v >> 6, below = v & 63;
    const uint64_t mw = marks[w];
    if (!((mw >> below) & 1))
        return 0;
    uint64_t r = rank[v / kSfrBlock] + __popcll(mw & ((1ull << below) - 1));
    const uint32_t w0 = (v / kSfrBlock) * (kSfrBlock / 64);
#pragma unroll
    for (uint32_t k = 0; k < kSfrBlock / 64 - 1; k++)
        r += w0 + k < w ? __popcll(marks[w0 + k]) : 0;
    return sf_field(vals, b, (uint32_t)r);
}

__device__ __forceinline__ uint64_t sfr_eval_edge(const uint64_t* marks, const uint64_t* rank, const uint64_t* vals,
                                                  uint64_t sigma, uint32_t b, uint32_t v0, uint32_t v1, uint32_t v2)
{
    const uint64_t s = sfr_value(marks, rank, vals, b, v0) + sfr_value(marks, rank, vals, b, v1) +
                       sfr_value(marks, rank, vals, b, v2);
    return s % sigma;
}

// ----- HEM split (Section 3): signatures, buckets by their top bits, an MPHF per bucket ------
// A u64 key's signature is 64 bits (a bijection of the key); a string key's is its whole 128-bit
// digest (a, b).  The top k bits of the first word pick the bucket; inside it the key is the
// digest pair (swap(first word), second word) -- (swap(sig), swap(sig)) for u64 keys,
// (swap(a), b) for strings, swap exchanging the 32-bit halves -- whose edge under the
// bucket's seed t is the edge of the digest (x ^ t, y ^ t).
__device__ __forceinline__ uint64_t hem_signature_u64(uint64_t key, uint64_t seed) { return fin((key ^ seed) + 4 * kGamma); }
__device__ __forceinline__ uint64_t hem_bucket_key(uint64_t sig) { return (sig << 32) | (sig >> 32); }

struct HemTables {
    const uint64_t* bucket_off;  // 2^k + 1 key offsets
    const uint64_t* code_off;    // 2^k + 1 code-word offsets
    const uint64_t* rank_off;    // 2^k + 1 rank-sample offsets
    const uint64_t* seeds;       // 2^k bucket seeds
    const uint64_t* codes;
    const uint64_t* rank;
    uint32_t k, gnum, gden;
};

__device__ __forceinline__ uint64_t eval_edge(const uint64_t* codes, const uint64_t* rank, uint32_t v0, uint32_t v1,
                                              uint32_t v2);

// f(key) from its signature's first word `top` (the bucket) and its bucket pair (x, y).
__device__ __forceinline__ uint64_t hem_eval_pair(const HemTables& t, uint64_t top, uint64_t x, uint64_t y)
{
    const uint64_t b = t.k ? top >> (64 - t.k) : 0;
    const uint64_t lo = t.bucket_off[b], nb = t.bucket_off[b + 1] - lo;
    const uint64_t num = nb * (uint64_t)t.gnum, den = 3ull * t.gden;  // nb < 2^32: no overflow
    const uint64_t P = (num + den - 1) / den;
    const uint64_t sd = t.seeds[b];
    uint32_t v0, v1, v2;
    edge_of_digest(x ^ sd, y ^ sd, P, v0, v1, v2);
    return lo + eval_edge(t.codes + t.code_off[b], t.rank + t.rank_off[b], v0, v1, v2);
}

// u64 keys: the 64-bit signature
__device__ __forceinline__ uint64_t hem_eval(const HemTables& t, uint64_t sig)
{
    const uint64_t x = hem_bucket_key(sig);
    return hem_eval_pair(t, sig, x, x);
}

// string keys: the 128-bit digest (a, b)
__device__ __forceinline__ uint64_t hem_eval_digest(const HemTables& t, uint64_t a, uint64_t b)
{
    return hem_eval_pair(t, a, hem_bucket_key(a), b);
}

__device__ __forceinline__ uint64_t eval_edge(const uint64_t* codes, const uint64_t* rank, uint32_t v0, uint32_t v1,
                                              uint32_t v2)
{
    uint32_t s = (code_at(codes, v0) % 3 + code_at(codes, v1) % 3 + code_at(codes, v2) % 3) % 3;
    uint32_t h = s == 0 ? v0 : (s == 1 ? v1 : v2);
    return rank_of(codes, rank, h);
}

}  // namespace mphx
