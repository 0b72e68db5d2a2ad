// Batched MWHC builds: many independent key buckets in one persistent launch.
//
// Each workgroup repeatedly takes the next bucket from a device queue (buckets ordered by
// decreasing size, so the longest jobs start first) and runs the whole build of that bucket
// by itself: hash (Section 3, tripartite as in Section 4.3), degree/label records (Section
// 4.1), synchronous peeling rounds (Section 4.2) separated by workgroup barriers, a new seed
// while a 2-core remains, assignment along the layers in reverse round order (Section 4.3),
// then the packed codes and rank samples (Section 5).  Buckets never wait for each other, so
// the kernel needs no grid-wide synchronisation and ends when the queue is empty.
//
// A bucket's state lives in a per-workgroup slot of global memory sized for the largest
// bucket; a bucket of up to 10^6 keys keeps its state within a few tens of MB, which stays in
// L2 / the MALL while the workgroup works on it.  Edges are recomputed from the key whenever
// needed (three SplitMix64 finalisers) instead of being stored.
#include "common.h"
#include "launch.h"

namespace mphx {

struct BatchArgs {
    const uint64_t* keys;
    const uint64_t* bucket_off;  // B + 1
    const uint32_t* order;       // B bucket ids, processing order
    uint32_t B;
    uint64_t seed;
    uint32_t gnum, gden, max_tries;
    const uint64_t* code_off;    // B + 1 word offsets into codes
    const uint64_t* rank_off;    // B + 1 offsets into rank
    uint64_t* codes;
    uint64_t* rank;
    BucketResult* results;
    uint8_t* slots;
    uint64_t slot_bytes;
    uint64_t max_n;              // largest bucket a slot can hold
    unsigned int* next;          // queue cursor
};

__device__ __forceinline__ uint64_t part_size_dev(uint64_t n, uint32_t gnum, uint32_t gden)
{
    // n < 2^32 and gnum < 2^32: the product fits in 64 bits
    uint64_t num = n * (uint64_t)gnum, den = 3ull * gden;
    return (num + den - 1) / den;
}

// Slot layout for a bucket of n keys and m vertices (offsets in bytes, 256-aligned pieces).
struct SlotLayout {
    uint64_t* rec;      // m
    uint32_t* front;    // m (codes as bytes after peeling)
    uint32_t* layer;    // n
    uint32_t* claim;    // ceil(n/4) words of claim bytes
    uint32_t* lstart;   // n + 2 layer starts
    uint32_t* bcount;   // ceil(m/512)
};

__host__ __device__ __forceinline__ uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

__host__ __device__ inline uint64_t slot_layout(uint8_t* base, uint64_t n, uint64_t m, SlotLayout* L)
{
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        uint8_t* p = base + off;
        off = align256(off + bytes);
        return p;
    };
    uint8_t* rec = take(8 * m);
    uint8_t* front = take(4 * m);
    uint8_t* layer = take(4 * n);
    uint8_t* claim = take(4 * ((n + 3) / 4));
    uint8_t* lstart = take(4 * (n + 2));
    uint8_t* bcount = take(4 * ((m + 511) / 512));
    if (L) {
        L->rec = reinterpret_cast<uint64_t*>(rec);
        L->front = reinterpret_cast<uint32_t*>(front);
        L->layer = reinterpret_cast<uint32_t*>(layer);
        L->claim = reinterpret_cast<uint32_t*>(claim);
        L->lstart = reinterpret_cast<uint32_t*>(lstart);
        L->bcount = reinterpret_cast<uint32_t*>(bcount);
    }
    return off;
}

uint64_t batch_slot_bytes(uint64_t max_n, uint32_t gnum, uint32_t gden)
{
    unsigned __int128 num = (unsigned __int128)max_n * gnum, den = (unsigned __int128)3 * gden;
    uint64_t P = (uint64_t)((num + den - 1) / den);
    return slot_layout(nullptr, max_n, 3 * P, nullptr);
}

// A bucket's state is read and written by exactly one workgroup, so its atomics and the loads
// of atomically updated words may use workgroup scope (kScope = __HIP_MEMORY_SCOPE_WORKGROUP)
// instead of agent scope; both are correct and give identical results.  Loads of atomically
// updated words always go through these helpers, never a plain load that could hit a stale L1
// line.
template <int kScope>
struct Sc {
    __device__ static __forceinline__ uint64_t ld(const uint64_t* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, kScope); }
    __device__ static __forceinline__ uint32_t ld(const uint32_t* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, kScope); }
    // degree before adding edge e at v (the batched build checks degrees as it goes)
    __device__ static __forceinline__ uint32_t rec_add(uint64_t* rec, uint32_t v, uint32_t e)
    {
        return Rec::deg(__hip_atomic_fetch_add(rec + v, Rec::kOne + e, __ATOMIC_RELAXED, kScope));
    }
    __device__ static __forceinline__ uint64_t rec_del(uint64_t* rec, uint32_t v, uint32_t e)
    {
        return __hip_atomic_fetch_add(rec + v, 0ull - (Rec::kOne + e), __ATOMIC_RELAXED, kScope);
    }
    __device__ static __forceinline__ uint32_t fetch_or(uint32_t* p, uint32_t x)
    {
        return __hip_atomic_fetch_or(p, x, __ATOMIC_RELAXED, kScope);
    }
    __device__ static __forceinline__ uint32_t claim_mask(const uint32_t* claim, uint32_t e)
    {
        return (ld(claim + (e >> 2)) >> (8 * (e & 3))) & 0xFFu;
    }
};

// Workgroup-wide exclusive scan of count values (in place is not needed: in -> out).
template <int kBlock>
__device__ void block_exclusive_scan(const uint32_t* in, uint64_t* out, uint32_t count)
{
    __shared__ uint64_t s_wsum[kBlock / kWave];
    __shared__ uint64_t s_carry;
    if (threadIdx.x == 0)
        s_carry = 0;
    __syncthreads();
    const uint32_t lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    for (uint32_t base = 0; base < count; base += kBlock) {
        uint32_t i = base + threadIdx.x;
        uint64_t x = i < count ? in[i] : 0;
        uint64_t incl = x;
        for (uint32_t d = 1; d < kWave; d <<= 1) {
            uint64_t y = __shfl_up(incl, d, kWave);
            if (lane >= d)
                incl += y;
        }
        if (lane == kWave - 1)
            s_wsum[w] = incl;
        __syncthreads();
        uint64_t pre = s_carry;
        for (uint32_t q = 0; q < w; q++)
            pre += s_wsum[q];
        if (i < count)
            out[i] = pre + incl - x;
        __syncthreads();
        if (threadIdx.x == kBlock - 1)
            s_carry = pre + incl;
        __syncthreads();
    }
}

// Workgroup-local append: one LDS atomic per wave.
__device__ __forceinline__ uint32_t block_append(uint32_t* counter, bool want1, bool want2)
{
    uint64_t b1 = __ballot(want1), b2 = __ballot(want2);
    uint32_t total = (uint32_t)(__popcll(b1) + __popcll(b2));
    uint32_t base = 0;
    if (total) {
        int leader = __ffsll((long long)__ballot(1)) - 1;
        if ((int)__lane_id() == leader)
            base = atomicAdd(counter, total);
        base = __builtin_amdgcn_readlane(base, leader);
    }
    return base + lanes_below(b1) + lanes_below(b2);
}

__device__ __forceinline__ void edge_of_key(uint64_t key, uint64_t seed, uint64_t P, uint32_t& v0, uint32_t& v1,
                                            uint32_t& v2)
{
    uint64_t s = key ^ seed;
    edge_of_digest(s, s, P, v0, v1, v2);
}

template <int kBlock, int kScope>
__device__ void build_bucket(const BatchArgs& a, uint32_t b, uint8_t* slot)
{
    __shared__ uint32_t s_ftail, s_ltail, s_err;
    const uint64_t k0 = a.bucket_off[b];
    const uint64_t n64 = a.bucket_off[b + 1] - k0;
    if (n64 > a.max_n) {  // larger than the slots were sized for: report, touch nothing
        if (threadIdx.x == 0) {
            a.results[b].seed_used = a.seed;
            a.results[b].tries = 0;
            a.results[b].status = -1;
            a.results[b].n_rounds = 0;
        }
        __syncthreads();
        return;
    }
    const uint32_t n = (uint32_t)n64;
    const uint64_t* keys = a.keys + k0;
    const uint64_t P = part_size_dev(n, a.gnum, a.gden);
    const uint32_t m = (uint32_t)(3 * P);
    SlotLayout L;
    slot_layout(slot, n, m, &L);
    const uint32_t tid = threadIdx.x;

    uint32_t t = 0, nrounds = 0;
    bool ok = false;
    int status = 0;
    uint64_t sd = a.seed;
    for (t = 0; t < a.max_tries; t++) {
        sd = a.seed + t;
        for (uint32_t v = tid; v < m; v += kBlock)
            L.rec[v] = 0;
        for (uint32_t w = tid; w < (n + 3) / 4; w += kBlock)
            L.claim[w] = 0;
        if (tid == 0) {
            s_ftail = 0;
            s_ltail = 0;
            s_err = 0;
        }
        __syncthreads();
        // records (AddEdge at the three vertices)
        for (uint32_t i = tid; i < n; i += kBlock) {
            uint32_t v0, v1, v2;
            edge_of_key(keys[i], sd, P, v0, v1, v2);
            uint32_t d = Sc<kScope>::rec_add(L.rec, v0, i);
            d = max(d, Sc<kScope>::rec_add(L.rec, v1, i));
            d = max(d, Sc<kScope>::rec_add(L.rec, v2, i));
            if (d >= kMaxDegree)
                s_err = 1;
        }
        __syncthreads();
        if (s_err) {
            status = -2;  // degree above 255: no seed helps a duplicate-heavy bucket
            break;
        }
        // round-0 frontier
        for (uint32_t base = 0; base < m; base += kBlock) {
            uint32_t v = base + tid;
            bool one = v < m && Rec::deg(Sc<kScope>::ld(L.rec + v)) == 1;
            uint32_t pos = block_append(&s_ftail, one, false);
            if (one)
                L.front[pos] = v;
        }
        __syncthreads();
        uint32_t flo = 0, fhi = s_ftail, r = 0;
        L.lstart[0] = 0;  // single writer is fine: every thread writes the same value
        for (;;) {
            const uint32_t llo = s_ltail;
            // claim
            for (uint32_t base = flo; base < fhi; base += kBlock) {
                uint32_t i = base + tid;
                bool first = false;
                uint32_t e = 0;
                if (i < fhi) {
                    uint32_t v = L.front[i];
                    uint64_t x = Sc<kScope>::ld(L.rec + v);
                    if (Rec::deg(x) == 1 && Rec::edge(x) < n) {
                        e = Rec::edge(x);
                        uint32_t k = part_of(v, P);
                        uint32_t sh = 8 * (e & 3);
                        uint32_t old = Sc<kScope>::fetch_or(&L.claim[e >> 2], (1u << k) << sh);
                        first = ((old >> sh) & 0xFFu) == 0;
                    }
                }
                uint32_t pos = block_append(&s_ltail, first, false);
                if (first)
                    L.layer[pos] = e;
            }
            __syncthreads();
            const uint32_t lhi = s_ltail;
            if (tid == 0)
                L.lstart[r + 1] = lhi;
            if (lhi == llo)
                break;
            // apply
            for (uint32_t base = llo; base < lhi; base += kBlock) {
                uint32_t i = base + tid;
                uint32_t p0 = 0, p1 = 0, np = 0;
                if (i < lhi) {
                    uint32_t e = L.layer[i];
                    uint32_t mask = Sc<kScope>::claim_mask(L.claim, e);
                    uint32_t v[3];
                    edge_of_key(keys[e], sd, P, v[0], v[1], v[2]);
#pragma unroll
                    for (int k = 0; k < 3; k++) {
                        if (!(mask & (1u << k)) && Rec::deg(Sc<kScope>::rec_del(L.rec, v[k], e)) == 2) {
                            if (np) p1 = v[k]; else p0 = v[k];
                            np++;
                        }
                    }
                }
                uint32_t pos = block_append(&s_ftail, np >= 1, np >= 2);
                if (np >= 1)
                    L.front[pos] = p0;
                if (np >= 2)
                    L.front[pos + 1] = p1;
            }
            __syncthreads();
            flo = fhi;
            fhi = s_ftail;
            r++;
        }
        nrounds = r;
        if (s_ltail == n) {
            ok = true;
            break;
        }
        __syncthreads();
    }
    if (!ok) {
        if (tid == 0) {
            a.results[b].seed_used = sd;
            a.results[b].tries = t < a.max_tries ? t + 1 : a.max_tries;
            a.results[b].status = status ? status : 1;
            a.results[b].n_rounds = nrounds;
        }
        __syncthreads();
        return;
    }
    // assignment, last layer first; codes as bytes in the frontier area
    uint8_t* code8 = reinterpret_cast<uint8_t*>(L.front);
    for (uint32_t v = tid; v < m; v += kBlock)
        code8[v] = 0;
    __syncthreads();
    for (int32_t r = (int32_t)nrounds - 1; r >= 0; r--) {
        const uint32_t lo = L.lstart[r], hi = L.lstart[r + 1];
        for (uint32_t i = lo + tid; i < hi; i += kBlock) {
            uint32_t e = L.layer[i];
            uint32_t k = __builtin_ctz(Sc<kScope>::claim_mask(L.claim, e));
            uint32_t v[3];
            edge_of_key(keys[e], sd, P, v[0], v[1], v[2]);
            uint32_t va = v[(k + 1) % 3], vb = v[(k + 2) % 3];
            uint32_t ca = code8[va], cb = code8[vb];
            uint32_t g = (k + 6 - (ca == 3 ? 0 : ca) - (cb == 3 ? 0 : cb)) % 3;
            code8[v[k]] = (uint8_t)(g ? g : 3);
        }
        __syncthreads();
    }
    // pack codes, count per 512 vertices, exclusive scan into the rank samples
    uint64_t* codes = a.codes + a.code_off[b];
    uint64_t* rank = a.rank + a.rank_off[b];
    const uint32_t nwords = (m + 31) / 32, nblocks = (m + 511) / 512;
    for (uint32_t base = 0; base < nwords; base += kBlock) {
        uint32_t w = base + tid;
        uint64_t x = 0;
        if (w < nwords) {
            if (32 * w + 32 <= m) {
                const uint4* p = reinterpret_cast<const uint4*>(code8 + 32 * w);
                uint4 c0 = p[0], c1 = p[1];
                uint32_t d[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
#pragma unroll
                for (int q = 0; q < 8; q++)
#pragma unroll
                    for (int u = 0; u < 4; u++)
                        x |= (uint64_t)((d[q] >> (8 * u)) & 3u) << (2 * (4 * q + u));
            } else {
                for (uint32_t q = 0; 32 * w + q < m; q++)
                    x |= (uint64_t)(code8[32 * w + q] & 3u) << (2 * q);
            }
            codes[w] = x;
        }
        uint32_t c = nz_pairs(x);
        c += __shfl_xor(c, 1, 16);
        c += __shfl_xor(c, 2, 16);
        c += __shfl_xor(c, 4, 16);
        c += __shfl_xor(c, 8, 16);
        if (w < nwords && (w & 15) == 0)
            L.bcount[w >> 4] = c;
    }
    __syncthreads();
    block_exclusive_scan<kBlock>(L.bcount, rank, nblocks);
    if (tid == 0) {
        a.results[b].seed_used = sd;
        a.results[b].tries = t + 1;
        a.results[b].status = 0;
        a.results[b].n_rounds = nrounds;
    }
    __syncthreads();
}

template <int kBlock, int kScope>
__global__ __launch_bounds__(kBlock) void k_batch(BatchArgs a)
{
    __shared__ uint32_t s_idx;
    uint8_t* slot = a.slots + (uint64_t)blockIdx.x * a.slot_bytes;
    for (;;) {
        if (threadIdx.x == 0)
            s_idx = atomicAdd(a.next, 1u);
        __syncthreads();
        const uint32_t idx = s_idx;
        __syncthreads();
        if (idx >= a.B)
            break;
        build_bucket<kBlock, kScope>(a, a.order[idx], slot);
    }
}

hipError_t launch_batch(const BatchLaunch& L, hipStream_t s)
{
    BatchArgs a;
    a.keys = L.keys;
    a.bucket_off = L.bucket_off;
    a.order = L.order;
    a.B = L.B;
    a.seed = L.seed;
    a.gnum = L.gnum;
    a.gden = L.gden;
    a.max_tries = L.max_tries;
    a.code_off = L.code_off;
    a.rank_off = L.rank_off;
    a.codes = L.codes;
    a.rank = L.rank;
    a.results = L.results;
    a.slots = L.slots;
    a.slot_bytes = L.slot_bytes;
    a.max_n = L.max_n;
    a.next = L.next;
    hipError_t err = launch_zero(L.next, sizeof(unsigned int), s);
    if (err != hipSuccess) return err;
    constexpr int W = __HIP_MEMORY_SCOPE_WORKGROUP, A = __HIP_MEMORY_SCOPE_AGENT;
    const bool wg = L.wg_scope;
    switch (L.block) {
    case 256: wg ? k_batch<256, W><<<L.grid, 256, 0, s>>>(a) : k_batch<256, A><<<L.grid, 256, 0, s>>>(a); break;
    case 512: wg ? k_batch<512, W><<<L.grid, 512, 0, s>>>(a) : k_batch<512, A><<<L.grid, 512, 0, s>>>(a); break;
    case 1024: wg ? k_batch<1024, W><<<L.grid, 1024, 0, s>>>(a) : k_batch<1024, A><<<L.grid, 1024, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mphx
