// Batched MWHC builds: many independent key sets ("buckets") in one persistent launch.
//
// Each workgroup repeatedly takes the next bucket from a device queue (buckets ordered by
// decreasing size, so the longest jobs start first) and runs the whole build of that bucket by
// itself: hash (Section 3, tripartite as in Section 4.3), degree/label records (Section 4.1),
// synchronous peeling rounds (Section 4.2) separated by workgroup barriers, a new seed while a
// 2-core remains, assignment along the layers in reverse round order (Section 4.3), then the
// packed codes and rank samples (Section 5).  Buckets never wait for each other, so the kernel
// needs no grid-wide synchronisation and ends when the queue is empty.
//
// Every bucket is described by its own key pointers and output pointers, so a batch can be
// one array split by offsets (mphx_build_batch_u64) or unrelated requests gathered by the
// build server.  The rounds follow the plain path's design: the atomic that takes a vertex
// from degree 2 to 1 returns the vertex's remaining edge, which is claimed for the next round
// at once with atomicMin((round << 2) | position) on the edge's state word (a claim on an edge
// that leaves in the current round cannot lower its state); layer slots are rewritten with
// the edge's vertices hinge first for the assignment.  u64 keys recompute their edge from the
// key when needed; string keys keep their edges in the slot.
#include "common.h"
#include "batch.h"
#include "launch.h"

namespace mphx {

__device__ __forceinline__ uint64_t part_size_dev(uint64_t n, uint32_t gnum, uint32_t gden)
{
    // n < 2^32 and gnum < 2^32: the product fits in 64 bits
    uint64_t num = n * (uint64_t)gnum, den = 3ull * gden;
    return (num + den - 1) / den;
}

// Slot layout for a bucket of n keys and m vertices (256-aligned pieces).
struct SlotLayout {
    uint64_t* rec;     // m records (codes as bytes after peeling)
    uint3* slots;      // n layer slots
    uint32_t* state;   // n edge states
    uint32_t* lstart;  // n + 2 layer starts
    uint32_t* bcount;  // ceil(m/512)
    uint3* edges;      // n edges (string keys only)
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
    uint8_t* slots = take(12 * n);
    uint8_t* state = take(4 * n);
    uint8_t* lstart = take(4 * (n + 2));
    uint8_t* bcount = take(4 * ((m + 511) / 512));
    uint8_t* edges = take(12 * n);
    if (L) {
        L->rec = reinterpret_cast<uint64_t*>(rec);
        L->slots = reinterpret_cast<uint3*>(slots);
        L->state = reinterpret_cast<uint32_t*>(state);
        L->lstart = reinterpret_cast<uint32_t*>(lstart);
        L->bcount = reinterpret_cast<uint32_t*>(bcount);
        L->edges = reinterpret_cast<uint3*>(edges);
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
    __device__ static __forceinline__ uint32_t fetch_min(uint32_t* p, uint32_t x)
    {
        return __hip_atomic_fetch_min(p, x, __ATOMIC_RELAXED, kScope);
    }
    __device__ static __forceinline__ uint32_t fetch_and(uint32_t* p, uint32_t x)
    {
        return __hip_atomic_fetch_and(p, x, __ATOMIC_RELAXED, kScope);
    }
};

// Workgroup-wide exclusive scan of count values (in -> out).
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

// Workgroup-local append: one LDS atomic per wave; lane j asks for want1 + want2 slots
// (want2 implies want1).
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

// In-place exclusive scan of count <= kBatchMaxBuckets LDS words; returns the total.
template <int kBlock>
__device__ uint32_t lds_exclusive_scan(uint32_t* a, uint32_t count, uint32_t* wtot)
{
    const uint32_t per = (count + kBlock - 1) / kBlock;
    const uint32_t b0 = threadIdx.x * per, b1 = min(b0 + per, count);
    uint32_t sum = 0;
    for (uint32_t j = b0; j < b1; j++)
        sum += a[j];
    const uint32_t lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    uint32_t incl = sum;
    for (uint32_t d = 1; d < kWave; d <<= 1) {
        uint32_t y = __shfl_up(incl, d, kWave);
        if (lane >= d)
            incl += y;
    }
    if (lane == kWave - 1)
        wtot[w] = incl;
    __syncthreads();
    uint32_t pre = 0, total = 0;
    for (uint32_t q = 0; q < kBlock / kWave; q++) {
        pre += q < w ? wtot[q] : 0u;
        total += wtot[q];
    }
    pre += incl - sum;
    for (uint32_t j = b0; j < b1; j++) {
        const uint32_t x = a[j];
        a[j] = pre;
        pre += x;
    }
    __syncthreads();
    return total;
}

// The partitioned record build works on LDS tiles of records and parts of at most
// kBatchMaxBuckets tiles; larger parts fall back to atomics.  Vertices per tile: 8192 (64 KB
// of records) for 1024-thread workgroups; 4096 for smaller ones, whose ~48 KB of LDS lets
// three share a compute unit.
template <int kBlock>
constexpr uint32_t batch_tile() { return kBlock >= 1024 ? 8192u : 4096u; }
constexpr uint32_t kBatchMaxBuckets = 2048;
// LDS shared by the two bucket builds: the partitioned record build's tile, counts and bounds,
// or a whole bucket's 4-byte records and edge states.  1024-thread workgroups take 158 KB (one
// per compute unit), 512-thread ones 78 KB (two), 256-thread ones 48 KB (three).
template <int kBlock>
constexpr uint32_t batch_part_bytes() { return batch_tile<kBlock>() * 8 + (2 * kBatchMaxBuckets + 1) * 4; }
template <int kBlock>
constexpr uint32_t batch_lds_bytes()
{
    return kBlock >= 1024 ? 158u * 1024 : (kBlock >= 512 ? 78u * 1024 : batch_part_bytes<kBlock>());
}
// A bucket whose records (m words) and states (n words) fit runs entirely in LDS.
template <int kBlock>
__device__ __forceinline__ bool bucket_fits_lds(uint64_t n, uint64_t m)
{
    return ((m + 3) & ~3ull) + n <= batch_lds_bytes<kBlock>() / 4;
}

// Digest of key i under seed sd for keys given by words: a u64 key x is the digest (x ^ sd,
// x ^ sd), a digest pair (x, y) the digest (x ^ sd, y ^ sd).
__device__ __forceinline__ void key_digest(const BatchArgs& a, const BucketDesc& d, uint32_t i, uint64_t sd,
                                           uint64_t& x, uint64_t& y)
{
    if (a.pairs) {
        const ulonglong2 w = reinterpret_cast<const ulonglong2*>(d.keys)[i];
        x = w.x ^ sd;
        y = w.y ^ sd;
    } else {
        x = y = d.keys[i] ^ sd;
    }
}

// Part-k local vertex of key i: recomputed from a key given by words, read from the stored
// edge else.
__device__ __forceinline__ uint32_t bucket_local(const BatchArgs& a, const BucketDesc& d, const SlotLayout& L,
                                                 uint32_t i, uint64_t sd, uint64_t P, uint32_t k)
{
    if (d.keys) {
        uint64_t x, y;
        key_digest(a, d, i, sd, x, y);
        return (uint32_t)range_reduce(fin((k == 2 ? y : x) + (uint64_t)(k + 1) * kGamma), P);
    }
    const uint3 ev = L.edges[i];
    return (k == 0 ? ev.x : (k == 1 ? ev.y : ev.z)) - (uint32_t)(k * P);
}

// The three part-local vertices of a key given by words, from its digest (x, y) under the try's
// seed (bucket_local for k = 0, 1, 2).
__device__ __forceinline__ uint3 digest_locals(uint64_t x, uint64_t y, uint64_t P)
{
    return make_uint3((uint32_t)range_reduce(fin(x + kGamma), P), (uint32_t)range_reduce(fin(x + 2 * kGamma), P),
                      (uint32_t)range_reduce(fin(y + 3 * kGamma), P));
}

// Edge of key i of a bucket: recomputed for keys given by words, stored for string keys.
__device__ __forceinline__ uint3 bucket_edge(const BatchArgs& a, const BucketDesc& d, const SlotLayout& L, uint32_t i,
                                             uint64_t sd, uint64_t P)
{
    if (d.keys) {
        uint64_t x, y;
        key_digest(a, d, i, sd, x, y);
        uint32_t v0, v1, v2;
        edge_of_digest(x, y, P, v0, v1, v2);
        return make_uint3(v0, v1, v2);
    }
    return L.edges[i];
}

__device__ __forceinline__ void write_result(BucketResult* r, uint64_t seed_used, uint32_t tries, int32_t status,
                                             uint32_t rounds)
{
    r->seed_used = seed_used;
    r->tries = tries;
    r->status = status;
    r->n_rounds = rounds;
}

// Codes (one byte per vertex, code8 in device memory or LDS) packed 2 bits per vertex into
// d.codes, counted per 512 vertices and scanned into the rank samples d.rank.
template <int kBlock>
__device__ void pack_codes(const uint8_t* code8, uint32_t m, const BucketDesc& d, const SlotLayout& L)
{
    const uint32_t tid = threadIdx.x;
    const uint32_t nwords = (m + 31) / 32, nblocks = (m + 511) / 512;
    for (uint32_t base = 0; base < nwords; base += kBlock) {
        uint32_t w = base + tid;
        uint64_t x = 0;
        if (w < nwords) {
            if (32 * w + 32 <= m) {
                const uint4* p = reinterpret_cast<const uint4*>(code8 + 32 * w);
                uint4 q0 = p[0], q1 = p[1];
                uint32_t dw[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
                for (int q = 0; q < 8; q++)
#pragma unroll
                    for (int u = 0; u < 4; u++)
                        x |= (uint64_t)((dw[q] >> (8 * u)) & 3u) << (2 * (4 * q + u));
            } else {
                for (uint32_t q = 0; 32 * w + q < m; q++)
                    x |= (uint64_t)(code8[32 * w + q] & 3u) << (2 * q);
            }
            d.codes[w] = x;
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
    block_exclusive_scan<kBlock>(L.bcount, d.rank, nblocks);
}

// The batch clock: per-phase workgroup time (wall-clock ticks, summed over workgroups) and work
// counts, added by the kernel instantiated with kClock (BatchArgs::clock); entry 0 is reserved
// for the tick rate, which the host fills in when it reads the clock.
enum : int {
    kClRecords = 1, kClDeletes, kClGroup, kClResolve, kClOther, kClAssign, kClPack, kClLds, kClQueue, kClLife,
    kClBuckets, kClKeys, kClTries, kClRounds, kClDels, kClRecs, kClLdsBuckets, kClLdsKeys
};
static_assert(kClLdsKeys + 1 == kBatchClockEntries, "batch clock entries");
__device__ unsigned long long g_batch_clock[kBatchClockEntries];

// Thread 0 marks phase boundaries right after workgroup barriers; the time since the last mark
// goes to the phase that ended.  Without kOn every member is empty.
template <bool kOn>
struct PhaseClock {
    uint64_t t = 0, recs = 0, dels = 0;
    uint64_t acc[kClPack + 1] = {};
    __device__ __forceinline__ void start()
    {
        if constexpr (kOn)
            t = wall_clock64();
    }
    __device__ __forceinline__ void mark(int k)
    {
        if constexpr (kOn) {
            if (threadIdx.x == 0) {
                const uint64_t t2 = wall_clock64();
                acc[k] += t2 - t;
                t = t2;
            }
        }
    }
    __device__ __forceinline__ void deletes(uint32_t c)
    {
        if constexpr (kOn)
            dels += c;
    }
    __device__ __forceinline__ void records(uint32_t c)
    {
        if constexpr (kOn)
            recs += c;
    }
    // every thread of the workgroup calls this once per bucket
    __device__ __forceinline__ void flush(uint64_t n, uint32_t tries, uint32_t rounds)
    {
        if constexpr (kOn) {
            uint64_t dsum = dels;
            for (int o = kWave / 2; o > 0; o >>= 1)
                dsum += __shfl_xor(dsum, o, kWave);
            if ((threadIdx.x & (kWave - 1)) == 0 && dsum)
                atomicAdd(&g_batch_clock[kClDels], (unsigned long long)dsum);
            dels = 0;
            if (threadIdx.x == 0) {
                for (int k = kClRecords; k <= kClPack; k++)
                    atomicAdd(&g_batch_clock[k], (unsigned long long)acc[k]);
                atomicAdd(&g_batch_clock[kClBuckets], 1ull);
                atomicAdd(&g_batch_clock[kClKeys], (unsigned long long)n);
                atomicAdd(&g_batch_clock[kClTries], (unsigned long long)tries);
                atomicAdd(&g_batch_clock[kClRounds], (unsigned long long)rounds);
                atomicAdd(&g_batch_clock[kClRecs], (unsigned long long)recs);
            }
        }
    }
};

template <int kBlock, int kScope, bool kClock>
__device__ void build_bucket(const BatchArgs& a, const BucketDesc& d, uint8_t* slot, uint8_t* lds)
{
    using S = Sc<kScope>;
    PhaseClock<kClock> clk;
    clk.start();
    constexpr uint32_t kBatchTile = batch_tile<kBlock>();
    __shared__ uint32_t s_ltail, s_err, s_degsum, s_ctail;
    __shared__ uint32_t s_l0part[3];  // where layer 0's appends of parts 0, 1, 2 end
    __shared__ uint32_t s_wtot[kBlock / kWave];
    unsigned long long* s_tab = reinterpret_cast<unsigned long long*>(lds);  // kBatchTile records
    uint32_t* s_cnt = reinterpret_cast<uint32_t*>(s_tab + kBatchTile);       // kBatchMaxBuckets
    uint32_t* s_bnd = s_cnt + kBatchMaxBuckets;                              // kBatchMaxBuckets + 1
    if (threadIdx.x == 0)
        s_degsum = 0;
    const uint32_t tid = threadIdx.x;
    if (d.n > a.max_n) {  // larger than the slots were sized for: report, touch nothing
        if (tid == 0)
            write_result(d.result, d.seed, 0, -1, 0);
        __syncthreads();
        return;
    }
    const uint32_t n = (uint32_t)d.n;
    const uint64_t P = part_size_dev(n, a.gnum, a.gden);
    const uint32_t m = (uint32_t)(3 * P);
    SlotLayout L;
    slot_layout(slot, n, m, &L);
    const uint64_t total = d.keys ? 0 : d.offs[n];
    // packed (vertex in tile, key) words: tiles of kPackTile vertices, keys below 2^20
    constexpr uint32_t kPackBits = 12, kPackTile = 1u << kPackBits;
    const uint32_t nbp = (uint32_t)((P + kPackTile - 1) / kPackTile);

    uint32_t t = 0, nrounds = 0;
    bool ok = false;
    int status = 0;
    uint64_t sd = d.seed;
    for (t = 0; t < a.max_tries; t++) {
        sd = d.seed + t;
        bool l0_in_slot = false;  // layer 0's slots carry their hinge part (partitioned build)
        for (uint32_t e = tid; e < n; e += kBlock)
            L.state[e] = kUnclaimed;
        if (tid == 0) {
            s_ltail = 0;
            s_err = 0;
        }
        const uint64_t sa = fin(sd + kGamma), sb = fin(sd + 2 * kGamma);
        if (!d.keys) {  // string keys: digest once, keep the edges
            for (uint32_t i = tid; i < n; i += kBlock) {
                uint64_t o0 = d.offs[i], o1 = d.offs[i + 1], ha, hb;
                digest_str(d.bytes, o0, o1 - o0, total, sa, sb, ha, hb);
                uint3 ev;
                edge_of_digest(ha, hb, P, ev.x, ev.y, ev.z);
                L.edges[i] = ev;
            }
        }
        __syncthreads();
        const uint32_t nbk = (uint32_t)((P + kBatchTile - 1) / kBatchTile);
        // Records of part k's tile at v0 (cnt vertices, accumulated in s_tab) written once; round
        // 0 rides along: a vertex of degree 1 in part k claims its edge unless a lower part
        // already did, so the hinge is the lowest part and each edge enters layer 0 once (the
        // parts run in order).  The claimed edges are appended to stage.
        auto write_tile = [&](uint32_t k, uint64_t v0, uint32_t cnt, uint32_t* stage, uint32_t& degsum) {
            for (uint32_t base = 0; base < cnt; base += kBlock) {
                const uint32_t v = base + tid;
                bool first = false;
                uint32_t e = 0;
                if (v < cnt) {
                    const uint64_t x = s_tab[v];
                    const uint32_t dg = Rec::deg(x);
                    degsum += dg;
                    if (dg > kMaxDegree)
                        s_err = 1;
                    L.rec[(uint64_t)k * P + v0 + v] = x;
                    if (dg == 1 && Rec::edge(x) < n) {
                        e = Rec::edge(x);
                        first = k == 0 || L.state[e] == kUnclaimed;
                        if (first)
                            L.state[e] = k;
                    }
                }
                const uint32_t pos = block_append(&s_ltail, first, false);
                if (first && pos < n)  // more only from wrapped records, flagged below
                    stage[pos] = e;
            }
        };
        // every degree field of part k at most 255 and their total n (no field wrapped); the
        // end of part k's layer-0 appends
        auto close_part = [&](uint32_t k, uint32_t degsum) {
            if (degsum)
                atomicAdd(&s_degsum, degsum);
            __syncthreads();
            if (tid == 0) {
                if (s_degsum != n)
                    s_err = 1;
                s_degsum = 0;
                s_l0part[k] = s_ltail;
            }
            __syncthreads();
        };
        constexpr uint32_t kU = 4;  // keys or pairs each thread loads before using any of them
        if (d.keys && n <= (1u << (32 - kPackBits)) && 3 * nbp <= kBatchMaxBuckets) {
            // Keys given by words: all three parts partitioned in one pass.  Each key's three
            // (vertex in tile, key) pairs are packed in a word (12 + 20 bits) and grouped by
            // (part, tile of kPackTile vertices); the keys are read and hashed twice in all.
            // The pairs (12n bytes) fill the slot area, layer 0 is staged in the free edge area.
            uint32_t* pairs = reinterpret_cast<uint32_t*>(L.slots);
            uint32_t* stage = reinterpret_cast<uint32_t*>(L.edges);
            for (uint32_t b = tid; b < 3 * nbp; b += kBlock)
                s_cnt[b] = 0;
            __syncthreads();
            for (uint32_t i0 = tid; i0 < n; i0 += kU * kBlock) {
                uint64_t x[kU], y[kU];
                for (uint32_t q = 0; q < kU; q++)
                    if (i0 + q * kBlock < n)
                        key_digest(a, d, i0 + q * kBlock, sd, x[q], y[q]);
                for (uint32_t q = 0; q < kU; q++) {
                    if (i0 + q * kBlock < n) {
                        const uint3 u = digest_locals(x[q], y[q], P);
                        atomicAdd(&s_cnt[u.x >> kPackBits], 1u);
                        atomicAdd(&s_cnt[nbp + (u.y >> kPackBits)], 1u);
                        atomicAdd(&s_cnt[2 * nbp + (u.z >> kPackBits)], 1u);
                    }
                }
            }
            __syncthreads();
            lds_exclusive_scan<kBlock>(s_cnt, 3 * nbp, s_wtot);
            for (uint32_t b = tid; b < 3 * nbp; b += kBlock)
                s_bnd[b] = s_cnt[b];
            if (tid == 0)
                s_bnd[3 * nbp] = 3 * n;
            __syncthreads();
            for (uint32_t i0 = tid; i0 < n; i0 += kU * kBlock) {
                uint64_t x[kU], y[kU];
                for (uint32_t q = 0; q < kU; q++)
                    if (i0 + q * kBlock < n)
                        key_digest(a, d, i0 + q * kBlock, sd, x[q], y[q]);
                for (uint32_t q = 0; q < kU; q++) {
                    const uint32_t i = i0 + q * kBlock;
                    if (i < n) {
                        const uint3 u = digest_locals(x[q], y[q], P);
                        const uint32_t hi_i = i << kPackBits;
                        pairs[atomicAdd(&s_cnt[u.x >> kPackBits], 1u)] = hi_i | (u.x & (kPackTile - 1));
                        pairs[atomicAdd(&s_cnt[nbp + (u.y >> kPackBits)], 1u)] = hi_i | (u.y & (kPackTile - 1));
                        pairs[atomicAdd(&s_cnt[2 * nbp + (u.z >> kPackBits)], 1u)] = hi_i | (u.z & (kPackTile - 1));
                    }
                }
            }
            __syncthreads();
            for (uint32_t k = 0; k < 3; k++) {
                uint32_t degsum = 0;
                for (uint32_t b = 0; b < nbp; b++) {
                    for (uint32_t v = tid; v < kPackTile; v += kBlock)
                        s_tab[v] = 0;
                    __syncthreads();
                    const uint32_t j1 = s_bnd[k * nbp + b + 1];
                    for (uint32_t j0 = s_bnd[k * nbp + b] + tid; j0 < j1; j0 += kU * kBlock) {
                        uint32_t pr[kU];
                        for (uint32_t q = 0; q < kU; q++)
                            if (j0 + q * kBlock < j1)
                                pr[q] = pairs[j0 + q * kBlock];
                        for (uint32_t q = 0; q < kU; q++)
                            if (j0 + q * kBlock < j1)
                                atomicAdd(&s_tab[pr[q] & (kPackTile - 1)],
                                          (unsigned long long)(Rec::kOne + (pr[q] >> kPackBits)));
                    }
                    __syncthreads();
                    const uint64_t v0 = (uint64_t)b * kPackTile;
                    write_tile(k, v0, (uint32_t)min<uint64_t>(kPackTile, P - v0), stage, degsum);
                    __syncthreads();
                }
                close_part(k, degsum);
            }
            // layer 0 to the front of the slots, each slot with its hinge part
            const uint32_t l0 = min(s_ltail, n);
            for (uint32_t j = tid; j < l0; j += kBlock)
                L.slots[j] = make_uint3(stage[j], j < s_l0part[0] ? 0u : (j < s_l0part[1] ? 1u : 2u), 0u);
            l0_in_slot = true;
        } else if (nbk <= kBatchMaxBuckets) {
            // Records part by part without device atomics: the part's (vertex, key) pairs are
            // grouped by tile of kBatchTile vertices (LDS counts, one scatter into the slot
            // area), each tile accumulated in LDS and written once.
            // The slot area (12n bytes) holds the pairs (8n) and, behind them, layer 0 (4n).
            uint2* pairs = reinterpret_cast<uint2*>(L.slots);
            uint32_t* stage = reinterpret_cast<uint32_t*>(pairs + n);
            for (uint32_t k = 0; k < 3; k++) {
                if (nbk > 1) {  // one tile: the keys go straight into it below
                    for (uint32_t b = tid; b < nbk; b += kBlock)
                        s_cnt[b] = 0;
                    __syncthreads();
                    for (uint32_t i = tid; i < n; i += kBlock)
                        atomicAdd(&s_cnt[bucket_local(a, d, L, i, sd, P, k) / kBatchTile], 1u);
                    __syncthreads();
                    lds_exclusive_scan<kBlock>(s_cnt, nbk, s_wtot);
                    for (uint32_t b = tid; b < nbk; b += kBlock)
                        s_bnd[b] = s_cnt[b];
                    if (tid == 0)
                        s_bnd[nbk] = n;
                    __syncthreads();
                    for (uint32_t i = tid; i < n; i += kBlock) {
                        const uint32_t u = bucket_local(a, d, L, i, sd, P, k);
                        const uint32_t pos = atomicAdd(&s_cnt[u / kBatchTile], 1u);
                        pairs[pos] = make_uint2(u % kBatchTile, i);
                    }
                    __syncthreads();
                }
                uint32_t degsum = 0;
                for (uint32_t b = 0; b < nbk; b++) {
                    for (uint32_t v = tid; v < kBatchTile; v += kBlock)
                        s_tab[v] = 0;
                    __syncthreads();
                    if (nbk == 1) {
                        for (uint32_t i = tid; i < n; i += kBlock)
                            atomicAdd(&s_tab[bucket_local(a, d, L, i, sd, P, k)],
                                      (unsigned long long)(Rec::kOne + i));
                    } else {
                        for (uint32_t j = s_bnd[b] + tid; j < s_bnd[b + 1]; j += kBlock) {
                            const uint2 pr = pairs[j];
                            atomicAdd(&s_tab[pr.x], (unsigned long long)(Rec::kOne + pr.y));
                        }
                    }
                    __syncthreads();
                    const uint64_t v0 = (uint64_t)b * kBatchTile;
                    write_tile(k, v0, (uint32_t)min<uint64_t>(kBatchTile, P - v0), stage, degsum);
                    __syncthreads();
                }
                close_part(k, degsum);
            }
            // Layer 0 moves to the front of the slots, each slot with its hinge part (the
            // appends came part by part).  Slot j overwrites staged entries at most j, so a
            // block-wide chunk is read in full before any of it is written.
            const uint32_t l0 = min(s_ltail, n);
            for (uint32_t base = 0; base < l0; base += kBlock) {
                const uint32_t j = base + tid;
                const uint32_t e = j < l0 ? stage[j] : 0u;
                __syncthreads();
                if (j < l0)
                    L.slots[j] = make_uint3(e, j < s_l0part[0] ? 0u : (j < s_l0part[1] ? 1u : 2u), 0u);
                __syncthreads();
            }
            l0_in_slot = true;
        } else {
            // very large bucket: records with device atomics, round 0 with atomicMin
            for (uint32_t v = tid; v < m; v += kBlock)
                L.rec[v] = 0;
            __syncthreads();
            for (uint32_t i = tid; i < n; i += kBlock) {
                const uint3 ev = bucket_edge(a, d, L, i, sd, P);
                uint32_t dg = S::rec_add(L.rec, ev.x, i);
                dg = max(dg, S::rec_add(L.rec, ev.y, i));
                dg = max(dg, S::rec_add(L.rec, ev.z, i));
                if (dg >= kMaxDegree)
                    s_err = 1;
            }
            __syncthreads();
            if (!s_err) {
                for (uint32_t base = 0; base < m; base += kBlock) {
                    uint32_t v = base + tid;
                    bool first = false;
                    uint32_t e = 0;
                    if (v < m) {
                        uint64_t x = S::ld(L.rec + v);
                        if (Rec::deg(x) == 1 && Rec::edge(x) < n) {
                            e = Rec::edge(x);
                            first = S::fetch_min(L.state + e, part_of(v, P)) == kUnclaimed;
                        }
                    }
                    uint32_t pos = block_append(&s_ltail, first, false);
                    if (first)
                        L.slots[pos].x = e;
                }
            }
        }
        __syncthreads();
        clk.mark(kClRecords);
        if (s_err) {
            status = -2;  // degree above 255: no seed helps a duplicate-heavy bucket
            break;
        }
        if (tid == 0)
            L.lstart[0] = 0;
        __syncthreads();
        uint32_t r = 0, lo = 0;
        // whether the current layer's slots carry their hinge part in .y (layer 0 from the
        // partitioned record build, layers resolved from claim lists); else it is read from
        // the edge state
        bool hinge_in_slot = l0_in_slot;
        auto hinge_of = [&](uint32_t i, uint32_t& e) {
            const uint3 s0 = L.slots[i];
            e = s0.x;
            return hinge_in_slot ? (s0.y & 3u) : (S::ld(L.state + e) & 3u);
        };
        for (;;) {
            // Layer r is [lo, hi).  Applying it claims round r + 1 at once: a vertex taken to
            // degree 1 claims its remaining edge, which is final unless that edge also leaves
            // in round r -- and then its state already holds round r, which the claim cannot
            // lower.  Every thread reads hi before any thread appends (barrier below).
            const uint32_t hi = s_ltail;
            __syncthreads();
            if (tid == 0)
                L.lstart[r + 1] = hi;
            if (lo == hi)
                break;
            const uint32_t rr = (r + 1) << 2;
            // A dense layer of a bucket given by key words may delete through a sorted list
            // instead of device atomics (Section 4.2's sorted update list, inside the
            // workgroup): its deletes, packed (vertex in tile, edge) like the record build's
            // pairs, are grouped by (part, tile of kPackTile vertices) in the free edge area;
            // each tile's records are loaded into LDS, the deletes applied with LDS atomics, and
            // the tile written back.  A delete that takes a vertex from degree 2 to 1 marks its
            // record (bit 63; degrees stay below 256 and sums below 2^28, so the bit is free);
            // a marked vertex still at degree 1 once the tile's deletes are done claims its
            // remaining edge -- the record's sum -- by clearing the part's bit in the edge's
            // state (no return value).  A scan of the states then appends the claimed edges,
            // each with its lowest claiming part as hinge and the claiming parts as the degree-1
            // parts: the layer and hinges the claim lists give.
            const uint32_t L2 = 2 * (hi - lo);
            constexpr uint32_t kClTile = kBatchTile * 8;  // claim-list tile: edges, one LDS byte each
            const uint32_t ncl = (n + kClTile - 1) / kClTile;
            const bool sorted_round = a.sort_div && d.keys && hinge_in_slot && (uint64_t)L2 * a.sort_div >= m &&
                                      n <= (1u << (32 - kPackBits)) && 3 * nbp <= kBatchMaxBuckets;
            const bool list_round = !sorted_round && a.claim_lists && d.keys && 8ull * (hi - lo) <= 3ull * n &&
                                    ncl <= kBatchMaxBuckets;
            if (!list_round && !sorted_round && hinge_in_slot) {
                // a layer resolved from claim lists left the states alone; the claims by
                // atomicMin below must find its edges taken, so they get their states now
                for (uint32_t i = lo + tid; i < hi; i += kBlock) {
                    const uint3 s0 = L.slots[i];
                    L.state[s0.x] = (r << 2) | (s0.y & 3u);
                }
                __syncthreads();
            }
            if (sorted_round) {
                constexpr uint64_t kMark = 1ull << 63;
                constexpr uint32_t kCollected = 0xFFFFFFF0u;  // a claimed edge, already appended
                uint32_t* se = reinterpret_cast<uint32_t*>(L.edges);  // the layer's edges, skip bits on top
                uint32_t* dl = se + n;                                // up to 2n packed deletes
                for (uint32_t b = tid; b < 3 * nbp; b += kBlock)
                    s_cnt[b] = 0;
                __syncthreads();
                for (uint32_t i = lo + tid; i < hi; i += kBlock) {
                    const uint3 s0 = L.slots[i];
                    const uint32_t e = s0.x, h = s0.y & 3u, ones = (s0.y >> 8) & 7u;
                    const uint3 ev = bucket_edge(a, d, L, e, sd, P);
                    const uint32_t vh = h == 0 ? ev.x : (h == 1 ? ev.y : ev.z);
                    const uint32_t va = h == 0 ? ev.y : (h == 1 ? ev.z : ev.x);
                    const uint32_t vb = h == 0 ? ev.z : (h == 1 ? ev.x : ev.y);
                    L.slots[i] = make_uint3(vh, va, vb);
                    const uint32_t pa = h == 2 ? 0u : h + 1, pb = h == 0 ? 2u : h - 1;  // parts of va, vb
                    const uint32_t sa = (ones >> pa) & 1u, sb = (ones >> pb) & 1u;    // degree 1: skip
                    se[i - lo] = e | sa << 30 | sb << 31;
                    clk.deletes(2u - sa - sb);
                    if (!sa)
                        atomicAdd(&s_cnt[pa * nbp + ((va - pa * (uint32_t)P) >> kPackBits)], 1u);
                    if (!sb)
                        atomicAdd(&s_cnt[pb * nbp + ((vb - pb * (uint32_t)P) >> kPackBits)], 1u);
                }
                __syncthreads();
                const uint32_t ndl = lds_exclusive_scan<kBlock>(s_cnt, 3 * nbp, s_wtot);
                for (uint32_t b = tid; b < 3 * nbp; b += kBlock)
                    s_bnd[b] = s_cnt[b];
                if (tid == 0)
                    s_bnd[3 * nbp] = ndl;
                __syncthreads();
                for (uint32_t i = lo + tid; i < hi; i += kBlock) {
                    const uint3 sl = L.slots[i];
                    const uint32_t w = se[i - lo], e = w & 0x3FFFFFFFu;
                    const uint32_t pa = part_of(sl.y, P), pb = part_of(sl.z, P);
                    const uint32_t la = sl.y - pa * (uint32_t)P, lb = sl.z - pb * (uint32_t)P;
                    if (!(w >> 30 & 1u))
                        dl[atomicAdd(&s_cnt[pa * nbp + (la >> kPackBits)], 1u)] = e << kPackBits | (la & (kPackTile - 1));
                    if (!(w >> 31))
                        dl[atomicAdd(&s_cnt[pb * nbp + (lb >> kPackBits)], 1u)] = e << kPackBits | (lb & (kPackTile - 1));
                }
                __syncthreads();
                for (uint32_t t = 0; t < 3 * nbp; t++) {
                    const uint32_t j1 = s_bnd[t + 1];
                    if (s_bnd[t] == j1)
                        continue;  // uniform per block
                    const uint32_t k = t / nbp;
                    const uint64_t tv = (uint64_t)(t - k * nbp) * kPackTile;
                    const uint64_t v0 = (uint64_t)k * P + tv;
                    const uint32_t cnt = (uint32_t)min<uint64_t>(kPackTile, P - tv);
                    for (uint32_t v = tid; v < cnt; v += kBlock)
                        s_tab[v] = S::ld(L.rec + v0 + v);
                    __syncthreads();
                    for (uint32_t j0 = s_bnd[t] + tid; j0 < j1; j0 += kU * kBlock) {
                        uint32_t dv[kU];
                        for (uint32_t q = 0; q < kU; q++)
                            if (j0 + q * kBlock < j1)
                                dv[q] = dl[j0 + q * kBlock];
                        for (uint32_t q = 0; q < kU; q++) {
                            if (j0 + q * kBlock < j1) {
                                unsigned long long* x = &s_tab[dv[q] & (kPackTile - 1)];
                                const uint64_t old = atomicAdd(x, 0ull - (Rec::kOne + (dv[q] >> kPackBits)));
                                if ((old >> 40 & 0xFFu) == 2)
                                    atomicOr(x, (unsigned long long)kMark);
                            }
                        }
                    }
                    __syncthreads();
                    for (uint32_t v = tid; v < cnt; v += kBlock) {
                        uint64_t x = s_tab[v];
                        if (x & kMark) {
                            x &= ~kMark;
                            if ((x >> 40 & 0xFFu) == 1)
                                S::fetch_and(L.state + Rec::edge(x), ~(1u << k));
                        }
                        L.rec[v0 + v] = x;
                    }
                    __syncthreads();
                }
                // the next layer: edges whose state lost part bits (and nothing else) this round
                for (uint32_t c0 = 0; c0 < n; c0 += kU * kBlock) {
                    uint32_t st[kU];
                    for (uint32_t q = 0; q < kU; q++) {
                        const uint32_t c = c0 + q * kBlock + tid;
                        st[q] = c < n ? S::ld(L.state + c) : kUnclaimed;
                    }
                    for (uint32_t q = 0; q < kU; q++) {
                        const uint32_t c = c0 + q * kBlock + tid;
                        const uint32_t bits = ~st[q] & 7u;
                        const bool hit = st[q] >= 0xFFFFFFF8u && bits != 0;
                        if (hit)
                            L.state[c] = kCollected;
                        const uint32_t pos = block_append(&s_ltail, hit, false);
                        if (hit)
                            L.slots[pos] = make_uint3(c, (uint32_t)__builtin_ctz(bits) | bits << 8, 0u);
                    }
                }
                __syncthreads();
                clk.mark(kClOther);
                lo = hi;
                r++;
                hinge_in_slot = true;  // the scan wrote each slot's hinge and degree-1 parts
                continue;
            }
            // A sparse layer of a bucket given by key words (whose edge area is free) may claim
            // through a list instead of atomicMin on the states, the plain path's claim lists
            // inside the workgroup: every delete that leaves a vertex at degree 1 records
            // (remaining edge, the vertex's part), and one that leaves it at degree 0 records a
            // cancel (its own edge, 4 | the vertex's part): the vertex fell 2 -> 1 -> 0 in this
            // round, so its claim named this edge, which leaves now.  The records are grouped
            // by tile of kClTile edges and each tile resolved in an LDS byte per edge (claim
            // bits 0..2, cancel bits 4..6): the lowest part claimed and not cancelled is the
            // hinge -- exactly the layer and hinges atomicMin gives.  The winner's slot gets
            // (edge, hinge | parts at degree 1 << 8): the next round reads the hinge there and
            // skips the deletes at the other degree-1 vertices, which drop to 0 and are never
            // read again.  No state is read or written; a later round that claims by atomicMin
            // first gives its layer's edges their states (above).
            if (list_round) {
                uint2* cl = reinterpret_cast<uint2*>(L.edges);  // 12n bytes: claims, then grouped
                uint2* cg = cl + 2 * (hi - lo);                 // at most two per layer edge each
                if (tid == 0)
                    s_ctail = 0;
                for (uint32_t b = tid; b < ncl; b += kBlock)
                    s_cnt[b] = 0;
                __syncthreads();
                for (uint32_t base = lo; base < hi; base += kBlock) {
                    const uint32_t i = base + tid;
                    uint2 c0 = make_uint2(0u, 0u), c1 = make_uint2(0u, 0u);
                    bool f0 = false, f1 = false;
                    if (i < hi) {
                        const uint3 s0 = L.slots[i];
                        const uint32_t e = s0.x;
                        const uint32_t h = hinge_in_slot ? (s0.y & 3u) : (S::ld(L.state + e) & 3u);
                        const uint32_t ones = hinge_in_slot ? (s0.y >> 8) & 7u : 0u;
                        const uint3 ev = bucket_edge(a, d, L, e, sd, P);
                        const uint32_t vh = h == 0 ? ev.x : (h == 1 ? ev.y : ev.z);
                        const uint32_t va = h == 0 ? ev.y : (h == 1 ? ev.z : ev.x);
                        const uint32_t vb = h == 0 ? ev.z : (h == 1 ? ev.x : ev.y);
                        L.slots[i] = make_uint3(vh, va, vb);
                        const uint32_t pa = h == 2 ? 0u : h + 1, pb = h == 0 ? 2u : h - 1;  // parts of va, vb
                        const bool sa = (ones >> pa) & 1u, sb = (ones >> pb) & 1u;
                        clk.deletes(2u - sa - sb);
                        const uint64_t oa = sa ? Rec::kOne : S::rec_del(L.rec, va, e);
                        const uint64_t ob = sb ? Rec::kOne : S::rec_del(L.rec, vb, e);
                        if (Rec::deg(oa) == 2) {
                            c0 = make_uint2((uint32_t)(Rec::edge(oa) - e), pa);
                            f0 = true;
                        } else if (Rec::deg(oa) == 1 && !sa) {
                            c0 = make_uint2(e, 4u | pa);
                            f0 = true;
                        }
                        if (Rec::deg(ob) == 2) {
                            c1 = make_uint2((uint32_t)(Rec::edge(ob) - e), pb);
                            f1 = true;
                        } else if (Rec::deg(ob) == 1 && !sb) {
                            c1 = make_uint2(e, 4u | pb);
                            f1 = true;
                        }
                        if (!f0) {  // the first requested slot holds the first record
                            c0 = c1;
                            f0 = f1;
                            f1 = false;
                        }
                        if (f0)
                            atomicAdd(&s_cnt[c0.x / kClTile], 1u);
                        if (f1)
                            atomicAdd(&s_cnt[c1.x / kClTile], 1u);
                    }
                    const uint32_t pos = block_append(&s_ctail, f0, f1);
                    if (f0)
                        cl[pos] = c0;
                    if (f1)
                        cl[pos + 1] = c1;
                }
                __syncthreads();
                clk.mark(kClDeletes);
                const uint32_t nc = s_ctail;
                clk.records(nc);
                if (nc <= kBatchTile && n < (1u << 24)) {
                    // Few records (a sparse round): resolve them in one LDS hash table keyed by
                    // edge, at most half full (open addressing, linear probing; an entry is the
                    // edge << 8 | its claim and cancel bits), instead of grouping them by tile --
                    // the same bits per edge, so the same winners.
                    uint32_t* htab = reinterpret_cast<uint32_t*>(s_tab);  // up to 2 kBatchTile entries
                    uint32_t lg = 6;
                    while ((1u << lg) < 2 * nc)
                        lg++;
                    const uint32_t mask = (1u << lg) - 1;
                    for (uint32_t j = tid; j <= mask; j += kBlock)
                        htab[j] = kUnclaimed;
                    __syncthreads();
                    for (uint32_t j = tid; j < nc; j += kBlock) {
                        const uint2 c = cl[j];
                        const uint32_t bit = 1u << c.y;
                        uint32_t h = (c.x * 0x9E3779B1u) >> (32 - lg);
                        for (;;) {
                            const uint32_t old = atomicCAS(&htab[h], kUnclaimed, c.x << 8 | bit);
                            if (old == kUnclaimed)
                                break;
                            if (old >> 8 == c.x) {
                                atomicOr(&htab[h], bit);
                                break;
                            }
                            h = (h + 1) & mask;
                        }
                    }
                    __syncthreads();
                    for (uint32_t base = 0; base < nc; base += kBlock) {
                        const uint32_t j = base + tid;
                        bool win = false;
                        uint32_t c = 0, hinge_word = 0;
                        if (j < nc) {
                            const uint2 cc = cl[j];
                            if (cc.y < 4) {
                                // the edge was inserted before any empty entry on its probe path
                                uint32_t h = (cc.x * 0x9E3779B1u) >> (32 - lg);
                                while (htab[h] >> 8 != cc.x)
                                    h = (h + 1) & mask;
                                const uint32_t t = htab[h] & 0xFFu;
                                const uint32_t live = t & ~(t >> 4) & 7u;
                                win = live != 0 && (uint32_t)__builtin_ctz(live) == cc.y;
                                c = cc.x;
                                hinge_word = cc.y | live << 8;
                            }
                        }
                        const uint32_t pos = block_append(&s_ltail, win, false);
                        if (win)
                            L.slots[pos] = make_uint3(c, hinge_word, 0u);
                    }
                    __syncthreads();
                    clk.mark(kClResolve);
                    lo = hi;
                    r++;
                    hinge_in_slot = true;
                    continue;
                }
                lds_exclusive_scan<kBlock>(s_cnt, ncl, s_wtot);
                for (uint32_t b = tid; b < ncl; b += kBlock)
                    s_bnd[b] = s_cnt[b];
                if (tid == 0)
                    s_bnd[ncl] = nc;
                __syncthreads();
                for (uint32_t j = tid; j < nc; j += kBlock) {
                    const uint2 c = cl[j];
                    cg[atomicAdd(&s_cnt[c.x / kClTile], 1u)] = c;
                }
                __syncthreads();
                clk.mark(kClGroup);
                uint32_t* tab = reinterpret_cast<uint32_t*>(s_tab);  // kClTile bytes
                for (uint32_t tl = 0; tl < ncl; tl++) {
                    const uint32_t j0 = s_bnd[tl], j1 = s_bnd[tl + 1];
                    if (j0 == j1)
                        continue;  // uniform per block
                    for (uint32_t j = j0 + tid; j < j1; j += kBlock)
                        tab[(cg[j].x % kClTile) >> 2] = 0u;
                    __syncthreads();
                    for (uint32_t j = j0 + tid; j < j1; j += kBlock) {
                        const uint2 c = cg[j];
                        atomicOr(&tab[(c.x % kClTile) >> 2], 1u << (8 * (c.x & 3) + c.y));
                    }
                    __syncthreads();
                    for (uint32_t base = j0; base < j1; base += kBlock) {
                        const uint32_t j = base + tid;
                        bool win = false;
                        uint32_t c = 0, hinge_word = 0;
                        if (j < j1) {
                            const uint2 cc = cg[j];
                            const uint32_t t = tab[(cc.x % kClTile) >> 2] >> (8 * (cc.x & 3));
                            const uint32_t live = t & ~(t >> 4) & 7u;
                            win = cc.y < 4 && live != 0 && (uint32_t)__builtin_ctz(live) == cc.y;
                            c = cc.x;
                            hinge_word = cc.y | live << 8;
                        }
                        const uint32_t pos = block_append(&s_ltail, win, false);
                        if (win)
                            L.slots[pos] = make_uint3(c, hinge_word, 0u);
                    }
                    __syncthreads();
                }
                clk.mark(kClResolve);
                lo = hi;
                r++;
                hinge_in_slot = true;  // the resolve wrote each slot's hinge and degree-1 parts
                continue;
            }
            for (uint32_t base = lo; base < hi; base += kBlock) {
                uint32_t i = base + tid;
                uint32_t c0 = 0, c1 = 0;
                bool f0 = false, f1 = false;
                if (i < hi) {
                    uint32_t e;
                    uint32_t h = hinge_of(i, e);
                    uint3 ev = bucket_edge(a, d, L, e, sd, P);
                    uint32_t vh = h == 0 ? ev.x : (h == 1 ? ev.y : ev.z);
                    uint32_t va = h == 0 ? ev.y : (h == 1 ? ev.z : ev.x);
                    uint32_t vb = h == 0 ? ev.z : (h == 1 ? ev.x : ev.y);
                    L.slots[i] = make_uint3(vh, va, vb);
                    uint64_t oa = S::rec_del(L.rec, va, e);
                    uint64_t ob = S::rec_del(L.rec, vb, e);
                    if (Rec::deg(oa) == 2) {
                        c0 = (uint32_t)(Rec::edge(oa) - e);
                        f0 = S::fetch_min(L.state + c0, rr | part_of(va, P)) == kUnclaimed;
                    }
                    if (Rec::deg(ob) == 2) {
                        c1 = (uint32_t)(Rec::edge(ob) - e);
                        f1 = S::fetch_min(L.state + c1, rr | part_of(vb, P)) == kUnclaimed;
                    }
                    if (!f0) {  // the first requested slot holds the first appended edge
                        c0 = c1;
                        f0 = f1;
                        f1 = false;
                    }
                }
                uint32_t pos = block_append(&s_ltail, f0, f1);
                if (f0)
                    L.slots[pos].x = c0;
                if (f1)
                    L.slots[pos + 1].x = c1;
            }
            __syncthreads();
            clk.mark(kClOther);
            lo = hi;
            r++;
            hinge_in_slot = false;  // the next layer was claimed by atomicMin
        }
        nrounds = r;
        const bool all = s_ltail == n;
        __syncthreads();
        clk.mark(kClDeletes);  // the empty-layer check that ended the rounds
        if (all) {
            ok = true;
            break;
        }
    }
    if (!ok) {
        if (tid == 0)
            write_result(d.result, sd, t < a.max_tries ? t + 1 : a.max_tries, status ? status : 1, nrounds);
        __syncthreads();
        clk.flush(n, t < a.max_tries ? t + 1 : a.max_tries, nrounds);
        return;
    }
    // assignment, last layer first; codes as bytes in the record area
    uint8_t* code8 = reinterpret_cast<uint8_t*>(L.rec);
    for (uint32_t v = tid; v < m; v += kBlock)
        code8[v] = 0;
    __syncthreads();
    for (int32_t r = (int32_t)nrounds - 1; r >= 0; r--) {
        const uint32_t lo = L.lstart[r], hi = L.lstart[r + 1];
        for (uint32_t i = lo + tid; i < hi; i += kBlock) {
            uint3 sl = L.slots[i];
            uint32_t k = part_of(sl.x, P);
            uint32_t ca = code8[sl.y], cb = code8[sl.z];
            uint32_t g = (k + 6 - (ca == 3 ? 0 : ca) - (cb == 3 ? 0 : cb)) % 3;
            code8[sl.x] = (uint8_t)(g ? g : 3);
        }
        __syncthreads();
    }
    clk.mark(kClAssign);
    pack_codes<kBlock>(code8, m, d, L);
    if (tid == 0)
        write_result(d.result, sd, t + 1, 0, nrounds);
    __syncthreads();
    clk.mark(kClPack);
    clk.flush(n, t + 1, nrounds);
}

// The same build for a bucket that fits in LDS: 4-byte records (degree in bits [24, 32), sum of
// incident edge ids in [0, 24): no carry while degrees stay <= 255 and ids below 2^16) and the
// edge states live in LDS, so every atomic of the rounds is an LDS atomic; the layer slots stay
// in the slot area.  Same rounds, hinges and layers as build_bucket, hence the same codes.
template <int kBlock>
__device__ void build_bucket_lds(const BatchArgs& a, const BucketDesc& d, uint8_t* slot, uint8_t* lds)
{
    __shared__ uint32_t s_ltail, s_err;
    constexpr uint32_t kOne32 = 1u << 24, kSum = kOne32 - 1;
    const uint32_t tid = threadIdx.x;
    const uint32_t n = (uint32_t)d.n;
    const uint64_t P = part_size_dev(n, a.gnum, a.gden);
    const uint32_t m = (uint32_t)(3 * P);
    SlotLayout L;
    slot_layout(slot, n, m, &L);
    uint32_t* rec = reinterpret_cast<uint32_t*>(lds);  // m records
    uint32_t* state = rec + ((m + 3) & ~3u);            // n edge states
    const uint64_t total = d.keys ? 0 : d.offs[n];

    uint32_t t = 0, nrounds = 0;
    bool ok = false;
    int status = 0;
    uint64_t sd = d.seed;
    for (t = 0; t < a.max_tries; t++) {
        sd = d.seed + t;
        for (uint32_t v = tid; v < m; v += kBlock)
            rec[v] = 0;
        for (uint32_t e = tid; e < n; e += kBlock)
            state[e] = kUnclaimed;
        if (tid == 0) {
            s_ltail = 0;
            s_err = 0;
        }
        const uint64_t sa = fin(sd + kGamma), sb = fin(sd + 2 * kGamma);
        if (!d.keys) {  // string keys: digest once, keep the edges
            for (uint32_t i = tid; i < n; i += kBlock) {
                uint64_t o0 = d.offs[i], o1 = d.offs[i + 1], ha, hb;
                digest_str(d.bytes, o0, o1 - o0, total, sa, sb, ha, hb);
                uint3 ev;
                edge_of_digest(ha, hb, P, ev.x, ev.y, ev.z);
                L.edges[i] = ev;
            }
        }
        __syncthreads();
        for (uint32_t i = tid; i < n; i += kBlock) {
            const uint3 ev = bucket_edge(a, d, L, i, sd, P);
            const uint32_t o0 = atomicAdd(&rec[ev.x], kOne32 + i);
            const uint32_t o1 = atomicAdd(&rec[ev.y], kOne32 + i);
            const uint32_t o2 = atomicAdd(&rec[ev.z], kOne32 + i);
            if (max(o0, max(o1, o2)) >= kMaxDegree * kOne32)  // a degree would pass 255
                s_err = 1;
        }
        __syncthreads();
        if (s_err) {
            status = -2;  // degree above 255: no seed helps a duplicate-heavy bucket
            break;
        }
        // round 0: a degree-1 vertex claims its edge; the lowest part wins
        for (uint32_t base = 0; base < m; base += kBlock) {
            const uint32_t v = base + tid;
            bool first = false;
            uint32_t e = 0;
            if (v < m) {
                const uint32_t x = rec[v];
                if ((x >> 24) == 1 && (x & kSum) < n) {
                    e = x & kSum;
                    first = atomicMin(&state[e], part_of(v, P)) == kUnclaimed;
                }
            }
            const uint32_t pos = block_append(&s_ltail, first, false);
            if (first)
                L.slots[pos].x = e;
        }
        if (tid == 0)
            L.lstart[0] = 0;
        __syncthreads();
        uint32_t r = 0, lo = 0;
        for (;;) {
            // as in build_bucket: applying layer r claims round r + 1
            const uint32_t hi = s_ltail;
            __syncthreads();
            if (tid == 0)
                L.lstart[r + 1] = hi;
            if (lo == hi)
                break;
            const uint32_t rr = (r + 1) << 2;
            for (uint32_t base = lo; base < hi; base += kBlock) {
                const uint32_t i = base + tid;
                uint32_t c0 = 0, c1 = 0;
                bool f0 = false, f1 = false;
                if (i < hi) {
                    const uint32_t e = L.slots[i].x;
                    const uint32_t h = state[e] & 3u;
                    const uint3 ev = bucket_edge(a, d, L, e, sd, P);
                    const uint32_t vh = h == 0 ? ev.x : (h == 1 ? ev.y : ev.z);
                    const uint32_t va = h == 0 ? ev.y : (h == 1 ? ev.z : ev.x);
                    const uint32_t vb = h == 0 ? ev.z : (h == 1 ? ev.x : ev.y);
                    L.slots[i] = make_uint3(vh, va, vb);
                    const uint32_t oa = atomicSub(&rec[va], kOne32 + e);
                    const uint32_t ob = atomicSub(&rec[vb], kOne32 + e);
                    if ((oa >> 24) == 2) {
                        c0 = (oa & kSum) - e;
                        f0 = atomicMin(&state[c0], rr | part_of(va, P)) == kUnclaimed;
                    }
                    if ((ob >> 24) == 2) {
                        c1 = (ob & kSum) - e;
                        f1 = atomicMin(&state[c1], rr | part_of(vb, P)) == kUnclaimed;
                    }
                    if (!f0) {  // the first requested slot holds the first appended edge
                        c0 = c1;
                        f0 = f1;
                        f1 = false;
                    }
                }
                const uint32_t pos = block_append(&s_ltail, f0, f1);
                if (f0)
                    L.slots[pos].x = c0;
                if (f1)
                    L.slots[pos + 1].x = c1;
            }
            __syncthreads();
            lo = hi;
            r++;
        }
        nrounds = r;
        const bool all = s_ltail == n;
        __syncthreads();
        if (all) {
            ok = true;
            break;
        }
    }
    if (!ok) {
        if (tid == 0)
            write_result(d.result, sd, t < a.max_tries ? t + 1 : a.max_tries, status ? status : 1, nrounds);
        __syncthreads();
        return;
    }
    // assignment, last layer first, with the codes as bytes in LDS over the records
    uint8_t* code8 = lds;
    for (uint32_t v = tid; v < m; v += kBlock)
        code8[v] = 0;
    __syncthreads();
    for (int32_t r = (int32_t)nrounds - 1; r >= 0; r--) {
        const uint32_t lo = L.lstart[r], hi = L.lstart[r + 1];
        for (uint32_t i = lo + tid; i < hi; i += kBlock) {
            const uint3 sl = L.slots[i];
            const uint32_t k = part_of(sl.x, P);
            const uint32_t ca = code8[sl.y], cb = code8[sl.z];
            const uint32_t g = (k + 6 - (ca == 3 ? 0 : ca) - (cb == 3 ? 0 : cb)) % 3;
            code8[sl.x] = (uint8_t)(g ? g : 3);
        }
        __syncthreads();
    }
    pack_codes<kBlock>(code8, m, d, L);
    if (tid == 0)
        write_result(d.result, sd, t + 1, 0, nrounds);
    __syncthreads();
}

// Waves per SIMD the launch shapes need resident: 1024 threads = 16 waves per compute unit, 512
// two workgroups per compute unit, 256 three.
template <int kBlock>
constexpr int batch_waves_per_eu() { return kBlock >= 512 ? 4 : 3; }

template <int kBlock, int kScope, bool kClock>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(batch_waves_per_eu<kBlock>())))
void k_batch(BatchArgs a)
{
    __shared__ uint32_t s_idx;
    __shared__ __align__(16) uint8_t s_lds[batch_lds_bytes<kBlock>()];
    uint8_t* slot = a.slots + (uint64_t)blockIdx.x * a.slot_bytes;
    uint64_t t_life = 0, t_q = 0, t_queue = 0, t_lds = 0, n_lds = 0, k_lds = 0;
    if constexpr (kClock)
        t_life = wall_clock64();
    for (;;) {
        if constexpr (kClock)
            t_q = wall_clock64();
        if (threadIdx.x == 0)
            s_idx = atomicAdd(a.next, 1u);
        __syncthreads();
        const uint32_t idx = s_idx;
        __syncthreads();
        if constexpr (kClock) {
            const uint64_t t2 = wall_clock64();
            t_queue += t2 - t_q;
            t_q = t2;
        }
        if (idx >= a.B)
            break;
        const BucketDesc d = a.descs[a.order ? a.order[idx] : idx];
        const bool in_lds = d.n <= a.max_n && bucket_fits_lds<kBlock>(d.n, 3 * part_size_dev(d.n, a.gnum, a.gden));
        if (in_lds && a.lds_path) {
            build_bucket_lds<kBlock>(a, d, slot, s_lds);
            if constexpr (kClock) {
                t_lds += wall_clock64() - t_q;
                n_lds++;
                k_lds += d.n;
            }
        } else {
            build_bucket<kBlock, kScope, kClock>(a, d, slot, s_lds);
        }
    }
    if constexpr (kClock) {
        if (threadIdx.x == 0) {
            atomicAdd(&g_batch_clock[kClQueue], (unsigned long long)t_queue);
            atomicAdd(&g_batch_clock[kClLds], (unsigned long long)t_lds);
            atomicAdd(&g_batch_clock[kClLdsBuckets], (unsigned long long)n_lds);
            atomicAdd(&g_batch_clock[kClLdsKeys], (unsigned long long)k_lds);
            atomicAdd(&g_batch_clock[kClLife], (unsigned long long)(wall_clock64() - t_life));
        }
    }
}

// Descriptors of the buckets of one key array (u64 keys or digest pairs, wpk words per key)
// split by offsets, with outputs at offsets.
__global__ __launch_bounds__(256) void k_batch_descs(BucketDesc* descs, const uint64_t* keys, const uint64_t* off,
                                                     uint32_t B, uint64_t seed, const uint64_t* code_off,
                                                     const uint64_t* rank_off, uint64_t* codes, uint64_t* rank,
                                                     BucketResult* results, uint32_t wpk)
{
    for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += gridDim.x * blockDim.x) {
        BucketDesc d;
        d.keys = keys + off[b] * wpk;
        d.bytes = nullptr;
        d.offs = nullptr;
        d.n = off[b + 1] - off[b];
        d.seed = seed;
        d.codes = codes + code_off[b];
        d.rank = rank + rank_off[b];
        d.result = results + b;
        descs[b] = d;
    }
}

hipError_t launch_batch_descs(BucketDesc* descs, const uint64_t* keys, const uint64_t* off, uint32_t B, uint64_t seed,
                              const uint64_t* code_off, const uint64_t* rank_off, uint64_t* codes, uint64_t* rank,
                              BucketResult* results, hipStream_t s, uint32_t words_per_key)
{
    if (B == 0) return hipSuccess;
    if (words_per_key != 1 && words_per_key != 2) return hipErrorInvalidValue;
    unsigned g = (B + 255) / 256;
    k_batch_descs<<<g < 4096 ? g : 4096, 256, 0, s>>>(descs, keys, off, B, seed, code_off, rank_off, codes, rank,
                                                      results, words_per_key);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchArgs& a, unsigned block, unsigned grid, bool wg_scope, hipStream_t s)
{
    hipError_t err = launch_zero(a.next, sizeof(unsigned int), s);
    if (err != hipSuccess) return err;
    constexpr int W = __HIP_MEMORY_SCOPE_WORKGROUP, A = __HIP_MEMORY_SCOPE_AGENT;
    if (a.clock) {  // the instantiation that clocks its phases
        switch (block) {
        case 256:
            wg_scope ? k_batch<256, W, true><<<grid, 256, 0, s>>>(a) : k_batch<256, A, true><<<grid, 256, 0, s>>>(a);
            break;
        case 512:
            wg_scope ? k_batch<512, W, true><<<grid, 512, 0, s>>>(a) : k_batch<512, A, true><<<grid, 512, 0, s>>>(a);
            break;
        case 1024:
            wg_scope ? k_batch<1024, W, true><<<grid, 1024, 0, s>>>(a)
                     : k_batch<1024, A, true><<<grid, 1024, 0, s>>>(a);
            break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (block) {
    case 256: wg_scope ? k_batch<256, W, false><<<grid, 256, 0, s>>>(a) : k_batch<256, A, false><<<grid, 256, 0, s>>>(a); break;
    case 512: wg_scope ? k_batch<512, W, false><<<grid, 512, 0, s>>>(a) : k_batch<512, A, false><<<grid, 512, 0, s>>>(a); break;
    case 1024:
        wg_scope ? k_batch<1024, W, false><<<grid, 1024, 0, s>>>(a) : k_batch<1024, A, false><<<grid, 1024, 0, s>>>(a);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t batch_clock_read(uint64_t* out, int max_entries, bool reset)
{
    unsigned long long h[kBatchClockEntries] = {};
    hipError_t err = hipMemcpyFromSymbol(h, HIP_SYMBOL(g_batch_clock), sizeof h, 0, hipMemcpyDeviceToHost);
    if (err != hipSuccess) return err;
    int dev = 0, khz = 0;
    err = hipGetDevice(&dev);
    if (err == hipSuccess)
        err = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    if (err != hipSuccess) return err;
    h[0] = (unsigned long long)khz * 1000ull;
    for (int i = 0; i < max_entries && i < kBatchClockEntries; i++)
        out[i] = h[i];
    if (reset) {
        const unsigned long long z[kBatchClockEntries] = {};
        err = hipMemcpyToSymbol(HIP_SYMBOL(g_batch_clock), z, sizeof z, 0, hipMemcpyHostToDevice);
    }
    return err;
}

const char* batch_clock_name(int i)
{
    static const char* const kNames[kBatchClockEntries] = {
        "tick_hz",  "records", "deletes",        "claim_grouping", "resolve",        "other_rounds",     "assign",
        "pack",     "lds_buckets", "queue",      "workgroup",      "device_buckets", "device_keys",      "tries",
        "rounds",   "deletes_issued", "list_records", "lds_bucket_count", "lds_keys"};
    return (i >= 0 && i < kBatchClockEntries) ? kNames[i] : "";
}

}  // namespace mphx
