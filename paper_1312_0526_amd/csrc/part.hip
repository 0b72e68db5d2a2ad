// Radix partitions of (key, value) pairs into LDS-sized buckets, and what is done per bucket:
//
// * Vertex records of a tripartite hypergraph (Section 4.1: degree and the label sum of the
//   incident edges, packed as in Rec) built without device atomics.  Part k holds the vertices
//   [kP, (k+1)P) and exactly one vertex of every edge.  Its n incidences (local vertex u,
//   edge e) are partitioned by u into buckets of 2^14 consecutive vertices -- first by the
//   group digit u >> 22 (at most 342 groups, since P < 2^32 / 3), then by the bucket digit
//   (u >> 14) & 255 inside each group -- and each bucket's 16384 records are accumulated with
//   LDS atomics and written out once.
// * The claims of one peeling round (edge c, position p), partitioned by c into buckets of
//   2^16 edges and resolved in LDS: the dedupe of Section 4.2 (an edge found from several
//   degree-1 vertices enters the layer once) with the lowest claimed position as the hinge.
//
// Every pass is a histogram / exclusive-scan / scatter over tiles of 8192 elements; a tile is
// ordered by digit in LDS before it is written, so the stores go out as runs of consecutive
// addresses.  The order inside a bucket is not fixed, which neither use depends on.  Group and
// bucket offsets come from the scans: the second pass lays out its tiles per group, and its
// scan is ordered (group, bucket digit, tile), so the scanned value at (group, digit, tile 0)
// is where that bucket starts.
#include "common.h"
#include "launch.h"

#include <algorithm>

namespace mphx {

namespace {

constexpr uint32_t kVxShift = 14;            // vertex buckets: 2^14 records = 128 KiB of LDS
constexpr uint32_t kClShift = 16;            // claim buckets: 2^16 edges, a byte each = 64 KiB
constexpr uint32_t kMaxGroups = 1024;        // first-pass digits: m >> kPartGrpShift < 1024 for m < 2^32
constexpr uint32_t kDigits = 256;            // second-pass digit: (key >> bucket shift) & 255
constexpr uint32_t kPtBlock = 512;           // two blocks per CU: one loads while the other writes
constexpr uint32_t kPtPer = 16;
constexpr uint32_t kPtTile = kPtBlock * kPtPer;
constexpr uint32_t kWaves = kPtBlock / kWave;
constexpr uint32_t kAccBlock = 1024;
constexpr uint32_t kResBlock = 512;
constexpr uint32_t kUpdPer = (1u << kVxShift) / kAccBlock;  // records per thread of an update bucket

static_assert(kVxShift + 8 == kPartGrpShift, "a vertex group holds 256 buckets");
static_assert(kPtTile == kPartTile, "first-pass tiles are the hashing kernels' tiles");
static_assert(kPtBlock >= kDigits, "one thread per digit");
static_assert(2 * kPtBlock >= kMaxGroups, "two groups per thread at most");
static_assert(kPartMaxGroups <= kMaxGroups, "the hashing kernels' digits fit the group tables");

// Exclusive prefix over a block of kB threads (one value per thread); wtot is kB / 64 words
// of LDS.
template <uint32_t kB = kPtBlock>
__device__ uint32_t block_exclusive(uint32_t x, uint32_t* wtot)
{
    const uint32_t lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    uint32_t incl = x;
    for (uint32_t d = 1; d < kWave; d <<= 1) {
        uint32_t y = __shfl_up(incl, d, kWave);
        if (lane >= d)
            incl += y;
    }
    if (lane == kWave - 1)
        wtot[w] = incl;
    __syncthreads();
    uint32_t pre = 0;
    for (uint32_t q = 0; q < w; q++)
        pre += wtot[q];
    __syncthreads();
    return pre + incl - x;
}

// Exclusive prefix of cnt[0, NH) into out[], NH <= 2 * kPtBlock (two entries per thread).
__device__ void groups_exclusive(const uint32_t* cnt, uint32_t NH, uint32_t* out, uint32_t* wtot)
{
    const uint32_t j0 = 2 * threadIdx.x, j1 = j0 + 1;
    const uint32_t a = j0 < NH ? cnt[j0] : 0u, b = j1 < NH ? cnt[j1] : 0u;
    const uint32_t ex = block_exclusive(a + b, wtot);
    if (j0 < NH)
        out[j0] = ex;
    if (j1 < NH)
        out[j1] = ex + a;
}

// Local vertex of part k: an id outside the part cannot come from the hashing kernels, but is
// counted as vertex 0 so that the passes stay consistent.
__device__ __forceinline__ uint32_t local_of(uint32_t v, uint32_t k, uint64_t P)
{
    uint64_t u = (uint64_t)v - (uint64_t)k * P;
    return u < P ? (uint32_t)u : 0u;
}

// First-pass sources: part k's column of the edge list as (local vertex, edge) pairs, or a
// list of (key, value) records.
struct EdgeColumn {
    using Rec = uint2;
    const uint32_t* edges;
    uint32_t k;
    uint64_t P;
    __device__ uint2 load(uint64_t i) const { return make_uint2(local_of(edges[3 * i + k], k, P), (uint32_t)i); }
};
// Records whose first 32-bit word carries the digits: (key, value) pairs, or the 16-byte
// signature records of the HEM split of string keys.
template <class R>
struct RecordsT {
    using Rec = R;
    const R* in;
    __device__ R load(uint64_t i) const { return in[i]; }
};
using Records = RecordsT<uint2>;

struct GroupInfo {
    const uint32_t* hstart;  // NH + 1 element offsets of the groups
    const uint32_t* tbase;   // NH + 1 tile offsets of the groups (second pass)
    __device__ GroupInfo(const uint32_t* g) : hstart(g), tbase(g + kMaxGroups + 1) {}
};

// ---- pass 1 histograms of a record list (the vertex build gets its own from hashing) -------
template <class Src>
__global__ __launch_bounds__(kPtBlock) void k_part_hist1(Src src, uint64_t n, uint32_t gsh, uint32_t NH,
                                                         uint64_t nt1, uint32_t* __restrict__ hist1)
{
    __shared__ uint32_t c[kMaxGroups];
    for (uint32_t j = threadIdx.x; j < kMaxGroups; j += kPtBlock)
        c[j] = 0;
    __syncthreads();
    const uint64_t t0 = (uint64_t)blockIdx.x * kPtTile;
    for (uint32_t q = 0; q < kPtPer; q++) {
        const uint64_t i = t0 + q * kPtBlock + threadIdx.x;
        if (i < n)
            atomicAdd(&c[src.load(i).x >> gsh], 1u);
    }
    __syncthreads();
    for (uint32_t h = threadIdx.x; h < NH; h += kPtBlock)
        hist1[(uint64_t)h * nt1 + blockIdx.x] = c[h];
}

// ---- pass 1 scatter: pairs grouped by key >> gsh -----------------------------------------------
template <class Src>
__global__ __launch_bounds__(kPtBlock) void k_part_scatter1(Src src, uint64_t n, uint32_t gsh, uint32_t NH,
                                                            uint64_t nt1, const uint32_t* __restrict__ off1,
                                                            typename Src::Rec* __restrict__ out)
{
    using R = typename Src::Rec;
    __shared__ R buf[kPtTile];
    __shared__ uint32_t cnt[kMaxGroups], lst[kMaxGroups], gof[kMaxGroups], wtot[kWaves];
    for (uint32_t j = threadIdx.x; j < kMaxGroups; j += kPtBlock)
        cnt[j] = 0;
    __syncthreads();
    const uint64_t t0 = (uint64_t)blockIdx.x * kPtTile;
    R p[kPtPer];
    uint32_t rk[kPtPer];
#pragma unroll
    for (uint32_t q = 0; q < kPtPer; q++) {
        const uint64_t i = t0 + q * kPtBlock + threadIdx.x;
        if (i < n) {
            p[q] = src.load(i);
            rk[q] = atomicAdd(&cnt[p[q].x >> gsh], 1u);
        }
    }
    __syncthreads();
    groups_exclusive(cnt, NH, lst, wtot);
    for (uint32_t h = threadIdx.x; h < NH; h += kPtBlock)
        gof[h] = off1[(uint64_t)h * nt1 + blockIdx.x];
    __syncthreads();
#pragma unroll
    for (uint32_t q = 0; q < kPtPer; q++) {
        const uint64_t i = t0 + q * kPtBlock + threadIdx.x;
        if (i < n)
            buf[lst[p[q].x >> gsh] + rk[q]] = p[q];
    }
    __syncthreads();
    const uint32_t total = (uint32_t)min<uint64_t>(kPtTile, n - t0);
    for (uint32_t s = threadIdx.x; s < total; s += kPtBlock) {
        const R x = buf[s];
        const uint32_t h = x.x >> gsh;
        out[(uint64_t)gof[h] + (s - lst[h])] = x;
    }
}

// ---- pass 1 scatter of all three parts from one read of the edges -------------------------------
// The same as k_part_scatter1 on EdgeColumn k = 0, 1, 2, with the tile's edges loaded once;
// off1 holds the three parts' scanned histograms back to back ([3][NH][nt1]).
__global__ __launch_bounds__(kPtBlock) void k_part_scatter1_x3(const uint32_t* __restrict__ edges, uint64_t n,
                                                               uint64_t P, uint32_t NH, uint64_t nt1,
                                                               const uint32_t* __restrict__ off1, uint2* __restrict__ out0,
                                                               uint2* __restrict__ out1, uint2* __restrict__ out2)
{
    __shared__ uint2 buf[kPtTile];
    __shared__ uint32_t cnt[kMaxGroups], lst[kMaxGroups], gof[kMaxGroups], wtot[kWaves];
    const uint64_t t0 = (uint64_t)blockIdx.x * kPtTile;
    uint32_t v[kPtPer][3];
#pragma unroll
    for (uint32_t q = 0; q < kPtPer; q++) {
        const uint64_t i = t0 + q * kPtBlock + threadIdx.x;
        if (i < n) {
            const uint32_t* t = edges + 3 * i;
            v[q][0] = t[0];
            v[q][1] = t[1];
            v[q][2] = t[2];
        }
    }
    const uint32_t total = (uint32_t)min<uint64_t>(kPtTile, n - t0);
#pragma unroll
    for (uint32_t k = 0; k < 3; k++) {
        for (uint32_t j = threadIdx.x; j < kMaxGroups; j += kPtBlock)
            cnt[j] = 0;
        __syncthreads();
        uint32_t rk[kPtPer];
#pragma unroll
        for (uint32_t q = 0; q < kPtPer; q++) {
            const uint64_t i = t0 + q * kPtBlock + threadIdx.x;
            if (i < n) {
                v[q][k] = local_of(v[q][k], k, P);
                rk[q] = atomicAdd(&cnt[v[q][k] >> kPartGrpShift], 1u);
            }
        }
        __syncthreads();
        groups_exclusive(cnt, NH, lst, wtot);
        const uint32_t* off = off1 + (uint64_t)k * NH * nt1;
        for (uint32_t h = threadIdx.x; h < NH; h += kPtBlock)
            gof[h] = off[(uint64_t)h * nt1 + blockIdx.x];
        __syncthreads();
#pragma unroll
        for (uint32_t q = 0; q < kPtPer; q++) {
            const uint64_t i = t0 + q * kPtBlock + threadIdx.x;
            if (i < n)
                buf[lst[v[q][k] >> kPartGrpShift] + rk[q]] = make_uint2(v[q][k], (uint32_t)i);
        }
        __syncthreads();
        uint2* out = k == 0 ? out0 : (k == 1 ? out1 : out2);
        for (uint32_t s = threadIdx.x; s < total; s += kPtBlock) {
            const uint2 x = buf[s];
            const uint32_t h = x.x >> kPartGrpShift;
            out[(uint64_t)gof[h] + (s - lst[h])] = x;
        }
        __syncthreads();  // buf, cnt and lst are reused by the next part
    }
}

// ---- group bounds and second-pass tile bases (one block) ---------------------------------------
__global__ __launch_bounds__(kPtBlock) void k_part_groups(const uint32_t* __restrict__ off1, uint32_t NH, uint64_t nt1,
                                                          uint64_t n, uint32_t* __restrict__ ginfo)
{
    __shared__ uint32_t hs[kMaxGroups + 1], tiles[kMaxGroups], tb[kMaxGroups], wtot[kWaves];
    for (uint32_t h = threadIdx.x; h < NH; h += kPtBlock)
        hs[h] = off1[(uint64_t)h * nt1];
    if (threadIdx.x == 0)
        hs[NH] = (uint32_t)n;
    __syncthreads();
    for (uint32_t h = threadIdx.x; h < NH; h += kPtBlock)
        tiles[h] = (hs[h + 1] - hs[h] + kPtTile - 1) / kPtTile;
    __syncthreads();
    groups_exclusive(tiles, NH, tb, wtot);
    __syncthreads();
    for (uint32_t h = threadIdx.x; h <= NH; h += kPtBlock) {
        ginfo[h] = hs[h];
        ginfo[kMaxGroups + 1 + h] = h < NH ? tb[h] : tb[NH - 1] + tiles[NH - 1];
    }
}

// Group of second-pass tile b (the one group whose tile range holds b); s_h is LDS.
__device__ __forceinline__ uint32_t group_of_tile(const GroupInfo& g, uint32_t NH, uint32_t b, uint32_t* s_h)
{
    for (uint32_t h = threadIdx.x; h < NH; h += kPtBlock)
        if (g.tbase[h] <= b && b < g.tbase[h + 1])
            *s_h = h;
    __syncthreads();
    return *s_h;
}

// ---- pass 2 histograms: bucket digits per (group, tile) ----------------------------------------
template <class R>
__global__ __launch_bounds__(kPtBlock) void k_part_hist2(const R* __restrict__ in, const uint32_t* __restrict__ ginfo,
                                                         uint32_t NH, uint32_t bsh, uint32_t* __restrict__ hist2)
{
    __shared__ uint32_t c[kDigits];
    __shared__ uint32_t s_h;
    const GroupInfo g(ginfo);
    const uint32_t b = blockIdx.x;
    const uint32_t T2 = g.tbase[NH];
    if (b >= T2) {  // beyond the last tile: zero entries keep the scan's tail exact
        if (threadIdx.x < kDigits)
            hist2[(uint64_t)b * kDigits + threadIdx.x] = 0;
        return;
    }
    if (threadIdx.x < kDigits)
        c[threadIdx.x] = 0;
    const uint32_t h = group_of_tile(g, NH, b, &s_h);
    const uint32_t j = b - g.tbase[h], tiles = g.tbase[h + 1] - g.tbase[h];
    const uint64_t lo = (uint64_t)g.hstart[h] + (uint64_t)j * kPtTile;
    const uint64_t hi = min<uint64_t>(lo + kPtTile, g.hstart[h + 1]);
    for (uint64_t i = lo + threadIdx.x; i < hi; i += kPtBlock)
        atomicAdd(&c[(in[i].x >> bsh) & (kDigits - 1)], 1u);
    __syncthreads();
    if (threadIdx.x < kDigits)
        hist2[(uint64_t)g.tbase[h] * kDigits + (uint64_t)threadIdx.x * tiles + j] = c[threadIdx.x];
}

// ---- pass 2 scatter: pairs grouped by bucket key >> bsh ----------------------------------------
template <class R>
__global__ __launch_bounds__(kPtBlock) void k_part_scatter2(const R* __restrict__ in, const uint32_t* __restrict__ ginfo,
                                                            uint32_t NH, uint32_t bsh, const uint32_t* __restrict__ off2,
                                                            R* __restrict__ out)
{
    __shared__ R buf[kPtTile];
    __shared__ uint32_t cnt[kDigits], lst[kDigits], gof[kDigits], wtot[kWaves];
    __shared__ uint32_t s_h;
    const GroupInfo g(ginfo);
    const uint32_t b = blockIdx.x;
    if (b >= g.tbase[NH])
        return;
    if (threadIdx.x < kDigits)
        cnt[threadIdx.x] = 0;
    const uint32_t h = group_of_tile(g, NH, b, &s_h);
    const uint32_t j = b - g.tbase[h], tiles = g.tbase[h + 1] - g.tbase[h];
    const uint64_t lo = (uint64_t)g.hstart[h] + (uint64_t)j * kPtTile;
    const uint32_t total = (uint32_t)(min<uint64_t>(lo + kPtTile, g.hstart[h + 1]) - lo);
    R p[kPtPer];
    uint32_t rk[kPtPer];
#pragma unroll
    for (uint32_t q = 0; q < kPtPer; q++) {
        const uint32_t i = q * kPtBlock + threadIdx.x;
        if (i < total) {
            p[q] = in[lo + i];
            rk[q] = atomicAdd(&cnt[(p[q].x >> bsh) & (kDigits - 1)], 1u);
        }
    }
    __syncthreads();
    const uint32_t x = threadIdx.x < kDigits ? cnt[threadIdx.x] : 0u;
    const uint32_t ex = block_exclusive(x, wtot);
    if (threadIdx.x < kDigits) {
        lst[threadIdx.x] = ex;
        gof[threadIdx.x] = off2[(uint64_t)g.tbase[h] * kDigits + (uint64_t)threadIdx.x * tiles + j];
    }
    __syncthreads();
#pragma unroll
    for (uint32_t q = 0; q < kPtPer; q++) {
        const uint32_t i = q * kPtBlock + threadIdx.x;
        if (i < total)
            buf[lst[(p[q].x >> bsh) & (kDigits - 1)] + rk[q]] = p[q];
    }
    __syncthreads();
    for (uint32_t s = threadIdx.x; s < total; s += kPtBlock) {
        const R q = buf[s];
        const uint32_t d = (q.x >> bsh) & (kDigits - 1);
        out[(uint64_t)gof[d] + (s - lst[d])] = q;
    }
}

// Start of bucket b (group b >> 8, digit b & 255) in the second pass's output; n past the end.
__device__ __forceinline__ uint64_t bucket_start(const GroupInfo& g, const uint32_t* off2, uint32_t NH, uint64_t n,
                                                 uint32_t b)
{
    const uint32_t h = b >> 8, d = b & 255u;
    if (h >= NH)
        return n;
    const uint32_t tiles = g.tbase[h + 1] - g.tbase[h];
    if (tiles == 0)
        return g.hstart[h];
    return off2[(uint64_t)g.tbase[h] * kDigits + (uint64_t)d * tiles];
}

// ---- per-bucket accumulation of part k's records in LDS ---------------------------------------
__global__ __launch_bounds__(kAccBlock) void k_part_accum(const uint2* __restrict__ in, const uint32_t* __restrict__ ginfo,
                                                         uint32_t NH, const uint32_t* __restrict__ off2, uint64_t n,
                                                         uint32_t k, uint64_t P, uint64_t* __restrict__ rec)
{
    __shared__ unsigned long long lrec[1u << kVxShift];
    const GroupInfo g(ginfo);
    const uint32_t b = blockIdx.x;
    for (uint32_t j = threadIdx.x; j < (1u << kVxShift); j += kAccBlock)
        lrec[j] = 0;
    const uint64_t lo = bucket_start(g, off2, NH, n, b);
    const uint64_t hi = bucket_start(g, off2, NH, n, b + 1);
    __syncthreads();
    for (uint64_t i = lo + threadIdx.x; i < hi; i += kAccBlock) {
        const uint2 p = in[i];
        atomicAdd(&lrec[p.x & ((1u << kVxShift) - 1)], (unsigned long long)(Rec::kOne + p.y));
    }
    __syncthreads();
    const uint64_t v0 = (uint64_t)b << kVxShift;
    const uint32_t cnt = (uint32_t)min<uint64_t>(1u << kVxShift, P - v0);
    uint64_t* dst = rec + (uint64_t)k * P + v0;
    for (uint32_t j = threadIdx.x; j < cnt; j += kAccBlock)
        dst[j] = lrec[j];
}

// ---- one round's update list applied per bucket of 2^14 vertices ---------------------------
// The bucket's deletes (vertex v, edge e) are summed per vertex in LDS -- degree and label sum
// are both additive -- and each touched record is read, reduced by its sum and written back
// once.  A record left at degree 1 had at least two edges when the round began, so its last
// edge is alive and not in this round's layer (an edge of the layer that had it as a non-hinge
// vertex sent a delete here, and it cannot be that edge's hinge, whose degree was 1): the
// record claims that edge for the next round, from its part.  A record left at 0 needs nothing.
__global__ __launch_bounds__(kAccBlock) void k_update_accum(const uint2* __restrict__ in,
                                                           const uint32_t* __restrict__ ginfo, uint32_t NH,
                                                           const uint32_t* __restrict__ off2, uint64_t count,
                                                           uint64_t m, uint64_t P, uint64_t* __restrict__ rec,
                                                           uint2* __restrict__ claims, uint64_t ccap,
                                                           unsigned long long* __restrict__ ccount, Ctrl* ctrl)
{
    __shared__ unsigned long long tab[1u << kVxShift];
    __shared__ uint32_t wtot[kAccBlock / kWave];
    __shared__ unsigned long long s_base;
    constexpr uint32_t kMask = (1u << kVxShift) - 1;
    const GroupInfo g(ginfo);
    const uint32_t b = blockIdx.x;
    const uint64_t lo = bucket_start(g, off2, NH, count, b);
    const uint64_t hi = bucket_start(g, off2, NH, count, b + 1);
    if (lo == hi)
        return;  // uniform per block
    for (uint32_t j = threadIdx.x; j < (1u << kVxShift); j += kAccBlock)
        tab[j] = 0;
    __syncthreads();
    for (uint64_t i = lo + threadIdx.x; i < hi; i += kAccBlock) {
        const uint2 d = in[i];
        atomicAdd(&tab[d.x & kMask], (unsigned long long)(Rec::kOne + d.y));
    }
    __syncthreads();
    // Each thread takes kUpdPer records, kAccBlock apart (coalesced), and has all their loads
    // in flight before it uses any; one device atomic places the bucket's claims.
    const uint64_t v0 = (uint64_t)b << kVxShift;
    const uint32_t cnt = (uint32_t)min<uint64_t>(1u << kVxShift, m - v0);
    unsigned long long d[kUpdPer];
    uint64_t x[kUpdPer];
#pragma unroll
    for (uint32_t q = 0; q < kUpdPer; q++) {
        const uint32_t j = q * kAccBlock + threadIdx.x;
        d[q] = j < cnt ? tab[j] : 0ull;
    }
#pragma unroll
    for (uint32_t q = 0; q < kUpdPer; q++)
        x[q] = d[q] ? rec[v0 + q * kAccBlock + threadIdx.x] : 0ull;
    uint32_t mine = 0, changed = 0;
#pragma unroll
    for (uint32_t q = 0; q < kUpdPer; q++) {
        if (d[q]) {
            changed++;
            x[q] -= d[q];
            rec[v0 + q * kAccBlock + threadIdx.x] = x[q];
            mine += Rec::deg(x[q]) == 1 ? 1u : 0u;
        }
    }
    // claims and changed records in one scan: claims in the low 16 bits (at most 2^14 each)
    const uint32_t pre = block_exclusive<kAccBlock>(mine | changed << 16, wtot);
    const uint32_t rank = pre & 0xFFFFu;
    if (threadIdx.x == kAccBlock - 1) {
        const uint32_t total = rank + mine, all = (pre >> 16) + changed;
        s_base = total ? atomicAdd(ccount, (unsigned long long)total) : 0ull;
        if (total)
            atomicAdd(&ctrl->ftail, (unsigned long long)total);
        atomicAdd(&ctrl->updates, (unsigned long long)(hi - lo));
        atomicAdd(&ctrl->touched, (unsigned long long)all);
    }
    __syncthreads();
    uint64_t at = s_base + rank;
#pragma unroll
    for (uint32_t q = 0; q < kUpdPer; q++) {
        if (d[q] && Rec::deg(x[q]) == 1) {
            const uint32_t v = (uint32_t)(v0 + q * kAccBlock + threadIdx.x);
            if (at < ccap)
                claims[at] = make_uint2((uint32_t)Rec::edge(x[q]), part_of(v, P));
            at++;
        }
    }
}

// ---- resolve one round's claims, bucket by bucket of 2^16 edges -----------------------------
// Every record is (edge c, position p) -- a claim from c's vertex in part p -- or
// (c, 4 | p) -- a cancel from the same vertex, which marks its claim stale (the vertex lost
// both its edges in one round).  Each (c, p) claims at most once and cancels at most once, so
// an edge's byte in the LDS table collects its claim bits (0..2) and cancel bits (4..6); the
// lowest position claimed and not cancelled is the hinge, and that claim is the winner and
// appends (c, hinge | live positions << 8) to the layer.  The grid is persistent: a block walks buckets b,
// b + grid, ... so sparse rounds cost few launches.
// 64 KiB table, 15 KiB appender and the bounds of kResWin buckets: two blocks per compute unit
using ClaimAppender = BlockAppender<uint2, kResBlock, 3 * kResBlock + kResBlock / 4 * 3>;
constexpr uint32_t kResGridPerCU = 2;
constexpr uint32_t kResWin = 128;

__global__ __launch_bounds__(kResBlock) void k_claims_resolve(const uint2* __restrict__ in,
                                                              const uint32_t* __restrict__ ginfo, uint32_t NH,
                                                              const uint32_t* __restrict__ off2, uint64_t count,
                                                              uint32_t nbuckets, uint3* __restrict__ slots,
                                                              const uint64_t* __restrict__ lstart,
                                                              unsigned long long* __restrict__ lcount, uint32_t r,
                                                              Ctrl* ctrl)
{
    __shared__ uint32_t tab[(1u << kClShift) / 4];
    __shared__ ClaimAppender app;
    __shared__ unsigned long long s_fresh;
    __shared__ uint32_t s_lo[kResWin + 1];  // bucket starts of the current window (count < 2^32)
    constexpr uint32_t kMask = (1u << kClShift) - 1;
    const GroupInfo g(ginfo);
    const uint64_t base = lstart[r];
    auto out = [slots, base](uint64_t i, uint2 v) { slots[base + i] = make_uint3(v.x, v.y, 0u); };
    if (threadIdx.x == 0)
        s_fresh = 0;
    app.init();
    unsigned long long fresh = 0;
    // a contiguous range of buckets per block; each window's bounds are read in parallel, so an
    // empty bucket costs no dependent global loads
    const uint32_t per = (nbuckets + gridDim.x - 1) / gridDim.x;
    const uint32_t b0 = (uint32_t)min<uint64_t>(nbuckets, (uint64_t)blockIdx.x * per);
    const uint32_t b1 = (uint32_t)min<uint64_t>(nbuckets, (uint64_t)b0 + per);
    for (uint32_t w0 = b0; w0 < b1; w0 += kResWin) {
        const uint32_t w1 = min(b1, w0 + kResWin);
        for (uint32_t j = threadIdx.x; j <= w1 - w0; j += kResBlock)
            s_lo[j] = (uint32_t)bucket_start(g, off2, NH, count, w0 + j);
        __syncthreads();
        for (uint32_t b = w0; b < w1; b++) {
            const uint64_t lo = s_lo[b - w0];
            const uint64_t hi = s_lo[b - w0 + 1];
            if (lo == hi)
                continue;  // uniform per block
            for (uint64_t i = lo + threadIdx.x; i < hi; i += kResBlock)
                tab[(in[i].x & kMask) >> 2] = 0u;
            __syncthreads();
            for (uint64_t i = lo + threadIdx.x; i < hi; i += kResBlock) {
                const uint2 c = in[i];
                atomicOr(&tab[(c.x & kMask) >> 2], 1u << (8 * (c.x & 3) + c.y));
            }
            __syncthreads();
            for (uint64_t i0 = lo; i0 < hi; i0 += kResBlock) {
                const uint64_t i = i0 + threadIdx.x;
                bool win = false;
                uint2 c = make_uint2(0u, 0u);
                if (i < hi) {
                    c = in[i];
                    const uint32_t t = tab[(c.x & kMask) >> 2] >> (8 * (c.x & 3));
                    const uint32_t live = t & ~(t >> 4) & 7u;
                    win = c.y < 4 && live != 0 && (uint32_t)__builtin_ctz(live) == c.y;
                    fresh += (c.y < 4 && ((live >> c.y) & 1u)) ? 1u : 0u;
                    c.y |= live << 8;  // the layer entry also names every position at degree 1
                }
                app.push(win, c, false, c, &lcount[r], out);
            }
            __syncthreads();  // the table is reused by the next bucket
        }
        __syncthreads();  // the window's bounds are reused by the next window
    }
    app.flush(&lcount[r], out);
    if (fresh)
        atomicAdd(&s_fresh, fresh);
    __syncthreads();
    if (threadIdx.x == 0 && s_fresh)
        atomicAdd(&ctrl->claims, s_fresh);
}

// Byte offsets inside the auxiliary buffer of one partition: first-pass histograms
// [NH][nt1], second-pass histograms [(nt1 + NH) * 256], group table, scan scratch.
struct AuxLayout {
    size_t hist1, hist2, ginfo, scan, scan_bytes, total;
};

AuxLayout aux_layout(uint64_t h1_entries, uint64_t n, uint32_t NH)
{
    const uint64_t nt1 = (n + kPtTile - 1) / kPtTile, h2 = (nt1 + NH) * kDigits;
    AuxLayout L{};
    size_t off = 0;
    auto take = [&off](size_t bytes) {
        off = (off + 255) & ~(size_t)255;
        size_t at = off;
        off += bytes;
        return at;
    };
    L.hist1 = take(h1_entries * 4);
    L.hist2 = take(h2 * 4);
    L.ginfo = take((2 * kMaxGroups + 2) * 4);
    L.scan_bytes = std::max(scan_scratch_bytes(h1_entries), scan_scratch_bytes(h2));
    L.scan = take(L.scan_bytes);
    L.total = off;
    return L;
}

uint32_t groups_of(uint64_t keys, uint32_t gsh) { return (uint32_t)((keys + (1ull << gsh) - 1) >> gsh); }
uint64_t tiles_of(uint64_t n) { return (n + kPtTile - 1) / kPtTile; }

// Build aux: three parts' first-pass histograms of n edges over P vertices.
AuxLayout build_aux(uint64_t n, uint64_t P)
{
    const uint32_t NH = groups_of(P, kPartGrpShift);
    return aux_layout(3ull * NH * tiles_of(n), n, NH);
}

// Claims aux: up to m claims keyed by edge ids below n.
AuxLayout claims_aux(uint64_t m, uint64_t n)
{
    const uint32_t NH = groups_of(n, kClShift + 8);
    return aux_layout((uint64_t)NH * tiles_of(m), m, NH);
}

// Update-list aux: up to m deletes keyed by vertex ids below m.
AuxLayout updates_aux(uint64_t m)
{
    const uint32_t NH = groups_of(m, kPartGrpShift);
    return aux_layout((uint64_t)NH * tiles_of(m), m, NH);
}

// Second pass + per-bucket kernel, after the first pass left the pairs grouped in mid.
template <class R, class Last>
hipError_t second_pass_then(uint64_t n, uint32_t gsh, uint32_t NH, const uint32_t* off1, R* mid, R* out,
                            const AuxLayout& L, uint8_t* base, Last last, hipStream_t s)
{
    const uint64_t nt1 = tiles_of(n), nt2 = nt1 + NH;
    uint32_t* hist2 = reinterpret_cast<uint32_t*>(base + L.hist2);
    uint32_t* ginfo = reinterpret_cast<uint32_t*>(base + L.ginfo);
    void* scan = base + L.scan;
    hipError_t err;
    k_part_groups<<<1, kPtBlock, 0, s>>>(off1, NH, nt1, n, ginfo);
    k_part_hist2<<<(unsigned)nt2, kPtBlock, 0, s>>>(mid, ginfo, NH, gsh - 8, hist2);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    err = launch_scan_u32(hist2, nt2 * kDigits, hist2, scan, L.scan_bytes, s);
    if (err != hipSuccess) return err;
    k_part_scatter2<<<(unsigned)nt2, kPtBlock, 0, s>>>(mid, ginfo, NH, gsh - 8, hist2, out);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    return last(ginfo, hist2);
}

// Both passes + per-bucket kernel, after the first-pass histograms (off1, scanned here).
template <class Src, class Last>
hipError_t partition_then(Src src, uint64_t n, uint32_t gsh, uint32_t NH, uint32_t* off1, typename Src::Rec* mid,
                          typename Src::Rec* out, const AuxLayout& L, uint8_t* base, Last last, hipStream_t s)
{
    const uint64_t nt1 = tiles_of(n);
    hipError_t err = launch_scan_u32(off1, (uint64_t)NH * nt1, off1, base + L.scan, L.scan_bytes, s);
    if (err != hipSuccess) return err;
    k_part_scatter1<Src><<<(unsigned)nt1, kPtBlock, 0, s>>>(src, n, gsh, NH, nt1, off1, mid);
    return second_pass_then(n, gsh, NH, off1, mid, out, L, base, last, s);
}

}  // namespace

size_t part_aux_bytes(uint64_t n, uint64_t P, bool lists)
{
    size_t b = build_aux(n, P).total;
    if (lists)
        b = std::max({b, claims_aux(3 * P, n).total, updates_aux(3 * P).total});
    return b;
}

PartHist1 part_hist1(void* aux, uint64_t n, uint64_t P)
{
    const AuxLayout L = build_aux(n, P);
    return PartHist1{reinterpret_cast<uint32_t*>(reinterpret_cast<uint8_t*>(aux) + L.hist1),
                     groups_of(P, kPartGrpShift), tiles_of(n)};
}

hipError_t launch_part_build(const uint32_t* edges, uint64_t n, uint64_t P, uint64_t* rec, uint2* pairs1,
                             uint2* pairs2, uint2* extra1, uint2* extra2, void* aux, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const AuxLayout L = build_aux(n, P);
    uint8_t* base = reinterpret_cast<uint8_t*>(aux);
    uint32_t* hist1 = reinterpret_cast<uint32_t*>(base + L.hist1);
    const uint32_t NH = groups_of(P, kPartGrpShift);
    const uint64_t nt1 = tiles_of(n), nb = (P + (1ull << kVxShift) - 1) >> kVxShift;
    if (NH > kPartMaxGroups || nt1 > 0x7FFFFFFFull || n >= 0xFFFFFFFFull) return hipErrorInvalidValue;
    if (extra1 && extra2) {
        // one first pass for the three parts, then each part's second pass and accumulation
        for (uint32_t k = 0; k < 3; k++) {
            uint32_t* off1 = hist1 + (uint64_t)k * NH * nt1;
            hipError_t err = launch_scan_u32(off1, (uint64_t)NH * nt1, off1, base + L.scan, L.scan_bytes, s);
            if (err != hipSuccess) return err;
        }
        k_part_scatter1_x3<<<(unsigned)nt1, kPtBlock, 0, s>>>(edges, n, P, NH, nt1, hist1, pairs1, extra1, extra2);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
        uint2* const first[3] = {pairs1, extra1, extra2};
        for (uint32_t k = 0; k < 3; k++) {
            err = second_pass_then(
                n, kPartGrpShift, NH, hist1 + (uint64_t)k * NH * nt1, first[k], pairs2, L, base,
                [&](const uint32_t* ginfo, const uint32_t* off2) {
                    k_part_accum<<<(unsigned)nb, kAccBlock, 0, s>>>(pairs2, ginfo, NH, off2, n, k, P, rec);
                    return hipGetLastError();
                },
                s);
            if (err != hipSuccess) return err;
        }
        return hipSuccess;
    }
    for (uint32_t k = 0; k < 3; k++) {
        uint32_t* off1 = hist1 + (uint64_t)k * NH * nt1;
        hipError_t err = partition_then(
            EdgeColumn{edges, k, P}, n, kPartGrpShift, NH, off1, pairs1, pairs2, L, base,
            [&](const uint32_t* ginfo, const uint32_t* off2) {
                k_part_accum<<<(unsigned)nb, kAccBlock, 0, s>>>(pairs2, ginfo, NH, off2, n, k, P, rec);
                return hipGetLastError();
            },
            s);
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

namespace {

unsigned resident_blocks(uint32_t per_cu)
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    return per_cu * (unsigned)cus;
}

}  // namespace

hipError_t launch_claims_resolve(const PeelState& st, uint32_t r, uint64_t count, bool in_tmp, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    const uint32_t gsh = kClShift + 8;
    const AuxLayout L = claims_aux(st.m, st.n);
    uint8_t* base = reinterpret_cast<uint8_t*>(st.aux);
    uint32_t* hist1 = reinterpret_cast<uint32_t*>(base + L.hist1);
    const uint32_t NH = groups_of(st.n, gsh);
    const uint64_t nt1 = tiles_of(count), nb = (st.n + (1ull << kClShift) - 1) >> kClShift;
    if (count > st.m || NH > kMaxGroups || nt1 > 0x7FFFFFFFull) return hipErrorInvalidValue;
    uint2* list = in_tmp ? st.claims_tmp : st.claims;
    uint2* other = in_tmp ? st.claims : st.claims_tmp;
    k_part_hist1<<<(unsigned)nt1, kPtBlock, 0, s>>>(Records{list}, count, gsh, NH, nt1, hist1);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    return partition_then(
        Records{list}, count, gsh, NH, hist1, other, list, L, base,
        [&](const uint32_t* ginfo, const uint32_t* off2) {
            const uint64_t grid = std::min<uint64_t>(nb, resident_blocks(kResGridPerCU));
            k_claims_resolve<<<(unsigned)grid, kResBlock, 0, s>>>(list, ginfo, NH, off2, count, (uint32_t)nb,
                                                                st.slots, st.lstart, st.lcount, r, st.ctrl);
            return hipGetLastError();
        },
        s);
}

// HEM: bucket_off[b] for b in [0, 2^k] from the second pass's scan
__global__ __launch_bounds__(256) void k_hem_bucket_off(const uint32_t* __restrict__ ginfo, uint32_t NH,
                                                        const uint32_t* __restrict__ off2, uint64_t n, uint32_t B,
                                                        uint64_t* __restrict__ bucket_off)
{
    const GroupInfo g(ginfo);
    for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b <= B; b += gridDim.x * blockDim.x)
        bucket_off[b] = bucket_start(g, off2, NH, n, b);
}

size_t hem_aux_bytes(uint64_t n, uint32_t k)
{
    const uint32_t NH = 1u << (k - 8);
    return aux_layout((uint64_t)NH * tiles_of(n), n, NH).total;
}

namespace {

template <class R>
hipError_t hem_partition(R* rec, uint64_t n, uint32_t k, R* tmp, uint64_t* bucket_off, void* aux, hipStream_t s)
{
    // the group digit is x >> (40 - k): k >= 9 keeps the shift below 32 (at least two groups)
    if (k < 9 || k > 18) return hipErrorInvalidValue;
    const uint32_t NH = 1u << (k - 8), gsh = 40 - k, B = 1u << k;
    const AuxLayout L = aux_layout((uint64_t)NH * tiles_of(n), n, NH);
    uint8_t* base = reinterpret_cast<uint8_t*>(aux);
    uint32_t* hist1 = reinterpret_cast<uint32_t*>(base + L.hist1);
    const uint64_t nt1 = tiles_of(n);
    if (n == 0) return launch_zero(bucket_off, (B + 1ull) * sizeof(uint64_t), s);
    if (nt1 > 0x7FFFFFFFull || n >= 0xFFFFFFFFull) return hipErrorInvalidValue;
    k_part_hist1<<<(unsigned)nt1, kPtBlock, 0, s>>>(RecordsT<R>{rec}, n, gsh, NH, nt1, hist1);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    return partition_then(
        RecordsT<R>{rec}, n, gsh, NH, hist1, tmp, rec, L, base,
        [&](const uint32_t* ginfo, const uint32_t* off2) {
            k_hem_bucket_off<<<(B + 256) / 256, 256, 0, s>>>(ginfo, NH, off2, n, B, bucket_off);
            return hipGetLastError();
        },
        s);
}

}  // namespace

hipError_t launch_hem_partition(uint2* rec, uint64_t n, uint32_t k, uint2* tmp, uint64_t* bucket_off, void* aux,
                                hipStream_t s)
{
    return hem_partition(rec, n, k, tmp, bucket_off, aux, s);
}

hipError_t launch_hem_partition(uint4* rec, uint64_t n, uint32_t k, uint4* tmp, uint64_t* bucket_off, void* aux,
                                hipStream_t s)
{
    return hem_partition(rec, n, k, tmp, bucket_off, aux, s);
}

// HEM beyond 2^18 buckets: each coarse bucket b (top kc bits) split, stably, by the next
// k - kc bits (at most 2) into fine buckets b * D + j, one workgroup per coarse bucket;
// fine_off[0 .. 2^k] written.
constexpr uint32_t kRefBlock = 256;

template <class R>
__global__ __launch_bounds__(kRefBlock) void k_hem_refine(const R* __restrict__ in,
                                                          const uint64_t* __restrict__ coarse_off, uint32_t nb,
                                                          uint32_t k, uint32_t d, R* __restrict__ out,
                                                          uint64_t* __restrict__ fine_off)
{
    __shared__ uint32_t s_cnt[4], s_wtot[kRefBlock / kWave][4];
    __shared__ uint64_t s_start[4];
    const uint32_t b = blockIdx.x, D = 1u << d, sh = 32 - k;
    const uint32_t lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const uint64_t lo = coarse_off[b], hi = coarse_off[b + 1];
    if (threadIdx.x < 4)
        s_cnt[threadIdx.x] = 0;
    __syncthreads();
    for (uint64_t i = lo + threadIdx.x; i < hi; i += kRefBlock)
        atomicAdd(&s_cnt[(in[i].x >> sh) & (D - 1)], 1u);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t at = lo;
        for (uint32_t j = 0; j < D; j++) {
            s_start[j] = at;
            fine_off[(uint64_t)b * D + j] = at;
            at += s_cnt[j];
        }
        if (b + 1 == nb)
            fine_off[(uint64_t)nb * D] = hi;
    }
    __syncthreads();
    for (uint64_t c = lo; c < hi; c += kRefBlock) {
        const uint64_t i = c + threadIdx.x;
        const bool have = i < hi;
        const R x = have ? in[i] : R{};
        const uint32_t dg = have ? (x.x >> sh) & (D - 1) : D;
        uint32_t below = 0;
        for (uint32_t j = 0; j < D; j++) {
            const uint64_t mj = __ballot(dg == j);
            if (lane == 0)
                s_wtot[w][j] = (uint32_t)__popcll(mj);
            if (dg == j)
                below = lanes_below(mj);
        }
        __syncthreads();
        if (have) {
            uint64_t pos = s_start[dg] + below;
            for (uint32_t q = 0; q < w; q++)
                pos += s_wtot[q][dg];
            out[pos] = x;
        }
        __syncthreads();
        if (threadIdx.x < D) {
            uint32_t t = 0;
            for (uint32_t q = 0; q < kRefBlock / kWave; q++)
                t += s_wtot[q][threadIdx.x];
            s_start[threadIdx.x] += t;
        }
        __syncthreads();
    }
}

template <class R>
hipError_t hem_refine(const R* in, const uint64_t* coarse_off, uint32_t kc, uint32_t k, R* out, uint64_t* fine_off,
                      hipStream_t s)
{
    if (kc < 9 || kc > 18 || k <= kc || k - kc > 2) return hipErrorInvalidValue;
    k_hem_refine<<<1u << kc, kRefBlock, 0, s>>>(in, coarse_off, 1u << kc, k, k - kc, out, fine_off);
    return hipGetLastError();
}

hipError_t launch_hem_refine(const uint2* in, const uint64_t* coarse_off, uint32_t kc, uint32_t k, uint2* out,
                             uint64_t* fine_off, hipStream_t s)
{
    return hem_refine(in, coarse_off, kc, k, out, fine_off, s);
}

hipError_t launch_hem_refine(const uint4* in, const uint64_t* coarse_off, uint32_t kc, uint32_t k, uint4* out,
                             uint64_t* fine_off, hipStream_t s)
{
    return hem_refine(in, coarse_off, kc, k, out, fine_off, s);
}

// Out-of-core HEM, first level: one chunk's signature records grouped by their top k - 8 bits
// (the partition's first pass alone) into out; the chunk's NH + 1 group starts are copied to
// host_gstart (pageable or pinned host memory, valid once the stream has reached the copy).
template <class R>
hipError_t hem_group_chunk(const R* csig, uint64_t cn, uint32_t k, R* out, void* aux, uint32_t* host_gstart,
                           hipStream_t s)
{
    if (k < 9 || k > 18 || cn == 0) return hipErrorInvalidValue;
    const uint32_t NH = 1u << (k - 8), gsh = 40 - k;
    const uint64_t nt1 = tiles_of(cn);
    if (nt1 > 0x7FFFFFFFull || cn >= 0xFFFFFFFFull) return hipErrorInvalidValue;
    const AuxLayout L = aux_layout((uint64_t)NH * nt1, cn, NH);
    uint8_t* base = reinterpret_cast<uint8_t*>(aux);
    uint32_t* hist1 = reinterpret_cast<uint32_t*>(base + L.hist1);
    uint32_t* ginfo = reinterpret_cast<uint32_t*>(base + L.ginfo);
    k_part_hist1<<<(unsigned)nt1, kPtBlock, 0, s>>>(RecordsT<R>{csig}, cn, gsh, NH, nt1, hist1);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    err = launch_scan_u32(hist1, (uint64_t)NH * nt1, hist1, base + L.scan, L.scan_bytes, s);
    if (err != hipSuccess) return err;
    k_part_scatter1<RecordsT<R>><<<(unsigned)nt1, kPtBlock, 0, s>>>(RecordsT<R>{csig}, cn, gsh, NH, nt1, hist1, out);
    k_part_groups<<<1, kPtBlock, 0, s>>>(hist1, NH, nt1, cn, ginfo);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    return hipMemcpyAsync(host_gstart, ginfo, (NH + 1) * sizeof(uint32_t), hipMemcpyDeviceToHost, s);
}

hipError_t launch_hem_group_chunk(const uint2* csig, uint64_t cn, uint32_t k, uint2* out, void* aux,
                                  uint32_t* host_gstart, hipStream_t s)
{
    return hem_group_chunk(csig, cn, k, out, aux, host_gstart, s);
}

hipError_t launch_hem_group_chunk(const uint4* csig, uint64_t cn, uint32_t k, uint4* out, void* aux,
                                  uint32_t* host_gstart, hipStream_t s)
{
    return hem_group_chunk(csig, cn, k, out, aux, host_gstart, s);
}

// Out-of-core HEM, second level: runs of grouped signatures copied into one batch buffer, one
// workgroup per run (runs are at most 2^16 records; the host checks every run against both
// buffers before the launch).
template <class R>
__global__ __launch_bounds__(256) void k_hem_gather(const R* __restrict__ src, const HemRun* __restrict__ runs,
                                                    R* __restrict__ dst)
{
    const HemRun r = runs[blockIdx.x];
    for (uint32_t i = threadIdx.x; i < r.len; i += 256)
        dst[r.dst + i] = src[r.src + i];
}

template <class R>
hipError_t hem_gather(const R* src, const HemRun* runs, uint32_t nruns, R* dst, hipStream_t s)
{
    if (nruns == 0) return hipSuccess;
    if (nruns > 0x7FFFFFFFu) return hipErrorInvalidValue;
    k_hem_gather<<<nruns, 256, 0, s>>>(src, runs, dst);
    return hipGetLastError();
}

hipError_t launch_hem_gather(const uint2* src, const HemRun* runs, uint32_t nruns, uint2* dst, hipStream_t s)
{
    return hem_gather(src, runs, nruns, dst, s);
}

hipError_t launch_hem_gather(const uint4* src, const HemRun* runs, uint32_t nruns, uint4* dst, hipStream_t s)
{
    return hem_gather(src, runs, nruns, dst, s);
}

hipError_t launch_update_apply(const PeelState& st, uint32_t r, uint64_t count, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    const AuxLayout L = updates_aux(st.m);
    uint8_t* base = reinterpret_cast<uint8_t*>(st.aux);
    uint32_t* hist1 = reinterpret_cast<uint32_t*>(base + L.hist1);
    const uint32_t NH = groups_of(st.m, kPartGrpShift);
    const uint64_t nt1 = tiles_of(count), nb = (st.m + (1ull << kVxShift) - 1) >> kVxShift;
    if (count > st.m || NH > kMaxGroups || nt1 > 0x7FFFFFFFull || nb > 0x7FFFFFFFull || !st.tripartite)
        return hipErrorInvalidValue;
    k_part_hist1<<<(unsigned)nt1, kPtBlock, 0, s>>>(Records{st.claims}, count, kPartGrpShift, NH, nt1, hist1);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    return partition_then(
        Records{st.claims}, count, kPartGrpShift, NH, hist1, st.claims_tmp, st.claims, L, base,
        [&](const uint32_t* ginfo, const uint32_t* off2) {
            k_update_accum<<<(unsigned)nb, kAccBlock, 0, s>>>(st.claims, ginfo, NH, off2, count, st.m, st.P,
                                                              st.rec, st.claims_tmp, st.m, st.ccount + r + 1,
                                                              st.ctrl);
            return hipGetLastError();
        },
        s);
}

}  // namespace mphx
