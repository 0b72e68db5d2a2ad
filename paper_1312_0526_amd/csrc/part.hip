// Vertex records of a tripartite hypergraph (Section 4.1: degree and the label sum of the
// incident edges, packed as in Rec) built without device atomics.
//
// Part k holds the vertices [kP, (k+1)P) and exactly one vertex of every edge.  Its n
// incidences (local vertex u, edge e) are partitioned by u into buckets of 2^14 consecutive
// vertices in two passes -- first by the group digit u >> 22 (at most 342 groups, since
// P < 2^32 / 3), then by the bucket digit (u >> 14) & 255 inside each group -- and each
// bucket's 16384 records are then accumulated with LDS atomics and written out once.  Every
// pass is a histogram / exclusive-scan / scatter over tiles of 16384 elements; a tile is
// ordered by digit in LDS before it is written, so the stores go out as runs of consecutive
// addresses.  The order inside a bucket is not fixed, which the commutative sum does not see.
//
// Group and bucket offsets come from the scans: the scatter of the second pass lays out
// tiles per group, and its scan is ordered (group, bucket digit, tile), so the scanned value
// at (group, digit, tile 0) is where that bucket starts.
#include "common.h"
#include "launch.h"

#include <algorithm>

namespace mphx {

namespace {

constexpr uint32_t kBkShift = 14;
constexpr uint32_t kBkSize = 1u << kBkShift;
constexpr uint32_t kGrpShift = kPartGrpShift;
constexpr uint32_t kMaxGroups = kPartMaxGroups;
constexpr uint32_t kDigits = 256;
constexpr uint32_t kPtBlock = 512;  // two blocks per CU: one loads while the other writes
constexpr uint32_t kPtPer = 16;
constexpr uint32_t kPtTile = kPtBlock * kPtPer;
constexpr uint32_t kWaves = kPtBlock / kWave;
constexpr uint32_t kAccBlock = 1024;

static_assert((kBkShift + 8) == kGrpShift, "a group holds 256 buckets");
static_assert(kPtTile == kPartTile, "first-pass tiles are the hashing kernels' tiles");
static_assert(kPtBlock > 342 && kPtBlock >= kDigits, "one thread per group and per digit");

// Exclusive prefix over the block (one value per thread); wtot is kWaves words of LDS.
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

// Local vertex of part k; an id outside the part is flagged and counted as vertex 0, so the
// histograms and scatters stay consistent and the caller reports the error.
__device__ __forceinline__ uint32_t local_of(uint32_t v, uint32_t k, uint64_t P, bool& bad)
{
    uint64_t u = (uint64_t)v - (uint64_t)k * P;
    if (u >= P) {
        bad = true;
        u = 0;
    }
    return (uint32_t)u;
}

struct GroupInfo {
    const uint32_t* hstart;  // NH + 1 element offsets of the groups
    const uint32_t* tbase;   // NH + 1 tile offsets of the groups (second pass)
    __device__ GroupInfo(const uint32_t* g) : hstart(g), tbase(g + kMaxGroups + 1) {}
};

// ---- pass 1 histograms, all three parts in one read of the edges ----------------------------
__global__ __launch_bounds__(kPtBlock) void k_part_hist1(const uint32_t* __restrict__ edges, uint64_t n, uint64_t P,
                                                         uint32_t NH, uint64_t nt1, uint32_t* __restrict__ hist1,
                                                         Ctrl* ctrl)
{
    __shared__ uint32_t c[3 * kMaxGroups];
    for (uint32_t j = threadIdx.x; j < 3 * kMaxGroups; j += kPtBlock)
        c[j] = 0;
    __syncthreads();
    const uint64_t t0 = (uint64_t)blockIdx.x * kPtTile;
    bool bad = false;
    for (uint32_t q = 0; q < kPtPer; q++) {
        const uint64_t e = t0 + q * kPtBlock + threadIdx.x;
        if (e < n) {
            for (uint32_t k = 0; k < 3; k++) {
                uint32_t u = local_of(edges[3 * e + k], k, P, bad);
                atomicAdd(&c[k * kMaxGroups + (u >> kGrpShift)], 1u);
            }
        }
    }
    if (bad)
        atomicOr(&ctrl->err, kErrBadEdge);
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < 3 * NH; j += kPtBlock) {
        const uint32_t k = j / NH, h = j - k * NH;
        hist1[((uint64_t)k * NH + h) * nt1 + blockIdx.x] = c[k * kMaxGroups + h];
    }
}

// ---- pass 1 scatter of part k: (u, e) pairs grouped by u >> 22 ------------------------------
__global__ __launch_bounds__(kPtBlock) void k_part_scatter1(const uint32_t* __restrict__ edges, uint64_t n, uint32_t k,
                                                            uint64_t P, uint32_t NH, uint64_t nt1,
                                                            const uint32_t* __restrict__ off1, uint2* __restrict__ out)
{
    __shared__ uint2 buf[kPtTile];
    __shared__ uint32_t cnt[kMaxGroups], lst[kMaxGroups], gof[kMaxGroups], wtot[kWaves];
    for (uint32_t j = threadIdx.x; j < kMaxGroups; j += kPtBlock)
        cnt[j] = 0;
    __syncthreads();
    const uint64_t t0 = (uint64_t)blockIdx.x * kPtTile;
    uint32_t u[kPtPer], rk[kPtPer];
    bool bad = false;
#pragma unroll
    for (uint32_t q = 0; q < kPtPer; q++) {
        const uint64_t e = t0 + q * kPtBlock + threadIdx.x;
        if (e < n) {
            u[q] = local_of(edges[3 * e + k], k, P, bad);
            rk[q] = atomicAdd(&cnt[u[q] >> kGrpShift], 1u);
        }
    }
    __syncthreads();
    const uint32_t x = threadIdx.x < NH ? cnt[threadIdx.x] : 0u;
    const uint32_t ex = block_exclusive(x, wtot);
    if (threadIdx.x < NH) {
        lst[threadIdx.x] = ex;
        gof[threadIdx.x] = off1[(uint64_t)threadIdx.x * nt1 + blockIdx.x];
    }
    __syncthreads();
#pragma unroll
    for (uint32_t q = 0; q < kPtPer; q++) {
        const uint64_t e = t0 + q * kPtBlock + threadIdx.x;
        if (e < n)
            buf[lst[u[q] >> kGrpShift] + rk[q]] = make_uint2(u[q], (uint32_t)e);
    }
    __syncthreads();
    const uint32_t total = (uint32_t)min<uint64_t>(kPtTile, n - t0);
    for (uint32_t s = threadIdx.x; s < total; s += kPtBlock) {
        const uint2 p = buf[s];
        const uint32_t h = p.x >> kGrpShift;
        out[(uint64_t)gof[h] + (s - lst[h])] = p;
    }
}

// ---- group bounds and second-pass tile bases of part k (one block) ---------------------------
__global__ __launch_bounds__(kPtBlock) void k_part_groups(const uint32_t* __restrict__ off1, uint32_t NH, uint64_t nt1,
                                                          uint64_t n, uint32_t* __restrict__ ginfo)
{
    __shared__ uint32_t hs[kMaxGroups + 1], wtot[kWaves];
    const uint32_t h = threadIdx.x;
    if (h < NH)
        hs[h] = off1[(uint64_t)h * nt1];
    if (h == 0)
        hs[NH] = (uint32_t)n;
    __syncthreads();
    const uint32_t tiles = h < NH ? (hs[h + 1] - hs[h] + kPtTile - 1) / kPtTile : 0u;
    const uint32_t ex = block_exclusive(tiles, wtot);
    if (h <= NH) {
        ginfo[h] = hs[h];
        if (h < NH)
            ginfo[kMaxGroups + 1 + h] = ex;
    }
    if (h == NH - 1)
        ginfo[kMaxGroups + 1 + NH] = ex + tiles;
}

// Group of second-pass tile b (the one group whose tile range holds b); s_h is LDS.
__device__ __forceinline__ uint32_t group_of_tile(const GroupInfo& g, uint32_t NH, uint32_t b, uint32_t* s_h)
{
    if (threadIdx.x < NH && g.tbase[threadIdx.x] <= b && b < g.tbase[threadIdx.x + 1])
        *s_h = threadIdx.x;
    __syncthreads();
    return *s_h;
}

// ---- pass 2 histograms of part k: bucket digits per (group, tile) -----------------------------
__global__ __launch_bounds__(kPtBlock) void k_part_hist2(const uint2* __restrict__ in, const uint32_t* __restrict__ ginfo,
                                                         uint32_t NH, uint32_t* __restrict__ hist2)
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
        atomicAdd(&c[(in[i].x >> kBkShift) & (kDigits - 1)], 1u);
    __syncthreads();
    if (threadIdx.x < kDigits)
        hist2[(uint64_t)g.tbase[h] * kDigits + (uint64_t)threadIdx.x * tiles + j] = c[threadIdx.x];
}

// ---- pass 2 scatter of part k: pairs grouped by bucket ----------------------------------------
__global__ __launch_bounds__(kPtBlock) void k_part_scatter2(const uint2* __restrict__ in, const uint32_t* __restrict__ ginfo,
                                                            uint32_t NH, const uint32_t* __restrict__ off2,
                                                            uint2* __restrict__ out)
{
    __shared__ uint2 buf[kPtTile];
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
    uint2 p[kPtPer];
    uint32_t rk[kPtPer];
#pragma unroll
    for (uint32_t q = 0; q < kPtPer; q++) {
        const uint32_t i = q * kPtBlock + threadIdx.x;
        if (i < total) {
            p[q] = in[lo + i];
            rk[q] = atomicAdd(&cnt[(p[q].x >> kBkShift) & (kDigits - 1)], 1u);
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
            buf[lst[(p[q].x >> kBkShift) & (kDigits - 1)] + rk[q]] = p[q];
    }
    __syncthreads();
    for (uint32_t s = threadIdx.x; s < total; s += kPtBlock) {
        const uint2 q = buf[s];
        const uint32_t d = (q.x >> kBkShift) & (kDigits - 1);
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
    __shared__ unsigned long long lrec[kBkSize];
    const GroupInfo g(ginfo);
    const uint32_t b = blockIdx.x;
    for (uint32_t j = threadIdx.x; j < kBkSize; j += kAccBlock)
        lrec[j] = 0;
    const uint64_t lo = bucket_start(g, off2, NH, n, b);
    const uint64_t hi = bucket_start(g, off2, NH, n, b + 1);
    __syncthreads();
    for (uint64_t i = lo + threadIdx.x; i < hi; i += kAccBlock) {
        const uint2 p = in[i];
        atomicAdd(&lrec[p.x & (kBkSize - 1)], (unsigned long long)(Rec::kOne + p.y));
    }
    __syncthreads();
    const uint64_t v0 = (uint64_t)b * kBkSize;
    const uint32_t cnt = (uint32_t)min<uint64_t>(kBkSize, P - v0);
    uint64_t* dst = rec + (uint64_t)k * P + v0;
    for (uint32_t j = threadIdx.x; j < cnt; j += kAccBlock)
        dst[j] = lrec[j];
}

}  // namespace

uint32_t part_groups(uint64_t P) { return (uint32_t)((P + (1ull << kGrpShift) - 1) >> kGrpShift); }
uint64_t part_tiles(uint64_t n) { return (n + kPtTile - 1) / kPtTile; }

size_t part_build_bytes(uint64_t n, uint64_t P, PartBuildLayout* L)
{
    const uint64_t NH = part_groups(P), nt1 = part_tiles(n);
    const uint64_t h1 = 3 * NH * nt1, h2 = (nt1 + NH) * kDigits;
    size_t off = 0;
    auto take = [&off](size_t bytes) {
        off = (off + 255) & ~(size_t)255;
        size_t at = off;
        off += bytes;
        return at;
    };
    size_t o_h1 = take(h1 * 4), o_h2 = take(h2 * 4), o_gi = take((2 * kMaxGroups + 2) * 4);
    size_t sb = std::max(scan_scratch_bytes(NH * nt1), scan_scratch_bytes(h2));
    size_t o_sc = take(sb);
    if (L) {
        L->hist1_off = o_h1;
        L->hist2_off = o_h2;
        L->ginfo_off = o_gi;
        L->scan_off = o_sc;
        L->scan_bytes = sb;
    }
    return off;
}

PartHist1 part_hist1(void* aux, uint64_t n, uint64_t P)
{
    PartBuildLayout L;
    part_build_bytes(n, P, &L);
    return PartHist1{reinterpret_cast<uint32_t*>(reinterpret_cast<uint8_t*>(aux) + L.hist1_off), part_groups(P),
                     part_tiles(n)};
}

hipError_t launch_part_build(const uint32_t* edges, uint64_t n, uint64_t P, uint64_t* rec, uint2* pairs1,
                             uint2* pairs2, void* aux, Ctrl* ctrl, bool hist1_done, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    PartBuildLayout L;
    part_build_bytes(n, P, &L);
    uint8_t* base = reinterpret_cast<uint8_t*>(aux);
    uint32_t* hist1 = reinterpret_cast<uint32_t*>(base + L.hist1_off);
    uint32_t* hist2 = reinterpret_cast<uint32_t*>(base + L.hist2_off);
    uint32_t* ginfo = reinterpret_cast<uint32_t*>(base + L.ginfo_off);
    void* scan = base + L.scan_off;
    const uint32_t NH = part_groups(P);
    const uint64_t nt1 = part_tiles(n), nt2 = nt1 + NH, nb = (P + kBkSize - 1) / kBkSize;
    if (NH > kMaxGroups || nt1 > 0x7FFFFFFFull || n >= 0xFFFFFFFFull) return hipErrorInvalidValue;
    if (!hist1_done)
        k_part_hist1<<<(unsigned)nt1, kPtBlock, 0, s>>>(edges, n, P, NH, nt1, hist1, ctrl);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    for (uint32_t k = 0; k < 3; k++) {
        uint32_t* off1 = hist1 + (uint64_t)k * NH * nt1;
        err = launch_scan_u32(off1, (uint64_t)NH * nt1, off1, scan, L.scan_bytes, s);
        if (err != hipSuccess) return err;
        k_part_scatter1<<<(unsigned)nt1, kPtBlock, 0, s>>>(edges, n, k, P, NH, nt1, off1, pairs1);
        k_part_groups<<<1, kPtBlock, 0, s>>>(off1, NH, nt1, n, ginfo);
        k_part_hist2<<<(unsigned)nt2, kPtBlock, 0, s>>>(pairs1, ginfo, NH, hist2);
        err = hipGetLastError();
        if (err != hipSuccess) return err;
        err = launch_scan_u32(hist2, nt2 * kDigits, hist2, scan, L.scan_bytes, s);
        if (err != hipSuccess) return err;
        k_part_scatter2<<<(unsigned)nt2, kPtBlock, 0, s>>>(pairs1, ginfo, NH, hist2, pairs2);
        k_part_accum<<<(unsigned)nb, kAccBlock, 0, s>>>(pairs2, ginfo, NH, hist2, n, k, P, rec);
        err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

}  // namespace mphx
