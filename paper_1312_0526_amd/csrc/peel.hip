// Peeling kernels for gfx950: packed incidence lists built with device atomics, synchronous
// frontier rounds (Section 4.2 layered peeling), and the canonical order.
//
// One round r is two launches:
//   claim(r): every frontier vertex that still has degree 1 reads its only edge e off its
//             packed record (Section 4.1 RetrieveEdge) and sets bit <its position> in e's
//             claim byte.  The first claimer appends e to the layer array, so each edge of the
//             layer appears once (the dedupe of Section 4.2).  Nothing else changes, so every
//             claimer sees the degrees of the start of the round.
//   apply(r): for each layer edge, hinge = lowest claimed position; the edge is deleted from
//             the vertices that did not claim it (DeleteEdge); a vertex whose degree drops
//             from 2 to 1 joins the next frontier.  Claimers had degree 1, so their only edge
//             is this one and they simply die with it.
// Round bounds are read from device memory, so rounds are enqueued without host round trips;
// a round after the last one finds an empty frontier and does nothing.
#include "common.h"
#include "launch.h"

namespace mphx {

// LDS-staged appender of the frontier / layer arrays (16 KB per block).
using Appender = BlockAppender<256, 4096>;

// ------------------------------------------------------------------------------------------
// Degree + label build from a caller-provided edge list, with validation.
// ------------------------------------------------------------------------------------------
template <class Rec>
__global__ __launch_bounds__(256) void k_edges_build(const uint32_t* __restrict__ edges, uint64_t n,
                                                     uint64_t m, uint64_t* __restrict__ rec, Ctrl* ctrl)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        uint32_t t0 = edges[3 * e], t1 = edges[3 * e + 1], t2 = edges[3 * e + 2];
        bool bad = t0 >= m || t1 >= m || t2 >= m || t0 == t1 || t0 == t2 || t1 == t2;
        if (bad) {
            atomicOr(&ctrl->err, kErrBadEdge);
            continue;
        }
        if constexpr (Rec::kind == 1) {
            uint32_t d = Rec::add_ret(rec, t0, (uint32_t)e);
            d = max(d, Rec::add_ret(rec, t1, (uint32_t)e));
            d = max(d, Rec::add_ret(rec, t2, (uint32_t)e));
            if (d >= kMaxDegree)
                atomicOr(&ctrl->err, kErrDegree);
        } else {
            Rec::add(rec, t0, (uint32_t)e);
            Rec::add(rec, t1, (uint32_t)e);
            Rec::add(rec, t2, (uint32_t)e);
        }
    }
}

// ------------------------------------------------------------------------------------------
// Round-0 frontier: every vertex of degree 1, compacted with one atomic per wave.
// ------------------------------------------------------------------------------------------
template <class Rec>
__global__ __launch_bounds__(256) void k_frontier_init(const uint64_t* __restrict__ rec, uint64_t m,
                                                       uint32_t* __restrict__ front, Ctrl* ctrl)
{
    __shared__ Appender app;
    app.init();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < m; base += stride) {
        uint64_t v = base + threadIdx.x;
        bool one = false;
        if (v < m) {
            uint32_t d = Rec::deg(rec[v]);
            one = d == 1;
            if (d > kMaxDegree)
                atomicOr(&ctrl->err, kErrDegree);
        }
        app.push(one, (uint32_t)v, false, 0u, &ctrl->ftail, front);
    }
    app.flush(&ctrl->ftail, front);
}

// ------------------------------------------------------------------------------------------
// Claim phase of round r.
// ------------------------------------------------------------------------------------------
template <class Rec, bool kTri>
__global__ __launch_bounds__(256) void k_claim(const uint64_t* __restrict__ rec, const uint32_t* __restrict__ front,
                                               const uint32_t* __restrict__ edges, uint32_t* __restrict__ hmask32,
                                               uint32_t* __restrict__ layer, uint64_t* __restrict__ fstart,
                                               Ctrl* ctrl, uint32_t r, uint64_t P, uint64_t n)
{
    const uint64_t lo = fstart[r];
    const uint64_t hi = *(volatile unsigned long long*)&ctrl->ftail;  // no push during a claim
    if (blockIdx.x == 0 && threadIdx.x == 0)
        fstart[r + 1] = hi;
    if (lo + (uint64_t)blockIdx.x * blockDim.x >= hi)
        return;  // whole block idle (uniform)
    __shared__ Appender app;
    __shared__ uint32_t nclaims;
    if (threadIdx.x == 0)
        nclaims = 0;
    app.init();
    uint32_t myclaims = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = lo + (uint64_t)blockIdx.x * blockDim.x; base < hi; base += stride) {
        uint64_t i = base + threadIdx.x;
        bool first = false, claimed = false;
        uint32_t e = 0;
        if (i < hi) {
            uint32_t v = front[i];
            uint64_t x = rec[v];
            if (Rec::deg(x) == 1 && Rec::edge(x) < n) {
                claimed = true;
                e = Rec::edge(x);
                uint32_t k;
                if constexpr (kTri) {
                    k = part_of(v, P);
                } else {
                    const uint32_t* t = edges + 3 * (uint64_t)e;
                    k = t[0] == v ? 0u : (t[1] == v ? 1u : 2u);
                }
                uint32_t sh = 8 * (e & 3);
                uint32_t old = atomicOr(&hmask32[e >> 2], (1u << k) << sh);
                first = ((old >> sh) & 0xFFu) == 0;
            }
        }
        myclaims += claimed;
        app.push(first, e, false, 0u, &ctrl->ltail, layer);
    }
    app.flush(&ctrl->ltail, layer);
    if (myclaims)
        atomicAdd(&nclaims, myclaims);
    __syncthreads();
    if (threadIdx.x == 0 && nclaims)
        atomicAdd(&ctrl->claims, (unsigned long long)nclaims);
}

// ------------------------------------------------------------------------------------------
// Apply phase of round r.  round_out (nullable) receives r for every layer edge.
// ------------------------------------------------------------------------------------------
template <class Rec>
__global__ __launch_bounds__(256) void k_apply(uint64_t* __restrict__ rec, uint32_t* __restrict__ front,
                                               const uint32_t* __restrict__ edges,
                                               const uint32_t* __restrict__ hmask32,
                                               const uint32_t* __restrict__ layer, uint64_t* __restrict__ lstart,
                                               uint32_t* __restrict__ round_out, Ctrl* ctrl, uint32_t r)
{
    const uint64_t lo = lstart[r];
    const uint64_t hi = *(volatile unsigned long long*)&ctrl->ltail;  // no claim during an apply
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        lstart[r + 1] = hi;
        if (hi == lo)
            atomicMin(&ctrl->nrounds, r);
    }
    if (lo + (uint64_t)blockIdx.x * blockDim.x >= hi)
        return;  // whole block idle (uniform)
    __shared__ Appender app;
    app.init();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = lo + (uint64_t)blockIdx.x * blockDim.x; base < hi; base += stride) {
        uint64_t i = base + threadIdx.x;
        uint32_t push0 = 0, push1 = 0;
        uint32_t npush = 0;
        if (i < hi) {
            uint32_t e = layer[i];
            uint32_t mask = claim_mask(hmask32, e);
            if (round_out)
                round_out[e] = r;
            const uint32_t* t = edges + 3 * (uint64_t)e;
            uint32_t v0 = t[0], v1 = t[1], v2 = t[2];
            if (!(mask & 1u) && Rec::del(rec, v0, e) == 2)
                push0 = v0, npush = 1;
            if (!(mask & 2u) && Rec::del(rec, v1, e) == 2) {
                if (npush) push1 = v1; else push0 = v1;
                npush++;
            }
            if (!(mask & 4u) && Rec::del(rec, v2, e) == 2) {
                if (npush) push1 = v2; else push0 = v2;
                npush++;
            }
        }
        app.push(npush >= 1, push0, npush >= 2, push1, &ctrl->ftail, front);
    }
    app.flush(&ctrl->ftail, front);
}

// ------------------------------------------------------------------------------------------
// Per-edge outputs of mphx_peel: core mask and hinge from round[] and the claim bytes.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_peel_finalize(const uint32_t* __restrict__ round,
                                                       const uint32_t* __restrict__ hmask32, uint64_t n,
                                                       uint8_t* __restrict__ core_mask, uint8_t* __restrict__ hinge)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        bool core = round[e] == kRoundCore;
        core_mask[e] = core ? 1 : 0;
        if (hinge) {
            uint32_t mask = claim_mask(hmask32, (uint32_t)e);
            hinge[e] = core ? 0xFF : (uint8_t)__builtin_ctz(mask);
        }
    }
}

// ------------------------------------------------------------------------------------------
// Canonical order: stable LSD counting sort of edge ids by key = round (2-core edges get key
// nrounds, after every layer), 8 bits per pass.  Each pass: per-tile digit histograms,
// one exclusive scan over (digit, tile), then a stable scatter per tile.
// ------------------------------------------------------------------------------------------
constexpr uint32_t kSortTile = 16384;
constexpr uint32_t kSortBlock = 256;

__device__ __forceinline__ uint32_t sort_key(const uint32_t* round, uint32_t id, uint32_t nrounds)
{
    uint32_t r = round[id];
    return r == kRoundCore ? nrounds : r;
}

__global__ __launch_bounds__(256) void k_sort_hist(const uint32_t* __restrict__ round,
                                                   const uint32_t* __restrict__ ids_in, uint64_t n,
                                                   uint32_t nrounds, uint32_t shift, uint32_t nbins,
                                                   uint32_t* __restrict__ tilehist, uint64_t ntiles)
{
    __shared__ uint32_t hist[256];
    hist[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t t0 = (uint64_t)blockIdx.x * kSortTile;
    const uint64_t t1 = min<uint64_t>(t0 + kSortTile, n);
    for (uint64_t j = t0 + threadIdx.x; j < t1; j += kSortBlock) {
        uint32_t id = ids_in ? ids_in[j] : (uint32_t)j;
        uint32_t d = (sort_key(round, id, nrounds) >> shift) & 255u;
        atomicAdd(&hist[d], 1u);
    }
    __syncthreads();
    if (threadIdx.x < nbins)
        tilehist[(uint64_t)threadIdx.x * ntiles + blockIdx.x] = hist[threadIdx.x];
}

__global__ __launch_bounds__(256) void k_sort_scatter(const uint32_t* __restrict__ round,
                                                      const uint32_t* __restrict__ ids_in, uint64_t n,
                                                      uint32_t nrounds, uint32_t shift, uint32_t nbins,
                                                      const uint32_t* __restrict__ tileoff, uint64_t ntiles,
                                                      uint32_t* __restrict__ ids_out)
{
    __shared__ uint32_t running[256];
    __shared__ uint32_t wcnt[kSortBlock / kWave][257];
    const uint32_t w = threadIdx.x / kWave;
    running[threadIdx.x] = threadIdx.x < nbins ? tileoff[(uint64_t)threadIdx.x * ntiles + blockIdx.x] : 0;
    for (uint32_t q = 0; q < kSortBlock / kWave; q++)
        wcnt[q][threadIdx.x] = 0;
    __syncthreads();
    const uint64_t t0 = (uint64_t)blockIdx.x * kSortTile;
    const uint64_t t1 = min<uint64_t>(t0 + kSortTile, n);
    for (uint64_t cbase = t0; cbase < t1; cbase += kSortBlock) {
        uint64_t j = cbase + threadIdx.x;
        bool valid = j < t1;
        uint32_t id = 0, d = 256;  // invalid lanes form their own group (digit 256)
        if (valid) {
            id = ids_in ? ids_in[j] : (uint32_t)j;
            d = (sort_key(round, id, nrounds) >> shift) & 255u;
        }
        uint64_t peers = __ballot(1);
        for (uint32_t bit = 0; bit < 9; bit++) {
            uint64_t b = __ballot((d >> bit) & 1u);
            peers &= ((d >> bit) & 1u) ? b : ~b;
        }
        uint32_t below = lanes_below(peers);
        if (valid && below == 0)
            wcnt[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t off = running[d] + below;
            for (uint32_t q = 0; q < w; q++)
                off += wcnt[q][d];
            ids_out[off] = id;
        }
        __syncthreads();
        uint32_t add = 0;
        for (uint32_t q = 0; q < kSortBlock / kWave; q++) {
            add += wcnt[q][threadIdx.x];
            wcnt[q][threadIdx.x] = 0;
        }
        running[threadIdx.x] += add;
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------------
// Host launchers
// ------------------------------------------------------------------------------------------
static inline unsigned grid_for(uint64_t count, unsigned cap)
{
    uint64_t g = (count + 255) / 256;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

hipError_t launch_edges_build(const uint32_t* edges, uint64_t n, uint64_t m, uint64_t* rec, Ctrl* ctrl,
                              int record, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    unsigned g = grid_for(n, 8192);
    if (record == 1)
        k_edges_build<RecSum><<<g, 256, 0, s>>>(edges, n, m, rec, ctrl);
    else
        k_edges_build<RecXor><<<g, 256, 0, s>>>(edges, n, m, rec, ctrl);
    return hipGetLastError();
}

hipError_t launch_frontier_init(const uint64_t* rec, uint64_t m, uint32_t* front, Ctrl* ctrl, int record,
                                 hipStream_t s)
{
    if (m == 0) return hipSuccess;
    unsigned g = grid_for(m, 8192);
    if (record == 1)
        k_frontier_init<RecSum><<<g, 256, 0, s>>>(rec, m, front, ctrl);
    else
        k_frontier_init<RecXor><<<g, 256, 0, s>>>(rec, m, front, ctrl);
    return hipGetLastError();
}

hipError_t launch_claim(const PeelState& st, uint32_t r, hipStream_t s)
{
    unsigned g = grid_for(st.m, st.grid_cap);
    if (st.record == 1) {
        if (st.tripartite)
            k_claim<RecSum, true><<<g, 256, 0, s>>>(st.rec, st.front, st.edges, st.hmask32, st.layer, st.fstart,
                                                    st.ctrl, r, st.P, st.n);
        else
            k_claim<RecSum, false><<<g, 256, 0, s>>>(st.rec, st.front, st.edges, st.hmask32, st.layer, st.fstart,
                                                     st.ctrl, r, st.P, st.n);
    } else {
        if (st.tripartite)
            k_claim<RecXor, true><<<g, 256, 0, s>>>(st.rec, st.front, st.edges, st.hmask32, st.layer, st.fstart,
                                                    st.ctrl, r, st.P, st.n);
        else
            k_claim<RecXor, false><<<g, 256, 0, s>>>(st.rec, st.front, st.edges, st.hmask32, st.layer, st.fstart,
                                                     st.ctrl, r, st.P, st.n);
    }
    return hipGetLastError();
}

hipError_t launch_apply(const PeelState& st, uint32_t r, hipStream_t s)
{
    unsigned g = grid_for(st.n, st.grid_cap);
    if (st.record == 1)
        k_apply<RecSum><<<g, 256, 0, s>>>(st.rec, st.front, st.edges, st.hmask32, st.layer, st.lstart, st.round_out,
                                          st.ctrl, r);
    else
        k_apply<RecXor><<<g, 256, 0, s>>>(st.rec, st.front, st.edges, st.hmask32, st.layer, st.lstart, st.round_out,
                                          st.ctrl, r);
    return hipGetLastError();
}

hipError_t launch_peel_finalize(const uint32_t* round, const uint32_t* hmask32, uint64_t n, uint8_t* core_mask,
                                uint8_t* hinge, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_peel_finalize<<<grid_for(n, 8192), 256, 0, s>>>(round, hmask32, n, core_mask, hinge);
    return hipGetLastError();
}

uint64_t sort_tiles(uint64_t n) { return (n + kSortTile - 1) / kSortTile; }

hipError_t launch_order_sort(const uint32_t* round, uint64_t n, uint32_t nrounds, uint32_t* order,
                             uint32_t* scratch_ids, uint32_t* tilehist, void* scan_scratch, size_t scan_bytes,
                             hipStream_t s)
{
    if (n == 0) return hipSuccess;
    uint32_t bits = 0;
    while (bits < 32 && (nrounds >> bits) != 0) bits++;
    uint32_t passes = bits == 0 ? 1 : (bits + 7) / 8;
    uint64_t ntiles = sort_tiles(n);
    const uint32_t* in = nullptr;
    for (uint32_t p = 0; p < passes; p++) {
        uint32_t shift = 8 * p;
        uint32_t nbins = (p + 1 == passes) ? ((nrounds >> shift) & 255u) + 1 : 256u;
        // the last pass writes `order`; earlier ones alternate so that this holds
        uint32_t* out = ((passes - 1 - p) % 2 == 0) ? order : scratch_ids;
        k_sort_hist<<<(unsigned)ntiles, kSortBlock, 0, s>>>(round, in, n, nrounds, shift, nbins, tilehist, ntiles);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
        err = launch_scan_u32(tilehist, (uint64_t)nbins * ntiles, tilehist, scan_scratch, scan_bytes, s);
        if (err != hipSuccess) return err;
        k_sort_scatter<<<(unsigned)ntiles, kSortBlock, 0, s>>>(round, in, n, nrounds, shift, nbins, tilehist, ntiles,
                                                              out);
        err = hipGetLastError();
        if (err != hipSuccess) return err;
        in = out;
    }
    return hipSuccess;
}

}  // namespace mphx
