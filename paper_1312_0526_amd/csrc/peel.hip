// Peeling kernels for gfx950: packed incidence records built with device atomics, synchronous
// frontier rounds (Section 4.2 layered peeling), and the canonical order.
//
// A vertex has degree 1 at the start of round r + 1 exactly when round r's deletions took it
// from degree 2 to 1 (or, for round 0, when the build left it at 1).  The thread whose atomic
// DeleteEdge takes a vertex from 2 to 1 gets the vertex's old record back, whose label sum holds
// the two remaining edges, so it knows the vertex's last edge at once and claims it for the
// next round on the spot: atomicMin(state[e], ((r + 1) << 2) | position).  The state word of an
// edge is unclaimed until its round, then (round << 2) | lowest claimed position -- the hinge.
// The first claimer (old value unclaimed) appends the edge to the next layer, so each edge
// enters one layer once (the dedupe of Section 4.2).  A vertex that drops to 1 and then to 0 in
// the same round claims an edge that leaves in that round; that edge's state already holds the
// round, which the later claim cannot lower, so nothing changes.
//
// One launch per round: apply(r) takes layer r = [lstart[r], lstart[r] + count[r]) -- count[r]
// was final when apply(r - 1) ended -- writes each edge's vertices back into its layer slot
// hinge first (for the assignment), deletes the edge at its two other vertices (the hinge has
// degree 1 and dies with it) and appends the next layer through count[r + 1].  Round bounds
// live in device memory, so rounds are enqueued without host round trips; a round after the
// last one finds an empty layer and does nothing.
//
// With claim lists (tripartite graphs), apply(r) appends (edge, position) claims instead of
// the atomicMin, and a deletion that takes a vertex from 1 to 0 appends a cancel for its own
// edge: if that vertex reached degree 1 earlier in the same round, its claim named exactly
// this edge, which leaves in this round, so the pair marks the claim stale.  The lists are
// then resolved bucket by bucket in LDS (part.hip); a resolved layer carries its hinge in the
// slot.  In a dense round apply(r) may instead append the deletes themselves (the degree update
// list of the sort-based round update of Section 4.2), which part.hip applies per vertex
// bucket.
#include "common.h"
#include "launch.h"

#include <type_traits>

namespace mphx {

constexpr int kPeelBlock = 256;
using LayerAppender = BlockAppender<uint32_t, kPeelBlock, 2048>;
using ClaimListAppender = BlockAppender<uint2, kPeelBlock, 2048>;
constexpr uint32_t kCancel = 4;  // claim-list record (edge, kCancel | position): a stale claim

// Position of vertex v in edge e (generic edge lists; tripartite ones use the part).
template <bool kTri>
__device__ __forceinline__ uint32_t position_in(const uint32_t* edges, uint32_t e, uint32_t v, uint64_t P)
{
    if constexpr (kTri) {
        return part_of(v, P);
    } else {
        const uint32_t* t = edges + 3 * (uint64_t)e;
        return t[0] == v ? 0u : (t[1] == v ? 1u : 2u);
    }
}

// ------------------------------------------------------------------------------------------
// Degree + label build from a caller-provided edge list, with validation.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_edges_build(const uint32_t* __restrict__ edges, uint64_t n, uint64_t m,
                                                     uint64_t* __restrict__ rec, Ctrl* ctrl)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        uint32_t t0 = edges[3 * e], t1 = edges[3 * e + 1], t2 = edges[3 * e + 2];
        bool bad = t0 >= m || t1 >= m || t2 >= m || t0 == t1 || t0 == t2 || t1 == t2;
        if (bad) {
            atomicOr(&ctrl->err, kErrBadEdge);
            continue;
        }
        Rec::add(rec, t0, (uint32_t)e);
        Rec::add(rec, t1, (uint32_t)e);
        Rec::add(rec, t2, (uint32_t)e);
    }
}

// ------------------------------------------------------------------------------------------
// Round 0: every vertex of degree 1 claims its edge; first claimers fill layer 0.  Also checks
// the degrees: a field above 255, or a total that differs from 3n (a wrapped field), means some
// degree exceeded 255.
// ------------------------------------------------------------------------------------------
template <bool kTri>
__global__ __launch_bounds__(kPeelBlock) void k_round0(const uint64_t* __restrict__ rec, uint64_t m,
                                                       const uint32_t* __restrict__ edges, uint64_t P, uint64_t n,
                                                       uint32_t* __restrict__ state, uint3* __restrict__ slots,
                                                       unsigned long long* __restrict__ lcount, Ctrl* ctrl)
{
    __shared__ LayerAppender app;
    __shared__ unsigned long long s_deg, s_ones, s_claims;
    if (threadIdx.x == 0)
        s_deg = s_ones = s_claims = 0;
    app.init();
    auto out = [slots](uint64_t i, uint32_t e) { slots[i].x = e; };
    unsigned long long mydeg = 0, myones = 0, myclaims = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < m; base += stride) {
        uint64_t v = base + threadIdx.x;
        bool first = false;
        uint32_t e = 0;
        if (v < m) {
            uint64_t x = rec[v];
            uint32_t d = Rec::deg(x);
            mydeg += d;
            if (d > kMaxDegree)
                atomicOr(&ctrl->err, kErrDegree);
            if (d == 1 && Rec::edge(x) < n) {
                e = Rec::edge(x);
                uint32_t old = atomicMin(&state[e], position_in<kTri>(edges, e, (uint32_t)v, P));
                first = old == kUnclaimed;
                myones++;
                myclaims++;
            }
        }
        app.push(first, e, false, 0u, &lcount[0], out);
    }
    app.flush(&lcount[0], out);
    if (mydeg) atomicAdd(&s_deg, mydeg);
    if (myones) atomicAdd(&s_ones, myones);
    if (myclaims) atomicAdd(&s_claims, myclaims);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_deg) atomicAdd(&ctrl->degsum, s_deg);
        if (s_ones) atomicAdd(&ctrl->ftail, s_ones);
        if (s_claims) atomicAdd(&ctrl->claims, s_claims);
    }
}

// ------------------------------------------------------------------------------------------
// Round 0 of a claim-list run (tripartite), without atomics and without edge states: the
// hinge of an edge is its lowest part at degree 1, so a degree-1 vertex of part k is the hinge
// exactly when the edge's vertices in parts below k have higher degrees -- read from the edge
// and from at most two records, all unchanged during the round.  The hinge alone appends the
// edge to layer 0, in vertex order, as (edge, part).  Same degree checks as k_round0.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kPeelBlock) void k_round0_lists(const uint64_t* __restrict__ rec, uint64_t m,
                                                             const uint32_t* __restrict__ edges, uint64_t P,
                                                             uint64_t n, uint3* __restrict__ slots,
                                                             unsigned long long* __restrict__ lcount, Ctrl* ctrl)
{
    __shared__ ClaimListAppender app;
    __shared__ unsigned long long s_deg, s_ones;
    if (threadIdx.x == 0)
        s_deg = s_ones = 0;
    app.init();
    auto out = [slots](uint64_t i, uint2 c) { slots[i] = make_uint3(c.x, c.y, 0u); };
    unsigned long long mydeg = 0, myones = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < m; base += stride) {
        const uint64_t v = base + threadIdx.x;
        bool hinge = false;
        uint32_t e = 0, k = 0;
        if (v < m) {
            const uint64_t x = rec[v];
            const uint32_t d = Rec::deg(x);
            mydeg += d;
            if (d > kMaxDegree)
                atomicOr(&ctrl->err, kErrDegree);
            if (d == 1 && Rec::edge(x) < n) {
                e = (uint32_t)Rec::edge(x);
                k = part_of((uint32_t)v, P);
                myones++;
                hinge = true;
                if (k > 0) {
                    const uint32_t* t = edges + 3 * (uint64_t)e;
                    const uint32_t u0 = t[0], u1 = k == 2 ? t[1] : 0u;
                    const uint64_t x0 = u0 < m ? rec[u0] : 0ull;
                    const uint64_t x1 = (k == 2 && u1 < m) ? rec[u1] : 0ull;
                    hinge = Rec::deg(x0) != 1 && (k == 1 || Rec::deg(x1) != 1);
                }
            }
        }
        app.push(hinge, make_uint2(e, k), false, make_uint2(e, k), &lcount[0], out);
    }
    app.flush(&lcount[0], out);
    if (mydeg) atomicAdd(&s_deg, mydeg);
    if (myones) atomicAdd(&s_ones, myones);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_deg) atomicAdd(&ctrl->degsum, s_deg);
        if (s_ones) {
            atomicAdd(&ctrl->ftail, s_ones);
            atomicAdd(&ctrl->claims, s_ones);
        }
    }
}

// Round 0 of a claim-list run whose round 0 deletes through an update list: the same hinge
// test, and the hinge then does what apply(0) would do -- it writes the edge's slot hinge
// first (vh, va, vb) to layer 0 and appends the deletes (va, e) and (vb, e) -- so layer 0 is
// read once, here.
using SlotAppender = BlockAppender<uint4, kPeelBlock, 4 * kPeelBlock>;
__global__ __launch_bounds__(kPeelBlock) void k_round0_updates(const uint64_t* __restrict__ rec, uint64_t m,
                                                               const uint32_t* __restrict__ edges, uint64_t P,
                                                               uint64_t n, uint3* __restrict__ slots,
                                                               unsigned long long* __restrict__ lcount,
                                                               uint2* __restrict__ dels,
                                                               unsigned long long* __restrict__ dcount, uint64_t dcap,
                                                               Ctrl* ctrl, const uint32_t* __restrict__ vin,
                                                               uint32_t* __restrict__ vout)
{
    __shared__ SlotAppender lapp;
    __shared__ ClaimListAppender dapp;
    __shared__ unsigned long long s_deg, s_ones;
    if (threadIdx.x == 0)
        s_deg = s_ones = 0;
    lapp.init();
    dapp.init();
    auto slot_out = [slots, vout](uint64_t i, uint4 t) {
        slots[i] = make_uint3(t.x, t.y, t.z);
        if (vout)
            vout[i] = t.w;  // a static function's value travels with the slot
    };
    auto del_out = [dels, dcap](uint64_t j, uint2 d) {
        if (j < dcap) dels[j] = d;  // past the capacity: counted, not stored; the host checks
    };
    unsigned long long mydeg = 0, myones = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < m; base += stride) {
        const uint64_t v = base + threadIdx.x;
        bool hinge = false;
        uint32_t e = 0, vh = 0, va = 0, vb = 0;
        if (v < m) {
            const uint64_t x = rec[v];
            const uint32_t d = Rec::deg(x);
            mydeg += d;
            if (d > kMaxDegree)
                atomicOr(&ctrl->err, kErrDegree);
            if (d == 1 && Rec::edge(x) < n) {
                e = (uint32_t)Rec::edge(x);
                const uint32_t k = part_of((uint32_t)v, P);
                myones++;
                const uint32_t* t = edges + 3 * (uint64_t)e;
                const uint32_t u0 = t[0], u1 = t[1], u2 = t[2];
                const uint64_t x0 = (k >= 1 && u0 < m) ? rec[u0] : 0ull;
                const uint64_t x1 = (k == 2 && u1 < m) ? rec[u1] : 0ull;
                hinge = (k == 0 || Rec::deg(x0) != 1) && (k < 2 || Rec::deg(x1) != 1);
                vh = k == 0 ? u0 : (k == 1 ? u1 : u2);
                va = k == 0 ? u1 : (k == 1 ? u2 : u0);
                vb = k == 0 ? u2 : (k == 1 ? u0 : u1);
            }
        }
        const uint32_t val = (hinge && vin) ? vin[e] : 0u;
        lapp.push(hinge, make_uint4(vh, va, vb, val), false, make_uint4(0u, 0u, 0u, 0u), &lcount[0], slot_out);
        dapp.push(hinge, make_uint2(va, e), hinge, make_uint2(vb, e), &dcount[0], del_out);
    }
    lapp.flush(&lcount[0], slot_out);
    dapp.flush(&dcount[0], del_out);
    if (mydeg) atomicAdd(&s_deg, mydeg);
    if (myones) atomicAdd(&s_ones, myones);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_deg) atomicAdd(&ctrl->degsum, s_deg);
        if (s_ones) {
            atomicAdd(&ctrl->ftail, s_ones);
            atomicAdd(&ctrl->claims, s_ones);
        }
    }
}

// Closes layer r without an apply (its slots were written by k_round0_updates).
__global__ void k_close_layer(uint64_t* __restrict__ lstart, const unsigned long long* __restrict__ lcount, Ctrl* ctrl,
                              uint32_t r)
{
    if (threadIdx.x == 0) {
        lstart[r + 1] = lstart[r] + lcount[r];
        if (lcount[r] == 0)
            atomicMin(&ctrl->nrounds, r);
    }
}

// ------------------------------------------------------------------------------------------
// Round r: delete layer r's edges and claim round r + 1.
// ------------------------------------------------------------------------------------------
template <bool kTri, ApplyMode kMode>
__global__ __launch_bounds__(kPeelBlock) void k_apply(uint64_t* __restrict__ rec, const uint32_t* __restrict__ edges,
                                                      uint32_t* __restrict__ state, uint3* __restrict__ slots,
                                                      uint64_t* __restrict__ lstart,
                                                      unsigned long long* __restrict__ lcount, uint2* __restrict__ claims,
                                                      unsigned long long* __restrict__ ccount,
                                                      unsigned long long* __restrict__ dcount, uint64_t ccap,
                                                      Ctrl* ctrl, uint32_t r, uint64_t P, bool hinge_in_slot,
                                                      const uint32_t* __restrict__ vin, uint32_t* __restrict__ vout)
{
    constexpr bool kList = kMode != ApplyMode::kAtomicClaims;
    constexpr bool kUpdates = kMode == ApplyMode::kUpdateList;
    const uint64_t lo = lstart[r];
    const uint64_t hi = lo + lcount[r];  // final: appended before this launch
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        lstart[r + 1] = hi;
        if (hi == lo)
            atomicMin(&ctrl->nrounds, r);
    }
    if (lo + (uint64_t)blockIdx.x * blockDim.x >= hi)
        return;  // whole block idle (uniform)
    using App = std::conditional_t<kList, ClaimListAppender, LayerAppender>;
    __shared__ App app;
    __shared__ unsigned long long s_push, s_claims;
    if (threadIdx.x == 0)
        s_push = s_claims = 0;
    app.init();
    unsigned long long mypush = 0, myclaims = 0;
    const uint32_t rr = (r + 1) << 2;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    // list records past the capacity are counted, not stored; the host checks the count
    unsigned long long* const tail = kUpdates ? &dcount[r] : &ccount[r + 1];
    auto to_list = [claims, ccap](uint64_t j, uint2 c) {
        if (j < ccap) claims[j] = c;
    };
    for (uint64_t base = lo + (uint64_t)blockIdx.x * blockDim.x; base < hi; base += stride) {
        uint64_t i = base + threadIdx.x;
        uint32_t c0 = 0, c1 = 0, p0 = 0, p1 = 0;
        bool f0 = false, f1 = false;
        if (i < hi) {
            const uint3 sl = slots[i];
            const uint32_t e = sl.x;
            // a resolved claim list leaves the hinge in the slot, with the positions of all the
            // edge's vertices that had degree 1 when the round began; atomic claims leave the
            // hinge in the state
            const uint32_t h = hinge_in_slot ? (sl.y & 3u) : (state[e] & 3u);
            const uint32_t ones = hinge_in_slot ? (sl.y >> 8) & 7u : 0u;
            const uint32_t* t = edges + 3 * (uint64_t)e;
            uint32_t v0 = t[0], v1 = t[1], v2 = t[2];
            uint32_t vh = h == 0 ? v0 : (h == 1 ? v1 : v2);
            uint32_t va = h == 0 ? v1 : (h == 1 ? v2 : v0);
            uint32_t vb = h == 0 ? v2 : (h == 1 ? v0 : v1);
            slots[i] = make_uint3(vh, va, vb);
            if (vin)  // a static function's value travels with the slot
                vout[i] = vin[e];
            // a vertex that had degree 1 when the round began drops to 0 with this edge and is
            // never read again: its delete can be skipped (old degree reads as 1, no record)
            const uint32_t pa = h == 2 ? 0u : h + 1, pb = h == 0 ? 2u : h - 1;
            if constexpr (kUpdates) {
                // the deletes themselves go to the update list
                f0 = !((ones >> pa) & 1u);
                f1 = !((ones >> pb) & 1u);
                c0 = va;
                p0 = e;
                c1 = vb;
                p1 = e;
            } else {
                uint64_t oa = ((ones >> pa) & 1u) ? Rec::kOne : Rec::del(rec, va, e);
                uint64_t ob = ((ones >> pb) & 1u) ? Rec::kOne : Rec::del(rec, vb, e);
                if (Rec::deg(oa) == 2) {
                    c0 = (uint32_t)(Rec::edge(oa) - e);
                    p0 = position_in<kTri>(edges, c0, va, P);
                    mypush++;
                    if constexpr (kList) {
                        f0 = true;
                    } else {
                        uint32_t old = atomicMin(&state[c0], rr | p0);
                        f0 = old == kUnclaimed;
                        myclaims += (f0 || (old >> 2) == r + 1) ? 1u : 0u;
                    }
                } else if (kList && Rec::deg(oa) == 1 && !((ones >> pa) & 1u)) {
                    // va leaves with this edge; if it reached degree 1 earlier in this round, its
                    // claim named this edge and is stale: cancel it
                    c0 = e;
                    p0 = kCancel | part_of(va, P);
                    f0 = true;
                }
                if (Rec::deg(ob) == 2) {
                    c1 = (uint32_t)(Rec::edge(ob) - e);
                    p1 = position_in<kTri>(edges, c1, vb, P);
                    mypush++;
                    if constexpr (kList) {
                        f1 = true;
                    } else {
                        uint32_t old = atomicMin(&state[c1], rr | p1);
                        f1 = old == kUnclaimed;
                        myclaims += (f1 || (old >> 2) == r + 1) ? 1u : 0u;
                    }
                } else if (kList && Rec::deg(ob) == 1 && !((ones >> pb) & 1u)) {
                    c1 = e;
                    p1 = kCancel | part_of(vb, P);
                    f1 = true;
                }
            }
            if (!f0) {  // the first requested slot holds the first appended entry
                c0 = c1;
                p0 = p1;
                f0 = f1;
                f1 = false;
            }
        }
        if constexpr (kList) {
            app.push(f0, make_uint2(c0, p0), f1, make_uint2(c1, p1), tail, to_list);
        } else {
            app.push(f0, c0, f1, c1, &lcount[r + 1], [slots, hi](uint64_t j, uint32_t x) { slots[hi + j].x = x; });
        }
    }
    if constexpr (kList) {
        app.flush(tail, to_list);
    } else {
        app.flush(&lcount[r + 1], [slots, hi](uint64_t j, uint32_t x) { slots[hi + j].x = x; });
    }
    if (mypush) atomicAdd(&s_push, mypush);
    if (myclaims) atomicAdd(&s_claims, myclaims);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_push) atomicAdd(&ctrl->ftail, s_push);
        if (s_claims) atomicAdd(&ctrl->claims, s_claims);
    }
}

// ------------------------------------------------------------------------------------------
// After a try that left a 2-core: which core edges share their vertex triple?  An edge is in
// the core exactly when its three vertices still have degree >= 2 (a peeled edge keeps its
// hinge at degree 1, the deletes skip it).  Pass 1 counts the core edges into ctrl->aux;
// pass 2 inserts each into an open-addressing table of edge ids (more slots than core edges,
// so every probe sequence ends) keyed by the triple, and a core edge whose triple is already
// there records the pair (first edge, this edge): ctrl->dups counts them, the first pcap are
// stored.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ bool core_edge(const uint64_t* rec, const uint32_t* edges, uint64_t e, uint3& t)
{
    t = make_uint3(edges[3 * e], edges[3 * e + 1], edges[3 * e + 2]);
    return Rec::deg(rec[t.x]) >= 2 && Rec::deg(rec[t.y]) >= 2 && Rec::deg(rec[t.z]) >= 2;
}

__global__ __launch_bounds__(256) void k_core_count(const uint64_t* __restrict__ rec,
                                                    const uint32_t* __restrict__ edges, uint64_t n, Ctrl* ctrl)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    unsigned long long c = 0;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        uint3 t;
        c += core_edge(rec, edges, e, t) ? 1u : 0u;
    }
    if (c)
        atomicAdd(&ctrl->aux, c);
}

__global__ __launch_bounds__(256) void k_core_pairs(const uint64_t* __restrict__ rec,
                                                    const uint32_t* __restrict__ edges, uint64_t n,
                                                    uint32_t* __restrict__ tab, uint64_t tmask,
                                                    uint2* __restrict__ pairs, uint32_t pcap, Ctrl* ctrl)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        uint3 t;
        if (!core_edge(rec, edges, e, t))
            continue;
        uint64_t h = fin(((uint64_t)t.x << 32 | t.y) ^ ((uint64_t)t.z * kGamma)) & tmask;
        for (;;) {
            const uint32_t old = atomicCAS(&tab[h], kUnclaimed, (uint32_t)e);
            if (old == kUnclaimed)
                break;
            if (edges[3 * (uint64_t)old] == t.x && edges[3 * (uint64_t)old + 1] == t.y &&
                edges[3 * (uint64_t)old + 2] == t.z) {
                const unsigned long long j = atomicAdd(&ctrl->dups, 1ull);
                if (j < pcap)
                    pairs[j] = make_uint2(old, (uint32_t)e);
                break;
            }
            h = (h + 1) & tmask;
        }
    }
}

hipError_t launch_core_count(const uint64_t* rec, const uint32_t* edges, uint64_t n, Ctrl* ctrl, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_core_count<<<(unsigned)std::min<uint64_t>((n + 255) / 256, 8192), 256, 0, s>>>(rec, edges, n, ctrl);
    return hipGetLastError();
}

hipError_t launch_core_pairs(const uint64_t* rec, const uint32_t* edges, uint64_t n, uint32_t* tab, uint64_t tsize,
                             uint2* pairs, uint32_t pcap, Ctrl* ctrl, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_core_pairs<<<(unsigned)std::min<uint64_t>((n + 255) / 256, 8192), 256, 0, s>>>(rec, edges, n, tab, tsize - 1,
                                                                                      pairs, pcap, ctrl);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Per-edge outputs of mphx_peel from the edge states.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_peel_finalize(const uint32_t* __restrict__ state, uint64_t n,
                                                       uint32_t* __restrict__ round, uint8_t* __restrict__ core_mask,
                                                       uint8_t* __restrict__ hinge)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        uint32_t s = state[e];
        bool core = s == kUnclaimed;
        round[e] = core ? kRoundCore : (s >> 2);
        core_mask[e] = core ? 1 : 0;
        if (hinge)
            hinge[e] = core ? 0xFF : (uint8_t)(s & 3u);
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

hipError_t launch_edges_build(const uint32_t* edges, uint64_t n, uint64_t m, uint64_t* rec, Ctrl* ctrl, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_edges_build<<<grid_for(n, 8192), 256, 0, s>>>(edges, n, m, rec, ctrl);
    return hipGetLastError();
}

hipError_t launch_round0(const PeelState& st, hipStream_t s)
{
    if (st.m == 0) return hipSuccess;
    unsigned g = grid_for(st.m, 8192);
    if (st.lists) {
        if (!st.tripartite) return hipErrorInvalidValue;
        if (st.round0_updates)
            k_round0_updates<<<g, kPeelBlock, 0, s>>>(st.rec, st.m, st.edges, st.P, st.n, st.slots, st.lcount,
                                                      st.claims, st.dcount, st.lcap, st.ctrl, st.vin, st.vout);
        else
            k_round0_lists<<<g, kPeelBlock, 0, s>>>(st.rec, st.m, st.edges, st.P, st.n, st.slots, st.lcount, st.ctrl);
    } else {
        // at least eight vertices per thread and at most 1024 blocks: every block ends with
        // four atomics on the same counters, which serialise (one thread per vertex made them
        // most of this kernel's time at 10^6 keys)
        g = grid_for((st.m + 7) / 8, 1024);
        if (st.tripartite)
            k_round0<true><<<g, kPeelBlock, 0, s>>>(st.rec, st.m, st.edges, st.P, st.n, st.state, st.slots,
                                                    st.lcount, st.ctrl);
        else
            k_round0<false><<<g, kPeelBlock, 0, s>>>(st.rec, st.m, st.edges, st.P, st.n, st.state, st.slots,
                                                     st.lcount, st.ctrl);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// r-hypergraphs, 2 <= r <= 8 (generic edge lists of r vertices each).  The same records,
// rounds and atomic claims as the three-vertex generic peel; an edge state is
// (round << 3) | hinge position, three bits holding positions below 8.
// ------------------------------------------------------------------------------------------
template <int kR>
__device__ __forceinline__ uint32_t position_r(const uint32_t* edges, uint32_t e, uint32_t v)
{
    const uint32_t* t = edges + (uint64_t)kR * e;
    uint32_t k = 0;
#pragma unroll
    for (uint32_t q = 1; q < kR; q++)
        if (t[q] == v)
            k = q;
    return k;
}

template <int kR>
__global__ __launch_bounds__(256) void k_edges_build_r(const uint32_t* __restrict__ edges, uint64_t n, uint64_t m,
                                                       uint64_t* __restrict__ rec, Ctrl* ctrl)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        uint32_t t[kR];
        bool bad = false;
#pragma unroll
        for (uint32_t q = 0; q < kR; q++) {
            t[q] = edges[(uint64_t)kR * e + q];
            bad = bad || t[q] >= m;
        }
#pragma unroll
        for (uint32_t a = 0; a < kR; a++)
#pragma unroll
            for (uint32_t b = a + 1; b < kR; b++)
                bad = bad || t[a] == t[b];
        if (bad) {
            atomicOr(&ctrl->err, kErrBadEdge);
            continue;
        }
#pragma unroll
        for (uint32_t q = 0; q < kR; q++)
            Rec::add(rec, t[q], (uint32_t)e);
    }
}

// Round 0 as k_round0: degree-1 vertices claim their edges, the lowest position wins.
template <int kR>
__global__ __launch_bounds__(kPeelBlock) void k_round0_r(const uint64_t* __restrict__ rec, uint64_t m,
                                                         const uint32_t* __restrict__ edges, uint64_t n,
                                                         uint32_t* __restrict__ state, uint3* __restrict__ slots,
                                                         unsigned long long* __restrict__ lcount, Ctrl* ctrl)
{
    __shared__ LayerAppender app;
    __shared__ unsigned long long s_deg, s_ones;
    if (threadIdx.x == 0)
        s_deg = s_ones = 0;
    app.init();
    auto out = [slots](uint64_t i, uint32_t e) { slots[i].x = e; };
    unsigned long long mydeg = 0, myones = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < m; base += stride) {
        const uint64_t v = base + threadIdx.x;
        bool first = false;
        uint32_t e = 0;
        if (v < m) {
            const uint64_t x = rec[v];
            const uint32_t d = Rec::deg(x);
            mydeg += d;
            if (d > kMaxDegree)
                atomicOr(&ctrl->err, kErrDegree);
            if (d == 1 && Rec::edge(x) < n) {
                e = Rec::edge(x);
                first = atomicMin(&state[e], position_r<kR>(edges, e, (uint32_t)v)) == kUnclaimed;
                myones++;
            }
        }
        app.push(first, e, false, 0u, &lcount[0], out);
    }
    app.flush(&lcount[0], out);
    if (mydeg) atomicAdd(&s_deg, mydeg);
    if (myones) atomicAdd(&s_ones, myones);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_deg) atomicAdd(&ctrl->degsum, s_deg);
        if (s_ones) {
            atomicAdd(&ctrl->ftail, s_ones);
            atomicAdd(&ctrl->claims, s_ones);
        }
    }
}

// Round r: every layer edge is deleted at its r - 1 vertices other than the hinge; a vertex
// taken to degree 1 claims its last edge for round r + 1 (lowest position wins, atomicMin).
template <int kR>
__global__ __launch_bounds__(kPeelBlock) void k_apply_r(uint64_t* __restrict__ rec, const uint32_t* __restrict__ edges,
                                                        uint32_t* __restrict__ state, uint3* __restrict__ slots,
                                                        uint64_t* __restrict__ lstart,
                                                        unsigned long long* __restrict__ lcount, Ctrl* ctrl, uint32_t r)
{
    const uint64_t lo = lstart[r];
    const uint64_t hi = lo + lcount[r];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        lstart[r + 1] = hi;
        if (hi == lo)
            atomicMin(&ctrl->nrounds, r);
    }
    if (lo + (uint64_t)blockIdx.x * blockDim.x >= hi)
        return;  // whole block idle (uniform)
    __shared__ LayerAppender app;
    __shared__ unsigned long long s_push, s_claims;
    if (threadIdx.x == 0)
        s_push = s_claims = 0;
    app.init();
    auto out = [slots, hi](uint64_t j, uint32_t x) { slots[hi + j].x = x; };
    unsigned long long mypush = 0, myclaims = 0;
    const uint32_t rr = (r + 1) << 3;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = lo + (uint64_t)blockIdx.x * blockDim.x; base < hi; base += stride) {
        const uint64_t i = base + threadIdx.x;
        uint32_t e = 0, h = 0;
        if (i < hi) {
            e = slots[i].x;
            h = state[e] & 7u;
        }
#pragma unroll
        for (uint32_t q = 0; q < kR; q++) {
            bool f = false;
            uint32_t c = 0;
            if (i < hi && q != h) {
                const uint32_t v = edges[(uint64_t)kR * e + q];
                const uint64_t old = Rec::del(rec, v, e);
                if (Rec::deg(old) == 2) {
                    c = (uint32_t)(Rec::edge(old) - e);
                    const uint32_t o = atomicMin(&state[c], rr | position_r<kR>(edges, c, v));
                    f = o == kUnclaimed;
                    mypush++;
                    myclaims += (f || (o >> 3) == r + 1) ? 1u : 0u;
                }
            }
            app.push(f, c, false, 0u, &lcount[r + 1], out);
        }
    }
    app.flush(&lcount[r + 1], out);
    if (mypush) atomicAdd(&s_push, mypush);
    if (myclaims) atomicAdd(&s_claims, myclaims);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_push) atomicAdd(&ctrl->ftail, s_push);
        if (s_claims) atomicAdd(&ctrl->claims, s_claims);
    }
}

__global__ __launch_bounds__(256) void k_peel_finalize_r(const uint32_t* __restrict__ state, uint64_t n,
                                                         uint32_t* __restrict__ round, uint8_t* __restrict__ core_mask,
                                                         uint8_t* __restrict__ hinge)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        const uint32_t s = state[e];
        const bool core = s == kUnclaimed;
        round[e] = core ? kRoundCore : (s >> 3);
        core_mask[e] = core ? 1 : 0;
        if (hinge)
            hinge[e] = core ? 0xFF : (uint8_t)(s & 7u);
    }
}

#define MPHX_FOR_R(R, CALL) \
    switch (R) {            \
    case 2: CALL(2); break; \
    case 3: CALL(3); break; \
    case 4: CALL(4); break; \
    case 5: CALL(5); break; \
    case 6: CALL(6); break; \
    case 7: CALL(7); break; \
    case 8: CALL(8); break; \
    default: return hipErrorInvalidValue; \
    }

hipError_t launch_edges_build_r(const uint32_t* edges, uint64_t n, uint64_t m, uint32_t r, uint64_t* rec, Ctrl* ctrl,
                                hipStream_t s)
{
    if (n == 0) return hipSuccess;
#define MPHX_CALL(K) k_edges_build_r<K><<<grid_for(n, 8192), 256, 0, s>>>(edges, n, m, rec, ctrl)
    MPHX_FOR_R(r, MPHX_CALL)
#undef MPHX_CALL
    return hipGetLastError();
}

hipError_t launch_round0_r(const PeelState& st, uint32_t r, hipStream_t s)
{
    if (st.m == 0) return hipSuccess;
    const unsigned g = grid_for(st.m, 8192);
#define MPHX_CALL(K) \
    k_round0_r<K><<<g, kPeelBlock, 0, s>>>(st.rec, st.m, st.edges, st.n, st.state, st.slots, st.lcount, st.ctrl)
    MPHX_FOR_R(r, MPHX_CALL)
#undef MPHX_CALL
    return hipGetLastError();
}

hipError_t launch_apply_r(const PeelState& st, uint32_t r, uint32_t round, hipStream_t s)
{
    const unsigned g = grid_for(st.n, st.grid_cap);
#define MPHX_CALL(K) \
    k_apply_r<K><<<g, kPeelBlock, 0, s>>>(st.rec, st.edges, st.state, st.slots, st.lstart, st.lcount, st.ctrl, round)
    MPHX_FOR_R(r, MPHX_CALL)
#undef MPHX_CALL
    return hipGetLastError();
}

hipError_t launch_peel_finalize_r(const uint32_t* state, uint64_t n, uint32_t* round, uint8_t* core_mask,
                                  uint8_t* hinge, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_peel_finalize_r<<<grid_for(n, 8192), 256, 0, s>>>(state, n, round, core_mask, hinge);
    return hipGetLastError();
}
#undef MPHX_FOR_R

hipError_t launch_apply(const PeelState& st, uint32_t r, bool hinge_in_slot, ApplyMode mode, hipStream_t s)
{
    unsigned g = grid_for(st.n, st.grid_cap);
    if (mode != ApplyMode::kAtomicClaims && !st.tripartite) return hipErrorInvalidValue;
#define MPHX_APPLY(TRI, MODE, HINGE)                                                                        \
    k_apply<TRI, MODE><<<g, kPeelBlock, 0, s>>>(st.rec, st.edges, st.state, st.slots, st.lstart, st.lcount, \
                                                st.claims, st.ccount, st.dcount, st.lcap, st.ctrl, r, st.P, HINGE,   \
                                                st.vin, st.vout)
    switch (mode) {
    case ApplyMode::kClaimList: MPHX_APPLY(true, ApplyMode::kClaimList, hinge_in_slot); break;
    case ApplyMode::kUpdateList: MPHX_APPLY(true, ApplyMode::kUpdateList, hinge_in_slot); break;
    default:
        if (st.tripartite)
            MPHX_APPLY(true, ApplyMode::kAtomicClaims, hinge_in_slot);
        else
            MPHX_APPLY(false, ApplyMode::kAtomicClaims, false);
    }
#undef MPHX_APPLY
    return hipGetLastError();
}

hipError_t launch_close_layer(const PeelState& st, uint32_t r, hipStream_t s)
{
    k_close_layer<<<1, 64, 0, s>>>(st.lstart, st.lcount, st.ctrl, r);
    return hipGetLastError();
}

hipError_t launch_peel_finalize(const uint32_t* state, uint64_t n, uint32_t* round, uint8_t* core_mask, uint8_t* hinge,
                                hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_peel_finalize<<<grid_for(n, 8192), 256, 0, s>>>(state, n, round, core_mask, hinge);
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
