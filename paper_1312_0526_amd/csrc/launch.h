// Internal host-side launchers of the gfx950 kernels (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "common.h"

namespace mphx {

// Everything one peeling run needs on the device.
struct PeelState {
    const uint32_t* edges;  // n x 3
    uint64_t n, m, P;       // P = part size when tripartite
    bool tripartite;
    unsigned grid_cap;      // max blocks of the grid-stride round kernels
    uint64_t* rec;          // m packed records
    uint3* slots;           // n layer slots of all rounds back to back: edge id, then vertices
    uint32_t* state;        // n edge states: unclaimed or (round << 2) | hinge
    uint64_t* lstart;       // rcap + 2 layer starts
    unsigned long long* lcount;  // rcap + 2 layer sizes (append cursors), zeroed per run
    Ctrl* ctrl;
    uint64_t rcap;          // rounds the start arrays can hold
    // Claim lists (tripartite only): instead of claiming an edge for the next round with a
    // device atomic, a vertex reaching degree 1 appends (edge, position); the list is then
    // partitioned by edge and resolved in LDS into the next layer.
    bool lists;
    uint2* claims;          // m (edge, position) claims of one round
    uint64_t lcap;          // records a round may keep in the list (<= m); more make the try
                            // fall back to atomic claims
    uint2* claims_tmp;      // m, the partition's other buffer
    unsigned long long* ccount;  // rcap + 2 claim counts: ccount[r] = claims that form layer r
    // Sorted update lists (dense rounds of a claim-list run): apply(r) appends one (vertex,
    // edge) delete per non-hinge vertex to st.claims instead of deleting with atomics; the
    // list is partitioned by vertex and applied bucket by bucket in LDS, which also yields
    // the next round's claims (into st.claims_tmp).
    unsigned long long* dcount;  // rcap + 2 update counts: dcount[r] = deletes of round r
    // round 0 writes layer 0's slots hinge first and its update list itself (claim lists only)
    bool round0_updates;
    // static functions: vin[e] = key e's value (nullable); whoever writes a layer slot hinge
    // first also writes vout[slot] = vin[edge], so the values reach the assignment in layer order
    const uint32_t* vin;
    uint32_t* vout;
    void* aux;              // partition histograms and scan scratch (part_aux_bytes)
};

// utilities (scan.hip)
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint64_t count, uint32_t value, hipStream_t s);
hipError_t launch_ctrl_init(Ctrl* ctrl, uint64_t* lstart, hipStream_t s);
size_t scan_scratch_bytes(uint64_t count);
// exclusive scans; in and out may alias
hipError_t launch_scan_u32(const uint32_t* in, uint64_t count, uint32_t* out, void* scratch, size_t scratch_bytes,
                           hipStream_t s);
// out has count_out entries; input entries past count_in read as 0
hipError_t launch_scan_u32_to_u64(const uint32_t* in, uint64_t count_in, uint64_t* out, uint64_t count_out,
                                  void* scratch, size_t scratch_bytes, hipStream_t s);

// partitioned record build of a tripartite edge list (part.hip).  First-pass tiles are
// kPartTile consecutive edges; the first-pass digit of part k's vertex v is
// (v - kP) >> kPartGrpShift.  The key-hashing kernels can count those digits per tile while
// they write the edges (PartHist1), which saves the build its own pass over the edges.
constexpr uint32_t kPartTile = 8192;
constexpr uint32_t kPartGrpShift = 22;
constexpr uint32_t kPartMaxGroups = 512;

struct PartHist1 {
    uint32_t* hist;  // [3][NH][nt1] counts, or nullptr
    uint32_t NH;
    uint64_t nt1;
};

// Auxiliary buffer of the partition passes: sized for the record build of n edges with part
// size P and, with claim lists, for resolving up to m = 3P claims.
size_t part_aux_bytes(uint64_t n, uint64_t P, bool lists);
PartHist1 part_hist1(void* aux, uint64_t n, uint64_t P);
// the hashing kernel has filled the first-pass histograms (part_hist1)
// extra1/extra2 (n pairs each, nullable): with both, one first pass serves all three parts
hipError_t launch_part_build(const uint32_t* edges, uint64_t n, uint64_t P, uint64_t* rec, uint2* pairs1,
                             uint2* pairs2, uint2* extra1, uint2* extra2, void* aux, hipStream_t s);
// Layer r from the count claims of round r - 1 (ccount[r] of them, known to the host), held in
// st.claims, or in st.claims_tmp when round r - 1 used update lists (in_tmp): the claims are
// partitioned by edge, cancelled ones dropped, each edge's lowest claimed position kept as its
// hinge; each winner fills a slot of layer r, (edge, hinge | positions at degree 1 << 8),
// through lcount[r].
hipError_t launch_claims_resolve(const PeelState& st, uint32_t r, uint64_t count, bool in_tmp, hipStream_t s);
// Round r's count deletes (vertex, edge) in st.claims, appended by apply(r) in update mode:
// partitioned by vertex into buckets of 2^14 records, each bucket's deletes summed in LDS and
// subtracted from its records once; a record left at degree 1 claims its last edge for round
// r + 1 into st.claims_tmp through ccount[r + 1].
hipError_t launch_update_apply(const PeelState& st, uint32_t r, uint64_t count, hipStream_t s);

// hashing and key generation (keys.hip); rec == nullptr hashes only
// h1.hist != nullptr (with rec == nullptr): also count the first-pass partition digits
hipError_t launch_hash_u64(const uint64_t* keys, uint64_t n, uint64_t seed, uint64_t P, uint32_t* edges,
                           uint64_t* rec, PartHist1 h1, hipStream_t s);
hipError_t launch_hash_str(const uint8_t* bytes, const uint64_t* offs, uint64_t n, uint64_t seed, uint64_t P,
                           uint32_t* edges, uint64_t* rec, PartHist1 h1, hipStream_t s);
hipError_t launch_gen_u64(uint64_t* keys, uint64_t n, uint64_t gen_seed, uint64_t start, hipStream_t s);
hipError_t launch_gen_buckets_u64(uint64_t* keys, const uint64_t* off, uint32_t B, hipStream_t s);
hipError_t launch_gen_str_lengths(uint32_t* lens, uint64_t n, uint64_t gen_seed, uint64_t start,
                                  const uint16_t* qtable, hipStream_t s);
hipError_t launch_gen_str_bytes(uint8_t* bytes, const uint64_t* offs, uint64_t n, uint64_t gen_seed, uint64_t start,
                                hipStream_t s);

// peeling (peel.hip)
hipError_t launch_edges_build(const uint32_t* edges, uint64_t n, uint64_t m, uint64_t* rec, Ctrl* ctrl,
                              hipStream_t s);
// Round 0: layer 0 from the degree-1 vertices -- atomicMin claims on the edge states, or with
// st.lists the hinge test on the records, which leaves (edge, hinge) in the slots -- or, with
// st.round0_updates, the hinge-first slots and round 0's update list (count in dcount[0]);
// layer 0 is then closed by launch_close_layer instead of an apply.
hipError_t launch_round0(const PeelState& st, hipStream_t s);
hipError_t launch_close_layer(const PeelState& st, uint32_t r, hipStream_t s);
// How apply(r) deletes layer r and finds round r + 1: atomic deletes with atomicMin claims on
// the edge states; atomic deletes with claims appended to st.claims (tripartite only); or
// deletes appended to st.claims as an update list (tripartite only), applied afterwards by
// launch_update_apply.
enum class ApplyMode { kAtomicClaims, kClaimList, kUpdateList };
// hinge_in_slot: layer r came from a resolved claim list
hipError_t launch_apply(const PeelState& st, uint32_t r, bool hinge_in_slot, ApplyMode mode, hipStream_t s);
hipError_t launch_peel_finalize(const uint32_t* state, uint64_t n, uint32_t* round, uint8_t* core_mask,
                                uint8_t* hinge, hipStream_t s);
uint64_t sort_tiles(uint64_t n);
hipError_t launch_order_sort(const uint32_t* round, uint64_t n, uint32_t nrounds, uint32_t* order,
                             uint32_t* scratch_ids, uint32_t* tilehist, void* scan_scratch, size_t scan_bytes,
                             hipStream_t s);

// assignment, ranking, lookup (solve.hip)
// 2-core edges of a failed try: their count (ctrl->aux), then pairs with equal vertex triples
// (tab: tsize entries, a power of two above the count, filled with kUnclaimed)
hipError_t launch_core_count(const uint64_t* rec, const uint32_t* edges, uint64_t n, Ctrl* ctrl, hipStream_t s);
hipError_t launch_core_pairs(const uint64_t* rec, const uint32_t* edges, uint64_t n, uint32_t* tab, uint64_t tsize,
                             uint2* pairs, uint32_t pcap, Ctrl* ctrl, hipStream_t s);
hipError_t launch_assign_round(const uint3* slots, const uint64_t* lstart, uint32_t r, uint64_t n_bound, uint64_t P,
                               uint8_t* code8, unsigned grid_cap, hipStream_t s);
// HEM split (keys.hip, part.hip): signature records, their partition into 2^k buckets in place
// (tmp: n more records; 9 <= k <= 18; larger k through launch_hem_refine) with
// bucket_off[0..2^k] written on the device, and lookups.  A u64 key's record is uint2 (high,
// low half of its signature: a u64 read gives the bucket key); a string key's is uint4 (high
// and low half of a, then b: two u64 reads give the bucket's digest pair (swap(a), b)).
hipError_t launch_hem_sig_u64(const uint64_t* keys, uint64_t n, uint64_t seed, uint2* rec, hipStream_t s);
hipError_t launch_hem_sig_str(const uint8_t* bytes, const uint64_t* offs, uint64_t n, uint64_t seed, uint4* rec,
                              hipStream_t s);
size_t hem_aux_bytes(uint64_t n, uint32_t k);
hipError_t launch_hem_partition(uint2* rec, uint64_t n, uint32_t k, uint2* tmp, uint64_t* bucket_off, void* aux,
                                hipStream_t s);
hipError_t launch_hem_partition(uint4* rec, uint64_t n, uint32_t k, uint4* tmp, uint64_t* bucket_off, void* aux,
                                hipStream_t s);
hipError_t launch_hem_lookup_u64(const HemTables& t, uint64_t seed, const uint64_t* keys, uint64_t n, uint64_t* out,
                                 hipStream_t s);
hipError_t launch_hem_lookup_str(const HemTables& t, uint64_t seed, const uint8_t* bytes, const uint64_t* offs,
                                 uint64_t n, uint64_t* out, hipStream_t s);
// static functions (solve.hip; string lookups in keys.hip)
hipError_t launch_sf_lookup_str_words(const uint64_t* words, uint64_t sigma, uint32_t b, uint64_t P, uint64_t seed,
                                      const uint8_t* bytes, const uint64_t* offs, uint64_t n, uint64_t* out,
                                      hipStream_t s);
// u holds m elements of sf_elem_bytes(b) bytes (u8 up to 8 bits, u16 up to 16, else u32)
uint32_t sf_elem_bytes(uint32_t b);
hipError_t launch_sf_assign_round(const uint3* slots, const uint32_t* vals, uint64_t count, uint64_t sigma,
                                  uint32_t b, void* u, hipStream_t s);
hipError_t launch_sf_pack(const void* u, uint64_t m, uint32_t b, uint64_t* words, hipStream_t s);
hipError_t launch_sf_lookup_u64(const uint64_t* words, uint64_t sigma, uint32_t b, uint64_t P, uint64_t seed,
                                const uint64_t* keys, uint64_t n, uint64_t* out, hipStream_t s);
hipError_t launch_sfr_marks(const void* u, uint64_t m, uint32_t b, uint64_t* marks, uint32_t* bcount, hipStream_t s);
hipError_t launch_sfr_compact(const void* u, uint64_t m, uint32_t b, const uint64_t* rank, uint64_t* vals,
                              uint64_t cap_words, hipStream_t s);
hipError_t launch_sfr_lookup_u64(const uint64_t* marks, const uint64_t* rank, const uint64_t* vals, uint64_t sigma,
                                 uint32_t b, uint64_t P, uint64_t seed, const uint64_t* keys, uint64_t n,
                                 uint64_t* out, hipStream_t s);
hipError_t launch_sfr_lookup_str_words(const uint64_t* marks, const uint64_t* rank, const uint64_t* vals,
                                       uint64_t sigma, uint32_t b, uint64_t P, uint64_t seed, const uint8_t* bytes,
                                       const uint64_t* offs, uint64_t n, uint64_t* out, hipStream_t s);
hipError_t launch_sf_check(const uint32_t* vals, uint64_t n, uint64_t sigma, Ctrl* ctrl, hipStream_t s);
hipError_t launch_pack_count(const uint8_t* code8, uint64_t m, uint64_t* codes, uint32_t* bcount, hipStream_t s);
hipError_t launch_lookup_u64(const uint64_t* codes, const uint64_t* rank, uint64_t P, uint64_t seed,
                             const uint64_t* keys, uint64_t n, uint64_t* out, hipStream_t s);
// string keys: the word-parallel digest of the hashing kernel, then the evaluation (keys.hip)
hipError_t launch_lookup_str_words(const uint64_t* codes, const uint64_t* rank, uint64_t P, uint64_t seed,
                                   const uint8_t* bytes, const uint64_t* offs, uint64_t n, uint64_t* out,
                                   hipStream_t s);
hipError_t launch_bijection(const uint64_t* vals, uint64_t n, uint32_t* bitmap, Ctrl* ctrl, hipStream_t s);

// r-hypergraph peel, 2 <= r <= 8 (peel.hip): edge lists of r vertices each; edge states are
// (round << 3) | hinge position; hipErrorInvalidValue for r outside [2, 8].
hipError_t launch_edges_build_r(const uint32_t* edges, uint64_t n, uint64_t m, uint32_t r, uint64_t* rec, Ctrl* ctrl,
                                hipStream_t s);
hipError_t launch_round0_r(const PeelState& st, uint32_t r, hipStream_t s);
hipError_t launch_apply_r(const PeelState& st, uint32_t r, uint32_t round, hipStream_t s);
hipError_t launch_peel_finalize_r(const uint32_t* state, uint64_t n, uint32_t* round, uint8_t* core_mask,
                                  uint8_t* hinge, hipStream_t s);

// Out-of-core HEM: a chunk's signature records grouped by their top k - 8 bits into out (aux:
// hem_aux_bytes(cn, k)), its NH + 1 group starts copied to host memory; runs of records
// gathered into a batch buffer; string offsets shifted down by base.
struct HemRun {
    uint64_t src, dst;
    uint32_t len, pad;
};
hipError_t launch_hem_group_chunk(const uint2* csig, uint64_t cn, uint32_t k, uint2* out, void* aux,
                                  uint32_t* host_gstart, hipStream_t s);
hipError_t launch_hem_group_chunk(const uint4* csig, uint64_t cn, uint32_t k, uint4* out, void* aux,
                                  uint32_t* host_gstart, hipStream_t s);
hipError_t launch_hem_gather(const uint2* src, const HemRun* runs, uint32_t nruns, uint2* dst, hipStream_t s);
hipError_t launch_hem_gather(const uint4* src, const HemRun* runs, uint32_t nruns, uint4* dst, hipStream_t s);
// More than 2^18 buckets: records partitioned into 2^kc coarse buckets (coarse_off, 2^kc + 1)
// split stably by the next k - kc <= 2 bits into out, with the 2^k + 1 fine offsets.
hipError_t launch_hem_refine(const uint2* in, const uint64_t* coarse_off, uint32_t kc, uint32_t k, uint2* out,
                             uint64_t* fine_off, hipStream_t s);
hipError_t launch_hem_refine(const uint4* in, const uint64_t* coarse_off, uint32_t kc, uint32_t k, uint4* out,
                             uint64_t* fine_off, hipStream_t s);
hipError_t launch_offs_rebase(uint64_t* offs, uint64_t count, uint64_t base, hipStream_t s);

// Streamed build (stream.hip): records as degree bytes (deg, (m + 3) & ~3 bytes, zeroed) and XOR
// packs of the two other endpoints' part-local ids (X, m words, zeroed); layers as slots
// (vh, va, vb) of part-local ids in runs by hinge part.
hipError_t launch_st_build(const uint64_t* keys, uint64_t cn, uint64_t seed, uint64_t P, uint8_t* deg, uint64_t* X,
                           Ctrl* ctrl, hipStream_t s);
hipError_t launch_st_claim(const uint8_t* deg, const uint64_t* X, uint64_t P, uint32_t k, uint3* slots, uint64_t cap,
                           unsigned long long* cursor, Ctrl* ctrl, hipStream_t s);
hipError_t launch_st_apply(const uint3* slots, uint64_t lo, uint64_t b1, uint64_t b2, uint64_t hi, uint64_t P,
                           uint8_t* deg, uint64_t* X, hipStream_t s);
hipError_t launch_st_assign(const uint3* slots, uint64_t lo, uint64_t b1, uint64_t b2, uint64_t hi, uint64_t P,
                            uint8_t* code8, hipStream_t s);
// f(key) for keys[0, cn) into out (nullable); with bitmap (n_total bits), each value is marked
// and ctrl->aux counts values >= n_total or marked twice
hipError_t launch_st_lookup(const uint64_t* codes, const uint64_t* rank, uint64_t P, uint64_t seed,
                            const uint64_t* keys, uint64_t cn, uint64_t* out, uint32_t* bitmap, uint64_t n_total,
                            Ctrl* ctrl, hipStream_t s);

}  // namespace mphx
