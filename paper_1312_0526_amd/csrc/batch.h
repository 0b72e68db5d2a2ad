// Internal declarations of the batched build (batch.hip; not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "common.h"

namespace mphx {

// One bucket of a batched launch: its keys (u64, or string bytes + offsets), its seed and
// where its outputs go.
struct BucketDesc {
    const uint64_t* keys;    // u64 keys, or nullptr for string keys
    const uint8_t* bytes;    // string bytes (4-byte aligned)
    const uint64_t* offs;    // n + 1 string offsets
    uint64_t n;
    uint64_t seed;
    uint64_t* codes;         // ceil(m/32) words
    uint64_t* rank;          // ceil(m/512) samples
    BucketResult* result;
};
static_assert(sizeof(BucketDesc) == 64, "BucketDesc is 64 bytes");

struct BatchArgs {
    const BucketDesc* descs;
    const uint32_t* order;   // processing order (nullable: descriptor order)
    uint32_t B;
    uint32_t gnum, gden, max_tries;
    uint8_t* slots;
    uint64_t slot_bytes;
    uint64_t max_n;          // largest bucket a slot can hold
    unsigned int* next;      // queue cursor
    uint32_t lds_path;       // 1: buckets that fit run in LDS
    uint32_t sort_div;       // > 0: a layer deletes through a sorted list when 2 * layer * sort_div >= m
    uint32_t pairs;          // 1: every bucket's keys are 128-bit digest pairs (2 u64 words per key:
                             // the edge under seed t is that of the digest (x ^ t, y ^ t))
    uint32_t claim_lists;    // 1: sparse rounds of buckets given by key words resolve their claims
                             // through a list grouped by edge tile, in LDS, instead of atomicMin
    uint32_t clock;          // 1: launch the kernel that adds its per-phase workgroup time and
                             // work counts to the device's batch clock
};

// batched builds (batch.hip)
uint64_t batch_slot_bytes(uint64_t max_n, uint32_t gnum, uint32_t gden);
// words_per_key: 1 for u64 keys, 2 for digest pairs (BatchArgs::pairs)
hipError_t launch_batch_descs(BucketDesc* descs, const uint64_t* keys, const uint64_t* off, uint32_t B, uint64_t seed,
                              const uint64_t* code_off, const uint64_t* rank_off, uint64_t* codes, uint64_t* rank,
                              BucketResult* results, hipStream_t s, uint32_t words_per_key = 1);
hipError_t launch_batch(const BatchArgs& a, unsigned block, unsigned grid, bool wg_scope, hipStream_t s);
// The batch clock of the current device: entry 0 is its tick rate in Hz, then per-phase ticks
// summed over workgroups and work counts (batch_clock_name(i)); reset zeroes them afterwards.
constexpr int kBatchClockEntries = 19;
hipError_t batch_clock_read(uint64_t* out, int max_entries, bool reset);
const char* batch_clock_name(int i);

}  // namespace mphx
