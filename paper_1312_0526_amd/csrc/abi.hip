// Host orchestration of the C ABI declared in include/mphx.h.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <memory>
#include <mutex>
#include <thread>
#include <string>
#include <vector>

#include "batch.h"
#include "launch.h"
#include "mphx.h"

using namespace mphx;

namespace {

thread_local std::string g_err;

struct Options {
    std::atomic<int> grid{0};          // 0 = automatic
    std::atomic<int> round_batch{64};  // rounds before the first termination check; later ones every
                                       // kLaterBatch (a peel at gamma 1.23 takes 57-64 rounds from
                                       // 10^5 keys up, so one batch usually covers it)
    std::atomic<int> timing{0};        // 1 = HIP events around every launch, per phase
    std::atomic<int> part_build{21};   // partitioned record build from n >= 2^part_build keys on,
                                       // device atomics below (0 = never): below ~2^21 keys the
                                       // records stay cache-resident and the build's one launch
                                       // beats the partition's dozen
    std::atomic<int> claim_lists{26};  // claim lists from n >= 2^claim_lists keys on (0 = never);
                                       // below 2^26 keys the per-round partition and resolve cost more
                                       // than the atomic claims they replace
    std::atomic<int> update_lists{16}; // claim-list rounds with 2 * layer >= m * update_lists / 100
                                       // delete through a sorted update list (0 = never)
    std::atomic<int> hem_block{1024};  // batched-kernel workgroup size for the HEM split's buckets
    std::atomic<int> hem_grid{0};      // its persistent grid (0 = one workgroup per compute unit)
    std::atomic<int64_t> list_cap{0};  // records a claim-list round may hold (0 = m, the buffers' size)
    std::atomic<int64_t> list_fallbacks{0};  // tries redone with atomic claims after a list overflowed
    std::atomic<int> batch_lds{1};     // 1 = batched buckets that fit run entirely in LDS
    std::atomic<int> batch_sort_deletes{4};  // sorted deletes for layers with 2 * layer * this >= m
                                             // (0: off; 4 takes layer 0 only, the one layer where
                                             // they beat the claim lists' device atomics)
    std::atomic<int> batch_claim_lists{1};   // sparse rounds of key-word buckets claim through lists
    std::atomic<int> batch_clock{0};   // 1 = batched launches run the kernel that clocks its phases
};

Options g_opt;

bool use_claim_lists(uint64_t n)
{
    const int b = g_opt.claim_lists.load();
    return b > 0 && n >= (1ull << b);
}

// ---- per-phase timing (HIP events on the caller's stream) ---------------------------------
enum Phase {
    PH_HASH, PH_BUILD, PH_FRONTIER, PH_APPLY, PH_RESOLVE, PH_ASSIGN, PH_RANK, PH_ORDER, PH_OTHER, PH_UPDATE, PH_COUNT
};
const char* const kPhaseNames[PH_COUNT] = {"hash",   "build", "frontier", "apply", "resolve",
                                           "assign", "rank",  "order",    "other", "update"};

struct Timers {
    struct Span { int phase; hipEvent_t a, b; };
    std::vector<hipEvent_t> pool;
    std::vector<Span> pending;
    double ms[PH_COUNT] = {};
    uint64_t launches[PH_COUNT] = {};
    hipEvent_t get()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    // Fold completed spans into the totals (the stream has been synchronised).
    void harvest()
    {
        for (auto& sp : pending) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, sp.a, sp.b) == hipSuccess) {
                ms[sp.phase] += t;
                launches[sp.phase] += 1;
            }
            pool.push_back(sp.a);
            pool.push_back(sp.b);
        }
        pending.clear();
    }
};
thread_local Timers g_timers;

struct Timed {
    int phase;
    hipStream_t s;
    hipEvent_t a = nullptr;
    Timed(int ph, hipStream_t st) : phase(ph), s(st)
    {
        if (g_opt.timing.load()) {
            a = g_timers.get();
            if (a && hipEventRecord(a, s) != hipSuccess) {
                g_timers.pool.push_back(a);
                a = nullptr;
            }
        }
    }
    ~Timed()
    {
        if (!a) return;
        hipEvent_t b = g_timers.get();
        if (b && hipEventRecord(b, s) == hipSuccess)
            g_timers.pending.push_back({phase, a, b});
        else {
            g_timers.pool.push_back(a);
            if (b) g_timers.pool.push_back(b);
        }
    }
};

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(call)                                                                             \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail(MPHX_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));             \
    } while (0)

constexpr uint64_t kRoundCapMax = 1ull << 22;

uint64_t round_cap(uint64_t n) { return std::min<uint64_t>(std::max<uint64_t>(n, 1), kRoundCapMax) + 1; }

// Bump allocator over the caller's workspace; with base == nullptr it only measures.
struct Carve {
    uint8_t* base;
    size_t off = 0;
    explicit Carve(void* b) : base((uint8_t*)b) {}
    template <class T>
    T* take(uint64_t count)
    {
        off = (off + 255) & ~(size_t)255;
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += (size_t)count * sizeof(T);
        return p;
    }
};

struct PeelLayout {
    Ctrl* ctrl;
    uint64_t *lstart, *rec;
    unsigned long long* lcount;
    uint32_t *state, *tilehist, *ids;
    uint3* slots;
    void* scan;
    size_t scan_bytes;
};

void layout_peel(Carve& c, uint64_t n, uint64_t m, PeelLayout& L)
{
    uint64_t rcap = round_cap(n);
    L.ctrl = c.take<Ctrl>(1);
    L.lstart = c.take<uint64_t>(rcap + 2);
    L.lcount = c.take<unsigned long long>(rcap + 2);
    L.rec = c.take<uint64_t>(m);
    L.slots = c.take<uint3>(n);
    L.state = c.take<uint32_t>(n);
    L.ids = reinterpret_cast<uint32_t*>(L.slots);  // sort scratch once the peel is over
    uint64_t hist_entries = 256 * sort_tiles(n);
    L.tilehist = c.take<uint32_t>(hist_entries);
    L.scan_bytes = scan_scratch_bytes(hist_entries);
    L.scan = c.take<uint8_t>(L.scan_bytes);
}

struct MphfLayout {
    Ctrl* ctrl;
    uint64_t *lstart, *rec;
    unsigned long long* lcount;
    uint32_t *edges, *state, *bcount;
    uint3* slots;
    uint2 *pairs1, *pairs2;  // the partitioned build's buffers, over slots and state
    void* aux;               // histograms and scan scratch of the partitions
    uint2 *claims, *claims_tmp;  // claim lists (m each), when used
    unsigned long long* ccount;  // claim counts per round
    unsigned long long* dcount;  // update-list counts per round
    uint32_t* vals;              // static functions without claim lists: the values in layer order
    void* scan;
    size_t scan_bytes;
};

// sf: a static-function build, whose values reach the assignment in layer order through n
// u32: the edge states with claim lists (unused there), else an array of their own.
void layout_mphf(Carve& c, uint64_t n, uint64_t m, bool lists, MphfLayout& L, bool sf = false)
{
    uint64_t rcap = round_cap(n);
    L.ctrl = c.take<Ctrl>(1);
    L.lstart = c.take<uint64_t>(rcap + 2);
    L.lcount = c.take<unsigned long long>(rcap + 2);
    L.edges = c.take<uint32_t>(3 * n);
    L.rec = c.take<uint64_t>(m);  // also the byte codes after peeling
    // slots (12n) then state (4n) in one region of 16n bytes, which the partitioned build
    // uses first as two buffers of n (vertex, edge) pairs
    uint8_t* region = c.take<uint8_t>(16 * n);
    L.slots = reinterpret_cast<uint3*>(region);
    L.state = reinterpret_cast<uint32_t*>(region ? region + 12 * n : nullptr);
    L.pairs1 = reinterpret_cast<uint2*>(region);
    L.pairs2 = reinterpret_cast<uint2*>(region ? region + 8 * n : nullptr);
    L.aux = c.take<uint8_t>(part_aux_bytes(n, m / 3, lists));
    L.ccount = c.take<unsigned long long>(2 * (rcap + 2));
    L.dcount = L.ccount ? L.ccount + rcap + 2 : nullptr;
    L.claims = lists ? c.take<uint2>(m) : nullptr;
    L.claims_tmp = lists ? c.take<uint2>(m) : nullptr;
    uint64_t nblocks = (m + 511) / 512;
    L.bcount = c.take<uint32_t>(nblocks);
    L.scan_bytes = scan_scratch_bytes(nblocks);
    L.scan = c.take<uint8_t>(L.scan_bytes);
    L.vals = (sf && !lists) ? c.take<uint32_t>(n) : nullptr;
}

bool aligned256(const void* p) { return ((uintptr_t)p & 255) == 0; }

int read_ctrl(Ctrl* dctrl, Ctrl& h, hipStream_t s)
{
    HIP_TRY(hipMemcpyAsync(&h, dctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return MPHX_OK;
}

// Apply grids: one 256-thread block per 256 layer edges, between 64 and 1024 blocks (four per
// compute unit; the kernels stride over larger layers).  A batch of rounds shares the grid of
// its first layer, so a larger cap launched thousands of idle blocks into the small rounds
// after it: 1024 against 8192 measured 2-4 % faster from 10^7 to 6x10^7 keys and no slower
// at 2^27 and 2^31.
unsigned auto_grid(uint64_t work)
{
    int g = g_opt.grid.load();
    if (g > 0) return (unsigned)g;
    uint64_t b = (work + 255) / 256;
    return (unsigned)std::min<uint64_t>(std::max<uint64_t>(b, 64), 1024);
}

constexpr uint32_t kLaterBatch = 16;

// Enqueue rounds in batches until a round finds an empty layer.  On return
// h.nrounds holds the number of non-empty layers and *peeled the number of peeled edges.
int run_rounds(PeelState& st, Ctrl& h, uint64_t* peeled, hipStream_t s)
{
    uint32_t r = 0;
    uint32_t batch = (uint32_t)std::max(1, g_opt.round_batch.load());
    unsigned long long next_layer = 0;
    HIP_TRY(hipMemcpyAsync(&next_layer, st.lcount, sizeof next_layer, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (;;) {
        uint64_t upto = std::min<uint64_t>((uint64_t)r + batch, st.rcap);
        // sized for the next layer; later rounds of the batch may be larger, which only costs
        // them more grid-stride iterations
        st.grid_cap = auto_grid(next_layer);
        for (; r < upto; r++) {
            Timed t(PH_APPLY, s);
            HIP_TRY(launch_apply(st, r, false, ApplyMode::kAtomicClaims, s));
        }
        HIP_TRY(hipMemcpyAsync(&next_layer, st.lcount + r, sizeof next_layer, hipMemcpyDeviceToHost, s));
        int rc = read_ctrl(st.ctrl, h, s);
        if (rc) return rc;
        if (h.nrounds != 0xFFFFFFFFu) {
            uint64_t p = 0;
            HIP_TRY(hipMemcpyAsync(&p, st.lstart + h.nrounds, sizeof p, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            *peeled = p;
            return MPHX_OK;
        }
        if (r >= st.rcap)
            return fail(MPHX_ERANGE, "more than %llu peeling rounds", (unsigned long long)st.rcap);
        batch = kLaterBatch;
    }
}

// Claim-list rounds.  Layer 0 comes from round 0's atomic claims, which keep it in vertex
// order (its hinges ascending, which the assignment's code writes profit from) and leave the
// hinge in the edge state.  Every apply appends the next layer's claims and cancels to the
// list, which is resolved into the next layer (the hinge lands in the slot).  One host read
// per round sizes the resolve.  A round whose list resolves to nothing ends the peel.
constexpr int kListOverflow = 1000;  // internal: a round's records exceeded the claim list

// Claim-list rounds.  Round r's layer comes from round r - 1's claims (resolve), then
// apply(r) deletes it.  A dense round -- twice its claim count, which bounds its deletes, at
// least update_lists percent of m -- appends its deletes to an update list applied per vertex
// bucket (Section 4.2's sort-based round update), which leaves the next claims in
// st.claims_tmp; a sparse round deletes with atomics and appends claims and cancels to
// st.claims.
int run_rounds_lists(PeelState& st, Ctrl& h, uint64_t* peeled, hipStream_t s)
{
    const uint64_t upd = (uint64_t)g_opt.update_lists.load();
    bool in_tmp = false;  // round r's claims sit in st.claims_tmp
    for (uint32_t r = 0;; r++) {
        if (r > st.rcap)
            return fail(MPHX_ERANGE, "more than %llu peeling rounds", (unsigned long long)st.rcap);
        unsigned long long est = 0;
        if (r > 0) {
            HIP_TRY(hipMemcpyAsync(&est, st.ccount + r, sizeof est, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            if (est > st.lcap)
                return kListOverflow;  // the list holds m records; no layer of a large random graph comes near
            Timed t(PH_RESOLVE, s);
            HIP_TRY(launch_claims_resolve(st, r, est, in_tmp, s));
        } else {
            HIP_TRY(hipMemcpyAsync(&est, st.lcount, sizeof est, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
        }
        st.grid_cap = auto_grid(est);  // the records bound the layer
        if (r == 0 && st.round0_updates) {
            // round 0 already wrote layer 0's slots and its update list
            HIP_TRY(launch_close_layer(st, 0, s));
            unsigned long long dels = 0;
            HIP_TRY(hipMemcpyAsync(&dels, st.dcount, sizeof dels, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            if (dels > st.lcap)
                return kListOverflow;  // layer 0 larger than m/2 edges: redo with atomic claims
            Timed t(PH_UPDATE, s);
            HIP_TRY(launch_update_apply(st, 0, dels, s));
            in_tmp = true;
            if (est == 0)
                break;
            continue;
        }
        // a layer of at most est edges deletes at most 2 est times, which the list must hold
        const bool updates = upd > 0 && 2 * est <= st.lcap && 200 * (unsigned __int128)est >= (unsigned __int128)upd * st.m;
        {
            Timed t(PH_APPLY, s);
            HIP_TRY(launch_apply(st, r, true, updates ? ApplyMode::kUpdateList : ApplyMode::kClaimList, s));
        }
        in_tmp = false;
        if (updates) {
            unsigned long long dels = 0;
            HIP_TRY(hipMemcpyAsync(&dels, st.dcount + r, sizeof dels, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            if (dels > st.lcap)
                return fail(MPHX_ERANGE, "update list of round %u overflowed (%llu deletes)", r, dels);
            Timed t(PH_UPDATE, s);
            HIP_TRY(launch_update_apply(st, r, dels, s));
            in_tmp = true;
        }
        if (est == 0)
            break;
    }
    int rc = read_ctrl(st.ctrl, h, s);
    if (rc) return rc;
    uint64_t p = 0;
    HIP_TRY(hipMemcpyAsync(&p, st.lstart + h.nrounds, sizeof p, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *peeled = p;
    return MPHX_OK;
}

int check_build_errors(Ctrl* dctrl, uint64_t n, hipStream_t s, uint64_t& first_front, uint32_t r = 3)
{
    Ctrl h;
    int rc = read_ctrl(dctrl, h, s);
    if (rc) return rc;
    first_front = h.ftail;
    if (h.err & kErrBadEdge)
        return fail(MPHX_EINVAL, "edge with a vertex id >= m or a repeated vertex");
    // every degree field at most 255 and their total exactly r n: no field overflowed
    if ((h.err & kErrDegree) || h.degsum != (uint64_t)r * n)
        return fail(MPHX_ERANGE, "a vertex has degree above %u", MPHX_MAX_DEGREE);
    return MPHX_OK;
}

// The round loop of an r-hypergraph peel: as run_rounds, with the r-vertex apply.
int run_rounds_r(PeelState& st, uint32_t r, Ctrl& h, uint64_t* peeled, hipStream_t s)
{
    uint32_t rd = 0;
    uint32_t batch = (uint32_t)std::max(1, g_opt.round_batch.load());
    unsigned long long next_layer = 0;
    HIP_TRY(hipMemcpyAsync(&next_layer, st.lcount, sizeof next_layer, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (;;) {
        uint64_t upto = std::min<uint64_t>((uint64_t)rd + batch, st.rcap);
        st.grid_cap = auto_grid(next_layer);
        for (; rd < upto; rd++) {
            Timed t(PH_APPLY, s);
            HIP_TRY(launch_apply_r(st, r, rd, s));
        }
        HIP_TRY(hipMemcpyAsync(&next_layer, st.lcount + rd, sizeof next_layer, hipMemcpyDeviceToHost, s));
        int rc = read_ctrl(st.ctrl, h, s);
        if (rc) return rc;
        if (h.nrounds != 0xFFFFFFFFu) {
            uint64_t p = 0;
            HIP_TRY(hipMemcpyAsync(&p, st.lstart + h.nrounds, sizeof p, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            *peeled = p;
            return MPHX_OK;
        }
        if (rd >= st.rcap)
            return fail(MPHX_ERANGE, "more than %llu peeling rounds", (unsigned long long)st.rcap);
        batch = kLaterBatch;
    }
}

}  // namespace

extern "C" {

const char* mphx_last_error(void) { return g_err.c_str(); }

uint64_t mphx_part_size(uint64_t n, uint32_t gamma_num, uint32_t gamma_den)
{
    if (gamma_den == 0) return 0;
    unsigned __int128 num = (unsigned __int128)n * gamma_num;
    unsigned __int128 den = (unsigned __int128)3 * gamma_den;
    return (uint64_t)((num + den - 1) / den);
}

int mphx_set_option(const char* key, int64_t value)
{
    if (!key) return fail(MPHX_EINVAL, "null option key");
    if (!strcmp(key, "grid")) {
        if (value < 0 || value > (1 << 20)) return fail(MPHX_EINVAL, "grid out of range");
        g_opt.grid = (int)value;
    } else if (!strcmp(key, "round_batch")) {
        if (value < 1 || value > 4096) return fail(MPHX_EINVAL, "round_batch out of range");
        g_opt.round_batch = (int)value;
    } else if (!strcmp(key, "timing")) {
        if (value != 0 && value != 1) return fail(MPHX_EINVAL, "timing must be 0 or 1");
        g_opt.timing = (int)value;
    } else if (!strcmp(key, "part_build")) {
        if (value < 0 || value > 32) return fail(MPHX_EINVAL, "part_build must be in 0..32");
        g_opt.part_build = (int)value;
    } else if (!strcmp(key, "claim_lists")) {
        if (value < 0 || value > 32) return fail(MPHX_EINVAL, "claim_lists must be in 0..32");
        g_opt.claim_lists = (int)value;
    } else if (!strcmp(key, "update_lists")) {
        if (value < 0 || value > 100) return fail(MPHX_EINVAL, "update_lists must be in 0..100");
        g_opt.update_lists = (int)value;
    } else if (!strcmp(key, "hem_block")) {
        if (value != 256 && value != 512 && value != 1024) return fail(MPHX_EINVAL, "hem_block must be 256, 512 or 1024");
        g_opt.hem_block = (int)value;
    } else if (!strcmp(key, "batch_lds")) {
        if (value != 0 && value != 1) return fail(MPHX_EINVAL, "batch_lds must be 0 or 1");
        g_opt.batch_lds = (int)value;
    } else if (!strcmp(key, "batch_sort_deletes")) {
        if (value < 0 || value > 1024) return fail(MPHX_EINVAL, "batch_sort_deletes must be in 0..1024");
        g_opt.batch_sort_deletes = (int)value;
    } else if (!strcmp(key, "batch_claim_lists")) {
        if (value != 0 && value != 1) return fail(MPHX_EINVAL, "batch_claim_lists must be 0 or 1");
        g_opt.batch_claim_lists = (int)value;
    } else if (!strcmp(key, "batch_clock")) {
        if (value != 0 && value != 1) return fail(MPHX_EINVAL, "batch_clock must be 0 or 1");
        g_opt.batch_clock = (int)value;
    } else if (!strcmp(key, "hem_grid")) {
        if (value < 0 || value > (1 << 16)) return fail(MPHX_EINVAL, "hem_grid must be in 0..65536");
        g_opt.hem_grid = (int)value;
    } else if (!strcmp(key, "list_cap")) {
        if (value < 0) return fail(MPHX_EINVAL, "list_cap must be >= 0");
        g_opt.list_cap = value;
    } else if (!strcmp(key, "list_fallbacks")) {
        if (value != 0) return fail(MPHX_EINVAL, "list_fallbacks can only be reset to 0");
        g_opt.list_fallbacks = 0;
    } else {
        return fail(MPHX_EINVAL, "unknown option '%s'", key);
    }
    return MPHX_OK;
}

int64_t mphx_get_option(const char* key)
{
    if (!key) return MPHX_EINVAL;
    if (!strcmp(key, "grid")) return g_opt.grid;
    if (!strcmp(key, "round_batch")) return g_opt.round_batch;
    if (!strcmp(key, "timing")) return g_opt.timing;
    if (!strcmp(key, "part_build")) return g_opt.part_build;
    if (!strcmp(key, "claim_lists")) return g_opt.claim_lists;
    if (!strcmp(key, "update_lists")) return g_opt.update_lists;
    if (!strcmp(key, "hem_block")) return g_opt.hem_block;
    if (!strcmp(key, "hem_grid")) return g_opt.hem_grid;
    if (!strcmp(key, "batch_lds")) return g_opt.batch_lds;
    if (!strcmp(key, "batch_sort_deletes")) return g_opt.batch_sort_deletes;
    if (!strcmp(key, "batch_claim_lists")) return g_opt.batch_claim_lists;
    if (!strcmp(key, "batch_clock")) return g_opt.batch_clock;
    if (!strcmp(key, "list_cap")) return g_opt.list_cap;
    if (!strcmp(key, "list_fallbacks")) return g_opt.list_fallbacks;
    fail(MPHX_EINVAL, "unknown option '%s'", key);
    return MPHX_EINVAL;
}

int mphx_phase_times(double* ms, uint64_t* launches, int max_phases, int reset)
{
    int k = std::min<int>(max_phases, PH_COUNT);
    for (int i = 0; i < k; i++) {
        if (ms) ms[i] = g_timers.ms[i];
        if (launches) launches[i] = g_timers.launches[i];
    }
    if (reset) {
        for (int i = 0; i < PH_COUNT; i++) {
            g_timers.ms[i] = 0;
            g_timers.launches[i] = 0;
        }
    }
    return PH_COUNT;
}

const char* mphx_phase_name(int i) { return (i >= 0 && i < PH_COUNT) ? kPhaseNames[i] : ""; }

int mphx_batch_clock(uint64_t* out, int max_entries, int reset)
{
    if (max_entries < 0 || (max_entries > 0 && !out)) return fail(MPHX_EINVAL, "null output");
    hipError_t err = batch_clock_read(out, max_entries, reset != 0);
    if (err != hipSuccess) return fail(MPHX_EDEVICE, "batch clock: %s", hipGetErrorString(err));
    return (int)kBatchClockEntries;
}

const char* mphx_batch_clock_name(int i) { return batch_clock_name(i); }

size_t mphx_peel_workspace_bytes(uint64_t n, uint64_t m)
{
    Carve c(nullptr);
    PeelLayout L;
    layout_peel(c, n, m, L);
    return c.off;
}

int mphx_peel(const uint32_t* edges, uint64_t n, uint64_t m, uint32_t* order, uint32_t* round, uint8_t* core_mask,
              uint8_t* hinge, void* ws, size_t ws_bytes, void* stream, mphx_peel_info* info)
{
    g_err.clear();
    hipStream_t s = (hipStream_t)stream;
    if (n >= 0xFFFFFFFFull || m > 0x100000000ull)
        return fail(MPHX_EINVAL, "n must be < 2^32 - 1 and m <= 2^32");
    if (n > 0 && (!edges || !order || !round || !core_mask))
        return fail(MPHX_EINVAL, "null pointer argument");
    if (!ws || !aligned256(ws))
        return fail(MPHX_EINVAL, "workspace must be non-null and 256-byte aligned");
    if (ws_bytes < mphx_peel_workspace_bytes(n, m))
        return fail(MPHX_ENOMEM, "workspace of %zu bytes, need %zu", ws_bytes, mphx_peel_workspace_bytes(n, m));
    if (info) memset(info, 0, sizeof *info);
    if (n == 0) return MPHX_OK;

    Carve c(ws);
    PeelLayout L;
    layout_peel(c, n, m, L);

    PeelState st{};
    st.edges = edges;
    st.n = n;
    st.m = m;
    st.P = 0;
    st.tripartite = false;
    st.rec = L.rec;
    st.slots = L.slots;
    st.state = L.state;
    st.lstart = L.lstart;
    st.lcount = L.lcount;
    st.ctrl = L.ctrl;
    st.rcap = round_cap(n);

    HIP_TRY(launch_zero(L.rec, m * sizeof(uint64_t), s));
    HIP_TRY(launch_fill_u32(L.state, n, kUnclaimed, s));
    HIP_TRY(launch_zero(L.lcount, (st.rcap + 2) * sizeof(unsigned long long), s));
    HIP_TRY(launch_ctrl_init(L.ctrl, L.lstart, s));
    {
        Timed t(PH_BUILD, s);
        HIP_TRY(launch_edges_build(edges, n, m, L.rec, L.ctrl, s));
    }
    {
        Timed t(PH_FRONTIER, s);
        HIP_TRY(launch_round0(st, s));
    }
    uint64_t f0 = 0;
    int rc = check_build_errors(L.ctrl, n, s, f0);
    if (rc) return rc;

    Ctrl h;
    uint64_t peeled = 0;
    rc = run_rounds(st, h, &peeled, s);
    if (rc) return rc;

    {
        Timed t(PH_ORDER, s);
        HIP_TRY(launch_peel_finalize(L.state, n, round, core_mask, hinge, s));
        HIP_TRY(launch_order_sort(round, n, h.nrounds, order, L.ids, L.tilehist, L.scan, L.scan_bytes, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    g_timers.harvest();
    if (info) {
        info->n_peeled = peeled;
        info->n_rounds = h.nrounds;
        info->frontier_total = h.ftail;
        info->claims = h.claims;
        info->frontier0 = f0;
    }
    return MPHX_OK;
}

size_t mphx_peel_r_workspace_bytes(uint64_t n, uint64_t m, uint32_t r)
{
    if (r < 2 || r > 8) return 0;
    return mphx_peel_workspace_bytes(n, m);
}

int mphx_peel_r(const uint32_t* edges, uint64_t n, uint64_t m, uint32_t r, uint32_t* order, uint32_t* round,
                uint8_t* core_mask, uint8_t* hinge, void* ws, size_t ws_bytes, void* stream, mphx_peel_info* info)
{
    g_err.clear();
    hipStream_t s = (hipStream_t)stream;
    if (r < 2 || r > 8) return fail(MPHX_EINVAL, "r must be in [2, 8]");
    if (n >= 0xFFFFFFFFull || m > 0x100000000ull)
        return fail(MPHX_EINVAL, "n must be < 2^32 - 1 and m <= 2^32");
    if (n > 0 && (!edges || !order || !round || !core_mask))
        return fail(MPHX_EINVAL, "null pointer argument");
    if (!ws || !aligned256(ws))
        return fail(MPHX_EINVAL, "workspace must be non-null and 256-byte aligned");
    if (ws_bytes < mphx_peel_r_workspace_bytes(n, m, r))
        return fail(MPHX_ENOMEM, "workspace of %zu bytes, need %zu", ws_bytes, mphx_peel_r_workspace_bytes(n, m, r));
    if (info) memset(info, 0, sizeof *info);
    if (n == 0) return MPHX_OK;

    Carve c(ws);
    PeelLayout L;
    layout_peel(c, n, m, L);
    PeelState st{};
    st.edges = edges;
    st.n = n;
    st.m = m;
    st.tripartite = false;
    st.rec = L.rec;
    st.slots = L.slots;
    st.state = L.state;
    st.lstart = L.lstart;
    st.lcount = L.lcount;
    st.ctrl = L.ctrl;
    st.rcap = round_cap(n);

    HIP_TRY(launch_zero(L.rec, m * sizeof(uint64_t), s));
    HIP_TRY(launch_fill_u32(L.state, n, kUnclaimed, s));
    HIP_TRY(launch_zero(L.lcount, (st.rcap + 2) * sizeof(unsigned long long), s));
    HIP_TRY(launch_ctrl_init(L.ctrl, L.lstart, s));
    {
        Timed t(PH_BUILD, s);
        HIP_TRY(launch_edges_build_r(edges, n, m, r, L.rec, L.ctrl, s));
    }
    {
        Timed t(PH_FRONTIER, s);
        HIP_TRY(launch_round0_r(st, r, s));
    }
    uint64_t f0 = 0;
    int rc = check_build_errors(L.ctrl, n, s, f0, r);
    if (rc) return rc;
    Ctrl h;
    uint64_t peeled = 0;
    rc = run_rounds_r(st, r, h, &peeled, s);
    if (rc) return rc;
    {
        Timed t(PH_ORDER, s);
        HIP_TRY(launch_peel_finalize_r(L.state, n, round, core_mask, hinge, s));
        HIP_TRY(launch_order_sort(round, n, h.nrounds, order, L.ids, L.tilehist, L.scan, L.scan_bytes, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    g_timers.harvest();
    if (info) {
        info->n_peeled = peeled;
        info->n_rounds = h.nrounds;
        info->frontier_total = h.ftail;
        info->claims = h.claims;
        info->frontier0 = f0;
    }
    return MPHX_OK;
}

size_t mphx_mphf_workspace_bytes(uint64_t n, uint32_t gamma_num, uint32_t gamma_den, int key_kind)
{
    (void)key_kind;
    uint64_t m = 3 * mphx_part_size(n, gamma_num, gamma_den);
    Carve c(nullptr);
    MphfLayout L;
    layout_mphf(c, n, m, use_claim_lists(n), L);
    return c.off;
}

size_t mphx_sf_workspace_bytes(uint64_t n, uint32_t gamma_num, uint32_t gamma_den, int key_kind)
{
    (void)key_kind;
    uint64_t m = 3 * mphx_part_size(n, gamma_num, gamma_den);
    Carve c(nullptr);
    MphfLayout L;
    layout_mphf(c, n, m, use_claim_lists(n), L, true);
    return c.off;
}

uint32_t mphx_sf_bits(uint64_t sigma)
{
    uint32_t b = 0;
    while (b < 64 && sigma > 0 && ((sigma - 1) >> b) != 0)
        b++;
    return b;
}

uint64_t mphx_sf_words(uint64_t n, uint32_t gamma_num, uint32_t gamma_den, uint64_t sigma)
{
    return (3 * mphx_part_size(n, gamma_num, gamma_den) * mphx_sf_bits(sigma) + 63) / 64;
}

}  // extern "C"

namespace {

struct KeySrc {
    int kind;  // MPHX_KEYS_U64 / MPHX_KEYS_STR
    const uint64_t* keys;
    const uint8_t* bytes;
    const uint64_t* offs;
};

// Are the keys of edges a and b equal?  (Only called on the failure path.)
int keys_equal(const KeySrc& k, uint64_t a, uint64_t b, bool& eq, hipStream_t s)
{
    if (k.kind == MPHX_KEYS_U64) {
        uint64_t x = 0, y = 0;
        HIP_TRY(hipMemcpyAsync(&x, k.keys + a, 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(&y, k.keys + b, 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        eq = x == y;
        return MPHX_OK;
    }
    uint64_t oa[2], ob[2];
    HIP_TRY(hipMemcpyAsync(oa, k.offs + a, 16, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(ob, k.offs + b, 16, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (oa[1] - oa[0] != ob[1] - ob[0]) {
        eq = false;
        return MPHX_OK;
    }
    std::vector<uint8_t> x(oa[1] - oa[0]), y(ob[1] - ob[0]);
    if (!x.empty()) {
        HIP_TRY(hipMemcpyAsync(x.data(), k.bytes + oa[0], x.size(), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(y.data(), k.bytes + ob[0], y.size(), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    eq = x == y;
    return MPHX_OK;
}

// After the last failed try: do identical core edges come from equal keys?  The core edges
// and the pairs of them with equal vertex triples are found on the device (the slot region,
// 16n bytes, is free once the tries are over); only the pairs' keys are read back.
int detect_duplicates(const KeySrc& k, const MphfLayout& L, uint64_t n, bool& dup, hipStream_t s)
{
    dup = false;
    HIP_TRY(launch_ctrl_init(L.ctrl, L.lstart, s));
    HIP_TRY(launch_core_count(L.rec, L.edges, n, L.ctrl, s));
    Ctrl h{};
    int rc = read_ctrl(L.ctrl, h, s);
    if (rc) return rc;
    const uint64_t core = h.aux;
    if (core < 2) return MPHX_OK;
    // at most 2/3 full: tsize <= 3 core <= 3n entries of 4 bytes, leaving >= 4n bytes of pairs
    uint64_t tsize = 2;
    while (tsize < core + core / 2 + 1)
        tsize <<= 1;
    uint32_t* tab = reinterpret_cast<uint32_t*>(L.slots);
    uint2* pairs = reinterpret_cast<uint2*>(tab + tsize);
    const uint32_t pcap = (uint32_t)std::min<uint64_t>((16 * n - 4 * tsize) / sizeof(uint2), 1024);
    HIP_TRY(launch_fill_u32(tab, tsize, kUnclaimed, s));
    HIP_TRY(launch_core_pairs(L.rec, L.edges, n, tab, tsize, pairs, pcap, L.ctrl, s));
    rc = read_ctrl(L.ctrl, h, s);
    if (rc) return rc;
    std::vector<uint2> hp((size_t)std::min<uint64_t>(h.dups, pcap));
    if (!hp.empty()) {
        HIP_TRY(hipMemcpyAsync(hp.data(), pairs, hp.size() * sizeof(uint2), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    for (const uint2& p : hp) {
        bool eq = false;
        rc = keys_equal(k, p.x, p.y, eq, s);
        if (rc) return rc;
        if (eq) {
            dup = true;
            break;
        }
    }
    return MPHX_OK;
}

// A static function's values and sigma (Section 3); absent for the MPHF.
struct SfArgs {
    const uint32_t* values;
    uint64_t sigma;
    // the ranked layout's outputs (Section 3, ranking structure); null for the plain layout
    uint64_t* marks = nullptr;
    uint64_t* rank = nullptr;
    uint64_t* vals = nullptr;
};

// The MPHF (codes + rank) or, with sf, the static function (codes = its packed fields).
int mphf_build(const KeySrc& k, uint64_t n, uint64_t seed, uint32_t gnum, uint32_t gden, uint32_t max_tries,
               uint64_t* codes, uint64_t* rank, void* ws, size_t ws_bytes, hipStream_t s, mphx_mphf_info* info,
               const SfArgs* sf = nullptr)
{
    g_err.clear();
    if (gnum == 0 || gden == 0) return fail(MPHX_EINVAL, "gamma must be a positive fraction");
    if (max_tries == 0) return fail(MPHX_EINVAL, "max_tries must be >= 1");
    if (n >= 0xFFFFFFFFull) return fail(MPHX_EINVAL, "n must be < 2^32 - 1");
    const uint64_t P = mphx_part_size(n, gnum, gden);
    const uint64_t m = 3 * P;
    if (m > 0x100000000ull) return fail(MPHX_EINVAL, "3P = %llu vertices exceed 2^32", (unsigned long long)m);
    if (n > 0) {
        if (k.kind == MPHX_KEYS_U64 && !k.keys) return fail(MPHX_EINVAL, "null keys");
        if (k.kind == MPHX_KEYS_STR && (!k.bytes || !k.offs)) return fail(MPHX_EINVAL, "null bytes/offs");
        if (k.kind == MPHX_KEYS_STR && ((uintptr_t)k.bytes & 3)) return fail(MPHX_EINVAL, "bytes must be 4-byte aligned");
        const bool no_fields = sf && mphx_sf_bits(sf->sigma) == 0;
        if (sf && sf->marks ? (!sf->values || !sf->rank || (!sf->vals && !no_fields))
                            : sf ? (!sf->values || (!codes && !no_fields)) : (!codes || !rank))
            return fail(MPHX_EINVAL, "null values or output");
    }
    if (sf && (sf->sigma == 0 || sf->sigma > 0x100000000ull)) return fail(MPHX_EINVAL, "sigma must be in [1, 2^32]");
    if (!ws || !aligned256(ws)) return fail(MPHX_EINVAL, "workspace must be non-null and 256-byte aligned");
    const bool lists = use_claim_lists(n);
    size_t need = sf ? mphx_sf_workspace_bytes(n, gnum, gden, k.kind) : mphx_mphf_workspace_bytes(n, gnum, gden, k.kind);
    if (ws_bytes < need) return fail(MPHX_ENOMEM, "workspace of %zu bytes, need %zu", ws_bytes, need);
    if (info) {
        memset(info, 0, sizeof *info);
        info->P = P;
        info->m = m;
        info->seed_used = seed;
    }
    if (n == 0) {
        if (info) info->tries = 1;
        return MPHX_OK;
    }

    Carve c(ws);
    MphfLayout L;
    layout_mphf(c, n, m, lists, L, sf != nullptr);
    if (sf) {  // every value below sigma
        HIP_TRY(launch_ctrl_init(L.ctrl, L.lstart, s));
        HIP_TRY(launch_sf_check(sf->values, n, sf->sigma, L.ctrl, s));
        Ctrl hc;
        int rc = read_ctrl(L.ctrl, hc, s);
        if (rc) return rc;
        if (hc.err & kErrValue) return fail(MPHX_EINVAL, "a value is not below sigma = %llu", (unsigned long long)sf->sigma);
    }

    PeelState st{};
    st.edges = L.edges;
    st.n = n;
    st.m = m;
    st.P = P;
    st.tripartite = true;
    st.rec = L.rec;
    st.slots = L.slots;
    st.state = L.state;
    st.lstart = L.lstart;
    st.lcount = L.lcount;
    st.ctrl = L.ctrl;
    st.rcap = round_cap(n);
    st.lists = lists;
    st.lcap = m;
    if (g_opt.list_cap.load() > 0)
        st.lcap = std::min<uint64_t>(m, (uint64_t)g_opt.list_cap.load());
    st.claims = L.claims;
    st.claims_tmp = L.claims_tmp;
    st.ccount = L.ccount;
    st.dcount = L.dcount;
    st.aux = L.aux;

    Ctrl h{};
    uint64_t peeled = 0;
    uint32_t t = 0;
    bool done = false;
    for (t = 0; t < max_tries; t++) {
        uint64_t sd = seed + t;
        const int pb = g_opt.part_build.load();
        const bool part = pb > 0 && n >= (1ull << pb);  // pb <= 32
        if (!part)
            HIP_TRY(launch_zero(L.rec, m * sizeof(uint64_t), s));
        HIP_TRY(launch_zero(L.lcount, (st.rcap + 2) * sizeof(unsigned long long), s));
        HIP_TRY(launch_zero(L.ccount, 2 * (st.rcap + 2) * sizeof(unsigned long long), s));
        HIP_TRY(launch_ctrl_init(L.ctrl, L.lstart, s));
        {
            // with the partitioned build the hash only writes the edges
            Timed tm(PH_HASH, s);
            uint64_t* fused = part ? nullptr : L.rec;
            const PartHist1 h1 = part ? part_hist1(L.aux, n, P) : PartHist1{nullptr, 0, 0};
            if (k.kind == MPHX_KEYS_U64)
                HIP_TRY(launch_hash_u64(k.keys, n, sd, P, L.edges, fused, h1, s));
            else
                HIP_TRY(launch_hash_str(k.bytes, k.offs, n, sd, P, L.edges, fused, h1, s));
        }
        if (part) {
            Timed tm(PH_BUILD, s);
            // the claim buffers (m >= n pairs each) are free until the rounds
            HIP_TRY(launch_part_build(L.edges, n, P, L.rec, L.pairs1, L.pairs2, L.claims, L.claims_tmp, L.aux, s));
        }
        // atomic claims keep per-edge states (after the build: they share the pair buffers);
        // claim lists carry the hinge in the layer slots from round 0 on
        if (!st.lists)
            HIP_TRY(launch_fill_u32(L.state, n, kUnclaimed, s));
        st.round0_updates = st.lists && g_opt.update_lists.load() > 0;
        if (sf) {
            // the values in layer order: over the edge states with claim lists; over the idle
            // claim buffers when a try fell back to atomic claims; else their own array
            st.vin = sf->values;
            st.vout = st.lists ? L.state : (L.claims ? reinterpret_cast<uint32_t*>(L.claims) : L.vals);
        }
        {
            Timed tm(PH_FRONTIER, s);
            HIP_TRY(launch_round0(st, s));
        }
        uint64_t f0 = 0;
        int rc = check_build_errors(L.ctrl, n, s, f0);
        if (rc) {
            if (info) { info->tries = t + 1; info->seed_used = sd; }
            return rc;
        }
        rc = st.lists ? run_rounds_lists(st, h, &peeled, s) : run_rounds(st, h, &peeled, s);
        if (rc == kListOverflow) {  // redo this try with atomic claims
            g_opt.list_fallbacks++;
            st.lists = false;
            t--;
            continue;
        }
        if (rc) return rc;
        if (info) {
            info->tries = t + 1;
            info->seed_used = sd;
            info->n_rounds = h.nrounds;
            info->n_core = n - peeled;
            info->frontier_total = h.ftail;
            info->claims = h.claims;
            info->frontier0 = f0;
            info->update_deletes = h.updates;
            info->update_records = h.touched;
        }
        if (peeled == n) {
            done = true;
            break;
        }
    }
    if (!done) {
        bool dup = false;
        int rc = detect_duplicates(k, L, n, dup, s);
        if (rc) return rc;
        if (dup) return fail(MPHX_EDUP, "duplicate keys: identical edges from equal keys stay in the 2-core");
        return fail(MPHX_ECORE, "2-core of %llu edges after %u tries", (unsigned long long)(n - peeled), max_tries);
    }

    // Assignment in reverse round order with exact grids from the layer bounds.
    std::vector<uint64_t> lb(h.nrounds + 1);
    HIP_TRY(hipMemcpyAsync(lb.data(), L.lstart, lb.size() * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (info) info->layer0 = h.nrounds ? lb[1] - lb[0] : 0;
    if (sf) {
        // u (one narrow element per vertex, over the records) solved layer by layer, then packed
        const uint32_t b = mphx_sf_bits(sf->sigma);
        void* u = L.rec;
        HIP_TRY(launch_zero(u, m * sf_elem_bytes(b), s));
        HIP_TRY(hipStreamSynchronize(s));
        for (int64_t r = (int64_t)h.nrounds - 1; r >= 0; r--) {
            Timed tm(PH_ASSIGN, s);
            HIP_TRY(launch_sf_assign_round(L.slots + lb[r], st.vout + lb[r], lb[r + 1] - lb[r], sf->sigma, b, u, s));
        }
        if (sf->marks) {
            // ranked layout: marks and per-block counts, their prefix, then the fields compacted
            Timed tm(PH_RANK, s);
            const uint64_t nb = (m + kSfrBlock - 1) / kSfrBlock;
            HIP_TRY(launch_sfr_marks(u, m, b, sf->marks, L.bcount, s));
            HIP_TRY(launch_scan_u32_to_u64(L.bcount, nb, sf->rank, nb + 1, L.scan, L.scan_bytes, s));
            if (b) {
                const uint64_t cap = mphx_sfr_val_words(n, sf->sigma);
                HIP_TRY(launch_zero(sf->vals, cap * sizeof(uint64_t), s));
                HIP_TRY(launch_sfr_compact(u, m, b, sf->rank, sf->vals, cap, s));
            }
        } else {
            Timed tm(PH_RANK, s);
            HIP_TRY(launch_sf_pack(u, m, b, codes, s));
        }
        HIP_TRY(hipStreamSynchronize(s));
        g_timers.harvest();
        return MPHX_OK;
    }
    uint8_t* code8 = reinterpret_cast<uint8_t*>(L.rec);
    HIP_TRY(launch_zero(code8, m, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int64_t r = (int64_t)h.nrounds - 1; r >= 0; r--) {
        uint64_t cnt = lb[r + 1] - lb[r];
        Timed tm(PH_ASSIGN, s);
        HIP_TRY(launch_assign_round(L.slots, L.lstart, (uint32_t)r, cnt, P, code8, 16384, s));
    }
    {
        Timed tm(PH_RANK, s);
        HIP_TRY(launch_pack_count(code8, m, codes, L.bcount, s));
        uint64_t nblocks = (m + 511) / 512;
        HIP_TRY(launch_scan_u32_to_u64(L.bcount, nblocks, rank, nblocks, L.scan, L.scan_bytes, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    g_timers.harvest();
    return MPHX_OK;
}

}  // namespace

extern "C" {

int mphx_mphf_build_u64(const uint64_t* keys, uint64_t n, uint64_t seed, uint32_t gamma_num, uint32_t gamma_den,
                        uint32_t max_tries, uint64_t* codes, uint64_t* rank, void* ws, size_t ws_bytes, void* stream,
                        mphx_mphf_info* info)
{
    KeySrc k{MPHX_KEYS_U64, keys, nullptr, nullptr};
    return mphf_build(k, n, seed, gamma_num, gamma_den, max_tries, codes, rank, ws, ws_bytes, (hipStream_t)stream,
                      info);
}

}  // extern "C"

namespace {

// Workspace of the allocation-free build: one array per device, held from the library's load
// to the end of the process.  Host code never passes the array's name to a kernel or a copy:
// on the host it is only a stand-in for the device symbol, so each device's address is looked
// up once (with that device current) and kept here.
constexpr size_t kStaticScratchBytes = 128ull << 20;
__device__ __attribute__((used)) __align__(256) uint8_t scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // by device ordinal

int static_scratch(void** out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr.size() <= (size_t)dev) g_scratch_ptr.resize((size_t)dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(MPHX_EDEVICE, "device %d: address of the static workspace: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MPHX_OK;
}

}  // namespace

extern "C" {

int mphx_mphf_build_u64_static(const uint64_t* keys, uint64_t n, uint64_t seed, uint32_t gamma_num,
                               uint32_t gamma_den, uint32_t max_tries, uint64_t* codes, uint64_t* rank, void* stream,
                               mphx_mphf_info* info)
{
    g_err.clear();
    if (gamma_num == 0 || gamma_den == 0) return fail(MPHX_EINVAL, "gamma must be a positive fraction");
    if (n >= 0xFFFFFFFFull) return fail(MPHX_EINVAL, "n must be < 2^32 - 1");
    const size_t need = mphx_mphf_workspace_bytes(n, gamma_num, gamma_den, MPHX_KEYS_U64);
    if (need > kStaticScratchBytes)
        return fail(MPHX_ENOMEM, "%llu keys need %zu bytes of workspace; the allocation-free build has %zu",
                    (unsigned long long)n, need, kStaticScratchBytes);
    void* ws = nullptr;
    int rc = static_scratch(&ws);
    if (rc) return rc;
    KeySrc k{MPHX_KEYS_U64, keys, nullptr, nullptr};
    return mphf_build(k, n, seed, gamma_num, gamma_den, max_tries, codes, rank, ws, kStaticScratchBytes,
                      (hipStream_t)stream, info);
}

int mphx_mphf_build_str(const uint8_t* bytes, const uint64_t* offs, uint64_t n, uint64_t seed, uint32_t gamma_num,
                        uint32_t gamma_den, uint32_t max_tries, uint64_t* codes, uint64_t* rank, void* ws,
                        size_t ws_bytes, void* stream, mphx_mphf_info* info)
{
    KeySrc k{MPHX_KEYS_STR, nullptr, bytes, offs};
    return mphf_build(k, n, seed, gamma_num, gamma_den, max_tries, codes, rank, ws, ws_bytes, (hipStream_t)stream,
                      info);
}

int mphx_sf_build_u64(const uint64_t* keys, const uint32_t* values, uint64_t n, uint64_t sigma, uint64_t seed,
                      uint32_t gamma_num, uint32_t gamma_den, uint32_t max_tries, uint64_t* words, void* ws,
                      size_t ws_bytes, void* stream, mphx_mphf_info* info)
{
    KeySrc k{MPHX_KEYS_U64, keys, nullptr, nullptr};
    SfArgs sf{values, sigma};
    return mphf_build(k, n, seed, gamma_num, gamma_den, max_tries, words, nullptr, ws, ws_bytes, (hipStream_t)stream,
                      info, &sf);
}

int mphx_sf_build_str(const uint8_t* bytes, const uint64_t* offs, const uint32_t* values, uint64_t n, uint64_t sigma,
                      uint64_t seed, uint32_t gamma_num, uint32_t gamma_den, uint32_t max_tries, uint64_t* words,
                      void* ws, size_t ws_bytes, void* stream, mphx_mphf_info* info)
{
    KeySrc k{MPHX_KEYS_STR, nullptr, bytes, offs};
    SfArgs sf{values, sigma};
    return mphf_build(k, n, seed, gamma_num, gamma_den, max_tries, words, nullptr, ws, ws_bytes, (hipStream_t)stream,
                      info, &sf);
}

uint64_t mphx_sfr_mark_words(uint64_t n, uint32_t gamma_num, uint32_t gamma_den)
{
    return (3 * mphx_part_size(n, gamma_num, gamma_den) + 63) / 64;
}

uint64_t mphx_sfr_rank_words(uint64_t n, uint32_t gamma_num, uint32_t gamma_den)
{
    return (3 * mphx_part_size(n, gamma_num, gamma_den) + kSfrBlock - 1) / kSfrBlock + 1;
}

uint64_t mphx_sfr_val_words(uint64_t n, uint64_t sigma)
{
    return (n * mphx_sf_bits(sigma) + 63) / 64;
}

int mphx_sfr_build_u64(const uint64_t* keys, const uint32_t* values, uint64_t n, uint64_t sigma, uint64_t seed,
                       uint32_t gamma_num, uint32_t gamma_den, uint32_t max_tries, uint64_t* marks, uint64_t* rank,
                       uint64_t* vals, void* ws, size_t ws_bytes, void* stream, mphx_mphf_info* info)
{
    KeySrc k{MPHX_KEYS_U64, keys, nullptr, nullptr};
    SfArgs sf{values, sigma, marks, rank, vals};
    if (n > 0 && !marks) return fail(MPHX_EINVAL, "null marks");
    return mphf_build(k, n, seed, gamma_num, gamma_den, max_tries, nullptr, nullptr, ws, ws_bytes,
                      (hipStream_t)stream, info, &sf);
}

int mphx_sfr_build_str(const uint8_t* bytes, const uint64_t* offs, const uint32_t* values, uint64_t n, uint64_t sigma,
                       uint64_t seed, uint32_t gamma_num, uint32_t gamma_den, uint32_t max_tries, uint64_t* marks,
                       uint64_t* rank, uint64_t* vals, void* ws, size_t ws_bytes, void* stream, mphx_mphf_info* info)
{
    KeySrc k{MPHX_KEYS_STR, nullptr, bytes, offs};
    SfArgs sf{values, sigma, marks, rank, vals};
    if (n > 0 && !marks) return fail(MPHX_EINVAL, "null marks");
    return mphf_build(k, n, seed, gamma_num, gamma_den, max_tries, nullptr, nullptr, ws, ws_bytes,
                      (hipStream_t)stream, info, &sf);
}

int mphx_sfr_lookup_u64(const uint64_t* marks, const uint64_t* rank, const uint64_t* vals, uint64_t sigma, uint64_t P,
                        uint64_t seed, const uint64_t* keys, uint64_t n, uint64_t* out, void* stream)
{
    g_err.clear();
    if (n == 0) return MPHX_OK;
    const uint32_t b = mphx_sf_bits(sigma);
    if (!marks || !rank || (!vals && b > 0) || !keys || !out || P == 0 || sigma == 0 || sigma > 0x100000000ull)
        return fail(MPHX_EINVAL, "null pointer, P = 0 or sigma out of [1, 2^32]");
    HIP_TRY(launch_sfr_lookup_u64(marks, rank, vals, sigma, b, P, seed, keys, n, out, (hipStream_t)stream));
    return MPHX_OK;
}

int mphx_sfr_lookup_str(const uint64_t* marks, const uint64_t* rank, const uint64_t* vals, uint64_t sigma, uint64_t P,
                        uint64_t seed, const uint8_t* bytes, const uint64_t* offs, uint64_t n, uint64_t* out,
                        void* stream)
{
    g_err.clear();
    if (n == 0) return MPHX_OK;
    const uint32_t b = mphx_sf_bits(sigma);
    if (!marks || !rank || (!vals && b > 0) || !bytes || !offs || !out || P == 0 || sigma == 0 ||
        sigma > 0x100000000ull)
        return fail(MPHX_EINVAL, "null pointer, P = 0 or sigma out of [1, 2^32]");
    if ((uintptr_t)bytes & 3) return fail(MPHX_EINVAL, "bytes must be 4-byte aligned");
    HIP_TRY(launch_sfr_lookup_str_words(marks, rank, vals, sigma, b, P, seed, bytes, offs, n, out,
                                        (hipStream_t)stream));
    return MPHX_OK;
}

int mphx_sf_lookup_u64(const uint64_t* words, uint64_t sigma, uint64_t P, uint64_t seed, const uint64_t* keys,
                       uint64_t n, uint64_t* out, void* stream)
{
    g_err.clear();
    if (n == 0) return MPHX_OK;
    const uint32_t b = mphx_sf_bits(sigma);
    if ((!words && b > 0) || !keys || !out || P == 0 || sigma == 0 || sigma > 0x100000000ull)
        return fail(MPHX_EINVAL, "null pointer, P = 0 or sigma out of [1, 2^32]");
    HIP_TRY(launch_sf_lookup_u64(words, sigma, b, P, seed, keys, n, out, (hipStream_t)stream));
    return MPHX_OK;
}

int mphx_sf_lookup_str(const uint64_t* words, uint64_t sigma, uint64_t P, uint64_t seed, const uint8_t* bytes,
                       const uint64_t* offs, uint64_t n, uint64_t* out, void* stream)
{
    g_err.clear();
    if (n == 0) return MPHX_OK;
    const uint32_t b = mphx_sf_bits(sigma);
    if ((!words && b > 0) || !bytes || !offs || !out || P == 0 || sigma == 0 || sigma > 0x100000000ull)
        return fail(MPHX_EINVAL, "null pointer, P = 0 or sigma out of [1, 2^32]");
    if ((uintptr_t)bytes & 3) return fail(MPHX_EINVAL, "bytes must be 4-byte aligned");
    HIP_TRY(launch_sf_lookup_str_words(words, sigma, b, P, seed, bytes, offs, n, out, (hipStream_t)stream));
    return MPHX_OK;
}

int mphx_mphf_lookup_u64(const uint64_t* codes, const uint64_t* rank, uint64_t P, uint64_t seed, const uint64_t* keys,
                         uint64_t n, uint64_t* out, void* stream)
{
    g_err.clear();
    if (n == 0) return MPHX_OK;
    if (!codes || !rank || !keys || !out || P == 0) return fail(MPHX_EINVAL, "null pointer or P = 0");
    HIP_TRY(launch_lookup_u64(codes, rank, P, seed, keys, n, out, (hipStream_t)stream));
    return MPHX_OK;
}

int mphx_mphf_lookup_str(const uint64_t* codes, const uint64_t* rank, uint64_t P, uint64_t seed, const uint8_t* bytes,
                         const uint64_t* offs, uint64_t n, uint64_t* out, void* stream)
{
    g_err.clear();
    if (n == 0) return MPHX_OK;
    if (!codes || !rank || !bytes || !offs || !out || P == 0) return fail(MPHX_EINVAL, "null pointer or P = 0");
    if ((uintptr_t)bytes & 3) return fail(MPHX_EINVAL, "bytes must be 4-byte aligned");
    HIP_TRY(launch_lookup_str_words(codes, rank, P, seed, bytes, offs, n, out, (hipStream_t)stream));
    return MPHX_OK;
}

int mphx_hash_u64(const uint64_t* keys, uint64_t n, uint64_t seed, uint64_t P, uint32_t* edges, void* stream)
{
    g_err.clear();
    if (n == 0) return MPHX_OK;
    if (!keys || !edges) return fail(MPHX_EINVAL, "null pointer");
    if (P == 0 || 3 * P > 0x100000000ull) return fail(MPHX_EINVAL, "P out of range");
    HIP_TRY(launch_hash_u64(keys, n, seed, P, edges, nullptr, PartHist1{nullptr, 0, 0}, (hipStream_t)stream));
    return MPHX_OK;
}

int mphx_hash_str(const uint8_t* bytes, const uint64_t* offs, uint64_t n, uint64_t seed, uint64_t P, uint32_t* edges,
                  void* stream)
{
    g_err.clear();
    if (n == 0) return MPHX_OK;
    if (!bytes || !offs || !edges) return fail(MPHX_EINVAL, "null pointer");
    if ((uintptr_t)bytes & 3) return fail(MPHX_EINVAL, "bytes must be 4-byte aligned");
    if (P == 0 || 3 * P > 0x100000000ull) return fail(MPHX_EINVAL, "P out of range");
    HIP_TRY(launch_hash_str(bytes, offs, n, seed, P, edges, nullptr, PartHist1{nullptr, 0, 0}, (hipStream_t)stream));
    return MPHX_OK;
}

size_t mphx_bijection_scratch_bytes(uint64_t n)
{
    uint64_t words = (n + 31) / 32;
    return (size_t)(((words * 4 + 255) & ~255ull) + sizeof(Ctrl));
}

int mphx_check_bijection(const uint64_t* vals, uint64_t n, void* scratch, uint64_t* n_bad, void* stream)
{
    g_err.clear();
    hipStream_t s = (hipStream_t)stream;
    if (!n_bad) return fail(MPHX_EINVAL, "null n_bad");
    *n_bad = 0;
    if (n == 0) return MPHX_OK;
    if (!vals || !scratch || !aligned256(scratch)) return fail(MPHX_EINVAL, "null or misaligned pointer");
    // bitmap words first, then one control slot for the violation counter
    uint64_t words = (n + 31) / 32;
    uint32_t* bitmap = reinterpret_cast<uint32_t*>(scratch);
    Ctrl* ctrl = reinterpret_cast<Ctrl*>(reinterpret_cast<uint8_t*>(scratch) + ((words * 4 + 255) & ~255ull));
    HIP_TRY(launch_zero(bitmap, words * 4, s));
    HIP_TRY(launch_zero(ctrl, sizeof(Ctrl), s));
    HIP_TRY(launch_bijection(vals, n, bitmap, ctrl, s));
    unsigned long long bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, &ctrl->aux, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *n_bad = bad;
    return MPHX_OK;
}

int mphx_gen_keys_u64(uint64_t* keys, uint64_t n, uint64_t gen_seed, uint64_t start, void* stream)
{
    g_err.clear();
    if (n && !keys) return fail(MPHX_EINVAL, "null keys");
    HIP_TRY(launch_gen_u64(keys, n, gen_seed, start, (hipStream_t)stream));
    return MPHX_OK;
}

int mphx_gen_buckets_u64(uint64_t* keys, const uint64_t* off, uint32_t B, void* stream)
{
    g_err.clear();
    if (B && (!keys || !off)) return fail(MPHX_EINVAL, "null pointer");
    HIP_TRY(launch_gen_buckets_u64(keys, off, B, (hipStream_t)stream));
    return MPHX_OK;
}

int mphx_gen_str_lengths(uint32_t* lens, uint64_t n, uint64_t gen_seed, uint64_t start, const uint16_t* qtable,
                         void* stream)
{
    g_err.clear();
    if (n && (!lens || !qtable)) return fail(MPHX_EINVAL, "null pointer");
    HIP_TRY(launch_gen_str_lengths(lens, n, gen_seed, start, qtable, (hipStream_t)stream));
    return MPHX_OK;
}

size_t mphx_scan_scratch_bytes(uint64_t count) { return scan_scratch_bytes(count); }

int mphx_gen_str_offsets(const uint32_t* lens, uint64_t n, uint64_t* offs, void* scratch, size_t scratch_bytes,
                         void* stream)
{
    g_err.clear();
    if (!offs || (n && !lens) || !scratch) return fail(MPHX_EINVAL, "null pointer");
    if (scratch_bytes < scan_scratch_bytes(n + 1)) return fail(MPHX_ENOMEM, "scan scratch too small");
    HIP_TRY(launch_scan_u32_to_u64(lens, n, offs, n + 1, scratch, scratch_bytes, (hipStream_t)stream));
    return MPHX_OK;
}

int mphx_gen_str_bytes(uint8_t* bytes, const uint64_t* offs, uint64_t n, uint64_t gen_seed, uint64_t start,
                       void* stream)
{
    g_err.clear();
    if (n && (!bytes || !offs)) return fail(MPHX_EINVAL, "null pointer");
    if ((uintptr_t)bytes & 3) return fail(MPHX_EINVAL, "bytes must be 4-byte aligned");
    HIP_TRY(launch_gen_str_bytes(bytes, offs, n, gen_seed, start, (hipStream_t)stream));
    return MPHX_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------------------------
// Batched builds
// ------------------------------------------------------------------------------------------
namespace {

static_assert(sizeof(mphx_bucket_result) == sizeof(BucketResult), "bucket result layouts agree");
static_assert(sizeof(mphx_mphf_info) == 88 && sizeof(mphx_peel_info) == 40, "info layouts as documented");
static_assert(sizeof(mphx_bucket) == sizeof(BucketDesc), "bucket descriptor layouts agree");

int batch_tuning(const mphx_batch_tuning* t, unsigned& block, unsigned& grid)
{
    block = (t && t->block) ? t->block : 1024;
    if (block != 256 && block != 512 && block != 1024)
        return fail(MPHX_EINVAL, "batch block must be 256, 512 or 1024");
    grid = t ? t->grid : 0;
    if (grid == 0) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        grid = (unsigned)cus;
    }
    if (grid > (1u << 20))
        return fail(MPHX_EINVAL, "batch grid too large");
    return MPHX_OK;
}

size_t batch_ws_bytes(uint32_t B, uint64_t max_bucket, uint32_t gnum, uint32_t gden, unsigned grid)
{
    return 256 + (((size_t)B * sizeof(BucketDesc) + 255) & ~(size_t)255) +
           (size_t)grid * batch_slot_bytes(max_bucket, gnum, gden);
}

int batch_enqueue(const uint64_t* keys, const uint64_t* bucket_off, const uint32_t* order, uint32_t B,
                  uint64_t max_bucket, uint64_t seed, uint32_t gnum, uint32_t gden, uint32_t max_tries,
                  const uint64_t* code_off, const uint64_t* rank_off, uint64_t* codes, uint64_t* rank,
                  mphx_bucket_result* results, void* ws, size_t ws_bytes, const mphx_batch_tuning* t,
                  hipStream_t s, bool pairs = false)
{
    if (gnum == 0 || gden == 0 || max_tries == 0) return fail(MPHX_EINVAL, "bad gamma or max_tries");
    if (B == 0) return MPHX_OK;
    if (!keys || !bucket_off || !order || !code_off || !rank_off || !codes || !rank || !results)
        return fail(MPHX_EINVAL, "null pointer argument");
    if (max_bucket >= 0xFFFFFFFFull || 3 * mphx_part_size(max_bucket, gnum, gden) > 0x100000000ull)
        return fail(MPHX_EINVAL, "max_bucket too large");
    unsigned block = 0, grid = 0;
    int rc = batch_tuning(t, block, grid);
    if (rc) return rc;
    if (!ws || !aligned256(ws)) return fail(MPHX_EINVAL, "workspace must be non-null and 256-byte aligned");
    size_t need = batch_ws_bytes(B, max_bucket, gnum, gden, grid);
    if (ws_bytes < need) return fail(MPHX_ENOMEM, "workspace of %zu bytes, need %zu", ws_bytes, need);
    uint8_t* base = reinterpret_cast<uint8_t*>(ws);
    BucketDesc* descs = reinterpret_cast<BucketDesc*>(base + 256);
    BatchArgs a{};
    a.descs = descs;
    a.order = order;
    a.B = B;
    a.gnum = gnum;
    a.gden = gden;
    a.max_tries = max_tries;
    a.next = reinterpret_cast<unsigned int*>(base);
    a.slots = base + 256 + (((size_t)B * sizeof(BucketDesc) + 255) & ~(size_t)255);
    a.slot_bytes = batch_slot_bytes(max_bucket, gnum, gden);
    a.max_n = max_bucket;
    a.lds_path = (uint32_t)g_opt.batch_lds.load();
    a.sort_div = (uint32_t)g_opt.batch_sort_deletes.load();
    a.claim_lists = (uint32_t)g_opt.batch_claim_lists.load();
    a.clock = (uint32_t)g_opt.batch_clock.load();
    a.pairs = pairs ? 1u : 0u;
    HIP_TRY(launch_batch_descs(descs, keys, bucket_off, B, seed, code_off, rank_off, codes, rank,
                               reinterpret_cast<BucketResult*>(results), s, pairs ? 2u : 1u));
    HIP_TRY(launch_batch(a, block, grid, !(t && t->scope == 1), s));
    return MPHX_OK;
}

}  // namespace

extern "C" {

int mphx_batch_layout(const uint64_t* bucket_off, uint32_t B, uint32_t gnum, uint32_t gden, uint64_t* code_off,
                      uint64_t* rank_off, uint32_t* order, uint64_t* max_bucket)
{
    g_err.clear();
    if (!bucket_off || !code_off || !rank_off || !order || !max_bucket) return fail(MPHX_EINVAL, "null pointer");
    if (gnum == 0 || gden == 0) return fail(MPHX_EINVAL, "bad gamma");
    uint64_t cw = 0, cr = 0, mx = 0;
    std::vector<std::pair<uint64_t, uint32_t>> sz(B);
    for (uint32_t b = 0; b < B; b++) {
        if (bucket_off[b + 1] < bucket_off[b]) return fail(MPHX_EINVAL, "bucket offsets decrease at %u", b);
        uint64_t n = bucket_off[b + 1] - bucket_off[b];
        uint64_t m = 3 * mphx_part_size(n, gnum, gden);
        if (n >= 0xFFFFFFFFull || m > 0x100000000ull) return fail(MPHX_EINVAL, "bucket %u too large", b);
        code_off[b] = cw;
        rank_off[b] = cr;
        cw += (m + 31) / 32;
        cr += (m + 511) / 512;
        mx = std::max(mx, n);
        sz[b] = {n, b};
    }
    code_off[B] = cw;
    rank_off[B] = cr;
    std::stable_sort(sz.begin(), sz.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
    for (uint32_t b = 0; b < B; b++) order[b] = sz[b].second;
    *max_bucket = mx;
    return MPHX_OK;
}

size_t mphx_batch_workspace_bytes(uint32_t B, uint64_t max_bucket, uint32_t gnum, uint32_t gden,
                                  const mphx_batch_tuning* t)
{
    unsigned block = 0, grid = 0;
    if (batch_tuning(t, block, grid)) return 0;
    return batch_ws_bytes(B, max_bucket, gnum, gden, grid);
}

// ---- HEM split (Section 3) ---------------------------------------------------------------
// Workspace: signature records and the partition's second buffer (8n each), the partition's
// histograms, the processing order and per-bucket results, and the batched build's scratch
// for buckets up to the bound below (bucket sizes are binomial around n / 2^k).
static uint64_t hem_max_bucket(uint64_t n, uint32_t k)
{
    const uint64_t mean = n >> k;
    uint64_t r = 1;
    while (r * r < mean) r++;
    return mean + 8 * r + 64;
}

// The batched kernel's shape for the HEM split's many equal buckets (library options).
static mphx_batch_tuning hem_tuning()
{
    mphx_batch_tuning t{};
    t.block = (uint32_t)g_opt.hem_block.load();
    t.grid = (uint32_t)g_opt.hem_grid.load();
    t.scope = 0;
    return t;
}

// Up to 2^18 buckets come straight from the two-pass partition; beyond, each of the 2^18
// coarse buckets is split by the next k - 18 bits.
static constexpr uint32_t kHemMaxK = 20, kHemCoarseK = 18;

}  // extern "C"

// Signature records: uint2 (8 bytes) for u64 keys, uint4 (16 bytes: the whole digest) for strings.
template <class R>
struct HemLayout {
    R *rec, *tmp;
    uint64_t* coff;  // coarse bucket offsets (k > 18 only)
    void* aux;
    uint32_t* order;
    mphx_bucket_result* results;
    uint8_t* batch;
    size_t batch_bytes;
};

template <class R>
static void layout_hem(Carve& c, uint64_t n, uint32_t k, uint32_t gnum, uint32_t gden, HemLayout<R>& L)
{
    const uint32_t B = 1u << k, kc = std::min(k, kHemCoarseK);
    L.rec = c.take<R>(n);
    L.tmp = c.take<R>(n);
    L.coff = k > kc ? c.take<uint64_t>((1ull << kc) + 1) : nullptr;
    L.aux = c.take<uint8_t>(hem_aux_bytes(n, kc));
    L.order = c.take<uint32_t>(B);
    L.results = c.take<mphx_bucket_result>(B);
    const mphx_batch_tuning t = hem_tuning();
    L.batch_bytes = mphx_batch_workspace_bytes(B, hem_max_bucket(n, k), gnum, gden, &t);
    L.batch = c.take<uint8_t>(L.batch_bytes);
}

extern "C" {

size_t mphx_hem_workspace_bytes(uint64_t n, uint32_t k, uint32_t gnum, uint32_t gden, int key_kind)
{
    if (k < 9 || k > kHemMaxK || gnum == 0 || gden == 0) return 0;
    Carve c(nullptr);
    if (key_kind == MPHX_KEYS_U64) {
        HemLayout<uint2> L;
        layout_hem(c, n, k, gnum, gden, L);
    } else if (key_kind == MPHX_KEYS_STR) {
        HemLayout<uint4> L;
        layout_hem(c, n, k, gnum, gden, L);
    } else {
        return 0;
    }
    return c.off;
}

int mphx_hem_capacity(uint64_t n, uint32_t k, uint32_t gnum, uint32_t gden, uint64_t* code_words,
                      uint64_t* rank_words)
{
    g_err.clear();
    if (k < 9 || k > kHemMaxK || gnum == 0 || gden == 0 || !code_words || !rank_words)
        return fail(MPHX_EINVAL, "k must be in [9, 20], gamma positive, outputs non-null");
    // sum over buckets of 3 ceil(n_b num / 3 den) <= n num / den + 3 * 2^k vertices
    const uint64_t B = 1ull << k;
    const uint64_t mv = (uint64_t)(((unsigned __int128)n * gnum + gden - 1) / gden) + 3 * B;
    *code_words = mv / 32 + B + 1;
    *rank_words = mv / 512 + B + 1;
    return MPHX_OK;
}

int mphx_build_batch_u64(const uint64_t* keys, const uint64_t* bucket_off, const uint32_t* order, uint32_t B,
                         uint64_t max_bucket, uint64_t seed, uint32_t gnum, uint32_t gden, uint32_t max_tries,
                         const uint64_t* code_off, const uint64_t* rank_off, uint64_t* codes, uint64_t* rank,
                         mphx_bucket_result* results, void* ws, size_t ws_bytes, const mphx_batch_tuning* t,
                         void* stream)
{
    g_err.clear();
    return batch_enqueue(keys, bucket_off, order, B, max_bucket, seed, gnum, gden, max_tries, code_off, rank_off,
                         codes, rank, results, ws, ws_bytes, t, (hipStream_t)stream);
}

uint32_t mphx_batch_tuning_candidates(mphx_batch_tuning* out, uint32_t cap)
{
    // The workgroup size fixes the LDS budget and tile (1024 threads: 158 KB, 8192-vertex
    // tiles, one workgroup per compute unit; 512: 78 KB and 4096, up to two; 256: 48 KB and
    // 4096, up to three), so each size comes with the grids its occupancy allows.
    unsigned block = 0, cus = 0;
    if (batch_tuning(nullptr, block, cus)) cus = 256;
    const mphx_batch_tuning c[] = {{1024, cus, 0, 0}, {512, cus, 0, 0}, {512, 2 * cus, 0, 0},
                                   {256, 2 * cus, 0, 0}, {256, 3 * cus, 0, 0}};
    const uint32_t n = (uint32_t)(sizeof(c) / sizeof(c[0]));
    for (uint32_t i = 0; i < n && i < cap && out; i++) out[i] = c[i];
    return n;
}

int mphx_batch_autotune_u64(const uint64_t* keys, const uint64_t* bucket_off, const uint32_t* order, uint32_t B,
                            uint64_t max_bucket, uint64_t seed, uint32_t gnum, uint32_t gden, uint32_t max_tries,
                            const uint64_t* code_off, const uint64_t* rank_off, uint64_t* codes, uint64_t* rank,
                            mphx_bucket_result* results, void* ws, size_t ws_bytes,
                            const mphx_batch_tuning* cands, uint32_t ncand, uint32_t reps, float* ms,
                            uint32_t* best, void* stream)
{
    g_err.clear();
    // every argument is checked before the first device call
    if (!cands || ncand == 0 || !best) return fail(MPHX_EINVAL, "candidates and best must be given");
    if (reps == 0 || reps > 100) return fail(MPHX_EINVAL, "reps must be in [1, 100]");
    if (gnum == 0 || gden == 0 || max_tries == 0) return fail(MPHX_EINVAL, "bad gamma or max_tries");
    std::vector<unsigned> grids(ncand);
    for (uint32_t i = 0; i < ncand; i++) {
        unsigned block = 0;
        int rc = batch_tuning(&cands[i], block, grids[i]);
        if (rc) return rc;
    }
    *best = 0;
    if (B == 0) {
        for (uint32_t i = 0; ms && i < ncand; i++) ms[i] = 0.0f;
        return MPHX_OK;
    }
    if (!keys || !bucket_off || !order || !code_off || !rank_off || !codes || !rank || !results)
        return fail(MPHX_EINVAL, "null pointer argument");
    if (!ws || !aligned256(ws)) return fail(MPHX_EINVAL, "workspace must be non-null and 256-byte aligned");

    hipStream_t s = (hipStream_t)stream;
    hipEvent_t ev[2] = {nullptr, nullptr};
    struct Events {
        hipEvent_t* e;
        ~Events()
        {
            for (int i = 0; i < 2; i++)
                if (e[i]) (void)hipEventDestroy(e[i]);
        }
    } guard{ev};
    HIP_TRY(hipEventCreate(&ev[0]));
    HIP_TRY(hipEventCreate(&ev[1]));
    float top = -1.0f;
    for (uint32_t i = 0; i < ncand; i++) {
        float t = -1.0f;  // -1: the candidate's workspace does not fit in ws_bytes
        if (batch_ws_bytes(B, max_bucket, gnum, gden, grids[i]) <= ws_bytes) {
            // one untimed build, then the best of reps; every build rewrites the same outputs
            for (uint32_t r = 0; r <= reps; r++) {
                HIP_TRY(hipEventRecord(ev[0], s));
                int rc = batch_enqueue(keys, bucket_off, order, B, max_bucket, seed, gnum, gden, max_tries, code_off,
                                       rank_off, codes, rank, results, ws, ws_bytes, &cands[i], s);
                if (rc) return rc;
                HIP_TRY(hipEventRecord(ev[1], s));
                HIP_TRY(hipEventSynchronize(ev[1]));
                float x = 0.0f;
                HIP_TRY(hipEventElapsedTime(&x, ev[0], ev[1]));
                if (r > 0 && (t < 0.0f || x < t)) t = x;
            }
            if (top < 0.0f || t < top) {
                top = t;
                *best = i;
            }
        }
        if (ms) ms[i] = t;
    }
    if (top < 0.0f) return fail(MPHX_ENOMEM, "no candidate's workspace fits in %zu bytes", ws_bytes);
    return MPHX_OK;
}

size_t mphx_batch_desc_workspace_bytes(uint64_t max_bucket, uint32_t gnum, uint32_t gden, const mphx_batch_tuning* t)
{
    unsigned block = 0, grid = 0;
    if (batch_tuning(t, block, grid)) return 0;
    return 256 + (size_t)grid * batch_slot_bytes(max_bucket, gnum, gden);
}

int mphx_build_batch(const mphx_bucket* buckets, uint32_t B, const uint32_t* order, uint64_t max_bucket,
                     uint32_t gnum, uint32_t gden, uint32_t max_tries, void* ws, size_t ws_bytes,
                     const mphx_batch_tuning* t, void* stream)
{
    g_err.clear();
    if (gnum == 0 || gden == 0 || max_tries == 0) return fail(MPHX_EINVAL, "bad gamma or max_tries");
    if (B == 0) return MPHX_OK;
    if (!buckets) return fail(MPHX_EINVAL, "null buckets");
    if (max_bucket >= 0xFFFFFFFFull || 3 * mphx_part_size(max_bucket, gnum, gden) > 0x100000000ull)
        return fail(MPHX_EINVAL, "max_bucket too large");
    unsigned block = 0, grid = 0;
    int rc = batch_tuning(t, block, grid);
    if (rc) return rc;
    if (!ws || !aligned256(ws)) return fail(MPHX_EINVAL, "workspace must be non-null and 256-byte aligned");
    size_t need = mphx_batch_desc_workspace_bytes(max_bucket, gnum, gden, t);
    if (ws_bytes < need) return fail(MPHX_ENOMEM, "workspace of %zu bytes, need %zu", ws_bytes, need);
    uint8_t* base = reinterpret_cast<uint8_t*>(ws);
    BatchArgs a{};
    a.descs = reinterpret_cast<const BucketDesc*>(buckets);
    a.order = order;
    a.B = B;
    a.gnum = gnum;
    a.gden = gden;
    a.max_tries = max_tries;
    a.next = reinterpret_cast<unsigned int*>(base);
    a.slots = base + 256;
    a.slot_bytes = batch_slot_bytes(max_bucket, gnum, gden);
    a.max_n = max_bucket;
    a.lds_path = (uint32_t)g_opt.batch_lds.load();
    a.sort_div = (uint32_t)g_opt.batch_sort_deletes.load();
    a.claim_lists = (uint32_t)g_opt.batch_claim_lists.load();
    a.clock = (uint32_t)g_opt.batch_clock.load();
    HIP_TRY(launch_batch(a, block, grid, !(t && t->scope == 1), (hipStream_t)stream));
    return MPHX_OK;
}

int mphx_graph_capture_batch_u64(const uint64_t* keys, const uint64_t* bucket_off, const uint32_t* order,
                                 uint32_t B, uint64_t max_bucket, uint64_t seed, uint32_t gnum, uint32_t gden,
                                 uint32_t max_tries, const uint64_t* code_off, const uint64_t* rank_off,
                                 uint64_t* codes, uint64_t* rank, mphx_bucket_result* results, void* ws,
                                 size_t ws_bytes, const mphx_batch_tuning* t, void** graph)
{
    g_err.clear();
    if (!graph) return fail(MPHX_EINVAL, "null graph pointer");
    *graph = nullptr;
    hipStream_t cs = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    int rc = MPHX_OK;
    if (e == hipSuccess) {
        rc = batch_enqueue(keys, bucket_off, order, B, max_bucket, seed, gnum, gden, max_tries, code_off, rank_off,
                           codes, rank, results, ws, ws_bytes, t, cs);
        hipError_t e2 = hipStreamEndCapture(cs, &g);
        if (rc == MPHX_OK && e2 != hipSuccess) e = e2;
    }
    hipGraphExec_t ex = nullptr;
    if (e == hipSuccess && rc == MPHX_OK)
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cs);
    if (rc) return rc;
    if (e != hipSuccess) return fail(MPHX_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
    *graph = ex;
    return MPHX_OK;
}

int mphx_graph_launch(void* graph, void* stream)
{
    g_err.clear();
    if (!graph) return fail(MPHX_EINVAL, "null graph");
    HIP_TRY(hipGraphLaunch((hipGraphExec_t)graph, (hipStream_t)stream));
    return MPHX_OK;
}

int mphx_graph_destroy(void* graph)
{
    g_err.clear();
    if (!graph) return MPHX_OK;
    HIP_TRY(hipGraphExecDestroy((hipGraphExec_t)graph));
    return MPHX_OK;
}


// The per-bucket results of a HEM build: seeds written, info filled, failed buckets reported.
static int hem_finish(uint32_t B, const mphx_bucket_result* results, uint64_t seed, uint64_t code_words,
                      uint64_t* seeds, hipStream_t s, mphx_mphf_info* info)
{
    std::vector<mphx_bucket_result> res(B);
    HIP_TRY(hipMemcpyAsync(res.data(), results, B * sizeof(mphx_bucket_result), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::vector<uint64_t> sd(B);
    uint32_t tries = 0, rounds = 0, failed = 0;
    int worst = MPHX_OK;
    for (uint32_t b = 0; b < B; b++) {
        sd[b] = res[b].seed_used;
        tries = std::max(tries, res[b].tries);
        rounds = std::max(rounds, res[b].n_rounds);
        if (res[b].status != MPHX_OK) {
            failed++;
            if (worst == MPHX_OK) worst = res[b].status;
        }
    }
    HIP_TRY(hipMemcpyAsync(seeds, sd.data(), B * sizeof(uint64_t), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    g_timers.harvest();
    if (info) {
        memset(info, 0, sizeof *info);
        info->m = code_words * 32;
        info->seed_used = seed;
        info->tries = tries;
        info->n_rounds = rounds;
        info->n_core = failed;
    }
    if (worst != MPHX_OK)
        return fail(worst == MPHX_ERANGE ? MPHX_ERANGE : MPHX_ECORE,
                    "%u of %u buckets failed (two keys with one signature, or a 2-core on every try): "
                    "build again with another seed", failed, B);
    return MPHX_OK;
}

}  // extern "C"

template <class R>
static int hem_build(const uint64_t* keys, const uint8_t* bytes, const uint64_t* offs, uint64_t n, uint32_t k,
                     uint64_t seed, uint32_t gnum, uint32_t gden, uint32_t max_tries, uint64_t* bucket_off,
                     uint64_t* code_off, uint64_t* rank_off, uint64_t* seeds, uint64_t* codes, uint64_t* rank,
                     void* ws, size_t ws_bytes, hipStream_t s, mphx_mphf_info* info)
{
    constexpr bool kStr = sizeof(R) == 16;
    const int kind = kStr ? MPHX_KEYS_STR : MPHX_KEYS_U64;
    g_err.clear();
    if (k < 9 || k > kHemMaxK) return fail(MPHX_EINVAL, "k must be in [9, 20]");
    if (gnum == 0 || gden == 0 || max_tries == 0) return fail(MPHX_EINVAL, "bad gamma or max_tries");
    if (n >= 0xFFFFFFFFull) return fail(MPHX_EINVAL, "n must be < 2^32 - 1");
    if (!bucket_off || !code_off || !rank_off || !seeds || !codes || !rank) return fail(MPHX_EINVAL, "null output");
    if (n > 0 && (kind == MPHX_KEYS_U64 ? !keys : (!bytes || !offs))) return fail(MPHX_EINVAL, "null keys");
    if (kind == MPHX_KEYS_STR && ((uintptr_t)bytes & 3)) return fail(MPHX_EINVAL, "bytes must be 4-byte aligned");
    if (!ws || !aligned256(ws)) return fail(MPHX_EINVAL, "workspace must be non-null and 256-byte aligned");
    const size_t need = mphx_hem_workspace_bytes(n, k, gnum, gden, kind);
    if (ws_bytes < need) return fail(MPHX_ENOMEM, "workspace of %zu bytes, need %zu", ws_bytes, need);
    const uint32_t B = 1u << k;
    const mphx_batch_tuning tune = hem_tuning();
    Carve c(ws);
    HemLayout<R> L;
    layout_hem(c, n, k, gnum, gden, L);
    {
        Timed tm(PH_HASH, s);
        if constexpr (kStr)
            HIP_TRY(launch_hem_sig_str(bytes, offs, n, seed, L.rec, s));
        else
            HIP_TRY(launch_hem_sig_u64(keys, n, seed, L.rec, s));
    }
    const uint32_t kc = std::min(k, kHemCoarseK);
    {
        Timed tm(PH_BUILD, s);
        HIP_TRY(launch_hem_partition(L.rec, n, kc, L.tmp, k > kc ? L.coff : bucket_off, L.aux, s));
        if (k > kc) HIP_TRY(launch_hem_refine(L.rec, L.coff, kc, k, L.tmp, bucket_off, s));
    }
    const R* bkeys = k > kc ? L.tmp : L.rec;  // the signatures in bucket order
    std::vector<uint64_t> bo(B + 1), co(B + 1), ro(B + 1);
    std::vector<uint32_t> order(B);
    HIP_TRY(hipMemcpyAsync(bo.data(), bucket_off, (B + 1) * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    uint64_t max_bucket = 0;
    int rc = mphx_batch_layout(bo.data(), B, gnum, gden, co.data(), ro.data(), order.data(), &max_bucket);
    if (rc) return rc;
    if (max_bucket > hem_max_bucket(n, k))
        return fail(MPHX_ENOMEM, "largest bucket %llu exceeds the workspace's bound %llu",
                    (unsigned long long)max_bucket, (unsigned long long)hem_max_bucket(n, k));
    HIP_TRY(hipMemcpyAsync(code_off, co.data(), (B + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(rank_off, ro.data(), (B + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(L.order, order.data(), B * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    {
        Timed tm(PH_OTHER, s);
        // the partitioned records read as u64 words are the bucket keys (u64 keys) or digest
        // pairs (strings)
        rc = batch_enqueue(reinterpret_cast<const uint64_t*>(bkeys), bucket_off, L.order, B, max_bucket, seed, gnum,
                           gden, max_tries, code_off, rank_off, codes, rank, L.results, L.batch, L.batch_bytes,
                           &tune, s, kStr);
        if (rc) return rc;
    }
    return hem_finish(B, L.results, seed, co[B], seeds, s, info);
}

extern "C" {

// ---- HEM split with the keys in host memory (key sets beyond HBM) ------------------------
// The keys stream through the device in chunks: each chunk's signatures are grouped by their
// top k - 8 bits into the resident signature array, so the device holds 8 bytes per key and
// never the keys.  Then batches of consecutive groups are gathered from every chunk,
// partitioned into their buckets and built by the batched kernel.  Each bucket's MPHF depends
// only on the set of its keys, so the result equals the in-HBM split's.
static constexpr uint32_t kHemRunMax = 1u << 16;    // records per gather run
static constexpr uint32_t kHemRunSlots = 1u << 16;  // runs per gather launch

}  // extern "C"

template <class R>
struct HemHostLayout {
    R *sig, *csig, *bsig, *btmp;
    uint8_t* stage;
    uint64_t* soffs;
    void *caux, *baux;
    uint64_t* lbo;
    uint64_t* lbo_c;  // a batch's coarse bucket offsets (k > 18 only)
    uint32_t* order;
    HemRun* runs;
    mphx_bucket_result* results;
    uint8_t* batch;
    size_t batch_bytes;
};

template <class R>
static void layout_hem_host(Carve& c, int kind, uint64_t n, uint32_t k, uint32_t gnum, uint32_t gden,
                            uint64_t chunk_keys, uint64_t chunk_bytes, uint64_t batch_keys, HemHostLayout<R>& L)
{
    const uint32_t B = 1u << k, kc = std::min(k, kHemCoarseK);
    L.sig = c.take<R>(n);
    if (kind == MPHX_KEYS_U64) {
        L.stage = reinterpret_cast<uint8_t*>(c.take<uint64_t>(chunk_keys));
        L.soffs = nullptr;
    } else {
        L.stage = c.take<uint8_t>(chunk_bytes);
        L.soffs = c.take<uint64_t>(chunk_keys + 1);
    }
    L.csig = c.take<R>(chunk_keys);
    L.caux = c.take<uint8_t>(hem_aux_bytes(chunk_keys, kc));
    L.bsig = c.take<R>(batch_keys);
    L.btmp = c.take<R>(batch_keys);
    L.baux = c.take<uint8_t>(hem_aux_bytes(batch_keys, kc));
    L.lbo = c.take<uint64_t>(B + 1);
    L.lbo_c = k > kc ? c.take<uint64_t>((1ull << kc) + 1) : nullptr;
    L.order = c.take<uint32_t>(B);
    L.runs = c.take<HemRun>(kHemRunSlots);
    L.results = c.take<mphx_bucket_result>(B);
    const mphx_batch_tuning t = hem_tuning();
    L.batch_bytes = mphx_batch_workspace_bytes(B, hem_max_bucket(n, k), gnum, gden, &t);
    L.batch = c.take<uint8_t>(L.batch_bytes);
}

extern "C" {

// Host-device copies for the streamed builds.  Pinned host memory is copied directly; pageable
// memory passes through two pinned staging buffers owned by the library.  Towards the device,
// host threads fill one buffer while the DMA engine drains the other (an event per buffer says
// when it is free); towards the host, the DMA engine fills one buffer while host threads empty
// the other.  The buffers live until the process ends; one streamed build uses them at a time.
class HostStager {
  public:
    static constexpr size_t kPiece = size_t(1) << 27;  // bytes per staged copy

    explicit HostStager(hipStream_t s) : s_(s), lock_(pool().mu) {}
    // later copies are ordered on stream s (those already made keep their events)
    void use_stream(hipStream_t s) { s_ = s; }
    ~HostStager()
    {
        for (hipEvent_t& e : ev_)
            if (e) {
                (void)hipEventSynchronize(e);
                (void)hipEventDestroy(e);
            }
    }

    hipError_t copy(void* dst, const void* src, size_t bytes)
    {
        if (bytes == 0) return hipSuccess;
        if (is_pinned(src)) return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s_);
        hipError_t berr = ensure_buffers();
        if (berr != hipSuccess) return berr;
        Pool& p = pool();
        for (size_t o = 0; o < bytes; o += kPiece) {
            const size_t len = std::min(kPiece, bytes - o);
            const int i = next_;
            next_ ^= 1;
            hipError_t err = hipEventSynchronize(ev_[i]);  // the buffer's previous copy has drained
            if (err != hipSuccess) return err;
            parallel_copy(p.buf[i], static_cast<const uint8_t*>(src) + o, len);
            err = hipMemcpyAsync(static_cast<uint8_t*>(dst) + o, p.buf[i], len, hipMemcpyHostToDevice, s_);
            if (err != hipSuccess) return err;
            err = hipEventRecord(ev_[i], s_);
            if (err != hipSuccess) return err;
        }
        return hipSuccess;
    }

    // Device to host; returns when dst holds the bytes (the stream is drained up to the copy).
    hipError_t copy_out(void* dst, const void* src, size_t bytes)
    {
        if (bytes == 0) return hipSuccess;
        if (is_pinned(dst)) {
            hipError_t err = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s_);
            return err != hipSuccess ? err : hipStreamSynchronize(s_);
        }
        hipError_t err = ensure_buffers();
        if (err != hipSuccess) return err;
        const size_t pieces = (bytes + kPiece - 1) / kPiece;
        auto len_of = [&](size_t j) { return std::min(kPiece, bytes - j * kPiece); };
        // piece j goes through buffer j & 1; before a buffer is refilled, its last use (an
        // earlier host-to-device copy, or piece j - 2, emptied below) has finished
        auto issue = [&](size_t j) {
            const int i = (int)(j & 1);
            hipError_t e = hipEventSynchronize(ev_[i]);
            if (e == hipSuccess)
                e = hipMemcpyAsync(pool().buf[i], static_cast<const uint8_t*>(src) + j * kPiece, len_of(j),
                                   hipMemcpyDeviceToHost, s_);
            return e == hipSuccess ? hipEventRecord(ev_[i], s_) : e;
        };
        err = issue(0);
        for (size_t j = 0; j < pieces && err == hipSuccess; j++) {
            if (j + 1 < pieces)
                err = issue(j + 1);
            if (err == hipSuccess)
                err = hipEventSynchronize(ev_[j & 1]);
            if (err == hipSuccess)
                parallel_copy(static_cast<uint8_t*>(dst) + j * kPiece, static_cast<const uint8_t*>(pool().buf[j & 1]),
                              len_of(j));
        }
        return err;
    }

  private:
    hipError_t ensure_buffers()
    {
        Pool& p = pool();
        if (!p.buf[0]) {
            for (void*& b : p.buf) {
                hipError_t e = hipHostMalloc(&b, kPiece, hipHostMallocDefault);
                if (e != hipSuccess) return e;
            }
        }
        for (hipEvent_t& e : ev_)
            if (!e) {
                hipError_t err = hipEventCreateWithFlags(&e, hipEventDisableTiming);
                if (err != hipSuccess) return err;
            }
        return hipSuccess;
    }

    struct Pool {
        std::mutex mu;
        void* buf[2] = {nullptr, nullptr};
    };
    static Pool& pool()
    {
        static Pool p;
        return p;
    }
    static bool is_pinned(const void* p)
    {
        hipPointerAttribute_t a;
        if (hipPointerGetAttributes(&a, p) != hipSuccess) {
            (void)hipGetLastError();  // pageable memory may be reported as an error: clear it
            return false;
        }
        return a.type == hipMemoryTypeHost;
    }
    static void parallel_copy(void* dst, const uint8_t* src, size_t len)
    {
        const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
        const size_t T = std::min<size_t>(std::min(8u, hw), std::max<size_t>(1, len >> 22));
        if (T <= 1) {
            memcpy(dst, src, len);
            return;
        }
        std::vector<std::thread> th;
        const size_t per = (len + T - 1) / T;
        for (size_t t = 0; t < T; t++) {
            const size_t a = t * per, b = std::min(len, a + per);
            if (a < b) th.emplace_back([=] { memcpy(static_cast<uint8_t*>(dst) + a, src + a, b - a); });
        }
        for (std::thread& x : th) x.join();
    }

    hipStream_t s_;
    std::lock_guard<std::mutex> lock_;
    hipEvent_t ev_[2] = {nullptr, nullptr};
    int next_ = 0;
};

static int hem_host_args(int kind, uint32_t k, uint32_t gnum, uint32_t gden, uint64_t chunk_keys,
                         uint64_t chunk_bytes, uint64_t batch_keys)
{
    if (k < 9 || k > kHemMaxK) return fail(MPHX_EINVAL, "k must be in [9, 20]");
    if (gnum == 0 || gden == 0) return fail(MPHX_EINVAL, "bad gamma");
    if (chunk_keys == 0 || chunk_keys >= 0x7FFFFFFFull) return fail(MPHX_EINVAL, "chunk_keys must be in [1, 2^31 - 1)");
    if (batch_keys == 0 || batch_keys >= 0x7FFFFFFFull) return fail(MPHX_EINVAL, "batch_keys must be in [1, 2^31 - 1)");
    if (kind == MPHX_KEYS_STR && chunk_bytes < 512) return fail(MPHX_EINVAL, "chunk_bytes must be at least 512");
    return MPHX_OK;
}

}  // extern "C"

template <class R>
static int hem_host_build(const uint64_t* hkeys, const uint8_t* hbytes, const uint64_t* hoffs, uint64_t n,
                          uint32_t k, uint64_t seed, uint32_t gnum, uint32_t gden, uint32_t max_tries,
                          uint64_t chunk_keys, uint64_t chunk_bytes, uint64_t batch_keys, uint64_t* bucket_off,
                          uint64_t* code_off, uint64_t* rank_off, uint64_t* seeds, uint64_t* codes, uint64_t* rank,
                          void* ws, size_t ws_bytes, hipStream_t s, mphx_mphf_info* info)
{
    constexpr bool kStr = sizeof(R) == 16;
    const int kind = kStr ? MPHX_KEYS_STR : MPHX_KEYS_U64;
    g_err.clear();
    int rc = hem_host_args(kind, k, gnum, gden, chunk_keys, chunk_bytes, batch_keys);
    if (rc) return rc;
    if (max_tries == 0) return fail(MPHX_EINVAL, "max_tries must be positive");
    if (!bucket_off || !code_off || !rank_off || !seeds || !codes || !rank) return fail(MPHX_EINVAL, "null output");
    if (n > 0 && (kind == MPHX_KEYS_U64 ? !hkeys : (!hbytes || !hoffs))) return fail(MPHX_EINVAL, "null keys");
    if (!ws || !aligned256(ws)) return fail(MPHX_EINVAL, "workspace must be non-null and 256-byte aligned");
    const size_t need = mphx_hem_host_workspace_bytes(n, k, gnum, gden, kind, chunk_keys, chunk_bytes, batch_keys);
    if (ws_bytes < need) return fail(MPHX_ENOMEM, "workspace of %zu bytes, need %zu", ws_bytes, need);
    if (kind == MPHX_KEYS_STR && n > 0)
        for (uint64_t i = 0; i < n; i++)
            if (hoffs[i + 1] < hoffs[i]) return fail(MPHX_EINVAL, "offsets decrease at key %llu", (unsigned long long)i);
    const uint32_t kc = std::min(k, kHemCoarseK), NH = 1u << (kc - 8), B = 1u << k;
    const uint32_t gshift = k - kc + 8;  // a group holds 2^gshift buckets
    const mphx_batch_tuning tune = hem_tuning();
    Carve c(ws);
    HemHostLayout<R> L;
    layout_hem_host(c, kind, n, k, gnum, gden, chunk_keys, chunk_bytes, batch_keys, L);

    // host buffers the stream copies from or into; the guard, destroyed first, lets every copy
    // finish before they go, on every return
    std::vector<uint64_t> cbase;
    std::vector<std::unique_ptr<uint32_t[]>> gst;  // per chunk: NH + 1 group starts (filled by the stream)
    std::vector<uint64_t> bo(B + 1, 0), co(B + 1, 0), ro(B + 1, 0), lbo(B + 1);
    std::vector<uint32_t> ord(B);
    std::vector<uint64_t> co_l(B + 1), ro_l(B + 1);
    std::vector<HemRun> runs;
    struct DrainOnExit {
        hipStream_t s;
        ~DrainOnExit() { (void)hipStreamSynchronize(s); }
    } drain{s};
    HostStager stager(s);  // destroyed before the drain: its events are waited for first

    // 1. stream the chunks: signatures, grouped into the resident array at the chunk's place
    {
        Timed tm(PH_HASH, s);
        for (uint64_t c0 = 0; c0 < n;) {
            uint64_t c1 = std::min(n, c0 + chunk_keys);
            if constexpr (!kStr) {
                HIP_TRY(stager.copy(L.stage, hkeys + c0, (c1 - c0) * sizeof(uint64_t)));
                HIP_TRY(launch_hem_sig_u64(reinterpret_cast<const uint64_t*>(L.stage), c1 - c0, seed, L.csig, s));
            } else {
                // the chunk's bytes from a 256-byte boundary, so every key keeps its alignment phase
                const uint64_t bbase = hoffs[c0] & ~255ull, limit = bbase + chunk_bytes;
                c1 = (uint64_t)(std::upper_bound(hoffs + c0 + 1, hoffs + c1 + 1, limit) - hoffs) - 1;
                if (c1 == c0)
                    return fail(MPHX_EINVAL, "key %llu does not fit in chunk_bytes - 255 bytes", (unsigned long long)c0);
                HIP_TRY(stager.copy(L.stage, hbytes + bbase, hoffs[c1] - bbase));
                HIP_TRY(stager.copy(L.soffs, hoffs + c0, (c1 - c0 + 1) * sizeof(uint64_t)));
                HIP_TRY(launch_offs_rebase(L.soffs, c1 - c0 + 1, bbase, s));
                HIP_TRY(launch_hem_sig_str(L.stage, L.soffs, c1 - c0, seed, L.csig, s));
            }
            gst.emplace_back(new uint32_t[NH + 1]);
            HIP_TRY(launch_hem_group_chunk(L.csig, c1 - c0, kc, L.sig + c0, L.caux, gst.back().get(), s));
            cbase.push_back(c0);
            c0 = c1;
        }
    }
    HIP_TRY(hipStreamSynchronize(s));
    const size_t C = cbase.size();
    std::vector<uint64_t> gsize(NH, 0);
    for (size_t j = 0; j < C; j++) {
        const uint64_t cn = (j + 1 < C ? cbase[j + 1] : n) - cbase[j];
        if (gst[j][0] != 0 || gst[j][NH] != cn) return fail(MPHX_EDEVICE, "chunk %zu: group starts inconsistent", j);
        for (uint32_t h = 0; h < NH; h++) gsize[h] += gst[j][h + 1] - gst[j][h];
    }

    // 2. batches of consecutive groups: gather, partition into buckets, build
    const uint64_t bound = hem_max_bucket(n, k);
    uint64_t kbase = 0, cw = 0, rw = 0;
    for (uint32_t g0 = 0; g0 < NH;) {
        uint32_t g1 = g0 + 1;
        uint64_t nb = gsize[g0];
        if (nb > batch_keys)
            return fail(MPHX_ENOMEM, "group %u holds %llu signatures, more than batch_keys", g0, (unsigned long long)nb);
        while (g1 < NH && nb + gsize[g1] <= batch_keys) nb += gsize[g1++];
        {
            Timed tm(PH_BUILD, s);
            uint64_t dst = 0;
            runs.clear();
            for (uint32_t h = g0; h < g1; h++)
                for (size_t j = 0; j < C; j++) {
                    const uint64_t src = cbase[j] + gst[j][h];
                    for (uint64_t len = gst[j][h + 1] - gst[j][h], o = 0; o < len; o += kHemRunMax) {
                        const uint32_t l = (uint32_t)std::min<uint64_t>(kHemRunMax, len - o);
                        if (src + o + l > n || dst + l > nb) return fail(MPHX_EDEVICE, "gather run out of range");
                        runs.push_back(HemRun{src + o, dst, l, 0});
                        dst += l;
                    }
                }
            if (dst != nb) return fail(MPHX_EDEVICE, "batch of groups [%u, %u) gathered %llu of %llu", g0, g1,
                                       (unsigned long long)dst, (unsigned long long)nb);
            for (size_t r0 = 0; r0 < runs.size(); r0 += kHemRunSlots) {
                const uint32_t cnt = (uint32_t)std::min<size_t>(kHemRunSlots, runs.size() - r0);
                HIP_TRY(hipMemcpyAsync(L.runs, runs.data() + r0, cnt * sizeof(HemRun), hipMemcpyHostToDevice, s));
                HIP_TRY(launch_hem_gather(L.sig, L.runs, cnt, L.bsig, s));
            }
            HIP_TRY(launch_hem_partition(L.bsig, nb, kc, L.btmp, k > kc ? L.lbo_c : L.lbo, L.baux, s));
            if (k > kc) HIP_TRY(launch_hem_refine(L.bsig, L.lbo_c, kc, k, L.btmp, L.lbo, s));
        }
        const R* bkeys = k > kc ? L.btmp : L.bsig;  // the batch's signatures in bucket order
        HIP_TRY(hipMemcpyAsync(lbo.data(), L.lbo, (B + 1) * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        const uint32_t b0 = g0 << gshift, Bb = (g1 - g0) << gshift;
        if (lbo[b0] != 0 || lbo[b0 + Bb] != nb) return fail(MPHX_EDEVICE, "batch bucket offsets inconsistent");
        uint64_t mb = 0;
        rc = mphx_batch_layout(&lbo[b0], Bb, gnum, gden, co_l.data(), ro_l.data(), &ord[b0], &mb);
        if (rc) return rc;
        if (mb > bound)
            return fail(MPHX_ENOMEM, "largest bucket %llu exceeds the workspace's bound %llu", (unsigned long long)mb,
                        (unsigned long long)bound);
        for (uint32_t j = 0; j <= Bb; j++) {
            bo[b0 + j] = kbase + lbo[b0 + j];
            co[b0 + j] = cw + co_l[j];
            ro[b0 + j] = rw + ro_l[j];
        }
        HIP_TRY(hipMemcpyAsync(code_off + b0, &co[b0], (Bb + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(rank_off + b0, &ro[b0], (Bb + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(L.order, &ord[b0], Bb * sizeof(uint32_t), hipMemcpyHostToDevice, s));
        {
            Timed tm(PH_OTHER, s);
            rc = batch_enqueue(reinterpret_cast<const uint64_t*>(bkeys), L.lbo + b0, L.order, Bb, mb, seed, gnum,
                               gden, max_tries, code_off + b0, rank_off + b0, codes, rank, L.results + b0, L.batch,
                               L.batch_bytes, &tune, s, kStr);
            if (rc) return rc;
        }
        kbase += nb;
        cw += co_l[Bb];
        rw += ro_l[Bb];
        g0 = g1;
    }
    HIP_TRY(hipMemcpyAsync(bucket_off, bo.data(), (B + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, s));
    return hem_finish(B, L.results, seed, co[B], seeds, s, info);
}

extern "C" {

int mphx_hem_build_u64(const uint64_t* keys, uint64_t n, uint32_t k, uint64_t seed, uint32_t gamma_num,
                       uint32_t gamma_den, uint32_t max_tries, uint64_t* bucket_off, uint64_t* code_off,
                       uint64_t* rank_off, uint64_t* seeds, uint64_t* codes, uint64_t* rank, void* ws,
                       size_t ws_bytes, void* stream, mphx_mphf_info* info)
{
    return hem_build<uint2>(keys, nullptr, nullptr, n, k, seed, gamma_num, gamma_den, max_tries, bucket_off, code_off,
                            rank_off, seeds, codes, rank, ws, ws_bytes, (hipStream_t)stream, info);
}

int mphx_hem_build_str(const uint8_t* bytes, const uint64_t* offs, uint64_t n, uint32_t k, uint64_t seed,
                       uint32_t gamma_num, uint32_t gamma_den, uint32_t max_tries, uint64_t* bucket_off,
                       uint64_t* code_off, uint64_t* rank_off, uint64_t* seeds, uint64_t* codes, uint64_t* rank,
                       void* ws, size_t ws_bytes, void* stream, mphx_mphf_info* info)
{
    return hem_build<uint4>(nullptr, bytes, offs, n, k, seed, gamma_num, gamma_den, max_tries, bucket_off, code_off,
                            rank_off, seeds, codes, rank, ws, ws_bytes, (hipStream_t)stream, info);
}

size_t mphx_hem_host_workspace_bytes(uint64_t n, uint32_t k, uint32_t gamma_num, uint32_t gamma_den, int kind,
                                     uint64_t chunk_keys, uint64_t chunk_bytes, uint64_t batch_keys)
{
    if (kind != MPHX_KEYS_U64 && kind != MPHX_KEYS_STR) return 0;
    if (k < 9 || k > kHemMaxK || gamma_num == 0 || gamma_den == 0 || chunk_keys == 0 || chunk_keys >= 0x7FFFFFFFull ||
        batch_keys == 0 || batch_keys >= 0x7FFFFFFFull || (kind == MPHX_KEYS_STR && chunk_bytes < 512))
        return 0;
    Carve c(nullptr);
    if (kind == MPHX_KEYS_U64) {
        HemHostLayout<uint2> L;
        layout_hem_host(c, kind, n, k, gamma_num, gamma_den, chunk_keys, chunk_bytes, batch_keys, L);
    } else {
        HemHostLayout<uint4> L;
        layout_hem_host(c, kind, n, k, gamma_num, gamma_den, chunk_keys, chunk_bytes, batch_keys, L);
    }
    return c.off;
}

int mphx_hem_build_host_u64(const uint64_t* keys, uint64_t n, uint32_t k, uint64_t seed, uint32_t gamma_num,
                            uint32_t gamma_den, uint32_t max_tries, uint64_t chunk_keys, uint64_t batch_keys,
                            uint64_t* bucket_off, uint64_t* code_off, uint64_t* rank_off, uint64_t* seeds,
                            uint64_t* codes, uint64_t* rank, void* ws, size_t ws_bytes, void* stream,
                            mphx_mphf_info* info)
{
    return hem_host_build<uint2>(keys, nullptr, nullptr, n, k, seed, gamma_num, gamma_den, max_tries,
                          chunk_keys, 0, batch_keys, bucket_off, code_off, rank_off, seeds, codes, rank, ws, ws_bytes,
                          (hipStream_t)stream, info);
}

int mphx_hem_build_host_str(const uint8_t* bytes, const uint64_t* offs, uint64_t n, uint32_t k, uint64_t seed,
                            uint32_t gamma_num, uint32_t gamma_den, uint32_t max_tries, uint64_t chunk_keys,
                            uint64_t chunk_bytes, uint64_t batch_keys, uint64_t* bucket_off, uint64_t* code_off,
                            uint64_t* rank_off, uint64_t* seeds, uint64_t* codes, uint64_t* rank, void* ws,
                            size_t ws_bytes, void* stream, mphx_mphf_info* info)
{
    return hem_host_build<uint4>(nullptr, bytes, offs, n, k, seed, gamma_num, gamma_den, max_tries,
                          chunk_keys, chunk_bytes, batch_keys, bucket_off, code_off, rank_off, seeds, codes, rank, ws,
                          ws_bytes, (hipStream_t)stream, info);
}

int mphx_hem_lookup_u64(const uint64_t* bucket_off, const uint64_t* code_off, const uint64_t* rank_off,
                        const uint64_t* seeds, const uint64_t* codes, const uint64_t* rank, uint32_t k,
                        uint32_t gamma_num, uint32_t gamma_den, uint64_t seed, const uint64_t* keys, uint64_t n,
                        uint64_t* out, void* stream)
{
    g_err.clear();
    if (n == 0) return MPHX_OK;
    if (!bucket_off || !code_off || !rank_off || !seeds || !codes || !rank || !keys || !out || k < 9 || k > kHemMaxK ||
        gamma_num == 0 || gamma_den == 0)
        return fail(MPHX_EINVAL, "null pointer, k outside [9, 20] or bad gamma");
    HemTables t{bucket_off, code_off, rank_off, seeds, codes, rank, k, gamma_num, gamma_den};
    HIP_TRY(launch_hem_lookup_u64(t, seed, keys, n, out, (hipStream_t)stream));
    return MPHX_OK;
}

int mphx_hem_lookup_str(const uint64_t* bucket_off, const uint64_t* code_off, const uint64_t* rank_off,
                        const uint64_t* seeds, const uint64_t* codes, const uint64_t* rank, uint32_t k,
                        uint32_t gamma_num, uint32_t gamma_den, uint64_t seed, const uint8_t* bytes,
                        const uint64_t* offs, uint64_t n, uint64_t* out, void* stream)
{
    g_err.clear();
    if (n == 0) return MPHX_OK;
    if (!bucket_off || !code_off || !rank_off || !seeds || !codes || !rank || !bytes || !offs || !out || k < 9 ||
        k > kHemMaxK || gamma_num == 0 || gamma_den == 0)
        return fail(MPHX_EINVAL, "null pointer, k outside [9, 20] or bad gamma");
    if ((uintptr_t)bytes & 3) return fail(MPHX_EINVAL, "bytes must be 4-byte aligned");
    HemTables t{bucket_off, code_off, rank_off, seeds, codes, rank, k, gamma_num, gamma_den};
    HIP_TRY(launch_hem_lookup_str(t, seed, bytes, offs, n, out, (hipStream_t)stream));
    return MPHX_OK;
}

}  // extern "C"

// ---- streamed build: keys in host memory, one hypergraph of up to 3 * 2^32 vertices ----------
namespace {

struct StreamLayout {
    uint8_t* deg;   // degree bytes, then the code bytes of the assignment
    uint64_t* X;    // XOR packs of the other two endpoints
    uint3* slots;   // the layer area
    uint64_t* stage[2];  // two chunks of keys: one copied in while the other is built from
    uint32_t* bcount;
    void* scan;
    size_t scan_bytes;
    Ctrl* ctrl;
    unsigned long long* cursor;  // layer append cursor, then the three run bounds of the round
};

void layout_stream(Carve& c, uint64_t m, uint64_t chunk_keys, uint64_t layer_slots, StreamLayout& L)
{
    const uint64_t nblocks = (m + 511) / 512;
    L.deg = c.take<uint8_t>((m + 15) & ~15ull);  // whole 16-byte groups for the round scans
    L.X = c.take<uint64_t>(m);
    L.slots = c.take<uint3>(layer_slots);
    L.stage[0] = c.take<uint64_t>(chunk_keys);
    L.stage[1] = c.take<uint64_t>(chunk_keys);
    L.bcount = c.take<uint32_t>(nblocks);
    L.scan_bytes = scan_scratch_bytes(nblocks);
    L.scan = c.take<uint8_t>(L.scan_bytes);
    L.ctrl = c.take<Ctrl>(1);
    L.cursor = c.take<unsigned long long>(4);
}

// P <= 2^32 (part-local ids are 32-bit) and at least one vertex per part
uint64_t stream_part_size(uint64_t n, uint32_t gnum, uint32_t gden)
{
    if (gnum == 0 || gden == 0 || n == 0) return 0;
    const uint64_t P = mphx_part_size(n, gnum, gden);
    return P <= (1ull << 32) ? P : 0;
}

}  // namespace

extern "C" {

size_t mphx_stream_workspace_bytes(uint64_t n, uint32_t gamma_num, uint32_t gamma_den, uint64_t chunk_keys,
                                   uint64_t layer_slots)
{
    const uint64_t P = stream_part_size(n, gamma_num, gamma_den);
    if (!P || chunk_keys == 0 || layer_slots == 0) return 0;
    Carve c(nullptr);
    StreamLayout L;
    layout_stream(c, 3 * P, chunk_keys, layer_slots, L);
    return c.off;
}

int mphx_mphf_build_stream_u64(const uint64_t* keys, uint64_t n, uint64_t seed, uint32_t gamma_num,
                               uint32_t gamma_den, uint32_t max_tries, uint64_t chunk_keys, uint64_t layer_slots,
                               void* host_layers, size_t host_layer_bytes, uint64_t* codes, uint64_t* rank, void* ws,
                               size_t ws_bytes, void* stream, mphx_mphf_info* info)
{
    g_err.clear();
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) return fail(MPHX_EINVAL, "the streamed build needs at least one key");
    if (!keys || !codes || !rank) return fail(MPHX_EINVAL, "null keys or outputs");
    if (max_tries == 0) return fail(MPHX_EINVAL, "max_tries must be >= 1");
    const uint64_t P = stream_part_size(n, gamma_num, gamma_den);
    if (!P) return fail(MPHX_EINVAL, "gamma must be a positive fraction and P = ceil(gamma n / 3) at most 2^32");
    const uint64_t m = 3 * P;
    if (chunk_keys == 0 || layer_slots == 0) return fail(MPHX_EINVAL, "chunk_keys and layer_slots must be positive");
    const bool spill = layer_slots < n;
    if (spill && (!host_layers || host_layer_bytes < 12 * n))
        return fail(MPHX_EINVAL, "layer_slots < n: host_layers must hold 12 n bytes");
    if (!ws || !aligned256(ws)) return fail(MPHX_EINVAL, "workspace must be non-null and 256-byte aligned");
    const size_t need = mphx_stream_workspace_bytes(n, gamma_num, gamma_den, chunk_keys, layer_slots);
    if (ws_bytes < need) return fail(MPHX_ENOMEM, "workspace of %zu bytes, need %zu", ws_bytes, need);
    if (info) {
        memset(info, 0, sizeof *info);
        info->P = P;
        info->m = m;
        info->seed_used = seed;
    }
    Carve c(ws);
    StreamLayout L;
    layout_stream(c, m, chunk_keys, layer_slots, L);
    uint8_t* const hl = static_cast<uint8_t*>(host_layers);

    // Key chunks reach the device on a copy stream of their own, double-buffered, so the
    // transfer of chunk i + 1 overlaps the record build of chunk i: ready[b] says a buffer
    // holds its chunk, freed[b] that its build has read it.
    struct CopyStream {
        hipStream_t cs = nullptr;
        hipEvent_t ready[2] = {nullptr, nullptr}, freed[2] = {nullptr, nullptr};
        ~CopyStream()
        {
            if (cs) {
                (void)hipStreamSynchronize(cs);
                (void)hipStreamDestroy(cs);
            }
            for (hipEvent_t e : {ready[0], ready[1], freed[0], freed[1]})
                if (e) (void)hipEventDestroy(e);
        }
    } cp;
    struct DrainOnExit {
        hipStream_t s;
        ~DrainOnExit() { (void)hipStreamSynchronize(s); }
    } drain{s};
    HIP_TRY(hipStreamCreateWithFlags(&cp.cs, hipStreamNonBlocking));
    for (hipEvent_t* e : {&cp.ready[0], &cp.ready[1], &cp.freed[0], &cp.freed[1]})
        HIP_TRY(hipEventCreateWithFlags(e, hipEventDisableTiming));
    HostStager stager(s);  // host key chunks (and spilled layers) go through its pinned buffers

    // per round: where its runs of hinge parts 0, 1, 2 start, and where it ends (device
    // positions without spilling, host slot positions with)
    std::vector<uint64_t> bounds;
    uint64_t peeled = 0;
    uint32_t rounds = 0;
    bool done = false;
    uint32_t t = 0;
    for (t = 0; t < max_tries && !done; t++) {
        const uint64_t sd = seed + t;
        HIP_TRY(launch_zero(L.deg, (m + 15) & ~15ull, s));
        HIP_TRY(launch_zero(L.X, m * sizeof(uint64_t), s));
        HIP_TRY(launch_zero(L.ctrl, sizeof(Ctrl), s));
        {
            Timed tm(PH_BUILD, s);
            stager.use_stream(cp.cs);
            HIP_TRY(hipEventRecord(cp.freed[0], s));
            HIP_TRY(hipEventRecord(cp.freed[1], s));
            for (uint64_t c0 = 0, i = 0; c0 < n; c0 += chunk_keys, i++) {
                const uint64_t cn = std::min(chunk_keys, n - c0);
                const int b = (int)(i & 1);
                HIP_TRY(hipStreamWaitEvent(cp.cs, cp.freed[b], 0));
                HIP_TRY(stager.copy(L.stage[b], keys + c0, cn * sizeof(uint64_t)));
                HIP_TRY(hipEventRecord(cp.ready[b], cp.cs));
                HIP_TRY(hipStreamWaitEvent(s, cp.ready[b], 0));
                HIP_TRY(launch_st_build(L.stage[b], cn, sd, P, L.deg, L.X, L.ctrl, s));
                HIP_TRY(hipEventRecord(cp.freed[b], s));
            }
            stager.use_stream(s);  // the build waited for every copy; later copies go on s
        }
        Ctrl h;
        int rc = read_ctrl(L.ctrl, h, s);
        if (rc) return rc;
        if (h.err & kErrDegree) {
            if (info) { info->tries = t + 1; info->seed_used = sd; }
            return fail(MPHX_ERANGE, "a vertex has degree above %u", MPHX_MAX_DEGREE);
        }
        bounds.clear();
        peeled = 0;
        uint64_t at = 0;  // device position of the next layer
        for (rounds = 0;; rounds++) {
            unsigned long long b[4];
            b[0] = spill ? 0 : at;
            HIP_TRY(hipMemcpyAsync(L.cursor, &b[0], sizeof b[0], hipMemcpyHostToDevice, s));
            {
                Timed tm(PH_FRONTIER, s);
                for (uint32_t k = 0; k < 3; k++) {
                    HIP_TRY(launch_st_claim(L.deg, L.X, P, k, L.slots, layer_slots, L.cursor, L.ctrl, s));
                    HIP_TRY(hipMemcpyAsync(L.cursor + 1 + k, L.cursor, sizeof b[0], hipMemcpyDeviceToDevice, s));
                }
            }
            HIP_TRY(hipMemcpyAsync(b + 1, L.cursor + 1, 3 * sizeof b[0], hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            if (b[3] > layer_slots)  // slots past the area were counted, not stored
                return fail(MPHX_ENOMEM, "round %u: the layer exceeds the layer area of %llu slots", rounds,
                            (unsigned long long)layer_slots);
            const uint64_t cnt = b[3] - b[0];
            if (cnt == 0) break;
            {
                Timed tm(PH_APPLY, s);
                HIP_TRY(launch_st_apply(L.slots, b[0], b[1], b[2], b[3], P, L.deg, L.X, s));
            }
            if (spill) {  // the round's slots to host memory; the area is reused by the next round
                Timed tm(PH_OTHER, s);
                HIP_TRY(stager.copy_out(hl + 12 * peeled, L.slots, 12 * cnt));
                for (int q = 0; q < 4; q++) bounds.push_back(peeled + (b[q] - b[0]));
            } else {
                for (int q = 0; q < 4; q++) bounds.push_back(b[q]);
                at = b[3];
            }
            if (info && rounds == 0) info->layer0 = cnt;
            peeled += cnt;
        }
        if (info) {
            info->tries = t + 1;
            info->seed_used = sd;
            info->n_rounds = rounds;
            info->n_core = n - peeled;
        }
        done = peeled == n;
    }
    if (!done)
        return fail(MPHX_ECORE, "2-core of %llu edges after %u tries", (unsigned long long)(n - peeled), max_tries);

    // assignment, last layer first (Section 4.3), the codes in the degree bytes (all zero now)
    uint8_t* code8 = L.deg;
    HIP_TRY(launch_zero(code8, (m + 3) & ~3ull, s));
    for (int64_t r = (int64_t)rounds - 1; r >= 0; r--) {
        const uint64_t* b = &bounds[4 * r];
        uint64_t lo = b[0];
        if (spill) {
            Timed tm(PH_OTHER, s);
            HIP_TRY(stager.copy(L.slots, hl + 12 * b[0], 12 * (b[3] - b[0])));
            lo = 0;
        }
        Timed tm(PH_ASSIGN, s);
        HIP_TRY(launch_st_assign(L.slots, lo, lo + (b[1] - b[0]), lo + (b[2] - b[0]), lo + (b[3] - b[0]), P, code8, s));
    }
    {
        Timed tm(PH_RANK, s);
        HIP_TRY(launch_pack_count(code8, m, codes, L.bcount, s));
        const uint64_t nblocks = (m + 511) / 512;
        HIP_TRY(launch_scan_u32_to_u64(L.bcount, nblocks, rank, nblocks, L.scan, L.scan_bytes, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    g_timers.harvest();
    return MPHX_OK;
}

int mphx_mphf_lookup_wide_u64(const uint64_t* codes, const uint64_t* rank, uint64_t P, uint64_t seed,
                              const uint64_t* keys, uint64_t n, uint64_t* out, void* stream)
{
    g_err.clear();
    if (n == 0) return MPHX_OK;
    if (!codes || !rank || !keys || !out || P == 0 || P > (1ull << 32)) return fail(MPHX_EINVAL, "bad arguments");
    HIP_TRY(launch_st_lookup(codes, rank, P, seed, keys, n, out, nullptr, n, nullptr, (hipStream_t)stream));
    return MPHX_OK;
}

size_t mphx_check_stream_workspace_bytes(uint64_t n, uint64_t chunk_keys)
{
    if (chunk_keys == 0) return 0;
    Carve c(nullptr);
    c.take<Ctrl>(1);
    c.take<uint32_t>((n + 31) / 32);
    c.take<uint64_t>(chunk_keys);
    return c.off;
}

int mphx_check_stream_u64(const uint64_t* codes, const uint64_t* rank, uint64_t P, uint64_t seed,
                          const uint64_t* keys, uint64_t n, uint64_t chunk_keys, void* ws, size_t ws_bytes,
                          void* stream, uint64_t* n_bad)
{
    g_err.clear();
    hipStream_t s = (hipStream_t)stream;
    if (!codes || !rank || (!keys && n) || !n_bad || P == 0 || P > (1ull << 32) || chunk_keys == 0)
        return fail(MPHX_EINVAL, "bad arguments");
    if (!ws || !aligned256(ws)) return fail(MPHX_EINVAL, "workspace must be non-null and 256-byte aligned");
    if (ws_bytes < mphx_check_stream_workspace_bytes(n, chunk_keys)) return fail(MPHX_ENOMEM, "workspace too small");
    Carve c(ws);
    Ctrl* ctrl = c.take<Ctrl>(1);
    uint32_t* bitmap = c.take<uint32_t>((n + 31) / 32);
    uint64_t* stage = c.take<uint64_t>(chunk_keys);
    struct DrainOnExit {
        hipStream_t s;
        ~DrainOnExit() { (void)hipStreamSynchronize(s); }
    } drain{s};
    HostStager stager(s);
    HIP_TRY(launch_zero(ctrl, sizeof(Ctrl), s));
    HIP_TRY(launch_zero(bitmap, ((n + 31) / 32) * sizeof(uint32_t), s));
    for (uint64_t c0 = 0; c0 < n; c0 += chunk_keys) {
        const uint64_t cn = std::min(chunk_keys, n - c0);
        HIP_TRY(stager.copy(stage, keys + c0, cn * sizeof(uint64_t)));
        HIP_TRY(launch_st_lookup(codes, rank, P, seed, stage, cn, nullptr, bitmap, n, ctrl, s));
    }
    Ctrl h;
    int rc = read_ctrl(ctrl, h, s);
    if (rc) return rc;
    *n_bad = h.aux;
    return MPHX_OK;
}

}  // extern "C"

