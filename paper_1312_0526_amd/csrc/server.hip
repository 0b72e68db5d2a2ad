// Build server: continuous admission of MWHC builds of mixed sizes under an HBM budget.
//
// The server owns one device pool of `budget` bytes and `slots` worker threads, each with its
// own HIP stream (default priority).  Requests wait in arrival order; whenever a worker is idle
// it admits the first waiting request whose workspace fits in the pool (first fit), so a later
// small request may pass a large one that does not fit yet -- but only a bounded number of
// times, after which the head of the queue blocks admission until it fits.  A request whose
// workspace exceeds what the pool can ever give it (the budget less the lane's reservation)
// fails at submission, so the head always fits once the running builds are done.  Admitted
// builds run concurrently on their streams and overlap on the device; each frees its workspace
// when done.  Destroying the server cancels the requests not admitted yet.
//
// Requests of at most `batch_max_keys` keys take a separate lane: one more worker gathers every
// such request waiting at that moment (same gamma and try limit, at most kLaneMax) and builds
// them all in one persistent batched launch, from a workspace reserved in the pool when the
// server starts.  Requests that arrive meanwhile form the next batch.
//
// Keys and outputs stay in caller-owned device memory; every build writes exactly what
// mphx_mphf_build_{u64,str} writes for the same request alone.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "launch.h"
#include "mphx.h"

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, cap) with 256-byte granularity.
struct PoolAlloc {
    size_t cap = 0;
    std::map<size_t, size_t> free_;  // offset -> size
    void init(size_t c)
    {
        cap = c & ~(size_t)255;
        free_.clear();
        if (cap) free_[0] = cap;
    }
    bool alloc(size_t bytes, size_t& off)
    {
        bytes = (bytes + 255) & ~(size_t)255;
        if (bytes == 0) bytes = 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                off = it->first;
                size_t rest = it->second - bytes;
                free_.erase(it);
                if (rest) free_[off + bytes] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = (bytes + 255) & ~(size_t)255;
        if (bytes == 0) bytes = 256;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Job {
    uint64_t ticket;
    mphx_request req;
    double t_submit;
    size_t ws_bytes;
    uint32_t skipped = 0;
};

constexpr uint32_t kMaxSkips = 8;   // times the queue head may be passed by later requests
constexpr uint32_t kLaneMax = 4096; // requests per batched launch
constexpr uint32_t kLaneGrid = 128; // workgroups of the batched launch

}  // namespace

struct mphx_server {
    int device = 0;
    size_t budget = 0;
    uint8_t* pool = nullptr;
    PoolAlloc alloc;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Job> pending;
    std::unordered_map<uint64_t, mphx_request_result> done;
    std::unordered_map<uint64_t, bool> known;
    std::vector<std::thread> workers;
    bool stopping = false;
    uint64_t next_ticket = 1;
    uint32_t running = 0;
    size_t in_use = 0, peak_in_use = 0;
    size_t job_cap = 0;  // largest workspace a plain request can ever be given

    // batching lane
    uint64_t lane_max = 0;                  // 0 = no lane
    std::deque<Job> lane_pending;
    uint8_t* lane_ws = nullptr;              // slots of the batched launch
    size_t lane_ws_bytes = 0;
    mphx_bucket* lane_descs = nullptr;       // device descriptors
    mphx_bucket_result* lane_results = nullptr;
    uint64_t lane_batches = 0;
    mphx_batch_tuning lane_tuning{1024, kLaneGrid, 0, 0};

    bool to_lane(const mphx_request& q) const { return lane_max && q.n <= lane_max; }

    void lane_worker()
    {
        (void)hipSetDevice(device);
        hipStream_t st = nullptr;
        (void)hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        std::vector<Job> batch;
        std::vector<mphx_bucket> hd;
        std::vector<mphx_bucket_result> hr;
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            while (lane_pending.empty() && !stopping)
                cv_work.wait(lk);
            if (lane_pending.empty() && stopping) break;
            const mphx_request& h = lane_pending.front().req;
            batch.clear();
            for (auto it = lane_pending.begin(); it != lane_pending.end() && batch.size() < kLaneMax;) {
                const mphx_request& q = it->req;
                if (q.gamma_num == h.gamma_num && q.gamma_den == h.gamma_den && q.max_tries == h.max_tries) {
                    batch.push_back(*it);
                    it = lane_pending.erase(it);
                } else {
                    ++it;
                }
            }
            running++;
            lk.unlock();

            std::sort(batch.begin(), batch.end(), [](const Job& x, const Job& y) { return x.req.n > y.req.n; });
            const uint32_t B = (uint32_t)batch.size();
            hd.resize(B);
            hr.assign(B, mphx_bucket_result{});
            uint64_t mx = 0;
            for (uint32_t i = 0; i < B; i++) {
                const mphx_request& q = batch[i].req;
                hd[i] = mphx_bucket{q.key_kind == MPHX_KEYS_U64 ? q.keys : nullptr,
                                    q.key_kind == MPHX_KEYS_U64 ? nullptr : q.bytes,
                                    q.key_kind == MPHX_KEYS_U64 ? nullptr : q.offs,
                                    q.n, q.seed, q.codes, q.rank, lane_results + i};
                mx = std::max(mx, q.n);
            }
            const double t_start = now_s();
            int status = MPHX_OK;
            if (hipMemcpyAsync(lane_descs, hd.data(), B * sizeof(mphx_bucket), hipMemcpyHostToDevice, st) !=
                hipSuccess)
                status = MPHX_EDEVICE;
            if (status == MPHX_OK)
                status = mphx_build_batch(lane_descs, B, nullptr, mx, batch[0].req.gamma_num, batch[0].req.gamma_den,
                                          batch[0].req.max_tries, lane_ws, lane_ws_bytes, &lane_tuning, st);
            if (status == MPHX_OK &&
                (hipMemcpyAsync(hr.data(), lane_results, B * sizeof(mphx_bucket_result), hipMemcpyDeviceToHost, st) !=
                     hipSuccess ||
                 hipStreamSynchronize(st) != hipSuccess))
                status = MPHX_EDEVICE;
            const double t_done = now_s();

            lk.lock();
            for (uint32_t i = 0; i < B; i++) {
                const mphx_request& q = batch[i].req;
                mphx_request_result r{};
                r.status = status == MPHX_OK ? hr[i].status : status;
                r.tries = hr[i].tries;
                r.n_rounds = hr[i].n_rounds;
                r.seed_used = hr[i].seed_used;
                r.P = mphx_part_size(q.n, q.gamma_num, q.gamma_den);
                r.m = 3 * r.P;
                r.t_submit = batch[i].t_submit;
                r.t_start = t_start;
                r.t_done = t_done;
                done[batch[i].ticket] = r;
            }
            lane_batches++;
            running--;
            cv_done.notify_all();
        }
        lk.unlock();
        (void)hipStreamDestroy(st);
    }

    // Take the next admissible job (called with mu held); false if none fits now.  A later
    // job admitted while the head does not fit counts as one pass of the head; once the head
    // has been passed kMaxSkips times, nothing behind it is admitted before it.
    bool admit(Job& out, size_t& off)
    {
        for (size_t i = 0; i < pending.size(); i++) {
            if (i > 0 && pending[0].skipped >= kMaxSkips)
                return false;
            if (alloc.alloc(pending[i].ws_bytes, off)) {
                if (i > 0) pending[0].skipped++;
                out = pending[i];
                pending.erase(pending.begin() + (long)i);
                return true;
            }
        }
        return false;
    }

    // Complete every request not admitted yet with MPHX_ECANCELED (called with mu held).
    void cancel_pending()
    {
        const double t = now_s();
        for (std::deque<Job>* q : {&pending, &lane_pending}) {
            for (const Job& j : *q) {
                mphx_request_result r{};
                r.status = MPHX_ECANCELED;
                r.P = mphx_part_size(j.req.n, j.req.gamma_num ? j.req.gamma_num : 1,
                                     j.req.gamma_den ? j.req.gamma_den : 1);
                r.m = 3 * r.P;
                r.t_submit = j.t_submit;
                r.t_start = r.t_done = t;
                done[j.ticket] = r;
            }
            q->clear();
        }
        cv_done.notify_all();
    }

    void worker()
    {
        (void)hipSetDevice(device);
        hipStream_t st = nullptr;
        (void)hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            Job job{};
            size_t off = 0;
            bool got = false;
            for (;;) {
                if (!pending.empty() && admit(job, off)) {
                    got = true;
                    break;
                }
                if (stopping && pending.empty()) break;
                cv_work.wait(lk);
            }
            if (!got) break;
            running++;
            in_use += job.ws_bytes;
            peak_in_use = std::max(peak_in_use, in_use);
            lk.unlock();

            mphx_request_result r{};
            r.t_submit = job.t_submit;
            r.t_start = now_s();
            mphx_mphf_info info{};
            const mphx_request& q = job.req;
            if (q.key_kind == MPHX_KEYS_U64)
                r.status = mphx_mphf_build_u64(q.keys, q.n, q.seed, q.gamma_num, q.gamma_den, q.max_tries, q.codes,
                                               q.rank, pool + off, job.ws_bytes, st, &info);
            else
                r.status = mphx_mphf_build_str(q.bytes, q.offs, q.n, q.seed, q.gamma_num, q.gamma_den, q.max_tries,
                                               q.codes, q.rank, pool + off, job.ws_bytes, st, &info);
            r.t_done = now_s();
            r.tries = info.tries;
            r.n_rounds = info.n_rounds;
            r.seed_used = info.seed_used;
            r.P = info.P;
            r.m = info.m;

            lk.lock();
            alloc.release(off, job.ws_bytes);
            in_use -= job.ws_bytes;
            running--;
            done[job.ticket] = r;
            cv_done.notify_all();
            cv_work.notify_all();
        }
        lk.unlock();
        (void)hipStreamDestroy(st);
    }
};

extern "C" {

int mphx_server_create(int device, size_t hbm_budget, uint32_t slots, uint64_t batch_max_keys, mphx_server** out)
{
    if (!out || slots == 0 || slots > 64 || hbm_budget < 256) return MPHX_EINVAL;
    *out = nullptr;
    if (hipSetDevice(device) != hipSuccess) return MPHX_EDEVICE;
    auto* s = new (std::nothrow) mphx_server();
    if (!s) return MPHX_ENOMEM;
    s->device = device;
    s->budget = hbm_budget & ~(size_t)255;
    if (hipMalloc((void**)&s->pool, s->budget) != hipSuccess) {
        delete s;
        return MPHX_ENOMEM;
    }
    s->alloc.init(s->budget);
    if (batch_max_keys) {
        // reserve the lane's workspace (sized for batch_max_keys keys at gamma 1.23),
        // descriptors and results; without room for it the server has no lane
        size_t ws = mphx_batch_desc_workspace_bytes(batch_max_keys, 123, 100, &s->lane_tuning);
        size_t extra = (size_t)kLaneMax * (sizeof(mphx_bucket) + sizeof(mphx_bucket_result)) + 512;
        size_t off = 0;
        if (ws && ws + extra < s->budget / 2 && s->alloc.alloc(ws + extra, off)) {
            s->lane_max = batch_max_keys;
            s->lane_ws = s->pool + off;
            s->lane_ws_bytes = ws;
            s->lane_descs = reinterpret_cast<mphx_bucket*>(s->pool + off + ((ws + 255) & ~(size_t)255));
            s->lane_results = reinterpret_cast<mphx_bucket_result*>(reinterpret_cast<uint8_t*>(s->lane_descs) +
                                                                    (size_t)kLaneMax * sizeof(mphx_bucket));
            s->in_use += ws + extra;
        }
    }
    // the lane's reservation sits at the pool's start: the rest is one free range
    s->job_cap = s->budget - s->in_use;
    for (uint32_t i = 0; i < slots; i++)
        s->workers.emplace_back([s] { s->worker(); });
    if (s->lane_max)
        s->workers.emplace_back([s] { s->lane_worker(); });
    *out = s;
    return MPHX_OK;
}

int mphx_server_submit(mphx_server* s, const mphx_request* req, uint64_t* ticket)
{
    if (!s || !req || !ticket) return MPHX_EINVAL;
    if (req->key_kind != MPHX_KEYS_U64 && req->key_kind != MPHX_KEYS_STR) return MPHX_EINVAL;
    Job j;
    j.req = *req;
    j.t_submit = now_s();
    j.ws_bytes = mphx_mphf_workspace_bytes(req->n, req->gamma_num ? req->gamma_num : 1,
                                           req->gamma_den ? req->gamma_den : 1, req->key_kind);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) return MPHX_EINVAL;
    j.ticket = s->next_ticket++;
    *ticket = j.ticket;
    s->known[j.ticket] = true;
    auto fail_now = [&](int status) {
        mphx_request_result r{};
        r.status = status;
        r.t_submit = r.t_start = r.t_done = j.t_submit;
        s->done[j.ticket] = r;
        s->cv_done.notify_all();
        return MPHX_OK;
    };
    const size_t ws_al = (j.ws_bytes + 255) & ~(size_t)255;
    if (s->to_lane(j.req)) {
        const mphx_request& q = j.req;
        // only if the request's own slots (at its gamma) fit the lane's reserved workspace
        size_t need = q.gamma_num && q.gamma_den && q.max_tries
                          ? mphx_batch_desc_workspace_bytes(q.n, q.gamma_num, q.gamma_den, &s->lane_tuning)
                          : 0;
        if (need && need <= s->lane_ws_bytes && (q.key_kind == MPHX_KEYS_U64 || ((uintptr_t)q.bytes & 3) == 0)) {
            s->lane_pending.push_back(j);
            s->cv_work.notify_all();
            return MPHX_OK;
        }
    }
    // beyond what the pool can ever give a plain build: fails at once instead of waiting forever
    if (ws_al > s->job_cap) return fail_now(MPHX_ENOMEM);
    s->pending.push_back(j);
    s->cv_work.notify_all();
    return MPHX_OK;
}

int mphx_server_poll(mphx_server* s, uint64_t ticket, mphx_request_result* res)
{
    if (!s) return MPHX_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->known.count(ticket)) return MPHX_EINVAL;
    auto it = s->done.find(ticket);
    if (it == s->done.end()) return 1;
    if (res) *res = it->second;
    return MPHX_OK;
}

int mphx_server_wait(mphx_server* s, uint64_t ticket, mphx_request_result* res)
{
    if (!s) return MPHX_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    if (!s->known.count(ticket)) return MPHX_EINVAL;
    s->cv_done.wait(lk, [&] { return s->done.count(ticket) > 0; });
    if (res) *res = s->done[ticket];
    return MPHX_OK;
}

int mphx_server_stats(mphx_server* s, mphx_server_stats_t* st)
{
    if (!s || !st) return MPHX_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    st->pending = (uint32_t)(s->pending.size() + s->lane_pending.size());
    st->running = s->running;
    st->completed = (uint64_t)s->done.size();
    st->budget = s->budget;
    st->in_use = s->in_use;
    st->peak_in_use = s->peak_in_use;
    return MPHX_OK;
}

double mphx_server_clock(void) { return now_s(); }

int mphx_server_destroy(mphx_server* s)
{
    if (!s) return MPHX_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
        s->cancel_pending();
    }
    s->cv_work.notify_all();
    for (auto& t : s->workers) t.join();
    (void)hipSetDevice(s->device);
    (void)hipFree(s->pool);
    delete s;
    return MPHX_OK;
}

}  // extern "C"
