// Build server: continuous admission of MWHC builds of mixed sizes under an HBM budget.
//
// The server owns one device pool of `budget` bytes and `slots` worker threads, each with its
// own HIP stream (default priority).  Requests wait in arrival order; whenever a worker is idle
// it admits the first waiting request whose workspace fits in the pool (first fit), so a later
// small request may pass a large one that does not fit yet -- but only a bounded number of
// times, after which the head of the queue blocks admission until it fits.  Admitted builds run
// concurrently on their streams and overlap on the device; each frees its workspace when done.
// Keys and outputs stay in caller-owned device memory; a build writes exactly what
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

constexpr uint32_t kMaxSkips = 8;  // times the queue head may be passed by later requests

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

    // Take the next admissible job (called with mu held); false if none fits now.
    bool admit(Job& out, size_t& off)
    {
        for (size_t i = 0; i < pending.size(); i++) {
            if (alloc.alloc(pending[i].ws_bytes, off)) {
                out = pending[i];
                pending.erase(pending.begin() + (long)i);
                return true;
            }
            if (i == 0 && ++pending[0].skipped > kMaxSkips)
                return false;  // the head has waited long enough: no more backfill
        }
        return false;
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

int mphx_server_create(int device, size_t hbm_budget, uint32_t slots, mphx_server** out)
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
    for (uint32_t i = 0; i < slots; i++)
        s->workers.emplace_back([s] { s->worker(); });
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
    if (((j.ws_bytes + 255) & ~(size_t)255) > s->budget) {
        mphx_request_result r{};
        r.status = MPHX_ENOMEM;
        r.t_submit = r.t_start = r.t_done = j.t_submit;
        s->done[j.ticket] = r;  // can never fit: fails at once instead of waiting forever
        s->cv_done.notify_all();
        return MPHX_OK;
    }
    s->pending.push_back(j);
    s->cv_work.notify_one();
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
    st->pending = (uint32_t)s->pending.size();
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
    }
    s->cv_work.notify_all();
    for (auto& t : s->workers) t.join();
    (void)hipSetDevice(s->device);
    (void)hipFree(s->pool);
    delete s;
    return MPHX_OK;
}

}  // extern "C"
