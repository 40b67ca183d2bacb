// Serving front end: continuous batching of independent eigenproblems.
//
// A server runs `max_inflight` worker slots on one GPU.  Each slot owns a
// solver handle and a stream; an idle slot forms the next batch from the
// oldest queued request and the later queued requests of the same precision
// that fit, runs it as one pass of the solver pipeline, publishes every
// request's result and frees its memory.  Requests that arrive while batches
// are on the GPU are admitted by the next slot that frees up, so batches of
// either precision overlap on the device.
//
// Memory.  The server owns one device arena of exactly the HBM budget,
// allocated at creation.  A batch runs on a region of it sized by the
// workspace query (mr3_workspace_bytes_batched: the whole level's
// eigenvectors in one round, clusters of two levels at once), so the solves
// allocate nothing and device use never exceeds the budget.  When the oldest
// request does not fit the largest free region it waits for a batch to end;
// when nothing else runs it gets the whole arena, which is at least its
// minimum work region (checked at submission), and runs with the tree walked
// in smaller groups.
//
// Eigenpairs of different matrices are independent (Section 3.1), so a batch
// gives each request what a solve of it alone gives, to the gates.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/mr3.h"
#include "mr3_internal.h"

namespace {

double steady_ms() {
    return std::chrono::duration<double, std::milli>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

int64_t wanted(const mr3_request& r) {
    if (r.range.range == MR3_RANGE_INDEX) return std::max<int64_t>(r.range.iu - r.range.il + 1, 0);
    return r.n;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// First-fit allocator of byte ranges of [0, cap) (the device arena), with
// coalescing of neighbouring free ranges.
struct ArenaMap {
    size_t cap = 0;
    std::map<size_t, size_t> free_;  // offset -> length
    void init(size_t c) {
        cap = c;
        free_.clear();
        if (c) free_[0] = c;
    }
    size_t largest() const {
        size_t m = 0;
        for (const auto& f : free_) m = std::max(m, f.second);
        return m;
    }
    bool take(size_t bytes, size_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
        return false;
    }
    void give(size_t off, size_t bytes) {
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

struct Entry {
    mr3_request r;
    size_t est = 0;       // full-speed work region of the request alone
    hipEvent_t ready = nullptr;  // recorded on the request's stream at submission
    bool done = false;
    bool claimed = false;  // a waiter has taken the ticket
    mr3_result res{};
};

}  // namespace

struct mr3_server_s {
    mr3_handle h = nullptr;   // the caller's handle (slot 0)
    std::vector<mr3_handle> owned;  // handles of the other slots
    int device = 0;
    mr3_executor_fn fn = nullptr;
    void* ctx = nullptr;
    size_t budget = 0;
    int max_batch = 1;
    int slots = 1;
    char* arena = nullptr;    // device memory (not with an executor)
    ArenaMap amap;
    std::vector<hipStream_t> streams;
    std::vector<mr3_handle> handles;
    std::vector<std::thread> workers;
    std::vector<hipEvent_t> event_pool;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Entry>> entries;
    uint64_t next_ticket = 1;
    int64_t next_batch = 0;
    int inflight = 0;
    bool stop = false;

    // Work region of a batch: the workspace query for the batch (or, with an
    // executor, the sum of the requests' estimates).
    size_t batch_bytes(const std::vector<mr3_request>& reqs) const {
        if (fn) {
            size_t t = 0;
            for (const auto& r : reqs) t += align256(mr3_request_bytes(r.n, wanted(r), r.precision));
            return t;
        }
        std::vector<int64_t> n;
        std::vector<mr3_range_desc> rg;
        for (const auto& r : reqs) {
            n.push_back(r.n);
            rg.push_back(r.range);
        }
        return align256(mr3_workspace_bytes_batched(h, (int64_t)reqs.size(), reqs[0].precision,
                                                    n.data(), rg.data()));
    }

    // run one batch on slot w; fills m and returns the status
    int execute(int w, std::vector<mr3_request>& reqs, std::vector<int64_t>& m, void* region,
                size_t region_bytes) {
        const int64_t c = (int64_t)reqs.size();
        if (fn) return fn(ctx, c, reqs.data(), m.data());
        std::vector<int64_t> n((size_t)c), ldz((size_t)c);
        std::vector<const void*> d((size_t)c), e((size_t)c);
        std::vector<void*> W((size_t)c), Z((size_t)c);
        std::vector<mr3_range_desc> rg((size_t)c);
        for (int64_t p = 0; p < c; ++p) {
            const mr3_request& r = reqs[p];
            n[p] = r.n;
            d[p] = r.d;
            e[p] = r.e ? r.e : r.d;
            W[p] = r.W;
            Z[p] = r.Z;
            ldz[p] = r.Z ? r.ldz : 1;
            rg[p] = r.range;
        }
        int rc = mr3_solve_ptrs(handles[w], reqs[0].precision, c, n.data(), d.data(), e.data(),
                                rg.data(), m.data(), W.data(), Z.data(), ldz.data(), region,
                                region_bytes, streams[w]);
        const hipError_t se = hipStreamSynchronize(streams[w]);
        if (rc == MR3_OK && se != hipSuccess) rc = MR3_ERR_HIP;
        return rc;
    }

    void run(int w) {
        if (!fn) (void)hipSetDevice(device);
        for (;;) {
            std::vector<uint64_t> batch;
            std::vector<mr3_request> reqs;
            std::vector<hipEvent_t> evs;
            size_t off = 0, bytes = 0;
            int64_t bid = 0;
            {
                std::unique_lock<std::mutex> lk(mu);
                for (;;) {
                    if (queue.empty()) {
                        if (stop) return;
                        cv_work.wait(lk);
                        continue;
                    }
                    Entry& head = *entries[queue.front()];
                    const size_t hole = amap.largest();
                    if (head.est <= hole) {
                        // the oldest request and later ones of its precision
                        // whose estimates fit the largest free region
                        const int prec = head.r.precision;
                        size_t sum = 0;
                        std::vector<uint64_t> cand;
                        for (uint64_t t : queue) {
                            if ((int)cand.size() >= max_batch) break;
                            const Entry& en = *entries[t];
                            if (en.r.precision != prec || sum + align256(en.est) > hole) continue;
                            sum += align256(en.est);
                            cand.push_back(t);
                        }
                        for (;;) {
                            reqs.clear();
                            for (uint64_t t : cand) reqs.push_back(entries[t]->r);
                            bytes = batch_bytes(reqs);
                            if (bytes <= hole || cand.size() == 1) break;
                            cand.pop_back();
                        }
                        bytes = std::min(bytes, hole);
                        batch = cand;
                    } else if (inflight == 0) {
                        // nothing else runs: the whole arena, at least the
                        // request's minimum region (checked at submission)
                        batch = {queue.front()};
                        reqs = {head.r};
                        bytes = hole;
                    } else {
                        cv_work.wait(lk);  // a running batch frees memory
                        continue;
                    }
                    if (!amap.take(bytes, &off)) {  // cannot happen: bytes <= largest hole
                        batch.clear();
                        reqs.clear();
                        cv_work.wait(lk);
                        continue;
                    }
                    break;
                }
                for (uint64_t t : batch) {
                    queue.erase(std::find(queue.begin(), queue.end(), t));
                    evs.push_back(entries[t]->ready);
                }
                ++inflight;
                bid = next_batch++;
            }
            // the solve reads the inputs after the work that produced them
            for (hipEvent_t ev : evs)
                if (ev) (void)hipStreamWaitEvent(streams[w], ev, 0);
            const double t0 = steady_ms();
            std::vector<int64_t> m(batch.size(), 0);
            std::vector<int> status(batch.size(), 0);
            void* region = arena ? arena + off : nullptr;
            int rc = execute(w, reqs, m, region, bytes);
            if (rc != MR3_OK && batch.size() > 1) {
                // isolate the failing request(s): solve each alone
                for (size_t i = 0; i < batch.size(); ++i) {
                    std::vector<mr3_request> one{reqs[i]};
                    std::vector<int64_t> m1(1, 0);
                    status[i] = execute(w, one, m1, region, bytes);
                    m[i] = m1[0];
                }
            } else {
                std::fill(status.begin(), status.end(), rc);
            }
            const double t1 = steady_ms();
            {
                std::lock_guard<std::mutex> lk(mu);
                amap.give(off, bytes);
                --inflight;
                for (size_t i = 0; i < batch.size(); ++i) {
                    Entry& en = *entries[batch[i]];
                    en.res.status = status[i];
                    en.res.m = m[i];
                    en.res.start_ms = t0;
                    en.res.done_ms = t1;
                    en.res.batch_id = bid;
                    en.res.batch_size = (int)batch.size();
                    en.res.slot = w;
                    en.done = true;
                    if (en.ready) {
                        event_pool.push_back(en.ready);
                        en.ready = nullptr;
                    }
                }
            }
            cv_done.notify_all();
            cv_work.notify_all();  // memory and a slot are free
        }
    }

    void release() {
        for (hipEvent_t ev : event_pool) (void)hipEventDestroy(ev);
        event_pool.clear();
        for (hipStream_t s : streams)
            if (s) (void)hipStreamDestroy(s);
        streams.clear();
        if (arena) (void)hipFree(arena);
        arena = nullptr;
        for (mr3_handle x : owned) (void)mr3_destroy(x);
        owned.clear();
    }
};

namespace {

int validate(const mr3_request* r) {
    if (!r) return -2;
    if (r->precision != 32 && r->precision != 64) return -2;
    if (r->n < 0) return -2;
    if (r->n > 0 && (!r->d || !r->W)) return -2;
    if (r->n > 1 && !r->e) return -2;
    const mr3_range_desc& g = r->range;
    if (g.range < 0 || g.range > 2) return -2;
    if (g.range == MR3_RANGE_VALUE && !(g.vl < g.vu)) return -2;
    if (g.range == MR3_RANGE_INDEX && (g.il < 1 || g.iu > r->n || g.il > g.iu)) return -2;
    if (r->Z && r->ldz < std::max<int64_t>(1, r->n)) return -2;
    return 0;
}

int create_common(mr3_server* s, mr3_handle h, mr3_executor_fn fn, void* ctx, size_t budget,
                  int max_batch, int max_inflight) {
    if (!s) return -1;
    if (budget == 0) return -3;
    if (max_batch < 1) return -4;
    if (max_inflight < 1 || max_inflight > 8) return -5;
    mr3_server_s* v = new mr3_server_s();
    v->h = h;
    v->fn = fn;
    v->ctx = ctx;
    v->budget = budget & ~(size_t)255;
    v->max_batch = max_batch;
    v->slots = max_inflight;
    v->amap.init(v->budget);
    v->streams.assign((size_t)max_inflight, nullptr);
    v->handles.assign((size_t)max_inflight, h);
    if (!fn) {
        v->device = mr3_handle_device(h);
        bool ok = hipSetDevice(v->device) == hipSuccess &&
                  hipMalloc(reinterpret_cast<void**>(&v->arena), v->budget) == hipSuccess;
        for (int w = 0; ok && w < max_inflight; ++w) {
            ok = hipStreamCreateWithFlags(&v->streams[w], hipStreamNonBlocking) == hipSuccess;
            if (ok && w > 0) {
                mr3_handle x = nullptr;
                ok = mr3_create(&x, v->device) == MR3_OK;
                if (ok) {
                    mr3_handle_copy_params(x, h);
                    v->owned.push_back(x);
                    v->handles[w] = x;
                }
            }
        }
        if (!ok) {
            v->release();
            delete v;
            return MR3_ERR_HIP;
        }
    }
    for (int w = 0; w < max_inflight; ++w) v->workers.emplace_back([v, w] { v->run(w); });
    *s = v;
    return MR3_OK;
}

}  // namespace

extern "C" {

size_t mr3_request_bytes(int64_t n, int64_t k, int precision) {
    if (n <= 0) return 4096;
    const int range = (k >= n) ? MR3_RANGE_ALL : MR3_RANGE_INDEX;
    return mr3_workspace_bytes(nullptr, n, range, std::max<int64_t>(k, 1),
                               precision == 32 ? 32 : 64);
}

int mr3_server_create(mr3_server* s, mr3_handle h, size_t hbm_budget_bytes, int max_batch) {
    if (!h) return -2;
    return create_common(s, h, nullptr, nullptr, hbm_budget_bytes, max_batch, 2);
}

int mr3_server_create_ex(mr3_server* s, mr3_handle h, size_t hbm_budget_bytes, int max_batch,
                         int max_inflight) {
    if (!h) return -2;
    return create_common(s, h, nullptr, nullptr, hbm_budget_bytes, max_batch, max_inflight);
}

int mr3_server_create_with_executor(mr3_server* s, mr3_executor_fn fn, void* ctx,
                                    size_t hbm_budget_bytes, int max_batch, int max_inflight) {
    if (!fn) return -2;
    return create_common(s, nullptr, fn, ctx, hbm_budget_bytes, max_batch, max_inflight);
}

int mr3_server_submit(mr3_server s, const mr3_request* r, uint64_t* ticket) {
    if (!s) return -1;
    const int v = validate(r);
    if (v) return v;
    if (!ticket) return -4;
    std::unique_ptr<Entry> en(new Entry());
    en->r = *r;
    en->est = mr3_request_bytes(r->n, wanted(*r), r->precision);
    // a request must be able to run alone in the whole arena
    const int range = wanted(*r) >= r->n ? MR3_RANGE_ALL : MR3_RANGE_INDEX;
    const size_t need = s->fn ? en->est
                              : mr3_workspace_min_bytes(s->h, r->n, range, std::max<int64_t>(wanted(*r), 1),
                                                        r->precision);
    if (need > s->budget) return -3;
    if (!s->fn) {
        // order the solve after the work that produced the request's inputs:
        // an event recorded now on the request's stream
        int prev = 0;
        (void)hipGetDevice(&prev);
        if (hipSetDevice(s->device) != hipSuccess) return MR3_ERR_HIP;
        hipEvent_t ev = nullptr;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if (!s->event_pool.empty()) {
                ev = s->event_pool.back();
                s->event_pool.pop_back();
            }
        }
        hipError_t e = hipSuccess;
        if (!ev) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(ev, (hipStream_t)r->stream);
        (void)hipSetDevice(prev);
        if (e != hipSuccess) {
            if (ev) (void)hipEventDestroy(ev);
            return MR3_ERR_HIP;
        }
        en->ready = ev;
    }
    en->res.submit_ms = steady_ms();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        const uint64_t t = s->next_ticket++;
        s->entries.emplace(t, std::move(en));
        s->queue.push_back(t);
        *ticket = t;
    }
    s->cv_work.notify_all();
    return MR3_OK;
}

int mr3_server_poll(mr3_server s, uint64_t ticket, int* done) {
    if (!s) return -1;
    if (!done) return -3;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->entries.find(ticket);
    if (it == s->entries.end()) return -2;
    *done = it->second->done ? 1 : 0;
    return MR3_OK;
}

int mr3_server_wait(mr3_server s, uint64_t ticket, mr3_result* out) {
    if (!s) return -1;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->entries.find(ticket);
    if (it == s->entries.end() || it->second->claimed) return -2;
    Entry* en = it->second.get();  // stable while the ticket is claimed
    en->claimed = true;
    s->cv_done.wait(lk, [&] { return en->done; });
    const mr3_result res = en->res;
    s->entries.erase(ticket);
    if (out) *out = res;
    return res.status;
}

int mr3_server_destroy(mr3_server s) {
    if (!s) return -1;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto& t : s->workers)
        if (t.joinable()) t.join();
    if (!s->fn) (void)hipSetDevice(s->device);
    for (auto& kv : s->entries)
        if (kv.second->ready) (void)hipEventDestroy(kv.second->ready);
    s->release();
    delete s;
    return MR3_OK;
}

}  // extern "C"
