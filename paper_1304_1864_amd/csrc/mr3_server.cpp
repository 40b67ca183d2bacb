// Serving front end: continuous batching of independent eigenproblems.
//
// One worker thread per server.  Requests wait in arrival order; when the
// device is free the worker forms the next batch from the oldest request and
// the later queued requests of the same precision that fit the batch limits
// (count and estimated workspace), runs the batch as one pass of the solver
// pipeline on the server's stream, and publishes every request's result.
// Eigenpairs of different matrices are independent (Section 3.1), so a batch
// gives each request what a solve of it alone gives.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
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

struct Entry {
    mr3_request r;
    size_t est = 0;
    bool done = false;
    mr3_result res{};
};

}  // namespace

struct mr3_server_s {
    mr3_handle h = nullptr;
    mr3_executor_fn fn = nullptr;
    void* ctx = nullptr;
    size_t budget = 0;
    int max_batch = 1;
    hipStream_t stream = nullptr;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, Entry> entries;
    uint64_t next_ticket = 1;
    int64_t next_batch = 0;
    bool stop = false;

    // run one batch; fills m and returns the status
    int execute(std::vector<mr3_request>& reqs, std::vector<int64_t>& m) {
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
        int rc = mr3_solve_ptrs(h, reqs[0].precision, c, n.data(), d.data(), e.data(), rg.data(),
                                m.data(), W.data(), Z.data(), ldz.data(), stream);
        const hipError_t se = hipStreamSynchronize(stream);
        if (rc == MR3_OK && se != hipSuccess) rc = MR3_ERR_HIP;
        return rc;
    }

    void run() {
        (void)(fn ? hipSuccess : hipSetDevice(mr3_handle_device(h)));
        for (;;) {
            std::vector<uint64_t> batch;
            std::vector<mr3_request> reqs;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] { return stop || !queue.empty(); });
                if (queue.empty()) return;  // stop requested and nothing left
                const int prec = entries[queue.front()].r.precision;
                size_t sum = 0;
                for (auto it = queue.begin(); it != queue.end() && (int)batch.size() < max_batch;) {
                    Entry& en = entries[*it];
                    if (en.r.precision == prec && (batch.empty() || sum + en.est <= budget)) {
                        sum += en.est;
                        batch.push_back(*it);
                        reqs.push_back(en.r);
                        it = queue.erase(it);
                    } else {
                        ++it;
                    }
                }
            }
            const int64_t bid = next_batch++;
            const double t0 = steady_ms();
            std::vector<int64_t> m(batch.size(), 0);
            std::vector<int> status(batch.size(), 0);
            int rc = execute(reqs, m);
            if (rc != MR3_OK && batch.size() > 1) {
                // isolate the failing request(s): solve each alone
                for (size_t i = 0; i < batch.size(); ++i) {
                    std::vector<mr3_request> one{reqs[i]};
                    std::vector<int64_t> m1(1, 0);
                    status[i] = execute(one, m1);
                    m[i] = m1[0];
                }
            } else {
                std::fill(status.begin(), status.end(), rc);
            }
            const double t1 = steady_ms();
            {
                std::lock_guard<std::mutex> lk(mu);
                for (size_t i = 0; i < batch.size(); ++i) {
                    Entry& en = entries[batch[i]];
                    en.res.status = status[i];
                    en.res.m = m[i];
                    en.res.start_ms = t0;
                    en.res.done_ms = t1;
                    en.res.batch_id = bid;
                    en.res.batch_size = (int)batch.size();
                    en.done = true;
                }
            }
            cv_done.notify_all();
        }
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
                  int max_batch) {
    if (!s) return -1;
    if (budget == 0) return -3;
    if (max_batch < 1) return -4;
    mr3_server_s* v = new mr3_server_s();
    v->h = h;
    v->fn = fn;
    v->ctx = ctx;
    v->budget = budget;
    v->max_batch = max_batch;
    if (!fn) {
        if (hipSetDevice(mr3_handle_device(h)) != hipSuccess ||
            hipStreamCreateWithFlags(&v->stream, hipStreamNonBlocking) != hipSuccess) {
            delete v;
            return MR3_ERR_HIP;
        }
    }
    v->worker = std::thread([v] { v->run(); });
    *s = v;
    return MR3_OK;
}

}  // namespace

extern "C" {

size_t mr3_request_bytes(int64_t n, int64_t k, int precision) {
    (void)precision;  // the working arrays are binary64 or double-double on both paths
    if (n <= 0) return 4096;
    // eigenvector tiles (binary64, both level parities) + root and child
    // representations and per-row arrays
    return (size_t)(16 * n * std::max<int64_t>(k, 0) + 256 * n + 65536);
}

int mr3_server_create(mr3_server* s, mr3_handle h, size_t hbm_budget_bytes, int max_batch) {
    if (!h) return -2;
    return create_common(s, h, nullptr, nullptr, hbm_budget_bytes, max_batch);
}

int mr3_server_create_with_executor(mr3_server* s, mr3_executor_fn fn, void* ctx,
                                    size_t hbm_budget_bytes, int max_batch) {
    if (!fn) return -2;
    return create_common(s, nullptr, fn, ctx, hbm_budget_bytes, max_batch);
}

int mr3_server_submit(mr3_server s, const mr3_request* r, uint64_t* ticket) {
    if (!s) return -1;
    const int v = validate(r);
    if (v) return v;
    if (!ticket) return -4;
    Entry en;
    en.r = *r;
    en.est = mr3_request_bytes(r->n, wanted(*r), r->precision);
    if (en.est > s->budget) return -3;
    en.res.submit_ms = steady_ms();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        const uint64_t t = s->next_ticket++;
        s->entries.emplace(t, en);
        s->queue.push_back(t);
        *ticket = t;
    }
    s->cv_work.notify_one();
    return MR3_OK;
}

int mr3_server_poll(mr3_server s, uint64_t ticket, int* done) {
    if (!s) return -1;
    if (!done) return -3;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->entries.find(ticket);
    if (it == s->entries.end()) return -2;
    *done = it->second.done ? 1 : 0;
    return MR3_OK;
}

int mr3_server_wait(mr3_server s, uint64_t ticket, mr3_result* out) {
    if (!s) return -1;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->entries.find(ticket);
    if (it == s->entries.end()) return -2;
    s->cv_done.wait(lk, [&] { return it->second.done; });
    const mr3_result res = it->second.res;
    s->entries.erase(it);
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
    if (s->worker.joinable()) s->worker.join();
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
    return MR3_OK;
}

}  // extern "C"
