// Driver for the AddressSanitizer / UndefinedBehaviorSanitizer build of the
// library's host code (no GPU needed): the workspace plan behind the
// workspace queries, and the serving scheduler with an executor callback in
// place of the device (several worker slots, concurrent submitters, the
// arena allocator, waits, destroy with requests in flight).
#include <cstdio>
#include <thread>
#include <vector>

#include "mr3.h"

static int exec_fn(void*, int64_t count, const mr3_request* reqs, int64_t* m) {
    for (int64_t i = 0; i < count; ++i)
        m[i] = reqs[i].range.range == MR3_RANGE_INDEX ? reqs[i].range.iu - reqs[i].range.il + 1
                                                      : reqs[i].n;
    return 0;
}

int main() {
    int bad = 0;
    for (int64_t n : {1, 7, 1000, 20000})
        for (int prec : {32, 64}) {
            const size_t full = mr3_workspace_bytes(nullptr, n, MR3_RANGE_ALL, 0, prec);
            const size_t low = mr3_workspace_min_bytes(nullptr, n, MR3_RANGE_INDEX, n / 3 + 1, prec);
            bad |= !(full > 0 && low > 0 && low <= full);
        }
    std::vector<int64_t> ns = {40, 300, 5000};
    std::vector<mr3_range_desc> rg(3);
    for (auto& r : rg) r.range = MR3_RANGE_ALL;
    rg[1].range = MR3_RANGE_INDEX;
    rg[1].il = 3;
    rg[1].iu = 90;
    bad |= mr3_workspace_bytes_batched(nullptr, 3, 64, ns.data(), rg.data()) == 0;
    mr3_server s = nullptr;
    const size_t budget = 3 * mr3_request_bytes(600, 600, 64);
    if (mr3_server_create_with_executor(&s, exec_fn, nullptr, budget, 8, 3) != 0) return 1;
    std::vector<std::thread> th;
    for (int k = 0; k < 4; ++k)
        th.emplace_back([&, k] {
            for (int i = 0; i < 60; ++i) {
                mr3_request r{};
                r.precision = ((i + k) & 1) ? 32 : 64;
                r.n = 50 + (i * 37 + k * 11) % 550;
                r.d = (void*)0x1000;
                r.e = (void*)0x2000;
                r.W = (void*)0x3000;
                r.range.range = (i % 3 == 0) ? MR3_RANGE_INDEX : MR3_RANGE_ALL;
                r.range.il = 1;
                r.range.iu = r.range.range == MR3_RANGE_INDEX ? r.n / 2 : r.n;
                r.ldz = r.n;
                uint64_t t = 0;
                if (mr3_server_submit(s, &r, &t) != 0) continue;
                if (i % 5 == 0) continue;  // left to destroy
                mr3_result res;
                if (mr3_server_wait(s, t, &res) != 0) bad = 1;
            }
        });
    for (auto& t : th) t.join();
    mr3_server_destroy(s);
    std::printf(bad ? "host sanitizer run: FAILED\n" : "host sanitizer run: ok\n");
    return bad;
}
