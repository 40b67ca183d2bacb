"""The serving scheduler on the host: batches are formed by an executor
callback instead of the device, so admission, batching, ordering, error
isolation and the ticket life cycle are checked without a GPU."""
import ctypes
import threading
import time

import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import paper_1304_1864_amd as mr3


class FakeExecutor:
    """Records every batch (request ids are carried in the W pointer) and
    returns m = number of wanted eigenpairs; ids in `fail` make any batch
    that holds them fail with MR3_ERR_NUMERIC."""

    def __init__(self, fail=(), hold=None):
        self.batches = []
        self.fail = set(fail)
        self.hold = hold
        self.lock = threading.Lock()
        self.cb = mr3.EXECUTOR_FN(self._run)

    def _run(self, ctx, count, reqs, m):
        if self.hold is not None:
            self.hold.wait(10)
        ids, precs = [], set()
        for i in range(count):
            r = reqs[i]
            ids.append(int(r.W))
            precs.add(r.precision)
            k = r.range.iu - r.range.il + 1 if r.range.range == mr3.RANGE_INDEX else r.n
            m[i] = k
        with self.lock:
            self.batches.append((ids, precs))
        return mr3.MR3_ERR_NUMERIC if self.fail & set(ids) else mr3.MR3_OK


def req(rid, n=100, precision=64, rng=None):
    r = mr3.mr3_request()
    r.precision = precision
    r.n = n
    r.d = 0x1000 + rid  # never dereferenced by the fake executor
    r.e = 0x2000 + rid
    r.W = rid
    r.Z = None
    r.ldz = n
    if rng is None:
        r.range.range, r.range.il, r.range.iu = mr3.RANGE_ALL, 1, n
    else:
        r.range.range, r.range.il, r.range.iu = rng
    return r


def make_server(ex, budget=1 << 30, max_batch=8, max_inflight=1):
    return mr3.mr3_server_create_with_executor(ex.cb, None, budget, max_batch, max_inflight)


def test_batches_group_precision_and_keep_arrival_order():
    hold = threading.Event()
    ex = FakeExecutor(hold=hold)
    s = make_server(ex, max_batch=4)
    # the first request occupies the worker until `hold` is set; the rest queue
    tickets = [mr3.mr3_server_submit(s, req(1, precision=64))]
    time.sleep(0.05)
    for i in range(2, 12):
        tickets.append(mr3.mr3_server_submit(s, req(i, precision=32 if i % 3 == 0 else 64)))
    hold.set()
    res = [mr3.mr3_server_wait(s, t) for t in tickets]
    mr3.mr3_server_destroy(s)
    assert all(r["status"] == 0 for r in res)
    seen = []
    for ids, precs in ex.batches:
        assert len(precs) == 1 and len(ids) <= 4
        seen += ids
        # inside a batch, requests keep their arrival order
        assert ids == sorted(ids)
    assert sorted(seen) == list(range(1, 12))
    # each batch starts with the oldest request still waiting
    waiting = list(range(1, 12))
    for ids, _ in ex.batches:
        assert ids[0] == waiting[0]
        for i in ids:
            waiting.remove(i)
    # results carry the batch bookkeeping
    for r in res:
        assert r["done_ms"] >= r["start_ms"] >= r["submit_ms"] - 1e-6
        assert 1 <= r["batch_size"] <= 4


def test_budget_limits_batches_and_rejects_oversized():
    hold = threading.Event()
    ex = FakeExecutor(hold=hold)
    one = mr3.mr3_request_bytes(1000, 1000, 64)
    s = make_server(ex, budget=int(2.5 * one), max_batch=64)
    with pytest.raises(mr3.MR3Error) as ei:
        mr3.mr3_server_submit(s, req(99, n=4000))
    assert ei.value.code == -3
    tickets = [mr3.mr3_server_submit(s, req(1, n=1000))]
    time.sleep(0.05)
    tickets += [mr3.mr3_server_submit(s, req(i, n=1000)) for i in range(2, 8)]
    hold.set()
    for t in tickets:
        mr3.mr3_server_wait(s, t)
    mr3.mr3_server_destroy(s)
    for ids, _ in ex.batches:
        assert len(ids) * one <= 2.5 * one
    assert max(len(ids) for ids, _ in ex.batches) == 2


def test_failing_request_is_isolated():
    ex = FakeExecutor(fail={5})
    hold = threading.Event()
    ex.hold = hold
    s = make_server(ex, max_batch=16)
    tickets = [mr3.mr3_server_submit(s, req(i)) for i in range(1, 9)]
    hold.set()
    status = {}
    for i, t in zip(range(1, 9), tickets):
        res = mr3.mr3_server_wait(s, t)
        status[i] = res["status"]
    mr3.mr3_server_destroy(s)
    assert status[5] == mr3.MR3_ERR_NUMERIC
    assert all(status[i] == 0 for i in status if i != 5)


def test_invalid_requests_and_tickets():
    ex = FakeExecutor()
    s = make_server(ex)
    bad = [req(1, precision=16), req(2, n=-1), req(3, rng=(mr3.RANGE_INDEX, 5, 2)),
           req(4, rng=(mr3.RANGE_INDEX, 0, 2)), req(5, rng=(mr3.RANGE_INDEX, 1, 101))]
    for r in bad:
        with pytest.raises(mr3.MR3Error) as ei:
            mr3.mr3_server_submit(s, r)
        assert ei.value.code == -2
    r = req(6)
    r.Z = 0x3000
    r.ldz = 50  # < n
    with pytest.raises(mr3.MR3Error):
        mr3.mr3_server_submit(s, r)
    with pytest.raises(mr3.MR3Error):
        mr3.mr3_server_poll(s, 12345)
    t = mr3.mr3_server_submit(s, req(7, rng=(mr3.RANGE_INDEX, 3, 12)))
    res = mr3.mr3_server_wait(s, t)
    assert res["m"] == 10
    with pytest.raises(mr3.MR3Error):  # ticket released by wait
        mr3.mr3_server_wait(s, t)
    mr3.mr3_server_destroy(s)


def test_concurrent_submitters_and_drain_on_destroy():
    ex = FakeExecutor()
    s = make_server(ex, max_batch=5)
    tickets, lock = [], threading.Lock()

    def client(base):
        for i in range(25):
            t = mr3.mr3_server_submit(s, req(base + i, n=50 + i))
            with lock:
                tickets.append(t)

    th = [threading.Thread(target=client, args=(1000 * (k + 1),)) for k in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    done = 0
    for t in tickets:
        while not mr3.mr3_server_poll(s, t):
            time.sleep(0.001)
        done += mr3.mr3_server_wait(s, t)["status"] == 0
    assert done == 100
    # queued work is finished by destroy
    for i in range(10):
        mr3.mr3_server_submit(s, req(9000 + i))
    mr3.mr3_server_destroy(s)
    ids = [i for b, _ in ex.batches for i in b]
    assert len(ids) == 110 and len(set(ids)) == 110


class SlowExecutor:
    """Each batch takes `delay(ids)` seconds; records when it ran, which
    requests it held, and the largest sum of request estimates in flight at
    once."""

    def __init__(self, delay):
        self.delay = delay
        self.lock = threading.Lock()
        self.inflight_bytes = 0
        self.max_inflight_bytes = 0
        self.max_concurrent = 0
        self.concurrent = 0
        self.cb = mr3.EXECUTOR_FN(self._run)

    def _run(self, ctx, count, reqs, m):
        ids, est = [], 0
        for i in range(count):
            r = reqs[i]
            ids.append(int(r.W))
            k = r.range.iu - r.range.il + 1 if r.range.range == mr3.RANGE_INDEX else r.n
            est += mr3.mr3_request_bytes(r.n, k, r.precision)
            m[i] = k
        with self.lock:
            self.inflight_bytes += est
            self.concurrent += 1
            self.max_inflight_bytes = max(self.max_inflight_bytes, self.inflight_bytes)
            self.max_concurrent = max(self.max_concurrent, self.concurrent)
        time.sleep(self.delay(ids))
        with self.lock:
            self.inflight_bytes -= est
            self.concurrent -= 1
        return mr3.MR3_OK


def test_later_request_overtakes_a_long_batch():
    """With two slots, a short request submitted while a long batch runs is
    admitted by the free slot and completes first (continuous batching)."""
    ex = SlowExecutor(lambda ids: 0.5 if 1 in ids else 0.01)
    s = make_server(ex, max_batch=8, max_inflight=2)
    t_long = mr3.mr3_server_submit(s, req(1, n=4000, precision=64))
    time.sleep(0.05)
    t_short = mr3.mr3_server_submit(s, req(2, n=100, precision=32))
    short = mr3.mr3_server_wait(s, t_short)
    assert not mr3.mr3_server_poll(s, t_long)
    long_ = mr3.mr3_server_wait(s, t_long)
    mr3.mr3_server_destroy(s)
    assert short["done_ms"] < long_["done_ms"]
    assert short["slot"] != long_["slot"]
    assert short["start_ms"] < long_["done_ms"]  # overlapped in time


def test_memory_in_flight_stays_within_the_budget():
    """Batches on several slots never hold more than the budget together, and
    every request runs."""
    one = mr3.mr3_request_bytes(1000, 1000, 64)
    budget = int(3.5 * one)
    ex = SlowExecutor(lambda ids: 0.02)
    s = make_server(ex, budget=budget, max_batch=2, max_inflight=4)
    tickets = [mr3.mr3_server_submit(s, req(i, n=1000)) for i in range(1, 25)]
    res = [mr3.mr3_server_wait(s, t) for t in tickets]
    mr3.mr3_server_destroy(s)
    assert all(r["status"] == 0 for r in res)
    assert ex.max_inflight_bytes <= budget
    assert ex.max_concurrent >= 2  # several batches did run at once
    assert len({r["slot"] for r in res}) >= 2


def test_a_ticket_has_one_waiter():
    hold = threading.Event()
    ex = FakeExecutor(hold=hold)
    s = make_server(ex)
    t = mr3.mr3_server_submit(s, req(1))
    first = {}
    th = threading.Thread(target=lambda: first.update(mr3.mr3_server_wait(s, t)))
    th.start()
    time.sleep(0.05)
    with pytest.raises(mr3.MR3Error) as ei:  # already claimed by the first waiter
        mr3.mr3_server_wait(s, t)
    assert ei.value.code == -2
    hold.set()
    th.join()
    assert first["status"] == 0
    mr3.mr3_server_destroy(s)


# ---------------------------------------------------------------------------
# property-based: random request streams through the scheduler
# ---------------------------------------------------------------------------


class RecordingExecutor:
    """Runs batches in a few milliseconds, failing those that hold a request
    of `fail`; records every batch with the request bytes in flight."""

    def __init__(self, fail):
        self.fail = set(fail)
        self.lock = threading.Lock()
        self.batches = []
        self.inflight = 0
        self.max_inflight = 0
        self.cb = mr3.EXECUTOR_FN(self._run)

    def _run(self, ctx, count, reqs, m):
        ids, precs, est = [], set(), 0
        for i in range(count):
            r = reqs[i]
            ids.append(int(r.W))
            precs.add(r.precision)
            k = r.range.iu - r.range.il + 1 if r.range.range == mr3.RANGE_INDEX else r.n
            est += mr3.mr3_request_bytes(r.n, k, r.precision)
            m[i] = k
        with self.lock:
            self.batches.append((ids, precs))
            self.inflight += est
            self.max_inflight = max(self.max_inflight, self.inflight)
        time.sleep(0.002)
        with self.lock:
            self.inflight -= est
        return mr3.MR3_ERR_NUMERIC if self.fail & set(ids) else mr3.MR3_OK


@st.composite
def stream(draw):
    count = draw(st.integers(1, 16))
    reqs = []
    for i in range(1, count + 1):
        n = draw(st.integers(1, 3000))
        prec = draw(st.sampled_from([32, 64]))
        rng = None
        if draw(st.booleans()):
            il = draw(st.integers(1, n))
            iu = draw(st.integers(il, n))
            rng = (mr3.RANGE_INDEX, il, iu)
        reqs.append((i, n, prec, rng))
    fail = draw(st.sets(st.integers(1, count), max_size=2))
    return reqs, fail


@settings(max_examples=40, deadline=None, derandomize=True, database=None,
          suppress_health_check=[HealthCheck.too_slow])
@given(stream(), st.integers(1, 8), st.integers(1, 4), st.floats(1.0, 4.0))
def test_random_streams_keep_the_scheduler_invariants(s_, max_batch, max_inflight, budget_factor):
    """Every request completes once, with its wanted count, alone in failing
    when it fails; batches hold one precision and at most max_batch
    requests; the request bytes in flight stay within the budget."""
    reqs, fail = s_
    sizes = []
    for i, n, prec, rng in reqs:
        k = rng[2] - rng[1] + 1 if rng else n
        sizes.append(mr3.mr3_request_bytes(n, k, prec))
    budget = int(max(sizes) * budget_factor)
    ex = RecordingExecutor(fail)
    srv = make_server(ex, budget=budget, max_batch=max_batch, max_inflight=max_inflight)
    tickets = [mr3.mr3_server_submit(srv, req(i, n=n, precision=prec, rng=rng))
               for i, n, prec, rng in reqs]
    results = [mr3.mr3_server_wait(srv, t) for t in tickets]
    mr3.mr3_server_destroy(srv)
    for (i, n, prec, rng), r in zip(reqs, results):
        k = rng[2] - rng[1] + 1 if rng else n
        if i in fail:
            assert r["status"] != 0
        else:
            assert r["status"] == 0 and r["m"] == k
    for ids, precs in ex.batches:
        assert len(precs) == 1 and 1 <= len(ids) <= max_batch
    assert ex.max_inflight <= budget
    ran_ok = {i for ids, _ in ex.batches for i in ids}
    assert {i for i, *_ in reqs} <= ran_ok
