"""Scheduler of the serving loop on the CPU, with a fake backend that sorts
with the oracle: admission under the memory cap, batches of one key type,
FIFO order, slots, rejection of requests that can never fit, and failure of
one batch without disturbing the others."""
import numpy as np
import pytest

import datagen
from paper_1511_03404_amd.serving import Request, Scheduler, serve, summarize


class FakeBackend:
    """Completes a batch `delay` scheduler steps after its launch; its
    'device time' is proportional to the batch's elements."""

    def __init__(self, delay=2, fail_batches=()):
        self.delay = delay
        self.fail_batches = set(fail_batches)
        self.launched = []
        self.steps = {}

    def launch(self, batch):
        if batch.id in self.fail_batches:
            raise RuntimeError("injected launch failure")
        self.launched.append(batch)
        self.steps[batch.id] = 0
        return batch.id

    def done(self, handle):
        self.steps[handle] += 1
        return self.steps[handle] >= self.delay

    def finish(self, batch):
        import oracle
        t = {}
        for r in batch.requests:
            keys, vals = r.payload
            r.result = oracle.sort(keys, vals)
            t[r.id] = r.arrival_s + 1e-3 * r.n
        return t


def make_requests(num, seed=1, lo=10, hi=14):
    reqs = []
    for q in datagen.requests(num, rate_per_s=1000.0, lo_log2=lo, hi_log2=hi, seed=seed):
        keys = datagen.keys("uniform", q["n"], q["bits"], seed=q["key_seed"])
        vals = datagen.values(q["n"], q["bits"]) if q["has_values"] else None
        reqs.append(Request(q["id"], q["n"], q["bits"], q["has_values"], q["arrival_s"],
                            payload=(keys, vals)))
    return reqs


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-4
        return self.t


def test_every_request_completes_once_and_correctly():
    reqs = make_requests(120)
    sch = Scheduler(FakeBackend(), mem_cap=1 << 30, slots=3, max_batch_elems=1 << 16)
    done = serve(sch, reqs, Clock(), open_loop=True, sleep=lambda s: None)
    assert sorted(r.id for r in done) == list(range(120))
    for r in done:
        keys, vals = r.payload
        k, v = r.result
        assert np.array_equal(k, np.sort(keys))
        if vals is not None:
            assert np.array_equal(v.astype(np.int64), np.argsort(keys, kind="stable"))
    s = summarize(done, 1.0)
    assert s["requests"] == 120 and s["p99_ms"] >= s["p50_ms"]


def test_batches_hold_one_key_type_and_respect_limits():
    reqs = make_requests(200)
    be = FakeBackend(delay=3)
    cap = 6 << 20
    sch = Scheduler(be, mem_cap=cap, slots=2, max_batch_elems=1 << 15, max_batch_requests=7)
    serve(sch, reqs, Clock(), open_loop=False, sleep=lambda s: None)
    assert sch.peak_mem <= cap
    for b in be.launched:
        assert len({r.kind for r in b.requests}) == 1
        assert len(b.requests) <= 7
        assert len(b.requests) == 1 or sum(r.n for r in b.requests) <= 1 << 15
    # requests of one kind are launched in arrival order
    order = [r.id for b in be.launched for r in b.requests]
    for kind in {r.kind for r in reqs}:
        ids = [i for i in order if reqs[i].kind == kind]
        assert ids == sorted(ids)


def test_never_more_batches_in_flight_than_slots():
    reqs = make_requests(100)
    be = FakeBackend(delay=5)
    sch = Scheduler(be, mem_cap=1 << 30, slots=2, max_batch_elems=1 << 12)
    clock = Clock()
    for r in reqs:
        r.arrival_s = 0.0
        sch.submit(r, 0.0)
    peak = 0
    while not sch.idle():
        sch.step(clock())
        peak = max(peak, len(sch.inflight))
    assert peak == 2


def test_request_that_can_never_fit_is_rejected_others_complete():
    reqs = make_requests(30)
    big = Request(999, 1 << 22, 64, True, 0.0, payload=None)
    sch = Scheduler(FakeBackend(), mem_cap=1 << 24, slots=2)
    done = serve(sch, reqs + [big], Clock(), open_loop=False, sleep=lambda s: None)
    assert [r.id for r in sch.rejected] == [999]
    assert sorted(r.id for r in done) == list(range(30))


def test_failed_batch_releases_memory_and_slot():
    reqs = make_requests(60)
    be = FakeBackend(fail_batches={2})
    sch = Scheduler(be, mem_cap=1 << 30, slots=2, max_batch_elems=1 << 14)
    done = serve(sch, reqs, Clock(), open_loop=False, sleep=lambda s: None)
    failed_ids = {r.id for r in sch.failed}
    assert failed_ids and all(r.batch_id == 2 for r in sch.failed)
    assert sorted([r.id for r in done] + sorted(failed_ids)) == list(range(60))
    assert sch.mem_used == 0 and sorted(sch.free_slots) == [0, 1]


def test_head_of_line_waits_for_memory():
    """A large head request waits for memory instead of being overtaken."""
    small = [Request(i, 1 << 10, 32, False, 0.0, payload=(np.zeros(1 << 10, np.uint32), None))
             for i in range(1, 4)]
    big = Request(0, 1 << 18, 32, False, 0.0, payload=(np.zeros(1 << 18, np.uint32), None))
    be = FakeBackend(delay=4)
    cap = big.footprint() + 10
    sch = Scheduler(be, mem_cap=cap, slots=4, max_batch_elems=1 << 20)
    sch.submit(small[0], 0.0)
    sch.step(0.0)                     # small[0] in flight
    for r in [big] + small[1:]:
        sch.submit(r, 0.0)
    while not sch.idle():
        sch.step(0.0)
    order = [b.requests[0].id for b in be.launched]
    assert order.index(0) < order.index(2)


class NullBackend:
    """Completes every batch at the next step, sorting nothing."""

    def launch(self, batch):
        return batch

    def done(self, handle):
        return True

    def finish(self, batch):
        return {r.id: 0.0 for r in batch.requests}


def test_forming_a_batch_does_not_scan_the_whole_queue():
    """A closed loop queues every request at once; a batch must cost
    O(batch), not O(queue), or the scheduler dominates at 10^5 requests."""
    import time
    qs = datagen.requests(100000, rate_per_s=1e6, lo_log2=10, hi_log2=24, seed=1)
    reqs = [Request(q["id"], q["n"], q["bits"], q["has_values"], 0.0) for q in qs]
    sch = Scheduler(NullBackend(), mem_cap=64 << 30, slots=4, max_batch_elems=1 << 25)
    t0 = time.perf_counter()
    done = serve(sch, reqs, lambda: 0.0, open_loop=False, sleep=lambda s: None)
    assert len(done) == 100000
    assert time.perf_counter() - t0 < 20.0
    # arrival order within each kind, one kind per batch
    for kind in {r.kind for r in reqs}:
        ids = [r.id for r in sorted(done, key=lambda r: (r.batch_id, r.id)) if r.kind == kind]
        assert ids == sorted(ids)
    batches = {}
    for r in done:
        batches.setdefault(r.batch_id, set()).add(r.kind)
    assert all(len(k) == 1 for k in batches.values())


def test_admission_uses_the_backend_batch_size():
    """A backend's batch size (here: a fixed workspace per batch plus a
    per-request term, not additive over requests) decides admission: the
    bytes held in flight never exceed the cap, and every batch's recorded
    bytes are the function's value for that batch."""
    calls = []

    def batch_bytes(kind, nreq, elems):
        calls.append((kind, nreq, elems))
        return (1 << 20) + 4096 * nreq + 12 * elems

    reqs = make_requests(150, seed=4)
    be = FakeBackend(delay=3)
    cap = 5 << 20
    sch = Scheduler(be, mem_cap=cap, slots=3, max_batch_elems=1 << 16,
                    batch_bytes=batch_bytes)
    done = serve(sch, reqs, Clock(), open_loop=False, sleep=lambda s: None)
    assert len(done) == 150 and not sch.rejected and calls
    assert sch.peak_mem <= cap
    for b in be.launched:
        assert b.bytes == batch_bytes(b.requests[0].kind, len(b.requests),
                                      sum(r.n for r in b.requests))
    # a request whose own batch could never fit is rejected, not queued
    sch2 = Scheduler(FakeBackend(), mem_cap=1 << 20, slots=1, batch_bytes=batch_bytes)
    assert not sch2.submit(reqs[0], 0.0) and sch2.rejected == [reqs[0]]
