"""Serving loop for the radix sort: continuous batching of sort requests.

Requests (n keys of 32 or 64 bits, with or without values) arrive over time.
The scheduler keeps pending requests in one FIFO per kind and a small number of
execution slots (HIP streams).  Whenever a slot is free it forms a batch:
the oldest pending request fixes the key type, and further pending requests
of that type join in arrival order while the batch stays under its element
budget and the device-memory cap (every byte of input staging, output and
scratch of the in-flight batches counts; ``HipBackend`` sizes a batch with
the library's own workspace formulas and caps admission by the device's
free memory).  A batch is one segmented sort
(``rs_segmented_sort``) or, for a single request, one plain sort; batches on
different slots overlap on the device.  Requests that arrive while others
run are admitted as soon as a slot and memory free up.

The scheduler (``Scheduler``) is independent of the device; ``HipBackend``
runs batches with the HIP library on torch streams.  Latency is
completion - arrival, with completion read from a GPU event timestamp.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Optional

GiB = 1 << 30


@dataclasses.dataclass
class Request:
    id: int
    n: int
    bits: int                 # 32 or 64
    has_values: bool
    arrival_s: float = 0.0    # seconds on the serving clock
    payload: object = None    # backend-specific input handle
    # filled in by the server
    batch_id: int = -1
    admit_s: float = float("nan")
    done_s: float = float("nan")
    result: object = None
    error: Optional[BaseException] = None

    @property
    def kind(self):
        return (self.bits, self.has_values)

    def footprint(self) -> int:
        """Device bytes the request occupies while in flight, as a batch of
        its own under the default estimate (staged input, output and scratch
        copies of keys and values)."""
        return default_batch_bytes(self.kind, 1, self.n)


def default_batch_bytes(kind, num_requests: int, elems: int) -> int:
    """Estimate of a batch's device bytes when the backend gives none: staged
    input, output and one scratch copy of the keys and values."""
    bits, has_values = kind
    return 3 * (bits // 8) * (2 if has_values else 1) * elems


@dataclasses.dataclass
class Batch:
    id: int
    slot: int
    requests: list
    handle: object = None
    bytes: int = 0


class Scheduler:
    """Admission and batch formation (no device code).

    backend must provide launch(batch) -> handle, done(handle) -> bool and
    finish(batch) -> {request id: completion seconds}; finish also stores
    each request's result.  An exception from launch or finish fails that
    batch's requests (their ``error`` is set), releases its memory and slot,
    and the rest carry on."""

    def __init__(self, backend, mem_cap: int = 64 * GiB, slots: int = 4,
                 max_batch_elems: int = 1 << 26, max_batch_requests: int = 256,
                 batch_bytes: Optional[Callable[[tuple, int, int], int]] = None):
        """batch_bytes(kind, number of requests, elements) gives the device
        bytes a batch occupies while in flight (default: default_batch_bytes);
        a backend passes its exact figure."""
        if slots < 1 or mem_cap <= 0:
            raise ValueError("need at least one slot and a positive memory cap")
        self.backend = backend
        self.mem_cap = mem_cap
        self.batch_bytes = batch_bytes or default_batch_bytes
        self.slots = slots
        self.max_batch_elems = max_batch_elems
        self.max_batch_requests = max_batch_requests
        # one FIFO per kind (key width, values); the oldest head overall
        # fixes the kind of the next batch, so forming a batch costs O(batch),
        # not O(queue)
        self.queues: dict[tuple, collections.deque] = {}
        self._seq = 0
        self.inflight: dict[int, Batch] = {}
        self.mem_used = 0
        self.free_slots = list(range(slots))
        self.completed: list = []
        self.failed: list = []
        self.rejected: list = []
        self.peak_mem = 0
        self.peak_inflight = 0
        self._next_batch = 0

    def submit(self, req: Request, now: float):
        if self.batch_bytes(req.kind, 1, req.n) > self.mem_cap:
            # could never fit: refuse it instead of blocking the queue
            self.rejected.append(req)
            return False
        self.queues.setdefault(req.kind, collections.deque()).append((self._seq, req))
        self._seq += 1
        return True

    @property
    def pending(self) -> list:
        """Pending requests in arrival order."""
        return [r for _, r in sorted((e for q in self.queues.values() for e in q),
                                     key=lambda e: e[0])]

    def _head_queue(self):
        best = None
        for q in self.queues.values():
            if q and (best is None or q[0][0] < best[0][0]):
                best = q
        return best

    def _form_batch(self):
        q = self._head_queue()
        head = q[0][1]
        if self.mem_used + self.batch_bytes(head.kind, 1, head.n) > self.mem_cap:
            return None
        # requests of a kind are served in arrival order: the first one of
        # the head's kind that does not fit closes the batch
        chosen, elems, nbytes = [], 0, 0
        while q:
            r = q[0][1]
            if not (len(chosen) < self.max_batch_requests
                    and (not chosen or elems + r.n <= self.max_batch_elems)):
                break
            grown = self.batch_bytes(head.kind, len(chosen) + 1, elems + r.n)
            if self.mem_used + grown > self.mem_cap:
                break
            q.popleft()
            chosen.append(r)
            elems += r.n
            nbytes = grown
        b = Batch(self._next_batch, self.free_slots.pop(), chosen, bytes=nbytes)
        self._next_batch += 1
        return b

    def step(self, now: float):
        """Retire finished batches, then launch batches while slots, memory
        and requests allow.  Returns the number of batches launched."""
        for bid in list(self.inflight):
            b = self.inflight[bid]
            try:
                if not self.backend.done(b.handle):
                    continue
                times = self.backend.finish(b)
            except Exception as e:  # the batch failed on the device side
                self._fail(b, e, now)
                continue
            del self.inflight[bid]
            for r in b.requests:
                r.done_s = times.get(r.id, now)
                self.completed.append(r)
            self._release(b)
        launched = 0
        while self.free_slots and self._head_queue() is not None:
            b = self._form_batch()
            if b is None:
                break
            for r in b.requests:
                r.batch_id = b.id
                r.admit_s = now
            self.mem_used += b.bytes
            self.peak_mem = max(self.peak_mem, self.mem_used)
            try:
                b.handle = self.backend.launch(b)
            except Exception as e:
                self._fail(b, e, now)
                continue
            self.inflight[b.id] = b
            self.peak_inflight = max(self.peak_inflight, len(self.inflight))
            launched += 1
        return launched

    def _release(self, b: Batch):
        self.mem_used -= b.bytes
        self.free_slots.append(b.slot)

    def _fail(self, b: Batch, err: BaseException, now: float):
        self.inflight.pop(b.id, None)
        for r in b.requests:
            r.error = err
            r.done_s = now
            self.failed.append(r)
        self._release(b)

    def idle(self) -> bool:
        return self._head_queue() is None and not self.inflight


def serve(scheduler: Scheduler, requests: list, clock: Callable[[], float],
          open_loop: bool = True, sleep: Callable[[float], None] = time.sleep,
          progress: Optional[Callable[[float, int, int], None]] = None,
          progress_every_s: float = 5.0):
    """Feed requests at their arrival times (open loop) or all at once
    (closed loop, arrival = 0) and run the scheduler until all complete.
    progress(now, submitted, finished) is called about every
    progress_every_s seconds of the serving clock."""
    reqs = sorted(requests, key=lambda r: r.arrival_s)
    if not open_loop:
        for r in reqs:
            r.arrival_s = 0.0
    i = 0
    next_report = progress_every_s
    while i < len(reqs) or not scheduler.idle():
        now = clock()
        if progress is not None and now >= next_report:
            progress(now, i, len(scheduler.completed) + len(scheduler.failed))
            next_report = now + progress_every_s
        while i < len(reqs) and reqs[i].arrival_s <= now:
            scheduler.submit(reqs[i], now)
            i += 1
        launched = scheduler.step(now)
        if not launched and i < len(reqs) and scheduler.idle():
            wait = reqs[i].arrival_s - clock()
            if wait > 0:
                sleep(min(wait, 0.001))
    return scheduler.completed


def percentile(xs, q):
    if not xs:
        return float("nan")
    s = sorted(xs)
    k = min(len(s) - 1, max(0, int(round(q / 100.0 * (len(s) - 1)))))
    return s[k]


def summarize(completed: list, makespan_s: float) -> dict:
    lat = [(r.done_s - r.arrival_s) * 1e3 for r in completed]
    keys = sum(r.n for r in completed)
    batches = len({r.batch_id for r in completed})
    return {"requests": len(completed), "keys": keys, "batches": batches,
            "makespan_s": round(makespan_s, 4),
            "Mkeys_s": round(keys / makespan_s / 1e6, 1) if makespan_s > 0 else None,
            "p50_ms": round(percentile(lat, 50), 3), "p99_ms": round(percentile(lat, 99), 3),
            "mean_ms": round(sum(lat) / len(lat), 3) if lat else None}


class HipBackend:
    """Runs batches on the GPU with the HIP library; torch supplies device
    memory, streams and events.  A request's payload is a pair of device
    tensors (keys, values or None) resident in HBM; a batch stages its
    requests' inputs contiguously, sorts them as one segmented sort (a single
    request: a plain sort) and leaves each result as a view of the batch's
    output."""

    def __init__(self, slots: int, device=0, max_batch_requests: int = 256,
                 keep_results: bool = True):
        import torch

        from . import context, segmented_sort, sort_keys, sort_pairs
        self.torch = torch
        self.keep_results = keep_results
        self.dev = torch.device("cuda", device)
        self.ctx = context(device)
        self._sort_keys, self._sort_pairs, self._seg = sort_keys, sort_pairs, segmented_sort
        self.streams = [torch.cuda.Stream(self.dev) for _ in range(slots)]
        # per-slot pinned staging of batch offsets; a slot's next batch only
        # starts after its previous one completed, so each slot's buffer is free
        self.max_requests = max_batch_requests
        self.off_pinned = [torch.empty(max_batch_requests + 1, dtype=torch.int64, pin_memory=True)
                           for _ in range(slots)]
        self.t0_event = torch.cuda.Event(enable_timing=True)
        self.t0_event.record()
        self.t0_wall = None

    def batch_bytes(self, kind, num_requests: int, elems: int) -> int:
        """Device bytes of a batch while in flight, from the library's own
        workspace formulas: the output, the staged inputs and offsets of a
        multi-request batch, and the sort's workspace."""
        bits, has_v = kind
        data = elems * (bits // 8) * (2 if has_v else 1)
        if num_requests <= 1:
            return data + self.ctx.workspace_bytes(bits, has_v, elems)
        return (2 * data + 8 * (num_requests + 1)
                + self.ctx.segmented_workspace_bytes(bits, has_v, elems, num_requests))

    def admission_cap(self, cap: int = 64 * GiB, reserve: int = 2 * GiB) -> int:
        """The admission cap: ``cap``, or the device's free memory less
        ``reserve`` when that is smaller."""
        free, _ = self.torch.cuda.mem_get_info(self.dev)
        return max(1, min(cap, free - reserve))

    def mark_clock_zero(self, wall_now: float):
        """Tie GPU event times to the serving clock: event 0 <-> wall_now."""
        torch = self.torch
        self.t0_event = torch.cuda.Event(enable_timing=True)
        self.t0_event.record(torch.cuda.current_stream(self.dev))
        self.t0_event.synchronize()
        self.t0_wall = wall_now

    def launch(self, batch: Batch):
        torch = self.torch
        s = self.streams[batch.slot]
        reqs = batch.requests
        bits, has_v = reqs[0].kind
        dt = torch.uint32 if bits == 32 else torch.uint64
        total = sum(r.n for r in reqs)
        # the payloads may still be in production on the caller's stream:
        # the slot's stream waits for it, and the caching allocator keeps
        # their memory for the slot's stream until it has used them
        s.wait_stream(torch.cuda.current_stream(self.dev))
        for r in reqs:
            for t in r.payload:
                if t is not None:
                    t.record_stream(s)
        with torch.cuda.stream(s):
            if len(reqs) == 1:
                k, v = reqs[0].payload
                ko = torch.empty(total, dtype=dt, device=self.dev)
                if has_v:
                    vo = torch.empty(total, dtype=dt, device=self.dev)
                    self._sort_pairs(k, v, ko, vo, ctx=self.ctx)
                else:
                    vo = None
                    self._sort_keys(k, ko, ctx=self.ctx)
                outs = [(ko, vo)]
            else:
                kin = torch.empty(total, dtype=dt, device=self.dev)
                vin = torch.empty(total, dtype=dt, device=self.dev) if has_v else None
                offs = [0]
                for r in reqs:
                    k, v = r.payload
                    a = offs[-1]
                    kin[a:a + r.n].copy_(k, non_blocking=True)
                    if has_v:
                        vin[a:a + r.n].copy_(v, non_blocking=True)
                    offs.append(a + r.n)
                if len(offs) > self.max_requests + 1:
                    raise ValueError("batch has more requests than the offsets staging holds")
                off_host = self.off_pinned[batch.slot][:len(offs)]
                off_host.copy_(torch.tensor(offs, dtype=torch.int64))
                off_dev = off_host.to(self.dev, non_blocking=True)
                ko, vo = self._seg(kin, vin, off_dev, ctx=self.ctx)
                outs = [(ko[offs[i]:offs[i + 1]], vo[offs[i]:offs[i + 1]] if has_v else None)
                        for i in range(len(reqs))]
                # keep staging alive until the stream has used it
                outs.append((kin, vin, off_dev, off_host))
            done = torch.cuda.Event(enable_timing=True)
            done.record(s)
        return (done, outs)

    def done(self, handle) -> bool:
        return handle[0].query()

    def finish(self, batch: Batch):
        done, outs = batch.handle
        t = self.t0_wall + self.t0_event.elapsed_time(done) * 1e-3
        if self.keep_results:
            for r, o in zip(batch.requests, outs):
                r.result = o
        batch.handle = None  # drop the batch's device buffers
        return {r.id: t for r in batch.requests}
