"""Serving loop on the GPU: requests of mixed sizes and key types, batched
with each other into segmented sorts and overlapped on several streams,
must each get exactly the result they get when sorted alone (tolerance 0:
integer sorts are bit-exact)."""
import numpy as np
import pytest
import torch

import datagen
from tests.certify import certify_stable_sort

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rs():
    import paper_1511_03404_amd as rs
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    rs.lib()
    return rs


def make(num, seed, hi_log2=18, rate_per_s=2000.0):
    from paper_1511_03404_amd.serving import Request
    pool = torch.from_numpy(datagen.MT19937(seed).u64(1 << 20)).cuda()
    idx32 = torch.arange(1 << hi_log2, dtype=torch.int64, device="cuda").to(torch.uint32)
    idx64 = torch.arange(1 << hi_log2, dtype=torch.int64, device="cuda").to(torch.uint64)
    reqs = []
    for q in datagen.requests(num, rate_per_s=rate_per_s, lo_log2=10, hi_log2=hi_log2, seed=seed):
        n, bits = q["n"], q["bits"]
        if bits == 32:
            src = pool.view(torch.uint32)
        else:
            src = pool
        off = q["key_seed"] % (src.numel() - n)
        keys = src[off:off + n]
        vals = (idx32 if bits == 32 else idx64)[:n] if q["has_values"] else None
        reqs.append(Request(q["id"], n, bits, q["has_values"], q["arrival_s"],
                            payload=(keys, vals)))
    return reqs


@pytest.mark.parametrize("open_loop", [False, True])
def test_each_result_same_alone_and_in_the_mix(rs, open_loop):
    import time
    from paper_1511_03404_amd.serving import HipBackend, Scheduler, serve
    # open loop: 120 arrivals within about 120 us, faster than three slots
    # drain them, so later arrivals queue and share batches whatever the
    # speed of the sort (at a rate the GPU keeps up with, nothing would queue)
    reqs = make(120, seed=3, rate_per_s=1e6 if open_loop else 2000.0)
    be = HipBackend(slots=3, max_batch_requests=16)
    sch = Scheduler(be, mem_cap=1 << 30, slots=3, max_batch_elems=1 << 19,
                    max_batch_requests=16)
    t0 = time.perf_counter()
    be.mark_clock_zero(0.0)
    done = serve(sch, reqs, lambda: time.perf_counter() - t0, open_loop=open_loop)
    torch.cuda.synchronize()
    assert len(done) == 120 and not sch.failed and not sch.rejected
    sizes = [len([r for r in done if r.batch_id == b]) for b in {r.batch_id for r in done}]
    assert max(sizes) > 1, "no request was batched with another"
    if not open_loop:
        assert sch.peak_inflight > 1, "batches never overlapped"
    for r in done:
        keys, vals = r.payload
        if vals is None:
            alone = rs.sort_keys(keys)
            torch.cuda.synchronize()
            assert torch.equal(r.result[0], alone), f"request {r.id}"
        else:
            ak, av = rs.sort_pairs(keys, vals)
            torch.cuda.synchronize()
            assert torch.equal(r.result[0], ak) and torch.equal(r.result[1], av), f"request {r.id}"
            kin = keys.cpu().numpy()
            assert certify_stable_sort(kin, r.result[0].cpu().numpy(),
                                       r.result[1].cpu().numpy()) is None
        assert r.done_s >= r.arrival_s
