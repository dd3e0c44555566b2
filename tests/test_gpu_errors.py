"""Errors found on the device are reported, and every kernel still exits.

* A wait on another workgroup (a tile claim or the decoupled look-back) is
  bounded.  The host forces each kind of wait to its bound with a test-only
  stall (a predecessor the wait treats as never published) and a tiny poll
  limit: the sort must end normally and the status query must say that the
  output is not valid.  No kernel faults or hangs: every wait gives up.
* A segment of 2^30 or more elements is left unsorted and reported as
  unsupported, while the other segments of the batch are sorted.
"""
import numpy as np
import pytest
import torch

import datagen

pytestmark = pytest.mark.gpu

TILE = 16384


@pytest.fixture(scope="module")
def rs():
    import paper_1511_03404_amd as rs
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    rs.lib()
    return rs


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("stall", [1, 2], ids=["lookback", "claim"])
@pytest.mark.parametrize("bits", [32, 64])
def test_bounded_waits_give_up_and_report(rs, oracle_lib, stall, bits):
    # a pass of up to 1024 tiles claims them in arrival order, with no
    # wait: the claim case needs more tiles (1100 of 16384 keys)
    n = (5 if stall == 1 else 1100) * TILE + 3
    print(f"case stall={stall} bits={bits} n={n}", flush=True)
    keys = datagen.keys("uniform", n, bits, seed=3)
    vals = datagen.values(n, bits)
    ctx = rs.Context(0)
    ws = torch.empty(ctx.workspace_bytes(bits, True, n), dtype=torch.uint8, device="cuda")
    ctx.debug_wait_set(spin_limit=32, stall=stall)
    kd, vd = dev(keys), dev(vals)
    rs.sort_pairs(kd, vd, ctx=ctx, workspace=ws)
    assert ctx.status(ws) == rs.RS_ERR_DEVICE
    with pytest.raises(rs.RSError):
        ctx.check(ws)
    # back to the default bound: the same workspace sorts correctly again
    ctx.debug_wait_set(spin_limit=1 << 22, stall=0)
    ko, vo = rs.sort_pairs(kd, vd, ctx=ctx, workspace=ws)
    assert ctx.status(ws) == rs.RS_OK
    ok, ov = oracle_lib.sort(keys, vals)
    assert np.array_equal(ko.cpu().numpy(), ok) and np.array_equal(vo.cpu().numpy(), ov)
    ctx.close()


def test_segmented_bounded_waits(rs, oracle_lib):
    sizes = [3 * TILE + 1, 17, 5000, 2 * TILE + 9]
    off = np.zeros(len(sizes) + 1, dtype=np.uint64)
    off[1:] = np.cumsum(sizes)
    total = int(off[-1])
    keys = datagen.keys("uniform", total, 32, seed=4)
    vals = datagen.values(total, 32)
    ctx = rs.Context(0)
    ws = torch.empty(ctx.segmented_workspace_bytes(32, True, total, len(sizes)),
                     dtype=torch.uint8, device="cuda")
    kd, vd, od = dev(keys), dev(vals), dev(off.view(np.int64))
    ctx.debug_wait_set(spin_limit=32, stall=1)
    rs.segmented_sort(kd, vd, od, ctx=ctx, workspace=ws)
    assert ctx.status(ws) == rs.RS_ERR_DEVICE
    ctx.debug_wait_set(spin_limit=1 << 22, stall=0)
    ko, vo = rs.segmented_sort(kd, vd, od, ctx=ctx, workspace=ws)
    assert ctx.status(ws) == rs.RS_OK
    ok, ov = oracle_lib.segmented_sort(keys, vals, off)
    assert np.array_equal(ko.cpu().numpy(), ok) and np.array_equal(vo.cpu().numpy(), ov)
    ctx.close()


def test_segment_of_2p30_elements_is_reported(rs, oracle_lib):
    """Keys only, 2^30 + 30000 elements in three segments; the middle one
    holds 2^30 elements, one more than a sort takes."""
    small = 10000
    big = 1 << 30
    total = big + 3 * small
    print(f"case segment of 2^30, total={total}", flush=True)
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    kd = torch.randint(-(1 << 31), 1 << 31, (total,), dtype=torch.int64, device="cuda",
                       generator=g).to(torch.int32)
    off = np.array([0, small, small + big, total], dtype=np.uint64)
    ctx = rs.Context(0)
    ko = torch.zeros_like(kd)
    ws = torch.empty(ctx.segmented_workspace_bytes(32, False, total, 3), dtype=torch.uint8,
                     device="cuda")
    rs.segmented_sort(kd, None, dev(off.view(np.int64)), ko, ctx=ctx, workspace=ws)
    assert ctx.status(ws) == rs.RS_ERR_UNSUPPORTED
    for a, b in ((0, small), (small + big, total)):
        ref, _ = oracle_lib.sort(kd[a:b].cpu().numpy().view(np.uint32))
        assert np.array_equal(ko[a:b].cpu().numpy().view(np.uint32), ref)
    ctx.close()
