"""rs_sort_noalloc (the entry point for callers that cannot allocate)
against rs_sort on the same inputs, bit for bit, through the C-ABI: two
calls in a row on the shared fixed scratch, the second smaller than the
first (so nothing left over from the first may leak into the second), for
every kind, and the oracle on the same inputs."""
import ctypes

import numpy as np
import pytest
import torch

import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rs():
    import paper_1511_03404_amd as rs
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    rs.lib()
    return rs


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def call(rs, f, ctx, bits, order, kd, vd, ko, vo, n, *ws):
    kt = rs.RS_KEY_U32 if bits == 32 else rs.RS_KEY_U64
    st = f(ctx.handle, kt, order, rs._ptr(kd), rs._ptr(vd), rs._ptr(ko), rs._ptr(vo), n, *ws,
           rs._stream(ctx.device))
    assert st == rs.RS_OK, rs.lib().rs_last_error()


@pytest.mark.parametrize("bits,pairs", [(32, False), (32, True), (64, False), (64, True)])
def test_noalloc_matches_rs_sort_twice_second_smaller(rs, oracle_lib, bits, pairs):
    L = rs.lib()
    ctx = rs.Context(0)
    per = (bits // 8) * (2 if pairs else 1)
    big = int(L.rs_sort_noalloc_scratch_bytes()) // per * 3 // 4  # near the limit
    for i, (n, dist, order) in enumerate([(big, "uniform", 0), (100003, "bucket", 0),
                                          (5000, "gaussian", rs.RS_ORDER_SIGNED)]):
        print(f"case noalloc bits={bits} pairs={pairs} call={i} n={n} dist={dist}", flush=True)
        keys = datagen.keys(dist, n, bits, seed=i + 1)
        vals = datagen.values(n, bits) if pairs else None
        kd = dev(keys)
        vd = dev(vals) if pairs else None
        ko_a, ko_b = torch.full_like(kd, 3), torch.full_like(kd, 5)
        vo_a = torch.full_like(vd, 3) if pairs else None
        vo_b = torch.full_like(vd, 5) if pairs else None
        call(rs, L.rs_sort_noalloc, ctx, bits, order, kd, vd, ko_a, vo_a, n)
        ws = torch.empty(ctx.workspace_bytes(bits, pairs, n), dtype=torch.uint8, device="cuda")
        call(rs, L.rs_sort, ctx, bits, order, kd, vd, ko_b, vo_b, n, rs._ptr(ws),
             ctypes.c_size_t(ws.numel()))
        torch.cuda.synchronize()
        assert torch.equal(ko_a, ko_b), f"keys differ from rs_sort, call {i}"
        if pairs:
            assert torch.equal(vo_a, vo_b), f"values differ from rs_sort, call {i}"
        ok, ov = oracle_lib.sort_ordered(keys, vals, "signed" if order else "unsigned")
        assert np.array_equal(ko_a.cpu().numpy(), ok)
        if pairs:
            assert np.array_equal(vo_a.cpu().numpy(), ov)
    ctx.close()


def test_noalloc_in_place(rs, oracle_lib):
    L = rs.lib()
    ctx = rs.Context(0)
    n = 300001
    keys = datagen.keys("uniform", n, 32, seed=4)
    vals = datagen.values(n, 32)
    kd, vd = dev(keys), dev(vals)
    call(rs, L.rs_sort_noalloc, ctx, 32, 0, kd, vd, kd, vd, n)
    torch.cuda.synchronize()
    ok, ov = oracle_lib.sort(keys, vals)
    assert np.array_equal(kd.cpu().numpy(), ok) and np.array_equal(vd.cpu().numpy(), ov)
    ctx.close()
