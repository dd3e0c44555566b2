"""GPU parity of every compiled digit-pass configuration -- digit widths of 4
to 8 bits and every tile shape -- against the oracle: the sort's result does
not depend on the digit width (paper, Section 2.6), so each configuration
must give the oracle's output bit for bit, on every distribution, in place
(odd pass counts end in the scratch copy) and in the segmented sort.  Then
the autotuner: the configuration it selects is the one later sorts and
captured graphs use, and they stay exact."""
import numpy as np
import pytest
import torch

import datagen
from tests.certify import certify_segmented

pytestmark = pytest.mark.gpu

KINDS = [(32, False), (32, True), (64, False), (64, True)]


def _config_cases():
    """(bits, pairs, index) for every compiled configuration of every kind,
    read from the library (rs_config_count is host-only), so a configuration
    added to the lists is tested without editing this file."""
    import paper_1511_03404_amd as rs
    return [(bits, pairs, i) for bits, pairs in KINDS for i in range(len(rs.configs(bits, pairs)))]


CASES = _config_cases()


def _seg_config_cases():
    import paper_1511_03404_amd as rs
    return [(bits, pairs, i) for bits, pairs in KINDS
            for i in range(len(rs.configs(bits, pairs, segmented=True)))]


SEG_CASES = _seg_config_cases()


@pytest.fixture(scope="module")
def rs():
    import paper_1511_03404_amd as rs
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    rs.lib()
    return rs


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def config_ctx(rs, bits, pairs, index):
    cfgs = rs.configs(bits, pairs)
    ctx = rs.Context(0)
    ctx.tune_set(bits, pairs, False, -1, index)
    if index < len(rs.configs(bits, pairs, segmented=True)):
        ctx.tune_set(bits, pairs, True, -1, index)
    return ctx, cfgs[index]


def sort(rs, ctx, keys, vals, in_place=False):
    kd = dev(keys)
    vd = dev(vals) if vals is not None else None
    if vd is None:
        out = rs.sort_keys(kd, kd if in_place else None, ctx=ctx)
        torch.cuda.synchronize()
        return host(out), None
    ko, vo = rs.sort_pairs(kd, vd, kd if in_place else None, vd if in_place else None, ctx=ctx)
    torch.cuda.synchronize()
    return host(ko), host(vo)


@pytest.mark.parametrize("bits,pairs,index", CASES)
def test_every_config_matches_oracle(rs, oracle_lib, bits, pairs, index):
    ctx, cfg = config_ctx(rs, bits, pairs, index)
    tile = cfg["threads"] * cfg["items"]
    for n in (3 * tile + 17, 100003):
        for dist in datagen.DISTRIBUTIONS:
            print(f"case bits={bits} pairs={pairs} cfg={cfg} n={n} dist={dist}", flush=True)
            keys = datagen.keys(dist, n, bits, seed=n + index)
            vals = datagen.values(n, bits) if pairs else None
            ok, ov = oracle_lib.sort(keys, vals)
            gk, gv = sort(rs, ctx, keys, vals)
            assert np.array_equal(gk, ok), f"keys differ: {cfg} n={n} {dist}"
            if pairs:
                assert np.array_equal(gv, ov), f"values differ: {cfg} n={n} {dist}"
    ctx.close()


@pytest.mark.parametrize("bits,pairs,index", CASES)
def test_every_config_grouped_claims(rs, oracle_lib, bits, pairs, index):
    """1025 tiles: passes claim them in XCD groups (except 32-bit keys
    alone, which always claim in arrival order), for every configuration."""
    ctx, cfg = config_ctx(rs, bits, pairs, index)
    n = 1025 * cfg["threads"] * cfg["items"] - 7
    print(f"case grouped bits={bits} pairs={pairs} cfg={cfg} n={n}", flush=True)
    keys = datagen.keys("uniform", n, bits, seed=index + 5)
    vals = datagen.values(n, bits) if pairs else None
    ok, ov = oracle_lib.sort(keys, vals)
    gk, gv = sort(rs, ctx, keys, vals)
    assert np.array_equal(gk, ok), f"keys differ: {cfg} n={n}"
    if pairs:
        assert np.array_equal(gv, ov), f"values differ: {cfg} n={n}"
    ctx.close()


@pytest.mark.parametrize("bits,pairs,index", CASES)
def test_every_config_in_place(rs, oracle_lib, bits, pairs, index):
    """In place, with every pass moving data and with the low digits all
    equal (skipped passes change the parity of the moving ones)."""
    ctx, cfg = config_ctx(rs, bits, pairs, index)
    n = 2 * cfg["threads"] * cfg["items"] + 5
    for shift in (0, 9):
        print(f"case in-place bits={bits} pairs={pairs} cfg={cfg} shift={shift}", flush=True)
        keys = datagen.keys("uniform", n, bits, seed=3)
        keys = (keys >> keys.dtype.type(shift)) << keys.dtype.type(shift)
        vals = datagen.values(n, bits) if pairs else None
        ok, ov = oracle_lib.sort(keys, vals)
        gk, gv = sort(rs, ctx, keys, vals, in_place=True)
        assert np.array_equal(gk, ok)
        if pairs:
            assert np.array_equal(gv, ov)
    ctx.close()


@pytest.mark.parametrize("bits,pairs,index", SEG_CASES)
def test_every_config_segmented(rs, oracle_lib, bits, pairs, index):
    """The segmented sort with this configuration's digit passes, out of
    place and in place (an odd pass count copies the large segments back)."""
    ctx, cfg = config_ctx(rs, bits, pairs, index)
    tile = cfg["threads"] * cfg["items"]
    sizes = [17, 5000, 0, 16385, 1, 3 * tile + 5, 70001, 2, 12000]
    off = np.zeros(len(sizes) + 1, dtype=np.uint64)
    off[1:] = np.cumsum(sizes)
    total = int(off[-1])
    keys = datagen.keys("gaussian", total, bits, seed=index)
    sizes_a = np.asarray(sizes, dtype=np.int64)
    vals = (np.arange(total) - np.repeat(off[:-1].astype(np.int64), sizes_a)).astype(keys.dtype) \
        if pairs else None
    ok, ov = oracle_lib.segmented_sort(keys, vals, off)
    offd = dev(off.view(np.int64))
    for in_place in (False, True):
        print(f"case segmented bits={bits} pairs={pairs} cfg={cfg} in_place={in_place}",
              flush=True)
        kd = dev(keys)
        vd = dev(vals) if pairs else None
        ko, vo = rs.segmented_sort(kd, vd, offd, kd if in_place else None,
                                   vd if in_place else None, ctx=ctx)
        torch.cuda.synchronize()
        assert np.array_equal(host(ko), ok)
        if pairs:
            assert np.array_equal(host(vo), ov)
            assert certify_segmented(keys, host(ko), host(vo), off) is None
    ctx.close()


def test_tuned_sort_is_used_and_exact(rs, oracle_lib):
    from paper_1511_03404_amd import tune
    ctx = rs.Context(0)
    n = (1 << 20) + 3
    res = tune.tune_sort(32, True, n, ctx=ctx, reps=2, warmup=1)
    print(f"tuned {res}", flush=True)
    assert ctx.tune_get(32, True, False, rs.size_class(n)) == res["index"]
    assert len(res["ms"]) == len(rs.configs(32, True))
    keys = datagen.keys("bucket", n, 32, seed=8)
    vals = datagen.values(n, 32)
    ok, ov = oracle_lib.sort(keys, vals)
    gk, gv = sort(rs, ctx, keys, vals)
    assert np.array_equal(gk, ok) and np.array_equal(gv, ov)
    ctx.close()


def test_tuned_segmented_graph_replay(rs, oracle_lib):
    """Tune on the caller's batch, capture the tuned enqueue in a graph and
    replay it: every replay equals the oracle."""
    from paper_1511_03404_amd import tune
    k, v, off = datagen.segmented(num_segments=300, lo_log2=4, hi_log2=18, bits=32, seed=4)
    kd, vd = dev(k), dev(v)
    offd = dev(off.view(np.int64))
    ctx = rs.Context(0)
    res = tune.tune_segmented(kd, vd, offd, ctx=ctx, reps=2, warmup=1)
    print(f"tuned {res}", flush=True)
    assert ctx.tune_get(32, True, True, rs.size_class(k.size)) == res["index"]
    ws = torch.empty(ctx.segmented_workspace_bytes(32, True, k.size, 300), dtype=torch.uint8,
                     device="cuda")
    ko, vo = torch.empty_like(kd), torch.empty_like(vd)
    rs.segmented_sort(kd, vd, offd, ko, vo, ctx=ctx, workspace=ws)  # warm-up outside capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rs.segmented_sort(kd, vd, offd, ko, vo, ctx=ctx, workspace=ws)
    ok, ov = oracle_lib.segmented_sort(k, v, off)
    for i in range(3):
        ko.fill_(3)
        vo.fill_(3)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(ko), ok) and np.array_equal(host(vo), ov), f"replay {i}"
    ctx.close()
