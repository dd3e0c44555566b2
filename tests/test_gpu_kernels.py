"""Per-kernel parity of the plain radix sort, so that a wrong result can be
traced to one kernel: the histogram kernel against the oracle's digit
histograms, and the state after each digit pass against the oracle's state
after the same number of counting-sort passes (the input stably sorted by
its low p*r bits; paper, Section 2.6).  Every compiled configuration (digit
widths and tile shapes), every kind, skewed and uniform keys, a ragged last
tile."""
import numpy as np
import pytest
import torch

import datagen

pytestmark = pytest.mark.gpu

KINDS = [(32, False), (32, True), (64, False), (64, True)]


def _counts():
    import paper_1511_03404_amd as rs
    return {k: len(rs.configs(*k)) for k in KINDS}


CASES = [(bits, pairs, i) for (bits, pairs), c in _counts().items() for i in range(c)]


@pytest.fixture(scope="module")
def rs():
    import paper_1511_03404_amd as rs
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    rs.lib()
    return rs


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("dist", ["uniform", "bucket", "sorted"])
@pytest.mark.parametrize("bits,pairs,index", CASES)
def test_histograms_and_each_pass(rs, oracle_lib, bits, pairs, index, dist):
    ctx = rs.Context(0)
    ctx.tune_set(bits, pairs, False, -1, index)
    cfg = rs.configs(bits, pairs)[index]
    r = cfg["radix_bits"]
    d = (bits + r - 1) // r
    n = 3 * cfg["threads"] * cfg["items"] + 1234
    print(f"case bits={bits} pairs={pairs} config={cfg} dist={dist} n={n}", flush=True)
    keys = datagen.keys(dist, n, bits, seed=index + 1)
    vals = datagen.values(n, bits) if pairs else None
    kd = dev(keys)
    vd = dev(vals) if pairs else None
    want_h = oracle_lib.digit_histograms(keys, r)
    for p in range(d + 1):
        hist, ko, vo = rs.sort_stages(kd, vd, passes=p, ctx=ctx)
        torch.cuda.synchronize()
        assert ctx.status(None) == rs.RS_OK
        h = hist.cpu().numpy().astype(np.uint64)
        assert h.shape == want_h.shape and np.array_equal(h, want_h), "histograms differ"
        sk, sv = oracle_lib.sort(keys, vals, r=r, passes=p)
        assert np.array_equal(ko.cpu().numpy(), sk), f"keys differ after {p} passes"
        if pairs:
            assert np.array_equal(vo.cpu().numpy(), sv), f"values differ after {p} passes"
    ctx.close()


@pytest.mark.parametrize("dist", ["uniform", "bucket"])
@pytest.mark.parametrize("n", [1 << 16, (1 << 16) + 1, 16 * 16384, 16 * 16384 + 1])
@pytest.mark.parametrize("bits,pairs", KINDS)
def test_histogram_modes(rs, oracle_lib, bits, pairs, n, dist):
    """Every way of building the histograms: up to 2^16 keys one workgroup
    per 4096 keys counting them key by key; up to 16 histogram workgroups
    (one per 16384 keys) each write a row block that the plan kernel sums;
    from 17 on they add into one cleared histogram.  Either way the
    histograms and every pass equal the oracle's."""
    ctx = rs.Context(0)
    ctx.tune_set(bits, pairs, False, -1, 0)
    cfg = rs.configs(bits, pairs)[0]
    r = cfg["radix_bits"]
    d = (bits + r - 1) // r
    print(f"case bits={bits} pairs={pairs} n={n} dist={dist}", flush=True)
    keys = datagen.keys(dist, n, bits, seed=n % 7 + 1)
    vals = datagen.values(n, bits) if pairs else None
    kd = dev(keys)
    vd = dev(vals) if pairs else None
    want_h = oracle_lib.digit_histograms(keys, r)
    for p in (0, 1, d):
        hist, ko, vo = rs.sort_stages(kd, vd, passes=p, ctx=ctx)
        torch.cuda.synchronize()
        assert ctx.status(None) == rs.RS_OK
        assert np.array_equal(hist.cpu().numpy().astype(np.uint64), want_h), "histograms differ"
        sk, sv = oracle_lib.sort(keys, vals, r=r, passes=p)
        assert np.array_equal(ko.cpu().numpy(), sk), f"keys differ after {p} passes"
        if pairs:
            assert np.array_equal(vo.cpu().numpy(), sv), f"values differ after {p} passes"
    ctx.close()
