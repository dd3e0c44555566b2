"""GPU parity of the batched segmented sort (one enqueue for many uneven
independent sorts) against the CPU oracle applied per segment."""
import numpy as np
import pytest
import torch

import datagen
from tests.certify import certify_segmented

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rs():
    import paper_1511_03404_amd as rs
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    rs.lib()
    return rs


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_seg(rs, keys, vals, offsets, total_out=None, in_place=False, sentinel=None):
    kd = dev(keys)
    vd = dev(vals) if vals is not None else None
    off = dev(np.asarray(offsets, dtype=np.uint64).view(np.int64))
    if in_place:
        ko, vo = kd, vd
    else:
        ko = torch.empty_like(kd)
        vo = torch.empty_like(vd) if vd is not None else None
        if sentinel is not None:
            ko.fill_(sentinel)
            if vo is not None:
                vo.fill_(sentinel)
    rs.segmented_sort(kd, vd, off, ko, vo)
    torch.cuda.synchronize()
    return ko.cpu().numpy(), (vo.cpu().numpy() if vo is not None else None)


def local_index(offsets, total, bits):
    off = np.asarray(offsets, dtype=np.int64)
    v = np.zeros(total, dtype=np.int64)
    sizes = np.diff(off)
    v[off[0]:off[-1]] = np.arange(off[-1] - off[0]) - np.repeat(off[:-1] - off[0], sizes)
    return v.astype(np.uint32 if bits == 32 else np.uint64)


CASES = {
    # sizes straddling every class boundary: empty, single, small cap 4096,
    # medium cap (16384, or 8192 for 64-bit pairs), tile multiples
    "edges": [0, 1, 2, 0, 4095, 4096, 4097, 8191, 8192, 8193, 16383, 16384, 16385, 1, 0,
              32768, 32769, 49153, 3, 100003],
    "all_tiny": [16, 17, 1, 0, 31, 64, 2, 5] * 40,
    "one_giant": [300001],
    "many_large": [20000 + 1237 * i for i in range(12)],
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("pairs", [False, True])
def test_segmented_matches_oracle(rs, oracle_lib, case, bits, pairs):
    sizes = CASES[case]
    off = np.zeros(len(sizes) + 1, dtype=np.uint64)
    off[1:] = np.cumsum(sizes)
    total = int(off[-1])
    print(f"case {case} bits={bits} pairs={pairs} total={total}", flush=True)
    keys = datagen.keys("bucket", total, bits, seed=len(sizes))
    keys[::3] = datagen.keys("uniform", keys[::3].size, bits, seed=7)
    vals = local_index(off, total, bits) if pairs else None
    gk, gv = run_seg(rs, keys, vals, off)
    ok, ov = oracle_lib.segmented_sort(keys, vals, off)
    assert np.array_equal(gk, ok)
    if pairs:
        assert np.array_equal(gv, ov)
        assert certify_segmented(keys, gk, gv, off) is None


@pytest.mark.parametrize("dist", datagen.DISTRIBUTIONS)
@pytest.mark.parametrize("bits", [32, 64])
def test_segmented_distributions(rs, oracle_lib, dist, bits):
    """Skewed inputs make whole waves share a digit (and partial last waves
    share one by chance): every distribution, every size class."""
    sizes = [17, 4000, 0, 9000, 16500, 1, 60482, 33333, 100000, 66]
    off = np.zeros(len(sizes) + 1, dtype=np.uint64)
    off[1:] = np.cumsum(sizes)
    total = int(off[-1])
    print(f"case dist={dist} bits={bits}", flush=True)
    keys = datagen.keys(dist, total, bits, seed=11)
    vals = local_index(off, total, bits)
    gk, gv = run_seg(rs, keys, vals, off)
    ok, ov = oracle_lib.segmented_sort(keys, vals, off)
    assert np.array_equal(gk, ok) and np.array_equal(gv, ov)


@pytest.mark.parametrize("bits", [32, 64])
def test_gaps_outside_segments_untouched(rs, oracle_lib, bits):
    """Segments need not cover the array: elements outside stay as they were
    in the output buffer."""
    total = 70000
    off = np.array([100, 5000, 5000, 40000, 69000], dtype=np.uint64)
    keys = datagen.keys("uniform", total, bits, seed=2)
    vals = datagen.keys("uniform", total, bits, seed=3)
    sent = 12345
    gk, gv = run_seg(rs, keys, vals, off, sentinel=sent)
    ok, ov = oracle_lib.segmented_sort(keys, vals, off)
    lo, hi = int(off[0]), int(off[-1])
    assert np.array_equal(gk[lo:hi], ok[lo:hi]) and np.array_equal(gv[lo:hi], ov[lo:hi])
    assert (gk[:lo] == sent).all() and (gk[hi:] == sent).all()
    assert (gv[:lo] == sent).all() and (gv[hi:] == sent).all()


@pytest.mark.parametrize("bits", [32, 64])
def test_in_place(rs, oracle_lib, bits):
    sizes = [3000, 0, 17000, 5, 40000, 9000]
    off = np.zeros(len(sizes) + 1, dtype=np.uint64)
    off[1:] = np.cumsum(sizes)
    total = int(off[-1])
    keys = datagen.keys("gaussian", total, bits, seed=4)
    vals = local_index(off, total, bits)
    gk, gv = run_seg(rs, keys, vals, off, in_place=True)
    ok, ov = oracle_lib.segmented_sort(keys, vals, off)
    assert np.array_equal(gk, ok) and np.array_equal(gv, ov)


def test_log_uniform_batch_certified(rs, oracle_lib):
    """2000 segments with log-uniform sizes in [16, 2^20] (the batched
    workload's size law at a tenth of its segment count): the segmented
    certificate on every element, the oracle on a sample of segments."""
    keys, vals, off = datagen.segmented(num_segments=2000, bits=32, seed=1)
    print(f"case log-uniform batch total={int(off[-1])}", flush=True)
    gk, gv = run_seg(rs, keys, vals, off)
    assert certify_segmented(keys, gk, gv, off) is None
    rng = np.random.RandomState(0)
    for s in rng.choice(2000, size=20, replace=False):
        a, b = int(off[s]), int(off[s + 1])
        ok, ov = oracle_lib.sort(keys[a:b], vals[a:b])
        assert np.array_equal(gk[a:b], ok) and np.array_equal(gv[a:b], ov)


def test_repeatable_with_caller_workspace(rs):
    keys, vals, off = datagen.segmented(num_segments=300, lo_log2=4, hi_log2=17, bits=64, seed=5)
    ctx = rs.context(0)
    ws = torch.empty(ctx.segmented_workspace_bytes(64, True, keys.size, 300), dtype=torch.uint8,
                     device="cuda")
    kd, vd = dev(keys), dev(vals)
    offd = dev(off.view(np.int64))
    outs = []
    for _ in range(2):
        ko, vo = rs.segmented_sort(kd, vd, offd, workspace=ws)
        torch.cuda.synchronize()
        outs.append((ko.cpu().numpy(), vo.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    assert certify_segmented(keys, outs[0][0], outs[0][1], off) is None


def certify_segmented_on_device(kin, kout, vout, offd, chunk=1 << 26):
    """The segmented certificate, computed on the device chunk by chunk
    (with value = index within the segment): every value lies in its
    segment, its input key equals the output key, and inside a segment the
    (key, value) pairs strictly increase.  Together these make each
    segment's values a permutation and its output the unique stable sort."""
    total = kin.numel()
    u = 0xFFFFFFFF
    for lo in range(0, total, chunk):
        hi = min(total, lo + chunk + 1)  # one element of overlap for the pairwise test
        idx = torch.arange(lo, hi, dtype=torch.int64, device="cuda")
        seg = torch.searchsorted(offd, idx, right=True) - 1
        start = offd[seg]
        size = offd[seg + 1] - start
        k = kout[lo:hi].to(torch.int64) & u
        v = vout[lo:hi].to(torch.int64) & u
        assert bool((v < size).all()), f"value outside its segment near {lo}"
        assert bool(((kin[start + v].to(torch.int64) & u) == k).all()), \
            f"key/value mismatch near {lo}"
        same = seg[1:] == seg[:-1]
        dk = k[1:] - k[:-1]
        dv = v[1:] - v[:-1]
        ok = (dk > 0) | ((dk == 0) & (dv > 0))
        assert bool((ok | ~same).all()), f"order broken inside a segment near {lo}"


def test_full_batch_20000_segments(rs, oracle_lib):
    """The batched workload at full size: 20,000 segments with log-uniform
    sizes in [16, 2^20] (about 1.9e9 pairs), uniform u32 keys, value = index
    within the segment.  Certified on the device on every element; a sample
    of segments (the largest, the smallest and random ones) against the
    oracle."""
    keys, vals, off = datagen.segmented(num_segments=20000, bits=32, seed=1)
    total = int(off[-1])
    print(f"case full segmented batch: 20000 segments, {total} pairs", flush=True)
    kd = torch.from_numpy(keys).cuda()
    vd = torch.from_numpy(vals).cuda()
    offd = torch.from_numpy(off.view(np.int64)).cuda()
    ctx = rs.context(0)
    ws = torch.empty(ctx.segmented_workspace_bytes(32, True, total, 20000), dtype=torch.uint8,
                     device="cuda")
    ko, vo = rs.segmented_sort(kd, vd, offd, ctx=ctx, workspace=ws)
    assert ctx.status(ws) == rs.RS_OK
    del ws
    certify_segmented_on_device(kd.view(torch.int32), ko.view(torch.int32), vo.view(torch.int32),
                                offd)
    sizes = np.diff(off.astype(np.int64))
    rng = np.random.RandomState(1)
    sample = set(rng.choice(20000, size=24, replace=False).tolist())
    sample |= {int(np.argmax(sizes)), int(np.argmin(sizes))}
    for s in sorted(sample):
        a, b = int(off[s]), int(off[s + 1])
        ok, ov = oracle_lib.sort(keys[a:b], vals[a:b])
        assert np.array_equal(ko[a:b].cpu().numpy(), ok), f"segment {s}"
        assert np.array_equal(vo[a:b].cpu().numpy(), ov), f"segment {s}"


@pytest.mark.parametrize("order,descending", [("unsigned", False), ("signed", True),
                                              ("float", False)])
@pytest.mark.parametrize("bits", [32, 64])
def test_trivial_and_skewed_passes_per_segment(rs, oracle_lib, order, descending, bits):
    """Large segments whose digits are the same for the whole segment at some
    passes (copied, not ranked) beside skewed and uniform ones, in one
    batch; with key orders, so the copy applies the order maps on the first
    and last pass."""
    n = 70001
    dt = np.uint32 if bits == 32 else np.uint64
    top = dt(bits - 8)
    parts = [
        datagen.keys("uniform", n, bits, seed=1),                  # every pass moves
        datagen.keys("uniform", n, bits, seed=2) & dt(0xFF),       # only the lowest digit moves
        datagen.keys("uniform", n, bits, seed=3) << top,           # only the top digit moves
        np.full(n, 12345, dtype=dt),                               # no pass moves
        datagen.keys("bucket", n, bits, seed=4),                   # skewed digits
        (datagen.keys("uniform", n, bits, seed=5) & dt(0xFF00)),   # only the second digit moves
    ]
    keys = np.concatenate(parts)
    off = np.arange(len(parts) + 1, dtype=np.uint64) * np.uint64(n)
    vals = local_index(off, keys.size, bits)
    print(f"case trivial/skewed segments bits={bits} order={order} desc={descending}", flush=True)
    kd, vd = dev(keys), dev(vals)
    ko, vo = rs.segmented_sort(kd, vd, dev(off.view(np.int64)), order=order,
                               descending=descending)
    torch.cuda.synchronize()
    ok, ov = oracle_lib.segmented_sort_ordered(keys, vals, off, order, descending)
    assert np.array_equal(ko.cpu().numpy(), ok) and np.array_equal(vo.cpu().numpy(), ov)
