"""The largest accepted sort, n = 2^30 - 1 elements, through the radix and
the merge path.  The oracle cannot run at this size, so the output is
checked on the device with the exact certificate of the stable sort (values
are input indices): every output value is an index whose input key equals
the output key, and the (key, value) pairs strictly increase.  Together
these mean the values are a permutation and the output is the stable sort."""
import pytest
import torch

pytestmark = pytest.mark.gpu

N = (1 << 30) - 1
CHUNK = 1 << 26


@pytest.fixture(scope="module")
def rs():
    import paper_1511_03404_amd as rs
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    rs.lib()
    return rs


def random_keys(n, mask, seed):
    """int32 tensor of n keys: 32 random bits per key, ANDed with mask (a
    narrow mask gives many equal keys and digits that are the same for all)."""
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    for lo in range(0, n, CHUNK):
        hi = min(n, lo + CHUNK)
        r = torch.randint(0, 1 << 32, (hi - lo,), dtype=torch.int64, device="cuda", generator=g)
        out[lo:hi] = ((r & mask) - ((r & mask) >> 31 << 32)).to(torch.int32)
    return out


def certify(kin, kout, vout):
    n = kin.numel()
    u = 0xFFFFFFFF
    for lo in range(0, n, CHUNK):
        hi = min(n, lo + CHUNK + 1)  # one element of overlap for the pairwise test
        k = kout[lo:hi].to(torch.int64) & u
        v = vout[lo:hi].to(torch.int64) & u
        assert bool((v < n).all()), f"value out of range near {lo}"
        assert bool(((kin[v].to(torch.int64) & u) == k).all()), f"key/value mismatch near {lo}"
        dk = k[1:] - k[:-1]
        dv = v[1:] - v[:-1]
        assert bool(((dk > 0) | ((dk == 0) & (dv > 0))).all()), f"order broken near {lo}"


@pytest.mark.parametrize("mask", [0xFFFFFFFF, 0x00FFFFFF])
def test_radix_sort_at_the_size_limit(rs, mask):
    print(f"case radix n={N} mask={mask:#x}", flush=True)
    kin = random_keys(N, mask, seed=1)
    vin = torch.arange(N, dtype=torch.int32, device="cuda")
    kout, vout = rs.sort_pairs(kin, vin)
    torch.cuda.synchronize()
    del vin
    certify(kin, kout, vout)


def test_merge_sort_at_the_size_limit(rs):
    print(f"case merge n={N}", flush=True)
    kin = random_keys(N, 0x00FFFFFF, seed=2)
    vin = torch.arange(N, dtype=torch.int32, device="cuda")
    kout, vout = rs.merge_sort(kin, vin)
    torch.cuda.synchronize()
    del vin
    certify(kin, kout, vout)
