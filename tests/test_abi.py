"""C-ABI of librs.so on the CPU: every symbol declared in include/rs.h is
exported, and argument errors are rejected on the host before any HIP call
(so they can be checked without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def rs():
    import paper_1511_03404_amd as rs
    if not os.path.exists(rs.LIB_PATH):
        from paper_1511_03404_amd import build
        build.build()
    return rs


def declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            names += re.findall(r"^\s*(?:rs_status|void|uint64_t|const char \*)\s*\*?\s*(rs_\w+)\s*\(",
                                text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("rs_sort_keys_u32", "rs_sort_keys_u64", "rs_sort_pairs_u32",
                 "rs_sort_pairs_u64", "rs_segmented_sort"):
        assert want in names


def test_every_declared_symbol_is_exported(rs):
    L = ctypes.CDLL(rs.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(declared_functions()) <= set(rs.EXPORTED) | {"rs_segmented_workspace_bytes"}


@pytest.fixture()
def ctx(rs):
    c = rs.Context(0)
    yield c
    c.close()


def call_keys(rs, ctx, kin, kout, n, ws=None, ws_bytes=0, bits=32):
    f = rs.lib().rs_sort_keys_u32 if bits == 32 else rs.lib().rs_sort_keys_u64
    return f(ctx.handle, kin, kout, n, ws, ws_bytes, None)


def test_context_and_workspace_need_no_gpu(rs, ctx):
    a = ctx.workspace_bytes(32, False, 1 << 20)
    b = ctx.workspace_bytes(32, True, 1 << 20)
    c = ctx.workspace_bytes(64, True, 1 << 20)
    assert 0 < a < b < c
    assert b >= (1 << 20) * 8  # one ping-pong copy of keys and values
    assert ctx.workspace_bytes(32, False, 0) > 0
    with pytest.raises(rs.RSError) as e:
        ctx.workspace_bytes(32, False, 1 << 30)
    assert e.value.status == rs.RS_ERR_UNSUPPORTED


def test_argument_errors(rs, ctx):
    L = rs.lib()
    fake = 0x7F0000000000  # never dereferenced: validation rejects first
    # n = 0 is a no-op even with NULL pointers
    assert call_keys(rs, ctx, None, None, 0) == rs.RS_OK
    assert call_keys(rs, ctx, None, fake, 10) == rs.RS_ERR_INVALID_ARGUMENT
    assert b"NULL" in L.rs_last_error()
    assert call_keys(rs, ctx, fake + 2, fake + 4096, 10) == rs.RS_ERR_INVALID_ARGUMENT
    assert b"aligned" in L.rs_last_error()
    assert call_keys(rs, ctx, fake, fake + 4, 8, bits=64) == rs.RS_ERR_INVALID_ARGUMENT
    # partial overlap of in and out
    assert call_keys(rs, ctx, fake, fake + 16, 100) == rs.RS_ERR_INVALID_ARGUMENT
    assert b"overlap" in L.rs_last_error()
    # too many elements
    assert call_keys(rs, ctx, fake, fake + (1 << 33), 1 << 30) == rs.RS_ERR_UNSUPPORTED
    # workspace too small / misaligned / overlapping
    need = ctx.workspace_bytes(32, False, 1000)
    ws = fake + (1 << 34)
    assert call_keys(rs, ctx, fake, fake + 8192, 1000, ws, need - 1) == rs.RS_ERR_INVALID_ARGUMENT
    assert b"workspace" in L.rs_last_error()
    assert call_keys(rs, ctx, fake, fake + 8192, 1000, ws + 4, need) == rs.RS_ERR_INVALID_ARGUMENT
    assert call_keys(rs, ctx, fake, fake + 8192, 1000, fake + 256, need) == rs.RS_ERR_INVALID_ARGUMENT
    # pairs: keys and values must not overlap
    f = L.rs_sort_pairs_u32
    assert f(ctx.handle, fake, fake + 8, fake + 8192, fake + 16384, 100, None, 0, None) \
        == rs.RS_ERR_INVALID_ARGUMENT
    assert f(ctx.handle, fake, None, fake + 8192, fake + 16384, 100, None, 0, None) \
        == rs.RS_ERR_INVALID_ARGUMENT
    # NULL context
    assert L.rs_sort_keys_u32(None, fake, fake + 8192, 10, None, 0, None) == rs.RS_ERR_INVALID_ARGUMENT


def test_status_strings(rs):
    L = rs.lib()
    for s in range(5):
        assert L.rs_status_string(s)
    assert L.rs_status_string(99) == b"unknown status"


def test_python_binding_rejects_host_tensors(rs):
    import torch
    with pytest.raises(ValueError):
        rs.sort_keys(torch.zeros(4, dtype=torch.int32))
    with pytest.raises(TypeError):
        rs.key_bits(torch.zeros(4, dtype=torch.float16))


def test_compiled_configurations(rs):
    """Every kind has its list: the default (index 0) at 8-bit digits, every
    digit width of 4..8 bits and 11-bit digits, tiles within one workgroup's
    limits; the segmented sort's list is the prefix without the wide digits."""
    for bits in (32, 64):
        for pairs in (False, True):
            cfgs = rs.configs(bits, pairs)
            seg = rs.configs(bits, pairs, segmented=True)
            assert cfgs[0]["radix_bits"] == 8
            assert {c["radix_bits"] for c in cfgs} == {4, 5, 6, 7, 8, 11}
            assert seg == cfgs[:len(seg)] and {c["radix_bits"] for c in seg} == {4, 5, 6, 7, 8}
            for c in cfgs:
                assert 256 <= c["threads"] <= 1024 and c["threads"] % 64 == 0
                assert c["threads"] * c["items"] * bits // 8 <= 128 * 1024
                if c["radix_bits"] <= 8:
                    # the lane-mask tables fit the staging
                    assert c["items"] >= 2 ** c["radix_bits"] // 32
                else:
                    # two digits per thread; tile positions are 16-bit
                    assert c["threads"] == 1024 and c["threads"] * c["items"] <= 1 << 16
    assert rs.configs(64, True)[0]["threads"] == 512  # registers of 16 u64 pairs per thread
    L = rs.lib()
    cnt = ctypes.c_int()
    assert L.rs_config_count(7, 0, ctypes.byref(cnt)) == rs.RS_ERR_INVALID_ARGUMENT
    assert L.rs_config_count(0, 0, None) == rs.RS_ERR_INVALID_ARGUMENT
    c = rs.Config()
    assert L.rs_config_get(0, 0, 99, ctypes.byref(c)) == rs.RS_ERR_INVALID_ARGUMENT
    assert L.rs_config_get(0, 0, -1, ctypes.byref(c)) == rs.RS_ERR_INVALID_ARGUMENT


def test_tune_table(rs, ctx):
    """Per kind, plain/segmented and size class; -1 resets; the workspace
    size follows the selected configuration."""
    assert ctx.tune_get(32, True, False, 26) == 0
    w0 = ctx.workspace_bytes(32, True, 1 << 26)
    cfgs = rs.configs(32, True)
    small = min(range(len(cfgs)), key=lambda i: cfgs[i]["threads"] * cfgs[i]["items"])
    ctx.tune_set(32, True, False, 26, small)
    assert ctx.tune_get(32, True, False, 26) == small
    assert ctx.tune_get(32, True, False, 25) == 0
    assert ctx.tune_get(32, True, True, 26) == 0
    assert ctx.tune_get(32, False, False, 25) == 0
    c32k = rs.configs(32, False)[ctx.tune_get(32, False, False, 26)]
    assert (c32k["threads"], c32k["items"], c32k["radix_bits"]) == (1024, 24, 8)
    c64p = rs.configs(64, True)[ctx.tune_get(64, True, False, 26)]
    assert (c64p["threads"], c64p["items"]) == (1024, 8)
    # smaller tiles: more look-back words in the workspace
    assert ctx.workspace_bytes(32, True, 1 << 26) > w0
    assert ctx.workspace_bytes(32, True, 1 << 25) == ctx.workspace_bytes(32, True, 1 << 25)
    wide = [i for i, c in enumerate(cfgs) if c["radix_bits"] == 11][0]
    with pytest.raises(rs.RSError):
        ctx.tune_set(32, True, True, -1, wide)  # the segmented sort has no wide digits
    ctx.tune_set(32, True, False, 26, wide)
    assert ctx.tune_get(32, True, False, 26) == wide
    ctx.tune_set(32, True, False, 26, -1)
    r4 = [i for i, c in enumerate(cfgs) if c["radix_bits"] == 4][0]
    ctx.tune_set(32, True, True, -1, r4)
    for cls in (0, 17, 39):
        assert ctx.tune_get(32, True, True, cls) == r4
    ctx.tune_set(32, True, True, -1, -1)
    assert ctx.tune_get(32, True, True, 17) == 0
    ctx.tune_set(32, True, False, 26, -1)
    # built-in choices of unset plain-sort classes: 1024 x 8 tiles up to 2^21
    # (64-bit pairs: 512 x 8 up to 2^19, 1024 x 8 above), the list's default
    # above (32-bit keys alone: 1024 x 24 from 2^26 on)
    for bits, pairs in ((32, False), (32, True), (64, False), (64, True)):
        c = rs.configs(bits, pairs)
        big = 39 if (bits, pairs) == (64, True) else 21
        for cls in ((20, 25, big) if (bits, pairs) == (64, True) else (0, 15, 17, big)):
            i = ctx.tune_get(bits, pairs, False, cls)
            assert (c[i]["threads"], c[i]["items"], c[i]["radix_bits"]) == (1024, 8, 8), (bits, pairs, cls)
        if (bits, pairs) == (64, True):
            for cls in (15, 19):
                i = ctx.tune_get(bits, pairs, False, cls)
                assert (c[i]["threads"], c[i]["items"]) == (512, 8), cls
        if big < 39:
            assert ctx.tune_get(bits, pairs, False, big + 1) == 0
        if (bits, pairs) == (32, False):
            for cls in (26, 30, 39):
                i = ctx.tune_get(bits, pairs, False, cls)
                assert (c[i]["threads"], c[i]["items"]) == (1024, 24), cls
        assert ctx.tune_get(bits, pairs, True, 17) == 0
    assert ctx.workspace_bytes(32, True, 1 << 26) == w0
    L = rs.lib()
    assert L.rs_tune_set(ctx.handle, 0, 1, 0, 40, 0) == rs.RS_ERR_INVALID_ARGUMENT
    assert L.rs_tune_set(ctx.handle, 0, 1, 0, 5, len(cfgs)) == rs.RS_ERR_INVALID_ARGUMENT
    assert L.rs_tune_set(ctx.handle, 2, 1, 0, 5, 0) == rs.RS_ERR_INVALID_ARGUMENT
    assert L.rs_tune_set(None, 0, 1, 0, 5, 0) == rs.RS_ERR_INVALID_ARGUMENT
    idx = ctypes.c_int()
    assert L.rs_tune_get(ctx.handle, 0, 1, 0, -1, ctypes.byref(idx)) == rs.RS_ERR_INVALID_ARGUMENT


def test_size_class(rs):
    assert [rs.size_class(n) for n in (0, 1, 2, 3, 4, 5, 1 << 26, (1 << 26) + 1)] == \
        [0, 0, 1, 2, 2, 3, 26, 27]


def test_tune_cache_round_trip(rs, ctx, tmp_path):
    """Saved tuning results load into another context; an entry whose
    configuration no longer matches the library's list is skipped."""
    from paper_1511_03404_amd import tune
    cfgs = rs.configs(64, False)
    good = {"key_bits": 64, "has_values": False, "segmented": True, "size_log2": 30,
            "n": 1 << 30, "index": 3, "config": cfgs[3], "ms": {}}
    stale = dict(good, size_log2=29, config=dict(cfgs[3], threads=999))
    path = tmp_path / "tune.json"
    tune.save([good, stale], str(path), "test")
    assert tune.load(str(path), ctx) == 1
    assert ctx.tune_get(64, False, True, 30) == 3
    assert ctx.tune_get(64, False, True, 29) == 0


def test_order_flag_errors(rs, ctx):
    """rs_sort and rs_segmented_sort_order reject contradictory or unknown
    order flags before any HIP call; the Python binding rejects unknown
    order names."""
    import torch
    L = rs.lib()
    fake = 0x7F0000000000
    need = ctx.workspace_bytes(32, False, 1000)
    ws = fake + (1 << 34)
    flags = rs.RS_ORDER_SIGNED | rs.RS_ORDER_FLOAT
    assert L.rs_sort(ctx.handle, 0, flags, fake, None, fake + 8192, None, 1000, ws, need,
                     None) == rs.RS_ERR_INVALID_ARGUMENT
    assert b"exclude" in L.rs_last_error()
    assert L.rs_sort(ctx.handle, 0, 8, fake, None, fake + 8192, None, 1000, ws, need,
                     None) == rs.RS_ERR_INVALID_ARGUMENT
    assert b"unknown order" in L.rs_last_error()
    assert L.rs_sort(ctx.handle, 0, rs.RS_ORDER_DESCENDING, None, None, None, None, 0, None, 0,
                     None) == rs.RS_OK
    assert L.rs_sort(ctx.handle, 5, 0, fake, None, fake + 8192, None, 1000, ws, need,
                     None) == rs.RS_ERR_INVALID_ARGUMENT
    assert L.rs_segmented_sort_order(ctx.handle, 0, 16, fake, None, fake + 8192, None,
                                     fake + 65536, 1, 1000, ws, need, None) \
        == rs.RS_ERR_INVALID_ARGUMENT
    with pytest.raises(ValueError):
        rs._order_flags(torch.empty(4, dtype=torch.int32), "reversed", False)
    assert rs._order_flags(torch.empty(4, dtype=torch.float32), None, True) \
        == rs.RS_ORDER_FLOAT | rs.RS_ORDER_DESCENDING
    assert rs._order_flags(torch.empty(4, dtype=torch.int64), None, False) == 0


def test_merge_sort_argument_errors(rs, ctx):
    """rs_merge_sort validates on the host like rs_sort."""
    L = rs.lib()
    fake = 0x7F0000000000
    assert L.rs_merge_sort(ctx.handle, 0, 0, None, None, None, None, 0, None, 0, None) == rs.RS_OK
    assert L.rs_merge_sort(ctx.handle, 0, 0, None, None, fake, None, 10, None, 0, None) \
        == rs.RS_ERR_INVALID_ARGUMENT
    assert L.rs_merge_sort(ctx.handle, 0, 3, fake, None, fake + 8192, None, 10, None, 0, None) \
        == rs.RS_ERR_INVALID_ARGUMENT
    assert L.rs_merge_sort(ctx.handle, 0, 0, fake, fake + 8192, fake + 16384, None, 10, None, 0,
                           None) == rs.RS_ERR_INVALID_ARGUMENT
    assert L.rs_merge_sort(ctx.handle, 0, 0, fake, None, fake + 16, None, 100, None, 0, None) \
        == rs.RS_ERR_INVALID_ARGUMENT
    assert b"overlap" in L.rs_last_error()
    assert L.rs_merge_sort(ctx.handle, 0, 0, fake, None, fake + (1 << 33), None, 1 << 30, None,
                           0, None) == rs.RS_ERR_UNSUPPORTED
    need = ctx.merge_workspace_bytes(32, True, 100000)
    assert need >= 100000 * 8
    assert ctx.merge_workspace_bytes(64, False, 8192) > 0
    ws = fake + (1 << 34)
    assert L.rs_merge_sort(ctx.handle, 0, 0, fake, fake + (1 << 20), fake + (1 << 21),
                           fake + (1 << 22), 100000, ws, need - 1, None) \
        == rs.RS_ERR_INVALID_ARGUMENT
    assert b"workspace" in L.rs_last_error()


def test_tiny_cap_setting(rs, ctx):
    L = rs.lib()
    assert ctx.tiny_cap() == 1024
    assert ctx.tiny_cap(0) == 0
    assert ctx.tiny_cap(1) == 0  # a cap below 2 turns the class off
    assert ctx.tiny_cap(777) == 777
    assert L.rs_segmented_tiny_cap_set(ctx.handle, 1025) == rs.RS_ERR_INVALID_ARGUMENT
    assert L.rs_segmented_tiny_cap_set(None, 8) == rs.RS_ERR_INVALID_ARGUMENT
    assert ctx.tiny_cap() == 777


def test_status_query_and_test_entry_points_validate_on_the_host(rs, ctx):
    """The device-status query and the test entry points reject bad
    arguments before any HIP call; a status query with no sort run on the
    context's own scratch is RS_OK without touching the device."""
    L = rs.lib()
    fake = 0x7F0000000000
    assert L.rs_workspace_status(None, None, None) == rs.RS_ERR_INVALID_ARGUMENT
    assert L.rs_workspace_status(ctx.handle, fake + 16, None) == rs.RS_ERR_INVALID_ARGUMENT
    assert b"aligned" in L.rs_last_error()
    assert L.rs_workspace_status(ctx.handle, None, None) == rs.RS_OK
    assert L.rs_debug_wait_set(ctx.handle, 0, 0) == rs.RS_ERR_INVALID_ARGUMENT
    assert L.rs_debug_wait_set(ctx.handle, 16, 4) == rs.RS_ERR_INVALID_ARGUMENT
    assert b"stall" in L.rs_last_error()
    assert L.rs_debug_wait_set(ctx.handle, 16, 3) == rs.RS_OK
    assert L.rs_debug_wait_set(ctx.handle, 1 << 22, 0) == rs.RS_OK
    st = L.rs_debug_sort_stages
    assert st(ctx.handle, 0, fake, None, fake + (1 << 20), None, 100, -1, None, None, 0,
              None) == rs.RS_ERR_INVALID_ARGUMENT
    assert st(ctx.handle, 7, fake, None, fake + (1 << 20), None, 100, 1, None, None, 0,
              None) == rs.RS_ERR_INVALID_ARGUMENT
    assert st(ctx.handle, 0, fake, fake + (1 << 21), fake + (1 << 20), None, 100, 1, None, None,
              0, None) == rs.RS_ERR_INVALID_ARGUMENT
    assert st(ctx.handle, 0, None, None, None, None, 0, 2, None, None, 0, None) == rs.RS_OK


def test_noalloc_rejects_what_its_scratch_cannot_hold(rs, ctx):
    """rs_sort_noalloc validates on the host: sizes whose workspace exceeds
    the fixed scratch are refused before any HIP call."""
    L = rs.lib()
    fake = 0x7F0000000000
    cap = L.rs_sort_noalloc_scratch_bytes()
    assert cap == 64 << 20
    n = 1 << 24  # 32-bit pairs: 128 MiB of ping-pong copy alone
    assert ctx.workspace_bytes(32, True, n) > cap
    assert L.rs_sort_noalloc(ctx.handle, 0, 0, fake, fake + (1 << 28), fake + (2 << 28),
                             fake + (3 << 28), n, None) == rs.RS_ERR_UNSUPPORTED
    assert b"scratch" in L.rs_last_error()
    assert L.rs_sort_noalloc(ctx.handle, 0, 0, fake, None, fake + (1 << 28), fake, 10,
                             None) == rs.RS_ERR_INVALID_ARGUMENT
    assert L.rs_sort_noalloc(None, 0, 0, fake, None, fake, None, 10,
                             None) == rs.RS_ERR_INVALID_ARGUMENT
    assert L.rs_sort_noalloc(ctx.handle, 0, 0, None, None, None, None, 0, None) == rs.RS_OK


def test_device_copy_validates_on_the_host(rs, ctx):
    L = rs.lib()
    fake = 0x7F0000000000
    assert L.rs_device_copy(ctx.handle, None, None, 0, None) == rs.RS_OK
    assert L.rs_device_copy(None, fake, fake + (1 << 20), 16, None) == rs.RS_ERR_INVALID_ARGUMENT
    assert L.rs_device_copy(ctx.handle, fake, fake + (1 << 20), 24, None) == \
        rs.RS_ERR_INVALID_ARGUMENT
    assert L.rs_device_copy(ctx.handle, fake + 8, fake + (1 << 20), 16, None) == \
        rs.RS_ERR_INVALID_ARGUMENT
    assert L.rs_device_copy(ctx.handle, fake, fake + 64, 128, None) == rs.RS_ERR_INVALID_ARGUMENT
    assert b"overlap" in L.rs_last_error()
