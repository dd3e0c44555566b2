"""MI355X (gfx950) LSD radix sort: Python binding of ``librs.so``.

The binding only marshals arguments: every step of the sort runs in the HIP
kernels of ``csrc/``.  PyTorch supplies device memory and the current stream.
If the library has not been built, every call raises; there is no CPU path.

A 32-bit sort takes ``torch.uint32``, ``torch.int32`` or ``torch.float32``
tensors, a 64-bit sort ``torch.uint64``, ``torch.int64`` or ``torch.float64``.
The order is chosen with ``order``: "unsigned" (the bit pattern read as an
unsigned integer; the default for integer tensors), "signed" (two's
complement) or "float" (IEEE total order of the bit patterns; the default
for float tensors), and ``descending``.  Values have the key's width.  All
sorts are stable (paper, Section 2.6): equal keys keep their input order.
``merge_sort`` gives the same result by the stable merge sort of Section 2.4.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librs.so")

RS_OK = 0
RS_ERR_INVALID_ARGUMENT = 1
RS_ERR_UNSUPPORTED = 2
RS_ERR_OUT_OF_MEMORY = 3
RS_ERR_DEVICE = 4
RS_KEY_U32 = 0
RS_KEY_U64 = 1
RS_ORDER_SIGNED = 1
RS_ORDER_FLOAT = 2
RS_ORDER_DESCENDING = 4
ORDERS = {"unsigned": 0, "signed": RS_ORDER_SIGNED, "float": RS_ORDER_FLOAT}
MAX_ELEMENTS = 1 << 30
# sorts up to this many elements run in one workgroup's LDS (one launch),
# whatever configuration the tune table selects
BLOCK_SORT_CAP = {(32, False): 16384, (32, True): 16384, (64, False): 16384, (64, True): 8192}

EXPORTED = (
    "rs_context_create", "rs_context_destroy", "rs_workspace_bytes",
    "rs_sort_keys_u32", "rs_sort_keys_u64", "rs_sort_pairs_u32", "rs_sort_pairs_u64",
    "rs_segmented_sort", "rs_segmented_workspace_bytes", "rs_status_string", "rs_last_error",
    "rs_profile_enable", "rs_profile_tag", "rs_profile_reset", "rs_profile_read",
    "rs_config_count", "rs_config_get", "rs_tune_set", "rs_tune_get",
    "rs_sort", "rs_segmented_sort_order", "rs_merge_sort", "rs_merge_workspace_bytes",
    "rs_segmented_tiny_cap_set", "rs_segmented_tiny_cap_get",
    "rs_workspace_status", "rs_debug_wait_set", "rs_debug_sort_stages",
    "rs_sort_noalloc", "rs_sort_noalloc_scratch_bytes", "rs_segmented_config_count",
    "rs_device_copy",
)


class Config(ctypes.Structure):
    """``rs_config``: digit width and tile shape of the digit passes."""
    _fields_ = [("radix_bits", ctypes.c_int), ("threads", ctypes.c_int), ("items", ctypes.c_int)]

    def as_dict(self):
        return {"radix_bits": self.radix_bits, "threads": self.threads, "items": self.items}

_lib = None
_lib_lock = threading.Lock()


class RSError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"rs status {status}: {message}")
        self.status = status


def lib():
    """The loaded ``librs.so``; raises if it has not been built."""
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(
                    "librs.so is not built; run `python -m paper_1511_03404_amd.build` "
                    "(there is no CPU fallback)")
            L = ctypes.CDLL(LIB_PATH)
            vp, u64, u32, ci = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
            sz = ctypes.c_size_t
            L.rs_context_create.argtypes = [ci, ctypes.POINTER(vp)]
            L.rs_context_destroy.argtypes = [vp]
            L.rs_context_destroy.restype = None
            L.rs_workspace_bytes.argtypes = [vp, ci, ci, u64, ctypes.POINTER(sz)]
            L.rs_sort_keys_u32.argtypes = [vp, vp, vp, u64, vp, sz, vp]
            L.rs_sort_keys_u64.argtypes = [vp, vp, vp, u64, vp, sz, vp]
            L.rs_sort_pairs_u32.argtypes = [vp, vp, vp, vp, vp, u64, vp, sz, vp]
            L.rs_sort_pairs_u64.argtypes = [vp, vp, vp, vp, vp, u64, vp, sz, vp]
            L.rs_segmented_sort.argtypes = [vp, ci, vp, vp, vp, vp, vp, u32, u64, vp, sz, vp]
            L.rs_segmented_workspace_bytes.argtypes = [vp, ci, ci, u64, u32, ctypes.POINTER(sz)]
            L.rs_status_string.argtypes = [ci]
            L.rs_status_string.restype = ctypes.c_char_p
            L.rs_profile_enable.argtypes = [vp, ci]
            L.rs_profile_tag.argtypes = [vp, ci]
            L.rs_profile_reset.argtypes = [vp]
            L.rs_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_char_p),
                                          ctypes.POINTER(ci), ctypes.POINTER(ctypes.c_float),
                                          ci, ctypes.POINTER(ci)]
            L.rs_last_error.argtypes = []
            L.rs_last_error.restype = ctypes.c_char_p
            L.rs_config_count.argtypes = [ci, ci, ctypes.POINTER(ci)]
            L.rs_segmented_config_count.argtypes = [ci, ci, ctypes.POINTER(ci)]
            L.rs_segmented_config_count.restype = ci
            L.rs_device_copy.argtypes = [vp, vp, vp, u64, vp]
            L.rs_device_copy.restype = ci
            L.rs_config_get.argtypes = [ci, ci, ci, ctypes.POINTER(Config)]
            L.rs_tune_set.argtypes = [vp, ci, ci, ci, ci, ci]
            L.rs_tune_get.argtypes = [vp, ci, ci, ci, ci, ctypes.POINTER(ci)]
            L.rs_sort.argtypes = [vp, ci, u32, vp, vp, vp, vp, u64, vp, sz, vp]
            L.rs_segmented_sort_order.argtypes = [vp, ci, u32, vp, vp, vp, vp, vp, u32, u64, vp,
                                                  sz, vp]
            L.rs_merge_sort.argtypes = [vp, ci, u32, vp, vp, vp, vp, u64, vp, sz, vp]
            L.rs_merge_workspace_bytes.argtypes = [vp, ci, ci, u64, ctypes.POINTER(sz)]
            L.rs_segmented_tiny_cap_set.argtypes = [vp, u32]
            L.rs_segmented_tiny_cap_get.argtypes = [vp, ctypes.POINTER(u32)]
            L.rs_workspace_status.argtypes = [vp, vp, vp]
            L.rs_debug_wait_set.argtypes = [vp, u32, u32]
            L.rs_debug_sort_stages.argtypes = [vp, ci, vp, vp, vp, vp, u64, ci, vp, vp, sz, vp]
            L.rs_sort_noalloc.argtypes = [vp, ci, u32, vp, vp, vp, vp, u64, vp]
            L.rs_sort_noalloc.restype = ci
            L.rs_sort_noalloc_scratch_bytes.argtypes = []
            L.rs_sort_noalloc_scratch_bytes.restype = u64
            for name in ("rs_context_create", "rs_workspace_bytes", "rs_sort_keys_u32",
                         "rs_sort_keys_u64", "rs_sort_pairs_u32", "rs_sort_pairs_u64",
                         "rs_segmented_sort", "rs_segmented_workspace_bytes",
                         "rs_profile_enable", "rs_profile_tag", "rs_profile_reset",
                         "rs_profile_read", "rs_config_count", "rs_config_get",
                         "rs_tune_set", "rs_tune_get", "rs_sort", "rs_segmented_sort_order",
                         "rs_merge_sort", "rs_merge_workspace_bytes",
                         "rs_segmented_tiny_cap_set", "rs_segmented_tiny_cap_get",
                         "rs_workspace_status", "rs_debug_wait_set", "rs_debug_sort_stages"):
                getattr(L, name).restype = ci
            _lib = L
    return _lib


def _check(status: int):
    if status != RS_OK:
        msg = lib().rs_last_error().decode(errors="replace")
        raise RSError(status, msg)


class Context:
    """An ``rs_context`` bound to one HIP device."""

    def __init__(self, device: int | None = None):
        if device is None:
            device = torch.cuda.current_device() if torch.cuda.is_available() else 0
        self.device = int(device)
        h = ctypes.c_void_p()
        _check(lib().rs_context_create(self.device, ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().rs_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self, key_bits: int, has_values: bool, n: int) -> int:
        out = ctypes.c_size_t()
        kt = RS_KEY_U32 if key_bits == 32 else RS_KEY_U64
        _check(lib().rs_workspace_bytes(self.handle, kt, int(has_values), n, ctypes.byref(out)))
        return out.value

    def tiny_cap(self, cap: int | None = None) -> int:
        """Segments of 2 .. cap elements are sorted by a bitonic network per
        wave (cap <= 1024, 0 sends them to the one-workgroup radix sort).
        Sets the cap if given; returns the cap in force."""
        if cap is not None:
            _check(lib().rs_segmented_tiny_cap_set(self.handle, int(cap)))
        out = ctypes.c_uint32()
        _check(lib().rs_segmented_tiny_cap_get(self.handle, ctypes.byref(out)))
        return out.value

    def merge_workspace_bytes(self, key_bits: int, has_values: bool, n: int) -> int:
        out = ctypes.c_size_t()
        kt = RS_KEY_U32 if key_bits == 32 else RS_KEY_U64
        _check(lib().rs_merge_workspace_bytes(self.handle, kt, int(has_values), n,
                                              ctypes.byref(out)))
        return out.value

    def segmented_workspace_bytes(self, key_bits: int, has_values: bool, total: int,
                                  num_segments: int) -> int:
        out = ctypes.c_size_t()
        kt = RS_KEY_U32 if key_bits == 32 else RS_KEY_U64
        _check(lib().rs_segmented_workspace_bytes(self.handle, kt, int(has_values), total,
                                                  num_segments, ctypes.byref(out)))
        return out.value

    # -- tune table (configuration per kind and size class) --------------
    def tune_set(self, key_bits: int, has_values: bool, segmented: bool, size_log2: int,
                 index: int):
        """Use configuration ``index`` (-1: the default) for sorts of this kind
        with ceil(log2 n) == size_log2 (-1: every size)."""
        kt = RS_KEY_U32 if key_bits == 32 else RS_KEY_U64
        _check(lib().rs_tune_set(self.handle, kt, int(has_values), int(segmented),
                                 int(size_log2), int(index)))

    def tune_get(self, key_bits: int, has_values: bool, segmented: bool, size_log2: int) -> int:
        kt = RS_KEY_U32 if key_bits == 32 else RS_KEY_U64
        out = ctypes.c_int()
        _check(lib().rs_tune_get(self.handle, kt, int(has_values), int(segmented),
                                 int(size_log2), ctypes.byref(out)))
        return out.value

    # -- device-side errors ----------------------------------------------
    def status(self, workspace: torch.Tensor | None = None) -> int:
        """Device-side status of the last sort that used ``workspace`` (None:
        the context's own scratch of the current stream): synchronises the
        current stream and returns the rs status code (RS_OK = 0)."""
        return lib().rs_workspace_status(self.handle, _ptr(workspace), _stream(self.device))

    def check(self, workspace: torch.Tensor | None = None):
        """Raise RSError if the last sort on ``workspace`` failed on the device
        (a segment of 2^30 or more elements, or a wait that gave up)."""
        _check(self.status(workspace))

    def debug_wait_set(self, spin_limit: int, stall: int = 0):
        """Test only: bound of the waits on other workgroups and the stall
        bits (1: look-back, 2: tile claims) that force those waits to their
        bound."""
        _check(lib().rs_debug_wait_set(self.handle, int(spin_limit), int(stall)))

    # -- per-kernel timing (HIP events around each launch) ---------------
    def profile_enable(self, on: bool = True):
        _check(lib().rs_profile_enable(self.handle, int(on)))

    def profile_tag(self, tag: int):
        _check(lib().rs_profile_tag(self.handle, int(tag)))

    def profile_reset(self):
        _check(lib().rs_profile_reset(self.handle))

    def profile_read(self):
        """List of (kernel name, tag, milliseconds); synchronises."""
        count = ctypes.c_int()
        _check(lib().rs_profile_read(self.handle, None, None, None, 0, ctypes.byref(count)))
        m = count.value
        if m == 0:
            return []
        names = (ctypes.c_char_p * m)()
        tags = (ctypes.c_int * m)()
        ms = (ctypes.c_float * m)()
        _check(lib().rs_profile_read(self.handle, names, tags, ms, m, ctypes.byref(count)))
        return [(names[i].decode(), tags[i], ms[i]) for i in range(m)]


def configs(key_bits: int, has_values: bool, segmented: bool = False) -> list[dict]:
    """The compiled digit-pass configurations for this kind, in index order
    (index 0 is the default); segmented=True: those the segmented sort can
    use (a prefix of the list)."""
    kt = RS_KEY_U32 if key_bits == 32 else RS_KEY_U64
    n = ctypes.c_int()
    f = lib().rs_segmented_config_count if segmented else lib().rs_config_count
    _check(f(kt, int(has_values), ctypes.byref(n)))
    out = []
    for i in range(n.value):
        c = Config()
        _check(lib().rs_config_get(kt, int(has_values), i, ctypes.byref(c)))
        out.append(c.as_dict())
    return out


def size_class(n: int) -> int:
    """ceil(log2 n): the tune table's size class of a sort of n elements."""
    return max(0, int(n - 1).bit_length()) if n > 1 else 0


_contexts: dict[int, Context] = {}


def context(device: int | None = None) -> Context:
    """Process-wide default context of a device."""
    if device is None:
        device = torch.cuda.current_device()
    c = _contexts.get(device)
    if c is None:
        c = _contexts[device] = Context(device)
    return c


_BITS = {torch.uint32: 32, torch.int32: 32, torch.float32: 32,
         torch.uint64: 64, torch.int64: 64, torch.float64: 64}


def key_bits(t: torch.Tensor) -> int:
    b = _BITS.get(t.dtype)
    if b is None:
        raise TypeError(f"unsupported dtype {t.dtype}; use (u)int32/float32 or (u)int64/float64")
    return b


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(device: int):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_tensor(t: torch.Tensor, name: str, bits: int, n: int):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if key_bits(t) != bits:
        raise TypeError(f"{name} must have the keys' width ({bits} bits)")
    if t.numel() != n or not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous with {n} elements")


def _order_flags(keys: torch.Tensor, order, descending: bool) -> int:
    if order is None:
        order = "float" if keys.dtype in (torch.float32, torch.float64) else "unsigned"
    if order not in ORDERS:
        raise ValueError(f"order must be one of {sorted(ORDERS)}")
    return ORDERS[order] | (RS_ORDER_DESCENDING if descending else 0)


def _workspace(ctx: Context, nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)


def sort_keys(keys: torch.Tensor, out: torch.Tensor | None = None, *, ctx: Context | None = None,
              workspace: torch.Tensor | None = None, order: str | None = None,
              descending: bool = False) -> torch.Tensor:
    """Stable sort of a 1-D key tensor (ascending unless ``descending``; see
    the module docstring for ``order``).  ``out`` may be ``keys`` (in
    place).  Asynchronous on the current stream."""
    bits = key_bits(keys)
    n = keys.numel()
    _check_tensor(keys, "keys", bits, n)
    if out is None:
        out = torch.empty_like(keys)
    _check_tensor(out, "out", bits, n)
    ctx = ctx or context(keys.device.index)
    if n == 0:
        return out
    flags = _order_flags(keys, order, descending)
    need = ctx.workspace_bytes(bits, False, n)
    ws = workspace if workspace is not None else _workspace(ctx, need, keys.device)
    if flags:
        kt = RS_KEY_U32 if bits == 32 else RS_KEY_U64
        _check(lib().rs_sort(ctx.handle, kt, flags, _ptr(keys), None, _ptr(out), None, n,
                             _ptr(ws), ws.numel(), _stream(ctx.device)))
        return out
    f = lib().rs_sort_keys_u32 if bits == 32 else lib().rs_sort_keys_u64
    _check(f(ctx.handle, _ptr(keys), _ptr(out), n, _ptr(ws), ws.numel(), _stream(ctx.device)))
    return out


def sort_pairs(keys: torch.Tensor, values: torch.Tensor, keys_out: torch.Tensor | None = None,
               values_out: torch.Tensor | None = None, *, ctx: Context | None = None,
               workspace: torch.Tensor | None = None, order: str | None = None,
               descending: bool = False):
    """Stable sort of (key, value) pairs by key.  Returns (keys_out, values_out)."""
    bits = key_bits(keys)
    n = keys.numel()
    _check_tensor(keys, "keys", bits, n)
    _check_tensor(values, "values", bits, n)
    keys_out = torch.empty_like(keys) if keys_out is None else keys_out
    values_out = torch.empty_like(values) if values_out is None else values_out
    _check_tensor(keys_out, "keys_out", bits, n)
    _check_tensor(values_out, "values_out", bits, n)
    ctx = ctx or context(keys.device.index)
    if n == 0:
        return keys_out, values_out
    flags = _order_flags(keys, order, descending)
    need = ctx.workspace_bytes(bits, True, n)
    ws = workspace if workspace is not None else _workspace(ctx, need, keys.device)
    if flags:
        kt = RS_KEY_U32 if bits == 32 else RS_KEY_U64
        _check(lib().rs_sort(ctx.handle, kt, flags, _ptr(keys), _ptr(values), _ptr(keys_out),
                             _ptr(values_out), n, _ptr(ws), ws.numel(), _stream(ctx.device)))
        return keys_out, values_out
    f = lib().rs_sort_pairs_u32 if bits == 32 else lib().rs_sort_pairs_u64
    _check(f(ctx.handle, _ptr(keys), _ptr(values), _ptr(keys_out), _ptr(values_out), n,
             _ptr(ws), ws.numel(), _stream(ctx.device)))
    return keys_out, values_out


def segmented_sort(keys: torch.Tensor, values: torch.Tensor | None, offsets: torch.Tensor,
                   keys_out: torch.Tensor | None = None, values_out: torch.Tensor | None = None,
                   *, ctx: Context | None = None, workspace: torch.Tensor | None = None,
                   order: str | None = None, descending: bool = False):
    """Sort every segment [offsets[s], offsets[s+1]) on its own, in one batch.
    ``offsets`` is a device int64/uint64 tensor of num_segments + 1 entries."""
    bits = key_bits(keys)
    n = keys.numel()
    _check_tensor(keys, "keys", bits, n)
    has_v = values is not None
    if has_v:
        _check_tensor(values, "values", bits, n)
    if offsets.dtype not in (torch.int64, torch.uint64) or not offsets.is_cuda \
            or not offsets.is_contiguous() or offsets.numel() < 1:
        raise ValueError("offsets must be a contiguous device int64 tensor of S+1 entries")
    keys_out = torch.empty_like(keys) if keys_out is None else keys_out
    _check_tensor(keys_out, "keys_out", bits, n)
    if has_v:
        values_out = torch.empty_like(values) if values_out is None else values_out
        _check_tensor(values_out, "values_out", bits, n)
    else:
        values_out = None
    ctx = ctx or context(keys.device.index)
    nseg = offsets.numel() - 1
    kt = RS_KEY_U32 if bits == 32 else RS_KEY_U64
    need = ctx.segmented_workspace_bytes(bits, has_v, n, nseg)
    ws = workspace if workspace is not None else _workspace(ctx, need, keys.device)
    flags = _order_flags(keys, order, descending)
    _check(lib().rs_segmented_sort_order(ctx.handle, kt, flags, _ptr(keys), _ptr(values),
                                         _ptr(keys_out), _ptr(values_out), _ptr(offsets), nseg, n,
                                         _ptr(ws), ws.numel(), _stream(ctx.device)))
    return keys_out, values_out


def merge_sort(keys: torch.Tensor, values: torch.Tensor | None = None,
               keys_out: torch.Tensor | None = None, values_out: torch.Tensor | None = None, *,
               ctx: Context | None = None, workspace: torch.Tensor | None = None,
               order: str | None = None, descending: bool = False):
    """Stable merge sort (the comparison-based counterpart of sort_keys /
    sort_pairs, same result).  Returns keys_out, or (keys_out, values_out)
    when values are given.  Asynchronous on the current stream."""
    bits = key_bits(keys)
    n = keys.numel()
    _check_tensor(keys, "keys", bits, n)
    has_v = values is not None
    if has_v:
        _check_tensor(values, "values", bits, n)
    keys_out = torch.empty_like(keys) if keys_out is None else keys_out
    _check_tensor(keys_out, "keys_out", bits, n)
    if has_v:
        values_out = torch.empty_like(values) if values_out is None else values_out
        _check_tensor(values_out, "values_out", bits, n)
    else:
        values_out = None
    ctx = ctx or context(keys.device.index)
    if n:
        flags = _order_flags(keys, order, descending)
        ws = workspace if workspace is not None else _workspace(
            ctx, ctx.merge_workspace_bytes(bits, has_v, n), keys.device)
        kt = RS_KEY_U32 if bits == 32 else RS_KEY_U64
        _check(lib().rs_merge_sort(ctx.handle, kt, flags, _ptr(keys), _ptr(values),
                                   _ptr(keys_out), _ptr(values_out), n, _ptr(ws), ws.numel(),
                                   _stream(ctx.device)))
    return (keys_out, values_out) if has_v else keys_out


def sort_stages(keys: torch.Tensor, values: torch.Tensor | None = None, passes: int = 0, *,
                ctx: Context | None = None):
    """Test only: the plain radix sort's kernels up to digit position
    ``passes`` (rs_debug_sort_stages), with the configuration the tune table
    selects.  Returns (the digit histograms as a device uint32 tensor
    [d, 2^r], the keys after those passes, the values after them or None)."""
    bits = key_bits(keys)
    n = keys.numel()
    _check_tensor(keys, "keys", bits, n)
    has_v = values is not None
    if has_v:
        _check_tensor(values, "values", bits, n)
    ctx = ctx or context(keys.device.index)
    kt = RS_KEY_U32 if bits == 32 else RS_KEY_U64
    cfg = configs(bits, has_v)[ctx.tune_get(bits, has_v, False, size_class(n))]
    r = cfg["radix_bits"]
    d = (bits + r - 1) // r
    hist = torch.zeros((d, 1 << r), dtype=torch.uint32, device=keys.device)
    ko = torch.empty_like(keys)
    vo = torch.empty_like(values) if has_v else None
    ws = _workspace(ctx, ctx.workspace_bytes(bits, has_v, n), keys.device)
    _check(lib().rs_debug_sort_stages(ctx.handle, kt, _ptr(keys), _ptr(values), _ptr(ko),
                                      _ptr(vo), n, int(passes), _ptr(hist), _ptr(ws), ws.numel(),
                                      _stream(ctx.device)))
    return hist, ko, vo


def device_copy(src: torch.Tensor, dst: torch.Tensor, *, ctx: Context | None = None):
    """Measurement helper: the library's plain copy of src into dst (device
    tensors of the same byte size, a multiple of 16)."""
    if not (src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("contiguous device tensors required")
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("src and dst must have the same byte size")
    ctx = ctx or context(src.device.index)
    _check(lib().rs_device_copy(ctx.handle, _ptr(src), _ptr(dst), nbytes, _stream(ctx.device)))
    return dst
