"""Elementwise primality of uint64 arrays on MI355X (gfx950).

A thin ctypes binding over ``libisprime.so`` (built from ``csrc/`` by
``_build.py``): argument marshalling only.  Every step of the computation
runs in the library's HIP kernels; there is no CPU path.  PyTorch supplies
device memory and streams.

    >>> import torch, paper_2108_04791_amd as isp
    >>> isp.isprime(torch.tensor([1, 2, 3, 4, 5], dtype=torch.uint64, device="cuda"))
    tensor([False,  True,  True, False,  True], device='cuda:0')

The inputs and outputs follow the paper's isprime_fast (section 1): an array
of any shape in, a logical array of the same shape out.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libisprime.so")

ISP_OK = 0
ISP_EINVAL = -1
ISP_ENOMEM = -2
ISP_EDEVICE = -3
ISP_EBUSY = -4
ISP_ETIMEDOUT = -5
ISP_ENOENT = -6
ISP_ERANGE = -7
ISP_ENOINIT = -8

_lib = None
_lock = threading.Lock()


class IsprimeError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        msg = "%s failed: %s (%d)" % (what, _strerror(status), status)
        if status == ISP_EDEVICE and _lib is not None:
            msg += ", hipError %d" % _lib.isp_last_device_error()
        super().__init__(msg)


class Config(ctypes.Structure):
    """Launch and algorithm parameters (mirrors isp_config); 0 = default."""
    _fields_ = [
        ("classify_block", ctypes.c_int32),
        ("classify_ept", ctypes.c_int32),
        ("classify_blocks_per_cu", ctypes.c_int32),
        ("filter_primes", ctypes.c_int32),
        ("sort_survivors", ctypes.c_int32),
        ("mr_block", ctypes.c_int32),
        ("mr_blocks_per_cu", ctypes.c_int32),
        ("mr_window", ctypes.c_int32),
        ("rest_test", ctypes.c_int32),
        ("wheel_log2", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerConfig(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_int32),
        ("max_inflight", ctypes.c_int32),
        ("mem_budget_bytes", ctypes.c_uint64),
        ("max_batch_elems", ctypes.c_uint64),
        ("max_batch_reqs", ctypes.c_int32),
        ("block_on_full", ctypes.c_int32),
        ("test_mode", ctypes.c_int32),
        ("test_fail_every", ctypes.c_int32),
        ("test_delay_us", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


# name: (restype, argtypes); every symbol include/isprime.h declares
_P, _SZ, _I, _U64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_uint64
SIGNATURES = {
    "isp_init": (_I, [_I]),
    "isp_shutdown": (None, []),
    "isprime_u64": (_I, [_P, _P, _SZ, _P]),
    "isprime_u64_noalloc": (_I, [_P, _P, _SZ, _P]),
    "isp_noalloc_max_len": (_SZ, []),
    "isprime_u64_batched": (_I, [_P, _P, _P, _SZ, _P]),
    "isprime_u64_batched_offsets": (_I, [_P, _P, _P, _SZ, _P]),
    "isprime_range_u64": (_I, [_U64, _P, _SZ, _P]),
    "isp_workspace_bytes": (_SZ, [_SZ]),
    "isp_range_workspace_bytes": (_SZ, [_U64, _SZ]),
    "isp_last_device_error": (_I, []),
    "isp_strerror": (ctypes.c_char_p, [_I]),
    "isp_get_config": (_I, [ctypes.POINTER(Config)]),
    "isp_set_config": (_I, [ctypes.POINTER(Config)]),
    "isp_montmul_u64": (_I, [_P, _P, _P, _P, _SZ, _P]),
    "isp_table": (_I, [_I, ctypes.POINTER(_P), ctypes.POINTER(_SZ)]),
    "isp_last_counts": (_I, [_P, ctypes.POINTER(_U64), ctypes.POINTER(_U64)]),
    "isp_profile": (_I, [_I]),
    "isp_profile_read": (_I, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_U64)]),
    "isp_table_rebuild": (_I, [_I, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "isp_wheel_table": (_I, [_I, ctypes.POINTER(_P), ctypes.POINTER(_SZ)]),
    "isp_server_create": (_I, [ctypes.POINTER(ServerConfig), ctypes.POINTER(_P)]),
    "isp_submit": (_I, [_P, _P, _P, _SZ, ctypes.POINTER(_U64)]),
    "isp_poll": (_I, [_P, _U64]),
    "isp_wait": (_I, [_P, _U64, ctypes.c_int64]),
    "isp_server_footprint": (_I, [_P, ctypes.POINTER(_U64), ctypes.POINTER(_U64)]),
    "isp_server_destroy": (_I, [_P]),
}


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(
                    "libisprime.so is not built (run `python -m paper_2108_04791_amd._build`); "
                    "this package has no CPU fallback")
            L = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(L, name)
                fn.restype = res
                fn.argtypes = args
            _lib = L
            _hip()
        return _lib


_hiprt = None


def _hip() -> ctypes.CDLL:
    """The HIP runtime the library links (for the table copy diagnostic)."""
    global _hiprt
    if _hiprt is None:
        h = ctypes.CDLL("libamdhip64.so", mode=ctypes.RTLD_GLOBAL)
        h.hipMemcpy.restype = ctypes.c_int
        h.hipMemcpy.argtypes = [_P, _P, _SZ, ctypes.c_int]
        _hiprt = h
    return _hiprt


def _strerror(status: int) -> str:
    if _lib is None:
        return "status %d" % status
    return _lib.isp_strerror(status).decode()


def _check(status: int, what: str) -> None:
    if status != ISP_OK:
        raise IsprimeError(status, what)


def _stream_handle(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _on_stream(stream, *tensors) -> None:
    """Before a call on a stream other than the current one: that stream
    waits for the current stream's work (copies and allocations made here,
    e.g. a .contiguous() copy of the input or a new output), and each
    tensor is recorded as used on it, so that the caching allocator does not
    hand its memory out again while the call may still read or write it."""
    if stream is None:
        return
    cur = torch.cuda.current_stream(stream.device)
    if stream == cur:
        return
    stream.wait_stream(cur)
    for t in tensors:
        if t is not None and t.is_cuda:
            t.record_stream(stream)


def _as_u64(t: torch.Tensor) -> torch.Tensor:
    if t.dtype not in (torch.uint64, torch.int64):
        raise TypeError("expected a torch.uint64 (or int64-viewed) tensor, got %s" % t.dtype)
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    return t.contiguous()


def init(device: int | None = None) -> None:
    """Build the device's sieve table now (otherwise on first use)."""
    if device is None:
        device = torch.cuda.current_device()
    _check(lib().isp_init(device), "isp_init")


def shutdown() -> None:
    lib().isp_shutdown()


def isprime_into(n: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
    """out[i] = 1 if n[i] is prime else 0 (uint8/bool out, same numel)."""
    n = _as_u64(n)
    if out.dtype not in (torch.uint8, torch.bool) or not out.is_contiguous():
        raise TypeError("out must be a contiguous uint8 or bool tensor")
    if out.numel() != n.numel():
        raise ValueError("out has %d elements, n has %d" % (out.numel(), n.numel()))
    with torch.cuda.device(n.device):
        _on_stream(stream, n, out)
        _check(lib().isprime_u64(n.data_ptr(), out.data_ptr(), n.numel(), _stream_handle(stream)),
               "isprime_u64")
    return out


def isprime_into_noalloc(n: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
    """isprime_into through the allocation-free entry point: the library
    allocates nothing during the call (its workspace is a static device
    array; init() must have run for the device).  n must already be a
    contiguous uint64/int64 device tensor: no copy is made here either."""
    if n.dtype not in (torch.uint64, torch.int64) or not n.is_cuda or not n.is_contiguous():
        raise TypeError("n must be a contiguous uint64 (or int64-viewed) device tensor")
    if out.dtype not in (torch.uint8, torch.bool) or not out.is_contiguous():
        raise TypeError("out must be a contiguous uint8 or bool tensor")
    if out.numel() != n.numel():
        raise ValueError("out has %d elements, n has %d" % (out.numel(), n.numel()))
    with torch.cuda.device(n.device):
        _on_stream(stream, n, out)
        _check(lib().isprime_u64_noalloc(n.data_ptr(), out.data_ptr(), n.numel(),
                                         _stream_handle(stream)), "isprime_u64_noalloc")
    return out


def noalloc_max_len() -> int:
    return lib().isp_noalloc_max_len()


def isprime(n: torch.Tensor, stream=None) -> torch.Tensor:
    """Boolean tensor of n's shape: True where the element is prime."""
    n = _as_u64(n)
    out = torch.empty(n.shape, dtype=torch.bool, device=n.device)
    return isprime_into(n, out, stream)


class Batch:
    """A prepared isprime_u64_batched call: the host arrays of device
    pointers and lengths are built once, so repeated calls over the same
    tensors cost one C call each.  The tensors must stay alive and keep
    their storage while the Batch is used."""

    def __init__(self, arrays, outs=None):
        self.arrays = [_as_u64(a) for a in arrays]
        if outs is None:
            outs = [torch.empty(a.shape, dtype=torch.bool, device=a.device) for a in self.arrays]
        if len(outs) != len(self.arrays):
            raise ValueError("one output per array")
        for a, o in zip(self.arrays, outs):
            if o.numel() != a.numel() or not o.is_contiguous() or o.dtype not in (torch.bool, torch.uint8):
                raise ValueError("each output must be a contiguous bool/uint8 tensor of its array's size")
        self.outs = list(outs)
        self.k = len(self.arrays)
        NP = ctypes.c_uint64 * max(self.k, 1)
        self._nps = NP(*[a.data_ptr() if a.numel() else 0 for a in self.arrays])
        self._ops = NP(*[o.data_ptr() if o.numel() else 0 for o in self.outs])
        self._lens = NP(*[a.numel() for a in self.arrays])
        self._device = self.arrays[0].device if self.k else None

    def run(self, stream=None):
        """Enqueue the call on `stream`; returns the outputs."""
        if self.k == 0:
            return self.outs
        with torch.cuda.device(self._device):
            _on_stream(stream, *self.arrays, *self.outs)
            _check(lib().isprime_u64_batched(ctypes.cast(self._nps, _P), ctypes.cast(self._ops, _P),
                                             ctypes.cast(self._lens, _P), self.k,
                                             _stream_handle(stream)),
                   "isprime_u64_batched")
        return self.outs


def isprime_batched(arrays, outs=None, stream=None):
    """Many arrays in one graph-replayed launch sequence; returns the outputs."""
    return Batch(arrays, outs).run(stream)


def isprime_batched_offsets(n: torch.Tensor, offsets: torch.Tensor, out: torch.Tensor | None = None,
                            stream=None) -> torch.Tensor:
    """Arrays laid end to end in one tensor: array a is n[offsets[a]:offsets[a+1]]
    (offsets: int64/uint64, on the device or the host).  Returns the bool
    verdicts over n's length (elements outside the arrays are left as
    they were in `out`, which is created zeroed when not given)."""
    n = _as_u64(n)
    if offsets.dtype not in (torch.uint64, torch.int64) or not offsets.is_contiguous():
        raise TypeError("offsets must be a contiguous uint64 / int64 tensor")
    if out is None:
        out = torch.zeros(n.shape, dtype=torch.bool, device=n.device)
    if out.numel() != n.numel() or not out.is_contiguous() or out.dtype not in (torch.bool, torch.uint8):
        raise ValueError("out must be a contiguous bool/uint8 tensor of n's size")
    num = offsets.numel() - 1
    if num < 0:
        raise ValueError("offsets needs at least one entry")
    if num > 0 and int(offsets[-1]) > n.numel():
        raise ValueError("offsets run past the end of n")
    with torch.cuda.device(n.device):
        _on_stream(stream, n, out, offsets if offsets.is_cuda else None)
        _check(lib().isprime_u64_batched_offsets(n.data_ptr(), out.data_ptr(), offsets.data_ptr(),
                                                 num, _stream_handle(stream)),
               "isprime_u64_batched_offsets")
    return out


def isprime_range(lo: int, length: int, out: torch.Tensor | None = None, stream=None,
                  device=None) -> torch.Tensor:
    """Boolean tensor: element i is True iff lo + i is prime (a contiguous
    interval; no input array)."""
    if out is None:
        out = torch.empty(length, dtype=torch.bool, device=device or "cuda")
    if out.numel() != length or not out.is_contiguous() or out.dtype not in (torch.bool, torch.uint8):
        raise ValueError("out must be a contiguous bool/uint8 tensor of `length` elements")
    with torch.cuda.device(out.device):
        _on_stream(stream, out)
        _check(lib().isprime_range_u64(lo, out.data_ptr() if length else None, length,
                                       _stream_handle(stream)), "isprime_range_u64")
    return out


def montmul(a: torch.Tensor, b: torch.Tensor, n: torch.Tensor, stream=None) -> torch.Tensor:
    """Diagnostic: a*b mod n on the device through Montgomery form (odd n >= 3)."""
    a, b, n = _as_u64(a), _as_u64(b), _as_u64(n)
    out = torch.empty_like(n)
    _on_stream(stream, a, b, n, out)
    _check(lib().isp_montmul_u64(a.data_ptr(), b.data_ptr(), n.data_ptr(), out.data_ptr(),
                                 n.numel(), _stream_handle(stream)), "isp_montmul_u64")
    return out


def table(device: int | None = None) -> torch.Tensor:
    """A copy of the device's sieve table (uint32, 2^26 words)."""
    if device is None:
        device = torch.cuda.current_device()
    ptr, words = _P(), _SZ()
    _check(lib().isp_table(device, ctypes.byref(ptr), ctypes.byref(words)), "isp_table")
    out = torch.empty(words.value, dtype=torch.int32, device="cuda:%d" % device)
    torch.cuda.synchronize(device)
    err = _hip().hipMemcpy(out.data_ptr(), ptr.value, words.value * 4, 3)  # device to device
    if err != 0:
        raise RuntimeError("table copy failed: hipError %d" % err)
    return out


def table_rebuild_ms(device: int | None = None):
    """Rebuild the device's tables in place; (sieve ms, wheel table ms) of
    the build kernels (HIP events).  Nothing may be in flight on the device."""
    if device is None:
        device = torch.cuda.current_device()
    ms, wms = ctypes.c_double(), ctypes.c_double()
    _check(lib().isp_table_rebuild(device, ctypes.byref(ms), ctypes.byref(wms)),
           "isp_table_rebuild")
    return ms.value, wms.value


def wheel_table(device: int | None = None) -> torch.Tensor:
    """A copy of the device's wheel table (uint32 words, 48 bits per 210 numbers)."""
    if device is None:
        device = torch.cuda.current_device()
    ptr, words = _P(), _SZ()
    _check(lib().isp_wheel_table(device, ctypes.byref(ptr), ctypes.byref(words)), "isp_wheel_table")
    out = torch.empty(words.value, dtype=torch.int32, device="cuda:%d" % device)
    torch.cuda.synchronize(device)
    err = _hip().hipMemcpy(out.data_ptr(), ptr.value, words.value * 4, 3)  # device to device
    if err != 0:
        raise RuntimeError("wheel table copy failed: hipError %d" % err)
    return out


def last_counts(stream=None):
    """(trial-filter survivors, base-2 passers) of the last call on the stream."""
    s, c = _U64(), _U64()
    _check(lib().isp_last_counts(_stream_handle(stream), ctypes.byref(s), ctypes.byref(c)),
           "isp_last_counts")
    return s.value, c.value


STAGES = ("classify", "filter2", "mr_base2", "mr_rest")


def profile(enable: bool) -> None:
    """Per-stage HIP-event timing of plain calls (calls become synchronous)."""
    _check(lib().isp_profile(1 if enable else 0), "isp_profile")


def profile_read() -> dict:
    """{stage: total ms} and the number of profiled calls under 'calls'."""
    ms = (ctypes.c_double * len(STAGES))()
    calls = _U64()
    _check(lib().isp_profile_read(ms, ctypes.byref(calls)), "isp_profile_read")
    d = dict(zip(STAGES, list(ms)))
    d["calls"] = calls.value
    return d


def get_config() -> dict:
    c = Config()
    _check(lib().isp_get_config(ctypes.byref(c)), "isp_get_config")
    return c.as_dict()


def set_config(**kw) -> dict:
    """Update some fields of the configuration; returns the previous one."""
    prev = get_config()
    c = Config(**{**prev, **kw})
    _check(lib().isp_set_config(ctypes.byref(c)), "isp_set_config")
    return prev


def workspace_bytes(n: int) -> int:
    return lib().isp_workspace_bytes(n)


class Server:
    """Continuous-batching request server over host buffers (isp_server_*)."""

    def __init__(self, device: int = 0, max_inflight: int = 0, mem_budget_bytes: int = 0,
                 max_batch_elems: int = 0, max_batch_reqs: int = 0, block_on_full: bool = True,
                 test_mode: int = 0, test_fail_every: int = 0, test_delay_us: int = 0):
        cfg = ServerConfig(device, max_inflight, mem_budget_bytes, max_batch_elems,
                           max_batch_reqs, 1 if block_on_full else 0, test_mode,
                           test_fail_every, test_delay_us, 0)
        h = _P()
        _check(lib().isp_server_create(ctypes.byref(cfg), ctypes.byref(h)), "isp_server_create")
        self._h = h
        self._keep = {}

    def submit(self, n, out) -> int:
        """Queue host arrays n (uint64) -> out (uint8); kept alive until waited on."""
        import numpy as np
        if n.dtype != np.uint64 or out.dtype != np.uint8 or n.size != out.size:
            raise TypeError("submit needs uint64 n and uint8 out of the same size")
        if not (n.flags["C_CONTIGUOUS"] and out.flags["C_CONTIGUOUS"]):
            raise ValueError("submit needs contiguous arrays")
        t = _U64()
        _check(lib().isp_submit(self._h, n.ctypes.data if n.size else None,
                                out.ctypes.data if out.size else None, n.size, ctypes.byref(t)),
               "isp_submit")
        self._keep[t.value] = (n, out)
        return t.value

    def poll(self, ticket: int) -> bool:
        r = lib().isp_poll(self._h, ticket)
        if r < 0:
            raise IsprimeError(r, "isp_poll")
        return r == 1

    def wait(self, ticket: int, timeout_us: int = -1) -> None:
        _check(lib().isp_wait(self._h, ticket, timeout_us), "isp_wait")
        self._keep.pop(ticket, None)

    def footprint(self):
        """(device bytes, pinned host bytes) reserved for the server's slots."""
        d, p = _U64(), _U64()
        _check(lib().isp_server_footprint(self._h, ctypes.byref(d), ctypes.byref(p)),
               "isp_server_footprint")
        return d.value, p.value

    def close(self) -> None:
        if self._h:
            _check(lib().isp_server_destroy(self._h), "isp_server_destroy")
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
