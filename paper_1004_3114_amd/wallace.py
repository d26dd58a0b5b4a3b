"""Python binding of libwallace.so (include/wallace.h), argument marshalling only.

Every pass of the generator runs in the library's HIP kernels. PyTorch is
used only to own device memory (the workspace and output tensors) and to
supply the current HIP stream. There is no CPU fallback: if the library is
missing, importing this module's entry points raises.

The functions ``wallace_*`` mirror the C ABI one to one (pointers are Python
ints). ``Generator`` and ``Batch`` wrap them for torch tensors.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIBRARY = os.path.join(_PKG, "libwallace.so")

WALLACE_OK = 0
WALLACE_EINVAL = -1
WALLACE_ENOSPC = -2
WALLACE_EHIP = -3
WALLACE_ECORRUPT = -4
WALLACE_EUNSUP = -5
WALLACE_ESTATE = -6
FLAG_CORRUPT = 1
FLAG_NONFINITE = 2


class WallaceError(RuntimeError):
    def __init__(self, code: int, what: str):
        detail = ""
        if code == WALLACE_EHIP and _lib is not None:
            detail = " [" + (_lib.wallace_last_error() or b"").decode() + "]"
        super().__init__(f"{what}: {strerror(code)} ({code}){detail}")
        self.code = code


class wallace_opts(ctypes.Structure):
    _fields_ = [("f", ctypes.c_int32), ("a_mode", ctypes.c_int32),
                ("reduce_mode", ctypes.c_int32), ("transform_mode", ctypes.c_int32),
                ("withhold_driver", ctypes.c_int32), ("check_workspace", ctypes.c_int32),
                ("restart_passes", ctypes.c_int32)]


_lib = None
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64
_sz = ctypes.c_size_t
_f32 = ctypes.c_float

# name -> (restype, argtypes); the names and order follow include/wallace.h
SIGNATURES = {
    "wallace_default_opts": (None, [ctypes.POINTER(wallace_opts)]),
    "wallace_strerror": (ctypes.c_char_p, [_i32]),
    "wallace_last_error": (ctypes.c_char_p, []),
    "wallace_workspace_bytes": (_i32, [_i32, _u32, ctypes.POINTER(wallace_opts),
                                       ctypes.POINTER(_sz)]),
    "wallace_init": (_i32, [_u64, _i32, _u32, ctypes.POINTER(wallace_opts), _vp, _sz,
                            _vp, ctypes.POINTER(_vp)]),
    "wallace_initial_pool": (_i32, [_u64, _i32, _u32, _vp, ctypes.POINTER(_u64)]),
    "wallace_fill": (_i32, [_vp, _vp, _u64, _vp]),
    "wallace_fill_normal": (_i32, [_vp, _vp, _u64, _f32, _f32, _vp]),
    "wallace_fill_static": (_i32, [_vp, _vp, _u64, _vp]),
    "wallace_sumsq": (_i32, [_vp, ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(_u64), _vp]),
    "wallace_read_pool": (_i32, [_vp, _vp, _vp]),
    "wallace_status": (_i32, [_vp, ctypes.POINTER(_u32), _vp]),
    "wallace_destroy": (_i32, [_vp]),
    "wallace_batch_workspace_bytes": (_i32, [_u32, _vp, _vp, ctypes.POINTER(_sz)]),
    "wallace_batch_init": (_i32, [_u32, _vp, _vp, _vp, ctypes.POINTER(wallace_opts), _vp,
                                  _sz, _vp, ctypes.POINTER(_vp)]),
    "wallace_batch_plan": (_i32, [_vp, _vp, _vp, _vp]),
    "wallace_fill_batched": (_i32, [_vp, _vp, _u64, _vp]),
    "wallace_batch_tune_bytes": (_i32, [_vp, ctypes.POINTER(_sz)]),
    "wallace_batch_tune": (_i32, [_vp, _vp, _sz, _vp]),
    "wallace_batch_tune_planned": (_i32, [_vp, _vp, _u64, _vp, _sz, _vp]),
    "wallace_batch_sumsq": (_i32, [_vp, _u32, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(_u64), _vp]),
    "wallace_batch_classes": (_i32, [_vp, _u32, _vp, ctypes.POINTER(_u32)]),
    "wallace_batch_status": (_i32, [_vp, ctypes.POINTER(_u32), _vp]),
    "wallace_batch_set_streams": (_i32, [_vp, _u32, ctypes.POINTER(_vp)]),
    "wallace_batch_destroy": (_i32, [_vp]),
}


def lib():
    """Load libwallace.so. Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBRARY):
        raise ImportError(f"{LIBRARY} is missing: run paper_1004_3114_amd.build.build() "
                          "(the HIP library is required; there is no fallback)")
    # torch first: the library and torch must share one HIP runtime in the
    # process, and the first libamdhip64.so.7 loaded serves both
    import torch  # noqa: F401
    L = ctypes.CDLL(LIBRARY)
    for name, (rt, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = rt
        fn.argtypes = args
    _lib = L
    return L


def strerror(code: int) -> str:
    try:
        return lib().wallace_strerror(code).decode()
    except ImportError:
        return "library not loaded"


def _check(code: int, what: str):
    if code != WALLACE_OK:
        raise WallaceError(code, what)


def make_opts(f=1, a_mode=0, reduce_mode=0, transform_mode=0, withhold_driver=0,
              check_workspace=0, restart_passes=0) -> wallace_opts:
    o = wallace_opts()
    lib().wallace_default_opts(ctypes.byref(o))
    o.f, o.a_mode, o.reduce_mode = f, a_mode, reduce_mode
    o.transform_mode, o.withhold_driver, o.check_workspace = (
        transform_mode, withhold_driver, check_workspace)
    o.restart_passes = restart_passes
    return o


def _stream_handle(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def initial_pool(seed: int, n: int, N: int):
    """The initial pool wallace_init uploads (host Box-Muller); needs no GPU."""
    out = np.empty(n * N, dtype=np.float32)
    rng = _u64()
    _check(lib().wallace_initial_pool(seed, n, N, out.ctypes.data, ctypes.byref(rng)),
           "wallace_initial_pool")
    return out, rng.value


def workspace_bytes(n: int, N: int, opts: Optional[wallace_opts] = None) -> int:
    b = _sz()
    _check(lib().wallace_workspace_bytes(n, N, ctypes.byref(opts) if opts else None,
                                         ctypes.byref(b)), "wallace_workspace_bytes")
    return b.value


def batch_extent(offsets, passes, n, N) -> int:
    """Floats of the output a planned batched fill writes: the largest
    offsets[g] + passes[g] * n[g] * N[g] (0 if nothing is written)."""
    ends = [int(o) + int(p) * int(a) * int(b) for o, p, a, b in zip(offsets, passes, n, N)
            if int(p)]
    return max(ends) if ends else 0


def check_batch_output(out, extent, device):
    """The checks a batched fill's output tensor must pass before its pointer
    is handed to the library: planned, float32, contiguous, on the
    workspace's device, at least `extent` elements."""
    import torch
    if extent is None:
        raise RuntimeError("Batch.fill before Batch.plan")
    if out.dtype != torch.float32:
        raise TypeError(f"batched output must be float32, not {out.dtype}")
    if not out.is_contiguous():
        raise ValueError("batched output must be contiguous")
    if out.device != device:
        raise ValueError(f"batched output on {out.device}, workspace on {device}")
    if out.numel() < extent:
        raise ValueError(f"batched output holds {out.numel()} floats, the plan writes {extent}")


class Generator:
    """One Wallace generator whose state lives in a torch-owned workspace."""

    def __init__(self, seed: int, n: int, N: int, device=None, stream=None, **opts):
        import torch
        self.n, self.N, self.nu = n, N, n * N
        self.opts = make_opts(**opts)
        nbytes = workspace_bytes(n, N, self.opts)
        dev = torch.device(device) if device is not None else torch.device("cuda")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        h = _vp()
        _check(lib().wallace_init(seed, n, N, ctypes.byref(self.opts), self._ws_ptr, nbytes,
                                  _stream_handle(stream), ctypes.byref(h)), "wallace_init")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.wallace_destroy(h)
            self._h = None

    def fill(self, out, count: Optional[int] = None, stream=None):
        """Fill a float32 CUDA tensor (first `count` elements) from the stream."""
        count = out.numel() if count is None else count
        assert out.dtype.itemsize == 4 and out.is_contiguous() and out.numel() >= count
        _check(lib().wallace_fill(self._h, out.data_ptr(), count, _stream_handle(stream)),
               "wallace_fill")
        return out

    def fill_static(self, out, count: Optional[int] = None, stream=None):
        """As fill, with the call's scratch in the library's static device
        array instead of the workspace (wallace_fill_static)."""
        count = out.numel() if count is None else count
        assert out.dtype.itemsize == 4 and out.is_contiguous() and out.numel() >= count
        _check(lib().wallace_fill_static(self._h, out.data_ptr(), count,
                                         _stream_handle(stream)), "wallace_fill_static")
        return out

    def fill_normal(self, out, mu: float, sigma: float, count: Optional[int] = None,
                    stream=None):
        count = out.numel() if count is None else count
        assert out.dtype.itemsize == 4 and out.is_contiguous() and out.numel() >= count
        _check(lib().wallace_fill_normal(self._h, out.data_ptr(), count, mu, sigma,
                                         _stream_handle(stream)), "wallace_fill_normal")
        return out

    def sumsq(self, stream=None):
        s = ctypes.c_double()
        p = _u64()
        _check(lib().wallace_sumsq(self._h, ctypes.byref(s), ctypes.byref(p),
                                   _stream_handle(stream)), "wallace_sumsq")
        return s.value, p.value

    def pool(self, stream=None) -> np.ndarray:
        out = np.empty(self.nu, dtype=np.float32)
        _check(lib().wallace_read_pool(self._h, out.ctypes.data, _stream_handle(stream)),
               "wallace_read_pool")
        return out

    def status(self, stream=None):
        f = _u32()
        rc = lib().wallace_status(self._h, ctypes.byref(f), _stream_handle(stream))
        return rc, f.value


class Batch:
    """G independent generators in one torch-owned workspace."""

    def __init__(self, seeds: Sequence[int], n: Sequence[int], N: Sequence[int], device=None,
                 stream=None, **opts):
        import torch
        self.G = len(seeds)
        self.seeds = np.ascontiguousarray(seeds, dtype=np.uint64)
        self.n = np.ascontiguousarray(n, dtype=np.int32)
        self.N = np.ascontiguousarray(N, dtype=np.uint32)
        assert self.n.size == self.G and self.N.size == self.G
        self.opts = make_opts(**opts)
        b = _sz()
        _check(lib().wallace_batch_workspace_bytes(self.G, self.n.ctypes.data,
                                                   self.N.ctypes.data, ctypes.byref(b)),
               "wallace_batch_workspace_bytes")
        dev = torch.device(device) if device is not None else torch.device("cuda")
        self.workspace = torch.empty(b.value + 256, dtype=torch.uint8, device=dev)
        ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        h = _vp()
        _check(lib().wallace_batch_init(self.G, self.seeds.ctypes.data, self.n.ctypes.data,
                                        self.N.ctypes.data, ctypes.byref(self.opts), ptr,
                                        b.value, _stream_handle(stream), ctypes.byref(h)),
               "wallace_batch_init")
        self._h = h
        # side streams for fills of several (n, N) classes, owned by torch
        self.side_streams = [torch.cuda.Stream(device=dev) for _ in range(3)]
        self.set_streams(self.side_streams)

    def set_streams(self, streams):
        """Hand the batch up to three side streams (torch streams) for its
        fills; an empty list returns to streams the library creates."""
        arr = (_vp * max(len(streams), 1))(*[int(x.cuda_stream) for x in streams])
        _check(lib().wallace_batch_set_streams(self._h, len(streams), arr),
               "wallace_batch_set_streams")
        self._streams_held = list(streams)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.wallace_batch_destroy(h)
            self._h = None

    def plan(self, offsets: Sequence[int], passes: Sequence[int], stream=None):
        self._offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
        self._passes = np.ascontiguousarray(passes, dtype=np.uint32)
        _check(lib().wallace_batch_plan(self._h, self._offsets.ctypes.data,
                                        self._passes.ctypes.data, _stream_handle(stream)),
               "wallace_batch_plan")
        self.extent = batch_extent(self._offsets, self._passes, self.n, self.N)

    def fill(self, out, stream=None):
        """Run the planned passes into `out` (a float32 CUDA tensor on the
        workspace's device holding at least `extent` elements)."""
        check_batch_output(out, getattr(self, "extent", None), self.workspace.device)
        _check(lib().wallace_fill_batched(self._h, out.data_ptr(), out.numel(),
                                          _stream_handle(stream)), "wallace_fill_batched")
        return out

    def tune(self, stream=None):
        import torch
        b = _sz()
        _check(lib().wallace_batch_tune_bytes(self._h, ctypes.byref(b)),
               "wallace_batch_tune_bytes")
        scratch = torch.empty(b.value + 256, dtype=torch.uint8, device=self.workspace.device)
        ptr = (scratch.data_ptr() + 255) // 256 * 256
        _check(lib().wallace_batch_tune(self._h, ptr, b.value, _stream_handle(stream)),
               "wallace_batch_tune")

    def tune_planned(self, out, stream=None):
        """Autotune every class on the planned fill itself, writing into
        `out` (checked like Batch.fill; its contents are overwritten)."""
        import torch
        check_batch_output(out, getattr(self, "extent", None), self.workspace.device)
        b = _sz()
        _check(lib().wallace_batch_tune_bytes(self._h, ctypes.byref(b)),
               "wallace_batch_tune_bytes")
        scratch = torch.empty(b.value + 256, dtype=torch.uint8, device=self.workspace.device)
        ptr = (scratch.data_ptr() + 255) // 256 * 256
        _check(lib().wallace_batch_tune_planned(self._h, out.data_ptr(), out.numel(), ptr,
                                                b.value, _stream_handle(stream)),
               "wallace_batch_tune_planned")

    def classes(self):
        """Per (n, N) class: its schedule (T, L, C), generator count and the
        block count of its planned launch."""
        cnt = _u32()
        _check(lib().wallace_batch_classes(self._h, 0, None, ctypes.byref(cnt)),
               "wallace_batch_classes")
        desc = np.zeros(7 * max(cnt.value, 1), dtype=np.int64)
        _check(lib().wallace_batch_classes(self._h, cnt.value, desc.ctypes.data,
                                           ctypes.byref(cnt)), "wallace_batch_classes")
        keys = ("n", "N", "T", "L", "C", "G", "blocks")
        return [dict(zip(keys, (int(v) for v in desc[7 * i:7 * i + 7])))
                for i in range(cnt.value)]

    def sumsq(self, g: int, stream=None):
        s = ctypes.c_double()
        p = _u64()
        _check(lib().wallace_batch_sumsq(self._h, g, ctypes.byref(s), ctypes.byref(p),
                                         _stream_handle(stream)), "wallace_batch_sumsq")
        return s.value, p.value

    def status(self, stream=None):
        f = _u32()
        rc = lib().wallace_batch_status(self._h, ctypes.byref(f), _stream_handle(stream))
        return rc, f.value
