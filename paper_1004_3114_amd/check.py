"""Binding of libwallace_check.so (include/wallace_check.h): device FP64
arithmetic checks and store-ceiling kernels, used by the tests and the
benchmark only. Argument marshalling only; the work runs in HIP kernels.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIBRARY = os.path.join(_PKG, "libwallace_check.so")

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64

SIGNATURES = {
    "wallace_check_chi2": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _u64, _vp]),
    "wallace_check_rotation": (_i32, [_vp, _vp, _vp, _u64, _vp]),
    "wallace_check_store_oneshot": (_i32, [_vp, _u64, ctypes.c_float, _i32, _vp]),
    "wallace_check_store_longlived": (_i32, [_vp, _u64, _u32, _u32, _u64, _u64, _u32, _vp]),
}

_lib = None


def lib():
    """Load libwallace_check.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBRARY):
        raise ImportError(f"{LIBRARY} is missing: run paper_1004_3114_amd.build.build()")
    import torch  # noqa: F401  (one HIP runtime per process, torch's)
    L = ctypes.CDLL(LIBRARY)
    for name, (rt, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = rt
        fn.argtypes = args
    _lib = L
    return L


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t):
    return None if t is None else t.data_ptr()


def _ok(code, what):
    if code != 0:
        raise RuntimeError(f"{what} failed with status {code}")


def chi2(xstar, sigma, r_nu, S=None, q=None, c=None, stream=None):
    """Device chi-squared scale over float64 CUDA tensors; returns c."""
    import torch
    c = torch.empty_like(xstar) if c is None else c
    n = xstar.numel()
    for t in (xstar, sigma, r_nu, S, q, c):
        assert t is None or (t.dtype == torch.float64 and t.is_contiguous() and t.numel() == n)
    _ok(lib().wallace_check_chi2(_ptr(xstar), _ptr(sigma), _ptr(r_nu), _ptr(S), _ptr(q),
                                 _ptr(c), n, _stream(stream)), "wallace_check_chi2")
    return c


def rotation(w, stream=None):
    """Device n = 2 rotation (cos, sin) for an int64 CUDA tensor of draws
    (their bit patterns are the uint64 draws)."""
    import torch
    assert w.dtype == torch.int64 and w.is_contiguous()
    cs = torch.empty(w.numel(), dtype=torch.float64, device=w.device)
    sn = torch.empty_like(cs)
    _ok(lib().wallace_check_rotation(_ptr(w), _ptr(cs), _ptr(sn), w.numel(), _stream(stream)),
        "wallace_check_rotation")
    return cs, sn


def store_oneshot(out, value=0.5, nontemporal=False, stream=None):
    _ok(lib().wallace_check_store_oneshot(_ptr(out), out.numel(), value, int(nontemporal),
                                          _stream(stream)), "wallace_check_store_oneshot")


def store_longlived(out, waves, chunks, wave_stride, chunk_stride, spin=0, stream=None):
    _ok(lib().wallace_check_store_longlived(_ptr(out), out.numel(), waves, chunks, wave_stride,
                                            chunk_stride, spin, _stream(stream)),
        "wallace_check_store_longlived")
