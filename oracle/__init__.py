"""Oracle for Wallace's normal generator (Brent 1997) -- TEST INFRASTRUCTURE.

A thin ctypes wrapper around ``wallace_oracle.c``: a plain, slow,
single-threaded CPU implementation written from the paper. Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import this
package; the GPU library never does, and the two share no code.

Parity pins live in ``tests/test_oracle_*.py``. Every oracle function is
pinned there by something other than itself (published vectors, closed forms,
invariants, brute force); see the header of ``wallace_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(_HERE, "wallace_oracle.c")
LIBRARY = os.path.join(_HERE, "liboracle.so")

SUM_F64, SUM_F32, SUM_F32_COMP = 0, 1, 2
A_PAIRS, A_FULL_ODD = 0, 1

CFLAGS = ["-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math",
          "-fPIC", "-shared"]


def build() -> str:
    """Compile the oracle with gcc (always recompiles)."""
    tmp = LIBRARY + ".tmp"
    subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, SOURCE, "-lm"])
    os.replace(tmp, LIBRARY)
    return LIBRARY


_lib = None

_u64p = ctypes.POINTER(ctypes.c_uint64)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_f32p = ctypes.POINTER(ctypes.c_float)
_f64p = ctypes.POINTER(ctypes.c_double)


def lib():
    """Load the oracle library, building it first if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBRARY):
        build()
    L = ctypes.CDLL(LIBRARY)
    L.wo_splitmix64.restype = ctypes.c_uint64
    L.wo_splitmix64.argtypes = [_u64p]
    L.wo_stride_pair.restype = None
    L.wo_stride_pair.argtypes = [ctypes.c_int, _u32p]
    L.wo_initial_pool64.restype = None
    L.wo_initial_pool64.argtypes = [_u64p, ctypes.c_int, ctypes.c_uint32, _f64p]
    L.wo_pass_params.restype = None
    L.wo_pass_params.argtypes = [_u64p, ctypes.c_int, ctypes.c_uint32,
                                 ctypes.c_int, _u32p, _u32p, _u32p]
    L.wo_pass_params_rot.restype = None
    L.wo_pass_params_rot.argtypes = [_u64p, ctypes.c_int, ctypes.c_uint32,
                                     ctypes.c_int, _u32p, _u32p, _u32p, _f64p]
    L.wo_rotation.restype = None
    L.wo_rotation.argtypes = [ctypes.c_uint64, _f64p, _f64p]
    L.wo_rotation_many.restype = None
    L.wo_rotation_many.argtypes = [_u64p, ctypes.c_size_t, _f64p, _f64p]
    L.wo_chi2_many.restype = None
    L.wo_chi2_many.argtypes = [_f64p, _f64p, _f64p, ctypes.c_size_t, _f64p, _f64p]
    L.wo_pass32_rot.restype = None
    L.wo_pass32_rot.argtypes = [ctypes.c_uint32, _u32p, _u32p, ctypes.c_float,
                                ctypes.c_float, _f32p, _f32p]
    L.wo_pass64_rot.restype = None
    L.wo_pass64_rot.argtypes = [ctypes.c_uint32, _u32p, _u32p, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double, _f64p, _f64p]
    for name, rt, pt in (("wo_sumsq_f64", ctypes.c_double, _f32p),
                         ("wo_sumsq_f32", ctypes.c_float, _f32p),
                         ("wo_sumsq_f32c", ctypes.c_double, _f32p),
                         ("wo_sumsq_d", ctypes.c_double, _f64p)):
        fn = getattr(L, name)
        fn.restype = rt
        fn.argtypes = [pt, ctypes.c_size_t]
    L.wo_scale32.restype = ctypes.c_float
    L.wo_scale32.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_size_t,
                             _f64p, _f64p]
    L.wo_pass32.restype = None
    L.wo_pass32.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_int,
                            _u32p, _u32p, ctypes.c_uint32, ctypes.c_float,
                            _f32p, _f32p]
    L.wo_pass64.restype = None
    L.wo_pass64.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_int,
                            _u32p, _u32p, ctypes.c_uint32, ctypes.c_double,
                            _f64p, _f64p]
    L.wo_matrix.restype = None
    L.wo_matrix.argtypes = [ctypes.c_int, ctypes.c_int, _f64p]
    L.wo_gen_create.restype = ctypes.c_void_p
    L.wo_gen_create.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32,
                                ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                ctypes.c_int]
    L.wo_gen64_create.restype = ctypes.c_void_p
    L.wo_gen64_create.argtypes = [ctypes.c_uint64, ctypes.c_int,
                                  ctypes.c_uint32, ctypes.c_int]
    L.wo_gen_set_restart.restype = None
    L.wo_gen_set_restart.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
    L.wo_gen_destroy.restype = None
    L.wo_gen_destroy.argtypes = [ctypes.c_void_p]
    L.wo_gen_pass.restype = None
    L.wo_gen_pass.argtypes = [ctypes.c_void_p]
    L.wo_gen_fill.restype = None
    L.wo_gen_fill.argtypes = [ctypes.c_void_p, _f32p, _f64p, ctypes.c_uint64]
    L.wo_gen_pool32.restype = _f32p
    L.wo_gen_pool32.argtypes = [ctypes.c_void_p]
    L.wo_gen_pool64.restype = _f64p
    L.wo_gen_pool64.argtypes = [ctypes.c_void_p]
    for name, rt in (("wo_gen_sigma", ctypes.c_double),
                     ("wo_gen_passes", ctypes.c_uint64),
                     ("wo_gen_rng", ctypes.c_uint64),
                     ("wo_gen_last_S", ctypes.c_double),
                     ("wo_gen_last_c64", ctypes.c_double)):
        fn = getattr(L, name)
        fn.restype = rt
        fn.argtypes = [ctypes.c_void_p]
    _lib = L
    return L


def _ptr(a: np.ndarray, typ):
    return a.ctypes.data_as(typ)


# ---------------------------------------------------------------------------
# Building blocks
# ---------------------------------------------------------------------------

def splitmix64(state: int):
    """Return (new_state, output) of one splitmix64 step."""
    s = ctypes.c_uint64(state)
    z = lib().wo_splitmix64(ctypes.byref(s))
    return s.value, z


def stride_pair(k: int):
    out = (ctypes.c_uint32 * 2)()
    lib().wo_stride_pair(k, out)
    return int(out[0]), int(out[1])


def initial_pool64(seed: int, n: int, N: int):
    """Box-Muller initial pool (FP64, unrounded) and the state after it."""
    s = ctypes.c_uint64(seed)
    pool = np.empty(n * N, dtype=np.float64)
    lib().wo_initial_pool64(ctypes.byref(s), n, N, _ptr(pool, _f64p))
    return pool, s.value


def pass_params(state: int, n: int, N: int, a_mode: int = A_PAIRS):
    """Return (a, b, signs, new_state) for one pass."""
    s = ctypes.c_uint64(state)
    a = np.empty(n, dtype=np.uint32)
    b = np.empty(n, dtype=np.uint32)
    signs = ctypes.c_uint32()
    lib().wo_pass_params(ctypes.byref(s), n, N, a_mode, _ptr(a, _u32p),
                         _ptr(b, _u32p), ctypes.byref(signs))
    return a, b, signs.value, s.value


def pass_params_rot(state: int, n: int, N: int, a_mode: int = A_PAIRS):
    """Return (a, b, signs, (cos, sin), new_state); the rotation is NaN for n != 2."""
    s = ctypes.c_uint64(state)
    a = np.empty(n, dtype=np.uint32)
    b = np.empty(n, dtype=np.uint32)
    signs = ctypes.c_uint32()
    rot = np.full(2, np.nan)
    lib().wo_pass_params_rot(ctypes.byref(s), n, N, a_mode, _ptr(a, _u32p),
                             _ptr(b, _u32p), ctypes.byref(signs), _ptr(rot, _f64p))
    return a, b, signs.value, (float(rot[0]), float(rot[1])), s.value


def rotation(w: int):
    """(cos theta, sin theta) of an n = 2 pass from its draw w (section 8)."""
    cs = ctypes.c_double()
    sn = ctypes.c_double()
    lib().wo_rotation(w, ctypes.byref(cs), ctypes.byref(sn))
    return cs.value, sn.value


def rotation_many(w: np.ndarray):
    """wo_rotation over an array of draws: (cos, sin) arrays."""
    w = np.ascontiguousarray(w, dtype=np.uint64)
    cs = np.empty(w.size, dtype=np.float64)
    sn = np.empty(w.size, dtype=np.float64)
    lib().wo_rotation_many(_ptr(w, _u64p), w.size, _ptr(cs, _f64p), _ptr(sn, _f64p))
    return cs, sn


def chi2_many(xstar, sigma, r):
    """Chi-squared target S and scale c (eq. 3) over arrays, r given."""
    xstar = np.ascontiguousarray(xstar, dtype=np.float64)
    sigma = np.ascontiguousarray(sigma, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    S = np.empty(xstar.size, dtype=np.float64)
    c = np.empty(xstar.size, dtype=np.float64)
    lib().wo_chi2_many(_ptr(xstar, _f64p), _ptr(sigma, _f64p), _ptr(r, _f64p), xstar.size,
                       _ptr(S, _f64p), _ptr(c, _f64p))
    return S, c


def pass32_rot(N, a, b, p, q, X):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    b = np.ascontiguousarray(b, dtype=np.uint32)
    X = np.ascontiguousarray(X, dtype=np.float32)
    Y = np.empty_like(X)
    lib().wo_pass32_rot(N, _ptr(a, _u32p), _ptr(b, _u32p), float(p), float(q),
                        _ptr(X, _f32p), _ptr(Y, _f32p))
    return Y


def pass64_rot(N, a, b, cs, sn, c, X):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    b = np.ascontiguousarray(b, dtype=np.uint32)
    X = np.ascontiguousarray(X, dtype=np.float64)
    Y = np.empty_like(X)
    lib().wo_pass64_rot(N, _ptr(a, _u32p), _ptr(b, _u32p), float(cs), float(sn), float(c),
                        _ptr(X, _f64p), _ptr(Y, _f64p))
    return Y


def sumsq_f64(y: np.ndarray) -> float:
    y = np.ascontiguousarray(y, dtype=np.float32)
    return lib().wo_sumsq_f64(_ptr(y, _f32p), y.size)


def sumsq_f32(y: np.ndarray) -> np.float32:
    y = np.ascontiguousarray(y, dtype=np.float32)
    return np.float32(lib().wo_sumsq_f32(_ptr(y, _f32p), y.size))


def sumsq_f32c(y: np.ndarray) -> float:
    y = np.ascontiguousarray(y, dtype=np.float32)
    return lib().wo_sumsq_f32c(_ptr(y, _f32p), y.size)


def sumsq_d(y: np.ndarray) -> float:
    y = np.ascontiguousarray(y, dtype=np.float64)
    return lib().wo_sumsq_d(_ptr(y, _f64p), y.size)


def scale32(xstar: float, sigma: float, nu: int):
    """Return (c32, S, c64) of the chi-squared rescaling (eq. 3)."""
    S = ctypes.c_double()
    c64 = ctypes.c_double()
    c32 = lib().wo_scale32(xstar, sigma, nu, ctypes.byref(S), ctypes.byref(c64))
    return np.float32(c32), S.value, c64.value


def pass32(n, N, mat, a, b, h, X, signs=0):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    b = np.ascontiguousarray(b, dtype=np.uint32)
    X = np.ascontiguousarray(X, dtype=np.float32)
    Y = np.empty_like(X)
    lib().wo_pass32(n, N, mat, _ptr(a, _u32p), _ptr(b, _u32p), signs,
                    float(h), _ptr(X, _f32p), _ptr(Y, _f32p))
    return Y


def pass64(n, N, mat, a, b, c, X, signs=0):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    b = np.ascontiguousarray(b, dtype=np.uint32)
    X = np.ascontiguousarray(X, dtype=np.float64)
    Y = np.empty_like(X)
    lib().wo_pass64(n, N, mat, _ptr(a, _u32p), _ptr(b, _u32p), signs,
                    float(c), _ptr(X, _f64p), _ptr(Y, _f64p))
    return Y


def matrix(n: int, mat: int) -> np.ndarray:
    M = np.empty(n * n, dtype=np.float64)
    lib().wo_matrix(n, mat, _ptr(M, _f64p))
    return M.reshape(n, n)


# ---------------------------------------------------------------------------
# Generators
# ---------------------------------------------------------------------------

class Gen:
    """FP32 generator (the bit-exact variant)."""

    fp64 = False

    def __init__(self, seed: int, n: int, N: int, sum_mode: int = SUM_F64,
                 a_mode: int = A_PAIRS, f: int = 1, withhold: int = 0, restart: int = 0):
        self.n, self.N, self.nu = n, N, n * N
        self._h = lib().wo_gen_create(seed, n, N, sum_mode, a_mode, f, withhold)
        lib().wo_gen_set_restart(self._h, restart)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.wo_gen_destroy(h)
            self._h = None

    def do_pass(self):
        lib().wo_gen_pass(self._h)

    def fill(self, count: int) -> np.ndarray:
        out = np.empty(count, dtype=np.float64 if self.fp64 else np.float32)
        if count:
            if self.fp64:
                lib().wo_gen_fill(self._h, None, _ptr(out, _f64p), count)
            else:
                lib().wo_gen_fill(self._h, _ptr(out, _f32p), None, count)
        return out

    @property
    def pool(self) -> np.ndarray:
        if self.fp64:
            p = lib().wo_gen_pool64(self._h)
        else:
            p = lib().wo_gen_pool32(self._h)
        return np.ctypeslib.as_array(p, shape=(self.nu,)).copy()

    @property
    def sigma(self) -> float:
        return lib().wo_gen_sigma(self._h)

    @property
    def passes(self) -> int:
        return lib().wo_gen_passes(self._h)

    @property
    def rng(self) -> int:
        return lib().wo_gen_rng(self._h)

    @property
    def last_S(self) -> float:
        return lib().wo_gen_last_S(self._h)

    @property
    def last_c64(self) -> float:
        return lib().wo_gen_last_c64(self._h)


class Gen64(Gen):
    """FP64 generator (the accuracy variant)."""

    fp64 = True

    def __init__(self, seed: int, n: int, N: int, a_mode: int = A_PAIRS, restart: int = 0):
        self.n, self.N, self.nu = n, N, n * N
        self._h = lib().wo_gen64_create(seed, n, N, a_mode)
        lib().wo_gen_set_restart(self._h, restart)
