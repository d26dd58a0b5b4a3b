"""Host-side checks of the C ABI (no GPU needed).

The library must load and export every entry point include/wallace.h
declares; argument errors must be reported before anything touches the GPU;
the host-side initial pool (section 5: Box-Muller) must match the oracle bit
for bit.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_1004_3114_amd import build as wbuild
from paper_1004_3114_amd import wallace as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wallace.h")


@pytest.fixture(scope="module", autouse=True)
def built_library():
    if not os.path.exists(W.LIBRARY):
        wbuild.build()
    return W.lib()


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wallace_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert len(names) >= 20
    lib = ctypes.CDLL(W.LIBRARY)
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(W.SIGNATURES), set(names) ^ set(W.SIGNATURES)


def test_check_library_exports_its_header():
    # libwallace_check.so (include/wallace_check.h): device arithmetic checks
    # and store-ceiling kernels for the tests and the benchmark
    from paper_1004_3114_amd import check as CK
    if not os.path.exists(CK.LIBRARY):
        wbuild.build()
    text = open(os.path.join(ROOT, "include", "wallace_check.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = sorted(set(re.findall(r"\b(wallace_check_[a-z_0-9]+)\s*\(", text)))
    assert len(names) == 4
    lib = ctypes.CDLL(CK.LIBRARY)
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(CK.SIGNATURES)
    # argument errors come back before any launch (null and misaligned
    # pointers, a layout that would end beyond the buffer)
    L = CK.lib()
    assert L.wallace_check_chi2(None, None, None, None, None, None, 5, None) == W.WALLACE_EINVAL
    assert L.wallace_check_chi2(None, None, None, None, None, None, 0, None) == W.WALLACE_OK
    assert L.wallace_check_rotation(None, None, None, 3, None) == W.WALLACE_EINVAL
    assert L.wallace_check_store_oneshot(None, 1024, 0.0, 0, None) == W.WALLACE_EINVAL
    assert L.wallace_check_store_oneshot(16, 1000, 0.0, 0, None) == W.WALLACE_EINVAL
    assert L.wallace_check_store_oneshot(8, 1024, 0.0, 0, None) == W.WALLACE_EINVAL
    assert L.wallace_check_store_longlived(16, 4096, 4, 2, 1024, 1024 * 4, 0, None) == \
        W.WALLACE_EINVAL  # last chunk ends at 3*1024 + 4096 + 1024 > 4096
    assert L.wallace_check_store_longlived(16, 1 << 20, 3, 1, 1024, 1024, 0, None) == \
        W.WALLACE_EINVAL  # waves not a multiple of 4


def test_strerror_and_defaults():
    assert W.strerror(0) == "ok"
    assert "workspace" in W.strerror(W.WALLACE_ENOSPC)
    o = W.make_opts()
    assert (o.f, o.a_mode, o.reduce_mode, o.transform_mode, o.withhold_driver,
            o.check_workspace, o.restart_passes) == (1, 0, 0, 0, 0, 0, 0)


@pytest.mark.parametrize("n,N,ok", [(4, 4, True), (4, 1024, True), (16, 16, True),
                                    (4, 2, False), (16, 8, False), (3, 64, False),
                                    (4, 100, False), (4, 0, False), (8, 64, False)])
def test_workspace_bytes_validation(n, N, ok):
    b = ctypes.c_size_t()
    rc = W.lib().wallace_workspace_bytes(n, N, None, ctypes.byref(b))
    assert (rc == W.WALLACE_OK) == ok
    if ok:
        assert b.value >= 4 * n * N + 256 and b.value % 256 == 0


def test_workspace_grows_with_streaming_pools():
    small = W.workspace_bytes(4, 1 << 14)
    big = W.workspace_bytes(4, 1 << 22)
    assert big >= 2 * 4 * 4 * (1 << 22)  # two pool buffers for the streaming pass
    assert small < 4 * 4 * (1 << 14) * 2


def test_init_argument_errors_before_gpu():
    L = W.lib()
    h = ctypes.c_void_p()
    o = W.make_opts()
    # bad shape, null workspace, misaligned workspace, too small, bad options
    assert L.wallace_init(1, 3, 64, ctypes.byref(o), 256, 1 << 20, None, ctypes.byref(h)) == W.WALLACE_EINVAL
    assert L.wallace_init(1, 4, 64, ctypes.byref(o), None, 1 << 20, None, ctypes.byref(h)) == W.WALLACE_EINVAL
    assert L.wallace_init(1, 4, 64, ctypes.byref(o), 256 + 8, 1 << 20, None, ctypes.byref(h)) == W.WALLACE_EINVAL
    assert L.wallace_init(1, 4, 64, ctypes.byref(o), 4096, 16, None, ctypes.byref(h)) == W.WALLACE_ENOSPC
    bad = W.make_opts(f=0)
    assert L.wallace_init(1, 4, 64, ctypes.byref(bad), 4096, 1 << 20, None, ctypes.byref(h)) == W.WALLACE_EINVAL
    bad = W.make_opts(reduce_mode=3)
    assert L.wallace_init(1, 4, 64, ctypes.byref(bad), 4096, 1 << 20, None, ctypes.byref(h)) == W.WALLACE_EINVAL
    bad = W.make_opts(f=3, restart_passes=10)  # restart interval must be a multiple of f
    assert L.wallace_init(1, 4, 64, ctypes.byref(bad), 4096, 1 << 20, None, ctypes.byref(h)) == W.WALLACE_EINVAL
    bad = W.make_opts(restart_passes=-1)
    assert L.wallace_init(1, 4, 64, ctypes.byref(bad), 4096, 1 << 20, None, ctypes.byref(h)) == W.WALLACE_EINVAL
    mm = W.make_opts(transform_mode=1)  # matrix cores only for n = 16
    assert L.wallace_init(1, 4, 1 << 20, ctypes.byref(mm), 4096, 1 << 40, None, ctypes.byref(h)) == W.WALLACE_EUNSUP
    # ... and for streamed pools of one tuple per thread (n = 16, 2^13 <= N <= 2^20)
    assert L.wallace_init(1, 16, 256, ctypes.byref(mm), 4096, 1 << 40, None, ctypes.byref(h)) == W.WALLACE_EUNSUP
    assert L.wallace_init(1, 16, 1 << 22, ctypes.byref(mm), 4096, 1 << 40, None, ctypes.byref(h)) == W.WALLACE_EUNSUP
    # streamed n = 16 pools take at most 4 tuples per thread: N = 2^22 is the largest
    assert L.wallace_init(1, 16, 1 << 23, None, 4096, 1 << 40, None, ctypes.byref(h)) == W.WALLACE_EUNSUP
    assert not h.value


def test_null_handles():
    L = W.lib()
    assert L.wallace_fill(None, 256, 10, None) == W.WALLACE_EINVAL
    assert L.wallace_fill_static(None, 256, 10, None) == W.WALLACE_EINVAL
    assert L.wallace_sumsq(None, None, None, None) == W.WALLACE_EINVAL
    assert L.wallace_destroy(None) == W.WALLACE_OK
    assert L.wallace_batch_destroy(None) == W.WALLACE_OK
    assert L.wallace_fill_batched(None, 256, 1 << 20, None) == W.WALLACE_EINVAL
    assert L.wallace_batch_plan(None, None, None, None) == W.WALLACE_EINVAL
    assert L.wallace_batch_set_streams(None, 0, None) == W.WALLACE_EINVAL
    assert L.wallace_batch_tune_planned(None, 256, 1 << 20, 256, 1 << 20, None) == W.WALLACE_EINVAL


def test_batch_output_checks_before_any_launch():
    # Batch.fill hands the library a raw pointer; the binding first checks
    # the tensor against the plan's extent (and the library checks out_len)
    import torch
    offsets = np.array([0, 3 * 1024, 10_000], dtype=np.uint64)
    passes = np.array([3, 2, 0], dtype=np.uint32)
    ext = W.batch_extent(offsets, passes, [4, 16, 4], [256, 64, 256])
    assert ext == 3 * 1024 + 2 * 1024
    cpu = torch.device("cpu")
    W.check_batch_output(torch.empty(ext, dtype=torch.float32), ext, cpu)
    with pytest.raises(ValueError):
        W.check_batch_output(torch.empty(ext - 1, dtype=torch.float32), ext, cpu)
    with pytest.raises(TypeError):
        W.check_batch_output(torch.empty(ext, dtype=torch.float16), ext, cpu)
    with pytest.raises(TypeError):
        W.check_batch_output(torch.empty(ext, dtype=torch.float64), ext, cpu)
    with pytest.raises(ValueError):
        W.check_batch_output(torch.empty(2 * ext, dtype=torch.float32)[::2], ext, cpu)
    with pytest.raises(ValueError):
        W.check_batch_output(torch.empty(ext, dtype=torch.float32), ext, torch.device("cuda", 0))
    with pytest.raises(RuntimeError):
        W.check_batch_output(torch.empty(ext, dtype=torch.float32), None, cpu)


def test_batch_workspace_validation():
    L = W.lib()
    b = ctypes.c_size_t()
    n = np.array([4, 16, 4], dtype=np.int32)
    N = np.array([256, 64, 1 << 14], dtype=np.uint32)
    assert L.wallace_batch_workspace_bytes(3, n.ctypes.data, N.ctypes.data, ctypes.byref(b)) == 0
    assert b.value >= 4 * (1024 + 1024 + 65536)
    N2 = np.array([256, 8, 1024], dtype=np.uint32)
    assert L.wallace_batch_workspace_bytes(3, n.ctypes.data, N2.ctypes.data, ctypes.byref(b)) == W.WALLACE_EINVAL
    N3 = np.array([256, 64, 1 << 20], dtype=np.uint32)  # too large to stay on chip
    assert L.wallace_batch_workspace_bytes(3, n.ctypes.data, N3.ctypes.data, ctypes.byref(b)) == W.WALLACE_EUNSUP
    # restarts are for single generators only (checked before the GPU)
    seeds = np.arange(3, dtype=np.uint64)
    o = W.make_opts(restart_passes=8)
    h = ctypes.c_void_p()
    assert L.wallace_batch_init(3, seeds.ctypes.data, n.ctypes.data, N.ctypes.data, ctypes.byref(o),
                                256, 1 << 30, None, ctypes.byref(h)) == W.WALLACE_EUNSUP


@pytest.mark.parametrize("seed,n,N", [(42, 4, 1024), (0, 4, 4), (7, 16, 16),
                                      (43, 4, 256), (12345, 16, 4096),
                                      (2 ** 64 - 1, 4, 64)])
def test_initial_pool_matches_oracle(seed, n, N):
    pool, rng = W.initial_pool(seed, n, N)
    ref64, ref_rng = oracle.initial_pool64(seed, n, N)
    assert rng == ref_rng
    assert np.array_equal(pool.view(np.uint32), ref64.astype(np.float32).view(np.uint32))


def test_initial_pool_matches_oracle_many_seeds():
    for seed in range(200):
        pool, _ = W.initial_pool(1000 + seed, 4, 256)
        ref64, _ = oracle.initial_pool64(1000 + seed, 4, 256)
        assert np.array_equal(pool.view(np.uint32), ref64.astype(np.float32).view(np.uint32))
