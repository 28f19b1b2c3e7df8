"""Device primitives (radix sort, scan, unique) against numpy, through the
test hooks of include/jp_testing.h."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hk():
    import torch
    import paper_2002_12459_amd as jp
    lib = jp._load()
    P = ctypes.c_void_p
    for f in ("jp_test_radix_sort_u64", "jp_test_radix_sort_u32", "jp_test_radix_sort_u128"):
        getattr(lib, f).argtypes = [P, P, ctypes.c_int64, ctypes.c_int32]
        getattr(lib, f).restype = ctypes.c_int
    lib.jp_test_exclusive_scan.argtypes = [P, P, P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    lib.jp_test_exclusive_scan.restype = ctypes.c_int
    lib.jp_test_unique_u64.argtypes = [P, P, ctypes.c_int64, P, ctypes.POINTER(ctypes.c_int64)]
    lib.jp_test_unique_u64.restype = ctypes.c_int
    h = jp.default_handle(0)
    h._bind_stream()
    return lib, h, torch


SIZES = [1, 2, 63, 64, 65, 1000, 4096, 4097, 100_003, 1_000_000]


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("bits", [6, 20, 40, 64])
def test_radix_sort_u64(hk, n, bits):
    lib, h, torch = hk
    rng = np.random.default_rng(n + bits)
    hi = (1 << bits) if bits < 64 else None
    a = rng.integers(0, hi if hi else 2**63, n, dtype=np.uint64 if bits == 64 else np.int64).astype(np.uint64)
    if bits == 64:
        a |= (rng.integers(0, 2, n).astype(np.uint64) << np.uint64(63))
    if n > 10:
        a[: n // 3] = a[0]  # heavy repeats
    t = torch.from_numpy(a.view(np.int64).copy()).cuda()
    assert lib.jp_test_radix_sort_u64(h._p, ctypes.c_void_p(t.data_ptr()), n, bits) == 0
    got = t.cpu().numpy().view(np.uint64)
    np.testing.assert_array_equal(got, np.sort(a))


@pytest.mark.parametrize("bits", [12, 38, 64])
def test_radix_sort_u64_many_tiles(hk, bits):
    """10M keys: thousands of tiles resolve their digit offsets by look-back."""
    lib, h, torch = hk
    n = 10_000_000
    rng = np.random.default_rng(bits)
    a = rng.integers(0, 2**63, n, dtype=np.int64).astype(np.uint64)
    if bits < 64:
        a &= np.uint64((1 << bits) - 1)
    else:
        a |= (rng.integers(0, 2, n).astype(np.uint64) << np.uint64(63))
    a[::7] = a[3]  # one very frequent key
    t = torch.from_numpy(a.view(np.int64).copy()).cuda()
    assert lib.jp_test_radix_sort_u64(h._p, ctypes.c_void_p(t.data_ptr()), n, bits) == 0
    np.testing.assert_array_equal(t.cpu().numpy().view(np.uint64), np.sort(a))


@pytest.mark.parametrize("n", [1, 65, 4097, 300_000, 3_000_000])
@pytest.mark.parametrize("bits", [40, 72, 128])
def test_radix_sort_u128(hk, n, bits):
    """16-byte keys: up to 16 digit passes (histograms counted in two launches)."""
    lib, h, torch = hk
    rng = np.random.default_rng(n * 3 + bits)
    lo = rng.integers(0, 2**63, n, dtype=np.int64).astype(np.uint64) | (rng.integers(0, 2, n).astype(np.uint64) << np.uint64(63))
    hi = rng.integers(0, 2**63, n, dtype=np.int64).astype(np.uint64) | (rng.integers(0, 2, n).astype(np.uint64) << np.uint64(63))
    if bits <= 64:
        hi[:] = 0
        if bits < 64:
            lo &= np.uint64((1 << bits) - 1)
    elif bits < 128:
        hi &= np.uint64((1 << (bits - 64)) - 1)
    if n > 10:
        lo[: n // 4] = lo[0]
        hi[: n // 4] = hi[0]
    words = np.stack([lo, hi], axis=1).reshape(-1)
    t = torch.from_numpy(words.view(np.int64).copy()).cuda()
    assert t.data_ptr() % 16 == 0
    assert lib.jp_test_radix_sort_u128(h._p, ctypes.c_void_p(t.data_ptr()), n, bits) == 0
    got = t.cpu().numpy().view(np.uint64).reshape(-1, 2)
    order = np.lexsort((lo, hi))
    np.testing.assert_array_equal(got[:, 0], lo[order])
    np.testing.assert_array_equal(got[:, 1], hi[order])


@pytest.mark.parametrize("n", SIZES + [10_000_000])
def test_radix_sort_u32(hk, n):
    lib, h, torch = hk
    rng = np.random.default_rng(n)
    a = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    t = torch.from_numpy(a.view(np.int32).copy()).cuda()
    assert lib.jp_test_radix_sort_u32(h._p, ctypes.c_void_p(t.data_ptr()), n, 32) == 0
    np.testing.assert_array_equal(t.cpu().numpy().view(np.uint32), np.sort(a))


@pytest.mark.parametrize("n", SIZES + [20_000_000])
def test_exclusive_scan(hk, n):
    lib, h, torch = hk
    rng = np.random.default_rng(n)
    a = rng.integers(0, 1000, n).astype(np.int64)
    t = torch.from_numpy(a).cuda()
    o = torch.empty_like(t)
    tot = ctypes.c_int64()
    assert lib.jp_test_exclusive_scan(h._p, ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(o.data_ptr()), n,
                                      ctypes.byref(tot)) == 0
    ex = np.concatenate([[0], np.cumsum(a)[:-1]])
    np.testing.assert_array_equal(o.cpu().numpy(), ex)
    assert tot.value == a.sum()


@pytest.mark.parametrize("n", SIZES)
def test_unique(hk, n):
    lib, h, torch = hk
    rng = np.random.default_rng(n)
    a = np.sort(rng.integers(0, max(2, n // 3), n)).astype(np.int64)
    t = torch.from_numpy(a).cuda()
    o = torch.empty_like(t)
    m = ctypes.c_int64()
    assert lib.jp_test_unique_u64(h._p, ctypes.c_void_p(t.data_ptr()), n, ctypes.c_void_p(o.data_ptr()),
                                  ctypes.byref(m)) == 0
    u = np.unique(a)
    assert m.value == u.size
    np.testing.assert_array_equal(o.cpu().numpy()[: m.value], u)
