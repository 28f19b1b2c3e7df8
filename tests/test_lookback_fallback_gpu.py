"""The look-back fallback of the single-pass scans and compactions.

Every scan and compaction tile waits a bounded time for each predecessor
tile's published status and otherwise computes that tile's sum from the
input itself.  On MI355X the fallback is not taken in normal runs, so these
tests force it on a handle of their own (wait limit 0: every status not yet
visible at the first read is recomputed) and check the primitives and whole
pipelines against numpy and the oracle.
"""
import ctypes

import numpy as np
import pytest

import datagen
import oracle

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("checks_mode")]


@pytest.fixture(scope="module")
def fb():
    import torch
    import paper_2002_12459_amd as jp
    lib = jp._load()
    P = ctypes.c_void_p
    lib.jp_test_set_lookback_wait.argtypes = [P, ctypes.c_int64]
    lib.jp_test_set_lookback_wait.restype = ctypes.c_int
    lib.jp_test_exclusive_scan.argtypes = [P, P, P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    lib.jp_test_exclusive_scan.restype = ctypes.c_int
    lib.jp_test_unique_u64.argtypes = [P, P, ctypes.c_int64, P, ctypes.POINTER(ctypes.c_int64)]
    lib.jp_test_unique_u64.restype = ctypes.c_int
    lib.jp_test_radix_sort_u64.argtypes = [P, P, ctypes.c_int64, ctypes.c_int32]
    lib.jp_test_radix_sort_u64.restype = ctypes.c_int
    h = jp.Handle(0, selector=None)
    assert lib.jp_test_set_lookback_wait(h._p, -1) == 1  # JP_EINVAL
    assert lib.jp_test_set_lookback_wait(h._p, 0) == 0
    h._bind_stream()
    return lib, h, torch


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.int32))).cuda()


@pytest.mark.parametrize("n", [4097, 300_000, 3_000_001])
def test_scan_with_fallback(fb, n):
    lib, h, torch = fb
    a = np.random.default_rng(n).integers(0, 1000, n).astype(np.int64)
    t = torch.from_numpy(a).cuda()
    out = torch.empty_like(t)
    tot = ctypes.c_int64()
    assert lib.jp_test_exclusive_scan(h._p, ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(out.data_ptr()), n,
                                      ctypes.byref(tot)) == 0
    ex = np.concatenate([[0], np.cumsum(a)[:-1]])
    np.testing.assert_array_equal(out.cpu().numpy(), ex)
    assert tot.value == int(a.sum())


@pytest.mark.parametrize("n", [5000, 2_000_003])
def test_unique_and_sort_with_fallback(fb, n):
    lib, h, torch = fb
    rng = np.random.default_rng(n)
    a = rng.integers(0, 1 << 40, n).astype(np.uint64)
    a[::5] = a[1]
    t = torch.from_numpy(a.view(np.int64).copy()).cuda()
    assert lib.jp_test_radix_sort_u64(h._p, ctypes.c_void_p(t.data_ptr()), n, 40) == 0
    s = np.sort(a)
    np.testing.assert_array_equal(t.cpu().numpy().view(np.uint64), s)
    out = torch.empty_like(t)
    m = ctypes.c_int64()
    assert lib.jp_test_unique_u64(h._p, ctypes.c_void_p(t.data_ptr()), n, ctypes.c_void_p(out.data_ptr()),
                                  ctypes.byref(m)) == 0
    u = np.unique(s)
    assert m.value == u.size
    np.testing.assert_array_equal(out[: m.value].cpu().numpy().view(np.uint64), u)


@pytest.mark.parametrize("kw", [{}, {"strategy": "fixed", "delta1": 30, "delta2": 6}])
def test_two_path_with_fallback(fb, kw):
    _, h, _ = fb
    (rx, ry), (sz, sy) = datagen.twopath_c2(0.01)
    x, z, st = h.two_path(dev(rx), dev(ry), dev(sz), dev(sy), **kw)
    ex, ez = oracle.two_path(rx, ry, sz, sy)
    np.testing.assert_array_equal(x.cpu().numpy(), ex)
    np.testing.assert_array_equal(z.cpu().numpy(), ez)


def test_star_with_fallback(fb):
    _, h, _ = fb
    rels = datagen.star_c3(0.01)
    cols, _ = h.star([(dev(a), dev(b)) for a, b in rels])
    exp = oracle.star(rels)
    for i in range(3):
        np.testing.assert_array_equal(cols[i].cpu().numpy(), exp[:, i])


def test_batch_with_fallback(fb):
    _, h, _ = fb
    insts = [datagen.batch_instance(i, lo=1e3, hi=3e4) for i in range(6)]
    r = h.two_path_batch_result([(dev(a[0]), dev(a[1]), dev(b[0]), dev(b[1])) for a, b in insts])
    try:
        x, z = r.to_torch()
        offs = r.batch_offsets()
    finally:
        r.free()
    for i, ((rx, ry), (sz, sy)) in enumerate(insts):
        ex, ez = oracle.two_path(rx, ry, sz, sy)
        np.testing.assert_array_equal(x[offs[i]:offs[i + 1]].cpu().numpy(), ex, err_msg=f"instance {i}")
        np.testing.assert_array_equal(z[offs[i]:offs[i + 1]].cpu().numpy(), ez, err_msg=f"instance {i}")
