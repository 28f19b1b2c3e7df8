"""Caller-supplied device memory (jp_set_allocator) through the C ABI.

Every device buffer of a call must come from the caller's functions and go
back to them; an allocator that runs dry must give JP_ENOMEM with every block
returned; the output stays the oracle's whatever the memory source.
"""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu

JP_ENOMEM = 2


@pytest.fixture(scope="module")
def jp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2002_12459_amd as jp
    return jp


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.int32))).cuda()


def failing_after(jp, n_ok):
    """torch-backed allocator whose (n_ok + 1)-th request returns NULL."""
    import torch
    state = {"calls": 0}

    def alloc(nbytes):
        state["calls"] += 1
        if state["calls"] > n_ok:
            return 0
        return torch.cuda.caching_allocator_alloc(nbytes, 0, torch.cuda.current_stream(0))

    return jp.DeviceAllocator(alloc, torch.cuda.caching_allocator_delete), state


def test_torch_allocator_sees_every_buffer(jp):
    (rx, ry), (sz, sy) = datagen.zipf_edges(40_000, 4_000, 800, 1.1, 7), datagen.zipf_edges(40_000, 4_000, 800, 1.1, 8)
    ex, ez = oracle.two_path(rx, ry, sz, sy)
    h = jp.Handle(0, selector=None, allocator="torch")
    a = h.allocator
    for kw in ({}, {"delta1": 20, "delta2": 8}, {"strategy": "light", "dedup": "global"}):
        x, z, st = h.two_path(dev(rx), dev(ry), dev(sz), dev(sy), **kw)
        np.testing.assert_array_equal(x.cpu().numpy(), ex)
        np.testing.assert_array_equal(z.cpu().numpy(), ez)
    # the result columns were freed after the copy: nothing is live except
    # the handle's own look-back status block
    assert a.n_alloc > 10 and a.n_alloc - a.n_free <= 1
    assert a.peak_bytes > 8 * ex.size
    h.close()
    assert a.live_bytes == 0 and a.n_alloc == a.n_free


def test_star_and_batch_on_caller_memory(jp):
    h = jp.Handle(0, selector=None, allocator="torch")
    rels = [datagen.zipf_edges(20_000, 3_000, 500, 1.3, 40 + i) for i in range(3)]
    (c0, c1, c2), _ = h.star([(dev(a), dev(b)) for a, b in rels], delta1=20, delta2=4)
    e = oracle.star(rels)
    for i, g in enumerate((c0, c1, c2)):
        np.testing.assert_array_equal(g.cpu().numpy(), e[:, i])
    insts = [datagen.batch_instance(i, hi=2e4) for i in range(6)]
    outs, _ = h.two_path_batch([tuple(dev(c) for c in (rx, ry, sz, sy)) for (rx, ry), (sz, sy) in insts])
    for ((rx, ry), (sz, sy)), (x, z) in zip(insts, outs):
        ex, ez = oracle.two_path(rx, ry, sz, sy)
        np.testing.assert_array_equal(x.cpu().numpy(), ex)
        np.testing.assert_array_equal(z.cpu().numpy(), ez)
    a = h.allocator
    h.close()
    assert a.live_bytes == 0 and a.n_alloc == a.n_free > 0


@pytest.mark.parametrize("n_ok", [0, 1, 5, 17, 40])
def test_allocator_running_dry_gives_enomem_and_leaks_nothing(jp, n_ok):
    rx, ry = datagen.zipf_edges(30_000, 3_000, 600, 1.2, 11)
    sz, sy = datagen.zipf_edges(30_000, 3_000, 600, 1.2, 12)
    h = jp.Handle(0, selector=None)
    a, state = failing_after(jp, n_ok)
    h.set_allocator(a)
    with pytest.raises(jp.JoinProjectError) as e:
        h.two_path(dev(rx), dev(ry), dev(sz), dev(sy), delta1=16, delta2=6)
    assert e.value.status == JP_ENOMEM
    # at most the handle's own look-back status block (kept between calls)
    # is still out; changing the source returns it
    assert a.live_bytes <= 8 << 16
    h.set_allocator(None)
    assert a.live_bytes == 0 and a.n_alloc == a.n_free
    # the handle still works once memory is available again
    x, z, _ = h.two_path(dev(rx), dev(ry), dev(sz), dev(sy), delta1=16, delta2=6)
    ex, ez = oracle.two_path(rx, ry, sz, sy)
    np.testing.assert_array_equal(x.cpu().numpy(), ex)
    np.testing.assert_array_equal(z.cpu().numpy(), ez)
    h.close()


def test_results_return_memory_to_their_own_source(jp):
    rx, ry = datagen.uniform_edges(5_000, 700, 300, 21)
    h = jp.Handle(0, selector=None, allocator="torch")
    first = h.allocator
    r = h.two_path_result(dev(rx), dev(ry), dev(rx), dev(ry))
    second = jp.torch_allocator(0)
    h.set_allocator(second)
    held = first.live_bytes
    assert held >= 8 * r.n
    x, z = r.to_torch()
    r.free()
    assert first.live_bytes == 0
    ex, ez = oracle.two_path(rx, ry, rx, ry)
    np.testing.assert_array_equal(x.cpu().numpy(), ex)
    np.testing.assert_array_equal(z.cpu().numpy(), ez)
    h.close()
    assert second.live_bytes == 0


def test_mixed_null_functions_are_rejected(jp):
    import ctypes
    lib = jp._load()
    h = jp.Handle(0, selector=None)
    a = jp.torch_allocator(0)
    assert lib.jp_set_allocator(h._p, a.c_alloc, jp._FREE_FN(), None) == 1
    assert lib.jp_set_allocator(None, a.c_alloc, a.c_free, None) == 1
    h.close()
