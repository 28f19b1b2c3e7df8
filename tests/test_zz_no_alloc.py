"""jp_two_path_static: the no-allocation entry point against jp_two_path.

Its pairs must equal jp_two_path's bit for bit, on two calls in a row (the
second on a smaller input, so stale contents of the shared device array from
the first call would show), at cost-model, forced-heavy and light-only
thresholds; it must make no request to the handle's allocator; and it must
refuse what does not fit with the documented status.
"""
import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu

JP_EINVAL, JP_ENOMEM, JP_ECAPACITY = 1, 2, 4


@pytest.fixture(scope="module")
def jp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2002_12459_amd as jp
    return jp


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.int32))).cuda()


def static_pairs(h, R, S, cap, **kw):
    import torch
    ox = torch.full((cap,), -7, dtype=torch.int32, device="cuda")
    oz = torch.full((cap,), -7, dtype=torch.int32, device="cuda")
    n, st = h.two_path_static(dev(R[0]), dev(R[1]), dev(S[0]), dev(S[1]), ox, oz, **kw)
    assert (ox[n:] == -7).all() and (oz[n:] == -7).all(), "wrote past the output"
    return ox[:n].cpu().numpy(), oz[:n].cpu().numpy(), st


def allocating_pairs(h, R, S, **kw):
    x, z, st = h.two_path(dev(R[0]), dev(R[1]), dev(S[0]), dev(S[1]), **kw)
    return x.cpu().numpy(), z.cpu().numpy(), st


@pytest.mark.parametrize("kw", [{}, {"delta1": 200, "delta2": 12}, {"strategy": "light"},
                                {"strategy": "light", "dedup": "global"}])
def test_static_matches_allocating_entry_point_twice(jp, kw):
    big = (datagen.zipf_edges(300_000, 30_000, 6_000, 1.1, 91), datagen.zipf_edges(280_000, 30_000, 6_000, 1.1, 92))
    small = (datagen.zipf_edges(20_000, 2_000, 400, 1.3, 93), datagen.zipf_edges(25_000, 2_000, 400, 1.3, 94))
    h = jp.Handle(0, selector=None, allocator="torch")
    for R, S in (big, small):
        ex, ez, est = allocating_pairs(h, R, S, **kw)
        a = h.allocator
        before = (a.n_alloc, a.n_free, a.live_bytes)
        x, z, st = static_pairs(h, R, S, ex.size + 1000, **kw)
        assert (a.n_alloc, a.n_free, a.live_bytes) == before, "the static entry point used the allocator"
        assert st["n_out"] == est["n_out"] == ex.size
        np.testing.assert_array_equal(x, ex)
        np.testing.assert_array_equal(z, ez)
        assert (st["J"], st["u"], st["v"], st["w"]) == (est["J"], est["u"], est["v"], est["w"])
    h.close()


def test_static_capacity_and_size_limits(jp):
    import torch
    R = datagen.uniform_edges(30_000, 3_000, 300, 5)
    h = jp.Handle(0, selector=None)
    ex, ez, _ = allocating_pairs(h, R, R)
    with pytest.raises(jp.JoinProjectError) as e:
        static_pairs(h, R, R, ex.size - 1)
    assert e.value.status == JP_ECAPACITY and e.value.n_out == ex.size
    x, z, _ = static_pairs(h, R, R, ex.size)  # exact fit
    np.testing.assert_array_equal(x, ex)
    np.testing.assert_array_equal(z, ez)
    # more than 2^19 edges per relation: refused before any device work
    big = torch.zeros((1 << 19) + 1, dtype=torch.int32, device="cuda")
    out = torch.empty(16, dtype=torch.int32, device="cuda")
    with pytest.raises(jp.JoinProjectError) as e:
        h.two_path_static(big, big, dev(R[0]), dev(R[1]), out, out.clone())
    assert e.value.status == JP_EINVAL
    # within the edge limit but with a join too large for the array: every
    # x meets every z through 8 y (J = 8 * 4000^2 = 1.28e8 witnesses)
    xs = np.repeat(np.arange(4000), 8)
    ys = np.tile(np.arange(8), 4000)
    with pytest.raises(jp.JoinProjectError) as e:
        static_pairs(h, (xs, ys), (xs, ys), 1 << 24, strategy="light", dedup="global")
    assert e.value.status == JP_ENOMEM
    # and the array is usable again afterwards
    x, z, _ = static_pairs(h, R, R, ex.size)
    np.testing.assert_array_equal(x, ex)
    np.testing.assert_array_equal(z, ez)
    h.close()
