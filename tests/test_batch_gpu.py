"""Batched two-path evaluation through the C ABI against the CPU oracle,
instance by instance."""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("checks_mode")]


@pytest.fixture(scope="module")
def jp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2002_12459_amd as jp
    return jp


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.int32))).cuda()


def run_batch(jp, insts, **kw):
    outs, st = jp.default_handle(0).two_path_batch([tuple(dev(c) for c in i) for i in insts], **kw)
    return [(x.cpu().numpy(), z.cpu().numpy()) for x, z in outs], st


def check(jp, insts, **kw):
    outs, st = run_batch(jp, insts, **kw)
    assert len(outs) == len(insts)
    for k, ((rx, ry, sz, sy), (x, z)) in enumerate(zip(insts, outs)):
        ex, ez = oracle.two_path(rx, ry, sz, sy)
        assert np.array_equal(x, ex) and np.array_equal(z, ez), f"instance {k}"
    return outs, st


def mixed_instances(signed):
    """Mixed batch; with signed ids the instances' id ranges add up to more
    than 2^31 values, which switches the batch to ranked ids."""
    insts = []
    (rx, ry) = datagen.selfjoin_c1()
    insts.append((rx, ry, rx, ry))
    for i in range(6):
        r = datagen.random_small(40 + 13 * i, 12, 7, seed=100 + i, dup=True, signed=signed and i % 2 == 1)
        s = datagen.random_small(35 + 11 * i, 9, 7, seed=200 + i, dup=True, signed=signed and i % 2 == 1)
        insts.append((r[0], r[1], s[0], s[1]))
    z = np.zeros(0, np.int32)
    insts.append((z, z, z, z))                                   # empty
    r = datagen.random_small(30, 5, 5, seed=7)
    insts.append((r[0], r[1], z, z))                             # S empty
    insts.append((np.array([5], np.int32), np.array([9], np.int32),
                  np.array([6], np.int32), np.array([8], np.int32)))  # no common y
    insts.append((np.array([-2**31, -2**31 + 5], np.int32), np.array([0, 0], np.int32),
                  np.array([2**31 - 1], np.int32), np.array([0], np.int32)))  # extreme ids
    (a, b), (c, d), _ = datagen.selector_instance(4, lo=2e3, hi=8e3)
    insts.append((a, b, c, d))
    return insts


@pytest.mark.parametrize("kw", [{}, {"strategy": "light"}, {"strategy": "fixed", "delta1": 3, "delta2": 2},
                                {"strategy": "fixed", "delta1": 1, "delta2": 1}, {"dedup": "global"},
                                {"strategy": "theory"}])
@pytest.mark.parametrize("signed", [False, True])
def test_mixed_batch_matches_oracle(jp, kw, signed):
    check(jp, mixed_instances(signed), **kw)


def test_empty_batch(jp):
    outs, st = run_batch(jp, [])
    assert outs == []


def test_all_instances_empty(jp):
    z = np.zeros(0, np.int32)
    outs, _ = run_batch(jp, [(z, z, z, z)] * 3)
    assert all(x.size == 0 and z_.size == 0 for x, z_ in outs)


def test_batch_shaped_like_the_serving_set(jp):
    """64 instances with the serving set's size mix, scaled down so the
    oracle checks every instance."""
    insts = [(r[0], r[1], s[0], s[1]) for r, s in datagen.batch_c4(64, lo=1e2, hi=2e4, seed0=5000)]
    outs, st = check(jp, insts)
    assert st["n_out"] == sum(x.size for x, _ in outs)


def test_batch_with_heavy_part(jp):
    insts = [(r[0], r[1], s[0], s[1]) for r, s in datagen.batch_c4(24, lo=2e3, hi=2e4, seed0=7000)]
    outs, st = check(jp, insts, strategy="fixed", delta1=20, delta2=4)
    assert st["u"] > 0 and st["v"] > 0 and st["w"] > 0 and st["nnz_heavy"] > 0


def test_full_int32_ranges_per_instance(jp):
    a = np.array([-2**31, 2**31 - 1, 0], np.int32)
    b = np.array([0, 1, 1], np.int32)
    insts = [(a, b, a, b), (a, b, a[::-1].copy(), b), (b, a, b, a)]
    check(jp, insts)
