"""Graph-captured batch plans (jp_two_path_batch_plan / jp_plan_launch).

A plan's replays must give the oracle's output for every instance, on
several replays in a row with other GPU work and waits between them; a too
small arena must give JP_ECAPACITY with a size that then works; changed
inputs must be refused before any replay.
"""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu

JP_ECAPACITY = 4


@pytest.fixture(scope="module")
def jp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2002_12459_amd as jp
    return jp


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.int32))).cuda()


@pytest.fixture(scope="module")
def insts():
    return [datagen.batch_instance(i, hi=3e4) for i in range(40)]


@pytest.fixture(scope="module")
def expected(insts):
    return [oracle.two_path(rx, ry, sz, sy) for (rx, ry), (sz, sy) in insts]


def check_outputs(plan, expected):
    outs = plan.outputs()
    assert len(outs) == len(expected)
    for i, ((x, z), (ex, ez)) in enumerate(zip(outs, expected)):
        np.testing.assert_array_equal(x.cpu().numpy(), ex, err_msg=f"instance {i}")
        np.testing.assert_array_equal(z.cpu().numpy(), ez, err_msg=f"instance {i}")


@pytest.mark.parametrize("kw", [{}, {"strategy": "light"}, {"delta1": 8, "delta2": 4}, {"dedup": "global"},
                                {"strategy": "mlp"}])
def test_plan_replays_match_the_oracle(jp, insts, expected, kw):
    import torch
    h = jp.Handle(0)
    cols = [tuple(dev(c) for c in (rx, ry, sz, sy)) for (rx, ry), (sz, sy) in insts]
    with pytest.raises(jp.JoinProjectError) as e:
        h.batch_plan(cols, arena_bytes=1 << 16, **kw)
    assert e.value.status == JP_ECAPACITY and e.value.arena_needed > 1 << 16
    plan = h.batch_plan(cols, arena_bytes=e.value.arena_needed, **kw)
    for rep in range(3):
        plan.launch()
        check_outputs(plan, expected)
        # eager work and a wait between replays
        outs, _ = h.two_path_batch(cols, **kw)
        torch.cuda.synchronize()
        for (x, z), (ex, ez) in zip(outs, expected):
            np.testing.assert_array_equal(x.cpu().numpy(), ex)
    plan.free()
    h.close()


def test_caller_arena_and_changed_inputs(jp, insts, expected):
    import torch
    h = jp.Handle(0)
    cols = [tuple(dev(c) for c in (rx, ry, sz, sy)) for (rx, ry), (sz, sy) in insts[:12]]
    probe = None
    try:
        h.batch_plan(cols, arena_bytes=256)
    except jp.JoinProjectError as e:
        probe = e.arena_needed
    assert probe
    arena = torch.empty(probe, dtype=torch.uint8, device="cuda")
    plan = h.batch_plan(cols, arena=arena)
    plan.launch()
    check_outputs(plan, expected[:12])
    # change one input column in place: the plan refuses to replay
    cols[3][1][:5] = cols[3][1][:5].flip(0) + 1
    with pytest.raises(jp.JoinProjectError) as e:
        plan.launch()
    assert e.value.status == JP_ECAPACITY
    plan.free()
    # a new plan on the new contents
    (rx, ry), (sz, sy) = insts[3]
    plan = h.batch_plan(cols, arena_bytes=4 * probe)
    plan.launch()
    outs = plan.outputs()
    ex, ez = oracle.two_path(rx, cols[3][1].cpu().numpy(), sz, sy)
    np.testing.assert_array_equal(outs[3][0].cpu().numpy(), ex)
    np.testing.assert_array_equal(outs[3][1].cpu().numpy(), ez)
    plan.free()
    h.close()


def test_single_instance_plan_with_heavy_product(jp):
    rx, ry = datagen.zipf_edges(60_000, 6_000, 1_200, 1.1, 77)
    sz, sy = datagen.zipf_edges(60_000, 6_000, 1_200, 1.1, 78)
    ex, ez = oracle.two_path(rx, ry, sz, sy)
    h = jp.Handle(0)
    cols = [(dev(rx), dev(ry), dev(sz), dev(sy))]
    plan = h.batch_plan(cols, arena_bytes=1 << 30, delta1=40, delta2=8, bmm="auto")
    for _ in range(4):
        plan.launch()
        (x, z), = plan.outputs()
        np.testing.assert_array_equal(x.cpu().numpy(), ex)
        np.testing.assert_array_equal(z.cpu().numpy(), ez)
    plan.free()
    h.close()
