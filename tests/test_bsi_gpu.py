"""Batched Boolean set intersection through the C ABI (jp_bsi) against the
oracle's per-query set intersection: every answer must match, for batches
with repeated queries, ids absent from the relations, and at thresholds that
exercise the light path, the heavy product and both."""
import numpy as np
import pytest

import datagen
import oracle
from tests.conftest import load_golden

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


def check(jp, rx, ry, sz, sy, tx, tz, **kw):
    want = oracle.bsi(rx, ry, sz, sy, tx, tz)
    ans, st = jp.default_handle(0).bsi(dev(rx), dev(ry), dev(sz), dev(sy), dev(tx), dev(tz), **kw)
    got = ans.cpu().numpy().astype(bool)
    assert got.size == want.size
    np.testing.assert_array_equal(got, want)
    return want, st


def mixed_batch(rx, sz, n, seed, pairs=None):
    """Queries: half from known intersecting pairs (when given), the rest
    random ids of the relations plus some ids that occur nowhere."""
    rng = np.random.default_rng(seed)
    parts_x, parts_z = [], []
    if pairs is not None and pairs[0].size:
        i = rng.integers(0, pairs[0].size, n // 2)
        parts_x.append(pairs[0][i])
        parts_z.append(pairs[1][i])
    m = n - sum(p.size for p in parts_x)
    parts_x.append(np.concatenate([rng.choice(rx, m - m // 8), rng.integers(-2**31, 2**31 - 1, m // 8)]))
    parts_z.append(np.concatenate([rng.choice(sz, m - m // 8), rng.integers(-2**31, 2**31 - 1, m // 8)]))
    tx = np.concatenate(parts_x).astype(np.int32)
    tz = np.concatenate(parts_z).astype(np.int32)
    p = rng.permutation(tx.size)
    return tx[p], tz[p]


@pytest.mark.parametrize("kw", [{"delta1": 2, "delta2": 2}, {"strategy": "light"}, {"delta1": 1, "delta2": 1}, {}])
def test_worked_example(jp, kw):
    rows = load_golden("two_path_example.txt")
    R = np.array([(int(r[1]), int(r[2])) for r in rows if r[0] == "R"])
    S = np.array([(int(r[1]), int(r[2])) for r in rows if r[0] == "S"])
    tx = [4, 4, 1, 2, 3, 6, 7, 5, 1, 4, 4]
    tz = [3, 4, 3, 2, 6, 2, 1, 5, 1, 4, 9]
    want, _ = check(jp, R[:, 0], R[:, 1], S[:, 0], S[:, 1], tx, tz, **kw)
    assert want.tolist() == [False, True, False, False, True, False, False, True, True, True, False]


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("d", [1, 2, None])
def test_random_small(jp, seed, d):
    x, y = datagen.random_small(800, 80, 50, seed=1200 + seed, dup=True, signed=seed % 2 == 1)
    rx, ry, sz, sy = x[0::2], y[0::2], x[1::2], y[1::2]
    tx, tz = mixed_batch(rx, sz, 300, seed, oracle.two_path(rx, ry, sz, sy))
    kw = {"strategy": "light"} if d is None else {"delta1": d, "delta2": d}
    check(jp, rx, ry, sz, sy, tx, tz, **kw)


@pytest.mark.parametrize("kw", [{}, {"strategy": "light"}, {"delta1": 30, "delta2": 6}])
@pytest.mark.parametrize("batch", [1, 100, 5000])
def test_zipf_batches(jp, kw, batch):
    rx, ry = datagen.zipf_edges(50_000, 5_000, 1_000, 1.1, 41)
    sz, sy = datagen.zipf_edges(50_000, 5_000, 1_000, 1.1, 42)
    tx, tz = mixed_batch(rx, sz, batch, batch, oracle.two_path(rx, ry, sz, sy))
    want, st = check(jp, rx, ry, sz, sy, tx, tz, **kw)
    if batch == 5000:
        assert want.any() and not want.all()


def test_empty_inputs(jp):
    a = dev([1, 2, 3])
    ans, _ = jp.default_handle(0).bsi(a, a, a, a, dev([]), dev([]))
    assert ans.numel() == 0
    ans, _ = jp.default_handle(0).bsi(dev([]), dev([]), a, a, a, a)
    assert not ans.cpu().numpy().any()
