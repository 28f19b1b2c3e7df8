"""Parity at the benchmark sizes: whole outputs against the oracle.

The 10M x 10M two-path input (cost-model, light-only and forced heavy
thresholds), the 3 x 2M star input and all 512 instances of the batched set
are compared element by element with the oracle's full output, with the
library's stage validation on ("checked") and off ("shipped", the
configuration the benchmark times).  The oracle runs its OpenMP variant
(pinned to the plain one by the CPU tests) or, for the batch, its plain form
on host threads, one instance per thread.
"""
import concurrent.futures as cf
import multiprocessing as mp

import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def jp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2002_12459_amd as jp
    return jp


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.int32))).cuda()


def host_threads():
    return max(1, min(16, oracle.cores()))


@pytest.fixture(scope="module")
def c2():
    return datagen.twopath_c2(1.0)


@pytest.fixture(scope="module")
def c2_oracle(c2):
    (rx, ry), (sz, sy) = c2
    return oracle.two_path_par(rx, ry, sz, sy, threads=host_threads())


@pytest.mark.parametrize("kw", [{}, {"strategy": "light"}, {"strategy": "fixed", "delta1": 1000, "delta2": 12}])
def test_two_path_10m(jp, c2, c2_oracle, checks_mode, kw):
    (rx, ry), (sz, sy) = c2
    ex, ez = c2_oracle
    h = jp.default_handle(0)
    x, z, st = h.two_path(dev(rx), dev(ry), dev(sz), dev(sy), **kw)
    assert st["n_out"] == x.numel() == ex.size
    np.testing.assert_array_equal(x.cpu().numpy(), ex)
    np.testing.assert_array_equal(z.cpu().numpy(), ez)
    assert st["J"] == oracle.join_size(rx, ry, sz, sy)
    if kw.get("strategy") == "fixed":
        assert st["u"] > 0 and st["v"] > 0 and st["w"] > 0 and st["nnz_heavy"] > 0


@pytest.fixture(scope="module")
def c3():
    return datagen.star_c3(1.0)


@pytest.fixture(scope="module")
def c3_oracle(c3):
    return oracle.star_par(c3, threads=host_threads())


@pytest.mark.parametrize("kw", [{}, {"strategy": "light"}, {"strategy": "fixed", "delta1": 20, "delta2": 4}])
def test_star_3x2m(jp, c3, c3_oracle, checks_mode, kw):
    h = jp.default_handle(0)
    cols, st = h.star([(dev(a), dev(b)) for a, b in c3], **kw)
    assert st["n_out"] == cols[0].numel() == c3_oracle.shape[0]
    for i in range(3):
        np.testing.assert_array_equal(cols[i].cpu().numpy(), c3_oracle[:, i])
    if kw.get("strategy") == "fixed":  # the chained product runs (119 heavy y; 13.5K, 3.4K, 0.5K heavy x)
        assert st["v"] > 0 and st["u"] > 0 and st["w"] > 0


@pytest.fixture(scope="module")
def c4():
    # numpy-only generation in fresh interpreters (nothing inherited from a
    # process that holds the GPU)
    with mp.get_context("spawn").Pool(host_threads()) as pool:
        return pool.map(datagen.batch_instance, range(512), chunksize=4)


def test_batch_512(jp, c4, checks_mode):
    """Every instance of the serving-style set in full against the oracle."""
    insts = c4
    h = jp.default_handle(0)
    r = h.two_path_batch_result([(dev(a[0]), dev(a[1]), dev(b[0]), dev(b[1])) for a, b in insts])
    try:
        x, z = r.to_torch()
        offs = r.batch_offsets()
    finally:
        r.free()
    assert offs[0] == 0 and offs[-1] == x.numel() and len(offs) == 513
    x, z = x.cpu().numpy(), z.cpu().numpy()

    def check(i):
        (rx, ry), (sz, sy) = insts[i]
        ex, ez = oracle.two_path(rx, ry, sz, sy)
        gx, gz = x[offs[i]:offs[i + 1]], z[offs[i]:offs[i + 1]]
        return i, ex.size, gx.size, bool(np.array_equal(gx, ex) and np.array_equal(gz, ez))

    # largest instances first, so the pool's last tasks are short
    order = sorted(range(512), key=lambda i: -insts[i][0][0].size)
    with cf.ThreadPoolExecutor(host_threads()) as ex:
        results = list(ex.map(check, order))
    bad = [(i, e, g) for i, e, g, ok in results if not ok]
    assert not bad, f"instances differing from the oracle (index, oracle size, GPU size): {bad[:10]}"


# ---------------------------------------------------------------------------
# The further rows at their benchmark sizes: set similarity join and batched
# set intersection on the 10M input, the k = 4 star on 4 x 500K edges.
# ---------------------------------------------------------------------------

def test_ssj_10m(jp, c2, checks_mode):
    """Pairs sharing >= 2 elements, with overlaps, in both orders."""
    (rx, ry), (sz, sy) = c2
    ex, ez, en = oracle.ssj(rx, ry, sz, sy, c=2)
    h = jp.default_handle(0)
    x, z, n, st = h.ssj(dev(rx), dev(ry), dev(sz), dev(sy), min_overlap=2)
    np.testing.assert_array_equal(x.cpu().numpy(), ex)
    np.testing.assert_array_equal(z.cpu().numpy(), ez)
    np.testing.assert_array_equal(n.cpu().numpy(), en)
    order = np.lexsort((ez, ex, -en.astype(np.int64)))  # overlap descending, then (x, z)
    x, z, n, st = h.ssj(dev(rx), dev(ry), dev(sz), dev(sy), min_overlap=2, ordered=True, delta1=1000, delta2=12)
    assert st["nnz_heavy"] > 0
    np.testing.assert_array_equal(x.cpu().numpy(), ex[order])
    np.testing.assert_array_equal(z.cpu().numpy(), ez[order])
    np.testing.assert_array_equal(n.cpu().numpy(), en[order])


@pytest.mark.parametrize("kw", [{}, {"strategy": "light"}, {"delta1": 1000, "delta2": 12}])
def test_bsi_10m(jp, c2, checks_mode, kw):
    (rx, ry), (sz, sy) = c2
    tx, tz = datagen.bsi_batch(rx, ry, sz, sy, 100_000, seed=17)
    want = oracle.bsi(rx, ry, sz, sy, tx, tz)
    ans, _ = jp.default_handle(0).bsi(dev(rx), dev(ry), dev(sz), dev(sy), dev(tx), dev(tz), **kw)
    np.testing.assert_array_equal(ans.cpu().numpy().astype(bool), want)
    assert 0.45 < want.mean() < 0.6


@pytest.fixture(scope="module")
def s4():
    return datagen.star4_c(1.0)


@pytest.fixture(scope="module")
def s4_oracle(s4):
    return oracle.star_par(s4, threads=host_threads())


@pytest.mark.parametrize("kw", [{}, {"strategy": "light"}, {"strategy": "fixed", "delta1": 200, "delta2": 10}])
def test_star4_4x500k(jp, s4, s4_oracle, checks_mode, kw):
    h = jp.default_handle(0)
    cols, st = h.star([(dev(a), dev(b)) for a, b in s4], **kw)
    assert st["n_out"] == cols[0].numel() == s4_oracle.shape[0]
    for i in range(4):
        np.testing.assert_array_equal(cols[i].cpu().numpy(), s4_oracle[:, i])
    assert st["J_L"] + st["J_H"] == st["J"] == oracle_star_join_size(s4)


def oracle_star_join_size(rels):
    """sum over y of the product of the k degrees, over distinct edges."""
    degs = []
    for a, b in rels:
        e = np.unique((a.astype(np.int64) << 32) | (b.astype(np.int64) & 0xffffffff))
        degs.append(np.bincount((e & 0xffffffff).astype(np.int64), minlength=1 << 20))
    n = min(d.size for d in degs)
    return int(np.prod(np.stack([d[:n] for d in degs]).astype(np.float64), axis=0).sum())
