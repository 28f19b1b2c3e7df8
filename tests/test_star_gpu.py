"""Star query Q*_3 parity: the HIP path through the C ABI against the CPU
oracle (bit-exact sorted tuples) and the numpy restatement of the Section 3.2
partition (J, light / heavy witness counts)."""
import itertools

import numpy as np
import pytest

import datagen
import oracle
from oracle import reference as ref
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


def run(jp, rels, **kw):
    cols, st = jp.default_handle(0).star([(dev(a), dev(b)) for a, b in rels], **kw)
    return np.stack([c.cpu().numpy() for c in cols], 1) if cols[0].numel() else np.zeros((0, len(rels)), np.int32), st


def check(jp, rels, **kw):
    exp = oracle.star(rels)
    got, st = run(jp, rels, **kw)
    assert got.shape == exp.shape, (got.shape, exp.shape, kw)
    np.testing.assert_array_equal(got, exp)
    return st


def example_rels():
    rows = load_golden("two_path_example.txt")
    R = [(int(r[1]), int(r[2])) for r in rows if r[0] == "R"]
    S = [(int(r[1]), int(r[2])) for r in rows if r[0] == "S"]
    rows = load_golden("star_example.txt")
    T = [(int(r[1]), int(r[2])) for r in rows if r[0] == "T"]
    rel = lambda E: (np.array([e[0] for e in E]), np.array([e[1] for e in E]))
    return [rel(R), rel(S), rel(T)]


def test_worked_example_star(jp):
    rels = example_rels()
    for d1, d2 in itertools.product([1, 2, 3, None], [1, 2, 3, None]):
        st = check(jp, rels, delta1=d1, delta2=d2, strategy="fixed")
        assert st["n_out"] == 80
        if d1 is not None and d2 is not None:
            r = ref.star_stats(rels, d1, d2)
            assert (st["J"], st["J_L"], st["J_H"]) == (r["J"], r["J_L"], r["J_H"]), (d1, d2)


@pytest.mark.parametrize("seed", range(8))
def test_random_small_star(jp, seed):
    rng = np.random.default_rng(seed)
    signed = seed % 2 == 1
    rels = [datagen.random_small(int(rng.integers(1, 300)), 30, 12, seed * 7 + i, dup=True, signed=signed)
            for i in range(3)]
    if signed:  # share y ids so the signed case still joins
        for i in (1, 2):
            rels[i] = (rels[i][0], rels[0][1][rng.integers(0, rels[0][1].size, rels[i][1].size)])
    for d1, d2 in [(1, 1), (2, 3), (4, 1), (None, None)]:
        st = check(jp, rels, delta1=d1, delta2=d2, strategy="fixed")
        if d1 is not None and seed < 4:
            r = ref.star_stats(rels, d1, d2)
            assert (st["J"], st["J_L"], st["J_H"]) == (r["J"], r["J_L"], r["J_H"])


def test_star_k2_is_two_path(jp):
    (rx, ry), (sz, sy) = datagen.twopath_c2(0.001)
    got, st = run(jp, [(rx, ry), (sz, sy)])
    ex, ez = oracle.two_path(rx, ry, sz, sy)
    np.testing.assert_array_equal(got[:, 0], ex)
    np.testing.assert_array_equal(got[:, 1], ez)


def test_star_degenerate(jp):
    e = np.zeros(0, np.int32)
    got, st = run(jp, [(e, e), ([1], [2]), ([3], [2])])
    assert got.shape[0] == 0
    got, st = run(jp, [([1], [1]), ([1], [2]), ([3], [2])])  # no common y
    assert got.shape[0] == 0
    check(jp, [([5], [9]), ([-7], [9]), ([2**31 - 1], [9])])


@pytest.mark.parametrize("scale", [0.005, 0.02])
def test_star_zipf_scaled(jp, scale):
    """The star workload's shape (Zipf(1.3) y, uniform x) at reduced scale,
    with light-only, theory and forced thresholds that create a heavy part."""
    rels = datagen.star_c3(scale)
    exp = oracle.star(rels)
    for kw in (dict(strategy="light"), dict(strategy="auto"), dict(delta1=8, delta2=3),
               dict(delta1=3, delta2=2)):
        got, st = run(jp, rels, **kw)
        np.testing.assert_array_equal(got, exp, err_msg=str(kw))


def test_star_communities_heavy(jp):
    """Dense communities: every in-community triple is an output; with low
    thresholds the heavy product carries them."""
    x, y = datagen.communities(3, 20, 12, 1.0, seed=2)
    st = check(jp, [(x, y)] * 3, delta1=3, delta2=3)
    assert st["nnz_heavy"] > 0 and st["n_out"] == 3 * 20 ** 3


def test_star_wide_keys(jp):
    """Rank widths summing to more than 64 bits use 128-bit sort keys."""
    n = 2_200_000
    rng = np.random.default_rng(3)
    rels = []
    for i in range(3):
        x = rng.permutation(n).astype(np.int32)
        y = (np.arange(n) // 2).astype(np.int32)
        rels.append((x, y))
    check(jp, rels, strategy="light")


# ---------------------------------------------------------------------------
# k > 3: V over the first ceil(k/2) relations, W over the rest (Section 3.2)
# ---------------------------------------------------------------------------

def example_rels4():
    rows = load_golden("star_example.txt")
    U = [(int(r[1]), int(r[2])) for r in rows if r[0] == "U"]
    return example_rels() + [(np.array([e[0] for e in U]), np.array([e[1] for e in U]))]


def test_worked_example_star4(jp):
    """Q*_4 over R, S, T, U: 237 output tuples and 286 witnesses at every
    threshold pair; the light / heavy split matches the restatement."""
    rels = example_rels4()
    for d1, d2 in itertools.product([1, 2, 3, None], [1, 2, 3, None]):
        st = check(jp, rels, delta1=d1, delta2=d2, strategy="fixed")
        assert st["n_out"] == 237 and st["J"] == 286
        if d1 is not None and d2 is not None:
            r = ref.star_stats(rels, d1, d2)
            assert (st["J_L"], st["J_H"]) == (r["J_L"], r["J_H"]), (d1, d2)
    st = check(jp, rels, delta1=2, delta2=2)
    assert st["J_H"] > 0 and st["nnz_heavy"] > 0


@pytest.mark.parametrize("k", [4, 5, 6])
@pytest.mark.parametrize("seed", range(4))
def test_random_small_star_k(jp, k, seed):
    rng = np.random.default_rng(100 * k + seed)
    signed = seed % 2 == 1
    rels = [datagen.random_small(int(rng.integers(1, 60)), 20, 8, 1000 * k + seed * 11 + i, dup=True, signed=signed)
            for i in range(k)]
    if signed:  # share y ids so the signed case still joins
        for i in range(1, k):
            rels[i] = (rels[i][0], rels[0][1][rng.integers(0, rels[0][1].size, rels[i][1].size)])
    for d1, d2 in [(1, 1), (2, 2), (3, 1), (None, None)]:
        st = check(jp, rels, delta1=d1, delta2=d2, strategy="fixed")
        if d1 is not None and seed < 2:
            r = ref.star_stats(rels, d1, d2)
            assert (st["J"], st["J_L"], st["J_H"]) == (r["J"], r["J_L"], r["J_H"])


@pytest.mark.parametrize("kw", [dict(strategy="light"), dict(strategy="auto"), dict(delta1=50, delta2=6),
                                dict(delta1=10, delta2=4), dict(delta1=10, delta2=4, bmm="f16")])
def test_star4_zipf(jp, kw):
    """Four 20K-edge Zipf(1.2) relations with independent y orders (J = 4.6M)."""
    rels = [datagen.zipf_edges(20_000, 5_000, 2_000, 1.2, 50 + i) for i in range(4)]
    check(jp, rels, **kw)


@pytest.mark.parametrize("k", [4, 5])
def test_star_k_communities_closed_form(jp, k):
    """Dense communities: every in-community k-tuple is an output (c m^k);
    with low thresholds the product of generated V and W rows carries them."""
    x, y = datagen.communities(3, 8, 6, 1.0, seed=4)
    st = check(jp, [(x, y)] * k, delta1=2, delta2=2)
    assert st["n_out"] == 3 * 8 ** k and st["nnz_heavy"] > 0
    st = check(jp, [(x, y)] * k, strategy="light")
    assert st["n_out"] == 3 * 8 ** k


def test_star4_wide_keys(jp):
    """Four rank widths of 18 bits (72 > 64) use 128-bit keys, light and heavy."""
    n = 140_000
    rng = np.random.default_rng(8)
    rels = [(rng.permutation(n).astype(np.int32), (np.arange(n) // 2).astype(np.int32)) for _ in range(4)]
    check(jp, rels, strategy="light")
    check(jp, rels, delta1=1, delta2=1)


def test_star4_dense_core_product(jp):
    """k = 4 over dense communities (2 of 32 x ids by 128 y ids, p = 0.5):
    J / |OUT| = 8, every witness heavy at Delta1 = Delta2 = 1, so the whole
    output comes from the product of generated 4,096-row V and W (24 of the
    2 * 32^4 in-community tuples share no y at this seed)."""
    x, y = datagen.communities(2, 32, 128, 0.5, seed=11)
    st = check(jp, [(x, y)] * 4, delta1=1, delta2=1)
    assert st["J_L"] == 0 and st["nnz_heavy"] == st["n_out"] == 2 * 32 ** 4 - 24
