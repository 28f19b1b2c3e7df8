"""Pins for the CPU oracle (no GPU).

The oracle (plain C, full join then sort-distinct) is checked against things
other than itself: brute force over all candidate pairs by set intersection,
the paper's worked examples, closed forms, and invariants the paper states.
"""
import itertools

import numpy as np
import pytest

import datagen
import oracle
from oracle import reference as ref
from tests.conftest import load_golden


# ---------------------------------------------------------------------------
# Brute force: for every candidate pair, test whether the neighbour sets meet.
# This is a different algorithm from the oracle's full join + sort.
# ---------------------------------------------------------------------------

def brute_two_path(rx, ry, sz, sy):
    nx, nz = {}, {}
    for a, b in zip(np.asarray(rx).tolist(), np.asarray(ry).tolist()):
        nx.setdefault(a, set()).add(b)
    for c, b in zip(np.asarray(sz).tolist(), np.asarray(sy).tolist()):
        nz.setdefault(c, set()).add(b)
    out = sorted((a, c) for a in nx for c in nz if nx[a] & nz[c])
    return out


def brute_star(rels):
    nbr = []
    for a, b in rels:
        m = {}
        for p, q in zip(np.asarray(a).tolist(), np.asarray(b).tolist()):
            m.setdefault(p, set()).add(q)
        nbr.append(m)
    out = []
    for t in itertools.product(*[sorted(m) for m in nbr]):
        common = set.intersection(*[nbr[i][t[i]] for i in range(len(t))])
        if common:
            out.append(t)
    return sorted(out)


def as_pairs(x, z):
    return list(zip(x.tolist(), z.tolist()))


@pytest.mark.parametrize("seed", range(12))
def test_two_path_matches_brute_force(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(0, 60))
    nx, ny = int(rng.integers(1, 12)), int(rng.integers(1, 12))
    rx, ry = datagen.random_small(n, nx, ny, seed, dup=bool(seed % 2), signed=bool(seed % 3 == 0))
    sz, sy = datagen.random_small(int(rng.integers(0, 60)), nx, ny, seed + 1000,
                                  dup=bool(seed % 2), signed=bool(seed % 3 == 0))
    if seed % 3 == 0:
        # share the y ids with R so the signed case still joins
        sy = ry[rng.integers(0, max(ry.size, 1), sy.size)] if ry.size else sy
    x, z = oracle.two_path(rx, ry, sz, sy)
    assert as_pairs(x, z) == brute_two_path(rx, ry, sz, sy)
    # sorted, distinct
    key = x.astype(np.int64) * (2**32) + z.astype(np.int64)
    assert np.all(np.diff(key) > 0)


@pytest.mark.parametrize("seed", range(6))
def test_star_matches_brute_force(seed):
    rng = np.random.default_rng(200 + seed)
    k = 2 + seed % 3
    rels = [datagen.random_small(int(rng.integers(0, 25)), 6, 5, seed * 10 + i, dup=True) for i in range(k)]
    t = oracle.star(rels)
    assert [tuple(r) for r in t.tolist()] == brute_star(rels)


def test_two_path_empty_and_disjoint():
    e = np.zeros(0, np.int32)
    x, z = oracle.two_path(e, e, e, e)
    assert x.size == 0 and z.size == 0
    x, z = oracle.two_path([1, 2], [5, 6], [3], [7])  # no common y
    assert x.size == 0
    assert oracle.join_size([1, 2], [5, 6], [3], [7]) == 0


def test_extreme_ids():
    lo, hi = -(2**31), 2**31 - 1
    rx = np.array([lo, hi, 0, lo], np.int32)
    ry = np.array([hi, lo, hi, lo], np.int32)
    x, z = oracle.two_path(rx, ry, rx, ry)
    assert as_pairs(x, z) == brute_two_path(rx, ry, rx, ry)
    assert x[0] == lo  # signed order


# ---------------------------------------------------------------------------
# The worked examples (Section 3.1 and 3.2)
# ---------------------------------------------------------------------------

def _example_two_path():
    rows = load_golden("two_path_example.txt")
    R = [(int(a), int(b), int(c)) for t, a, b, c in (r for r in rows if r[0] == "R")]
    S = [(int(a), int(b), int(c)) for t, a, b, c in (r for r in rows if r[0] == "S")]
    mats = {r[0]: np.array(list(map(int, r[1:]))).reshape(3, 3) for r in rows if r[0] in ("M1", "M2", "M")}
    return R, S, mats


def test_worked_example_two_path_output():
    R, S, _ = _example_two_path()
    rx, ry = np.array([r[0] for r in R]), np.array([r[1] for r in R])
    sz, sy = np.array([s[0] for s in S]), np.array([s[1] for s in S])
    x, z = oracle.two_path(rx, ry, sz, sy)
    assert as_pairs(x, z) == brute_two_path(rx, ry, sz, sy)
    # derived from the figure by brute force: 26 distinct pairs, J = 35
    assert len(x) == 26
    assert oracle.join_size(rx, ry, sz, sy) == 35


def test_worked_example_partition_and_matrices():
    """At Delta1 = Delta2 = 2 the figure's coloured edges are R^- and S^-,
    and the heavy matrices are the printed M1 and M2."""
    R, S, mats = _example_two_path()
    rx, ry = np.array([r[0] for r in R]), np.array([r[1] for r in R])
    sz, sy = np.array([s[0] for s in S]), np.array([s[1] for s in S])
    st = ref.two_path_stats(rx, ry, sz, sy, 2, 2)
    assert st["X"] == [4, 5, 6] and st["Y"] == [4, 5, 6] and st["Z"] == [4, 5, 6]
    xh, yh, zh = set(st["X"]), set(st["Y"]), set(st["Z"])
    for a, b, light in R:
        assert (not (a in xh and b in yh)) == bool(light), (a, b)
    for c, b, light in S:
        assert (not (c in zh and b in yh)) == bool(light), (c, b)
    np.testing.assert_array_equal(st["M1"], mats["M1"])
    np.testing.assert_array_equal(st["M2"], mats["M2"])
    # The product of the printed matrices: every entry but [6][6] as printed.
    M = st["M"]
    P = mats["M"]
    mask = np.ones((3, 3), bool)
    mask[2, 2] = False
    np.testing.assert_array_equal(M[mask], P[mask])
    assert M[2, 2] == 1 and P[2, 2] == 3  # misprint; both nonzero
    assert (M > 0).all() and (P > 0).all()  # the Boolean support agrees
    # light witnesses: 19 distinct pairs; union with the 9 heavy pairs is 26
    assert st["J_L"] == 19 and len(st["light_pairs"]) == 19
    assert st["nnz_heavy"] == 9
    assert len(st["light_pairs"] | st["heavy_pairs"]) == 26
    assert st["light_pairs"] & st["heavy_pairs"] == {(4, 4), (6, 6)}


def test_worked_example_star():
    R, S, _ = _example_two_path()
    rows = load_golden("star_example.txt")
    T = [(int(r[1]), int(r[2])) for r in rows if r[0] == "T"]
    U = [(int(r[1]), int(r[2])) for r in rows if r[0] == "U"]
    rel = lambda E: (np.array([e[0] for e in E]), np.array([e[1] for e in E]))
    Rr, Sr, Tr, Ur = rel([r[:2] for r in R]), rel([s[:2] for s in S]), rel(T), rel(U)
    t3 = oracle.star([Rr, Sr, Tr])
    assert [tuple(r) for r in t3.tolist()] == brute_star([Rr, Sr, Tr])
    assert len(t3) == 80
    t4 = oracle.star([Rr, Sr, Tr, Ur])
    assert [tuple(r) for r in t4.tolist()] == brute_star([Rr, Sr, Tr, Ur])
    assert len(t4) == 237
    # The printed V rows (4,5), (6,6) and W columns follow the V/W definition
    # (membership of every (a_i, y) in R_i); the printed V row (4,4) does not.
    def adj(rr):
        m = {}
        for a, b in zip(*rr):
            m.setdefault(int(a), set()).add(int(b))
        return m
    aR, aS, aT, aU = adj(Rr), adj(Sr), adj(Tr), adj(Ur)
    for r in rows:
        if r[0] in ("V", "W"):
            a, c = int(r[1]), int(r[2])
            bits = [int(v) for v in r[3:]]
            first, second = (aR, aS) if r[0] == "V" else (aT, aU)
            expect = [int(b in first[a] and b in second[c]) for b in (4, 5, 6)]
            if r[0] == "V" and (a, c) == (4, 4):
                assert expect == [1, 0, 0] and bits == [1, 1, 1]
            else:
                assert expect == bits, r


# ---------------------------------------------------------------------------
# Closed forms
# ---------------------------------------------------------------------------

def test_communities_closed_form():
    """Example 1: c disjoint communities of m x values fully connected through
    their community's y values give c*m^2 self-join pairs."""
    c, m = 5, 7
    x, y = datagen.communities(c, m, 4, 1.0, seed=3)
    ox, oz = oracle.two_path(x, y, x, y)
    assert len(ox) == c * m * m
    # sparse communities: pairs never cross communities, so at most c*m^2
    xs, ys = datagen.communities(c, m, 4, 0.3, seed=3)
    sx, sz = oracle.two_path(xs, ys, xs, ys)
    assert len(sx) <= c * m * m and np.all(sx // m == sz // m)
    # star over full communities: every in-community triple, c*m^3
    xf, yf = datagen.communities(3, 4, 3, 1.0, seed=1)
    assert len(oracle.star([(xf, yf)] * 3)) == 3 * 4 ** 3


def test_complete_bipartite_and_single_y():
    X = np.arange(7)
    Z = np.arange(100, 105)
    Y = np.arange(3)
    rx, ry = np.repeat(X, Y.size), np.tile(Y, X.size)
    sz, sy = np.repeat(Z, Y.size), np.tile(Y, Z.size)
    x, z = oracle.two_path(rx, ry, sz, sy)
    assert len(x) == X.size * Z.size
    # single shared y: |X| * |Z|
    x, z = oracle.two_path(X, np.zeros(7), Z, np.zeros(5))
    assert len(x) == 35


def test_perfect_matching_is_diagonal():
    n = 50
    rng = np.random.default_rng(5)
    x = rng.permutation(n)
    y = rng.permutation(n)
    ox, oz = oracle.two_path(x, y, x, y)
    assert np.array_equal(ox, np.arange(n)) and np.array_equal(oz, np.arange(n))


# ---------------------------------------------------------------------------
# Invariants stated in the paper
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(4))
def test_selfjoin_symmetry_bounds_and_duplicates(seed):
    x, y = datagen.uniform_edges(300, 60, 40, seed)
    ox, oz = oracle.two_path(x, y, x, y)
    pairs = set(as_pairs(ox, oz))
    assert all((c, a) in pairs for a, c in pairs)  # symmetric
    dom = np.unique(x)
    assert all((a, a) in pairs for a in dom.tolist())  # full diagonal
    J = oracle.join_size(x, y, x, y)
    n = len(x)
    # Section 5: |dom x| <= |OUT| <= min(|dom x|^2, J) and J <= N sqrt(|OUT|)
    assert dom.size <= len(pairs) <= min(dom.size ** 2, J)
    assert J <= n * np.sqrt(len(pairs)) + 1e-9
    # idempotent under repeated rows
    x2 = np.concatenate([x, x[: 50]])
    y2 = np.concatenate([y, y[: 50]])
    dx, dz = oracle.two_path(x2, y2, x2, y2)
    assert np.array_equal(dx, ox) and np.array_equal(dz, oz)
    assert oracle.join_size(x2, y2, x2, y2) == J


def test_monotone_under_insertion():
    x, y = datagen.uniform_edges(200, 40, 30, 9)
    a, b = oracle.two_path(x[:150], y[:150], x[:150], y[:150])
    c, d = oracle.two_path(x, y, x, y)
    assert set(as_pairs(a, b)) <= set(as_pairs(c, d))


def test_join_size_matches_enumeration():
    for seed in range(5):
        rx, ry = datagen.random_small(80, 15, 10, seed, dup=True)
        sz, sy = datagen.random_small(70, 15, 10, seed + 50, dup=True)
        er = set(zip(rx.tolist(), ry.tolist()))
        es = set(zip(sz.tolist(), sy.tolist()))
        J = sum(1 for a, b in er for c, d in es if b == d)
        assert oracle.join_size(rx, ry, sz, sy) == J


@pytest.mark.parametrize("d1,d2", [(1, 1), (1, 3), (2, 2), (3, 1), (5, 5), (1000, 1000)])
def test_partition_is_exact_at_any_threshold(d1, d2):
    """Correctness argument of Section 3.1: the light output unioned with the
    heavy product's support is the query result whatever the thresholds, and
    light plus heavy witnesses partition the full join."""
    rx, ry = datagen.random_small(120, 25, 12, 31)
    sz, sy = datagen.random_small(110, 25, 12, 32)
    st = ref.two_path_stats(rx, ry, sz, sy, d1, d2)
    x, z = oracle.two_path(rx, ry, sz, sy)
    assert sorted(st["light_pairs"] | st["heavy_pairs"]) == as_pairs(x, z)
    assert st["J_L"] + st["J_H"] == st["J"] == oracle.join_size(rx, ry, sz, sy)
    for rule in (ref.Y_RULE_MAX, ref.Y_RULE_R_ONLY):
        s2 = ref.two_path_stats(rx, ry, sz, sy, d1, d2, y_rule=rule)
        assert sorted(s2["light_pairs"] | s2["heavy_pairs"]) == as_pairs(x, z)


@pytest.mark.parametrize("d1,d2", [(1, 1), (2, 1), (2, 3), (100, 100)])
def test_star_partition_is_exact(d1, d2):
    rels = [datagen.random_small(40, 8, 6, 70 + i) for i in range(3)]
    st = ref.star_stats(rels, d1, d2)
    t = oracle.star(rels)
    assert sorted(st["light"] | st["heavy"]) == [tuple(r) for r in t.tolist()]
    assert st["J_L"] + st["J_H"] == st["J"]


# ---------------------------------------------------------------------------
# Lemma 3 closed forms against a direct minimisation of the idealised cost
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,out", [(1e6, 1e3), (1e6, 1e5), (1e6, 1e6), (1e6, 3e7), (1e5, 1e9)])
def test_lemma3_minimiser(n, out):
    d1, d2 = ref.theory_thresholds(n, out)
    f0 = ref.idealized_cost(n, out, d1, d2)
    grid = np.exp(np.linspace(0, np.log(n), 400))
    best = min(ref.idealized_cost(n, out, a, b) for a in grid for b in grid)
    assert f0 <= best * (1 + 1e-3)


def test_k3_example_exponents():
    """Section 3.2 example (k=3, OUT = N^(3/2)): D2 = N^(6/16), D1 = N^(7/16)
    balance N D1^2 = OUT D2 = (N/D2)^3 (the omega = 2 product cost with
    beta = N/D1), giving N^(15/8)."""
    N = 1e8
    out = N ** 1.5
    d2 = N ** (6 / 16)
    d1 = N ** (7 / 16)
    a = N * d1 ** 2
    b = out * d2
    c = (N / d2) ** 2 * (N / d1) * (N / d2) / (N / d1)  # M(U,V,W) = UVW/beta
    assert np.isclose(np.log(a), np.log(b)) and np.isclose(np.log(b), np.log(c))
    assert np.isclose(np.log(a) / np.log(N), 15 / 8)


def test_out_estimate_within_bounds():
    for seed in range(3):
        x, y = datagen.uniform_edges(400, 80, 50, seed)
        ox, _ = oracle.two_path(x, y, x, y)
        J = oracle.join_size(x, y, x, y)
        dom = np.unique(x).size
        est = ref.out_estimate(dom, dom, J, len(x))
        assert dom <= est <= min(dom * dom, J)


# ---------------------------------------------------------------------------
# Star partition (Section 3.2) pinned to hand-worked cases
# ---------------------------------------------------------------------------

def _example_star_rels():
    R, S, _ = _example_two_path()
    rows = load_golden("star_example.txt")
    T = [(int(r[1]), int(r[2])) for r in rows if r[0] == "T"]
    U = [(int(r[1]), int(r[2])) for r in rows if r[0] == "U"]
    rel = lambda E: (np.array([e[0] for e in E]), np.array([e[1] for e in E]))
    return rel([r[:2] for r in R]), rel([s[:2] for s in S]), rel(T), rel(U)


def test_star_example_partition_by_hand():
    """The star example at Delta1 = Delta2 = 2, worked by hand from the
    Section 3.2 definitions.

    x-degrees in R: x1 1, x2 2, x3 2, x4 3, x5 3, x6 3, so R^- holds the
    tuples of x1, x2, x3.  y-degrees (R, S, T, U): y1 (2,1,2,1), y2 (2,2,2,1),
    y3 (1,2,2,1), y4 (3,2,3,3), y5 (3,3,3,4), y6 (3,4,3,3).  The y light in
    every other relation (S, T for Q*_3; S, T, U for Q*_4) are y1, y2, y3, so
    R^diamond holds the R tuples at those y.  The example's remark that R^-
    equals R^diamond does not hold under the definitions.
    J = sum over y of the degree products: Q*_3 4+8+4+18+27+36 = 97,
    Q*_4 4+8+4+54+108+108 = 286.
    """
    Rr, Sr, Tr, Ur = _example_star_rels()
    minus = {(1, 6), (2, 1), (2, 2), (3, 5), (3, 3)}
    diamond = {(2, 1), (2, 2), (3, 3), (4, 1), (6, 2)}
    for rels, J in (([Rr, Sr, Tr], 97), ([Rr, Sr, Tr, Ur], 286)):
        _, parts, _, _ = ref.star_parts(rels, 2, 2)
        assert parts[0]["minus"] == minus
        assert parts[0]["diamond"] == diamond
        assert parts[0]["plus"] == {(4, 4), (4, 6), (5, 4), (5, 5), (5, 6), (6, 4), (6, 5)}
        st = ref.star_stats(rels, 2, 2)
        assert st["J"] == J and st["J_L"] + st["J_H"] == J


def test_star_plus_needs_y_heavy_in_some_other_relation():
    """R_i^+ = R_i minus R_i^- minus R_i^diamond: heavy x and y heavy in at
    least one OTHER relation.  Delta1 = Delta2 = 1.

    Case A: y0 and y1 each have degree 2 in R1 and R2 and 1 in R3; x0, x1
    have degree 2 in R1 and R2, x0 degree 2 in R3.  Every tuple sees its y
    heavy in another relation (R3's tuples see R1 and R2), so all
    2*2*1 witnesses per y are heavy: J = J_H = 8.  (Requiring y heavy in
    every other relation would make J_H = 0.)
    Case B: R2 = R3 = {(0,0), (0,1)}: y light in R2 and R3, so R1's tuples are
    in R1^diamond and no witness is heavy: J = 4, J_H = 0.  (Counting R1's own
    y-degree would make J_H = 4.)
    """
    full = (np.array([0, 1, 0, 1]), np.array([0, 0, 1, 1]))
    one = (np.array([0, 0]), np.array([0, 1]))
    st = ref.star_stats([full, full, one], 1, 1)
    assert (st["J"], st["J_L"], st["J_H"]) == (8, 0, 8)
    assert st["u"] == [2, 2, 1] and st["v"] == 2
    assert st["heavy"] == {(0, 0, 0), (0, 1, 0), (1, 0, 0), (1, 1, 0)}
    st = ref.star_stats([full, one, one], 1, 1)
    assert (st["J"], st["J_L"], st["J_H"]) == (4, 4, 0)
    assert st["heavy"] == set()
    _, parts, _, _ = ref.star_parts([full, one, one], 1, 1)
    assert parts[0]["diamond"] == {(0, 0), (1, 0), (0, 1), (1, 1)}
    assert parts[1]["plus"] == {(0, 0), (0, 1)}


# ---------------------------------------------------------------------------
# Section 5 indexes and the output estimate, pinned to a hand-made instance
# ---------------------------------------------------------------------------

HAND_R = ([1, 1, 2, 3, 3, 4], [10, 11, 10, 11, 12, 13])
HAND_S = ([7, 8, 7, 9, 7, 8, 9, 8], [10, 10, 11, 12, 12, 12, 13, 14])


def test_degree_summary_by_hand():
    """Worked by hand.  S's (8, 14) is dangling (no y 14 in R) and dropped.
    deg_R(y): 10:2 11:2 12:1 13:1; deg_S(y): 10:2 11:1 12:3 13:1.
    Key degree (larger of the two): 10:2 11:2 12:3 13:1.
      y index: degree 1 -> {13}, sum 1*1 = 1; degree 2 -> {10, 11}, sum
               2*2 + 2*1 = 6; degree 3 -> {12}, sum 1*3 = 3.
      x index: deg_R(x) x1:2 x2:1 x3:2 x4:1; witnesses of x (sum of deg_S
               over its y): x1 2+1 = 3, x2 2, x3 1+3 = 4, x4 1; degree 1 ->
               count 2, sum 3; degree 2 -> count 2, sum 7.
      cdfx:    smallest key degree among the y of x: x1 2, x2 2, x3 2, x4 1.
      z index: deg_S(z) z7:3 z8:2 z9:2.
    J = 4 + 2 + 3 + 1 = 10, N = max(6, 7) = 7.
    With deg_R alone as the key: y keys 10:2 11:2 12:1 13:1, y index
    degree 1 -> {12, 13}, sum 3 + 1 = 4; degree 2 -> sum 6; cdfx x3 -> 1.
    """
    d = ref.degree_summary(*HAND_R, *HAND_S)
    assert (d["n_r"], d["n_s"], d["dom_x"], d["dom_y"], d["dom_z"], d["J"]) == (6, 7, 4, 4, 3, 10)

    def same(idx, deg, cnt, sm=None):
        np.testing.assert_array_equal(idx[0], deg)
        np.testing.assert_array_equal(idx[1], cnt)
        if sm is None:
            assert idx[2] is None
        else:
            np.testing.assert_array_equal(idx[2], sm)

    same(d["y"], [1, 2, 3], [1, 2, 1], [1.0, 6.0, 3.0])
    same(d["x"], [1, 2], [2, 2], [3.0, 7.0])
    same(d["xcdf"], [1, 2], [1, 3])
    same(d["z"], [2, 3], [2, 1])
    r = ref.degree_summary(*HAND_R, *HAND_S, y_rule=ref.Y_RULE_R_ONLY)
    same(r["y"], [1, 2], [2, 2], [4.0, 6.0])
    same(r["xcdf"], [1, 2], [2, 2])
    same(r["x"], [1, 2], [2, 2], [3.0, 7.0])


def test_out_estimate_by_hand():
    """Section 5 estimate on the hand-made instance: lower bound
    max(|dom x|, (J/N)^2) = max(4, (10/7)^2) = 4, upper bound
    min(|dom x| |dom z|, J) = min(12, 10) = 10, geometric mean sqrt(40).
    (The arithmetic mean would be 7.)  The true |OUT| is 8: x1 {7,8},
    x2 {7,8}, x3 {7,8,9}, x4 {9}."""
    d = ref.degree_summary(*HAND_R, *HAND_S)
    assert d["out_est"] == pytest.approx(np.sqrt(40.0), rel=1e-12)
    assert ref.out_estimate(4, 3, 10, 7) == pytest.approx(6.324555320336759, rel=1e-12)
    ox, oz = oracle.two_path(*HAND_R, *HAND_S)
    assert as_pairs(ox, oz) == [(1, 7), (1, 8), (2, 7), (2, 8), (3, 7), (3, 8), (3, 9), (4, 9)]
    # (J/N)^2 as the lower bound: |dom x| = 5, |dom z| = 1000, J = 2000,
    # N = 100: lo = max(5, 400) = 400, hi = min(5000, 2000) = 2000
    assert ref.out_estimate(5, 1000, 2000, 100) == pytest.approx(np.sqrt(400.0 * 2000.0), rel=1e-12)
    # bounds that cross (lo > hi) collapse to the upper bound
    assert ref.out_estimate(5, 1000, 1000, 10) == pytest.approx(1000.0, rel=1e-12)


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_parallel_oracle_matches_plain(threads):
    """The multi-threaded variants split R (R_1) by first-column ranges; they
    must give exactly the single-thread result, including signed extremes
    and repeated rows."""
    for seed in range(4):
        rx, ry = datagen.random_small(400, 60, 25, seed, dup=True, signed=seed % 2 == 1)
        sz, sy = datagen.random_small(380, 60, 25, seed + 9, dup=True, signed=seed % 2 == 1)
        if seed % 2:
            sy = ry[np.random.default_rng(seed).integers(0, ry.size, sy.size)]
        a = oracle.two_path(rx, ry, sz, sy)
        b = oracle.two_path(rx, ry, sz, sy, threads=threads)
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_array_equal(a[1], b[1])
        rels = [datagen.random_small(150, 20, 8, seed * 3 + i, dup=True) for i in range(3)]
        np.testing.assert_array_equal(oracle.star(rels), oracle.star(rels, threads=threads))
    e = np.zeros(0, np.int32)
    assert oracle.two_path(e, e, [1], [2], threads=threads)[0].size == 0
    x, y = datagen.selfjoin_c1()
    a = oracle.two_path(x, y, x, y)
    b = oracle.two_path(x, y, x, y, threads=threads)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


# ---------------------------------------------------------------------------
# Set similarity join and Boolean set intersection (Section 2.1): pinned by
# brute force over all set pairs (Python sets), the worked example's overlaps
# worked out by hand, and closed forms.
# ---------------------------------------------------------------------------

def brute_overlaps(rx, ry, sz, sy):
    nx, nz = {}, {}
    for a, b in zip(np.asarray(rx).tolist(), np.asarray(ry).tolist()):
        nx.setdefault(a, set()).add(b)
    for c, b in zip(np.asarray(sz).tolist(), np.asarray(sy).tolist()):
        nz.setdefault(c, set()).add(b)
    return {(a, c): len(nx[a] & nz[c]) for a in nx for c in nz if nx[a] & nz[c]}


def example_relations():
    rows = load_golden("two_path_example.txt")
    R = np.array([(int(r[1]), int(r[2])) for r in rows if r[0] == "R"])
    S = np.array([(int(r[1]), int(r[2])) for r in rows if r[0] == "S"])
    return R[:, 0], R[:, 1], S[:, 0], S[:, 1]


def test_ssj_worked_example_by_hand():
    rx, ry, sz, sy = example_relations()
    hand = {(int(a), int(b)): int(c) for a, b, c in load_golden("ssj_example.txt")}
    assert len(hand) == 26 and sum(hand.values()) == 35
    for c in (1, 2, 3, 4):
        x, z, n = oracle.ssj(rx, ry, sz, sy, c=c)
        want = sorted((k, v) for k, v in hand.items() if v >= c)
        assert list(zip(zip(x.tolist(), z.tolist()), n.tolist())) == want
    x, z, n = oracle.ssj(rx, ry, sz, sy, c=2, order=1)
    assert list(zip(x.tolist(), z.tolist(), n.tolist()))[:2] == [(5, 5, 3), (4, 4, 2)]
    assert len(x) == 8


def two_relations(n, n_x, n_y, seed, signed):
    """R and S drawn as one relation split by row parity, so that with signed
    ids both use the same element ids."""
    x, y = datagen.random_small(2 * n, n_x, n_y, seed=seed, dup=True, signed=signed)
    return x[0::2], y[0::2], x[1::2], y[1::2]


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("c", [1, 2, 3])
def test_ssj_matches_brute_force(seed, c):
    rx, ry, sz, sy = two_relations(60 + 7 * seed, 15, 12, 500 + seed, seed % 2 == 1)
    ov = brute_overlaps(rx, ry, sz, sy)
    x, z, n = oracle.ssj(rx, ry, sz, sy, c=c)
    assert list(zip(zip(x.tolist(), z.tolist()), n.tolist())) == sorted((k, v) for k, v in ov.items() if v >= c)
    # ordered: overlap descending, ties by (x, z)
    x, z, n = oracle.ssj(rx, ry, sz, sy, c=c, order=1)
    want = sorted(((k, v) for k, v in ov.items() if v >= c), key=lambda kv: (-kv[1], kv[0]))
    assert list(zip(zip(x.tolist(), z.tolist()), n.tolist())) == want


def test_ssj_overlap_one_is_the_two_path_and_counts_sum_to_j():
    rx, ry = datagen.zipf_edges(3000, 300, 80, 1.2, 71)
    sz, sy = datagen.zipf_edges(2500, 250, 80, 1.2, 72)
    x, z, n = oracle.ssj(rx, ry, sz, sy, c=1)
    ex, ez = oracle.two_path(rx, ry, sz, sy)
    np.testing.assert_array_equal(x, ex)
    np.testing.assert_array_equal(z, ez)
    assert int(n.sum()) == oracle.join_size(rx, ry, sz, sy)
    assert (n >= 1).all()


def test_ssj_communities_closed_form():
    # c communities of m sets over g elements each, every set holds all g
    # elements of its community: every in-community pair overlaps in g.
    c_, m, g = 5, 7, 4
    xs = np.repeat(np.arange(c_ * m), g)
    ys = (np.arange(c_ * m)[:, None] // m * g + np.arange(g)[None, :]).ravel()
    for c in (1, g, g + 1):
        x, z, n = oracle.ssj(xs, ys, xs, ys, c=c)
        assert x.size == (c_ * m * m if c <= g else 0)
        assert (n == g).all()


def test_bsi_matches_brute_force_and_the_example():
    rx, ry, sz, sy = example_relations()
    q = [(4, 3, 0), (4, 4, 1), (1, 3, 0), (2, 2, 0), (3, 6, 1), (6, 2, 0), (7, 1, 0), (5, 5, 1), (1, 1, 1)]
    got = oracle.bsi(rx, ry, sz, sy, [a for a, _, _ in q], [b for _, b, _ in q])
    assert got.tolist() == [bool(v) for _, _, v in q]
    for seed in range(6):
        rx, ry, sz, sy = two_relations(80, 20, 15, 700 + seed, seed % 2 == 0)
        ov = brute_overlaps(rx, ry, sz, sy)
        rng = np.random.default_rng(seed)
        tx = np.concatenate([rng.choice(rx, 40), rng.integers(-5, 30, 10)]).astype(np.int32)
        tz = np.concatenate([rng.choice(sz, 40), rng.integers(-5, 30, 10)]).astype(np.int32)
        got = oracle.bsi(rx, ry, sz, sy, tx, tz)
        assert got.tolist() == [(a, b) in ov for a, b in zip(tx.tolist(), tz.tolist())]
    assert oracle.bsi(rx, ry, sz, sy, [], []).size == 0


# ---------------------------------------------------------------------------
# Sampled output-size estimate (a selector input): its generator pinned to
# SplitMix64's published first outputs, the estimate to a closed form and to
# the exact |OUT| it approaches over many seeds.
# ---------------------------------------------------------------------------

def test_splitmix64_reference_outputs():
    # SplitMix64 seeded with 0: state advances by 0x9e3779b97f4a7c15 per call
    # (Steele, Lea, Flood; the reference sequence for seed 0)
    outs = [ref.splitmix64(i * 0x9E3779B97F4A7C15 & ref.MASK64) for i in range(3)]
    assert outs == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_sampled_estimate_closed_form_on_communities():
    # c communities of m sets over g elements, each set holding all g: every x
    # reaches exactly m z, so every draw counts m and the estimate is c m^2
    c_, m, g = 6, 9, 4
    xs = np.repeat(np.arange(c_ * m), g)
    ys = (np.arange(c_ * m)[:, None] // m * g + np.arange(g)[None, :]).ravel()
    for seed in (0, 7, 123456789):
        D, k, n, est = ref.sampled_out_estimate(xs, ys, xs, ys, seed)
        assert (k, n) == (c_ * m, c_ * m) and D == k * m and est == c_ * m * m


def test_sampled_estimate_is_unbiased():
    rx, ry = datagen.zipf_edges(1500, 400, 60, 1.1, 91)
    sz, sy = datagen.zipf_edges(1500, 400, 60, 1.1, 92)
    out = oracle.two_path(rx, ry, sz, sy)[0].size
    ests = [ref.sampled_out_estimate(rx, ry, sz, sy, seed, draws=64)[3] for seed in range(300)]
    assert abs(np.mean(ests) / out - 1) < 0.03
