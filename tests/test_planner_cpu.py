"""Algorithm 2 (Section 5) in the library, on the host, against its numpy
restatement under oracle/.  The paper prints no optimizer numbers, so both
are pinned to hand-worked searches on hand-made degree summaries: every cost
term, the step of Delta1, the Delta2 rule with its rounding, the tie rule of
each mode and the plain-join rule, each worked out on paper."""
import numpy as np
import pytest

import datagen
import paper_2002_12459_amd as jp
from oracle import reference as ref


def cals():
    base = jp.default_calibration()
    yield base
    lit = dict(base, literal=1)
    yield lit
    yield dict(base, light_once=0)
    cheap_mm = dict(base, mm_s=[s * 1e-3 for s in base["mm_s"]], t_byte=0.0)
    yield cheap_mm
    dear_mm = dict(base, mm_s=[s * 1e6 for s in base["mm_s"]])
    yield dear_mm
    yield dict(base, t_seq=1e-12, eps=0.2)


def instances():
    yield datagen.communities(6, 40, 30, 0.6, seed=1) * 2
    (rx, ry), (sz, sy) = datagen.twopath_c2(0.002)
    yield rx, ry, sz, sy
    x, y = datagen.zipf_edges(6000, 300, 200, 1.4, seed=9)
    yield x, y, x, y
    x, y = datagen.uniform_edges(3000, 400, 60, 4)
    yield x, y, x, y


@pytest.mark.parametrize("inst", range(4))
def test_library_search_matches_restatement(inst):
    rx, ry, sz, sy = list(instances())[inst]
    s = ref.degree_summary(rx, ry, sz, sy)
    for cal in cals():
        got = jp.plan_summary(s, cal)
        exp = ref.algorithm2(s, cal)
        assert got[0] == exp[0] and got[1] == exp[1], (inst, cal, got, exp)
        assert np.isclose(got[2], exp[2], rtol=1e-9) and np.isclose(got[3], exp[3], rtol=1e-9)


def test_small_join_uses_plain_join():
    """J <= 20 N: Algorithm 2 keeps the worst-case optimal join."""
    x, y = datagen.uniform_edges(2000, 500, 500, 1)
    s = ref.degree_summary(x, y, x, y)
    assert s["J"] <= 20 * 2000
    assert jp.plan_summary(s)[:2] == (None, None)


def test_free_product_drives_delta_down_and_dear_product_keeps_light():
    x, y = datagen.communities(6, 40, 30, 0.6, seed=1)
    s = ref.degree_summary(x, y, x, y)
    base = jp.default_calibration()
    free = dict(base, mm_s=[0.0] * len(base["mm_s"]), t_byte=0.0)
    d1, d2, c, clo = jp.plan_summary(s, free)
    assert d1 is not None and d1 <= 2 and c < clo
    dear = dict(base, mm_s=[1e9] * len(base["mm_s"]))
    d1, d2, c, clo = jp.plan_summary(s, dear)
    # no y is heavy at the chosen Delta1: the plan has no product
    assert d1 is None or d1 >= int(s["y"][0][-1])


def test_summary_validation():
    s = ref.degree_summary(*datagen.communities(2, 5, 4, 1.0, seed=1) * 2)
    bad = dict(s, y=(s["y"][0][::-1].copy(), s["y"][1], s["y"][2]))
    if len(s["y"][0]) > 1:
        with pytest.raises(jp.JoinProjectError):
            jp.plan_summary(bad)


def _hand_summary():
    """A degree summary written by hand (no instance behind it), small enough
    that every cost of the search can be worked out on paper.  N = 100 and an
    output estimate of 1000 give Delta2 = floor(Delta1 / 10), at least 1."""
    i64 = lambda *v: np.array(v, dtype=np.int64)
    f64 = lambda *v: np.array(v, dtype=np.float64)
    return dict(
        n_r=100, n_s=100, dom_x=10, dom_y=5, dom_z=10, J=5000, out_est=1000.0,
        y=(i64(2, 50), i64(3, 2), f64(12.0, 4988.0)),   # key degrees; sums of deg_R * deg_S
        x=(i64(5, 20), i64(6, 4), f64(600.0, 4400.0)),  # deg_R(x); witnesses per degree
        xcdf=(i64(2, 50), i64(7, 3), None),
        z=(i64(5, 20), i64(6, 4), None),
    )


def _hand_cal(literal):
    # light cost = witnesses only; heavy cost = u * v * w (one product entry, p = 1)
    return dict(t_witness=1.0, t_seq=0.0, t_byte=0.0, t_x=0.0, eps=0.5, literal=literal,
                mm_p=[1.0], mm_s=[1.0])


@pytest.mark.parametrize("impl", ["library", "restatement"])
def test_algorithm2_hand_worked_search(impl):
    """Algorithm 2 on a hand-made summary, with the costs worked out by hand.

    Light-only cost: all 5000 + 5000 witnesses = 10000.  Non-literal search
    (eps = 0.5), starting at the largest key degree:
      (50, 5): light 5000 + 600, v = 0 heavy y, no product        -> 5600
      (25, 2): light 12, product 10 x 2 x 10                      -> 212
      (12, 1), (6, 1), (3, 1): the same sets, 212 (ties continue)
      (1, 1): light 0, product 10 x 5 x 10 = 500 > 212            -> stop at (3, 1).
    Literal search (eps = 0.95, ties stop), starting at Delta1 = N = 100:
      (100, 10): 5600;  (5, 1): 212;  next Delta1 = floor(0.25) = 0 -> stop at (5, 1).
    """
    s = _hand_summary()
    plan = jp.plan_summary if impl == "library" else ref.algorithm2
    for literal, want in ((0, (3, 1)), (1, (5, 1))):
        d1, d2, c, clo = plan(s, _hand_cal(literal))
        assert (d1, d2) == want, (literal, d1, d2)
        assert c == pytest.approx(212.0, rel=1e-12) and clo == pytest.approx(10000.0, rel=1e-12)


@pytest.mark.parametrize("impl", ["library", "restatement"])
def test_algorithm2_hand_worked_light_once(impl):
    """The light-x term counted once.  J = 5000; key degrees 2 (x3, sum 12)
    and 50 (x2, sum 4988); nine x of degree 1 (4900 witnesses) and one of
    degree 30 (100 witnesses), z alike; T_I = 1, product u v w.

    Printed sum (light_once 0): light only 5000 + 5000 = 10000; (50, 5)
    5000 + 4900 = 9900; (25, 2) 12 + 4900 + product 1*2*1 = 4914, the same
    to (3, 1); (1, 1) 0 + 4900 + 1*5*1 = 4905, lower again, and the search
    ends there: (1, 1).
    Counted once: light only 5000 + 5000 (1 - 1) = 5000; (50, 5) 5000 +
    4900 * 0 = 5000; (25, 2) 12 + 4900 (1 - 12/5000) + 2 = 4902.24, the same
    to (3, 1); (1, 1) 0 + 4900 + 5 = 4905 is higher: stop at (3, 1)."""
    i64 = lambda *v: np.array(v, dtype=np.int64)
    f64 = lambda *v: np.array(v, dtype=np.float64)
    s = dict(_hand_summary(), y=(i64(2, 50), i64(3, 2), f64(12.0, 4988.0)),
             x=(i64(1, 30), i64(9, 1), f64(4900.0, 100.0)), z=(i64(1, 30), i64(9, 1), None))
    plan = jp.plan_summary if impl == "library" else ref.algorithm2
    d1, d2, c, clo = plan(s, dict(_hand_cal(0), light_once=0))
    assert (d1, d2) == (1, 1)
    assert c == pytest.approx(4905.0, rel=1e-12) and clo == pytest.approx(10000.0, rel=1e-12)
    d1, d2, c, clo = plan(s, dict(_hand_cal(0), light_once=1))
    assert (d1, d2) == (3, 1)
    assert c == pytest.approx(4902.24, rel=1e-12) and clo == pytest.approx(5000.0, rel=1e-12)


@pytest.mark.parametrize("impl", ["library", "restatement"])
def test_algorithm2_hand_worked_product_floor(impl):
    """A product below the table's smallest cube costs that cube's time.
    Table: one cube p = 10 at 1000.  (50, 5): 5600, no product.  (25, 2):
    u v w = 200, p = 5.8 < 10, so 12 + 1000 = 1012 (scaled, it would be
    12 + 1000 * 200 / 1000 = 212); the same to (3, 1); (1, 1): u v w = 500,
    p = 7.9, 0 + 1000 = 1000, lower: the search ends at (1, 1).  Scaled
    down, (1, 1) would cost 500 > 212 and the search would stop at (3, 1)."""
    s = _hand_summary()
    plan = jp.plan_summary if impl == "library" else ref.algorithm2
    d1, d2, c, clo = plan(s, dict(_hand_cal(0), mm_p=[10.0], mm_s=[1000.0]))
    assert (d1, d2) == (1, 1)
    assert c == pytest.approx(1000.0, rel=1e-12) and clo == pytest.approx(10000.0, rel=1e-12)


@pytest.mark.parametrize("impl", ["library", "restatement"])
def test_algorithm2_hand_worked_no_gain(impl):
    """The same summary with a product 100 times dearer: (25, 2) then costs
    12 + 20000, more than (50, 5) at 5600, so the search stops at once; 5600
    beats the light-only 10000, so (50, 5) is returned.  With the product 10^4
    times dearer and J below 20 N the plain join is kept instead."""
    s = _hand_summary()
    plan = jp.plan_summary if impl == "library" else ref.algorithm2
    cal = dict(_hand_cal(0), mm_s=[100.0])
    d1, d2, c, clo = plan(s, cal)
    assert (d1, d2) == (50, 5) and c == pytest.approx(5600.0, rel=1e-12)
    small = dict(s, J=2000)  # J <= 20 N
    d1, d2, c, clo = plan(small, dict(_hand_cal(0), mm_s=[1e4]))
    assert (d1, d2) == (None, None) and c == pytest.approx(10000.0, rel=1e-12)


@pytest.mark.parametrize("impl", ["library", "restatement"])
def test_algorithm2_hand_worked_all_terms(impl):
    """Every term of the cost at 1 (T_I, T_m per x, T_s, T_m per byte):
    light-only = 10000 + 10 + 10 * 10 = 10110.  (50, 5): 5600 + 10 + 10 * 10
    = 5710.  (25, 2): 12 + 10 + 7 * 10 (x whose smallest key degree is at
    most 25) + product 200 + bytes 10 * 2 + 10 * 2 = 332, the same down to
    (3, 1); (1, 1): 0 + 10 + 0 + 500 + 100 = 610 stops the search."""
    s = _hand_summary()
    plan = jp.plan_summary if impl == "library" else ref.algorithm2
    cal = dict(_hand_cal(0), t_x=1.0, t_seq=1.0, t_byte=1.0)
    d1, d2, c, clo = plan(s, cal)
    assert (d1, d2) == (3, 1)
    assert c == pytest.approx(332.0, rel=1e-12) and clo == pytest.approx(10110.0, rel=1e-12)


@pytest.mark.parametrize("impl", ["library", "restatement"])
def test_algorithm2_hand_worked_delta2_rounding(impl):
    """A summary where the search ends at a Delta2 that rounding decides.
    Key degrees 2 (x3), 20, 50; x and z degrees 3 (x6) and 20 (x4); product
    cost 5 u v w.  (50, 5): 5600 with no heavy y.  (25, floor 2.5 = 2): light
    12 + 400, product 5 * 10 * 1 * 10 -> 912.  (12, 1): light 12, product
    5 * 10 * 2 * 10 -> 1012, worse: the search stops at (25, 2).  Rounding
    Delta2 up instead would take (25, 3) at 1092 and end at (3, 1)."""
    i64 = lambda *v: np.array(v, dtype=np.int64)
    f64 = lambda *v: np.array(v, dtype=np.float64)
    s = dict(_hand_summary(), y=(i64(2, 20, 50), i64(3, 1, 1), f64(12.0, 400.0, 4588.0)),
             x=(i64(3, 20), i64(6, 4), f64(600.0, 4400.0)), z=(i64(3, 20), i64(6, 4), None))
    plan = jp.plan_summary if impl == "library" else ref.algorithm2
    d1, d2, c, clo = plan(s, dict(_hand_cal(0), mm_s=[5.0]))
    assert (d1, d2) == (25, 2)
    assert c == pytest.approx(912.0, rel=1e-12) and clo == pytest.approx(10000.0, rel=1e-12)


@pytest.mark.parametrize("n,out", [(1e6, 1e3), (1e6, 1e5), (1e6, 1e6), (1e6, 3e7), (1e5, 1e9), (1e4, 1e12),
                                   (2000, 8301), (10, 0.5), (7, 6.324555320336759)])
def test_library_theory_thresholds_match_lemma3(n, out):
    """The library's THEORY thresholds are Lemma 3's minimisers (the
    restatement, itself checked against a grid minimisation in
    test_oracle.py) rounded down and clamped to [1, N]."""
    n = int(n)
    a, b = ref.theory_thresholds(n, out)
    clamp = lambda t: 1 if t < 1 else (n if t >= n else int(np.floor(t)))
    assert jp.plan_theory(n, out) == (clamp(a), clamp(b))


def test_library_theory_hand_values():
    """Worked by hand: N = 10^6, OUT = 10^3 (OUT <= N): Delta1 = 10^(3/3) = 10,
    Delta2 = 10^6 / 10^2 = 10^4.  N = 1000, OUT = 10^6 (OUT > N):
    Delta1 = Delta2 = (2 10^6 / 1001000)^(1/3) = 1.2594..., floor 1.
    N = 10^6, OUT = 7 10^6: (2 10^12 / 8 10^6)^(1/3) = 250000^(1/3) = 62.99."""
    assert jp.plan_theory(10**6, 1e3) == (10, 10**4)
    assert jp.plan_theory(1000, 1e6) == (1, 1)
    assert jp.plan_theory(10**6, 7e6) == (62, 62)
    assert jp.plan_theory(0, 5.0) == (None, None)
    assert jp.plan_theory(100, 0.0) == (None, None)


def test_library_out_estimate_by_hand():
    """The hand-made instance of test_oracle.py: sqrt(4 * 10) for
    |dom x| = 4, |dom z| = 3, J = 10, N = 7; (J/N)^2 as the lower bound;
    crossing bounds collapse to the upper bound; empty join gives 0."""
    assert jp.estimate_out(4, 3, 10, 7) == pytest.approx(np.sqrt(40.0), rel=1e-12)
    assert jp.estimate_out(5, 1000, 2000, 100) == pytest.approx(np.sqrt(400.0 * 2000.0), rel=1e-12)
    assert jp.estimate_out(5, 1000, 1000, 10) == pytest.approx(1000.0, rel=1e-12)
    assert jp.estimate_out(5, 5, 0, 10) == 0.0


def test_heavy_cost_terms():
    """jp_heavy_cost: M-hat (nearest cube scaled, floored at the smallest)
    plus T_m per byte of the u x v and w x v matrices; 0 without a product."""
    cal = dict(_hand_cal(0), mm_p=[10.0, 100.0], mm_s=[5.0, 2000.0], t_byte=0.5)
    assert jp.heavy_cost(0, 10, 10, cal) == 0.0 and jp.heavy_cost(10, 0, 10, cal) == 0.0
    # p = 80: nearest cube 100, scaled 2000 * 80^3 / 100^3 = 1024; bytes 0.5 * (80*80 + 80*80) = 6400
    assert jp.heavy_cost(80, 80, 80, cal) == pytest.approx(1024.0 + 6400.0, rel=1e-12)
    # p = 2: below the smallest cube, its time 5; bytes 0.5 * (2*2 + 2*2) = 4
    assert jp.heavy_cost(2, 2, 2, cal) == pytest.approx(5.0 + 4.0, rel=1e-12)


def test_selector_candidates_rule():
    assert jp.selector_candidates(10.0, [1.0, 10.0, 11.0, 0.0, 99.0]) == [True, False, False, True, True]


@pytest.mark.parametrize("impl", ["library", "restatement"])
def test_algorithm2_hand_worked_padded_inner_dimension(impl):
    """The product priced on v padded to a multiple of k_pad = 4.  The hand
    summary's (25, 2) has u v w = 10 x 2 x 10: padded 10 x 4 x 10 = 400, so
    12 + 400 = 412; the same to (3, 1); (1, 1) has v = 5, padded 8:
    0 + 800 > 412, so the search stops at (3, 1) with cost 412."""
    s = _hand_summary()
    plan = jp.plan_summary if impl == "library" else ref.algorithm2
    d1, d2, c, clo = plan(s, dict(_hand_cal(0), k_pad=4))
    assert (d1, d2) == (3, 1)
    assert c == pytest.approx(412.0, rel=1e-12) and clo == pytest.approx(10000.0, rel=1e-12)


def test_heavy_cost_pads_the_inner_dimension():
    cal = dict(_hand_cal(0), mm_p=[1.0], mm_s=[1.0], t_byte=1.0, k_pad=128)
    # v = 1 is priced as 128: M-hat 3 * 128 * 3 = 1152, bytes 3 * 128 + 3 * 128 = 768
    assert jp.heavy_cost(3, 1, 3, cal) == pytest.approx(1152.0 + 768.0, rel=1e-12)
    assert jp.heavy_cost(3, 1, 3, dict(cal, k_pad=1)) == pytest.approx(9.0 + 6.0, rel=1e-12)
