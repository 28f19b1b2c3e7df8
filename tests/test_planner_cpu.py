"""Algorithm 2 (Section 5) in the library, on the host, against its numpy
restatement under oracle/ (a second implementation: the paper prints no
optimizer numbers, so beyond these invariants the search is parity-unpinned)."""
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
