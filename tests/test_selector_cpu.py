"""What the trained threshold selector gains over the cost model (no GPU).

The selector's training data is the library's own timing sweep on MI355X:
every instance was run at each of the 65 threshold cells, with the cost
model (Algorithm 2), Lemma 3's thresholds and sqrt(N) thresholds timed
beside them.  The held-out instances were not used in training.  Here the
committed weights are evaluated with the fp64 reference network: the cell
it picks on each held-out instance is compared with the fastest cell.
Outputs are identical at every cell (checked during the sweep and by the
GPU tests), so this is purely a time comparison.
"""
import gzip
import json
import math
import os

import numpy as np
import pytest

from oracle import mlp

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.join(os.path.dirname(HERE), "paper_2002_12459_amd")
WEIGHTS = os.path.join(PKG, "selector_mi355x.json")
TABLE = os.path.join(PKG, "selector_sweep_mi355x.jsonl.gz")

pytestmark = pytest.mark.skipif(not (os.path.exists(WEIGHTS) and os.path.exists(TABLE)),
                                reason="selector weights or sweep table not present")


def _load():
    with open(WEIGHTS) as fh:
        w = json.load(fh)
    with gzip.open(TABLE, "rt") as fh:
        recs = [json.loads(line) for line in fh if line.strip()]
    return w, recs


def _holdout(w, recs):
    meta = w["meta"]
    lim = {"zipf": meta["holdout_from"], "clustered": meta["holdout_from_clustered"],
           "dense": meta.get("holdout_from_dense", 0)}
    return [r for r in recs if r["i"] >= lim[r.get("family", "zipf")]]


def _candidates(r):
    """The library's rule: light only (cell 64) and every cell whose heavy
    part's estimate is below the light-only plan's estimate."""
    if "heavy" not in r:
        return np.ones(65, dtype=bool)
    h = np.asarray(r["heavy"], dtype=np.float64)
    ok = h < r["est"][64]
    ok[64] = True
    return ok


def _picks(w, recs):
    x = np.asarray([r["features"] for r in recs], dtype=np.float32)
    xin = (x - np.asarray(w["mean"], np.float32)) / np.asarray(w["scale"], np.float32)
    y, _ = mlp.forward(np.asarray(w["params"], np.float64), w["n_out"], xin.astype(np.float64))
    for i, r in enumerate(recs):
        y[i, ~_candidates(r)] = np.inf
    return y.argmin(axis=1)


def _geo(v):
    return float(np.exp(np.mean(np.log(v))))


def _best(r):
    return min(t for t in r["t"] if t is not None)


def test_weights_match_the_layout():
    w, _ = _load()
    assert w["n_out"] == 65
    assert len(w["params"]) == mlp.param_count(65)
    assert len(w["mean"]) == len(w["scale"]) == 16 and min(w["scale"]) > 0


def test_holdout_is_disjoint_and_large_enough():
    w, recs = _load()
    te = _holdout(w, recs)
    assert len(te) >= 100
    assert len({(r.get("family", "zipf"), r["i"]) for r in recs}) == len(recs)


def test_selector_beats_the_cost_model_on_held_out_instances():
    w, recs = _load()
    te = _holdout(w, recs)
    skip = w["meta"]["skip_ratio"]
    ks = _picks(w, te)
    mlp_regret = [skip if r["t"][k] is None else r["t"][k] / _best(r) for r, k in zip(te, ks)]
    cost_regret = [r["auto"]["t"] / _best(r) for r in te]
    g_mlp, g_cost = _geo(mlp_regret), _geo(cost_regret)
    # within 10% of the best swept cell (geometric mean), and better than Algorithm 2
    assert g_mlp <= 1.10, g_mlp
    assert g_mlp < g_cost, (g_mlp, g_cost)
    for fam in sorted({r.get("family", "zipf") for r in te}):
        sel = [i for i, r in enumerate(te) if r.get("family", "zipf") == fam]
        assert _geo([mlp_regret[i] for i in sel]) <= 1.15, fam


def _light_only(r):
    """The light-only cell (no heavy part) is the last of the 65."""
    return r["t"][-1]


def test_selector_is_no_worse_than_light_only_where_the_product_pays():
    """On held-out instances where some plan with a heavy part beats light
    only by more than 10%, the selector's pick must on average beat light only."""
    w, recs = _load()
    te = [r for r in _holdout(w, recs) if _light_only(r) is not None and _best(r) < 0.9 * _light_only(r)]
    if len(te) < 5:
        pytest.skip(f"only {len(te)} held-out instances where the product pays")
    skip = w["meta"]["skip_ratio"]
    ks = _picks(w, te)
    ratio = [(skip * _best(r) if r["t"][k] is None else r["t"][k]) / _light_only(r) for r, k in zip(te, ks)]
    assert _geo(ratio) < 1.0, _geo(ratio)
