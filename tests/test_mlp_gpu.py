"""Selector network kernels (forward, loss gradient, Adam) through the C ABI
against the fp64 reference, and the AUTO_MLP strategy end to end."""
import numpy as np
import pytest

import datagen
import oracle
from oracle import mlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def jp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2002_12459_amd as jp
    return jp


@pytest.fixture(scope="module")
def h(jp):
    return jp.Handle(0, selector=None)


def f32(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float32))).cuda()


def problem(k, b, seed):
    rng = np.random.default_rng(seed)
    p = mlp.init_params(k, seed) + rng.normal(0, 0.05, mlp.param_count(k))
    p = p.astype(np.float32).astype(np.float64)  # what the GPU sees
    x = rng.normal(0, 1, (b, 16)).astype(np.float32).astype(np.float64)
    t = rng.normal(0, 1, (b, k)).astype(np.float32).astype(np.float64)
    m = (rng.random((b, k)) < 0.7).astype(np.float64)
    if b:
        m[0, :] = 0.0
    return p, x, t, m


# fp32 forward over 16 + 64 + 64 products per output: relative error well
# below 1e-5 of the output scale.
@pytest.mark.parametrize("k,b", [(65, 1), (65, 300), (1, 17), (256, 9), (130, 3)])
def test_forward_matches_reference(jp, h, k, b):
    p, x, _, _ = problem(k, b, k * 1000 + b)
    y = h.mlp_forward(f32(p), f32(x), n_out=k).cpu().numpy()
    ey, _ = mlp.forward(p, k, x)
    scale = max(1.0, np.abs(ey).max())
    assert np.abs(y - ey).max() <= 2e-5 * scale


def test_forward_empty_batch(jp, h):
    import torch
    p, _, _, _ = problem(65, 0, 5)
    y = h.mlp_forward(f32(p), torch.empty((0, 16), dtype=torch.float32, device="cuda"))
    assert y.shape == (0, 65)


# The gradient sums per-sample terms with fp32 atomics: compare against the
# fp64 backward pass relative to the largest gradient entry.
@pytest.mark.parametrize("k,b", [(65, 1), (65, 257), (3, 40), (256, 5)])
def test_gradient_matches_reference(jp, h, k, b):
    p, x, t, m = problem(k, b, 7 * k + b)
    g, loss = h.mlp_grad(f32(p), f32(x), f32(t), f32(m))
    eL, eg = mlp.loss_and_grad(p, k, x, t, m)
    g = g.cpu().numpy()
    assert abs(float(loss.item()) - eL) <= 1e-5 * max(1.0, abs(eL))
    assert np.abs(g - eg).max() <= 1e-5 * max(1e-3, np.abs(eg).max())


def test_gradient_is_overwritten(jp, h):
    import torch
    p, x, t, m = problem(65, 8, 11)
    g = torch.full((mlp.param_count(65),), 7.0, dtype=torch.float32, device="cuda")
    loss = torch.full((1,), 7.0, dtype=torch.float32, device="cuda")
    h.mlp_grad(f32(p), f32(x), f32(t), f32(np.zeros_like(m)), grad=g, loss=loss)
    assert float(loss.item()) == 0.0 and float(g.abs().max().item()) == 0.0


def test_adam_matches_reference(jp, h):
    rng = np.random.default_rng(3)
    n = mlp.param_count(65)
    p = rng.normal(0, 1, n).astype(np.float32).astype(np.float64)
    m = np.zeros(n)
    v = np.zeros(n)
    tp, tm, tv = f32(p), f32(m), f32(v)
    for step in range(1, 6):
        g = rng.normal(0, 1, n).astype(np.float32).astype(np.float64)
        h.mlp_adam(tp, tm, tv, f32(g), step, lr=1e-2)
        p, m, v = mlp.adam_step(p, m, v, g, step, 1e-2)
    assert np.abs(tp.cpu().numpy() - p).max() <= 1e-5
    assert np.abs(tm.cpu().numpy() - m).max() <= 1e-6
    assert np.abs(tv.cpu().numpy() - v).max() <= 1e-6


def test_training_with_kernels_follows_reference(jp, h):
    """Twenty full-batch Adam steps on the GPU track the fp64 reference run."""
    k, b = 65, 64
    p, x, t, m = problem(k, b, 21)
    tp, tm, tv = f32(p), f32(np.zeros_like(p)), f32(np.zeros_like(p))
    tx, tt, tw = f32(x), f32(t), f32(m)
    rp, rm, rv = p.copy(), np.zeros_like(p), np.zeros_like(p)
    losses = []
    for step in range(1, 21):
        g, loss = h.mlp_grad(tp, tx, tt, tw)
        losses.append(float(loss.item()))
        h.mlp_adam(tp, tm, tv, g, step, lr=3e-3)
        _, rg = mlp.loss_and_grad(rp, k, x, t, m)
        rp, rm, rv = mlp.adam_step(rp, rm, rv, rg, step, 3e-3)
    assert losses[-1] < 0.8 * losses[0]
    assert np.abs(tp.cpu().numpy() - rp).max() <= 1e-3
    assert mlp.loss(tp.cpu().numpy().astype(np.float64), k, x, t, m) == pytest.approx(
        mlp.loss(rp, k, x, t, m), rel=1e-3)


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.int32))).cuda()


def test_auto_mlp_picks_a_best_scored_cell_and_stays_exact(jp):
    (rx, ry), (sz, sy), _ = datagen.selector_instance(3, lo=5e3, hi=2e4)
    hd = jp.Handle(0, selector=None)
    d1a, d2a, feats = hd.plan_two_path(dev(rx), dev(ry), dev(sz), dev(sy))
    mean = np.array(feats, dtype=np.float64)
    scale = np.ones(16)
    k = 65
    p = mlp.init_params(k, 99).astype(np.float32).astype(np.float64)
    hd.set_selector(p.tolist(), (mean - 0.5).tolist(), scale.tolist())
    x, z, st = hd.two_path(dev(rx), dev(ry), dev(sz), dev(sy), strategy="mlp")
    ex, ez = oracle.two_path(rx, ry, sz, sy)
    assert np.array_equal(x.cpu().numpy(), ex) and np.array_equal(z.cpu().numpy(), ez)
    assert st["strategy"] == 4
    # the reference network's scores on the same normalised features
    xin = (np.array(feats, dtype=np.float32) - (mean - 0.5).astype(np.float32)) / scale.astype(np.float32)
    score, _ = mlp.forward(p, k, xin.astype(np.float64)[None, :])
    score = score[0]
    cells = list(zip(*jp.selector_cells(feats)))
    inf = jp.DELTA_INF
    picked = (st["delta1"] if st["delta1"] != inf else None, st["delta2"] if st["delta2"] != inf else None)
    # candidates: light only and the cells whose heavy part alone is
    # estimated below the light-only plan (the library's rule)
    d1s, d2s = jp.selector_cells(feats)
    est, dims = hd.plan_cells(dev(rx), dev(ry), dev(sz), dev(sy), d1s, d2s)
    cal = hd.get_calibration()
    cand = jp.selector_candidates(est[-1], [jp.heavy_cost(u, v, w, cal) for u, v, w in dims])
    best = min(s for s, ok in zip(score, cand) if ok)
    ok = [c for c, s, q in zip(cells, score, cand) if q and s <= best + 1e-4]
    assert picked in ok
    # the planning entry point makes the same choice
    d1, d2, _ = hd.plan_two_path(dev(rx), dev(ry), dev(sz), dev(sy), strategy="mlp")
    assert (d1, d2) == picked
    # without weights AUTO_MLP is Algorithm 2
    hd.clear_selector()
    _, _, st2 = hd.two_path(dev(rx), dev(ry), dev(sz), dev(sy), strategy="mlp")
    assert st2["strategy"] == 0
    assert (st2["delta1"], st2["delta2"]) == (d1a if d1a is not None else inf, d2a if d2a is not None else inf)
    hd.close()


def test_auto_mlp_skips_cells_whose_product_alone_exceeds_light_only(jp):
    """A network whose lowest score is on a cell that the candidate rule
    excludes (its heavy part alone estimated above the light-only plan)
    does not get that cell."""
    (rx, ry), (sz, sy), _ = datagen.selector_instance(3, lo=5e3, hi=2e4)
    hd = jp.Handle(0, selector=None)
    _, _, feats = hd.plan_two_path(dev(rx), dev(ry), dev(sz), dev(sy))
    d1s, d2s = jp.selector_cells(feats)
    est, dims = hd.plan_cells(dev(rx), dev(ry), dev(sz), dev(sy), d1s, d2s)
    cal = hd.get_calibration()
    heavy = [jp.heavy_cost(u, v, w, cal) for u, v, w in dims]
    cand = jp.selector_candidates(est[-1], heavy)
    excluded = [k for k, q in enumerate(cand) if not q]
    if not excluded:
        hd.close()
        pytest.skip("no cell of this instance is excluded")
    k = 65
    p = np.zeros(mlp.param_count(k))
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p, k)
    b3[:] = 0.0
    b3[excluded[0]] = -100.0  # the excluded cell scores lowest by far
    alt = next(j for j, q in enumerate(cand) if q and j != 64) if any(cand[:64]) else 64
    b3[alt] = -50.0            # the best candidate
    hd.set_selector(mlp.pack(W1, b1, W2, b2, W3, b3).tolist(), np.zeros(16).tolist(), np.ones(16).tolist())
    x, z, st = hd.two_path(dev(rx), dev(ry), dev(sz), dev(sy), strategy="mlp")
    inf = jp.DELTA_INF
    got = (None if st["delta1"] == inf else st["delta1"], None if st["delta2"] == inf else st["delta2"])
    assert got == (d1s[alt], d2s[alt])
    ex, ez = oracle.two_path(rx, ry, sz, sy)
    assert np.array_equal(x.cpu().numpy(), ex) and np.array_equal(z.cpu().numpy(), ez)
    hd.close()


def test_every_selector_cell_is_exact(jp):
    """The output does not depend on which of the 65 cells is used."""
    (rx, ry), (sz, sy), _ = datagen.selector_instance(8, lo=3e3, hi=1e4)
    hd = jp.Handle(0, selector=None)
    _, _, feats = hd.plan_two_path(dev(rx), dev(ry), dev(sz), dev(sy))
    ex, ez = oracle.two_path(rx, ry, sz, sy)
    d1s, d2s = jp.selector_cells(feats)
    for d1, d2 in zip(d1s, d2s):
        x, z, st = hd.two_path(dev(rx), dev(ry), dev(sz), dev(sy), delta1=d1, delta2=d2)
        assert np.array_equal(x.cpu().numpy(), ex) and np.array_equal(z.cpu().numpy(), ez), (d1, d2)
    hd.close()


def test_plan_cells_heavy_dims(jp):
    (rx, ry), (sz, sy), _ = datagen.selector_instance(5, lo=2e4, hi=5e4)
    from oracle import reference as ref
    hd = jp.Handle(0, selector=None)
    cells = [(2, 1), (8, 3), (40, 10), (None, None)]
    est, dims = hd.plan_cells(dev(rx), dev(ry), dev(sz), dev(sy), [c[0] for c in cells], [c[1] for c in cells])
    a, b, c, d = ref.reduce_two_path(rx, ry, sz, sy)

    def deg(v):
        return np.unique(v, return_counts=True)

    (_, dx), (yr, dyr), (ys, dys), (_, dz) = deg(a), deg(b), deg(d), deg(c)
    assert np.array_equal(yr, ys)
    key = np.maximum(dyr, dys)
    big = 2**62
    for (d1, d2), e, (u, v, w) in zip(cells, est, dims):
        d1 = big if d1 is None else d1
        d2 = big if d2 is None else d2
        assert (u, v, w) == (int((dx > d2).sum()), int((key > d1).sum()), int((dz > d2).sum())), (d1, d2)
        assert e > 0
    hd.close()
