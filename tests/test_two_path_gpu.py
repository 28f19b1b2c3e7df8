"""Two-path parity: the HIP path through the C ABI against the CPU oracle.

Outputs must match bit for bit as sorted distinct pair sets; the reported
partition statistics must match the numpy restatement of Algorithm 1.
"""
import itertools

import numpy as np
import pytest

import datagen
import oracle
from oracle import reference as ref
from tests.conftest import load_golden

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("checks_mode")]

INF = None


@pytest.fixture(scope="module")
def jp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2002_12459_amd as jp
    return jp


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.int32))).cuda()


def run(jp, rx, ry, sz, sy, **kw):
    x, z, st = jp.default_handle(0).two_path(dev(rx), dev(ry), dev(sz), dev(sy), **kw)
    return x.cpu().numpy(), z.cpu().numpy(), st


def check_equal(jp, rx, ry, sz, sy, **kw):
    ex, ez = oracle.two_path(rx, ry, sz, sy)
    x, z, st = run(jp, rx, ry, sz, sy, **kw)
    assert x.size == ex.size, (x.size, ex.size, kw)
    np.testing.assert_array_equal(x, ex)
    np.testing.assert_array_equal(z, ez)
    return st


def test_worked_example(jp):
    rows = load_golden("two_path_example.txt")
    R = np.array([(int(r[1]), int(r[2])) for r in rows if r[0] == "R"])
    S = np.array([(int(r[1]), int(r[2])) for r in rows if r[0] == "S"])
    st = check_equal(jp, R[:, 0], R[:, 1], S[:, 0], S[:, 1], delta1=2, delta2=2)
    assert (st["u"], st["v"], st["w"]) == (3, 3, 3)
    assert st["J"] == 35 and st["J_L"] == 19 and st["J_H"] == 16 and st["nnz_heavy"] == 9
    assert st["n_out"] == 26


def test_selfjoin_2000_fixed_sqrt(jp):
    x, y = datagen.selfjoin_c1()
    d = int(np.sqrt(len(x)))  # 44
    st = check_equal(jp, x, y, x, y, delta1=d, delta2=d)
    assert st["delta1"] == 44 and st["delta2"] == 44


DELTAS = [1, 2, 3, 4, 6, 8, 12, 16, 44, None]


def test_selfjoin_2000_threshold_invariance(jp):
    """The output does not depend on the thresholds (Section 3.1 correctness
    argument); the partition statistics follow Algorithm 1."""
    x, y = datagen.selfjoin_c1()
    ex, ez = oracle.two_path(x, y, x, y)
    for d1, d2 in itertools.product(DELTAS, DELTAS):
        gx, gz, st = run(jp, x, y, x, y, delta1=d1, delta2=d2, strategy="fixed")
        np.testing.assert_array_equal(gx, ex, err_msg=f"{d1},{d2}")
        np.testing.assert_array_equal(gz, ez, err_msg=f"{d1},{d2}")
        if d1 in (1, 4, 12) and d2 in (2, 6, 44):
            r = ref.two_path_stats(x, y, x, y, d1, d2)
            for k in ("u", "v", "w", "J", "J_L", "J_H", "nnz_heavy", "dom_x", "dom_y", "dom_z"):
                assert st[k] == r[k], (k, d1, d2, st[k], r[k])


@pytest.mark.parametrize("seed", range(10))
def test_random_small(jp, seed):
    rng = np.random.default_rng(seed)
    signed = seed % 2 == 0
    nx, ny = int(rng.integers(1, 40)), int(rng.integers(1, 30))
    rx, ry = datagen.random_small(int(rng.integers(1, 400)), nx, ny, seed, dup=True, signed=signed)
    sz, sy = datagen.random_small(int(rng.integers(1, 400)), nx, ny, seed + 99, dup=True, signed=signed)
    if signed:
        sy = ry[rng.integers(0, ry.size, sy.size)]
    for d1, d2 in [(1, 1), (2, 3), (5, 1), (None, None)]:
        for rule in ("max", "r_only"):
            check_equal(jp, rx, ry, sz, sy, delta1=d1, delta2=d2, strategy="fixed", y_rule=rule)


def test_empty_and_degenerate(jp):
    e = np.zeros(0, np.int32)
    x, z, st = run(jp, e, e, e, e)
    assert x.size == 0 and st["n_out"] == 0
    x, z, st = run(jp, [1, 2], [3, 4], e, e)
    assert x.size == 0
    # no common y
    x, z, st = run(jp, [1, 2], [3, 4], [5], [6])
    assert x.size == 0
    # a single tuple each
    check_equal(jp, [7], [9], [-3], [9])
    # all ids identical
    check_equal(jp, [5] * 10, [5] * 10, [5] * 3, [5] * 3)
    # extreme ids
    lo, hi = -(2**31), 2**31 - 1
    check_equal(jp, [lo, hi, 0, lo], [hi, lo, hi, lo], [hi, lo, 0], [lo, lo, hi])


def test_auto_and_theory(jp):
    x, y = datagen.uniform_edges(20000, 3000, 400, 11)
    for strat in ("auto", "theory", "light"):
        check_equal(jp, x, y, x, y, strategy=strat)


@pytest.mark.parametrize("scale", [0.002, 0.01])
def test_zipf_scaled(jp, scale):
    """Skewed two-path input (Zipf y, uniform x) at a reduced scale, several
    threshold settings, R != S."""
    (rx, ry), (sz, sy) = datagen.twopath_c2(scale)
    ex, ez = oracle.two_path(rx, ry, sz, sy)
    for kw in (dict(strategy="light"), dict(delta1=50, delta2=8), dict(delta1=3, delta2=3), dict(strategy="auto")):
        x, z, st = run(jp, rx, ry, sz, sy, **kw)
        np.testing.assert_array_equal(x, ex, err_msg=str(kw))
        np.testing.assert_array_equal(z, ez, err_msg=str(kw))


@pytest.mark.parametrize("bmm", ["auto", "i8_t128", "i8_t256", "bitpop", "f16"])
def test_communities_dense_heavy(jp, bmm):
    """Dense communities: the heavy product carries most of the output."""
    # p = 0.5 over 150 y per community: two x of a community miss a common y
    # with probability 0.75^150 (about 1e-19), so every in-community pair is out.
    x, y = datagen.communities(4, 300, 150, 0.5, seed=5)
    st = check_equal(jp, x, y, x, y, delta1=10, delta2=10, bmm=bmm)
    assert st["nnz_heavy"] > 0 and st["n_out"] == 4 * 300 * 300
    assert st["bmm"] == {"bitpop": 2, "f16": 5}.get(bmm, 1 if bmm != "auto" else st["bmm"])


@pytest.mark.parametrize("kind", ["i8", "i8_t128", "i8_t256", "bitpop", "f16", "auto"])
@pytest.mark.parametrize("u,w,k", [(1, 1, 1), (37, 130, 200), (128, 128, 128), (257, 129, 1000), (600, 515, 77),
                                   (1100, 1300, 390), (513, 2049, 256), (1, 1, 5000), (100, 90, 20000),
                                   (129, 300, 9000)])
def test_bool_matmul_kernel(jp, u, w, k, kind):
    import torch
    rng = np.random.default_rng(u * 7 + w)
    ld = -(-k // 128) * 128
    A = np.zeros((u, ld), np.int8)
    B = np.zeros((w, ld), np.int8)
    A[:, :k] = rng.random((u, k)) < 0.02
    B[:, :k] = rng.random((w, k)) < 0.02
    C = A.astype(np.int64) @ B.astype(np.int64).T
    ei, ej = np.nonzero(C)
    rows, cols, ms = jp.default_handle(0).bool_matmul(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), k=k,
                                                      kind=kind)
    got = sorted(zip(rows.cpu().numpy().tolist(), cols.cpu().numpy().tolist()))
    assert got == sorted(zip(ei.tolist(), ej.tolist()))


def test_bool_matmul_counts_do_not_overflow(jp):
    """All-ones rows: counts equal K (here 4096 > int8 range); still exact."""
    import torch
    u, w, k = 64, 64, 4096
    A = torch.ones((u, k), dtype=torch.int8).cuda()
    B = torch.zeros((w, k), dtype=torch.int8)
    B[::2] = 1
    for kind in ("i8_t128", "i8_t256", "bitpop", "f16"):
        rows, cols, _ = jp.default_handle(0).bool_matmul(A, B.cuda(), kind=kind)
        assert rows.numel() == u * (w // 2)
        assert set(cols.cpu().numpy().tolist()) == set(range(0, w, 2))


def test_bool_matmul_more_tiles_than_one_grid(jp):
    """600000 x 600000 output (22M tiles of 128 x 128, more work-items than one
    dispatch can count): one-hot rows at column i % 128, so C[i][j] > 0 iff
    i and j agree mod 128; the count has a closed form."""
    import torch
    u = w = 600_000
    A = torch.zeros((u, 128), dtype=torch.int8, device="cuda")
    idx = torch.arange(u, device="cuda")
    A[idx, idx % 128] = 1
    per = np.bincount(np.arange(u) % 128, minlength=128).astype(np.int64)
    for kind in ("i8_t128", "i8_t256", "bitpop", "f16"):
        nnz, _ = jp.default_handle(0).bool_matmul_count(A, A, kind=kind)
        assert nnz == int((per * per).sum()), kind


@pytest.mark.parametrize("spacing", [1, 3, 5])
def test_spaced_z_ids(jp, spacing):
    """z ids spread over a range up to 5x their count (the per-x dedup keys z
    by id offset up to 4x, by rank beyond), with and without a heavy part."""
    x, y = datagen.communities(3, 120, 80, 0.3, seed=9)
    (zx, zy) = datagen.communities(3, 110, 80, 0.3, seed=10)
    sz = (zx.astype(np.int64) * spacing - 1000).astype(np.int32)
    check_equal(jp, x, y, sz, zy, strategy="light")
    st = check_equal(jp, x, y, sz, zy, strategy="fixed", delta1=10, delta2=10)
    assert st["nnz_heavy"] > 0


def test_dedup_unit_class_boundaries(jp):
    """x values whose candidate counts (cnt + cnt // 2 here) sit on both sides
    of the per-x class limits of the duplicate removal (up to 2560: packed
    with other x; up to 5120: a unit of its own; up to 20480: z windows
    sized to fit a unit's sort; more: bitmap windows), plus counts around
    4096, 8192 and 32768, interleaved, with duplicates inside every x."""
    rng = np.random.default_rng(11)
    counts = [1, 2, 63, 64, 65, 128, 129, 255, 256, 257, 511, 512, 513, 1023, 1024, 1025, 1706, 1707, 1708,
              2730, 2731, 2732, 3413, 3414, 4095, 4096, 4097, 5461, 5462, 9000, 13653, 13654, 21845, 21846,
              3, 700, 512, 5461, 2731, 1707, 3414, 512, 2]
    rx, ry, sz, sy = [], [], [], []
    nz = 40000
    for i, cnt in enumerate(counts):
        # x = i meets two lists: y = 2i (cnt distinct z) and y = 2i + 1 (half of them again)
        zs = rng.choice(nz, cnt, replace=False)
        half = zs[: max(1, cnt // 2)]
        rx += [i, i]
        ry += [2 * i, 2 * i + 1]
        sz += zs.tolist() + half.tolist()
        sy += [2 * i] * cnt + [2 * i + 1] * half.size
    check_equal(jp, rx, ry, sz, sy, strategy="light")
    check_equal(jp, rx, ry, sz, sy, strategy="fixed", delta1=600, delta2=1)


def test_dedup_crowded_and_wide_windows(jp):
    """Skewed z windows: an x whose candidates all fall in the lower half of
    a 1.3M-wide z range, an x whose candidates crowd into one narrow range,
    and an x with 1.3M candidates (many bitmap windows)."""
    rng = np.random.default_rng(5)
    Z = 1_300_000
    z_crowd = rng.choice(600_000, 6000, replace=False)          # x = 0: 6000 z in the lower half
    z_narrow = rng.choice(20_000, 5000, replace=False) + 700_000  # x = 2: 5000 z in a narrow range
    rx = [0, 1, 2, 2]
    ry = [0, 1, 2, 0]
    sz = z_crowd.tolist() + list(range(Z)) + z_narrow.tolist()
    sy = [0] * z_crowd.size + [1] * Z + [2] * z_narrow.size
    check_equal(jp, rx, ry, sz, sy, strategy="light")


@pytest.mark.parametrize("dedup", ["global", "segmented"])
def test_dedup_strategies(jp, dedup):
    """Both duplicate-removal strategies (one device-wide sort; per-x on-chip
    sort / bitmap) give the oracle's output, with and without a heavy part."""
    (rx, ry), (sz, sy) = datagen.twopath_c2(0.005)
    ex, ez = oracle.two_path(rx, ry, sz, sy)
    for kw in (dict(strategy="light"), dict(delta1=20, delta2=5)):
        x, z, st = run(jp, rx, ry, sz, sy, dedup=dedup, **kw)
        np.testing.assert_array_equal(x, ex, err_msg=str(kw))
        np.testing.assert_array_equal(z, ez, err_msg=str(kw))


@pytest.mark.parametrize("dedup", ["global", "segmented"])
def test_large_x_and_wide_z_domain(jp, dedup):
    """x values with far more witnesses than one on-chip unit holds, over a z
    domain wider than one bitmap window (more than 2^19 distinct z)."""
    rng = np.random.default_rng(7)
    nz = 700_000
    sz = np.concatenate([np.arange(nz), rng.integers(0, nz, 50_000)]).astype(np.int32)
    sy = np.concatenate([np.zeros(nz), rng.integers(1, 2000, 50_000)]).astype(np.int32)
    rx = np.concatenate([np.arange(6), rng.integers(0, 5000, 20_000)]).astype(np.int32)
    ry = np.concatenate([np.zeros(6), rng.integers(1, 2000, 20_000)]).astype(np.int32)
    ex, ez = oracle.two_path(rx, ry, sz, sy)
    for kw in (dict(strategy="light"), dict(delta1=30, delta2=6)):
        x, z, st = run(jp, rx, ry, sz, sy, dedup=dedup, **kw)
        assert x.size == ex.size
        np.testing.assert_array_equal(x, ex)
        np.testing.assert_array_equal(z, ez)


def _planner_instances():
    x, y = datagen.communities(6, 40, 30, 0.6, seed=1)
    yield x, y, x, y
    (rx, ry), (sz, sy) = datagen.twopath_c2(0.002)
    yield rx, ry, sz, sy
    x, y = datagen.zipf_edges(6000, 300, 200, 1.4, seed=9)
    yield x, y, x, y


@pytest.mark.parametrize("inst", range(3))
def test_device_summary_drives_the_same_choice(jp, inst):
    """The degree indexes built on the GPU give Algorithm 2 the same inputs as
    the numpy restatement: the chosen thresholds agree, and the features are
    the documented logs of sizes and degree quantiles."""
    rx, ry, sz, sy = list(_planner_instances())[inst]
    h = jp.default_handle(0)
    cal = h.get_calibration()
    for c in (cal, dict(cal, mm_s=[s * 1e-3 for s in cal["mm_s"]], t_byte=0.0)):
        h.set_calibration(c)
        d1, d2, f = h.plan_two_path(dev(rx), dev(ry), dev(sz), dev(sy))
        s = ref.degree_summary(rx, ry, sz, sy)
        e1, e2, _, _ = ref.algorithm2(s, c)
        assert (d1, d2) == (e1, e2), (inst, d1, d2, e1, e2)
    h.set_calibration(cal)
    assert np.isclose(f[0], np.log(s["n_r"]), rtol=1e-5) and np.isclose(f[1], np.log(s["n_s"]), rtol=1e-5)
    assert np.isclose(f[14], np.log(1 + s["x"][0][-1]), rtol=1e-5)
    assert np.isclose(f[15], np.log(1 + s["z"][0][-1]), rtol=1e-5)
    # and the whole pipeline under the optimizer's thresholds is exact
    check_equal(jp, rx, ry, sz, sy, strategy="auto")


def test_f16_product_refuses_counts_beyond_its_exact_range(jp):
    """fp16 operands with fp32 accumulation are exact below 2^24: a product
    whose inner dimension reaches 2^24 is refused before any launch."""
    import torch
    A = torch.zeros((1, 1 << 24), dtype=torch.int8, device="cuda")
    with pytest.raises(jp.JoinProjectError) as e:
        jp.default_handle(0).bool_matmul_count(A, A, kind="f16")
    assert e.value.status == 5  # JP_EPRECISION
    nnz, _ = jp.default_handle(0).bool_matmul_count(A[:, :(1 << 24) - 128], A[:, :(1 << 24) - 128], kind="f16")
    assert nnz == 0


def test_f16_product_end_to_end(jp):
    rx, ry = datagen.zipf_edges(40_000, 4_000, 800, 1.1, 81)
    sz, sy = datagen.zipf_edges(40_000, 4_000, 800, 1.1, 82)
    st = check_equal(jp, rx, ry, sz, sy, delta1=20, delta2=8, bmm="f16")
    assert st["bmm"] == 5 and st["nnz_heavy"] > 0


def test_self_join_symmetric_product_many_tiles(jp):
    """A self-join whose heavy part spans 6 x 6 tiles of 256: the product runs
    on the 21 tiles on and above the diagonal and mirrors the rest."""
    x, y = datagen.communities(6, 250, 100, 0.5, seed=9)
    st = check_equal(jp, x, y, x, y, delta1=10, delta2=10, bmm="i8_t256")
    assert st["u"] == st["w"] == 1500 and st["nnz_heavy"] == 6 * 250 * 250
    # the same relation passed as two different column pairs: no symmetry assumed
    st2 = check_equal(jp, x, y, x.copy(), y.copy(), delta1=10, delta2=10, bmm="i8_t256")
    assert st2["nnz_heavy"] == st["nnz_heavy"]


@pytest.mark.parametrize("seed", [0, 1, 12345, 2**63 + 5])
def test_sampled_out_estimate_matches_the_restatement(jp, seed):
    """The sampled output-size estimate (a selector input): the same draws of
    x and the same exact distinct counts as the numpy restatement."""
    cases = [datagen.zipf_edges(20_000, 3_000, 500, 1.2, 61) + datagen.zipf_edges(20_000, 3_000, 500, 1.2, 62),
             datagen.random_small(600, 300, 40, seed=63, dup=True, signed=True) * 2,
             ]
    if seed == 0:  # more than 2^20 distinct z: a device sort counts the draws, not LDS bitmaps
        cases.append(datagen.zipf_edges(3_000, 3_000, 500, 1.2, 64) +
                     datagen.zipf_edges(3_000_000, 2_000_000, 500, 0.8, 65))
    for rx, ry, sz, sy in cases:
        D, k, n, est = ref.sampled_out_estimate(rx, ry, sz, sy, seed)
        x, z, st = run(jp, rx, ry, sz, sy, strategy="light", seed=seed, sampled_out=True)
        assert (st["sample_distinct"], st["sample_draws"], st["dom_x"]) == (D, k, n)
        if len(sz) > 1_000_000:
            assert st["dom_z"] > 1 << 20
        assert st["out_sampled"] == pytest.approx(est, rel=1e-12)
