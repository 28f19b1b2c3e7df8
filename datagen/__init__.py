"""Seeded synthetic edge-list generators.

This module only draws inputs. It holds none of the join-project arithmetic, so
the CPU oracle and the GPU path can both be fed from it without sharing any of
the method's code. Every generator is deterministic in its seed (numpy PCG64).

Relations are binary and returned as two int32 numpy arrays ``(a, y)``: the
first column is the free variable (x, z or x_i), the second the join variable y
(the paper's problem statement, Section 2.1).

Workload shapes (the paper's datasets are not available, so these stand in):

* ``uniform_edges``: i.i.d. uniform (x, y) on a square, first n distinct kept.
* ``zipf_edges``: x uniform over ``n_x`` ids; the y *rank* follows a truncated
  Zipf(s) rank-frequency law over ``n_y`` ids, mapped to ids through a seeded
  permutation of its own (two relations drawn with different seeds therefore
  have independent y-degree orders); first n distinct (x, y) in draw order.
* ``communities``: c disjoint communities of m x-ids times g y-ids with edge
  probability p (the community structure of the paper's Example 1).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "uniform_edges",
    "zipf_edges",
    "communities",
    "random_small",
    "selfjoin_c1",
    "twopath_c2",
    "star_c3",
    "star4_c",
    "bsi_batch",
    "batch_c4",
    "batch_instance",
    "selector_instance",
    "selector_instance_clustered",
    "selector_instance_dense",
]


def _first_distinct(draw, n: int, n_y: int, rng, max_rounds: int = 64):
    """Draw (x, y) batches with ``draw(rng, m)`` until ``n`` distinct pairs exist.

    Keeps the first ``n`` distinct pairs in draw order.  Each round draws
    ``max(1024, 1.15 (n - have) + 16)`` pairs, where ``have`` is the number of
    distinct pairs drawn so far.  The pairs seen so far are kept as sorted
    per-round chunks, so a round costs time in its own size only.
    """
    chunks = []      # sorted distinct keys first seen in each round
    firsts = []      # their global draw positions
    bxs, bys = [], []
    have = 0
    drawn = 0
    for _ in range(max_rounds):
        if have >= n:
            pos = np.sort(np.concatenate(firsts))[:n]
            xs = np.concatenate(bxs)
            ys = np.concatenate(bys)
            return xs[pos].astype(np.int32), ys[pos].astype(np.int32)
        m = max(1024, int((n - have) * 1.15) + 16)
        bx, by = draw(rng, m)
        bx = bx.astype(np.int64)
        by = by.astype(np.int64)
        key = bx * n_y + by
        uk, first = np.unique(key, return_index=True)
        new = np.ones(uk.size, dtype=bool)
        for ch in chunks:
            j = np.searchsorted(ch, uk)
            j = np.minimum(j, ch.size - 1)
            new &= ch[j] != uk
        chunks.append(uk[new])
        firsts.append(first[new] + drawn)
        bxs.append(bx)
        bys.append(by)
        have += int(new.sum())
        drawn += m
    raise RuntimeError("could not draw enough distinct pairs; domain too small")


def uniform_edges(n: int, n_x: int, n_y: int, seed: int):
    """First ``n`` distinct (x, y) of i.i.d. uniform draws on [0,n_x) x [0,n_y)."""
    if n > n_x * n_y:
        raise ValueError("n exceeds the number of possible pairs")
    rng = np.random.default_rng(seed)

    def draw(r, m):
        return r.integers(0, n_x, m), r.integers(0, n_y, m)

    return _first_distinct(draw, n, n_y, rng)


def zipf_table(n_y: int, s: float) -> np.ndarray:
    """CDF of the truncated rank-frequency Zipf law P(rank=k) ~ k^-s, k=1..n_y."""
    w = np.arange(1, n_y + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    return cdf


def zipf_edges(n: int, n_x: int, n_y: int, s: float, seed: int):
    """x uniform in [0,n_x), y = perm(Zipf(s) rank over n_y), first n distinct."""
    rng = np.random.default_rng(seed)
    cdf = zipf_table(n_y, s)
    perm = rng.permutation(n_y)

    def draw(r, m):
        x = r.integers(0, n_x, m)
        rank = np.searchsorted(cdf, r.random(m), side="right")
        rank = np.minimum(rank, n_y - 1)
        return x, perm[rank]

    return _first_distinct(draw, n, n_y, rng)


def communities(c: int, m: int, g: int, p: float, seed: int):
    """c disjoint communities: x-block i (m ids) joined to y-block i (g ids).

    Each of the m*g possible edges of a community is present with probability
    p; every x and every y of a community is guaranteed at least one edge.
    """
    rng = np.random.default_rng(seed)
    xs, ys = [], []
    for i in range(c):
        mask = rng.random((m, g)) < p
        # guarantee no isolated vertex inside a community
        mask[np.arange(m), rng.integers(0, g, m)] = True
        mask[rng.integers(0, m, g), np.arange(g)] = True
        a, b = np.nonzero(mask)
        xs.append(a + i * m)
        ys.append(b + i * g)
    return (np.concatenate(xs).astype(np.int32), np.concatenate(ys).astype(np.int32))


def random_small(n: int, n_x: int, n_y: int, seed: int, dup: bool = False, signed: bool = False):
    """Tiny random relation for brute-force checks.

    With ``dup`` some rows are repeated (bag input); with ``signed`` the ids are
    spread over the whole int32 range including negatives and the extremes.
    """
    rng = np.random.default_rng(seed)
    x = rng.integers(0, n_x, n)
    y = rng.integers(0, n_y, n)
    if signed:
        xmap = rng.choice(np.arange(-(2**31), 2**31, 2**21, dtype=np.int64), n_x, replace=False)
        ymap = rng.choice(np.arange(-(2**31), 2**31, 2**21, dtype=np.int64), n_y, replace=False)
        xmap[0] = -(2**31)
        ymap[-1] = 2**31 - 1
        x, y = xmap[x], ymap[y]
    if dup and n > 0:
        k = max(1, n // 4)
        idx = rng.integers(0, n, k)
        x = np.concatenate([x, x[idx]])
        y = np.concatenate([y, y[idx]])
        p = rng.permutation(x.size)
        x, y = x[p], y[p]
    return x.astype(np.int32), y.astype(np.int32)


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------

def selfjoin_c1(seed: int = 1):
    """Self-join input: 2,000 distinct (x, y), both uniform in [0, 500)."""
    return uniform_edges(2000, 500, 500, seed)


def twopath_c2(scale: float = 1.0):
    """Two-path input pair: |R|=|S|=10M, 1M x/z ids, 200K y ids, Zipf(1.1) y.

    ``scale`` shrinks every size proportionally (for tests on the CPU).
    Seeds 2 (R) and 3 (S).
    """
    n = int(10_000_000 * scale)
    nx = max(1, int(1_000_000 * scale))
    ny = max(1, int(200_000 * scale))
    r = zipf_edges(n, nx, ny, 1.1, seed=2)
    s = zipf_edges(n, nx, ny, 1.1, seed=3)
    return r, s


def star_c3(scale: float = 1.0):
    """Star input: three relations of 2M edges, 500K x ids, 100K y ids, Zipf(1.3)."""
    n = int(2_000_000 * scale)
    nx = max(1, int(500_000 * scale))
    ny = max(1, int(100_000 * scale))
    return [zipf_edges(n, nx, ny, 1.3, seed=4 + i) for i in range(3)]


def star4_c(scale: float = 1.0):
    """Four-relation star input (k = 4): 500K edges each, 125K x ids, 25K y
    ids, Zipf(1.3) y with independent y orders (seeds 60..63); about 2.1e8
    witnesses."""
    n = int(500_000 * scale)
    nx = max(1, int(125_000 * scale))
    ny = max(1, int(25_000 * scale))
    return [zipf_edges(n, nx, ny, 1.3, seed=60 + i) for i in range(4)]


def bsi_batch(rx, ry, sz, sy, n: int, seed: int):
    """A batch of n set-intersection queries (a, c) over R(x, y) and S(z, y):
    half are drawn by picking a row (a, b) of R and then a row (c, b) of S
    with the same element b (a query that shares at least b), 3/8 pick a and
    c independently from the rows of R and S (sets in proportion to their
    size), and 1/8 name ids drawn uniformly from the int32 range."""
    rng = np.random.default_rng(seed)
    rx, ry, sz, sy = (np.asarray(v) for v in (rx, ry, sz, sy))
    order = np.argsort(sy, kind="stable")
    sy_sorted = sy[order]
    n_share = n // 2
    n_abs = n // 8
    n_ind = n - n_share - n_abs
    i = rng.integers(0, rx.size, 4 * n_share + 16)
    lo = np.searchsorted(sy_sorted, ry[i], side="left")
    hi = np.searchsorted(sy_sorted, ry[i], side="right")
    ok = hi > lo
    i, lo, hi = i[ok][:n_share], lo[ok][:n_share], hi[ok][:n_share]
    j = order[lo + (rng.random(i.size) * (hi - lo)).astype(np.int64)]
    n_ind += n_share - i.size
    tx = np.concatenate([rx[i], rng.choice(rx, n_ind), rng.integers(-2**31, 2**31 - 1, n_abs)])
    tz = np.concatenate([sz[j], rng.choice(sz, n_ind), rng.integers(-2**31, 2**31 - 1, n_abs)])
    p = rng.permutation(n)
    return tx[p].astype(np.int32), tz[p].astype(np.int32)


def batch_instance(i: int, lo: float = 1e3, hi: float = 1e6, seed0: int = 1000):
    """Instance i of the batched set: ((rx, ry), (sz, sy)), see ``batch_c4``."""
    rng = np.random.default_rng(seed0 + i)
    e = int(round(float(np.exp(rng.uniform(np.log(lo), np.log(hi))))))
    s = float(rng.uniform(0.6, 1.6))
    nx = max(2, -(-e // 10))
    ny = max(2, -(-e // 50))
    e = min(e, nx * ny // 2)
    sub = int(rng.integers(0, 2**31 - 1))
    r = zipf_edges(e, nx, ny, s, seed=sub)
    t = zipf_edges(e, nx, ny, s, seed=sub + 1)
    return r, t


def batch_c4(n_inst: int = 512, lo: float = 1e3, hi: float = 1e6, seed0: int = 1000):
    """Batched set: instance i has E_i ~ log-uniform[lo,hi] edges per relation.

    The Zipf exponent is U[0.6,1.6]; |dom x| = |dom z| = ceil(E/10) and
    |dom y| = ceil(E/50) (the same ratios as the single two-path input).
    Returns a list of ((rx, ry), (sz, sy)) tuples.
    """
    return [batch_instance(i, lo, hi, seed0) for i in range(n_inst)]


def selector_instance(i: int, lo: float = 1e5, hi: float = 2e7, seed0: int = 10_000,
                      scale: float = 1.0):
    """Instance i of the threshold-selector set: |R|=|S| log-uniform in [lo,hi].

    Zipf exponent U[0.5,1.8]; domains in the same ratios as the batched set.
    """
    rng = np.random.default_rng(seed0 + i)
    e = int(round(float(np.exp(rng.uniform(np.log(lo), np.log(hi)))) * scale))
    s = float(rng.uniform(0.5, 1.8))
    nx = max(2, -(-e // 10))
    ny = max(2, -(-e // 50))
    e = min(e, nx * ny // 2)
    sub = int(rng.integers(0, 2**31 - 1))
    return zipf_edges(e, nx, ny, s, seed=sub), zipf_edges(e, nx, ny, s, seed=sub + 1), s


def selector_instance_clustered(i: int, lo: float = 1e5, hi: float = 1e7, seed0: int = 30_000):
    """Instance i of the clustered selector set: dense communities plus a sparse part.

    |R| = |S| ~ E log-uniform in [lo, hi].  A fraction f ~ U[0.3, 0.9] of the
    edges forms c ~ U{1..200} communities (the structure of the paper's
    Example 1): each has m x-ids and g y-ids with edge probability
    p ~ U[0.05, 0.5], where d = m p ~ log-uniform [4, 400] (capped so that
    f E d <= 5e8) and g = f E / (c d).  S uses the same y blocks with its own
    z blocks and draws.  The rest is a Zipf part as in ``selector_instance``
    (exponent U[0.5, 1.8], domains E/10 and E/50) on ids above the
    communities'.  Returns ((rx, ry), (sz, sy), params).
    """
    rng = np.random.default_rng(seed0 + i)
    e = int(round(float(np.exp(rng.uniform(np.log(lo), np.log(hi))))))
    f = float(rng.uniform(0.3, 0.9))
    c = int(rng.integers(1, 201))
    p = float(rng.uniform(0.05, 0.5))
    d = float(np.exp(rng.uniform(np.log(4.0), np.log(400.0))))
    d = min(d, 5e8 / max(f * e, 1.0))
    m = max(2, int(round(d / p)))
    g = max(2, int(round(f * e / (c * max(d, 1.0)))))
    s = float(rng.uniform(0.5, 1.8))
    sub = int(rng.integers(0, 2**31 - 1))
    cx, cy = communities(c, m, g, p, seed=sub)
    dz, dy = communities(c, m, g, p, seed=sub + 1)
    es = max(1, e - cx.size)
    nx = max(2, -(-es // 10))
    ny = max(2, -(-es // 50))
    es = min(es, nx * ny // 2)
    (zx, zy) = zipf_edges(es, nx, ny, s, seed=sub + 2)
    (wz, wy) = zipf_edges(es, nx, ny, s, seed=sub + 3)
    ox, oy = c * m, c * g
    rx = np.concatenate([cx, zx + ox]).astype(np.int32)
    ry = np.concatenate([cy, zy + oy]).astype(np.int32)
    sz = np.concatenate([dz, wz + ox]).astype(np.int32)
    sy = np.concatenate([dy, wy + oy]).astype(np.int32)
    return (rx, ry), (sz, sy), {"e": e, "f": f, "c": c, "m": m, "g": g, "p": p, "s": s}


def selector_instance_dense(i: int, lo: float = 1e5, hi: float = 2e7, seed0: int = 50_000, jmax: float = 3e9):
    """Instance i of the dense selector set: few large dense communities, the
    shape of the paper's dense datasets and of Example 1, where a pair of
    sets shares many elements (the case the matrix product serves).

    |R| = |S| ~ E log-uniform in [lo, hi].  A fraction f ~ U[0.7, 1.0] of the
    edges forms c ~ U{1..8} communities with edge probability p ~ U[0.1, 0.5]
    and g = r / p^2 y-ids, where r ~ log-uniform [4, 128] is about the number
    of elements two sets of a community share; each community has
    m = f E p / (c r) x-ids (at least 2; fewer when the join size
    f E m p would exceed jmax).  S uses the same y blocks with its own z
    blocks and draws.  The rest is a Zipf part as in ``selector_instance``
    on ids above the communities'.  Returns ((rx, ry), (sz, sy), params).
    """
    rng = np.random.default_rng(seed0 + i)
    e = int(round(float(np.exp(rng.uniform(np.log(lo), np.log(hi))))))
    f = float(rng.uniform(0.7, 1.0))
    c = int(rng.integers(1, 9))
    p = float(rng.uniform(0.1, 0.5))
    r = float(np.exp(rng.uniform(np.log(4.0), np.log(128.0))))
    g = max(2, int(round(r / (p * p))))
    m = max(2, int(round(f * e / (c * g * p))))
    m = max(2, min(m, int(jmax / max(f * e * p, 1.0))))
    s = float(rng.uniform(0.5, 1.8))
    sub = int(rng.integers(0, 2**31 - 1))
    cx, cy = communities(c, m, g, p, seed=sub)
    dz, dy = communities(c, m, g, p, seed=sub + 1)
    es = max(1, e - cx.size)
    nx = max(2, -(-es // 10))
    ny = max(2, -(-es // 50))
    es = min(es, nx * ny // 2)
    (zx, zy) = zipf_edges(es, nx, ny, s, seed=sub + 2)
    (wz, wy) = zipf_edges(es, nx, ny, s, seed=sub + 3)
    ox, oy = c * m, c * g
    rx = np.concatenate([cx, zx + ox]).astype(np.int32)
    ry = np.concatenate([cy, zy + oy]).astype(np.int32)
    sz = np.concatenate([dz, wz + ox]).astype(np.int32)
    sy = np.concatenate([dy, wy + oy]).astype(np.int32)
    return (rx, ry), (sz, sy), {"e": e, "f": f, "c": c, "m": m, "g": g, "p": p, "r": r, "s": s}

