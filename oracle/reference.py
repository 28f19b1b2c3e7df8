"""Numpy restatements of the method's intermediate quantities.  TEST INFRASTRUCTURE.

These check the statistics the GPU path reports (partition sizes, light
witness count, heavy product nonzeros) against the paper's definitions:

* Section 3.1 (two-path): relations are split at integer thresholds
  Delta1 (join variable y) and Delta2 (free variables x, z); a tuple is light
  when one of its values has degree at most the threshold.  Light tuples are
  joined combinatorially, heavy tuples go through the 0/1 matrix product
  M = M1 x M2, and the two outputs are unioned (Algorithm 1).
* Section 3.2 (star): R_i^- holds light x_i, R_i^diamond holds tuples whose y
  is light in every other relation, R_i^+ the rest; the heavy part is the
  product of the grouped matrices V and W.
* Lemma 3 (Section 3.1 analysis): closed-form thresholds for omega = 2.
* Section 5: output-size estimate from |dom x| and the full join size.

Readings of the paper where it is ambiguous (y classification shared by both
relations with the larger degree deciding, light means degree <= threshold,
relations are sets, dangling tuples removed first) are the ones listed in the
design notes; each function names the reading it uses.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

Y_RULE_MAX = 0
Y_RULE_R_ONLY = 1
INF = np.iinfo(np.int64).max


def distinct_edges(a, b):
    """Set semantics: remove repeated rows (relations are sets)."""
    k = np.unique(np.stack([np.asarray(a, np.int64), np.asarray(b, np.int64)], 1), axis=0)
    return k[:, 0], k[:, 1]


def reduce_two_path(rx, ry, sz, sy):
    """Distinct edges of R and S, keeping only y present in both relations.

    Removing tuples that contribute to no output is the preprocessing step the
    paper assumes before partitioning (Section 3.1).
    """
    rx, ry = distinct_edges(rx, ry)
    sz, sy = distinct_edges(sz, sy)
    common = np.intersect1d(ry, sy)
    kr = np.isin(ry, common)
    ks = np.isin(sy, common)
    return rx[kr], ry[kr], sz[ks], sy[ks]


def _deg(v):
    u, c = np.unique(v, return_counts=True)
    return dict(zip(u.tolist(), c.tolist()))


def two_path_stats(rx, ry, sz, sy, delta1, delta2, y_rule=Y_RULE_MAX):
    """Partition sizes and witness counts of Algorithm 1 at (delta1, delta2).

    Returns a dict with n_r, n_s (after reduction), dom sizes, u, v, w (heavy
    x, y, z counts), J (full join size), J_L (light witnesses: the disjoint
    classes R^- join S and R^+ join S^-), J_H (heavy witnesses) and
    nnz_heavy (nonzeros of M1 x M2), plus the heavy count matrix itself and the
    distinct light pairs.
    """
    rx, ry, sz, sy = reduce_two_path(rx, ry, sz, sy)
    dRx, dRy, dSy, dSz = _deg(rx), _deg(ry), _deg(sy), _deg(sz)
    xh = {a for a, d in dRx.items() if d > delta2}
    zh = {c for c, d in dSz.items() if d > delta2}
    if y_rule == Y_RULE_MAX:
        yh = {b for b in dRy if max(dRy[b], dSy[b]) > delta1}
    else:
        yh = {b for b in dRy if dRy[b] > delta1}
    J = sum(dRy[b] * dSy[b] for b in dRy)
    # Per y: light / heavy x in R and z in S.
    Rby, Sby = {}, {}
    for a, b in zip(rx.tolist(), ry.tolist()):
        Rby.setdefault(b, []).append(a)
    for c, b in zip(sz.tolist(), sy.tolist()):
        Sby.setdefault(b, []).append(c)
    J_L = 0
    J_H = 0
    light_pairs = set()
    for b in Rby:
        xs, zs = Rby[b], Sby[b]
        if b not in yh:
            J_L += len(xs) * len(zs)
            light_pairs.update((a, c) for a in xs for c in zs)
        else:
            Lx = [a for a in xs if a not in xh]
            Hx = [a for a in xs if a in xh]
            Lz = [c for c in zs if c not in zh]
            Hz = [c for c in zs if c in zh]
            J_L += len(Lx) * len(zs) + len(Hx) * len(Lz)
            J_H += len(Hx) * len(Hz)
            light_pairs.update((a, c) for a in Lx for c in zs)
            light_pairs.update((a, c) for a in Hx for c in Lz)
    X = sorted(xh)
    Y = sorted(yh)
    Z = sorted(zh)
    xi = {a: i for i, a in enumerate(X)}
    yi = {b: i for i, b in enumerate(Y)}
    zi = {c: i for i, c in enumerate(Z)}
    M1 = np.zeros((len(X), len(Y)), np.int64)
    M2 = np.zeros((len(Y), len(Z)), np.int64)
    for a, b in zip(rx.tolist(), ry.tolist()):
        if a in xi and b in yi:
            M1[xi[a], yi[b]] = 1
    for c, b in zip(sz.tolist(), sy.tolist()):
        if c in zi and b in yi:
            M2[yi[b], zi[c]] = 1
    M = M1 @ M2
    heavy_pairs = {(X[i], Z[j]) for i, j in zip(*np.nonzero(M))}
    return dict(
        n_r=int(rx.size), n_s=int(sz.size),
        dom_x=len(dRx), dom_y=len(dRy), dom_z=len(dSz),
        u=len(X), v=len(Y), w=len(Z),
        J=int(J), J_L=int(J_L), J_H=int(J_H),
        nnz_heavy=int(np.count_nonzero(M)),
        X=X, Y=Y, Z=Z, M1=M1, M2=M2, M=M,
        light_pairs=light_pairs, heavy_pairs=heavy_pairs,
    )


def star_stats(rels, delta1, delta2):
    """Star partition of Section 3.2 for k relations at (delta1, delta2).

    A tuple (a,b) of R_i is in R_i^- when a has degree <= delta2 in R_i, in
    R_i^diamond when b has degree <= delta1 in every other relation, and in
    R_i^+ otherwise.  A witness (a_1..a_k, b) is heavy when every tuple is in
    its R_i^+.  Returns J, J_L, J_H, the heavy x counts u_i, the number of
    y values that can carry a heavy witness, the distinct heavy tuples and the
    distinct light tuples.
    """
    k = len(rels)
    R = [distinct_edges(a, b) for a, b in rels]
    common = R[0][1]
    for a, b in R[1:]:
        common = np.intersect1d(common, b)
    R = [(a[np.isin(b, common)], b[np.isin(b, common)]) for a, b in R]
    dx = [_deg(a) for a, _ in R]
    dy = [_deg(b) for _, b in R]
    by = []
    for a, b in R:
        m = {}
        for p, q in zip(a.tolist(), b.tolist()):
            m.setdefault(q, []).append(p)
        by.append(m)
    J = J_L = J_H = 0
    heavy, light = set(), set()
    hy = 0
    for b in np.unique(common).tolist():
        heavy_in = [dy[i][b] > delta1 for i in range(k)]
        lists = [by[i][b] for i in range(k)]

        def plus(i, a):
            # a heavy in R_i and b heavy in some other relation
            return dx[i][a] > delta2 and any(heavy_in[j] for j in range(k) if j != i)

        n_hw = 1
        Hs = []
        for i in range(k):
            H = [a for a in lists[i] if plus(i, a)]
            Hs.append(H)
            n_hw *= len(H)
        tot = 1
        for L in lists:
            tot *= len(L)
        J += tot
        J_H += n_hw
        J_L += tot - n_hw
        if sum(heavy_in) >= 2:
            hy += 1
        for t in itertools.product(*lists):
            if all(plus(i, t[i]) for i in range(k)):
                heavy.add(t)
            else:
                light.add(t)
    u = [sum(1 for a, d in dx[i].items() if d > delta2) for i in range(k)]
    return dict(J=J, J_L=J_L, J_H=J_H, u=u, v=hy, heavy=heavy, light=light)


def theory_thresholds(n: int, out: float):
    """Lemma 3 minimisers of f(D1,D2) = N + N D1 + OUT D2 + N^2/(D2 min(D1,D2)).

    Case OUT <= N: D1 = OUT^(1/3), D2 = N / OUT^(2/3).
    Case OUT > N:  D1 = D2 = (2 N^2 / (N + OUT))^(1/3).
    Real-valued (before rounding to integers).
    """
    if out <= n:
        return out ** (1.0 / 3.0), n / out ** (2.0 / 3.0)
    d = (2.0 * n * n / (n + out)) ** (1.0 / 3.0)
    return d, d


def idealized_cost(n: float, out: float, d1: float, d2: float) -> float:
    """The function f that Lemma 3 minimises (omega = 2)."""
    return n + n * d1 + out * d2 + n * n / (d2 * min(d1, d2))


def out_estimate(dom_x: int, dom_z: int, J: int, N: int) -> float:
    """Section 5 output-size estimate: geometric mean of the lower bound
    max(|dom x|, (J/N)^2) and the upper bound min(|dom x| |dom z|, J)."""
    lo = max(float(dom_x), (J / max(N, 1)) ** 2)
    hi = min(float(dom_x) * float(dom_z), float(J))
    lo = min(lo, hi)
    return math.sqrt(lo * hi)
