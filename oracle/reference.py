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
* Section 5: output-size estimate from |dom x| and the full join size, the
  degree indexes, and Algorithm 2's cost-based threshold search (the paper
  prints no numbers for it; tests/test_planner_cpu.py pins it to searches
  worked out by hand).
* A sampled output-size estimate (a selector input; not in the paper):
  draws of x values by the splitmix64 generator, exact distinct z per drawn
  x, scaled to all x.

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


def star_parts(rels, delta1, delta2):
    """The Section 3.2 partition of every relation of a star query.

    After dropping tuples whose y is missing from some relation (they join
    nothing), relation i is split as the paper defines it:
      R_i^-       tuples (a, b) whose a has degree <= delta2 in R_i;
      R_i^diamond tuples (a, b) whose b has degree <= delta1 in every OTHER
                  relation R_j, j != i (R_i's own y-degree is not consulted);
      R_i^+       R_i minus (R_i^- union R_i^diamond).
    R_i^- and R_i^diamond may overlap.  Returns (relations as lists of
    distinct (a, b) tuples, per-relation dicts of the three sets, x-degree
    and y-degree maps).
    """
    k = len(rels)
    R = [distinct_edges(a, b) for a, b in rels]
    common = R[0][1]
    for a, b in R[1:]:
        common = np.intersect1d(common, b)
    R = [(a[np.isin(b, common)], b[np.isin(b, common)]) for a, b in R]
    dx = [_deg(a) for a, _ in R]
    dy = [_deg(b) for _, b in R]
    tuples = [list(zip(a.tolist(), b.tolist())) for a, b in R]
    parts = []
    for i in range(k):
        minus = {(a, b) for a, b in tuples[i] if dx[i][a] <= delta2}
        diamond = {(a, b) for a, b in tuples[i] if all(dy[j][b] <= delta1 for j in range(k) if j != i)}
        plus = set(tuples[i]) - minus - diamond
        parts.append({"minus": minus, "diamond": diamond, "plus": plus})
    return tuples, parts, dx, dy


def star_stats(rels, delta1, delta2):
    """Witness classes of the star method of Section 3.2 at (delta1, delta2).

    A witness (a_1..a_k, b) of the full join goes to the matrix product when
    every (a_i, b) lies in R_i^+ (step 3); otherwise some tuple lies in R_i^-
    or R_i^diamond and steps 1-2 enumerate it.  Returns J, J_L, J_H, the
    heavy x counts u_i (x with degree > delta2), the number of y that carry a
    heavy witness, the distinct heavy and light output tuples, and the
    partition itself (see star_parts).
    """
    k = len(rels)
    tuples, parts, dx, dy = star_parts(rels, delta1, delta2)
    by = []
    for i in range(k):
        m = {}
        for a, b in tuples[i]:
            m.setdefault(b, []).append(a)
        by.append(m)
    J = J_L = J_H = 0
    heavy, light = set(), set()
    hy = 0
    for b in sorted(by[0]):
        lists = [by[i][b] for i in range(k)]
        n_hw = 1
        for i in range(k):
            n_hw *= sum(1 for a in lists[i] if (a, b) in parts[i]["plus"])
        tot = 1
        for L in lists:
            tot *= len(L)
        J += tot
        J_H += n_hw
        J_L += tot - n_hw
        if n_hw:
            hy += 1
        for t in itertools.product(*lists):
            if all((t[i], b) in parts[i]["plus"] for i in range(k)):
                heavy.add(t)
            else:
                light.add(t)
    u = [sum(1 for a, d in dx[i].items() if d > delta2) for i in range(k)]
    return dict(J=J, J_L=J_L, J_H=J_H, u=u, v=hy, heavy=heavy, light=light, parts=parts)


def theory_thresholds(n: int, out: float):
    """Lemma 3 minimisers of f(D1,D2) = N + N D1 + OUT D2 + N^2/(D2 min(D1,D2)).

    Case OUT <= N: D1 = OUT^(1/3), D2 = N / OUT^(2/3).
    Case OUT > N:  D1 = D2 = (2 N^2 / (N + OUT))^(1/3).
    Real-valued (before rounding to integers).
    Cube roots are the real cube root (np.cbrt), exact on perfect cubes, so
    that rounding down an exact cube gives the cube root itself.
    """
    if out <= n:
        c = float(np.cbrt(out))
        return c, n / (c * c)
    d = float(np.cbrt(2.0 * n * n / (n + out)))
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


# ---------------------------------------------------------------------------
# Algorithm 2 (Section 5): cost-based threshold search on degree indexes.
# ---------------------------------------------------------------------------

def degree_summary(rx, ry, sz, sy, y_rule=Y_RULE_MAX):
    """The Section 5 indexes of a two-path instance as sorted degree vectors.

    Returns a dict with sizes, J, the output estimate, and four indexes, each a
    tuple (deg, count, sum) of numpy arrays with ascending distinct degrees:
      y    key degree of y; sum = deg_R(y) * deg_S(y)  (sum(y_delta))
      x    deg_R(x); sum = witnesses of x              (sum(x_delta))
      xcdf per x the smallest key degree of its y      (cdfx(y_delta))
      z    deg_S(z)                                    (count(z_delta))
    """
    rx, ry, sz, sy = reduce_two_path(rx, ry, sz, sy)
    dRy, dSy = _deg(ry), _deg(sy)
    dRx, dSz = _deg(rx), _deg(sz)
    key = {b: (dRy[b] if y_rule == Y_RULE_R_ONLY else max(dRy[b], dSy[b])) for b in dRy}
    wx, mk = {}, {}
    for a, b in zip(rx.tolist(), ry.tolist()):
        wx[a] = wx.get(a, 0) + dSy[b]
        mk[a] = min(mk.get(a, 1 << 62), key[b])

    def index(degs, sums=None):
        d = np.array(sorted(set(degs.values())), dtype=np.int64)
        cnt = np.array([sum(1 for v in degs.values() if v == t) for t in d], dtype=np.int64)
        if sums is None:
            return d, cnt, None
        sm = np.array([float(sum(sums[k] for k, v in degs.items() if v == t)) for t in d])
        return d, cnt, sm

    J = sum(dRy[b] * dSy[b] for b in dRy)
    N = max(len(rx), len(sz))
    return dict(
        n_r=len(rx), n_s=len(sz), dom_x=len(dRx), dom_y=len(dRy), dom_z=len(dSz), J=int(J),
        out_est=out_estimate(len(dRx), len(dSz), int(J), N) if J else 0.0,
        y=index(key, {b: dRy[b] * dSy[b] for b in dRy}),
        x=index(dRx, wx),
        xcdf=index(mk),
        z=index(dSz),
    )


def _le(index, delta):
    """(count, sum) of the values with degree <= delta (binary search)."""
    d, cnt, sm = index
    p = int(np.searchsorted(d, delta, side="right"))
    c = int(cnt[:p].sum())
    s = float(sm[:p].sum()) if sm is not None else 0.0
    return c, s


def algorithm2(s, cal):
    """Cost-based optimizer of Section 5, in the paper's order.

    cal: dict with t_witness (T_I), t_seq (T_s), t_byte (T_m per byte), t_x
    (T_m per x value), eps, literal, and the product table mm_p / mm_s.
    Readings: N = max(|R|, |S|); Delta2 = floor(N Delta1 / OUT) clamped to
    [1, N] from the first step on; the start is Delta1 = N when literal, else
    the largest key degree; the search stops when the cost does not decrease
    (literal) or strictly increases; the light cost is
      T_I sum(y_D1) + T_I sum(x_D2) + T_m |dom x| + T_s cdfx(y_D1) |dom x|
    and the heavy cost M-hat(u,v,w) + T_m (u v + w v), M-hat taken from the
    nearest cube of the table scaled by u v w / p^3, or the smallest cube's
    time when p is below it, and v priced as the next multiple of k_pad when
    k_pad > 1 (missing k_pad: v itself); the result is the plain
    join when J <= 20 N or when no candidate beats it.  With light_once (a
    reading of Section 5's sum indexes as counts of work done once per light
    witness) the light-x term becomes sum(x_D2) (1 - sum(y_D1) / J): the
    witnesses of light x at light y, already counted in sum(y_D1), are taken
    out in the proportion they would have if x and y degree classes were
    independent, and a plan without a product is priced at all J witnesses
    (nothing leaves the light side).  A missing light_once means 0 (the
    printed sum).
    Returns (delta1, delta2, cost, cost_light_only); None stands for infinity.
    """
    N = max(s["n_r"], s["n_s"])
    out = max(s["out_est"], 1.0)

    kp = int(cal.get("k_pad", 1))

    def padded(v):  # the product's inner dimension as priced (k_pad > 1: next multiple)
        return -(-v // kp) * kp if kp > 1 else v

    def mm_hat(u, v, w):
        if min(u, v, w) <= 0:
            return 0.0
        p = (u * v * w) ** (1.0 / 3.0)
        j = int(np.argmin(cal["mm_p"]))
        if p <= cal["mm_p"][j]:  # below the smallest measured cube: its time
            return cal["mm_s"][j]
        i = int(np.argmin([abs(q - p) for q in cal["mm_p"]]))
        return cal["mm_s"][i] * (u * v * w) / cal["mm_p"][i] ** 3

    def cost(d1, d2):
        cy, sy_ = _le(s["y"], d1)
        cx, sx_ = _le(s["x"], d2)
        cc, _ = _le(s["xcdf"], d1)
        cz, _ = _le(s["z"], d2)
        u, v, w = s["dom_x"] - cx, s["dom_y"] - cy, s["dom_z"] - cz
        wit = sy_ + sx_
        if cal.get("light_once", 0) and s["J"] > 0:
            if u > 0 and v > 0 and w > 0:
                wit = sy_ + sx_ * max(0.0, 1.0 - sy_ / s["J"])
            else:  # no product: every witness stays light
                wit = float(s["J"])
        light = cal["t_witness"] * wit + cal["t_x"] * s["dom_x"] + cal["t_seq"] * cc * s["dom_x"]
        heavy = 0.0
        if u > 0 and v > 0 and w > 0:
            vp = padded(v)
            heavy = mm_hat(u, vp, w) + cal["t_byte"] * (u * vp + w * vp)
        return light + heavy

    big = 1 << 62
    light_only = cost(big, big)
    if s["J"] <= 20 * N or N <= 0:
        return None, None, light_only, light_only
    eps = 0.95 if cal["literal"] else cal["eps"]

    def d2_of(d1):
        t = N * d1 / out
        return 1 if t < 1 else (N if t >= N else int(math.floor(t)))

    d1 = max(N, 1) if cal["literal"] else max(int(s["y"][0][-1]), 1)
    d2 = d2_of(d1)
    prev = cost(d1, d2)
    for _ in range(10000):
        nd1 = int(math.floor((1 - eps) * d1))
        if nd1 >= d1:
            nd1 = d1 - 1
        if nd1 < 1:
            break
        nd2 = d2_of(nd1)
        c = cost(nd1, nd2)
        if (prev <= c) if cal["literal"] else (prev < c):
            break
        prev, d1, d2 = c, nd1, nd2
    if not prev < light_only:
        return None, None, light_only, light_only
    return d1, d2, prev, light_only


MASK64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """Steele, Lea and Flood's SplitMix64 output function applied to state
    x + 0x9e3779b97f4a7c15 (the generator's next value for state x)."""
    z = (x + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def sampled_out_estimate(rx, ry, sz, sy, seed: int, draws: int = 1024):
    """Sampled |OUT| estimate.  After set semantics and dangling-tuple
    removal (reduce_two_path), the distinct x values in ascending order are
    x_0 < ... < x_{n-1}; draw i (0 <= i < k, k = min(draws, n)) picks x of
    index splitmix64(seed + i) mod n (with replacement); D is the sum over
    the draws of |{c : exists b, (x, b) in R, (c, b) in S}|.  Returns
    (D, k, n) and the estimate D n / k."""
    rx, ry, sz, sy = reduce_two_path(rx, ry, sz, sy)
    xs = np.unique(rx)
    n = int(xs.size)
    if n == 0:
        return 0, 0, 0, 0.0
    k = min(int(draws), n)
    nbr = {}
    for a, b in zip(rx.tolist(), ry.tolist()):
        nbr.setdefault(a, []).append(b)
    zs_of_y = {}
    for c, b in zip(sz.tolist(), sy.tolist()):
        zs_of_y.setdefault(b, set()).add(c)
    D = 0
    for i in range(k):
        x = int(xs[splitmix64((seed + i) & MASK64) % n])
        reach = set()
        for b in nbr[x]:
            reach |= zs_of_y[b]
        D += len(reach)
    return D, k, n, D * n / k
