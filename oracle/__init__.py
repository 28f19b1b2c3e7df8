"""CPU oracle for the join-project queries.  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_2002_12459_amd``) and never imports it.

* ``two_path`` / ``star`` / ``join_size``: plain C (``oracle.c``), the query
  definitions of Section 2.1 evaluated as Proposition 1 says (full join, then
  project and deduplicate by sorting).
* ``ssj`` / ``bsi``: the set-similarity join (pairs with at least c common
  elements, with their overlap; plain or ordered by overlap) and Boolean set
  intersection (one answer per queried pair) of Section 2.1, by their
  definitions (full join and run lengths; a merge of the two sets per query).
* ``two_path_par`` / ``star_par``: the same computation split over OpenMP
  threads by ranges of the first output column (timed CPU baseline, and the
  check of full-size outputs).
* ``reference``: numpy restatements of the method's intermediate quantities
  (degrees, heavy/light partition, light witness count, heavy counts,
  thresholds), used to check the GPU path's statistics.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc (plain -O2)."""
    if force or not os.path.exists(_LIB_PATH):
        src = os.path.join(_HERE, "oracle.c")
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        i32p = ctypes.POINTER(ctypes.c_int32)
        lib.orc_join_size.restype = ctypes.c_int64
        lib.orc_join_size.argtypes = [i32p, i32p, ctypes.c_int64, i32p, i32p, ctypes.c_int64]
        lib.orc_two_path.restype = ctypes.c_int
        lib.orc_two_path.argtypes = [i32p, i32p, ctypes.c_int64, i32p, i32p, ctypes.c_int64,
                                     ctypes.POINTER(i32p), ctypes.POINTER(i32p),
                                     ctypes.POINTER(ctypes.c_int64)]
        lib.orc_star.restype = ctypes.c_int
        lib.orc_star.argtypes = [ctypes.c_int, ctypes.POINTER(i32p), ctypes.POINTER(i32p),
                                 ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(i32p),
                                 ctypes.POINTER(ctypes.c_int64)]
        lib.orc_two_path_par.restype = ctypes.c_int
        lib.orc_two_path_par.argtypes = [i32p, i32p, ctypes.c_int64, i32p, i32p, ctypes.c_int64, ctypes.c_int,
                                         ctypes.POINTER(i32p), ctypes.POINTER(i32p),
                                         ctypes.POINTER(ctypes.c_int64)]
        lib.orc_star_par.restype = ctypes.c_int
        lib.orc_star_par.argtypes = [ctypes.c_int, ctypes.POINTER(i32p), ctypes.POINTER(i32p),
                                     ctypes.POINTER(ctypes.c_int64), ctypes.c_int, ctypes.POINTER(i32p),
                                     ctypes.POINTER(ctypes.c_int64)]
        lib.orc_ssj.restype = ctypes.c_int
        lib.orc_ssj.argtypes = [i32p, i32p, ctypes.c_int64, i32p, i32p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                                ctypes.POINTER(i32p), ctypes.POINTER(i32p), ctypes.POINTER(i32p),
                                ctypes.POINTER(ctypes.c_int64)]
        lib.orc_bsi.restype = ctypes.c_int
        lib.orc_bsi.argtypes = [i32p, i32p, ctypes.c_int64, i32p, i32p, ctypes.c_int64, i32p, i32p,
                                ctypes.c_int64, ctypes.POINTER(ctypes.c_uint8)]
        lib.orc_free.restype = None
        lib.orc_free.argtypes = [ctypes.c_void_p]
        _lib = lib
    return _lib


def _col(a) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a), dtype=np.int32)
    return a


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def join_size(rx, ry, sz, sy) -> int:
    """Full join size J over distinct edges (Section 5, indexing pass)."""
    lib = _load()
    rx, ry, sz, sy = map(_col, (rx, ry, sz, sy))
    j = lib.orc_join_size(_ptr(rx), _ptr(ry), rx.size, _ptr(sz), _ptr(sy), sz.size)
    if j < 0:
        raise ValueError("orc_join_size failed")
    return int(j)


def cores() -> int:
    """Host threads this process may run on."""
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except (AttributeError, OSError):
        return max(1, os.cpu_count() or 1)


def two_path(rx, ry, sz, sy, threads: int = 0):
    """Distinct (x, z) of Q(x,z) = R(x,y), S(z,y), sorted by (x, z) signed.

    threads = 0: the plain single-thread oracle; threads >= 1: the OpenMP
    variant with that many threads."""
    lib = _load()
    rx, ry, sz, sy = map(_col, (rx, ry, sz, sy))
    if rx.size != ry.size or sz.size != sy.size:
        raise ValueError("column lengths differ")
    ox = ctypes.POINTER(ctypes.c_int32)()
    oz = ctypes.POINTER(ctypes.c_int32)()
    n = ctypes.c_int64(0)
    if threads:
        rc = lib.orc_two_path_par(_ptr(rx), _ptr(ry), rx.size, _ptr(sz), _ptr(sy), sz.size, int(threads),
                                  ctypes.byref(ox), ctypes.byref(oz), ctypes.byref(n))
    else:
        rc = lib.orc_two_path(_ptr(rx), _ptr(ry), rx.size, _ptr(sz), _ptr(sy), sz.size,
                              ctypes.byref(ox), ctypes.byref(oz), ctypes.byref(n))
    if rc != 0:
        raise MemoryError(f"orc_two_path failed ({rc})")
    try:
        m = n.value
        x = np.ctypeslib.as_array(ox, shape=(max(m, 1),))[:m].copy()
        z = np.ctypeslib.as_array(oz, shape=(max(m, 1),))[:m].copy()
    finally:
        lib.orc_free(ox)
        lib.orc_free(oz)
    return x, z


def two_path_par(rx, ry, sz, sy, threads: int | None = None):
    """``two_path`` on ``threads`` OpenMP threads (default: all cores)."""
    return two_path(rx, ry, sz, sy, threads=threads or cores())


def star_par(rels, threads: int | None = None):
    """``star`` on ``threads`` OpenMP threads (default: all cores)."""
    return star(rels, threads=threads or cores())


def star(rels, threads: int = 0):
    """Distinct tuples of the star query over ``rels = [(x_i, y_i), ...]``.

    Returns an int32 array of shape (n_out, k), rows sorted lexicographically.
    threads as for ``two_path``.
    """
    lib = _load()
    k = len(rels)
    if not 1 <= k <= 8:
        raise ValueError("k must be in [1, 8]")
    cols = [(_col(a), _col(b)) for a, b in rels]
    for a, b in cols:
        if a.size != b.size:
            raise ValueError("column lengths differ")
    P = ctypes.POINTER(ctypes.c_int32)
    xs = (P * k)(*[_ptr(a) for a, _ in cols])
    ys = (P * k)(*[_ptr(b) for _, b in cols])
    ns = (ctypes.c_int64 * k)(*[a.size for a, _ in cols])
    out = P()
    n = ctypes.c_int64(0)
    if threads:
        rc = lib.orc_star_par(k, xs, ys, ns, int(threads), ctypes.byref(out), ctypes.byref(n))
    else:
        rc = lib.orc_star(k, xs, ys, ns, ctypes.byref(out), ctypes.byref(n))
    if rc != 0:
        raise MemoryError(f"orc_star failed ({rc})")
    try:
        m = n.value
        t = np.ctypeslib.as_array(out, shape=(max(m, 1) * k,))[: m * k].copy()
    finally:
        lib.orc_free(out)
    return t.reshape(m, k)


def ssj(rx, ry, sz, sy, c: int = 1, order: int = 0):
    """Set similarity join: (x, z, overlap) int32 arrays of the pairs whose
    sets share at least ``c`` elements; order 0 by (x, z), order 1 by overlap
    descending then (x, z)."""
    lib = _load()
    rx, ry, sz, sy = map(_col, (rx, ry, sz, sy))
    if rx.size != ry.size or sz.size != sy.size:
        raise ValueError("column lengths differ")
    P = ctypes.POINTER(ctypes.c_int32)
    ox, oz, oc = P(), P(), P()
    n = ctypes.c_int64(0)
    rc = lib.orc_ssj(_ptr(rx), _ptr(ry), rx.size, _ptr(sz), _ptr(sy), sz.size, int(c), int(order),
                     ctypes.byref(ox), ctypes.byref(oz), ctypes.byref(oc), ctypes.byref(n))
    if rc != 0:
        raise (ValueError if rc == -1 else MemoryError)(f"orc_ssj failed ({rc})")
    try:
        m = n.value
        out = [np.ctypeslib.as_array(p, shape=(max(m, 1),))[:m].copy() for p in (ox, oz, oc)]
    finally:
        for p in (ox, oz, oc):
            lib.orc_free(p)
    return tuple(out)


def bsi(rx, ry, sz, sy, tx, tz):
    """Boolean set intersection: a bool array, True where the set of tx[i] in
    R and the set of tz[i] in S intersect."""
    lib = _load()
    rx, ry, sz, sy, tx, tz = map(_col, (rx, ry, sz, sy, tx, tz))
    if rx.size != ry.size or sz.size != sy.size or tx.size != tz.size:
        raise ValueError("column lengths differ")
    ans = np.zeros(max(tx.size, 1), dtype=np.uint8)
    rc = lib.orc_bsi(_ptr(rx), _ptr(ry), rx.size, _ptr(sz), _ptr(sy), sz.size, _ptr(tx), _ptr(tz), tx.size,
                     ans.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    if rc != 0:
        raise (ValueError if rc == -1 else MemoryError)(f"orc_bsi failed ({rc})")
    return ans[: tx.size].astype(bool)
