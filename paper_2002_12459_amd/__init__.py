"""MI355X (gfx950) join-project: Python binding of libjoinproject.

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch provides device memory and the current stream.  The
binding refuses to run when the native library is missing (no fallback).

    import paper_2002_12459_amd as jp
    x, z = jp.two_path(rx, ry, sz, sy)                # AUTO_COST thresholds
    x, z = jp.two_path(rx, ry, sz, sy, delta1=44, delta2=44)
    t = jp.star([(x1, y1), (x2, y2), (x3, y3)])       # tuple columns
"""
from __future__ import annotations

import ctypes
import os
import threading

__all__ = [
    "LIB_PATH", "JoinProjectError", "Handle", "Result", "two_path", "star", "bool_matmul",
    "default_handle", "STRATEGY", "BMM", "Y_RULE", "DEDUP", "DELTA_INF", "selector_cells", "mlp_param_count",
    "SELECTOR_PATH", "load_selector_file", "plan_theory", "estimate_out", "DeviceAllocator", "torch_allocator",
    "product_shape_class", "load_product_table", "PRODUCT_TABLE_PATH",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libjoinproject.so")
# Trained threshold-selector weights for MI355X (written by selector.py).
SELECTOR_PATH = os.path.join(_HERE, "selector_mi355x.json")
# Product kernel per shape class measured on MI355X (written by autotune.py).
PRODUCT_TABLE_PATH = os.path.join(_HERE, "autotune_mi355x.json")
N_FEATURES = 16
N_CELLS = 65

DELTA_INF = 2**63 - 1
STRATEGY = {"auto": 0, "cost": 0, "theory": 1, "fixed": 2, "light": 3, "mlp": 4}
BMM = {"auto": 0, "i8": 1, "bitpop": 2, "i8_t128": 3, "i8_t256": 4, "f16": 5}
Y_RULE = {"max": 0, "r_only": 1}
DEDUP = {"auto": 0, "global": 1, "segmented": 2}
STATUS = {0: "JP_OK", 1: "JP_EINVAL", 2: "JP_ENOMEM", 3: "JP_EHIP", 4: "JP_ECAPACITY",
          5: "JP_EPRECISION", 6: "JP_EINTERNAL"}
FLAG_TIMING = 1
FLAG_SAMPLED_OUT = 2


class JoinProjectError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("delta1", ctypes.c_int64), ("delta2", ctypes.c_int64), ("strategy", ctypes.c_int32),
                ("bmm", ctypes.c_int32), ("y_rule", ctypes.c_int32), ("dedup", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("flags", ctypes.c_uint64)]


class Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("n_r", "n_s", "dom_x", "dom_y", "dom_z", "delta1", "delta2")] + \
               [(n, ctypes.c_int32) for n in ("strategy", "bmm", "dedup", "arity")] + \
               [(n, ctypes.c_int64) for n in ("u", "v", "w", "J", "J_L", "J_H", "nnz_heavy", "n_out")] + \
               [(n, ctypes.c_double) for n in ("bmm_ops", "ms_ingest", "ms_plan", "ms_light", "ms_heavy",
                                               "ms_bmm", "ms_dedup", "ms_total", "ms_kernel_dedup",
                                               "dedup_alg_bytes")] + \
               [("dedup_units", ctypes.c_int64), ("out_est", ctypes.c_double), ("out_sampled", ctypes.c_double),
                ("sample_draws", ctypes.c_int64), ("sample_distinct", ctypes.c_int64)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class Calibration(ctypes.Structure):
    _fields_ = [("t_witness", ctypes.c_double), ("t_seq", ctypes.c_double), ("t_byte", ctypes.c_double),
                ("t_x", ctypes.c_double), ("eps", ctypes.c_double), ("literal", ctypes.c_int32),
                ("n_mm", ctypes.c_int32), ("mm_p", ctypes.c_double * 24), ("mm_s", ctypes.c_double * 24),
                ("light_once", ctypes.c_int32), ("k_pad", ctypes.c_int32)]

    def as_dict(self):
        return {"t_witness": self.t_witness, "t_seq": self.t_seq, "t_byte": self.t_byte, "t_x": self.t_x,
                "eps": self.eps, "literal": self.literal, "mm_p": list(self.mm_p[: self.n_mm]),
                "mm_s": list(self.mm_s[: self.n_mm]), "light_once": self.light_once, "k_pad": self.k_pad}

    @classmethod
    def from_dict(cls, d):
        c = cls()
        for k in ("t_witness", "t_seq", "t_byte", "t_x", "eps"):
            setattr(c, k, float(d[k]))
        c.literal = int(d.get("literal", 0))
        c.light_once = int(d.get("light_once", 0))
        c.k_pad = int(d.get("k_pad", 1))
        c.n_mm = len(d["mm_p"])
        for i, (a, b) in enumerate(zip(d["mm_p"], d["mm_s"])):
            c.mm_p[i] = a
            c.mm_s[i] = b
        return c


class DegreeIndex(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("deg", ctypes.c_void_p), ("count", ctypes.c_void_p), ("sum", ctypes.c_void_p)]


class TwoPathSummary(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("n_r", "n_s", "dom_x", "dom_y", "dom_z", "J")] + \
               [("out_est", ctypes.c_double)] + [(n, DegreeIndex) for n in ("y", "x", "xcdf", "z")]


class Instance(ctypes.Structure):
    _fields_ = [("r_x", ctypes.c_void_p), ("r_y", ctypes.c_void_p), ("n_r", ctypes.c_int64),
                ("s_z", ctypes.c_void_p), ("s_y", ctypes.c_void_p), ("n_s", ctypes.c_int64)]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

_lib = None
_lock = threading.Lock()


def _load():
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2002_12459_amd.build.build()")
        # torch first: it brings its own HIP runtime, and a process that has
        # loaded the system one before it finds no GPU through torch
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.jp_create.argtypes = [ctypes.POINTER(P), ctypes.c_int]
        lib.jp_destroy.argtypes = [P]
        lib.jp_destroy.restype = None
        lib.jp_set_stream.argtypes = [P, P]
        lib.jp_set_allocator.argtypes = [P, _ALLOC_FN, _FREE_FN, P]
        lib.jp_last_error.argtypes = [P]
        lib.jp_last_error.restype = ctypes.c_char_p
        lib.jp_default_options.argtypes = [ctypes.POINTER(Options)]
        lib.jp_default_options.restype = None
        lib.jp_two_path.argtypes = [P, P, P, i64, P, P, i64, ctypes.POINTER(Options), ctypes.POINTER(P)]
        lib.jp_two_path_static.argtypes = [P, P, P, i64, P, P, i64, ctypes.POINTER(Options), P, P, i64,
                                           ctypes.POINTER(i64), ctypes.POINTER(Stats)]
        lib.jp_ssj.argtypes = [P, P, P, i64, P, P, i64, i64, ctypes.c_int32, ctypes.POINTER(Options),
                               ctypes.POINTER(P)]
        lib.jp_bsi.argtypes = [P, P, P, i64, P, P, i64, P, P, i64, ctypes.POINTER(Options), P,
                               ctypes.POINTER(Stats)]
        lib.jp_two_path_batch_plan.argtypes = [P, ctypes.c_int32, ctypes.POINTER(Instance), ctypes.POINTER(Options),
                                               P, i64, ctypes.POINTER(P), ctypes.POINTER(i64)]
        lib.jp_plan_launch.argtypes = [P, P]
        lib.jp_plan_result.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(i64), ctypes.POINTER(i64)]
        lib.jp_plan_copy.argtypes = [P, P, ctypes.POINTER(P)]
        lib.jp_plan_free.argtypes = [P]
        lib.jp_plan_free.restype = None
        lib.jp_product_shape_class.argtypes = [i64, i64, i64]
        lib.jp_product_shape_class.restype = ctypes.c_uint64
        lib.jp_set_product_table.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64),
                                             ctypes.POINTER(ctypes.c_int32)]
        lib.jp_star.argtypes = [P, ctypes.c_int, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(i64),
                                ctypes.POINTER(Options), ctypes.POINTER(P)]
        lib.jp_result_size.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_int32)]
        lib.jp_result_columns.argtypes = [P, ctypes.POINTER(P)]
        lib.jp_result_copy.argtypes = [P, P, ctypes.POINTER(P)]
        lib.jp_result_stats.argtypes = [P, ctypes.POINTER(Stats)]
        lib.jp_result_free.argtypes = [P]
        lib.jp_result_free.restype = None
        lib.jp_bool_matmul.argtypes = [P, P, P, i64, i64, i64, i64, ctypes.c_int32, P, P, i64,
                                       ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double)]
        lib.jp_default_calibration.argtypes = [ctypes.POINTER(Calibration)]
        lib.jp_default_calibration.restype = None
        lib.jp_set_calibration.argtypes = [P, ctypes.POINTER(Calibration)]
        lib.jp_get_calibration.argtypes = [P, ctypes.POINTER(Calibration)]
        lib.jp_plan_summary.argtypes = [ctypes.POINTER(TwoPathSummary), ctypes.POINTER(Calibration),
                                        ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double)]
        lib.jp_plan_two_path.argtypes = [P, P, P, i64, P, P, i64, ctypes.POINTER(Options), ctypes.POINTER(i64),
                                         ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_float)]
        lib.jp_plan_theory.argtypes = [i64, ctypes.c_double, ctypes.POINTER(i64), ctypes.POINTER(i64)]
        lib.jp_estimate_out.argtypes = [i64, i64, i64, i64]
        lib.jp_estimate_out.restype = ctypes.c_double
        lib.jp_two_path_batch.argtypes = [P, ctypes.c_int32, ctypes.POINTER(Instance), ctypes.POINTER(Options),
                                          ctypes.POINTER(P)]
        lib.jp_result_batch_offsets.argtypes = [P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(i64)]
        lib.jp_plan_cells.argtypes = [P, P, P, i64, P, P, i64, ctypes.POINTER(Options), ctypes.c_int32,
                                      ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(i64)]
        lib.jp_selector_cells.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.POINTER(i64), ctypes.POINTER(i64)]
        lib.jp_heavy_cost.argtypes = [ctypes.POINTER(Calibration), i64, i64, i64]
        lib.jp_heavy_cost.restype = ctypes.c_double
        lib.jp_selector_cells.restype = ctypes.c_int32
        lib.jp_mlp_param_count.argtypes = [ctypes.c_int32]
        lib.jp_mlp_param_count.restype = i64
        lib.jp_set_selector.argtypes = [P, ctypes.POINTER(ctypes.c_float), ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]
        lib.jp_mlp_forward.argtypes = [P, P, ctypes.c_int32, P, i64, P]
        lib.jp_mlp_grad.argtypes = [P, P, ctypes.c_int32, P, P, P, i64, P, P]
        f32 = ctypes.c_float
        lib.jp_mlp_adam.argtypes = [P, P, P, P, P, i64, ctypes.c_int32, f32, f32, f32, f32]
        for f in ("jp_create", "jp_set_stream", "jp_set_allocator", "jp_two_path", "jp_two_path_static", "jp_ssj", "jp_bsi", "jp_two_path_batch_plan",
                  "jp_plan_launch", "jp_plan_result", "jp_plan_copy", "jp_set_product_table", "jp_star", "jp_result_size",
                  "jp_result_columns", "jp_result_copy", "jp_result_stats", "jp_bool_matmul",
                  "jp_set_calibration", "jp_get_calibration", "jp_plan_summary", "jp_plan_two_path",
                  "jp_plan_cells", "jp_set_selector", "jp_mlp_forward", "jp_mlp_grad", "jp_mlp_adam",
                  "jp_two_path_batch", "jp_result_batch_offsets", "jp_plan_theory"):
            getattr(lib, f).restype = ctypes.c_int
        _lib = lib
    return _lib


def _torch():
    import torch
    return torch


def _col(t, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != torch.int32:
        raise TypeError(f"{name} must be int32")
    if t.dim() != 1 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous 1-D tensor")
    return t


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr() if t.numel() else 0)


class Result:
    """A library-owned result; columns stay valid until ``free()``."""

    def __init__(self, handle, ptr):
        self._h = handle
        self._p = ptr
        lib = _load()
        n = ctypes.c_int64()
        a = ctypes.c_int32()
        lib.jp_result_size(ptr, ctypes.byref(n), ctypes.byref(a))
        self.n = n.value
        self.arity = a.value
        s = Stats()
        lib.jp_result_stats(ptr, ctypes.byref(s))
        self.stats = s.as_dict()

    def batch_offsets(self):
        """Instance slices of a batched result (list of n_inst + 1 ints), or None."""
        lib = _load()
        n = ctypes.c_int32()
        lib.jp_result_batch_offsets(self._p, ctypes.byref(n), None)
        if n.value == 0:
            return None
        offs = (ctypes.c_int64 * (n.value + 1))()
        lib.jp_result_batch_offsets(self._p, ctypes.byref(n), offs)
        return list(offs)

    def to_torch(self):
        """Copy the columns into new int32 torch tensors (stream-ordered)."""
        torch = _torch()
        dev = torch.device("cuda", self._h.device)
        cols = [torch.empty(self.n, dtype=torch.int32, device=dev) for _ in range(self.arity)]
        if self.n:
            arr = (ctypes.c_void_p * self.arity)(*[c.data_ptr() for c in cols])
            self._h._check(_load().jp_result_copy(self._h._p, self._p, arr))
        return cols

    def free(self):
        if self._p:
            _load().jp_result_free(self._p)
            self._p = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Plan:
    """A graph-captured batched evaluation; ``launch()`` replays it."""

    def __init__(self, handle, ptr, n_inst, keep, arena, arena_needed):
        self._h, self._p, self.n_inst = handle, ptr, n_inst
        self._keep, self._arena = keep, arena  # the graph reads these columns / this arena
        self.arena_needed = arena_needed

    def launch(self):
        self._h._bind_stream()
        self._h._check(_load().jp_plan_launch(self._h._p, self._p))

    def outputs(self):
        """[(x, z), ...] per instance: copies of the plan's output columns."""
        torch = _torch()
        n = ctypes.c_int64()
        offs = (ctypes.c_int64 * (self.n_inst + 1))()
        self._h._check(_load().jp_plan_result(self._p, None, ctypes.byref(n), offs))
        dev = torch.device("cuda", self._h.device)
        x = torch.empty(n.value, dtype=torch.int32, device=dev)
        z = torch.empty(n.value, dtype=torch.int32, device=dev)
        if n.value:
            self._h._bind_stream()
            arr = (ctypes.c_void_p * 2)(x.data_ptr(), z.data_ptr())
            self._h._check(_load().jp_plan_copy(self._h._p, self._p, arr))
        return [(x[offs[i]:offs[i + 1]], z[offs[i]:offs[i + 1]]) for i in range(self.n_inst)]

    def free(self):
        if self._p:
            _load().jp_plan_free(self._p)
            self._p = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _f32(t, name, n=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float32 CUDA tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must hold {n} values")
    return t


def product_shape_class(u, w, ld):
    """Shape class of a u x ld by w x ld product (JP_BMM_AUTO's table key)."""
    return int(_load().jp_product_shape_class(int(u), int(w), int(ld)))


def load_product_table(path=PRODUCT_TABLE_PATH):
    """{shape class: kind name} of an autotune file (JSON)."""
    import json
    with open(path) as fh:
        d = json.load(fh)
    return {int(e["class"]): e["kind"] for e in d["entries"]}


def load_selector_file(path=SELECTOR_PATH):
    """(params, mean, scale) lists of a selector weight file (JSON)."""
    import json
    with open(path) as fh:
        d = json.load(fh)
    return d["params"], d["mean"], d["scale"]


class DeviceAllocator:
    """Allocation callbacks handed to ``jp_set_allocator``.

    ``alloc(nbytes) -> int`` returns a device address (0 when out of memory)
    and ``free(ptr)`` takes it back.  The wrapper counts live bytes, the peak
    and the calls, and turns a Python exception in ``alloc`` into NULL (the
    library then reports JP_ENOMEM)."""

    def __init__(self, alloc, free):
        self._alloc, self._free = alloc, free
        self.live = {}
        self.live_bytes = self.peak_bytes = self.n_alloc = self.n_free = 0

        def a(nbytes, _user):
            try:
                ptr = int(self._alloc(int(nbytes)) or 0)
            except Exception:
                ptr = 0
            if ptr:
                self.live[ptr] = int(nbytes)
                self.live_bytes += int(nbytes)
                self.peak_bytes = max(self.peak_bytes, self.live_bytes)
                self.n_alloc += 1
            return ptr or None

        def f(ptr, _user):
            if not ptr:
                return
            self.live_bytes -= self.live.pop(ptr, 0)
            self.n_free += 1
            try:
                self._free(ptr)
            except Exception:
                pass

        self.c_alloc = _ALLOC_FN(a)
        self.c_free = _FREE_FN(f)


def torch_allocator(device: int) -> DeviceAllocator:
    """PyTorch's caching allocator, on torch's current stream of ``device``."""
    torch = _torch()

    def alloc(nbytes):
        return torch.cuda.caching_allocator_alloc(nbytes, device, torch.cuda.current_stream(device))

    return DeviceAllocator(alloc, torch.cuda.caching_allocator_delete)


class Handle:
    """One library handle per device; work goes to torch's current stream.

    ``selector="default"`` installs the packaged MI355X selector weights when
    the file exists (used by strategy "mlp"); None leaves the handle without
    a selector, so "mlp" behaves as "auto".  ``allocator``: "torch"
    (PyTorch's caching allocator: the library and torch share one pool of
    device memory), "builtin" (the library's own caching pool, which saves
    the Python callback of each of the 60 to 90 buffers of an evaluation) or
    a ``DeviceAllocator``.  ``product_table="default"`` installs the packaged
    autotuned product kernel table (autotune.py) when the file exists; a
    dict {shape class: kind name} installs that one; None none."""

    def __init__(self, device: int = 0, selector="default", allocator="torch", product_table="default"):
        lib = _load()
        self.device = device
        self.allocator = None
        p = ctypes.c_void_p()
        st = lib.jp_create(ctypes.byref(p), device)
        if st != 0:
            raise JoinProjectError(st, f"jp_create({device}) failed")
        self._p = p
        if allocator != "builtin":
            self.set_allocator(torch_allocator(device) if allocator == "torch" else allocator)
        if product_table == "default":
            if os.path.exists(PRODUCT_TABLE_PATH):
                self.set_product_table(load_product_table(PRODUCT_TABLE_PATH))
        elif product_table is not None:
            self.set_product_table(product_table)
        if selector == "default":
            if os.path.exists(SELECTOR_PATH):
                self.set_selector(*load_selector_file(SELECTOR_PATH))
        elif selector is not None:
            self.set_selector(*selector)

    def _check(self, st):
        if st != 0:
            raise JoinProjectError(st, _load().jp_last_error(self._p).decode())

    def set_allocator(self, allocator):
        """Route the handle's device memory through ``allocator`` (a
        DeviceAllocator), or back to the built-in pool with None."""
        lib = _load()
        if allocator is None:
            self._check(lib.jp_set_allocator(self._p, _ALLOC_FN(), _FREE_FN(), None))
        else:
            self._check(lib.jp_set_allocator(self._p, allocator.c_alloc, allocator.c_free, None))
        # results made with the previous allocator hold this handle, and the
        # handle holds every allocator it used, so callbacks outlive them
        self._old_allocators = getattr(self, "_old_allocators", []) + [self.allocator]
        self.allocator = allocator

    def _bind_stream(self):
        torch = _torch()
        s = torch.cuda.current_stream(self.device)
        self._check(_load().jp_set_stream(self._p, ctypes.c_void_p(s.cuda_stream)))

    def _options(self, delta1, delta2, strategy, bmm, y_rule, dedup, timing, seed, sampled_out=False):
        o = Options()
        _load().jp_default_options(ctypes.byref(o))
        if delta1 is not None or delta2 is not None or strategy == "fixed":
            if strategy in (None, "auto"):
                strategy = "fixed"
            o.delta1 = DELTA_INF if delta1 is None else int(delta1)
            o.delta2 = DELTA_INF if delta2 is None else int(delta2)
        if strategy is not None:
            o.strategy = STRATEGY[strategy]
        o.bmm = BMM[bmm]
        o.y_rule = Y_RULE[y_rule]
        o.dedup = DEDUP[dedup]
        if seed is not None:
            o.seed = seed
        o.flags = (FLAG_TIMING if timing else 0) | (FLAG_SAMPLED_OUT if sampled_out else 0)
        return o

    def two_path_result(self, rx, ry, sz, sy, delta1=None, delta2=None, strategy=None, bmm="auto",
                        y_rule="max", dedup="auto", timing=False, seed=None, sampled_out=False) -> Result:
        rx, ry, sz, sy = (_col(t, n) for t, n in ((rx, "r_x"), (ry, "r_y"), (sz, "s_z"), (sy, "s_y")))
        if rx.numel() != ry.numel() or sz.numel() != sy.numel():
            raise ValueError("column lengths differ")
        self._bind_stream()
        o = self._options(delta1, delta2, strategy, bmm, y_rule, dedup, timing, seed, sampled_out)
        out = ctypes.c_void_p()
        self._check(_load().jp_two_path(self._p, _ptr(rx), _ptr(ry), rx.numel(), _ptr(sz), _ptr(sy), sz.numel(),
                                        ctypes.byref(o), ctypes.byref(out)))
        return Result(self, out)

    def two_path(self, rx, ry, sz, sy, **kw):
        r = self.two_path_result(rx, ry, sz, sy, **kw)
        try:
            x, z = r.to_torch()
            return x, z, r.stats
        finally:
            r.free()

    def two_path_static(self, rx, ry, sz, sy, out_x, out_z, delta1=None, delta2=None, strategy=None, bmm="auto",
                        y_rule="max", dedup="auto", seed=None):
        """jp_two_path_static: the pairs go into the caller's int32 CUDA
        tensors out_x / out_z (capacity = their length) and the library
        allocates no device memory.  Returns (n_out, stats); raises
        JoinProjectError (JP_ECAPACITY with .n_out set when they are too short)."""
        rx, ry, sz, sy, out_x, out_z = (_col(t, n) for t, n in ((rx, "r_x"), (ry, "r_y"), (sz, "s_z"), (sy, "s_y"),
                                                                 (out_x, "out_x"), (out_z, "out_z")))
        if rx.numel() != ry.numel() or sz.numel() != sy.numel() or out_x.numel() != out_z.numel():
            raise ValueError("column lengths differ")
        self._bind_stream()
        o = self._options(delta1, delta2, strategy, bmm, y_rule, dedup, False, seed)
        n = ctypes.c_int64()
        s = Stats()
        st = _load().jp_two_path_static(self._p, _ptr(rx), _ptr(ry), rx.numel(), _ptr(sz), _ptr(sy), sz.numel(),
                                        ctypes.byref(o), _ptr(out_x), _ptr(out_z), out_x.numel(), ctypes.byref(n),
                                        ctypes.byref(s))
        if st != 0:
            err = JoinProjectError(st, _load().jp_last_error(self._p).decode())
            err.n_out = n.value
            raise err
        return n.value, s.as_dict()

    def ssj_result(self, rx, ry, sz, sy, min_overlap=1, ordered=False, delta1=None, delta2=None, strategy=None,
                   bmm="auto", y_rule="max", timing=False, seed=None) -> Result:
        """Set similarity join: pairs whose sets share >= min_overlap elements."""
        rx, ry, sz, sy = (_col(t, n) for t, n in ((rx, "r_x"), (ry, "r_y"), (sz, "s_z"), (sy, "s_y")))
        if rx.numel() != ry.numel() or sz.numel() != sy.numel():
            raise ValueError("column lengths differ")
        self._bind_stream()
        o = self._options(delta1, delta2, strategy, bmm, y_rule, "global", timing, seed)
        out = ctypes.c_void_p()
        self._check(_load().jp_ssj(self._p, _ptr(rx), _ptr(ry), rx.numel(), _ptr(sz), _ptr(sy), sz.numel(),
                                   int(min_overlap), 1 if ordered else 0, ctypes.byref(o), ctypes.byref(out)))
        return Result(self, out)

    def ssj(self, rx, ry, sz, sy, **kw):
        """(x, z, overlap, stats): int32 tensors of the pairs and their overlaps."""
        r = self.ssj_result(rx, ry, sz, sy, **kw)
        try:
            x, z, cnt = r.to_torch()
            return x, z, cnt, r.stats
        finally:
            r.free()

    def bsi(self, rx, ry, sz, sy, tx, tz, delta1=None, delta2=None, strategy=None, bmm="auto", y_rule="max",
            dedup="auto", timing=False, seed=None):
        """Batched Boolean set intersection: (answers, stats), answers a uint8
        CUDA tensor with answers[i] = 1 iff the set of tx[i] in R and the set
        of tz[i] in S intersect."""
        torch = _torch()
        rx, ry, sz, sy, tx, tz = (_col(t, n) for t, n in ((rx, "r_x"), (ry, "r_y"), (sz, "s_z"), (sy, "s_y"),
                                                          (tx, "t_x"), (tz, "t_z")))
        if rx.numel() != ry.numel() or sz.numel() != sy.numel() or tx.numel() != tz.numel():
            raise ValueError("column lengths differ")
        self._bind_stream()
        o = self._options(delta1, delta2, strategy, bmm, y_rule, dedup, timing, seed)
        ans = torch.empty(tx.numel(), dtype=torch.uint8, device=tx.device)
        s = Stats()
        self._check(_load().jp_bsi(self._p, _ptr(rx), _ptr(ry), rx.numel(), _ptr(sz), _ptr(sy), sz.numel(), _ptr(tx),
                                   _ptr(tz), tx.numel(), ctypes.byref(o), _ptr(ans), ctypes.byref(s)))
        return ans, s.as_dict()

    def two_path_batch_result(self, instances, delta1=None, delta2=None, strategy=None, bmm="auto", y_rule="max",
                              dedup="auto", timing=False, seed=None) -> Result:
        """All instances [(r_x, r_y, s_z, s_y), ...] in one evaluation."""
        descs = (Instance * max(len(instances), 1))()
        keep = []
        for i, (rx, ry, sz, sy) in enumerate(instances):
            rx, ry, sz, sy = (_col(t, n) for t, n in ((rx, "r_x"), (ry, "r_y"), (sz, "s_z"), (sy, "s_y")))
            if rx.numel() != ry.numel() or sz.numel() != sy.numel():
                raise ValueError(f"instance {i}: column lengths differ")
            keep.extend([rx, ry, sz, sy])
            descs[i] = Instance(_ptr(rx), _ptr(ry), rx.numel(), _ptr(sz), _ptr(sy), sz.numel())
        self._bind_stream()
        o = self._options(delta1, delta2, strategy, bmm, y_rule, dedup, timing, seed)
        out = ctypes.c_void_p()
        self._check(_load().jp_two_path_batch(self._p, len(instances), descs, ctypes.byref(o), ctypes.byref(out)))
        return Result(self, out)

    def batch_plan(self, instances, arena_bytes=0, arena=None, delta1=None, delta2=None, strategy=None,
                   bmm="auto", y_rule="max", dedup="auto", seed=None):
        """A graph-captured plan of the batch (see jp_two_path_batch_plan).
        arena: an optional uint8 CUDA tensor used as the plan's arena.
        Raises JoinProjectError with .arena_needed set on JP_ECAPACITY."""
        descs = (Instance * max(len(instances), 1))()
        keep = []
        for i, (rx, ry, sz, sy) in enumerate(instances):
            rx, ry, sz, sy = (_col(t, n) for t, n in ((rx, "r_x"), (ry, "r_y"), (sz, "s_z"), (sy, "s_y")))
            if rx.numel() != ry.numel() or sz.numel() != sy.numel():
                raise ValueError(f"instance {i}: column lengths differ")
            keep.extend([rx, ry, sz, sy])
            descs[i] = Instance(_ptr(rx), _ptr(ry), rx.numel(), _ptr(sz), _ptr(sy), sz.numel())
        if arena is not None:
            arena_bytes = arena.numel() * arena.element_size()
        self._bind_stream()
        o = self._options(delta1, delta2, strategy, bmm, y_rule, dedup, False, seed)
        p = ctypes.c_void_p()
        need = ctypes.c_int64()
        st = _load().jp_two_path_batch_plan(self._p, len(instances), descs, ctypes.byref(o),
                                            _ptr(arena) if arena is not None else None, int(arena_bytes),
                                            ctypes.byref(p), ctypes.byref(need))
        if st != 0:
            err = JoinProjectError(st, _load().jp_last_error(self._p).decode())
            err.arena_needed = need.value
            raise err
        return Plan(self, p, len(instances), keep, arena, need.value)

    def two_path_batch(self, instances, **kw):
        """Per-instance outputs [(x, z), ...] (views of two shared tensors) and the stats."""
        r = self.two_path_batch_result(instances, **kw)
        try:
            x, z = r.to_torch()
            offs = r.batch_offsets() or [0] * (len(instances) + 1)
            return [(x[offs[i]:offs[i + 1]], z[offs[i]:offs[i + 1]]) for i in range(len(instances))], r.stats
        finally:
            r.free()

    def star_result(self, rels, delta1=None, delta2=None, strategy=None, bmm="auto", dedup="auto",
                    timing=False, seed=None) -> Result:
        k = len(rels)
        cols = [(_col(a, f"x{i}"), _col(b, f"y{i}")) for i, (a, b) in enumerate(rels)]
        for a, b in cols:
            if a.numel() != b.numel():
                raise ValueError("column lengths differ")
        self._bind_stream()
        o = self._options(delta1, delta2, strategy, bmm, "max", dedup, timing, seed)
        xs = (ctypes.c_void_p * k)(*[_ptr(a) for a, _ in cols])
        ys = (ctypes.c_void_p * k)(*[_ptr(b) for _, b in cols])
        ns = (ctypes.c_int64 * k)(*[a.numel() for a, _ in cols])
        out = ctypes.c_void_p()
        self._check(_load().jp_star(self._p, k, xs, ys, ns, ctypes.byref(o), ctypes.byref(out)))
        return Result(self, out)

    def star(self, rels, **kw):
        r = self.star_result(rels, **kw)
        try:
            return r.to_torch(), r.stats
        finally:
            r.free()

    def bool_matmul(self, A, Bt, k=None, kind="i8", cap=None):
        """Nonzero coordinates of A @ Bt.T for 0/1 int8 device matrices (rows
        padded to a multiple of 128 bytes).  Returns (rows, cols, ms)."""
        torch = _torch()
        if A.dtype != torch.int8 or Bt.dtype != torch.int8 or not (A.is_cuda and Bt.is_cuda):
            raise TypeError("A and Bt must be int8 CUDA tensors")
        if A.dim() != 2 or Bt.dim() != 2 or A.shape[1] != Bt.shape[1]:
            raise ValueError("A and Bt must be 2-D with equal row length")
        A = A.contiguous()
        Bt = Bt.contiguous()
        u, ld = A.shape
        w = Bt.shape[0]
        k = ld if k is None else k
        if cap is None:
            cap = u * w
        self._bind_stream()
        rows = torch.empty(max(cap, 1), dtype=torch.int32, device=A.device)
        cols = torch.empty(max(cap, 1), dtype=torch.int32, device=A.device)
        nnz = ctypes.c_int64()
        ms = ctypes.c_double()
        self._check(_load().jp_bool_matmul(self._p, _ptr(A), _ptr(Bt), u, w, k, ld, BMM[kind], _ptr(rows),
                                           _ptr(cols), cap, ctypes.byref(nnz), ctypes.byref(ms)))
        return rows[: nnz.value], cols[: nnz.value], ms.value

    def bool_matmul_count(self, A, Bt, k=None, kind="i8"):
        """Number of nonzero entries of A @ Bt.T (nothing is stored) and the
        kernel's device time in ms."""
        torch = _torch()
        if A.dtype != torch.int8 or Bt.dtype != torch.int8 or not (A.is_cuda and Bt.is_cuda):
            raise TypeError("A and Bt must be int8 CUDA tensors")
        A = A.contiguous()
        Bt = Bt.contiguous()
        u, ld = A.shape
        w = Bt.shape[0]
        k = ld if k is None else k
        self._bind_stream()
        nnz = ctypes.c_int64()
        ms = ctypes.c_double()
        st = _load().jp_bool_matmul(self._p, _ptr(A), _ptr(Bt), u, w, k, ld, BMM[kind], None, None, 0,
                                    ctypes.byref(nnz), ctypes.byref(ms))
        if st not in (0, 4):  # JP_ECAPACITY reports the count
            self._check(st)
        return nnz.value, ms.value

    def set_product_table(self, table):
        """Product kernel per shape class: {class (int): "i8_t128" | "i8_t256" | "bitpop"}."""
        items = list(table.items())
        cls = (ctypes.c_uint64 * max(len(items), 1))(*[int(k) for k, _ in items])
        kinds = (ctypes.c_int32 * max(len(items), 1))(*[BMM[v] for _, v in items])
        self._check(_load().jp_set_product_table(self._p, len(items), cls, kinds))

    def set_calibration(self, cal):
        c = cal if isinstance(cal, Calibration) else Calibration.from_dict(cal)
        self._check(_load().jp_set_calibration(self._p, ctypes.byref(c)))

    def get_calibration(self):
        c = Calibration()
        self._check(_load().jp_get_calibration(self._p, ctypes.byref(c)))
        return c.as_dict()

    def plan_two_path(self, rx, ry, sz, sy, strategy="auto", y_rule="max", seed=None):
        """Thresholds the optimizer picks (None = infinity) and the 16 selector features."""
        rx, ry, sz, sy = (_col(t, n) for t, n in ((rx, "r_x"), (ry, "r_y"), (sz, "s_z"), (sy, "s_y")))
        self._bind_stream()
        o = self._options(None, None, strategy, "auto", y_rule, "auto", False, seed)
        d1, d2 = ctypes.c_int64(), ctypes.c_int64()
        f = (ctypes.c_float * 16)()
        self._check(_load().jp_plan_two_path(self._p, _ptr(rx), _ptr(ry), rx.numel(), _ptr(sz), _ptr(sy),
                                             sz.numel(), ctypes.byref(o), ctypes.byref(d1), ctypes.byref(d2), f))
        inf = lambda v: None if v == DELTA_INF else v
        return inf(d1.value), inf(d2.value), list(f)

    def plan_cells(self, rx, ry, sz, sy, delta1, delta2, y_rule="max"):
        """Cost-model seconds and heavy (u, v, w) of each threshold pair
        (None = infinity) on one instance."""
        rx, ry, sz, sy = (_col(t, n) for t, n in ((rx, "r_x"), (ry, "r_y"), (sz, "s_z"), (sy, "s_y")))
        n = len(delta1)
        if len(delta2) != n:
            raise ValueError("delta1 and delta2 differ in length")
        self._bind_stream()
        o = self._options(None, None, "auto", "auto", y_rule, "auto", False, None)
        conv = lambda v: DELTA_INF if v is None else int(v)
        a = (ctypes.c_int64 * max(n, 1))(*[conv(v) for v in delta1])
        b = (ctypes.c_int64 * max(n, 1))(*[conv(v) for v in delta2])
        est = (ctypes.c_double * max(n, 1))()
        dims = (ctypes.c_int64 * max(3 * n, 1))()
        self._check(_load().jp_plan_cells(self._p, _ptr(rx), _ptr(ry), rx.numel(), _ptr(sz), _ptr(sy), sz.numel(),
                                          ctypes.byref(o), n, a, b, est, dims))
        return list(est[:n]), [tuple(dims[3 * i: 3 * i + 3]) for i in range(n)]

    def set_selector(self, params, mean, scale):
        """Install selector weights (sequences of floats: parameters, 16 feature
        means, 16 feature scales)."""
        npar = mlp_param_count(N_CELLS)
        if len(params) != npar or len(mean) != N_FEATURES or len(scale) != N_FEATURES:
            raise ValueError(f"selector needs {npar} parameters and 16 means / scales")
        P = (ctypes.c_float * npar)(*[float(v) for v in params])
        M = (ctypes.c_float * N_FEATURES)(*[float(v) for v in mean])
        S = (ctypes.c_float * N_FEATURES)(*[float(v) for v in scale])
        self._check(_load().jp_set_selector(self._p, P, N_CELLS, M, S))

    def clear_selector(self):
        self._check(_load().jp_set_selector(self._p, None, 0, None, None))

    def mlp_forward(self, params, x, n_out=N_CELLS):
        """Forward pass of the selector network on a (batch, 16) float32 CUDA tensor."""
        torch = _torch()
        _f32(params, "params", mlp_param_count(n_out))
        _f32(x, "x")
        b = x.numel() // N_FEATURES
        if x.numel() != b * N_FEATURES:
            raise ValueError("x must have 16 columns")
        y = torch.empty((b, n_out), dtype=torch.float32, device=x.device)
        self._bind_stream()
        self._check(_load().jp_mlp_forward(self._p, _ptr(params), n_out, _ptr(x), b, _ptr(y)))
        return y

    def mlp_grad(self, params, x, target, weight, grad=None, loss=None):
        """Loss gradient (written into / returned as a new tensor) and loss."""
        torch = _torch()
        b, n_out = target.shape
        _f32(params, "params", mlp_param_count(n_out))
        _f32(x, "x", b * N_FEATURES)
        _f32(target, "target")
        _f32(weight, "weight", b * n_out)
        if grad is None:
            grad = torch.empty_like(params)
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=params.device)
        _f32(grad, "grad", params.numel())
        _f32(loss, "loss", 1)
        self._bind_stream()
        self._check(_load().jp_mlp_grad(self._p, _ptr(params), n_out, _ptr(x), _ptr(target), _ptr(weight), b,
                                         _ptr(grad), _ptr(loss)))
        return grad, loss

    def mlp_adam(self, params, m, v, grad, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        """One Adam step in place on params, m, v."""
        n = params.numel()
        for t, nm in ((params, "params"), (m, "m"), (v, "v"), (grad, "grad")):
            _f32(t, nm, n)
        self._bind_stream()
        self._check(_load().jp_mlp_adam(self._p, _ptr(params), _ptr(m), _ptr(v), _ptr(grad), n, int(step),
                                         float(lr), float(beta1), float(beta2), float(eps)))

    def close(self):
        if getattr(self, "_p", None):
            _load().jp_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_handles = {}


def default_handle(device: int | None = None) -> Handle:
    torch = _torch()
    if device is None:
        device = torch.cuda.current_device()
    h = _handles.get(device)
    if h is None:
        h = _handles[device] = Handle(device)
    return h


def two_path(rx, ry, sz, sy, **kw):
    """Distinct (x, z) of Q(x,z) = R(x,y), S(z,y) as two sorted int32 tensors."""
    x, z, _ = default_handle(rx.device.index).two_path(rx, ry, sz, sy, **kw)
    return x, z


def star(rels, **kw):
    """Distinct tuples of the star query, as a list of k sorted int32 columns."""
    cols, _ = default_handle(rels[0][0].device.index).star(rels, **kw)
    return cols


def bool_matmul(A, Bt, **kw):
    return default_handle(A.device.index).bool_matmul(A, Bt, **kw)


def selector_cells(features):
    """The 65 (delta1, delta2) cells the selector scores for these 16
    features (None = infinity)."""
    f = (ctypes.c_float * N_FEATURES)(*[float(v) for v in features])
    a = (ctypes.c_int64 * N_CELLS)()
    b = (ctypes.c_int64 * N_CELLS)()
    n = _load().jp_selector_cells(f, a, b)
    inf = lambda v: None if v == DELTA_INF else v
    return [inf(v) for v in a[:n]], [inf(v) for v in b[:n]]


def mlp_param_count(n_out=N_CELLS):
    return int(_load().jp_mlp_param_count(n_out))


def heavy_cost(u, v, w, cal=None):
    """Heavy part of Algorithm 2's cost for dimensions (u, v, w), seconds
    (M-hat plus the heavy matrices' bytes; calibration dict or None)."""
    c = None if cal is None else (cal if isinstance(cal, Calibration) else Calibration.from_dict(cal))
    return float(_load().jp_heavy_cost(ctypes.byref(c) if c is not None else None, int(u), int(v), int(w)))


def selector_candidates(est_light, heavy):
    """Cells the selector may take: light only (the last) and every cell whose
    heavy-part estimate is below the light-only plan's estimate."""
    return [k == len(heavy) - 1 or h < est_light for k, h in enumerate(heavy)]


def default_calibration():
    c = Calibration()
    _load().jp_default_calibration(ctypes.byref(c))
    return c.as_dict()


def plan_theory(n, out):
    """Lemma 3 thresholds (integers, None = infinity) for N = n and output
    estimate out.  Runs on the host."""
    d1, d2 = ctypes.c_int64(), ctypes.c_int64()
    st = _load().jp_plan_theory(int(n), float(out), ctypes.byref(d1), ctypes.byref(d2))
    if st != 0:
        raise JoinProjectError(st, "jp_plan_theory failed")
    inf = lambda v: None if v == DELTA_INF else v
    return inf(d1.value), inf(d2.value)


def estimate_out(dom_x, dom_z, J, n):
    """Section 5 output-size estimate (host)."""
    return float(_load().jp_estimate_out(int(dom_x), int(dom_z), int(J), int(n)))


def plan_summary(summary, cal=None):
    """Algorithm 2 on a host summary (dict as returned by the oracle's
    degree_summary: sizes, J, out_est and (deg, count, sum) indexes).  Runs on
    the host; no GPU needed.  Returns (delta1, delta2, cost, cost_light_only)
    with None for infinity."""
    import numpy as np
    keep = []

    def idx(t):
        d, c, s = t
        d = np.ascontiguousarray(d, dtype=np.int64)
        c = np.ascontiguousarray(c, dtype=np.int64)
        keep.extend([d, c])
        di = DegreeIndex()
        di.n = d.size
        di.deg = d.ctypes.data
        di.count = c.ctypes.data
        if s is not None:
            s = np.ascontiguousarray(s, dtype=np.float64)
            keep.append(s)
            di.sum = s.ctypes.data
        return di

    ts = TwoPathSummary()
    for k in ("n_r", "n_s", "dom_x", "dom_y", "dom_z", "J"):
        setattr(ts, k, int(summary[k]))
    ts.out_est = float(summary["out_est"])
    ts.y, ts.x, ts.xcdf, ts.z = (idx(summary[k]) for k in ("y", "x", "xcdf", "z"))
    c = None if cal is None else (cal if isinstance(cal, Calibration) else Calibration.from_dict(cal))
    d1, d2 = ctypes.c_int64(), ctypes.c_int64()
    cost, clo = ctypes.c_double(), ctypes.c_double()
    st = _load().jp_plan_summary(ctypes.byref(ts), ctypes.byref(c) if c is not None else None, ctypes.byref(d1),
                                 ctypes.byref(d2), ctypes.byref(cost), ctypes.byref(clo))
    if st != 0:
        raise JoinProjectError(st, "jp_plan_summary failed")
    inf = lambda v: None if v == DELTA_INF else v
    return inf(d1.value), inf(d2.value), cost.value, clo.value
