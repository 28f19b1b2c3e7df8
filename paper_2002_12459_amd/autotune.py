"""Autotuner of the heavy product kernel (MI355X).

For a grid of product shapes (u rows of A, w rows of B^T, row stride ld
bytes, 0/1 int8 entries at density 1/8) it times every product kernel
(int8 MFMA with 128 x 128 block tiles, int8 MFMA with 256 x 256 block tiles,
bit-packed AND + popcount) through jp_bool_matmul in count-only mode, best of
``--reps`` runs after a warm-up, and keeps the fastest per shape class (the
log2 buckets of u, w and ld, jp_product_shape_class).  The table is written
as JSON and installed in every Handle (jp_set_product_table), so that
JP_BMM_AUTO picks the kernel without a timed race, also inside captured
plans.

    python -m paper_2002_12459_amd.autotune --out paper_2002_12459_amd/autotune_mi355x.json
"""
from __future__ import annotations

import argparse
import json
import sys
import time

KINDS = ("i8_t128", "i8_t256", "bitpop")


def shapes():
    """(u, w, ld) of the sweep: square and skewed heavy parts, short and long K."""
    out = []
    for u in (1024, 4096, 16384, 65536, 131072):
        for ld in (128, 512, 2048, 8192):
            out.append((u, u, ld))
    for u, w in ((1024, 65536), (65536, 1024), (4096, 131072), (131072, 4096)):
        for ld in (128, 2048):
            out.append((u, w, ld))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--max-ops", type=float, default=3e14, help="skip shapes with more int8 operations")
    a = ap.parse_args(argv)
    import torch

    import paper_2002_12459_amd as jp
    h = jp.Handle(0, product_table=None, allocator="builtin")
    g = torch.Generator(device="cuda").manual_seed(1)
    entries = []
    for u, w, ld in shapes():
        ops = 2.0 * u * w * ld
        if ops > a.max_ops:
            continue
        A = (torch.rand((u, ld), device="cuda", generator=g) < 0.125).to(torch.int8)
        B = (torch.rand((w, ld), device="cuda", generator=g) < 0.125).to(torch.int8)
        times = {}
        for kind in KINDS:
            h.bool_matmul_count(A, B, kind=kind)
            best = None
            for _ in range(a.reps):
                _, ms = h.bool_matmul_count(A, B, kind=kind)
                best = ms if best is None else min(best, ms)
            times[kind] = best
        kind = min(times, key=times.get)
        cls = jp.product_shape_class(u, w, ld)
        entries.append({"class": cls, "u": u, "w": w, "ld": ld, "kind": kind, "ms": times,
                        "tops": ops / (times[kind] * 1e-3) / 1e12})
        print(f"u={u} w={w} ld={ld}: {kind} " + " ".join(f"{k}={v:.3f}ms" for k, v in times.items()),
              flush=True)
        del A, B
    with open(a.out, "w") as fh:
        json.dump({"device": torch.cuda.get_device_name(0), "time": time.strftime("%Y-%m-%d"),
                   "entries": entries}, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
