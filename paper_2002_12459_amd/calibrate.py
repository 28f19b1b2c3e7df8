"""Measure the cost-based optimizer's constants on this GPU.

    python -m paper_2002_12459_amd.calibrate [out.json]

* product table: the int8 heavy product on p x p x p random 0/1 operands
  (density 1/256) for p in 1024 .. 20480 (the table of Section 5, here for
  this library's kernel);
* T_I (t_witness): device time of a light-only evaluation per light witness;
* T_m per byte (t_byte): time per byte to clear and fill a heavy matrix;
* T_m per x (t_x): fixed per-x cost of the light path.
Writes JSON that Handle.set_calibration accepts.
"""
from __future__ import annotations

import json
import sys
import time


def main(out_path="calibration.json"):
    import numpy as np
    import torch

    import datagen
    import paper_2002_12459_amd as jp

    h = jp.Handle(0)
    cal = jp.default_calibration()
    ps, ts = [], []
    for p in (1024, 2048, 4096, 8192, 12288, 16384, 20480):
        g = torch.Generator(device="cuda").manual_seed(p)
        A = (torch.rand((p, p), device="cuda", generator=g) < 1 / 256).to(torch.int8)
        B = (torch.rand((p, p), device="cuda", generator=g) < 1 / 256).to(torch.int8)
        cap = p * p
        h.bool_matmul(A, B, cap=cap)  # warm-up
        best = min(h.bool_matmul(A, B, cap=cap)[2] for _ in range(3))
        ps.append(float(p))
        ts.append(best * 1e-3)
        print(f"[calibrate] p={p}: {best:.3f} ms, {2 * p ** 3 / (best * 1e-3) / 1e12:.1f} TOP/s", flush=True)
        del A, B
    cal["mm_p"], cal["mm_s"] = ps, ts

    (rx, ry), (sz, sy) = datagen.twopath_c2(0.25)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()
    Rx, Ry, Sz, Sy = T(rx), T(ry), T(sz), T(sy)
    r = h.two_path_result(Rx, Ry, Sz, Sy, strategy="light", timing=True)
    r.free()
    r = h.two_path_result(Rx, Ry, Sz, Sy, strategy="light", timing=True)
    st = r.stats
    r.free()
    cal["t_witness"] = (st["ms_dedup"] + st["ms_light"]) * 1e-3 / max(st["J_L"], 1)
    cal["t_x"] = st["ms_ingest"] * 1e-3 / max(st["dom_x"] + st["dom_z"], 1)
    buf = torch.empty(1 << 30, dtype=torch.int8, device="cuda")
    buf.zero_()  # first touch outside the timed loop
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        buf.zero_()
    torch.cuda.synchronize()
    cal["t_byte"] = (time.perf_counter() - t0) / 5 / buf.numel() * 2  # clear + scattered fill
    print(f"[calibrate] t_witness={cal['t_witness']:.3e} t_x={cal['t_x']:.3e} t_byte={cal['t_byte']:.3e}", flush=True)
    with open(out_path, "w") as f:
        json.dump(cal, f, indent=1)
    print(f"[calibrate] wrote {out_path}")


if __name__ == "__main__":
    main(*sys.argv[1:])
