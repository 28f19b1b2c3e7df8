"""Benchmark: distinct (x,z) output pairs per second of the two-path
join-project on one MI355X, plus the heavy product's int8 TOPS.

Workload: Q(x,z) = R(x,y), S(z,y) with |R| = |S| = 10M distinct int32 edges,
1M x/z ids, 200K y ids, y degrees Zipf(1.1) (independent y-rank permutations
for R and S), x/z uniform; thresholds from the cost model.  Inputs are
seeded synthetic data, generated on the host and resident in HBM before the
timed region.  One step = one full evaluation (index build, thresholds,
partition, light expansion, heavy product, union, duplicate removal, sorted
output in HBM).

A second leg measures the batched mode on the serving-style set: 512
independent two-path instances, edge counts log-uniform in [1K, 1M], Zipf
exponent U[0.6, 1.6], evaluated in one call; it is reported under "batched"
next to the time of the same instances evaluated one call each, and as a
captured plan replayed as one HIP graph.  Further legs: the same 10M input
with the learned selector's thresholds ("selector") and at forced thresholds
that give the int8 product a large shape ("heavy_bmm"); the star query over
three 2M-edge Zipf(1.3) relations ("star") and a 4-relation star
("star_k4"); a dense-core self-join of 8 communities ("dense_core"), where
the cost model sends most witnesses to the matrix product; the set
similarity join at overlap >= 2 ("ssj") and batched set intersection
("bsi") on the 10M input; the paper's five-run, middle-three timing
("paper_protocol"); the whole output against the oracle ("parity"); and the
oracle itself on the host cores ("cpu_baseline").

    python bench.py [--steps K] [--warmup W] [--gpus 1]
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
INT8_PEAK_TOPS = 5000.0        # MI355X dense int8 MFMA, TOP/s

# HBM bytes moved by one k_dedup launch on this workload, from two
# rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each
# scaled by what the same counter reads for a 1 GiB device copy (FETCH_SIZE
# reads half of the copy's 1 GiB: x2; WRITE_SIZE reads it in full: x1); see
# profiles/k_dedup_two_path_10M_traffic.md.  Valid only for the dedup source
# whose SHA-256 is given (None: not measured for the current source).
DEDUP_TRAFFIC = {"sha256": "41f302bc8b638cc89b25e2ae8f9053f0aadcc4924c5f44146ce085e63f9e39ff",
                 "bytes_per_launch": 1844558510}


def dedup_traffic():
    import hashlib
    with open(os.path.join(ROOT, "paper_2002_12459_amd", "csrc", "dedup.hip"), "rb") as fh:
        digest = hashlib.sha256(fh.read()).hexdigest()
    return DEDUP_TRAFFIC["bytes_per_launch"] if digest == DEDUP_TRAFFIC["sha256"] else None


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--scale", type=float, default=1.0, help="shrink the workload (testing only)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-bmm", action="store_true")
    p.add_argument("--cpu-sample", type=float, default=0.3,
                   help="fraction of x ids in the single-thread oracle sample")
    p.add_argument("--no-batch", action="store_true")
    p.add_argument("--batch-instances", type=int, default=512)
    p.add_argument("--no-star", action="store_true")
    p.add_argument("--no-dense", action="store_true")
    p.add_argument("--no-ssj", action="store_true", help="skip the set-similarity and set-intersection legs")
    return p.parse_args()


def _batch_instance(i):
    import datagen
    return datagen.batch_instance(i)


def batched_leg(h, insts, steps, warmup):
    """Batched evaluation of all instances vs one call per instance, and the
    graph-captured plan of the same batch."""
    import torch

    import paper_2002_12459_amd as jp
    dev = torch.device("cuda:0")
    T = lambda v: torch.from_numpy(v).to(dev)
    tin = [(T(r[0]), T(r[1]), T(s[0]), T(s[1])) for r, s in insts]
    for _ in range(warmup):
        h.two_path_batch_result(tin).free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = h.two_path_batch_result(tin)
        n, st = r.n, r.stats
        r.free()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    # the same instances one call each (after one warm-up pass)
    for q in tin:
        h.two_path_result(*q).free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_single = 0
    for q in tin:
        r = h.two_path_result(*q)
        n_single += r.n
        r.free()
    torch.cuda.synchronize()
    ds = time.perf_counter() - t0
    if n_single != n:
        raise RuntimeError(f"batched output size {n} differs from per-instance total {n_single}")
    # the same batch as a graph-captured plan: replays of one HIP graph
    try:
        h.batch_plan(tin, arena_bytes=256)
        raise RuntimeError("a 256-byte arena was accepted")
    except jp.JoinProjectError as e:
        need = e.arena_needed
    plan = h.batch_plan(tin, arena_bytes=need)
    plan.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.launch()
    torch.cuda.synchronize()
    dg = (time.perf_counter() - t0) / steps
    n_plan = sum(int(x.numel()) for x, _ in plan.outputs())
    plan.free()
    if n_plan != n:
        raise RuntimeError(f"plan output size {n_plan} differs from the batched call's {n}")
    return {"workload": f"{len(insts)} two-path instances, |R|=|S| log-uniform [1K,1M], Zipf U[0.6,1.6], "
                        f"x/z ids E/10, y ids E/50; one batched call, cost-model thresholds",
            "edges_r": int(sum(q[0].numel() for q in tin)), "n_out": n, "J": st["J"],
            "ms_per_step": dt * 1e3, "pairs_per_s": n / dt, "instances_per_s": len(insts) / dt,
            "delta1": st["delta1"], "delta2": st["delta2"],
            "per_instance_calls_ms": ds * 1e3, "speedup_vs_per_instance_calls": ds / dt,
            "graph_replay": {"ms_per_step": dg * 1e3, "pairs_per_s": n / dg, "arena_bytes": need,
                             "note": "one HIP graph of the whole batched evaluation, replayed; the launch "
                                     "first fingerprints the inputs on the device"}}


def star_leg(h, rels, steps):
    """Star query over three relations: cost-model thresholds, then forced
    thresholds that give the chained heavy product work."""
    import torch
    dev = torch.device("cuda:0")
    tin = [(torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)) for a, b in rels]
    h.star_result(tin).free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = h.star_result(tin)
        n, st = r.n, r.stats
        r.free()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    out = {"workload": "star k=3: 3 relations of 2M distinct edges, 500K x ids, 100K y ids, Zipf(1.3) y "
                       "(independent y-rank permutations), cost-model thresholds",
           "n_out": n, "J": st["J"], "ms_per_step": dt * 1e3, "tuples_per_s": n / dt,
           "delta1": st["delta1"], "delta2": st["delta2"]}
    d1, d2 = 20, 4  # after dangling tuples go: 119 y heavy in two relations, 13.5K / 3.4K / 0.5K heavy x
    h.star_result(tin, delta1=d1, delta2=d2).free()
    r = h.star_result(tin, delta1=d1, delta2=d2, timing=True)
    nf, sf = r.n, r.stats
    r.free()
    if nf != n:
        raise RuntimeError(f"star output size {nf} at forced thresholds differs from {n}")
    out["forced"] = {"delta1": d1, "delta2": d2, "ms_total": sf["ms_total"], "ms_bmm": sf["ms_bmm"],
                     "bmm_ops": sf["bmm_ops"],
                     "tops": sf["bmm_ops"] / (sf["ms_bmm"] * 1e-3) / 1e12 if sf["ms_bmm"] > 0 else None}
    return out


def ssj_leg(h, T, steps):
    """Set similarity join on the two-path input: pairs sharing >= 2 and >= 3
    elements, plain and ordered by overlap."""
    import torch
    Rx, Ry, Sz, Sy = T
    out = {"workload": "set similarity join on the 10M two-path input (overlap >= c), cost-model thresholds"}
    for c, ordered in ((2, False), (2, True), (3, False)):
        h.ssj_result(Rx, Ry, Sz, Sy, min_overlap=c, ordered=ordered).free()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            r = h.ssj_result(Rx, Ry, Sz, Sy, min_overlap=c, ordered=ordered)
            n, st = r.n, r.stats
            r.free()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        out[f"c{c}{'_ordered' if ordered else ''}"] = {"ms_per_step": dt * 1e3, "n_out": n, "J": st["J"],
                                                      "witnesses_per_s": st["J"] / dt,
                                                      "delta1": st["delta1"], "delta2": st["delta2"]}
    return out


def bsi_leg(h, T, host, steps):
    """Batched set intersection over the two-path input's relations: batches
    of 1K, 10K and 100K queries."""
    import numpy as np
    import torch
    import datagen
    Rx, Ry, Sz, Sy = T
    out = {"workload": "batched Boolean set intersection over the 10M relations (half the queries share a sampled "
                       "element, 3/8 independent set ids, 1/8 absent ids), cost-model thresholds"}
    for b in (1_000, 10_000, 100_000):
        tx, tz = datagen.bsi_batch(*host, b, seed=b)
        Tx = torch.from_numpy(tx).cuda()
        Tz = torch.from_numpy(tz).cuda()
        h.bsi(Rx, Ry, Sz, Sy, Tx, Tz)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ans, st = h.bsi(Rx, Ry, Sz, Sy, Tx, Tz)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        out[f"batch{b}"] = {"ms_per_batch": dt * 1e3, "queries_per_s": b / dt,
                            "answered_true": int(ans.sum().item()), "filtered_edges_r": st["n_r"],
                            "pairs_of_filtered_query": st["n_out"]}
    return out


def star4_leg(h, rels, steps):
    """Star query with k = 4: cost-model thresholds, then forced thresholds
    that give the product of generated V and W rows work."""
    import torch
    dev = torch.device("cuda:0")
    tin = [(torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)) for a, b in rels]
    h.star_result(tin).free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = h.star_result(tin)
        n, st = r.n, r.stats
        r.free()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    out = {"workload": "star k=4: 4 relations of 500K distinct edges, 125K x ids, 25K y ids, Zipf(1.3) y "
                       "(independent y-rank permutations), cost-model thresholds",
           "n_out": n, "J": st["J"], "ms_per_step": dt * 1e3, "tuples_per_s": n / dt,
           "delta1": st["delta1"], "delta2": st["delta2"]}
    # the product's own workload: dense communities, where every witness is
    # heavy at Delta1 = Delta2 = 1 (4 communities of 64 x ids by 512 y ids,
    # p = 0.5: |OUT| = 4 * 64^4 by closed form, J / |OUT| = 32)
    import datagen
    x, y = datagen.communities(4, 64, 512, 0.5, seed=12)
    X, Y = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
    dense = [(X, Y)] * 4
    h.star_result(dense, delta1=1, delta2=1).free()
    r = h.star_result(dense, delta1=1, delta2=1, timing=True)
    nf, sf = r.n, r.stats
    r.free()
    out["dense_product"] = {"workload": "k=4 star over 4 communities of 64 x ids by 512 y ids at p=0.5 "
                                        f"({x.size} edges per relation), Delta1 = Delta2 = 1",
                            "n_out": nf, "closed_form_n_out": 4 * 64 ** 4, "J": sf["J"], "rows_v": sf["u"],
                            "v": sf["v"], "rows_w": sf["w"], "ms_total": sf["ms_total"], "ms_bmm": sf["ms_bmm"],
                            "bmm_ops": sf["bmm_ops"],
                            "tops": sf["bmm_ops"] / (sf["ms_bmm"] * 1e-3) / 1e12 if sf["ms_bmm"] > 0 else None}
    if nf != 4 * 64 ** 4:
        raise RuntimeError(f"k=4 dense star output size {nf} differs from the closed form")
    return out


def dense_leg(h, edges, steps):
    """Dense-core self-join (communities): the case where the product pays."""
    import torch
    dev = torch.device("cuda:0")
    x = torch.from_numpy(edges[0]).to(dev)
    y = torch.from_numpy(edges[1]).to(dev)
    h.two_path_result(x, y, x, y).free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = h.two_path_result(x, y, x, y)
        n, st = r.n, r.stats
        r.free()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    r = h.two_path_result(x, y, x, y, timing=True)
    sp = r.stats
    r.free()
    # the same product with fp16 operands and fp32 accumulation (exact: v < 2^24)
    h.two_path_result(x, y, x, y, bmm="f16").free()
    r = h.two_path_result(x, y, x, y, bmm="f16", timing=True)
    sf = r.stats
    nf = r.n
    r.free()
    if nf != n:
        raise RuntimeError(f"fp16 product output size {nf} differs from {n}")
    f16 = {"ms_bmm": sf["ms_bmm"], "tops": sf["bmm_ops"] / (sf["ms_bmm"] * 1e-3) / 1e12 if sf["ms_bmm"] > 0 else None,
           "peak_tops": 2500.0, "ms_total": sf["ms_total"]}
    return {"f16_product": f16, "workload": f"dense-core self-join: 8 communities of 4096 x ids by 2048 y ids, edge probability 0.25 "
                        f"({int(x.numel())} edges), cost-model thresholds",
            "n_out": n, "closed_form_n_out": 8 * 4096 * 4096, "J": st["J"], "ms_per_step": dt * 1e3,
            "pairs_per_s": n / dt, "delta1": st["delta1"], "delta2": st["delta2"], "u": sp["u"], "v": sp["v"],
            "w": sp["w"], "ms_bmm": sp["ms_bmm"],
            "bmm_tops": sp["bmm_ops"] / (sp["ms_bmm"] * 1e-3) / 1e12 if sp["ms_bmm"] > 0 else None,
            "bmm_ops_executed": sp["bmm_ops"], "bmm_ops_full_product": 2.0 * sp["u"] * sp["v"] * sp["w"],
            "note": "self-join: M2^T = M1, the product runs on the tiles on and above the diagonal (mirrored)"}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); the library runs on a single GPU.",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np

    # batched-set generation in worker processes, forked before this process
    # touches the GPU
    pool = batch_async = None
    if not a.no_batch:
        import multiprocessing as mp
        pool = mp.get_context("fork").Pool(min(12, os.cpu_count() or 1))
        batch_async = pool.map_async(_batch_instance, range(a.batch_instances))

    import torch

    import datagen
    import paper_2002_12459_amd as jp

    t0 = time.time()
    (rx, ry), (sz, sy) = datagen.twopath_c2(a.scale)
    log(f"generated |R|={rx.size} |S|={sz.size} in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    T = lambda v: torch.from_numpy(np.ascontiguousarray(v, dtype=np.int32)).to(dev)
    Rx, Ry, Sz, Sy = T(rx), T(ry), T(sz), T(sy)
    h = jp.Handle(0, allocator="builtin")  # the library's own pool: no Python callback per buffer

    def step(**kw):
        r = h.two_path_result(Rx, Ry, Sz, Sy, **kw)
        n, st = r.n, r.stats
        r.free()
        return n, st

    if batch_async is not None:
        batch_async.wait()  # no host work competes with the timed region
    for i in range(a.warmup):
        n, st = step()
        log(f"warmup {i}: |OUT|={n} strategy={st['strategy']} d1={st['delta1']} d2={st['delta2']}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_out = None
    for i in range(a.steps):
        n, st = step()
        n_out = n
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / a.steps
    log(f"timed {a.steps} steps: {dt * 1e3:.2f} ms/step, |OUT|={n_out}")

    # the paper's protocol (Section 7): 5 runs, each timed on its own, mean
    # of the middle 3
    runs = []
    for _ in range(5):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        runs.append(time.perf_counter() - t1)
    mid3 = sorted(runs)[1:4]
    protocol = {"runs_ms": [r * 1e3 for r in runs], "middle3_mean_ms": sum(mid3) / 3 * 1e3,
                "value": n_out / (sum(mid3) / 3)}

    # one more evaluation with per-phase / dominant-kernel device timing
    _, ph = step(timing=True)
    log("phases ms: " + ", ".join(f"{k[3:]}={ph[k]:.3f}" for k in ph if k.startswith("ms_")))
    log(f"J={ph['J']} J_L={ph['J_L']} J_H={ph['J_H']} u={ph['u']} v={ph['v']} w={ph['w']} units={ph['dedup_units']}")
    dom_ms = ph["ms_kernel_dedup"]
    dom_bytes = ph["dedup_alg_bytes"]
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9 if dom_ms > 0 else None
    roofline = {"kernel": "k_dedup (per-x witness gather + on-chip sort/bitmap dedup)", "bound": "hbm",
                "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": dedup_traffic(),
                "alg_bytes_per_launch": dom_bytes, "ms_per_launch": dom_ms}

    # the learned selector on the same input (when weights are installed)
    selector = None
    if os.path.exists(jp.SELECTOR_PATH):
        step(strategy="mlp")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            n_m, st_m = step(strategy="mlp")
        torch.cuda.synchronize()
        dm = (time.perf_counter() - t0) / a.steps
        selector = {"strategy": "learned selector (AUTO_MLP)", "ms_per_step": dm * 1e3, "value": n_m / dm,
                    "delta1": st_m["delta1"], "delta2": st_m["delta2"], "speedup_vs_cost_model": dt / dm}
        log(f"selector: {dm * 1e3:.2f} ms/step (d1={st_m['delta1']} d2={st_m['delta2']})")

    # heavy product at forced thresholds (the cost model keeps this workload light)
    bmm = None
    if not a.no_bmm:
        d1, d2 = 1000, 12
        step(delta1=d1, delta2=d2)  # warm-up of the product kernel
        nb, pb = step(delta1=d1, delta2=d2, timing=True)
        if pb["ms_bmm"] > 0:
            tops = pb["bmm_ops"] / (pb["ms_bmm"] * 1e-3) / 1e12
            bmm = {"delta1": d1, "delta2": d2, "u": pb["u"], "v": pb["v"], "w": pb["w"],
                   "nnz": pb["nnz_heavy"], "ms": pb["ms_bmm"], "tops": tops, "peak_tops": INT8_PEAK_TOPS,
                   "frac": tops / INT8_PEAK_TOPS, "n_out": nb, "ms_total": pb["ms_total"]}
            log(f"heavy product u={pb['u']} v={pb['v']} w={pb['w']}: {pb['ms_bmm']:.2f} ms, {tops:.1f} TOP/s")

    batched = None
    if batch_async is not None:
        t0 = time.time()
        insts = batch_async.get()
        pool.close()
        log(f"batched set ready ({time.time() - t0:.1f}s wait)")
        batched = batched_leg(h, insts, max(1, min(a.steps, 3)), 1)
        log(f"batched: {batched['ms_per_step']:.1f} ms per call for {len(insts)} instances, "
            f"{batched['pairs_per_s']:.3g} pairs/s; one call per instance: {batched['per_instance_calls_ms']:.1f} ms; "
            f"graph replay {batched['graph_replay']['ms_per_step']:.1f} ms")
        del insts

    star = None
    if not a.no_star:
        t0 = time.time()
        rels = datagen.star_c3(a.scale)
        log(f"star input generated in {time.time() - t0:.1f}s")
        star = star_leg(h, rels, max(1, min(a.steps, 3)))
        log(f"star: {star['ms_per_step']:.2f} ms/step, |OUT|={star['n_out']} (d1={star['delta1']} d2={star['delta2']}); "
            f"forced product {star['forced']['ms_bmm']:.2f} ms, {star['forced']['tops'] or 0:.1f} TOP/s")
        del rels

    ssj = bsi = None
    if not a.no_ssj:
        ssj = ssj_leg(h, (Rx, Ry, Sz, Sy), max(1, min(a.steps, 3)))
        log("ssj: " + ", ".join(f"{k} {v['ms_per_step']:.2f} ms ({v['n_out']} pairs)" for k, v in ssj.items()
                                if isinstance(v, dict)))
        bsi = bsi_leg(h, (Rx, Ry, Sz, Sy), (rx, ry, sz, sy), max(1, min(a.steps, 3)))
        log("bsi: " + ", ".join(f"{k} {v['ms_per_batch']:.2f} ms" for k, v in bsi.items() if isinstance(v, dict)))

    star4 = None
    if not a.no_star:
        rels4 = datagen.star4_c(a.scale)
        star4 = star4_leg(h, rels4, max(1, min(a.steps, 3)))
        dp = star4["dense_product"]
        log(f"star k=4: {star4['ms_per_step']:.2f} ms/step, |OUT|={star4['n_out']}; dense product "
            f"{dp['ms_bmm']:.2f} ms, {dp['tops'] or 0:.1f} TOP/s, whole call {dp['ms_total']:.2f} ms")
        del rels4

    dense = None
    if not a.no_dense and a.scale == 1.0:
        t0 = time.time()
        edges = datagen.communities(8, 4096, 2048, 0.25, seed=7)
        log(f"dense-core input ({edges[0].size} edges) generated in {time.time() - t0:.1f}s")
        dense = dense_leg(h, edges, max(1, min(a.steps, 3)))
        log(f"dense core: {dense['ms_per_step']:.2f} ms/step, |OUT|={dense['n_out']} (closed form "
            f"{dense['closed_form_n_out']}), d1={dense['delta1']} d2={dense['delta2']} u={dense['u']} v={dense['v']} "
            f"w={dense['w']}, product {dense['ms_bmm']:.2f} ms")
        del edges

    # CPU oracle on the same input: all host cores (3 runs, mean) and one
    # thread (one run); the all-core output is also compared with the GPU's
    cpu = None
    parity = None
    if not a.no_cpu_baseline:
        import oracle
        threads = max(1, min(16, oracle.cores()))
        t_all = []
        for _ in range(3):
            t0 = time.perf_counter()
            ox, oz = oracle.two_path_par(rx, ry, sz, sy, threads=threads)
            t_all.append(time.perf_counter() - t0)
        r = h.two_path_result(Rx, Ry, Sz, Sy)
        gx, gz = r.to_torch()
        r.free()
        equal = bool(gx.numel() == ox.size and np.array_equal(gx.cpu().numpy(), ox)
                     and np.array_equal(gz.cpu().numpy(), oz))
        parity = {"against": "oracle, whole output", "n_out_gpu": int(gx.numel()), "n_out_oracle": int(ox.size),
                  "equal": equal}
        del gx, gz
        lim = int(a.cpu_sample * max(int(1_000_000 * a.scale), 1))
        m = rx < lim
        t0 = time.perf_counter()
        sx, _ = oracle.two_path(rx[m], ry[m], sz, sy)
        t1 = time.perf_counter() - t0
        ta = sum(t_all) / len(t_all)
        cpu = {"value": ox.size / ta, "unit": "pairs/s", "cores": threads, "kind": "oracle",
               "sample": f"the whole input ({rx.size} + {sz.size} edges, {ox.size} distinct pairs): full join, "
                         f"qsort, unique per x-range chunk on {threads} OpenMP threads; mean of 3 runs "
                         f"({', '.join(f'{t:.2f}' for t in t_all)} s)",
               "single_thread": {"value": sx.size / t1, "cores": 1,
                                 "sample": f"R restricted to x < {lim} ({int(m.sum())} edges), all of S; "
                                           f"{sx.size} distinct pairs in {t1:.1f} s (one run)"},
               "cpu_model": cpu_model(), "nproc": os.cpu_count(), "affinity_cores": oracle.cores()}
        log(f"cpu oracle: {cpu['sample']}; one thread: {cpu['single_thread']['sample']}; parity {equal}")
        del ox, oz

    out = {
        "metric": "distinct (x,z) output pairs/sec for two-path join-project, + heavy-BMM int8 TOPS",
        "value": n_out / dt,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "two-path R(x,y),S(z,y): |R|=|S|=10M, 1M x/z ids, 200K y ids, Zipf(1.1) y, "
                               "cost-model thresholds" if a.scale == 1.0 else f"two-path scaled x{a.scale}",
                   "n_out": n_out, "J": ph["J"], "delta1": ph["delta1"], "delta2": ph["delta2"]},
        "paper_protocol": protocol,
        "parity": parity,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "heavy_bmm": bmm,
        "batched": batched,
        "selector": selector,
        "star": star,
        "dense_core": dense,
        "ssj": ssj,
        "bsi": bsi,
        "star_k4": star4,
        "phases_ms": {k[3:]: ph[k] for k in ph if k.startswith("ms_")},
    }
    print(json.dumps(out), flush=True)
    if parity is not None and not parity["equal"]:
        log("GPU output differs from the oracle")
        sys.exit(1)


if __name__ == "__main__":
    main()
