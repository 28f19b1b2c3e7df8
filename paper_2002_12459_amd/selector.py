"""Training data, training and evaluation of the learned threshold selector.

The selector (strategy "mlp") scores the 65 threshold cells of
``selector_cells`` (an 8 x 8 geometric grid of (Delta1, Delta2) plus light
only) from the 16 instance features of ``Handle.plan_two_path`` and runs the
cell with the lowest predicted log time ratio.  Any cell gives the exact
result (the partition argument of Section 3.1 holds for every threshold
pair), so the selector only affects speed.  It stands in for the search of
Algorithm 2 (Section 5), which stays the fallback.

    # time every cell on generated instances (GPU), one JSON line per instance
    python -m paper_2002_12459_amd.selector sweep --first 0 --count 300 --out sweep.jsonl
    # train with the library's own forward / gradient / Adam kernels (GPU)
    python -m paper_2002_12459_amd.selector train --data sweep*.jsonl --holdout-from 1000 \\
        --out selector_mi355x.json --report report.json

Instances: three families, each indexed from 0.  "zipf":
``datagen.selector_instance`` (|R| = |S| log-uniform, Zipf y degrees with
exponent U[0.5, 1.8], x / y domains |R|/10 and |R|/50; the output is close to
the join size, few duplicates).  "clustered":
``datagen.selector_instance_clustered`` (dense communities, as in the
paper's Example 1, plus a Zipf part; many duplicate witnesses).  "dense":
``datagen.selector_instance_dense`` (a few large dense communities whose
sets share tens to about a hundred elements: the shape of the paper's
dense datasets, where the product pays).
Instances whose full join J = sum_y deg_R(y) deg_S(y) exceeds ``--jmax`` are
recorded as rejected and not timed: their run time is dominated by writing an
output close to |dom x| |dom z| pairs whatever the thresholds.

Cell timing: wall time of one jp_two_path call (result freed), best of
``--reps`` runs after one warm-up.  A cell is not run when the cost model
(``Handle.plan_cells``) predicts a product of more than ``--max-ops``
operations, heavy matrices of more than ``--max-bytes`` bytes, or more than
``--skip-ratio`` times the light-only estimate; a cell whose warm-up takes
more than ``--skip-ratio`` times the measured light-only time is not
repeated.  Such cells count as ``--skip-ratio`` times slower than the best.
"""
from __future__ import annotations

import argparse
import functools
import json
import math
import os
import sys
import time

N_CELLS = 65
N_FEATURES = 16


# ---------------------------------------------------------------------------- sweep

def _generate(i, family, lo, hi, jmax):
    import numpy as np

    import datagen
    if family == "clustered":
        (rx, ry), (sz, sy), prm = datagen.selector_instance_clustered(i, lo=lo, hi=hi)
        s = prm["s"]
    elif family == "dense":
        (rx, ry), (sz, sy), prm = datagen.selector_instance_dense(i, lo=lo, hi=hi, jmax=jmax)
        s = prm["s"]
    else:
        (rx, ry), (sz, sy), s = datagen.selector_instance(i, lo=lo, hi=hi)
    ny = int(max(ry.max(), sy.max())) + 1
    J = int((np.bincount(ry, minlength=ny).astype(np.int64) * np.bincount(sy, minlength=ny)).sum())
    if J > jmax:
        return i, None, s, J
    return i, (rx, ry, sz, sy), s, J


def _key(rec):
    return rec.get("family", "zipf"), rec["i"]


def _done_indices(paths):
    """Instances already swept cleanly (records whose cells disagreed on the
    output size are swept again)."""
    done = set()
    for p in paths:
        if not os.path.exists(p):
            continue
        with open(p) as fh:
            for line in fh:
                line = line.strip()
                if line:
                    r = json.loads(line)
                    if not r.get("mismatch"):
                        done.add(_key(r))
    return done


def sweep(args):
    import multiprocessing as mp

    done = _done_indices(args.resume + [args.out])
    todo = [i for i in range(args.first, args.first + args.count) if (args.family, i) not in done]
    # workers only run numpy; they are forked before this process touches the GPU
    pool = mp.get_context("fork").Pool(args.workers)
    gen = pool.imap(functools.partial(_generate, family=args.family, lo=args.lo, hi=args.hi, jmax=args.jmax), todo)

    import numpy as np
    import torch

    import paper_2002_12459_amd as jp

    h = jp.Handle(0, selector=None, allocator="builtin")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()
    t_start = time.perf_counter()
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    out = open(args.out, "a")
    n_done = 0
    for i, data, s, J in gen:
        rec = {"family": args.family, "i": i, "s": s, "J": J}
        if data is None:
            rec["rejected"] = True
            out.write(json.dumps(rec) + "\n")
            out.flush()
            print(f"[sweep] {i}: rejected (J={J:.3g})", flush=True)
            continue
        rx, ry, sz, sy = data
        R = (T(rx), T(ry), T(sz), T(sy))
        n = int(max(rx.size, sz.size))
        rec["n"] = n

        def run(reps, limit=None, **kw):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = h.two_path_result(*R, **kw)
            torch.cuda.synchronize()
            best = time.perf_counter() - t0
            st = r.stats
            r.free()
            if limit is not None and best > limit:
                return best, st, False
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = h.two_path_result(*R, **kw)
                torch.cuda.synchronize()
                best = min(best, time.perf_counter() - t0)
                r.free()
            return best, st, True

        d1a, d2a, feats = h.plan_two_path(*R)
        d1s, d2s = jp.selector_cells(feats)
        est, dims = h.plan_cells(*R, d1s, d2s)
        rec["features"] = feats
        rec["cells"] = [[a, b] for a, b in zip(d1s, d2s)]
        rec.update(_cell_estimates(h, est, dims))
        t = [None] * N_CELLS
        full = [False] * N_CELLS
        t_light, st, full[64] = run(args.reps, strategy="light")
        t[64] = t_light
        n_out = st["n_out"]
        mismatch = 0
        for k in range(64):
            u, v, w = dims[k]
            vpad = -(-v // 128) * 128
            if (2.0 * u * v * w > args.max_ops or (u + w) * vpad > args.max_bytes
                    or est[k] > args.skip_ratio * est[64]):
                continue
            t[k], st, full[k] = run(args.reps, limit=args.skip_ratio * t_light, strategy="fixed", delta1=d1s[k],
                                    delta2=d2s[k])
            mismatch += st["n_out"] != n_out
        for name, kw in (("auto", {"strategy": "auto"}), ("theory", {"strategy": "theory"}),
                         ("sqrtN", {"strategy": "fixed", "delta1": math.isqrt(n), "delta2": math.isqrt(n)})):
            tt, st, _ = run(args.reps, limit=args.skip_ratio * t_light, **kw)
            rec[name] = {"t": tt, "d1": st["delta1"] if st["delta1"] != jp.DELTA_INF else None,
                         "d2": st["delta2"] if st["delta2"] != jp.DELTA_INF else None}
            mismatch += st["n_out"] != n_out
        rec["t"] = t
        rec["full"] = full
        rec["n_out"] = n_out
        rec["mismatch"] = mismatch
        out.write(json.dumps(rec) + "\n")
        out.flush()
        n_done += 1
        best = min(x for x in t if x is not None)
        el = time.perf_counter() - t_start
        print(f"[sweep] {i}: n={n} s={s:.2f} J={J:.3g} out={n_out:.3g} best={best * 1e3:.2f} ms "
              f"light={t_light * 1e3:.2f} auto={rec['auto']['t'] * 1e3:.2f} timed={sum(x is not None for x in t)} "
              f"mismatch={mismatch} elapsed={el:.0f}s", flush=True)
        if mismatch:
            print(f"[sweep] {i}: OUTPUT SIZE DIFFERS BETWEEN CELLS", flush=True)
        if el > args.time_budget:
            print(f"[sweep] time budget reached after {n_done} instances", flush=True)
            break
    out.close()
    pool.terminate()
    h.close()


def _cell_estimates(h, est, dims):
    """Cost-model seconds of every cell and of its heavy part alone (the
    selector's candidate rule compares the latter with the light-only cell's
    estimate), with the handle's calibration."""
    import paper_2002_12459_amd as jp
    cal = h.get_calibration()
    return {"est": [float(e) for e in est], "heavy": [jp.heavy_cost(u, v, w, cal) for u, v, w in dims],
            "uvw": [list(d) for d in dims]}


def candidates(rec):
    """Cells the selector may take on a swept instance (all when the record
    holds no estimates)."""
    import paper_2002_12459_amd as jp
    if "heavy" not in rec:
        return [True] * N_CELLS
    return jp.selector_candidates(rec["est"][N_CELLS - 1], rec["heavy"])


def masked_argmin(scores, recs):
    """Per row, the candidate cell with the smallest score."""
    import numpy as np
    s = np.array(scores, dtype=np.float64, copy=True)
    for i, r in enumerate(recs):
        s[i, ~np.asarray(candidates(r))] = np.inf
    return s.argmin(axis=1)


def retime(args):
    """Time the cost model's plan again on instances already swept (after a
    change of the cost model or its calibration), and recompute the cells'
    cost-model estimates, keeping every other column."""
    import multiprocessing as mp

    recs = [r for r in load_records(args.data) if r.get("family", "zipf") == args.family and "t" in r]
    by_i = {r["i"]: r for r in recs}
    pool = mp.get_context("fork").Pool(args.workers)
    gen = pool.imap(functools.partial(_generate, family=args.family, lo=args.lo, hi=args.hi, jmax=args.jmax),
                    sorted(by_i))

    import numpy as np
    import torch

    import paper_2002_12459_amd as jp

    h = jp.Handle(0, selector=None, allocator="builtin")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()
    out = open(args.out, "a")
    t_start = time.perf_counter()
    for i, data, s, J in gen:
        rec = by_i[i]
        if data is None:
            continue
        R = tuple(T(a) for a in data)
        d1s = [c[0] for c in rec["cells"]]
        d2s = [c[1] for c in rec["cells"]]
        est, dims = h.plan_cells(*R, d1s, d2s)
        rec.update(_cell_estimates(h, est, dims))
        r = h.two_path_result(*R, strategy="auto")
        st = r.stats
        r.free()
        best = None
        for _ in range(args.reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = h.two_path_result(*R, strategy="auto")
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            r.free()
            best = dt if best is None else min(best, dt)
        if st["n_out"] != rec["n_out"]:
            print(f"[retime] {i}: OUTPUT SIZE DIFFERS ({st['n_out']} vs {rec['n_out']})", flush=True)
            rec["mismatch"] = rec.get("mismatch", 0) + 1
        old = rec["auto"]["t"]
        rec["auto"] = {"t": best, "d1": st["delta1"] if st["delta1"] != jp.DELTA_INF else None,
                       "d2": st["delta2"] if st["delta2"] != jp.DELTA_INF else None}
        out.write(json.dumps(rec) + "\n")
        out.flush()
        print(f"[retime] {i}: auto {old * 1e3:.2f} -> {best * 1e3:.2f} ms (d1={rec['auto']['d1']}, "
              f"d2={rec['auto']['d2']}) elapsed={time.perf_counter() - t_start:.0f}s", flush=True)
    out.close()
    pool.terminate()
    h.close()


# ---------------------------------------------------------------------------- train

def load_records(paths):
    """Clean records (every cell gave the same output size), one per
    (family, instance), the last one read winning."""
    recs = {}
    for p in paths:
        with open(p) as fh:
            for line in fh:
                line = line.strip()
                if line:
                    r = json.loads(line)
                    if not r.get("mismatch"):
                        recs[_key(r)] = r
    return [recs[k] for k in sorted(recs)]


def targets(rec, skip_ratio):
    """Per-cell log(t / t_best), capped at log(skip_ratio); untimed cells take the cap."""
    t = rec["t"]
    best = min(x for x in t if x is not None)
    cap = math.log(skip_ratio)
    return [cap if x is None else min(math.log(x / best), cap) for x in t]


def regret(rec, k, skip_ratio):
    t = rec["t"]
    best = min(x for x in t if x is not None)
    return skip_ratio if t[k] is None else t[k] / best


def _init_params(seed):
    """He-style initial weights (zero biases) in the library's flat layout."""
    import numpy as np
    rng = np.random.default_rng(seed)
    parts = [rng.normal(0, math.sqrt(2.0 / 16), 64 * 16), np.zeros(64),
             rng.normal(0, math.sqrt(2.0 / 64), 64 * 64), np.zeros(64),
             rng.normal(0, math.sqrt(1.0 / 64), N_CELLS * 64), np.zeros(N_CELLS)]
    return np.concatenate(parts).astype(np.float32)


def _summary(vals):
    import numpy as np
    a = np.asarray(vals, dtype=np.float64)
    return {"geomean": float(np.exp(np.log(a).mean())), "p50": float(np.percentile(a, 50)),
            "p90": float(np.percentile(a, 90)), "max": float(a.max()), "n": int(a.size)}


def train(args):
    import numpy as np
    import torch

    import paper_2002_12459_amd as jp

    recs = [r for r in load_records(args.data) if not r.get("rejected")]
    if args.table_out:
        import gzip
        keep = ("family", "i", "n", "s", "J", "n_out", "features", "t", "auto", "theory", "sqrtN", "est", "heavy",
                "uvw")
        with gzip.open(args.table_out, "wt") as fh:
            for r in recs:
                fh.write(json.dumps({k: r.get(k, "zipf" if k == "family" else None) for k in keep}) + "\n")
    hold = {"zipf": args.holdout_from, "clustered": args.holdout_from_clustered, "dense": args.holdout_from_dense}
    tr = [r for r in recs if r["i"] < hold[_key(r)[0]]]
    te = [r for r in recs if r["i"] >= hold[_key(r)[0]]]
    every = max(2, int(round(1.0 / args.val_frac)))  # every k-th training instance validates
    fit = [r for k, r in enumerate(tr) if k % every != every - 1]
    val = [r for k, r in enumerate(tr) if k % every == every - 1]
    X = lambda rs: np.asarray([r["features"] for r in rs], dtype=np.float32)
    Y = lambda rs: np.asarray([targets(r, args.skip_ratio) for r in rs], dtype=np.float32)
    mean = X(fit).mean(axis=0)
    scale = X(fit).std(axis=0)
    scale = np.where(scale > 1e-3, scale, 1.0).astype(np.float32)
    norm = lambda rs: torch.from_numpy((X(rs) - mean) / scale).cuda()

    h = jp.Handle(0, selector=None)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    xf, tf = norm(fit), dev(Y(fit))
    # errors near an instance's best cells decide its pick: weight each target
    # by exp(-target / tau) (1 at the best cell, 1/e at a cell e^tau times slower)
    wf = torch.exp(-tf / args.weight_tau) if args.weighted else torch.ones_like(tf)
    xv = norm(val)

    def picks(params, xs, rs):
        return masked_argmin(h.mlp_forward(params, xs).cpu().numpy(), rs)

    def geo_regret(params, rs, xs):
        ks = picks(params, xs, rs)
        return float(np.exp(np.mean([math.log(regret(r, int(k), args.skip_ratio)) for r, k in zip(rs, ks)])))

    # one run per seed; the parameters with the best validation regret over
    # all runs and checkpoints are kept
    best_p, best_val, best_seed, log = None, math.inf, None, []
    t0 = time.perf_counter()
    for seed in range(args.seed, args.seed + args.seeds):
        p = dev(_init_params(seed))
        m = torch.zeros_like(p)
        v = torch.zeros_like(p)
        grad = torch.empty_like(p)
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        for step in range(1, args.steps + 1):
            lr = args.lr * 0.5 * (1.0 + math.cos(math.pi * (step - 1) / args.steps))
            h.mlp_grad(p, xf, tf, wf, grad=grad, loss=loss)
            h.mlp_adam(p, m, v, grad, step, lr=lr)
            if step % args.eval_every == 0 or step == args.steps:
                vr = geo_regret(p, val, xv)
                log.append({"seed": seed, "step": step, "loss": float(loss.item()), "val_regret": vr})
                print(f"[train] seed {seed} step {step}: loss {loss.item():.4f} val geo-regret {vr:.4f}", flush=True)
                if vr < best_val:
                    best_val, best_p, best_seed = vr, p.clone(), seed
    t_train = time.perf_counter() - t0

    params = best_p.cpu().numpy().astype(np.float64)
    with open(args.out, "w") as fh:
        json.dump({"n_out": N_CELLS, "params": [float(x) for x in params], "mean": [float(x) for x in mean],
                   "scale": [float(x) for x in scale],
                   "meta": {"n_fit": len(fit), "n_val": len(val), "steps": args.steps, "lr": args.lr,
                            "skip_ratio": args.skip_ratio, "val_regret": best_val, "seed": best_seed,
                            "seeds": [args.seed, args.seed + args.seeds], "weighted": bool(args.weighted),
                            "weight_tau": args.weight_tau,
                            "holdout_from": args.holdout_from,
                            "holdout_from_clustered": args.holdout_from_clustered,
                            "holdout_from_dense": args.holdout_from_dense}}, fh)
    report = {"train_seconds": t_train, "log": log, "val_regret": best_val}
    if te:
        xt = norm(te)
        ks = picks(best_p, xt, te)
        best = lambda r: min(x for x in r["t"] if x is not None)
        rows = {"mlp": [regret(r, int(k), args.skip_ratio) for r, k in zip(te, ks)]}
        for name in ("auto", "theory", "sqrtN"):
            rows[name] = [r[name]["t"] / best(r) for r in te]
        rows["light_only"] = [regret(r, 64, args.skip_ratio) for r in te]
        fam = [_key(r)[0] for r in te]
        report["holdout"] = {k: _summary(vv) for k, vv in rows.items()}
        report["holdout_n"] = len(te)
        report["holdout_by_family"] = {
            f: {k: _summary([x for x, g in zip(vv, fam) if g == f]) for k, vv in rows.items()}
            for f in sorted(set(fam))}
        report["mlp_picks"] = {"light_only": int(sum(int(k) == 64 for k in ks)), "grid": int(sum(int(k) != 64 for k in ks))}
        for k, s_ in report["holdout"].items():
            print(f"[eval] {k:10s} geomean {s_['geomean']:.3f} p50 {s_['p50']:.3f} p90 {s_['p90']:.3f} "
                  f"max {s_['max']:.2f}", flush=True)
        for f, d in report["holdout_by_family"].items():
            print(f"[eval] {f}: mlp {d['mlp']['geomean']:.3f} auto {d['auto']['geomean']:.3f} "
                  f"light {d['light_only']['geomean']:.3f} (n={d['mlp']['n']})", flush=True)
    if args.report:
        with open(args.report, "w") as fh:
            json.dump(report, fh, indent=1)
    h.close()


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_2002_12459_amd.selector")
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("sweep")
    a.add_argument("--family", choices=["zipf", "clustered", "dense"], default="zipf")
    a.add_argument("--first", type=int, default=0)
    a.add_argument("--count", type=int, default=100)
    a.add_argument("--out", required=True)
    a.add_argument("--resume", nargs="*", default=[], help="earlier sweep files: skip their instances")
    a.add_argument("--lo", type=float, default=1e5)
    a.add_argument("--hi", type=float, default=2e6)
    a.add_argument("--jmax", type=float, default=1e9)
    a.add_argument("--reps", type=int, default=2)
    a.add_argument("--max-ops", type=float, default=4e14)
    a.add_argument("--max-bytes", type=float, default=16e9)
    a.add_argument("--skip-ratio", type=float, default=30.0)
    a.add_argument("--workers", type=int, default=12)
    a.add_argument("--time-budget", type=float, default=900.0)
    c = sub.add_parser("retime")
    c.add_argument("--data", nargs="+", required=True)
    c.add_argument("--family", choices=["zipf", "clustered", "dense"], default="dense")
    c.add_argument("--out", required=True)
    c.add_argument("--lo", type=float, default=1e5)
    c.add_argument("--hi", type=float, default=2e6)
    c.add_argument("--jmax", type=float, default=1e9)
    c.add_argument("--reps", type=int, default=2)
    c.add_argument("--workers", type=int, default=12)
    b = sub.add_parser("train")
    b.add_argument("--data", nargs="+", required=True)
    b.add_argument("--holdout-from", type=int, default=1000, help="first held-out zipf instance")
    b.add_argument("--holdout-from-clustered", type=int, default=450, help="first held-out clustered instance")
    b.add_argument("--holdout-from-dense", type=int, default=200, help="first held-out dense instance")
    b.add_argument("--val-frac", type=float, default=0.1)
    b.add_argument("--steps", type=int, default=4000)
    b.add_argument("--lr", type=float, default=3e-3)
    b.add_argument("--eval-every", type=int, default=100)
    b.add_argument("--skip-ratio", type=float, default=30.0)
    b.add_argument("--seed", type=int, default=0)
    b.add_argument("--weighted", type=int, default=1, help="weight targets by exp(-target / tau)")
    b.add_argument("--weight-tau", type=float, default=0.3)
    b.add_argument("--seeds", type=int, default=5, help="runs from seeds seed .. seed + seeds - 1")
    b.add_argument("--out", required=True)
    b.add_argument("--report", default=None)
    b.add_argument("--table-out", default=None, help="write the clean sweep table (gzip JSON lines) here")
    args = ap.parse_args(argv)
    if args.cmd == "sweep":
        sweep(args)
    elif args.cmd == "retime":
        retime(args)
    else:
        train(args)


if __name__ == "__main__":
    sys.exit(main())
