"""Scale sweep on one GPU: h-degree throughput and exact decomposition time
as the graph grows (the single-GPU part of the paper's scalability study,
Section V, Exp-6, on synthetic stand-ins for its datasets).

Workloads: R-MAT (a/b/c/d .57/.19/.19/.05, edge factor 8 below scale 20 and
16 from it, seed 1) at a range of scales, and Chung-Lu power-law graphs
(beta 2.5, mean degree 10, seed 1) at a range of sizes.  For each graph and
h it reports khdeg_compute over all vertices (median of several runs,
GTEPS by the scanned-arc count of khdeg_scanned_arcs) and, where it fits
the time budget, one exact decomposition (host-driven rounds, bounded
schedule).  Every run prints one JSON line.

    python -m paper_2006_03372_amd.sweep --rmat 16,18,20,22 --chung-lu 100000,400000 --h 2,3

With --schedules LIST it instead times one exact decomposition per listed
schedule (KHC_OPT_SCHEDULE 1 bounded, 2 local update, 0 plain, 3 bounded
with decremented (h-1)-degree bounds; plain at h = 2 only) of every graph
and h, and checks that all schedules give the same cores.  --driver 1 runs
those decompositions in the persistent kernel instead of host-driven rounds.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def measure(ctx, g, desc, h, steps, decompose):
    import torch
    gr = ctx.graph(g)
    out = {"graph": desc, "n": g.n, "edges": g.num_edges, "h": h}
    if steps > 0:
        te = ctx.scanned_arcs(gr, h)
        torch.cuda.synchronize()
        te_total = int(te.cpu().numpy().view(np.uint64).sum())
        del te
        ctx.hdeg(gr, h)
        torch.cuda.synchronize()
        times = []
        for _ in range(steps):
            t0 = time.perf_counter()
            ctx.hdeg(gr, h)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        t = float(np.median(times))
        out.update({"hdeg_ms": round(t * 1e3, 2), "traversed_edges": te_total, "gteps": round(te_total / t / 1e9, 1)})
    if decompose:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.set_progress(lambda r, removed, level: _log(f"  {desc} h={h}: {time.perf_counter() - t0:.0f} s, "
                                                        f"round {r}, {removed} removed"), 20000)
        core, _, st = ctx.core(gr, h)
        torch.cuda.synchronize()
        ctx.set_progress(None)
        out.update({"decompose_s": round(time.perf_counter() - t0, 3), "rounds": st["rounds"],
                    "max_core": int(core.max().item()), "h_recomputes": st["h_recomputes"]})
    gr.close()
    return out


def schedules(ctx, g, desc, h, order=(1, 2, 0), driver=0):
    import torch
    from . import khcore
    gr = ctx.graph(g)
    ref = None
    for sched in order:
        if sched == 0 and h >= 3:
            continue
        ctx.set_option(khcore.OPT_SCHEDULE, sched)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.set_progress(lambda r, removed, level: _log(f"  schedule {sched}: {time.perf_counter() - t0:.0f} s, "
                                                        f"round {r}, {removed} removed, level {level}"), 20000)
        core, _, st = ctx.core(gr, h)
        torch.cuda.synchronize()
        ctx.set_progress(None)
        t = time.perf_counter() - t0
        c = core.cpu().numpy()
        ref = c if ref is None else ref
        print(json.dumps({"graph": desc, "h": h, "schedule": sched, "driver": driver,
                          "s": round(t, 3), "rounds": st["rounds"],
                          "local_rounds": st["local_rounds"], "h_recomputes": st["h_recomputes"],
                          "hm1_recomputes": st["hm1_recomputes"], "same": bool((c == ref).all())}), flush=True)
    ctx.set_option(khcore.OPT_SCHEDULE, 3)  # the default
    gr.close()


def main():
    from . import khcore, synth
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--rmat", default="16,18,20", help="R-MAT scales")
    ap.add_argument("--chung-lu", default="", help="Chung-Lu sizes")
    ap.add_argument("--chung-lu-mean", type=float, default=10.0)
    ap.add_argument("--schedules", default="", help="comma list of schedules to time instead, e.g. 1,2,0")
    ap.add_argument("--h", default="2,3")
    ap.add_argument("--steps", type=int, default=3, help="timed khdeg_compute runs (0: decomposition only)")
    ap.add_argument("--decompose-max", type=int, default=400000,
                    help="decompose graphs with at most this many non-isolated vertices (h=2) "
                         "or a quarter of it (h>=3)")
    ap.add_argument("--driver", type=int, default=0, choices=(0, 1),
                    help="with --schedules: 0 host-driven rounds, 1 the persistent kernel")
    a = ap.parse_args()
    ctx = khcore.Context(0)
    ctx.set_option(khcore.OPT_DRIVER, a.driver)
    graphs = []
    for sc in [int(x) for x in a.rmat.split(",") if x]:
        ef = 16 if sc >= 20 else 8
        graphs.append((lambda sc=sc, ef=ef: synth.rmat(sc, ef, seed=1), f"R-MAT scale {sc} ef {ef}"))
    for n in [int(x) for x in a.chung_lu.split(",") if x]:
        m = a.chung_lu_mean
        graphs.append((lambda n=n, m=m: synth.chung_lu(n, m, 2.5, seed=1), f"Chung-Lu n={n} mean {m:g}"))
    for make, desc in graphs:
        t0 = time.time()
        g = make()
        live = int(np.count_nonzero(g.degrees()))
        _log(f"{desc}: n={g.n} edges={g.num_edges} ({time.time() - t0:.1f} s)")
        for h in [int(x) for x in a.h.split(",")]:
            if a.schedules:
                schedules(ctx, g, desc, h, tuple(int(x) for x in a.schedules.split(",")), a.driver)
                continue
            limit = a.decompose_max if h <= 2 else a.decompose_max // 4
            res = measure(ctx, g, desc, h, a.steps, live <= limit)
            print(json.dumps(res), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
