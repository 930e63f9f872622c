"""Benchmark: h-hop degrees of every vertex of R-MAT scale 20 at h = 3.

One step = khdeg_compute over all vertices of the graph (every live vertex
gets its exact h-hop degree by the multi-source bounded BFS kernels).  The
throughput is in GTEPS: traversed edges, where the work of one vertex is the
number of arcs a scalar bounded BFS from it examines (khdeg_scanned_arcs),
divided by the step time, 10^9 per second.

After the timed steps, the exact (k,h)-core decomposition is timed once on
R-MAT scale 16 (edge factor 8) at h = 3 (--decompose-scale 20 times the
R-MAT-20 graph instead, which takes minutes).

Prints one JSON line.  Only one GPU is used; --gpus above 1 exits.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "h-hop BFS GTEPS + (k,h)-core wall time, R-MAT-20 h=3; learned-mode error"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def profiled_traffic(path=os.path.join(ROOT, "profiles", "level_kernel_rmat20_h3.md")):
    """HBM-side bytes per launch of the counting level from the committed
    rocprofv3 counter summary, or None when the BFS source has changed
    since the counters were taken."""
    import hashlib
    try:
        text = open(path).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        line = line.strip()
        for key in ("traffic_bytes_per_launch:", "source_sha256:"):
            if line.startswith(key):
                vals[key] = line.split(":", 1)[1].strip()
    if vals.get("source_sha256:") != level_source_hash():
        return None
    return float(vals["traffic_bytes_per_launch:"])


def level_source_hash():
    """sha256 over the sources the BFS level kernel is built from."""
    import hashlib
    h = hashlib.sha256()
    for name in ("khc_bfs.hip", "khc_level.h", "khc_internal.h"):
        with open(os.path.join(ROOT, "paper_2006_03372_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def decomposition(ctx, scale, edge_factor, h, log, tune=False):
    """One exact decomposition, host-driven rounds (wall time, statistics);
    with tune, the width and waves per CU come from khc_autotune (trials cut
    after 256 rounds, not timed)."""
    import torch
    from paper_2006_03372_amd import khcore, synth
    g = synth.rmat(scale, edge_factor, seed=1)
    gr = ctx.graph(g)
    ctx.set_option(khcore.OPT_DRIVER, 0)
    ctx.set_option(khcore.OPT_MAX_WIDTH, 32)
    ctx.set_option(khcore.OPT_WAVES_PER_CU, 8)
    tuned = None
    if tune:
        t0 = time.perf_counter()
        tuned = ctx.autotune(gr, h, rounds=256)
        log(f"autotune {time.perf_counter() - t0:.0f} s: width {tuned['width_words']}, "
            f"{tuned['waves_per_cu']} waves/CU")
    t0 = time.perf_counter()
    ctx.set_progress(lambda r, removed, level: log(f"  decomposition {time.perf_counter() - t0:.0f} s: "
                                                   f"round {r}, {removed} removed, level {level}"), 20000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    core, _, st = ctx.core(gr, h)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.set_progress(None)
    gr.close()
    setting = ("autotuned: W={}, {} waves/CU".format(tuned["width_words"], tuned["waves_per_cu"]) if tuned
               else "W=32, 8 waves/CU")
    return {"workload": f"khcore_decompose, R-MAT scale {scale} (ef {edge_factor}, seed 1), h={h}, "
                        f"bounded schedule, host-driven rounds, {setting}",
            "n": g.n, "edges": g.num_edges, "wall_s": round(wall, 3), "rounds": st["rounds"],
            "h_recomputes": st["h_recomputes"], "hm1_recomputes": st["hm1_recomputes"],
            "max_core": int(core.max().item())}


def cpu_baseline(g, h, budget_s=15.0, seed=0):
    """The oracle's scalar bounded BFS on a bounded random sample of the
    sources, single thread: traversed edges per second."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    deg = g.degrees()
    cand = np.flatnonzero(deg > 0).astype(np.uint32)
    rng = np.random.default_rng(seed)
    order = rng.permutation(cand)
    done_te, done_v, t_used = 0, 0, 0.0
    chunk = 16
    while t_used < budget_s and done_v < order.size:
        verts = order[done_v:done_v + chunk]
        t = time.perf_counter()
        _, te = oracle.hdeg_list(g, h, verts)
        t_used += time.perf_counter() - t
        done_te += int(te.sum())
        done_v += verts.size
    return {"value": done_te / t_used / 1e9, "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": f"{done_v} random non-isolated sources of the same graph, h={h}, "
                      f"scalar bounded BFS (oracle_hdeg_list), {t_used:.1f} s"}


def batched(ctx, count, h, log):
    """Batched decomposition of `count` Chung-Lu graphs (the first of the
    256-graph batch: n ~ U{500..20000}, mean degree ~ U[4,16], beta 2.5,
    seeds 7 + i): autotuned persistent kernel in a hipGraph, then the same
    graphs one at a time with host-driven rounds; the cores must agree."""
    import numpy as np
    import torch
    from paper_2006_03372_amd import khcore, synth
    graphs = synth.batch_chung_lu(256)[:count]
    bg = ctx.batch(graphs)
    t0 = time.perf_counter()
    tune = ctx.autotune(bg, h, rounds=32)
    t_tune = time.perf_counter() - t0
    log(f"autotune {t_tune:.1f} s: width {tune['width_words']} words, {tune['waves_per_cu']} waves/CU")
    ctx.set_progress(lambda r, removed, level: log(f"  batched {time.perf_counter() - t0:.0f} s: round {r}, "
                                                   f"{removed} removed"), 20000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    core, _, st = ctx.core(bg, h)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    ctx.set_progress(None)
    cb = core.cpu().numpy().view(np.uint32)
    bg.close()
    ctx.set_option(khcore.OPT_DRIVER, 0)
    ctx.set_option(khcore.OPT_MAX_WIDTH, 32)
    ctx.set_option(khcore.OPT_WAVES_PER_CU, 8)
    same, off, t_loop = True, 0, 0.0
    for i, g in enumerate(graphs):
        gr = ctx.graph(g)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c, _, _ = ctx.core(gr, h)
        torch.cuda.synchronize()
        t_loop += time.perf_counter() - t0
        same &= bool((c.cpu().numpy().view(np.uint32) == cb[off:off + g.n]).all())
        off += g.n
        gr.close()
        if (i + 1) % 32 == 0:
            log(f"  loop of single decompositions: {i + 1} graphs, {t_loop:.0f} s")
    return {"workload": f"{count} Chung-Lu graphs (n ~ U{{500..20000}}, mean ~ U[4,16], beta 2.5), h={h}",
            "vertices": int(off), "persistent_s": round(t_batch, 2), "rounds": st["rounds"],
            "autotune": {"width_words": tune["width_words"], "waves_per_cu": tune["waves_per_cu"],
                         "seconds": round(t_tune, 1)},
            "loop_of_singles_s": round(t_loop, 2), "speedup": round(t_loop / t_batch, 3), "cores_identical": same}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=int, default=20)
    ap.add_argument("--edge-factor", type=int, default=16)
    ap.add_argument("--h", type=int, default=3)
    ap.add_argument("--width", type=int, default=32)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--decompose-scale", type=int, default=16,
                    help="R-MAT scale of the timed decomposition (0: skip; 20 takes minutes)")
    ap.add_argument("--tune", action="store_true",
                    help="autotune width and waves per CU before the timed decomposition")
    ap.add_argument("--batched", type=int, default=0, metavar="COUNT",
                    help="also time the batched decomposition of COUNT Chung-Lu graphs (256 takes minutes)")
    ap.add_argument("--profile-pass", action="store_true",
                    help="one untimed-warmup-free step without the work count or CPU leg, for profilers")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this build measures the single-GPU path "
              "(--gpus 1); multi-GPU sharding is not implemented.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2006_03372_amd import khcore, synth

    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": nbytes, "copies": 3}))
        return
    if args.profile_pass:
        args.warmup, args.steps, args.no_cpu, args.decompose_scale = 0, 1, True, 0

    t = time.time()
    g = synth.rmat(args.scale, args.edge_factor, seed=1)
    log(f"generated R-MAT scale {args.scale} ef {args.edge_factor}: n={g.n} edges={g.num_edges} "
        f"({time.time() - t:.1f} s)")
    ctx = khcore.Context(0)
    ctx.set_option(khcore.OPT_MAX_WIDTH, args.width)
    gr = ctx.graph(g)
    h = args.h

    te_total = 0
    if not args.profile_pass:
        te = ctx.scanned_arcs(gr, h)
        torch.cuda.synchronize()
        te_total = int(te.cpu().numpy().view(np.uint64).sum())
        del te
        log(f"traversed-edge total at h={h}: {te_total:.4e}")

    for i in range(args.warmup):
        ctx.hdeg(gr, h)
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")

    ctx.set_option(khcore.OPT_PROFILE, 1)
    ctx.profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        out = ctx.hdeg(gr, h)
        torch.cuda.synchronize()
        log(f"step {i + 1}/{args.steps} done")
    t1 = time.perf_counter()
    prof = ctx.profile_read(reset=True)
    ctx.set_option(khcore.OPT_PROFILE, 0)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    gteps = te_total / (ms_per_step / 1e3) / 1e9

    last = prof["level_last"]
    avg_ms = last["ms"] / max(last["launches"], 1)
    avg_bytes = last["bytes"] / max(last["launches"], 1)
    achieved = avg_bytes / (avg_ms / 1e3) / 1e9
    traffic = profiled_traffic() if (args.scale, args.edge_factor, h, args.width) == (20, 16, 3, 32) else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else round(traffic / 1e9, 3),
                "traffic_unit": "GB per launch (rocprofv3 FETCH_SIZE+WRITE_SIZE, copy-calibrated)",
                "kernel": f"level_kernel<W,LAST> (counting level), {last['launches']} launches, "
                          f"avg {avg_ms:.3f} ms, {avg_bytes / 1e9:.3f} GB algorithmic per launch"
                          + ("" if traffic is None else
                             f"; rocprof FETCH+WRITE {traffic / 1e9:.3f} GB per launch = "
                             f"{traffic / (avg_ms / 1e3) / 1e9:.0f} GB/s")}

    result = {
        "metric": METRIC, "value": round(gteps, 2), "unit": "GTEPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"khdeg_compute, all vertices, R-MAT scale {args.scale} "
                               f"(ef {args.edge_factor}, a/b/c/d .57/.19/.19/.05, seed 1), h={h}",
                   "n": g.n, "edges": g.num_edges, "h": h, "max_width_words": args.width,
                   "traversed_edges": te_total},
        "kernels": {k: {"launches": v["launches"], "ms": round(v["ms"], 2)} for k, v in prof.items()},
        "roofline": roofline,
    }
    if not args.no_cpu:
        log("timing the CPU oracle on a sample ...")
        result["cpu_baseline"] = cpu_baseline(g, h)
    gr.close()
    if args.decompose_scale:
        ef = 16 if args.decompose_scale >= 20 else 8
        log(f"timing the decomposition of R-MAT scale {args.decompose_scale} at h={h} ...")
        result["decomposition"] = decomposition(ctx, args.decompose_scale, ef, h, log, tune=args.tune)
    if args.batched:
        log(f"timing the batched decomposition of {args.batched} graphs ...")
        result["batched"] = batched(ctx, args.batched, h, log)
    ctx.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
