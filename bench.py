"""Benchmark: h-hop degrees of every vertex of R-MAT scale 20 at h = 3, the
exact (k,h)-core decompositions of the same graph, and the learned-mode
error.

One step = khdeg_compute over all vertices of the graph (every live vertex
gets its exact h-hop degree by the multi-source bounded BFS kernels).  The
throughput is in GTEPS: traversed edges, where the work of one vertex is the
number of arcs a scalar bounded BFS from it examines (khdeg_scanned_arcs),
divided by the step time, 10^9 per second.

After the timed steps, outside the timed region: the exact (k,h)-core
decompositions of the same graph at h = 3 and 4 (wall time), and the
learned-mode error (the estimating mode on R-MAT-18 at h = 4 with a network
trained on R-MAT-16 graphs, against the exact decomposition).

Parity is checked in the same run, outside the timed region: the last
step's degrees against the CPU oracle on the sampled vertices the CPU
baseline computes, and the decompositions' core numbers and removal rounds
by the peeling-order certificate on sampled vertices.  A mismatch exits
with status 1.

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
LEVEL_PROFILE = os.path.join(ROOT, "profiles", "level_kernel_rmat20_h3.md")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def level_source_hash():
    """sha256 over the sources the BFS level kernel is built from."""
    import hashlib
    h = hashlib.sha256()
    for name in ("khc_bfs.hip", "khc_level.h", "khc_internal.h"):
        with open(os.path.join(ROOT, "paper_2006_03372_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def profiled_counters(path=LEVEL_PROFILE):
    """Calibrated HBM-side bytes per launch of the counting level from the
    committed rocprofv3 counter summary (machine-readable lines), or None
    when the BFS sources have changed since the counters were taken."""
    try:
        text = open(path).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        line = line.strip()
        if ":" in line:
            key, val = line.split(":", 1)
            vals[key.strip()] = val.strip()
    if vals.get("source_sha256") != level_source_hash() or "traffic_bytes_per_launch" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch"])


def profiled_traffic(path=LEVEL_PROFILE):
    return profiled_counters(path)


def level_bytes(g, W, last=True):
    """Per pull launch over the whole graph (no live mask), in bytes:
    compulsory = what must cross between HBM and the chip if every array the
    launch touches crosses once: per non-isolated row its schedule entry
    (4 B), row offset (8 B) and own words (8W B), the column ids (4 B per
    arc) and the frontier words once (8W B per non-isolated row); a
    non-counting level also writes the new words (frontier and visited,
    16W B per row at most, not counted here).
    modeled = the same rows plus one frontier gather of 8W B per arc, as if
    no gather hit a cache (the per-arc model of the level)."""
    import numpy as np
    rows = int(np.count_nonzero(g.degrees()))
    compulsory = rows * (4 + 8 + 8 * W) + g.nnz * 4 + rows * 8 * W
    modeled = rows * (4 + 8 + 8 * W) + g.nnz * (4 + 8 * W)
    return compulsory, modeled


def cpu_baseline(g, h, budget_s=10.0, seed=0):
    """The oracle's scalar bounded BFS on bounded random samples of the
    sources: traversed edges per second, first on one thread, then with the
    per-vertex loop split over every host thread this process may use
    (OMP_NUM_THREADS caps it).  The all-thread rate is the reported value.
    Also returns the sampled vertices and their oracle h-degrees for the
    parity check."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    deg = g.degrees()
    cand = np.flatnonzero(deg > 0).astype(np.uint32)
    rng = np.random.default_rng(seed)
    order = rng.permutation(cand)
    threads = oracle.host_threads()
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        threads = max(1, min(threads, int(os.environ["OMP_NUM_THREADS"])))
    done_v = 0
    got = []
    rates = {}
    for nthr, chunk in ((1, 16), (threads, 16 * threads)):
        te_sum, t_used, first = 0, 0.0, done_v
        while t_used < budget_s and done_v < order.size:
            verts = order[done_v:done_v + chunk]
            t = time.perf_counter()
            d, te = oracle.hdeg_list(g, h, verts, threads=nthr)
            t_used += time.perf_counter() - t
            got.append(d)
            te_sum += int(te.sum())
            done_v += verts.size
        rates[nthr] = (te_sum / t_used / 1e9, done_v - first, t_used)
    v1, n1, t1 = rates[1]
    vt, nt, tt = rates[threads]
    res = {"value": vt, "unit": "GTEPS", "cores": threads, "kind": "oracle", "value_1core": v1,
           "sample": f"{nt} random non-isolated sources of the same graph on {threads} threads ({tt:.1f} s), "
                     f"after {n1} others on 1 thread ({v1:.3f} GTEPS, {t1:.1f} s); h={h}, scalar bounded "
                     f"BFS per source (oracle_hdeg_list)"}
    return res, order[:done_v], np.concatenate(got)


def certificate_check(g, h, core, rnd, count, seed=3):
    """Peeling-order certificate of the oracle on `count` random
    non-isolated vertices (conditions (i), (ii)) and on all vertices (iii)."""
    import numpy as np
    import oracle
    rng = np.random.default_rng(seed)
    cand = np.flatnonzero(g.degrees() > 0).astype(np.uint32)
    verts = rng.choice(cand, size=min(count, cand.size), replace=False).astype(np.uint32)
    threads = oracle.host_threads()
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        threads = max(1, min(threads, int(os.environ["OMP_NUM_THREADS"])))
    t = time.perf_counter()
    fail = oracle.certificate(g, h, core, rnd, verts, threads=threads)
    return {"vertices": int(verts.size), "violations": [int(x) for x in fail],
            "cpu_s": round(time.perf_counter() - t, 1), "threads": threads}


def decomposition(ctx, g, desc, h, log, tune=False, cert=300):
    """One exact decomposition, host-driven rounds (wall time, statistics),
    then the certificate on `cert` sampled vertices (not timed); with tune,
    the width and waves per CU come from khc_autotune (trials cut after 256
    rounds, not timed)."""
    import numpy as np
    import torch
    from paper_2006_03372_amd import khcore
    gr = ctx.graph(g)
    ctx.set_option(khcore.OPT_DRIVER, 0)
    ctx.set_option(khcore.OPT_MAX_WIDTH, 32)
    ctx.set_option(khcore.OPT_WAVES_PER_CU, 16)
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
    core, rnd, st = ctx.core(gr, h, with_round=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.set_progress(None)
    gr.close()
    c = core.cpu().numpy().view(np.uint32)
    r = rnd.cpu().numpy().view(np.uint32)
    setting = ("autotuned: W={}, {} waves/CU".format(tuned["width_words"], tuned["waves_per_cu"]) if tuned
               else "W=32, 16 waves/CU")
    out = {"workload": f"khcore_decompose, {desc}, h={h}, bounded schedule with decremented (h-1)-degree bounds "
                       f"(KHC_OPT_SCHEDULE 3), host-driven rounds, {setting}",
           "n": g.n, "edges": g.num_edges, "wall_s": round(wall, 3), "rounds": st["rounds"],
           "h_recomputes": st["h_recomputes"], "hm1_recomputes": st["hm1_recomputes"],
           "max_core": int(c.max())}
    if cert:
        log(f"certificate on {cert} sampled vertices ...")
        out["certificate"] = certificate_check(g, h, c, r, cert)
    return out


def learned_leg(ctx, log, h=4, train_count=32, test_scale=18):
    """The metric's learned-mode error: the network trained on the exact
    h-degrees of peeling states of `train_count` R-MAT-16 graphs (seeds
    101..), then the estimating mode (khcore_decompose_approx) on R-MAT of
    `test_scale` against the exact decomposition: exact fraction, mean
    absolute core error, the paper's precision and the speedup."""
    import numpy as np
    import torch
    from paper_2006_03372_amd import khcore, learned, synth
    ctx.set_option(khcore.OPT_SCHEDULE, 3)
    ctx.set_option(khcore.OPT_MAX_WIDTH, 32)
    ctx.set_option(khcore.OPT_WAVES_PER_CU, 16)
    t0 = time.perf_counter()
    graphs = [synth.rmat(16, 8, seed=101 + i) for i in range(train_count)]
    X, t = learned.training_set(ctx, graphs, h)
    net = ctx.mlp(seed=7)
    losses = net.train(X, t, epochs=10, batch=4096, lr=2e-3, seed=1)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"learned mode: {X.shape[0]} training samples, {t_train:.0f} s")
    del X, t
    ef = 16 if test_scale >= 20 else 8
    g = synth.rmat(test_scale, ef, seed=1)
    gr = ctx.graph(g)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    exact, _, _ = ctx.core(gr, h)
    torch.cuda.synchronize()
    t_exact = time.perf_counter() - t0
    t0 = time.perf_counter()
    approx, _, st = ctx.core_approx(gr, h, net)
    torch.cuda.synchronize()
    t_approx = time.perf_counter() - t0
    gr.close()
    net.close()
    acc = learned.accuracy(exact.cpu().numpy().view(np.uint32), approx.cpu().numpy().view(np.uint32))
    return {"workload": f"khcore_decompose_approx, R-MAT scale {test_scale} (ef {ef}, seed 1), h={h}; network "
                        f"trained on {train_count} R-MAT scale 16 graphs (seeds 101..{100 + train_count})",
            "exact_fraction": round(acc["exact_fraction"], 5), "mae": round(acc["mae"], 3),
            "precision": round(acc["precision"], 6), "approx_s": round(t_approx, 2),
            "exact_s": round(t_exact, 2), "speedup_vs_exact": round(t_exact / t_approx, 3),
            "train_s": round(t_train, 1), "loss_last": float(losses[-1])}


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


def calibrate(kind, mib):
    """Counter calibration workloads of known size (run under rocprofv3
    --pmc): a plain device copy of `mib` MiB, or a gather of random 256-byte
    rows of a `mib` MiB table (as many rows as the table has; the indices
    add 8 bytes per row)."""
    import torch
    nbytes = mib << 20
    if kind == "copy":
        src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read": nbytes, "bytes_written": nbytes, "runs": 3}))
        return
    rows = nbytes // 256
    table = torch.ones((rows, 32), dtype=torch.int64, device="cuda")
    idx = torch.randint(0, rows, (rows,), dtype=torch.int64, device="cuda",
                        generator=torch.Generator(device="cuda").manual_seed(1))
    out = torch.empty_like(table)
    ms = []
    for _ in range(3):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        torch.index_select(table, 0, idx, out=out)
        b.record()
        b.synchronize()
        ms.append(a.elapsed_time(b))
    torch.cuda.synchronize()
    moved = rows * (256 + 8) + rows * 256
    # the rate of this access pattern on this GPU (random 256-byte rows read
    # with 16-byte loads, rows written in order), a practical ceiling beside
    # the HBM peak for the BFS level's gathers
    print(json.dumps({"calibration": "gather", "rows": rows, "bytes_read": rows * (256 + 8),
                      "bytes_written": rows * 256, "runs": 3, "ms": [round(x, 3) for x in ms],
                      "GBs_best": round(moved / (min(ms) * 1e-3) / 1e9, 1)}))


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
    ap.add_argument("--decompose-scale", type=int, default=20,
                    help="R-MAT scale of the timed decomposition (0: skip; 20: the benchmark graph itself)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-mode error leg")
    ap.add_argument("--decompose-h", default="3,4",
                    help="h values of the timed decompositions (the --h one is reported as 'decomposition')")
    ap.add_argument("--cert", type=int, default=300,
                    help="sampled vertices of the decomposition's certificate check (0: skip)")
    ap.add_argument("--tune", action="store_true",
                    help="autotune width and waves per CU before the timed decomposition")
    ap.add_argument("--batched", type=int, default=0, metavar="COUNT",
                    help="also time the batched decomposition of COUNT Chung-Lu graphs (256 takes minutes)")
    ap.add_argument("--profile-pass", action="store_true",
                    help="one untimed-warmup-free step without the work count or CPU leg, for profilers")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (counter calibration)")
    ap.add_argument("--calibrate-gather", type=int, default=0, metavar="MIB",
                    help="only gather random 256-byte rows of a MIB MiB table three times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: it measures the single-GPU path "
              "(--gpus 1); multi-GPU sharding is not implemented.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2006_03372_amd import khcore, synth

    if args.calibrate_copy:
        return calibrate("copy", args.calibrate_copy)
    if args.calibrate_gather:
        return calibrate("gather", args.calibrate_gather)
    if args.profile_pass:
        args.warmup, args.steps, args.no_cpu, args.decompose_scale = 0, 1, True, 0
        args.no_learned = True

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
    compulsory, modeled = level_bytes(g, args.width)
    counted = profiled_counters() if (args.scale, args.edge_factor, h, args.width) == (20, 16, 3, 32) else None
    if counted is not None:
        achieved = counted / (avg_ms / 1e3) / 1e9
        basis = "rocprofv3 FETCH_SIZE+WRITE_SIZE per launch (gather-calibrated), committed profile"
    else:
        achieved = compulsory / (avg_ms / 1e3) / 1e9
        basis = "compulsory bytes per launch (no counter profile for the current sources)"
    frac = achieved / HBM_PEAK_GBS
    if frac > 1.0:
        log(f"roofline fraction {frac:.3f} above 1: the byte count is wrong")
        sys.exit(1)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(frac, 4),
                "traffic": None if counted is None else round(counted / 1e9, 3),
                "traffic_unit": "GB per launch",
                "basis": basis,
                "kernel": f"level_kernel<{args.width},true> (counting level), {last['launches']} launches, "
                          f"avg {avg_ms:.3f} ms (HIP events on the library stream)",
                "compulsory_GB_per_launch": round(compulsory / 1e9, 3),
                "compulsory_GBs": round(compulsory / (avg_ms / 1e3) / 1e9, 1),
                "modeled_request_GB_per_launch": round(modeled / 1e9, 3),
                "modeled_request_GBs": round(modeled / (avg_ms / 1e3) / 1e9, 1)}

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
    bad = False
    if not args.no_cpu:
        log("timing the CPU oracle on a sample ...")
        base, verts, ref = cpu_baseline(g, h)
        result["cpu_baseline"] = base
        got = out.cpu().numpy().view(np.uint32)[verts]
        mism = int(np.count_nonzero(got != ref))
        result["parity"] = {"hdeg_sampled_vertices": int(verts.size), "hdeg_mismatches": mism}
        bad |= mism != 0
    gr.close()
    if args.decompose_scale:
        if args.decompose_scale == args.scale:
            dg, desc = g, f"R-MAT scale {args.scale} (ef {args.edge_factor}, seed 1)"
        else:
            ef = 16 if args.decompose_scale >= 20 else 8
            dg, desc = synth.rmat(args.decompose_scale, ef, seed=1), f"R-MAT scale {args.decompose_scale} " \
                                                                     f"(ef {ef}, seed 1)"
        for dh in [int(x) for x in args.decompose_h.split(",") if x]:
            log(f"timing the decomposition of {desc} at h={dh} ...")
            key = "decomposition" if dh == h else f"decomposition_h{dh}"
            result[key] = decomposition(ctx, dg, desc, dh, log, tune=args.tune, cert=args.cert)
            cert = result[key].get("certificate")
            bad |= bool(cert and any(cert["violations"]))
    if not args.no_learned:
        log("learned mode: training, then the estimating decomposition against exact ...")
        result["learned_mode"] = learned_leg(ctx, log)
    if args.batched:
        log(f"timing the batched decomposition of {args.batched} graphs ...")
        result["batched"] = batched(ctx, args.batched, h, log)
        bad |= not result["batched"]["cores_identical"]
    ctx.close()
    print(json.dumps(result), flush=True)
    if bad:
        log("PARITY FAILURE: see the parity / certificate fields")
        sys.exit(1)


if __name__ == "__main__":
    main()
