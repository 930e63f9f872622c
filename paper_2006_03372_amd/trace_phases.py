"""Split the rocprofv3 kernel trace of one host-driven decomposition into
the phases of a peeling round.

    python -m paper_2006_03372_amd.trace_phases run_kernel_trace.csv

Walks the dispatches in start order from the first peel_init_kernel and
assigns each kernel to a phase by the round structure of the host driver
(khc_peel.hip):
  clean    keymin / collect of the cleaning loop;
  h_bfs    multi-source BFS kernels after a collect (h-degree recomputes);
  round    select, the affected-set BFS levels, kill;
  hm1_bfs  BFS kernels after a kill ((h-1)-degree recomputes);
  bounds   lower bounds, finish, dirty-flag updates;
  readback the small device-to-host copies of the round counters.
The idle time before each kernel (the GPU waiting for the host) is charged
to the phase of that kernel.
"""
from __future__ import annotations

import csv
import sys
from collections import defaultdict

BFS_KERNELS = ("batch_reset_kernel", "batch_seed_kernel", "level_kernel", "batch_end_kernel", "scatter",
               "check_ids", "row_count")


def phase_of(name: str, state: str) -> tuple[str, str]:
    """(phase of this kernel, state after it)."""
    if "keymin_kernel" in name or "collect_kernel" in name:
        return "clean", "clean"
    if "select_kernel" in name or "affected_kernel" in name or "kill_kernel" in name:
        return "round", "round"
    if "lower_bound_kernel" in name or "finish_kernel" in name or "set_flag_kernel" in name:
        return "bounds", state
    if any(b in name for b in BFS_KERNELS):
        return {"clean": "h_bfs", "round": "hm1_bfs"}.get(state, "init"), state
    if "copyBuffer" in name:
        return "readback", state
    return "other", state


def split(path: str):
    rows = []
    with open(path) as f:
        for r in csv.DictReader(f):
            rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]))
    rows.sort()
    first = next(i for i, r in enumerate(rows) if "peel_init_kernel" in r[2])
    rows = rows[first:]
    busy, idle, count = defaultdict(float), defaultdict(float), defaultdict(int)
    state = "init"
    prev_end = rows[0][0]
    for start, end, name in rows:
        ph, state = phase_of(name, state)
        busy[ph] += (end - start) / 1e6
        idle[ph] += max(0, start - prev_end) / 1e6
        count[ph] += 1
        prev_end = max(prev_end, end)
    span = (rows[-1][1] - rows[0][0]) / 1e6
    return span, len(rows), busy, idle, count


def main():
    span, n, busy, idle, count = split(sys.argv[1])
    print(f"span {span:.1f} ms, {n} dispatches")
    print("| phase | dispatches | busy ms | idle ms | % of span |")
    print("|---|---|---|---|---|")
    for ph in sorted(busy, key=lambda p: -(busy[p] + idle[p])):
        print(f"| {ph} | {count[ph]} | {busy[ph]:.1f} | {idle[ph]:.1f} | {100 * (busy[ph] + idle[ph]) / span:.1f} |")


if __name__ == "__main__":
    main()
