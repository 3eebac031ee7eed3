#!/usr/bin/env python3
"""Benchmark of the hybrid vectorized merge sort on one MI355X.

Workload (one "step"): sort 2^28 int32 keys for each of six seeded
distributions (uniform, gaussian, sorted, reverse, 16 distinct, zipf 1.1),
out of place from a pristine device copy, so every step sorts the same
inputs.  Inputs are resident in HBM before the timed region; the timed region
is exactly `--steps` steps bracketed by device synchronisation.

Printed: one JSON line with keys/s (whole job), HBM GB/s of the merge passes
measured live with HIP events recorded by the library around each merge
kernel inside the timed steps, the roofline of that kernel, and the CPU
oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import paper_2409_03970_amd as hv  # noqa: E402
from paper_2409_03970_amd import inputs  # noqa: E402

METRIC = "keys/sec + HBM GB/s per pass (int32, 1M–1G keys); learned vs binary co-rank"
HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    # name: (log2 n, distributions)
    "sort_2p28_six": (28, inputs.DISTRIBUTIONS),
    "sort_2p20_uniform": (20, ("uniform",)),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_events(k):
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(k)]
    for e in ev:            # materialise the underlying hipEvent_t
        e.record()
    torch.cuda.synchronize()
    return ev


def cpu_baseline(dists, log2n, seed=0, sample_log2=24):
    """The oracle (single thread, as written) on the first 2^sample_log2 keys
    of each distribution's input."""
    import oracle
    total_keys, total_s = 0, 0.0
    for d in dists:
        x = inputs.keys(1 << min(sample_log2, log2n), d, seed=seed, device="cpu").numpy()
        t0 = time.perf_counter()
        oracle.sort(x)
        total_s += time.perf_counter() - t0
        total_keys += x.size
    return {"value": total_keys / total_s, "unit": "keys/s", "cores": 1, "kind": "oracle",
            "sample": f"first 2^{min(sample_log2, log2n)} keys of each of the {len(dists)} "
                      f"inputs ({', '.join(dists)}), sorted once each by the single-threaded "
                      f"oracle merge sort; {total_s:.1f} s of CPU time"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="sort_2p28_six", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--keys-per-lane", type=int, default=0)
    ap.add_argument("--block-threads", type=int, default=0)
    ap.add_argument("--merge-tile", type=int, default=0)
    ap.add_argument("--wave-levels", type=int, default=0, help="levels + 1; 0 = default")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the sort is a single-GPU library)", file=sys.stderr)
        sys.exit(2)

    log2n, dists = WORKLOADS[args.workload]
    n = 1 << log2n
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    opts = {"keys_per_lane": args.keys_per_lane, "block_threads": args.block_threads,
            "merge_tile": args.merge_tile, "wave_levels": args.wave_levels}
    o_probe = hv._opts(opts)
    ws_bytes = hv.lib().hvms_sort_workspace_bytes(n, 0, o_probe)
    R = args.keys_per_lane or 16
    NT = args.block_threads or 512
    tile = R * NT
    passes = max(0, int(np.ceil(np.log2(max(1, -(-n // tile))))))

    log(f"generating {len(dists)} x 2^{log2n} keys")
    xs = [inputs.keys(n, d, seed=0, device=dev) for d in dists]
    out = torch.empty(n, dtype=torch.int32, device=dev)
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev)
    n_ev = 2 + 2 * passes
    ev_sets = [[make_events(n_ev) for _ in dists] for _ in range(args.steps)]

    def step(events=None):
        for i, x in enumerate(xs):
            o = dict(opts)
            if events is not None:
                o["events"] = events[i]
            hv.hvms_sort_i32(x, out, ws, opts=o)

    log("warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # parity spot check of the last output against the input (cheap properties)
    last = out[: min(n, 1 << 22)]
    assert bool((last[1:] >= last[:-1]).all()), "output not sorted"

    log("timed")
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record()
    for s in range(args.steps):
        step(ev_sets[s])
    t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = t0.elapsed_time(t1)
    ms_step = ms_total / args.steps
    keys_per_s = args.steps * len(dists) * n / (ms_total / 1e3)

    # per-kernel times from the library's trace events
    bs_ms, pass_ms = [], [[] for _ in range(passes)]
    for s in range(args.steps):
        for i in range(len(dists)):
            ev = ev_sets[s][i]
            bs_ms.append(ev[0].elapsed_time(ev[1]))
            for p in range(passes):
                pass_ms[p].append(ev[2 + 2 * p].elapsed_time(ev[3 + 2 * p]))
    merge_ms = float(np.mean([t for p in pass_ms for t in p])) if passes else float("nan")
    pass_bytes = 8.0 * n                      # read + write every key once
    achieved = pass_bytes / (merge_ms / 1e3) / 1e9 if passes else 0.0
    per_pass_gbs = [round(pass_bytes / (np.mean(p) / 1e3) / 1e9, 1) for p in pass_ms]

    per_dist = {}
    for i, d in enumerate(dists):
        t = []
        for s in range(args.steps):
            ev = ev_sets[s][i]
            t.append(ev[0].elapsed_time(ev[-1]) if passes else ev[0].elapsed_time(ev[1]))
        per_dist[d] = round(n / (np.mean(t) / 1e3) / 1e9, 3)

    rec = {
        "metric": METRIC,
        "value": keys_per_s,
        "unit": "keys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32",
        "data": "synthetic",
        "config": {
            "workload": f"sort of 2^{log2n} int32 keys, each of: {', '.join(dists)}",
            "n": n, "distributions": list(dists), "keys_per_lane": R, "block_threads": NT,
            "block_tile": tile, "merge_tile": args.merge_tile or 8192, "merge_passes": passes,
            "parallelism": "single GPU",
        },
        "roofline": {
            "kernel": "merge_pass_kernel (global merge pass)",
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "bytes_per_launch": pass_bytes, "avg_launch_ms": merge_ms,
        },
        "merge_pass_gbs": per_pass_gbs,
        "block_sort_ms": float(np.mean(bs_ms)) if bs_ms else None,
        "gkeys_per_s_by_distribution": per_dist,
        "wall_s_timed": wall,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        rec["cpu_baseline"] = cpu_baseline(dists, log2n)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
