"""Autotuner for the sort's tile shapes.

Searches keys per lane (R), block-sort threads, cross-lane merge levels, the
merge tile and the merge kernel variant for one operation and size bucket,
timing every candidate with HIP events through the C ABI.  A candidate
counts only if its output is bit-identical to the default configuration's
output on the same input (the default itself is checked against the CPU
oracle by the test suite).  Winners are cached in JSON, keyed by
(architecture, CU count, operation, log2 size bucket):

    python -m paper_2409_03970_amd.tune --op sort --log2n 28
    python -m paper_2409_03970_amd.tune --op segmented --nseg 200000

The library itself never reads the cache; the allocating conveniences of the
Python binding (sort, sort_pairs, segmented_sort) use a cached entry when
they are called without explicit options.
"""
import argparse
import itertools
import json
import math
import os
import statistics
import sys

import torch

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")


def _key(op, log2n):
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(props, "gcnArchName", "gfx").split(":")[0]
    return f"{arch}:{props.multi_processor_count}:{op}:{int(log2n)}"


def load_cache(path=CACHE):
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def tuned_options(op, n, path=CACHE, two_way=False):
    """Cached options for (op, nearest size bucket) on this device, or None
    (two_way: the best configuration restricted to two-way passes)."""
    if not torch.cuda.is_available() or n <= 0:
        return None
    cache = load_cache(path)
    if not cache:
        return None
    log2n = max(0, int(round(math.log2(n))))
    best = None
    for k, v in cache.items():
        parts = k.split(":")
        if len(parts) != 4 or ":".join(parts[:3]) != _key(op, 0).rsplit(":", 1)[0]:
            continue
        d = abs(int(parts[3]) - log2n)
        o = v.get("two_way", {}).get("options") if two_way else v["options"]
        if o is not None and d <= 2 and (best is None or d < best[0]):
            best = (d, o)
    return dict(best[1]) if best else None


def candidates(op):
    shapes = [(16, 256), (16, 512), (16, 1024), (8, 1024), (32, 256), (32, 512)]
    if op == "sort":
        shapes.append((32, 1024))
    out = []
    pair_op = op in ("sort_pairs", "segmented_pairs")
    for (R, NT), K, TM, V, W in itertools.product(shapes, (6, 5, 4), (2048, 4096, 8192, 16384),
                                                  (2, 3), (2, 4)):
        if TM > 2 * R * NT:
            continue
        if TM == 16384 and (op != "sort" or W != 4):  # four-way key passes only
            continue
        if TM == 2048 and not (pair_op and W == 4):  # four-way pair passes only
            continue
        if op != "sort" and R * NT * 8 > 163840:
            continue
        if W == 4 and (V == 3 or (pair_op and TM not in (2048, 4096))):
            continue
        if op == "segmented_pairs" and (R, NT) == (16, 1024):  # pair tile + piece table > LDS
            continue
        out.append(dict(keys_per_lane=R, block_threads=NT, wave_levels=K + 1, merge_tile=TM,
                        merge_variant=V, merge_ways=W))
    return out


def _time(fn, reps):
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return statistics.median(ts)


def tune(op="sort", log2n=24, nseg=200000, seg_max=65536, reps=5, seed=0, path=CACHE,
         cands=None, verbose=True, dists=("uniform",), seg_min=1):
    """Times every candidate (and the defaults) on the operation's workload
    and records the fastest in the cache.  Segmented ops: nseg segments of
    sizes log-uniform in [seg_min, seg_max].  dists (sort / sort_pairs): the key
    distributions the objective sums over, each a separate input of 2^log2n
    keys; every candidate must reproduce the defaults' outputs exactly."""
    import paper_2409_03970_amd as hv
    from paper_2409_03970_amd import inputs
    dev = torch.device("cuda", torch.cuda.current_device())
    if op in ("segmented", "segmented_pairs"):
        pairs = op == "segmented_pairs"
        sizes = inputs.log_uniform_sizes(nseg, seg_min, seg_max, seed=seed)
        offs = inputs.offsets_from_sizes(sizes)
        n = int(offs[-1])
        d_off = offs.to(dev)
        max_seg = int(sizes.max())
        if tuple(dists) == ("uniform",):
            keys = inputs.keys(n, "uniform", seed=seed, device=dev)
            seg_id = torch.repeat_interleave(torch.arange(nseg, device=dev), sizes.to(dev))
            vals = (torch.arange(n, device=dev) - offs.to(dev)[seg_id]).to(torch.int32)
        else:  # each segment drawn from one of the given distributions
            pick = inputs.segment_distributions(nseg, seed=seed)
            idx = torch.tensor([inputs.DISTRIBUTIONS.index(d) for d in dists])
            keys, vals = inputs.segment_pairs(sizes, idx[pick % len(dists)], seed=seed,
                                              device=dev)
        out = torch.empty_like(keys)
        if pairs:  # each segment's values: the index inside the segment
            vout = torch.empty_like(vals)

        def run(o):
            ws = hv._workspace(hv.lib().hvms_segmented_workspace_bytes(
                n, nseg, max_seg, int(pairs), hv._opts(o)), dev)
            if pairs:
                return lambda: hv.hvms_segmented_sort_pairs_i32(keys, vals, out, vout, d_off, n,
                                                                max_seg, ws, opts=o)
            return lambda: hv.hvms_segmented_sort_i32(keys, out, d_off, n, max_seg, ws, opts=o)
        log2n = int(round(math.log2(n)))
        outputs = (out, vout) if pairs else (out,)
    elif op in ("sort", "sort_pairs"):
        n = 1 << log2n
        keyset = [inputs.keys(n, d, seed=seed, device=dev) for d in dists]
        vals = torch.arange(n, device=dev, dtype=torch.int32)
        outs = [torch.empty_like(keyset[0]) for _ in dists]
        vout = torch.empty_like(vals)

        def run(o):
            pairs = op == "sort_pairs"
            ws = hv._workspace(hv.lib().hvms_sort_workspace_bytes(n, int(pairs), hv._opts(o)), dev)

            def go():
                for keys, out in zip(keyset, outs):
                    if pairs:
                        hv.hvms_sort_pairs_i32(keys, vals, out, vout, ws, opts=o)
                    else:
                        hv.hvms_sort_i32(keys, out, ws, opts=o)
            return go
        outputs = tuple(outs) + ((vout,) if op == "sort_pairs" else ())
    else:
        raise ValueError(op)

    default = {}
    f = run(default)
    f()
    torch.cuda.synchronize()
    ref = [t.clone() for t in outputs]
    base_ms = _time(f, reps)
    results = [(base_ms, default)]
    for o in (cands or candidates(op)):
        f = run(o)
        f()
        torch.cuda.synchronize()
        if not all(torch.equal(a, b) for a, b in zip(outputs, ref)):
            raise RuntimeError(f"candidate {o} changed the output")
        ms = _time(f, reps)
        results.append((ms, o))
        if verbose:
            print(f"  {ms:8.3f} ms  {o}", flush=True)
    results.sort(key=lambda r: r[0])
    best_ms, best = results[0]
    cache = load_cache(path)
    entry = {"options": best, "ms": best_ms, "default_ms": base_ms, "n": n,
             "candidates": len(results)}
    entry["dists"] = list(dists)
    if op in ("segmented", "segmented_pairs"):
        entry["segments"] = [nseg, seg_min, seg_max]
    # the best configuration with two-way passes only, for comparison
    two = next((r for r in results if r[1].get("merge_ways", 2) == 2), None)
    if two is not None:
        entry["two_way"] = {"options": two[1], "ms": two[0]}
    cache[_key(op, log2n)] = entry
    with open(path, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    if verbose:
        print(f"{op} 2^{log2n}: best {best_ms:.3f} ms {best} (default {base_ms:.3f} ms)",
              flush=True)
    return best, best_ms, base_ms


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--op", default="sort",
                    choices=["sort", "sort_pairs", "segmented", "segmented_pairs"])
    ap.add_argument("--log2n", type=int, default=24)
    ap.add_argument("--nseg", type=int, default=200000)
    ap.add_argument("--seg-min", type=int, default=1)
    ap.add_argument("--seg-max", type=int, default=65536)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--dists", default="uniform",
                    help="comma-separated key distributions whose total time is minimised "
                         "(sort / sort_pairs), e.g. uniform,gaussian,sorted,reverse,distinct16,zipf")
    ap.add_argument("--path", default=CACHE, help="tuning cache to update (default: the package's)")
    a = ap.parse_args()
    tune(a.op, a.log2n, a.nseg, a.seg_max, a.reps, path=a.path, dists=tuple(a.dists.split(",")),
         seg_min=a.seg_min)


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    main()
