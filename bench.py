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


# committed counter summaries per merge kernel (two-way, four-way) and the
# sources whose hash they record
COUNTERS = {
    2: (os.path.join(ROOT, "profiles", "merge_pass_counters_sort_2p28_six.md"),
        ("paper_2409_03970_amd/csrc/merge_common.h", "paper_2409_03970_amd/csrc/merge.hip",
         "paper_2409_03970_amd/csrc/common.h")),
    4: (os.path.join(ROOT, "profiles", "merge4_pass_counters_sort_2p28_six.md"),
        ("paper_2409_03970_amd/csrc/merge_common.h", "paper_2409_03970_amd/csrc/merge4.hip",
         "paper_2409_03970_amd/csrc/common.h")),
}


def counter_traffic(ways=2):
    """HBM bytes per merge launch from the committed FETCH_SIZE / WRITE_SIZE
    runs of that merge kernel, or None once its sources differ from the ones
    the counters were taken on."""
    import hashlib
    try:
        path, sources = COUNTERS[ways]
        text = open(path).read()
        h = hashlib.sha256(b"".join(open(os.path.join(ROOT, p), "rb").read()
                                    for p in sources)).hexdigest()[:16]
        fields = dict(line.split(":", 1) for line in text.splitlines()
                      if line.startswith(("merge_pass_traffic_bytes:", "kernel_source_sha256_16:")))
        if fields["kernel_source_sha256_16"].split()[0] != h:
            return None
        return float(fields["merge_pass_traffic_bytes"])
    except (OSError, KeyError, ValueError):
        return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_events(k):
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(k)]
    for e in ev:            # materialise the underlying hipEvent_t
        e.record()
    torch.cuda.synchronize()
    return ev


def _host_cpu():
    """Host CPU model name and the cores this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return model, usable, os.cpu_count()


def cpu_baseline(dists, log2n, seed=0):
    """The oracle as written (a single-threaded merge sort) on the full
    headline inputs: one sort of each distribution's 2^log2n keys, the six
    sorts running at once on six host threads, so the measured rate is the
    host's six-core rate for this workload.  Beside it: the per-sort
    single-thread rate, the 2^20-key uniform input (five sorts, one thread),
    and the C++ library's std::sort on the same full inputs (context)."""
    import concurrent.futures
    import oracle
    dev = torch.device("cuda", 0)
    xs = [inputs.keys(1 << log2n, d, seed=seed, device=dev).cpu().numpy() for d in dists]
    torch.cuda.empty_cache()

    def timed(fn, x):
        t0 = time.perf_counter()
        fn(x)
        return time.perf_counter() - t0

    def concurrent_run(fn):
        with concurrent.futures.ThreadPoolExecutor(len(xs)) as ex:
            w0 = time.perf_counter()
            per = list(ex.map(lambda x: timed(fn, x), xs))
            return time.perf_counter() - w0, per

    oracle.lib()
    oracle.std_sort(xs[0][:16])                     # load both libraries first
    wall, per = concurrent_run(oracle.sort)
    n_all = sum(x.size for x in xs)
    small = inputs.keys(1 << 20, "uniform", seed=seed, device=dev).cpu().numpy()
    t_small = [timed(oracle.sort, small) for _ in range(5)]
    std_wall, std_per = concurrent_run(oracle.std_sort)
    model, usable, total = _host_cpu()
    return {"value": n_all / wall, "unit": "keys/s", "cores": len(xs), "kind": "oracle",
            "sample": f"the full headline workload: one sort of each of the {len(xs)} inputs of "
                      f"2^{log2n} keys ({', '.join(dists)}) by the single-threaded oracle merge "
                      f"sort, the {len(xs)} sorts at once on {len(xs)} host threads; "
                      f"{wall:.1f} s wall",
            "per_sort_single_thread_keys_per_s": round(n_all / sum(per), 1),
            "per_distribution_s": {d: round(t, 2) for d, t in zip(dists, per)},
            "uniform_2p20_single_thread_keys_per_s": round(small.size / float(np.median(t_small)), 1),
            "uniform_2p20_s": [round(t, 4) for t in t_small],
            "context_std_sort": {"value": n_all / std_wall, "unit": "keys/s", "cores": len(xs),
                                 "per_sort_single_thread_keys_per_s": round(n_all / sum(std_per), 1),
                                 "wall_s": round(std_wall, 2)},
            "host_cpu_model": model, "host_cores_usable": usable, "host_cores_total": total}


def merge_passes(n, tile, ways=2):
    """Merge launches of a sort: the two-way levels first, then (ways = 4)
    one launch per two levels."""
    levels = max(0, int(np.ceil(np.log2(max(1, -(-n // tile))))))
    return levels - (levels // 2 if ways == 4 else 0)


def four_way_bench(x, ref_out, opts):
    """The opt-in four-way merge passes (two merge levels per trip through
    HBM) against the two-way default on the same input."""
    o4 = dict(opts, merge_ways=4, merge_variant=0)
    n = x.numel()
    tile = (o4.get("keys_per_lane") or 16) * (o4.get("block_threads") or 512)
    passes = merge_passes(n, tile, 4)
    ws = torch.empty(max(hv.lib().hvms_sort_workspace_bytes(n, 0, hv._opts(o4)), 1),
                     dtype=torch.uint8, device=x.device)
    out = torch.empty_like(x)
    ms = _median_ms(lambda: hv.hvms_sort_i32(x, out, ws, opts=o4))
    equal = bool(torch.equal(out, ref_out))
    ev = make_events(2 + 2 * passes)
    hv.hvms_sort_i32(x, out, ws, opts=dict(o4, events=ev))
    torch.cuda.synchronize()
    merge = [ev[2 + 2 * p].elapsed_time(ev[3 + 2 * p]) for p in range(passes)]
    # launches between two merge launches: the co-rank grid and the
    # four-way co-rank records of the next pass
    corank = [ev[1 + 2 * p].elapsed_time(ev[2 + 2 * p]) for p in range(passes)]
    levels = max(0, int(np.ceil(np.log2(max(1, -(-n // tile))))))
    p2 = levels - 2 * (levels // 2)  # two-way launches come first
    four = merge[p2:]
    return {"ms": round(ms, 3), "gkeys_per_s": round(n / ms / 1e6, 3), "merge_launches": passes,
            "two_way_launches": p2, "options": o4, "merge_ms": [round(t, 3) for t in merge],
            "corank_ms": [round(t, 3) for t in corank],
            "four_way_pass_gbs_mean": round(8.0 * n / (np.mean(four) / 1e3) / 1e9, 1) if four else None,
            "block_sort_ms": round(ev[0].elapsed_time(ev[1]), 3), "equal_to_two_way": equal}


def key_types_bench(n):
    """uint32 and float32 keys (tuned sort options) against int32 on the
    same number of keys; the key map is fused into the first and last
    launches, so the rates should match.  Then int64, uint64 and float64
    keys (tuned key-value options: 64-bit keys run on those kernels)."""
    dev = torch.device("cuda", 0)
    from paper_2409_03970_amd import tune
    opts = tune.tuned_options("sort", n) or {}
    ws = hv._workspace(hv.lib().hvms_sort_workspace_bytes(n, 0, hv._opts(opts)), dev)
    g = torch.Generator(device=dev).manual_seed(0)
    res = {}
    bits = torch.randint(-2**31, 2**31 - 1, (n,), dtype=torch.int32, device=dev, generator=g)
    out = torch.empty_like(bits)
    cases = (("int32", bits, out, hv.hvms_sort_i32),
             ("uint32", bits.view(torch.uint32), out.view(torch.uint32), hv.hvms_sort_u32))
    for name, x, y, fn in cases:
        ms = _median_ms(lambda: fn(x, y, ws, opts=opts))
        mono = out ^ (-2**31) if name == "uint32" else out   # unsigned order as signed
        res[name] = {"ms": round(ms, 3), "gkeys_per_s": round(n / ms / 1e6, 3),
                     "sorted": bool((mono[1:] >= mono[:-1]).all())}
    f = torch.randn(n, device=dev, generator=g) * 1e3
    f[f == 0] = 1.0
    fo = torch.empty_like(f)
    ms = _median_ms(lambda: hv.hvms_sort_f32(f, fo, ws, opts=opts))
    res["float32"] = {"ms": round(ms, 3), "gkeys_per_s": round(n / ms / 1e6, 3),
                      "sorted": bool((fo[1:] >= fo[:-1]).all())}
    del ws, bits, out, f, fo
    torch.cuda.empty_cache()
    # 64-bit keys run on the key-value kernels (16 bytes per key per pass)
    o64 = tune.tuned_options("sort_pairs", n) or {}
    tile = (o64.get("keys_per_lane") or 16) * (o64.get("block_threads") or 512)
    passes = merge_passes(n, tile, o64.get("merge_ways") or 2)
    ws = hv._workspace(hv.lib().hvms_sort64_workspace_bytes(n, hv._opts(o64)), dev)
    x = torch.randint(-2**63, 2**63 - 1, (n,), dtype=torch.int64, device=dev, generator=g)
    y = torch.empty_like(x)
    for name, fn, xv, yv in (("int64", hv.hvms_sort_i64, x, y),
                             ("uint64", hv.hvms_sort_u64, x.view(torch.uint64),
                              y.view(torch.uint64)),
                             ("float64", hv.hvms_sort_f64, None, None)):
        if name == "float64":
            del x, y
            xv = torch.randn(n, dtype=torch.float64, device=dev, generator=g) * 1e3
            xv[xv == 0] = 1.0
            yv = torch.empty_like(xv)
        ms = _median_ms(lambda: fn(xv, yv, ws, opts=o64))
        ev = make_events(2 + 2 * passes)
        fn(xv, yv, ws, opts=dict(o64, events=ev))
        torch.cuda.synchronize()
        pm = [ev[2 + 2 * p].elapsed_time(ev[3 + 2 * p]) for p in range(passes)]
        mono = yv.view(torch.int64)
        if name == "uint64":
            mono = mono ^ (-2**63)                    # unsigned order as signed
        elif name == "float64":
            mono = yv
        res[name] = {"ms": round(ms, 3), "gkeys_per_s": round(n / ms / 1e6, 3),
                     "merge_pass_gbs_mean": round(16.0 * n / (np.mean(pm) / 1e3) / 1e9, 1)
                     if pm else None,
                     "sorted": bool((mono[1:] >= mono[:-1]).all())}
    res["options_64bit"] = o64
    return res


def merge_table3_bench(n):
    """Table 3 analog: the two per-thread mergers of a merge pass -- serial
    (the serial part of the hybrid merger) and the bitonic network in
    registers -- at VT = 8, 16 and 32 outputs per thread (merge tiles 2048,
    8192, 16384), on one pass over 2^28 uniform keys in sorted runs of
    16,384.  Times the whole pass (co-rank kernel + merge kernel)."""
    dev = torch.device("cuda", 0)
    base = {"keys_per_lane": 32, "block_threads": 512}
    res = {}
    for dist in ("uniform", "sorted", "distinct16"):
        x = inputs.keys(n, dist, seed=3, device=dev)
        runs = hv.sort_runs(x, 14, opts=base)
        del x
        out = torch.empty_like(runs)
        ref = None
        for tm, vt in ((2048, 8), (8192, 16), (16384, 32)):
            for name, var in (("serial", 2), ("bitonic", 4)):
                o = dict(base, merge_tile=tm, merge_variant=var)
                ws = hv._workspace(hv.lib().hvms_merge_workspace_bytes(n, 16384, hv._opts(o)), dev)
                ms = _median_ms(lambda: hv.hvms_merge_pass_i32(runs, out, 16384, ws, opts=o))
                if ref is None:
                    ref = out.clone()
                res[f"{dist}_2x{vt}_{name}"] = {
                    "ms": round(ms, 4), "gbs": round(8.0 * n / (ms / 1e3) / 1e9, 1),
                    "equal": bool(torch.equal(out, ref))}
        del runs, out, ref
        torch.cuda.empty_cache()
    return res


_M64 = (1 << 64) - 1


def _s64(c):
    """A 64-bit constant as the signed value torch's int64 holds."""
    return c - (1 << 64) if c >= 1 << 63 else c


def gpu_multiset_hash(t, chunk=1 << 26):
    """Sum over the keys of a 64-bit mix of each key (SplitMix64's output
    function), modulo 2^64, on the device: equal for any two arrangements of
    one multiset, different with probability about 2^-64 otherwise.  A
    certificate that a sort output is a permutation of its input."""
    total = torch.zeros((), dtype=torch.int64, device=t.device)
    for a in range(0, t.numel(), chunk):
        z = t[a:a + chunk].to(torch.int64) & 0xFFFFFFFF
        z = z + _s64(0x9E3779B97F4A7C15)
        z = (z ^ ((z >> 30) & ((1 << 34) - 1))) * _s64(0xBF58476D1CE4E5B9)
        z = (z ^ ((z >> 27) & ((1 << 37) - 1))) * _s64(0x94D049BB133111EB)
        z = z ^ ((z >> 31) & ((1 << 33) - 1))
        total += z.sum()
    return int(total.item()) & _M64


def sort_certificate(x, y):
    """y is nondecreasing and a permutation of x (multiset hash)."""
    return bool((y[1:] >= y[:-1]).all()) and gpu_multiset_hash(x) == gpu_multiset_hash(y)


def _median_ms(fn, reps=3):
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


def _mode_stats(x, out, ws, opts, params, mode, radius=12):
    """One co-rank mode on one input: sort time (median), the co-rank phase
    of every merge pass (library events, a run without statistics), then
    the co-rank statistics of one more run (mean and p99 probes; for the
    predicting modes fallback rate, mean / p99 bound / max |error|)."""
    n = x.numel()
    st = torch.zeros(hv.STATS_WORDS, dtype=torch.int64, device=x.device)
    o = dict(opts, corank_mode=mode, radius_log2=radius, cdf_params=params)
    ms = _median_ms(lambda: hv.hvms_sort_i32(x, out, ws, opts=o))
    R = opts.get("keys_per_lane") or 16
    NT = opts.get("block_threads") or 512
    passes = merge_passes(n, R * NT, opts.get("merge_ways") or 2)
    ev = make_events(2 + 2 * passes)
    hv.hvms_sort_i32(x, out, ws, opts=dict(o, events=ev))
    torch.cuda.synchronize()
    cr_ms = [ev[1 + 2 * p].elapsed_time(ev[2 + 2 * p]) for p in range(passes)]
    o["stats"] = st
    hv.hvms_sort_i32(x, out, ws, opts=o)
    torch.cuda.synchronize()
    c = st.cpu().tolist()
    s = hv.corank_stats(c)
    r = {"ms": round(ms, 3), "gkeys_per_s": round(n / ms / 1e6, 3),
         "probes_per_corank": s["probes_mean"], "probes_p99": s["probes_p99"],
         "corank_ms_per_pass": [round(t, 4) for t in cr_ms],
         "corank_ms_total": round(sum(cr_ms), 3)}
    if mode != hv.CORANK_BINARY:
        r.update(fallback_rate=s.get("fallback_rate"), mean_abs_err=s.get("abs_err_mean"),
                 abs_err_p99_at_most=s.get("abs_err_p99_at_most"), max_err=s.get("max_err"),
                 predicted_coranks=s.get("predicted", 0))
    return r


def corank_modes(xs, dists, out, ws, opts, opts4=None, ws4=None):
    """Binary vs learned vs linear co-rank on the same 2^28 inputs in the
    best two-way shape (the two-way co-rank is the one the model predicts),
    and with opts4 the co-rank time of the tuned four-way shape, whose
    co-ranks are selected in the runs directly in every mode."""
    res = {}
    for x, d in zip(xs, dists):
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        params = hv.fit_cdf_model(x, frac=0.01, steps=300, batch=65536, lr=3e-3, seed=1)
        t1.record()
        torch.cuda.synchronize()
        r = {"train_ms": round(t0.elapsed_time(t1), 2)}
        for name, mode in (("binary", hv.CORANK_BINARY), ("learned", hv.CORANK_LEARNED),
                           ("linear", hv.CORANK_LINEAR)):
            r[name] = _mode_stats(x, out, ws, opts, params, mode)
        if opts4 is not None:
            r["four_way"] = _mode_stats(x, out, ws4, opts4, params, hv.CORANK_BINARY)
        res[d] = r
    return res


def pairs_bench(n):
    """Key-value sort of 2^28 (key, original index) pairs."""
    dev = torch.device("cuda", 0)
    k, v = inputs.pairs(n, "uniform", seed=0, device=dev)
    ko, vo = torch.empty_like(k), torch.empty_like(v)
    from paper_2409_03970_amd import tune
    opts = tune.tuned_options("sort_pairs", n) or {}
    ws = hv._workspace(hv.lib().hvms_sort_workspace_bytes(n, 1, hv._opts(opts)), dev)
    tile = (opts.get("keys_per_lane") or 16) * (opts.get("block_threads") or 512)
    passes = merge_passes(n, tile, opts.get("merge_ways") or 2)
    ev = make_events(2 + 2 * passes)
    ms = _median_ms(lambda: hv.hvms_sort_pairs_i32(k, v, ko, vo, ws, opts=opts))
    hv.hvms_sort_pairs_i32(k, v, ko, vo, ws, opts=dict(opts, events=ev))
    torch.cuda.synchronize()
    pm = [ev[2 + 2 * p].elapsed_time(ev[3 + 2 * p]) for p in range(passes)]
    # certificate: keys nondecreasing and every payload still points at its key
    ok = bool((ko[1:] >= ko[:-1]).all()) and bool(torch.equal(k[vo.long()], ko))
    return {"ms": round(ms, 3), "gkeys_per_s": round(n / ms / 1e6, 3), "options": opts,
            "merge_pass_gbs_mean": round(16.0 * n / (np.mean(pm) / 1e3) / 1e9, 1) if pm else None,
            "certificate_ok": ok}


def by_key_bench(n):
    """Stable sort of 2^28 uniform int32 keys carrying 64-bit payloads (the
    payload is the input index, which makes the certificate cheap)."""
    dev = torch.device("cuda", 0)
    k = inputs.keys(n, "uniform", seed=0, device=dev)
    v = torch.arange(n, dtype=torch.int64, device=dev)
    ko, vo = torch.empty_like(k), torch.empty_like(v)
    from paper_2409_03970_amd import tune
    opts = tune.tuned_options("sort_pairs", n) or {}
    ws = hv._workspace(hv.lib().hvms_sort_by_key_workspace_bytes(n, hv._opts(opts)), dev)
    ms = _median_ms(lambda: hv.hvms_sort_by_key_i32_p64(k, v, ko, vo, ws, opts=opts))
    # certificate: keys nondecreasing, each payload still points at its key,
    # and equal keys keep their input order
    ok = (bool((ko[1:] >= ko[:-1]).all()) and bool(torch.equal(k[vo], ko))
          and bool(((ko[1:] > ko[:-1]) | (vo[1:] > vo[:-1])).all()))
    return {"ms": round(ms, 3), "gkeys_per_s": round(n / ms / 1e6, 3), "options": opts,
            "certificate_ok": ok}


def sort_dist_bench(dist, reps=5, log2n=28):
    """2^log2n keys of one distribution, the tuned options, `reps` timed sorts
    (a short run for kernel traces and counters of one input)."""
    dev = torch.device("cuda", 0)
    n = 1 << log2n
    x = inputs.keys(n, dist, seed=0, device=dev)
    out = torch.empty_like(x)
    from paper_2409_03970_amd import tune
    opts = tune.tuned_options("sort", n) or {}
    ws = hv._workspace(hv.lib().hvms_sort_workspace_bytes(n, 0, hv._opts(opts)), dev)
    ms = _median_ms(lambda: hv.hvms_sort_i32(x, out, ws, opts=opts), reps=reps)
    return {"dist": dist, "n": n, "ms": round(ms, 3), "gkeys_per_s": round(n / ms / 1e6, 2),
            "options": opts, "certified": sort_certificate(x, out)}


def batched_bench(per_array=True):
    """200,000 arrays, sizes log-uniform in [1, 65536]: one batched call
    (eager and as a replayed HIP graph) against one plain sort per array."""
    dev = torch.device("cuda", 0)
    sizes = inputs.log_uniform_sizes(200000, 1, 65536, seed=0)
    offs = inputs.offsets_from_sizes(sizes)
    n = int(offs[-1])
    d_off = offs.to(dev)
    max_seg = int(sizes.max())
    k = inputs.keys(n, "uniform", seed=3, device=dev)
    out = torch.empty_like(k)
    from paper_2409_03970_amd import tune
    opts = tune.tuned_options("segmented", n) or {}
    ws = hv._workspace(hv.lib().hvms_segmented_workspace_bytes(n, sizes.numel(), max_seg, 0,
                                                                 hv._opts(opts)), dev)
    eager_ms = _median_ms(lambda: hv.hvms_segmented_sort_i32(k, out, d_off, n, max_seg, ws,
                                                             opts=opts))
    ref = out.clone()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            hv.hvms_segmented_sort_i32(k, out, d_off, n, max_seg, ws, opts=opts)
    torch.cuda.current_stream().wait_stream(s)
    graph_ms = _median_ms(g.replay)
    graph_ok = bool(torch.equal(out, ref))
    if not per_array:
        return {"keys": n, "segments": int(sizes.numel()), "options": opts,
                "batched_ms": round(eager_ms, 3), "graph_ms": round(graph_ms, 3),
                "graph_replay_equal": graph_ok}
    # plain sort per array, same inputs, one ABI call each (workspace sized once)
    ws2 = hv._workspace(hv.lib().hvms_sort_workspace_bytes(max_seg, 0, None), dev)
    L = hv.lib()
    st = hv._stream(None)
    kp, op = k.data_ptr(), out.data_ptr()
    wp, wb = (ws2.data_ptr(), ws2.numel()) if ws2 is not None else (None, 0)
    offl = offs.tolist()

    def per_array():
        for i in range(len(offl) - 1):
            m = offl[i + 1] - offl[i]
            if m:
                L.hvms_sort_i32(hv._vp(kp + 4 * offl[i]), hv._vp(op + 4 * offl[i]), m,
                                hv._vp(wp), wb, st, None)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    per_array()
    b.record()
    torch.cuda.synchronize()
    per_ms = a.elapsed_time(b)
    per_ok = bool(torch.equal(out, ref))
    return {"keys": n, "segments": int(sizes.numel()), "options": opts,
            "batched_ms": round(eager_ms, 3), "batched_gkeys_per_s": round(n / eager_ms / 1e6, 2),
            "graph_ms": round(graph_ms, 3), "graph_gkeys_per_s": round(n / graph_ms / 1e6, 2),
            "per_array_plain_sort_ms": round(per_ms, 1),
            "per_array_gkeys_per_s": round(n / per_ms / 1e6, 3),
            "graph_replay_equal": graph_ok, "per_array_equal": per_ok}


def learned_bench():
    """2^30 keys from the 8-Gaussian + lognormal mixture: co-rank modes."""
    dev = torch.device("cuda", 0)
    n = 1 << 30
    x = inputs.keys(n, "mixture", seed=0, device=dev)
    out = torch.empty_like(x)
    from paper_2409_03970_amd import tune
    opts = tune.tuned_options("sort", n) or {}
    ws = hv._workspace(hv.lib().hvms_sort_workspace_bytes(n, 0, hv._opts(opts)), dev)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    params = hv.fit_cdf_model(x, frac=0.01, steps=400, batch=65536, lr=3e-3, seed=2)
    t1.record()
    torch.cuda.synchronize()
    res = {"n": n, "train_ms_incl_sample_sort": round(t0.elapsed_time(t1), 2)}
    ref = None
    for name, mode in (("binary", hv.CORANK_BINARY), ("learned", hv.CORANK_LEARNED),
                       ("linear", hv.CORANK_LINEAR)):
        res[name] = _mode_stats(x, out, ws, opts, params, mode, radius=13)
        # each mode's output as it is produced: the binary one certified
        # (nondecreasing, a permutation of the input), the others identical
        if ref is None:
            res[name]["output_certified"] = sort_certificate(x, out)
            ref = out.clone()
        else:
            res[name]["output_equals_binary"] = bool(torch.equal(out, ref))
    res["sorted_ok"] = bool(res["binary"]["output_certified"] and
                            res["learned"]["output_equals_binary"] and
                            res["linear"]["output_equals_binary"])
    res["options"] = opts
    # the same modes in the best two-way shape, where every co-rank of a
    # pass is a predicted two-way co-rank (the tuned four-way shape selects
    # its co-ranks in the runs directly, so there the modes coincide)
    o2 = tune.tuned_options("sort", n, two_way=True)
    if o2 and o2.get("merge_ways", 2) == 2 and o2 != opts:
        ws2 = hv._workspace(hv.lib().hvms_sort_workspace_bytes(n, 0, hv._opts(o2)), dev)
        tw = {"options": o2}
        for name, mode in (("binary", hv.CORANK_BINARY), ("learned", hv.CORANK_LEARNED),
                           ("linear", hv.CORANK_LINEAR)):
            r = _mode_stats(x, out, ws2, o2, params, mode, radius=13)
            r["output_equals_binary"] = bool(torch.equal(out, ref))
            tw[name] = r
        res["two_way"] = tw
        res["sorted_ok"] = bool(res["sorted_ok"] and all(tw[m]["output_equals_binary"]
                                                         for m in ("binary", "learned", "linear")))
        del ws2
    return res


def small_bench():
    """1,048,576 uniform keys (fits in L2 / infinity cache): launch bound."""
    dev = torch.device("cuda", 0)
    n = 1 << 20
    x = inputs.keys(n, "uniform", seed=0, device=dev)
    out = torch.empty_like(x)
    from paper_2409_03970_amd import tune
    opts = tune.tuned_options("sort", n) or {}
    ws = hv._workspace(hv.lib().hvms_sort_workspace_bytes(n, 0, hv._opts(opts)), dev)
    ms = _median_ms(lambda: hv.hvms_sort_i32(x, out, ws, opts=opts), reps=20)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            hv.hvms_sort_i32(x, out, ws, opts=opts)
    torch.cuda.current_stream().wait_stream(s)
    gms = _median_ms(g.replay, reps=20)
    return {"ms": round(ms, 4), "gkeys_per_s": round(n / ms / 1e6, 2), "graph_ms": round(gms, 4),
            "graph_gkeys_per_s": round(n / gms / 1e6, 2), "options": opts}


def config5_bench(max_groups=None, per_segment=True, base_opts=None):
    """50,000 segments, sizes log-uniform in [256, 4194304] (about 2.2e10
    (key, index) pairs, each segment one of the six distributions), generated
    super-group by super-group (about 2^31 pairs each, bounded scratch).
    Times only the sort calls: batched with the learned co-rank (a model
    trained per group, training timed apart), batched with binary co-rank,
    and one plain pair sort per segment."""
    dev = torch.device("cuda", 0)
    nseg = 50000
    sizes = inputs.log_uniform_sizes(nseg, 256, 4194304, seed=0)
    dists = inputs.segment_distributions(nseg, seed=0)
    offs = inputs.offsets_from_sizes(sizes).tolist()
    t = {"learned": 0.0, "binary": 0.0, "per_segment": 0.0, "train": 0.0}
    from paper_2409_03970_amd import tune
    # the tuned shape for batched key-value segments (else the defaults)
    base = dict(base_opts if base_opts is not None
                else (tune.tuned_options("segmented_pairs", 1 << 31) or {}))
    stats = torch.zeros(hv.STATS_WORDS, dtype=torch.int64, device=dev)
    total, ok = 0, True
    L = hv.lib()
    for gi, (s0, s1, _) in enumerate(hv.segment_groups(offs, 1 << 31)):
        if max_groups is not None and gi >= max_groups:
            break
        log(f"  segments {s0}..{s1}")
        sz = sizes[s0:s1]
        k0, v0 = inputs.segment_pairs(sz, dists[s0:s1], s0, seed=0, device=dev)
        offs_local = inputs.offsets_from_sizes(sz)
        params = {}

        def learned(kg, gi):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            p = hv.fit_cdf_model(kg, frac=0.01, steps=150, batch=32768, lr=3e-3, seed=gi)
            b.record()
            torch.cuda.synchronize()
            t["train"] += a.elapsed_time(b)
            params[gi] = p
            return dict(base, corank_mode=hv.CORANK_LEARNED, cdf_params=p, stats=stats)

        res = {}
        # the group workspace is allocated before the timed calls
        gws = hv._workspace(hv.grouped_workspace_bytes(offs_local, 1 << 30, base or None), dev)
        for mode in ("learned", "binary"):
            k, v = k0.clone(), v0.clone()
            torch.cuda.synchronize()
            if mode == "learned":
                hv.segmented_sort_pairs_grouped(k, v, offs_local, 1 << 30, opts_for_group=learned,
                                                ws=gws)
                k, v = k0.clone(), v0.clone()      # first run trained the models
                fn = (lambda kg, gi: dict(base, corank_mode=hv.CORANK_LEARNED,
                                          cdf_params=params[gi]))
            else:
                fn = (lambda kg, gi: dict(base)) if base else None
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            hv.segmented_sort_pairs_grouped(k, v, offs_local, 1 << 30, opts_for_group=fn,
                                            ws=gws)
            b.record()
            torch.cuda.synchronize()
            t[mode] += a.elapsed_time(b)
            res[mode] = (k, v)
        ok &= bool(torch.equal(res["learned"][0], res["binary"][0]))
        ok &= bool(torch.equal(res["learned"][1], res["binary"][1]))
        del res, gws
        if not per_segment:
            total += k0.numel()
            del k0, v0
            torch.cuda.empty_cache()
            continue
        # one plain pair sort per segment, same inputs
        k, v = k0.clone(), v0.clone()
        maxs = int(sz.max())
        ws = hv._workspace(L.hvms_sort_workspace_bytes(maxs, 1, None), dev)
        wp, wb = (ws.data_ptr(), ws.numel()) if ws is not None else (None, 0)
        st = hv._stream(None)
        ol = offs_local.tolist()
        kp, vp = k.data_ptr(), v.data_ptr()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for i in range(len(ol) - 1):
            m = ol[i + 1] - ol[i]
            L.hvms_sort_pairs_i32(hv._vp(kp + 4 * ol[i]), hv._vp(vp + 4 * ol[i]),
                                  hv._vp(kp + 4 * ol[i]), hv._vp(vp + 4 * ol[i]), m,
                                  hv._vp(wp), wb, st, None)
        b.record()
        torch.cuda.synchronize()
        t["per_segment"] += a.elapsed_time(b)
        total += k0.numel()
        del k, v, k0, v0, ws
        torch.cuda.empty_cache()
    c = stats.cpu().tolist()
    return {"pairs": total, "segments": nseg, "options": base, "learned_equals_binary": ok,
            "batched_learned_ms": round(t["learned"], 1),
            "batched_learned_gpairs_per_s": round(total / t["learned"] / 1e6, 2),
            "batched_binary_ms": round(t["binary"], 1),
            "batched_binary_gpairs_per_s": round(total / t["binary"] / 1e6, 2),
            "per_segment_plain_ms": round(t["per_segment"], 1),
            "per_segment_gpairs_per_s": (round(total / t["per_segment"] / 1e6, 2)
                                         if t["per_segment"] else None),
            "training_ms_all_groups": round(t["train"], 1),
            "learned_corank": hv.corank_stats(c)}


def _graph_ms(fn, launches=20, reps=3):
    """Time of one call of fn (which enqueues one launch) from `reps`
    replays of a graph holding `launches` calls: no launch gaps."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()                                    # warm up outside the capture
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            for _ in range(launches):
                fn()
    torch.cuda.current_stream().wait_stream(s)
    return _median_ms(g.replay, reps) / launches


TABLE_N_LOG2 = 23   # 32 MiB of keys: held in the last-level cache, so the
                    # in-register work, not HBM, sets the time


def table2_bench(only_once=False):
    """The paper's Table 2 on the GPU: the time to leave every run of
    X = R * 2^k keys sorted (column network, then k cross-lane merge levels)
    for R = 4, 8, 16, 32 and, at R = 16, the three column networks of Table 1
    (60 / 63 / 80 comparators).  2^23 keys resident in the last-level cache,
    256-thread workgroups, each measured as the mean of 20 launches replayed
    from a captured graph; G keys/s per (R, network, X).  only_once: one
    launch per variant at X = 64 R, in a fixed order (for counters)."""
    dev = torch.device("cuda", 0)
    n = 1 << TABLE_N_LOG2
    x = inputs.keys(n, "uniform", seed=0, device=dev)
    out = torch.empty_like(x)
    res = {}
    for R, net, name in ((4, 0, "R4"), (8, 0, "R8"), (16, 0, "R16*"), (16, 1, "R16-oddeven"),
                         (16, 2, "R16-bitonic"), (32, 0, "R32")):
        o = {"keys_per_lane": R, "block_threads": 256, "column_network": net}
        if only_once:
            hv.hvms_sort_runs_i32(x, out, int(np.log2(R * 64)), opts=o)
            continue
        row = {}
        for k in range(0, 7):
            X = R << k
            ms = _graph_ms(lambda: hv.hvms_sort_runs_i32(x, out, int(np.log2(X)), opts=o))
            row[f"X={X}"] = round(n / ms / 1e6, 2)
        res[name] = row
    torch.cuda.synchronize()
    return {"n": n, "gkeys_per_s": res,
            "note": "2^23 keys in the last-level cache, launches replayed from a graph"}


def table3_bench(only_once=False):
    """The paper's Table 3 on the GPU: the hybrid in-register merger (a run
    per lane, cross-lane flip, then in-lane half-cleaners) against the pure
    cross-lane one (runs across lanes, every stage a lane exchange), merging
    pairs of sorted runs of X = 8, 16, 32 keys.  Each launch repeats the
    merge 16 times on the registers; G merged keys/s = 16 n / time, from 20
    launches replayed from a graph over 2^23 cache-resident keys."""
    dev = torch.device("cuda", 0)
    n = 1 << TABLE_N_LOG2
    reps = 16
    res = {}
    for x_log2 in (3, 4, 5):
        X = 1 << x_log2
        x = inputs.keys(n, "uniform", seed=1, device=dev)
        runs = hv.sort_runs(x, x_log2, opts={"keys_per_lane": 8 if X == 8 else 16,
                                             "block_threads": 256})
        out = torch.empty_like(runs)
        for form, name in ((0, "hybrid"), (1, "vector")):
            if only_once:
                hv.hvms_merge_runs_i32(runs, out, x_log2, form, reps)
                continue
            ms = _graph_ms(lambda: hv.hvms_merge_runs_i32(runs, out, x_log2, form, reps))
            res[f"2x{X}_{name}"] = {"ms": round(ms, 4),
                                    "gkeys_per_s": round(reps * n / ms / 1e6, 1)}
    torch.cuda.synchronize()
    return {"n": n, "reps_per_launch": reps, "results": res}


def measure(opts, xs, dists, out, steps, warmup):
    """Times `steps` sorts of every input with HIP events (warm-up first),
    plus the library's own events around the block stage and every merge
    launch.  Returns rates and per-kernel times."""
    n = xs[0].numel()
    dev = xs[0].device
    ws_bytes = hv.lib().hvms_sort_workspace_bytes(n, 0, hv._opts(opts))
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev)
    R = opts.get("keys_per_lane") or 16
    NT = opts.get("block_threads") or 512
    ways = opts.get("merge_ways") or 2
    passes = merge_passes(n, R * NT, ways)
    levels = merge_passes(n, R * NT, 2)
    first_dominant = levels - 2 * (levels // 2) if ways == 4 else 0  # two-way launches first
    ev_sets = [[make_events(2 + 2 * passes) for _ in dists] for _ in range(steps)]

    def step(events=None):
        for i, x in enumerate(xs):
            o = dict(opts)
            if events is not None:
                o["events"] = events[i]
            hv.hvms_sort_i32(x, out, ws, opts=o)

    log("warmup")
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # parity spot check of the last output (cheap properties)
    if warmup > 0:
        last = out[: min(n, 1 << 22)]
        assert bool((last[1:] >= last[:-1]).all()), "output not sorted"

    log("timed")
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record()
    for st in range(steps):
        step(ev_sets[st])
    t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = t0.elapsed_time(t1)

    bs_ms, pass_ms = [], [[] for _ in range(passes)]
    per_dist = {}
    for i, d in enumerate(dists):
        t = []
        for st in range(steps):
            ev = ev_sets[st][i]
            bs_ms.append(ev[0].elapsed_time(ev[1]))
            for p in range(passes):
                pass_ms[p].append(ev[2 + 2 * p].elapsed_time(ev[3 + 2 * p]))
            t.append(ev[0].elapsed_time(ev[-1]) if passes else ev[0].elapsed_time(ev[1]))
        per_dist[d] = round(n / (np.mean(t) / 1e3) / 1e9, 3)
    dom = [t for p in pass_ms[first_dominant:] for t in p]
    merge_ms = float(np.mean(dom)) if dom else float("nan")
    pass_bytes = 8.0 * n                      # read + write every key once
    return {
        "R": R, "NT": NT, "passes": passes, "ws": ws,
        "keys_per_s": steps * len(dists) * n / (ms_total / 1e3),
        "ms_step": ms_total / steps, "wall": wall, "merge_ms": merge_ms,
        "achieved": pass_bytes / (merge_ms / 1e3) / 1e9 if dom else 0.0,
        "per_pass_gbs": [round(pass_bytes / (np.mean(p) / 1e3) / 1e9, 1) for p in pass_ms],
        "bs_ms": bs_ms, "per_dist": per_dist,
    }


# single measurements for traces and counters (--only)
ONLY = {
    "learned_2p30_mixture": lambda: learned_bench(),
    "sort_2p28_uniform": lambda: sort_dist_bench("uniform"),
    "sort_2p28_sorted": lambda: sort_dist_bench("sorted"),
    "batched_200k_segments": lambda: batched_bench(per_array=False),
    "batched_learned_pairs_first_group": lambda: config5_bench(max_groups=1, per_segment=False),
    "table2": lambda: table2_bench(),
    "table3": lambda: table3_bench(),
    "table2_once": lambda: table2_bench(only_once=True),
    "table3_once": lambda: table3_bench(only_once=True),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="sort_2p28_six", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true", help="headline workload only")
    ap.add_argument("--all", action="store_true",
                    help="accepted for compatibility: every extra runs by default")
    ap.add_argument("--profile-copy", action="store_true",
                    help="also copy one input once with torch (a plain copy of known size "
                         "that calibrates the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--keys-per-lane", type=int, default=0)
    ap.add_argument("--block-threads", type=int, default=0)
    ap.add_argument("--merge-tile", type=int, default=0)
    ap.add_argument("--wave-levels", type=int, default=0, help="levels + 1; 0 = default")
    ap.add_argument("--only", choices=sorted(ONLY),
                    help="diagnostic: run just this measurement (no headline) and print "
                         "its record; used by the kernel traces and counter profiles")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the sort is a single-GPU library)", file=sys.stderr)
        sys.exit(2)
    if args.only:
        dev = torch.device("cuda", 0)
        torch.cuda.set_device(dev)
        if args.profile_copy:  # a plain 1 GiB copy of known size (counter calibration)
            a = torch.zeros(1 << 28, dtype=torch.int32, device=dev)
            torch.empty_like(a).copy_(a)
            torch.cuda.synchronize()
            del a
        rec = {"only": args.only, **ONLY[args.only]()}
        print(json.dumps(rec), flush=True)
        return

    log2n, dists = WORKLOADS[args.workload]
    n = 1 << log2n
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    opts = {"keys_per_lane": args.keys_per_lane, "block_threads": args.block_threads,
            "merge_tile": args.merge_tile, "wave_levels": args.wave_levels}
    if not any(opts.values()):
        from paper_2409_03970_amd import tune
        opts = tune.tuned_options("sort", n) or opts
    opts = {k: int(v) for k, v in opts.items()}
    log(f"generating {len(dists)} x 2^{log2n} keys")
    xs = [inputs.keys(n, d, seed=0, device=dev) for d in dists]
    out = torch.empty(n, dtype=torch.int32, device=dev)
    M = measure(opts, xs, dists, out, args.steps, args.warmup)
    R, NT, tile, passes = M["R"], M["NT"], M["R"] * M["NT"], M["passes"]
    keys_per_s, ms_step, wall = M["keys_per_s"], M["ms_step"], M["wall"]
    merge_ms, achieved, per_pass_gbs = M["merge_ms"], M["achieved"], M["per_pass_gbs"]
    bs_ms, per_dist = M["bs_ms"], M["per_dist"]
    pass_bytes = 8.0 * n
    ways = opts.get("merge_ways") or 2
    ws = M["ws"]

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
            "block_tile": tile, "merge_tile": opts.get("merge_tile") or min(8192, 2 * tile),
            "wave_levels": (opts.get("wave_levels") or 7) - 1,
            "merge_variant": opts.get("merge_variant") or 2, "merge_passes": passes,
            "merge_ways": opts.get("merge_ways") or 2,
            "parallelism": "single GPU",
            # the headline mean includes the presorted inputs, whose tiles are
            # copied rather than merged: the rate of each input beside it
            "gkeys_per_s_by_distribution": per_dist,
        },
        "roofline": {
            "kernel": ("merge4_pipe_kernel (four-way merge pass: two merge levels per launch)"
                       if ways == 4 else "merge_pass_pipe_kernel (two-way merge pass)"),
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": counter_traffic(ways) if log2n == 28 else None,
            "bytes_per_launch": pass_bytes, "avg_launch_ms": merge_ms,
            "merge_levels_per_launch": 2 if ways == 4 else 1,
        },
        "merge_pass_gbs": per_pass_gbs,
        "block_sort_ms": float(np.mean(bs_ms)) if bs_ms else None,
        "gkeys_per_s_by_distribution": per_dist,
        "wall_s_timed": wall,
    }
    if args.profile_copy:
        out.copy_(xs[0])
        torch.cuda.synchronize()
    if not args.quick:
        log("corank_modes_2p28")
        try:
            # the co-rank the model predicts is the two-way pass's: compare
            # the modes on the best two-way configuration
            oc = opts
            if ways == 4:
                from paper_2409_03970_amd import tune
                oc = tune.tuned_options("sort", n, two_way=True) or {
                    "keys_per_lane": 32, "block_threads": 512, "wave_levels": 7,
                    "merge_tile": 8192}
                oc = {k: int(v) for k, v in oc.items()}
            wsc = torch.empty(max(hv.lib().hvms_sort_workspace_bytes(n, 0, hv._opts(oc)), 1),
                              dtype=torch.uint8, device=dev)
            rec["corank_modes_2p28"] = dict(
                corank_modes(xs, dists, out, wsc, oc, opts if ways == 4 else None, ws),
                options=oc, options_four_way=opts if ways == 4 else None)
            del wsc
        except Exception as e:  # an extra must never cost the headline line
            rec["corank_modes_2p28"] = {"error": repr(e)}
        log("key_types_2p28")
        try:
            rec["key_types_2p28"] = key_types_bench(n)
        except Exception as e:
            rec["key_types_2p28"] = {"error": repr(e)}
        if ways == 4:
            # the best configuration with two-way passes on the same inputs:
            # one merge level per trip through HBM, at a higher share of the
            # bandwidth per launch
            log("two_way_2p28")
            try:
                from paper_2409_03970_amd import tune
                o2 = tune.tuned_options("sort", n, two_way=True) or {
                    "keys_per_lane": 32, "block_threads": 512, "wave_levels": 7,
                    "merge_tile": 8192}
                o2 = {k: int(v) for k, v in o2.items()}
                M2 = measure(o2, xs, dists, out, args.steps, 1)
                rec["two_way_2p28"] = {
                    "value": M2["keys_per_s"], "options": o2,
                    "gkeys_per_s_by_distribution": M2["per_dist"],
                    "merge_pass_gbs": M2["per_pass_gbs"], "avg_launch_ms": M2["merge_ms"],
                    "frac": round(M2["achieved"] / HBM_PEAK_GBS, 4),
                    "traffic": counter_traffic(2),
                    "block_sort_ms": float(np.mean(M2["bs_ms"]))}
                del M2
            except Exception as e:
                rec["two_way_2p28"] = {"error": repr(e)}
        else:
            log("four_way_2p28")
            try:
                hv.hvms_sort_i32(xs[0], out, ws, opts=opts)
                rec["four_way_2p28_" + dists[0]] = four_way_bench(xs[0], out, opts)
            except Exception as e:
                rec["four_way_2p28_" + dists[0]] = {"error": repr(e)}
        del xs, out, ws, M
        torch.cuda.empty_cache()
        extras = (("in_register_sort_table2", table2_bench),
                  ("in_register_merge_table3", table3_bench),
                  ("merge_pass_mergers", lambda: merge_table3_bench(n)),
                  ("pairs_2p28", lambda: pairs_bench(n)),
                  ("sort_by_key_p64_2p28", lambda: by_key_bench(n)),
                  ("batched_learned_pairs_50k_segments", config5_bench),
                  ("batched_200k_segments", batched_bench),
                  ("learned_2p30_mixture", learned_bench),
                  ("small_2p20", small_bench))
        for name, fn in extras:
            if fn is None:
                continue
            log(name)
            try:
                rec[name] = fn()
            except Exception as e:  # an extra must never cost the headline line
                rec[name] = {"error": repr(e)}
            torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        rec["cpu_baseline"] = cpu_baseline(dists, log2n)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
