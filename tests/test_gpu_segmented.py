"""GPU parity of the batched segmented sort against the CPU oracle, through the
C ABI, including replays of a captured HIP graph."""
import numpy as np
import pytest
import torch

import oracle
import paper_2409_03970_amd as hv
from paper_2409_03970_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _say(*a):
    print(*a, flush=True)


def _run(sizes, dist="uniform", seed=0, opts=None, pairs=False):
    sizes = torch.as_tensor(sizes, dtype=torch.int64)
    offs = inputs.offsets_from_sizes(sizes)
    n = int(offs[-1])
    k = inputs.keys(n, dist, seed=seed, device=DEV)
    offs_np = offs.numpy()
    if pairs:
        v = torch.cat([torch.arange(int(s), dtype=torch.int32) for s in sizes.tolist()]).to(DEV) \
            if n else torch.empty(0, dtype=torch.int32, device=DEV)
        ko, vo = hv.segmented_sort_pairs(k, v, offs, opts=opts)
        ek, ev = oracle.segmented_sort_pairs(k.cpu().numpy(), v.cpu().numpy(), offs_np)
        assert np.array_equal(ko.cpu().numpy(), ek) and np.array_equal(vo.cpu().numpy(), ev)
    else:
        y = hv.segmented_sort(k, offs, opts=opts)
        assert np.array_equal(y.cpu().numpy(), oracle.segmented_sort(k.cpu().numpy(), offs_np))


@pytest.mark.parametrize("seed", range(3))
def test_log_uniform_sizes(seed):
    _say("segmented log-uniform", seed)
    _run(inputs.log_uniform_sizes(3000, 1, 65536, seed=seed), seed=seed)


def test_edge_sizes():
    # empty, one, around the lane / wave / tile sizes and several merge passes
    sizes = [0, 1, 0, 2, 15, 16, 17, 31, 33, 1023, 1024, 1025, 8191, 8192, 8193, 0, 16383,
             16384, 16385, 40000, 65536, 65537, 131072 + 5, 3, 0]
    _run(sizes, seed=1)
    _run(sizes[::-1], dist="distinct16", seed=2)


def test_single_segment_equals_plain_sort():
    n = 300007
    k = inputs.keys(n, "zipf", seed=3, device=DEV)
    y = hv.segmented_sort(k, torch.tensor([0, n]))
    assert torch.equal(y, hv.sort(k))


def test_all_empty_and_none():
    k = torch.empty(0, dtype=torch.int32, device=DEV)
    assert hv.segmented_sort(k, torch.zeros(5, dtype=torch.int64)).numel() == 0
    assert hv.segmented_sort(k, torch.zeros(1, dtype=torch.int64)).numel() == 0


def test_keys_outside_segments_untouched():
    n = 50000
    k = inputs.keys(n, "uniform", seed=4, device=DEV)
    offs = torch.tensor([100, 5000, 5000, 30000, 49000], dtype=torch.int64)
    out = torch.full_like(k, -7)
    hv.segmented_sort(k, offs, out=out)
    o = out.cpu().numpy()
    assert np.all(o[:100] == -7) and np.all(o[49000:] == -7)
    want = oracle.segmented_sort(k.cpu().numpy(), offs.numpy())
    assert np.array_equal(o[100:49000], want[100:49000])


@pytest.mark.parametrize("dist", ["distinct16", "sorted", "reverse", "zipf"])
def test_distributions(dist):
    _run(inputs.log_uniform_sizes(800, 1, 40000, seed=5), dist=dist, seed=5)


@pytest.mark.parametrize("opt", [dict(keys_per_lane=R, block_threads=NT, merge_tile=TM, wave_levels=K + 1,
                                      merge_variant=V)
                                 for R, NT in [(16, 256), (16, 512), (16, 1024), (8, 512), (32, 256), (32, 512)]
                                 for TM in (2048, 4096, 8192) if TM <= 2 * R * NT
                                 for K in (6, 2) for V in (2, 3)],
                         ids=lambda o: "R{keys_per_lane}_NT{block_threads}_TM{merge_tile}_K{wave_levels}_V{merge_variant}".format(**o))
def test_every_tuning(opt):
    _run(inputs.log_uniform_sizes(400, 1, 70000, seed=6), seed=6, opts=opt)


@pytest.mark.parametrize("dist", ["uniform", "distinct16"])
def test_pairs(dist):
    _say("segmented pairs", dist)
    _run(inputs.log_uniform_sizes(600, 1, 50000, seed=7), dist=dist, seed=7, pairs=True)


@pytest.mark.parametrize("opt", [dict(keys_per_lane=16, block_threads=256, merge_tile=4096),
                                 dict(keys_per_lane=8, block_threads=1024, merge_tile=8192),
                                 dict(keys_per_lane=32, block_threads=512, merge_tile=2048)])
def test_pairs_tunings(opt):
    _run(inputs.log_uniform_sizes(300, 1, 40000, seed=8), dist="zipf", seed=8, pairs=True, opts=opt)


def test_offsets_on_device_and_in_place():
    sizes = inputs.log_uniform_sizes(500, 1, 30000, seed=9)
    offs = inputs.offsets_from_sizes(sizes)
    n = int(offs[-1])
    k = inputs.keys(n, "uniform", seed=9, device=DEV)
    want = oracle.segmented_sort(k.cpu().numpy(), offs.numpy())
    hv.segmented_sort(k, offs.to(DEV), out=k)
    assert np.array_equal(k.cpu().numpy(), want)


def test_graph_capture_replays():
    sizes = inputs.log_uniform_sizes(2000, 1, 65536, seed=10)
    offs = inputs.offsets_from_sizes(sizes)
    n = int(offs[-1])
    k = inputs.keys(n, "uniform", seed=10, device=DEV)
    d_off = offs.to(DEV)
    out = torch.empty_like(k)
    max_seg = int(sizes.max())
    ws = torch.empty(hv.lib().hvms_segmented_workspace_bytes(n, sizes.numel(), max_seg, 0, None),
                     dtype=torch.uint8, device=DEV)
    eager = torch.empty_like(k)
    hv.hvms_segmented_sort_i32(k, eager, d_off, n, max_seg, ws)
    torch.cuda.synchronize()
    assert np.array_equal(eager.cpu().numpy(), oracle.segmented_sort(k.cpu().numpy(), offs.numpy()))
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            hv.hvms_segmented_sort_i32(k, out, d_off, n, max_seg, ws)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(4):
        out.fill_(-1)
        junk = hv.sort(inputs.keys(70000, "zipf", seed=rep, device=DEV))   # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep
        assert junk.numel() == 70000


def test_full_size_200k_segments():
    # 200,000 segments, sizes log-uniform in [1, 65536] (about 1.18e9 keys)
    sizes = inputs.log_uniform_sizes(200000, 1, 65536, seed=0)
    offs = inputs.offsets_from_sizes(sizes)
    n = int(offs[-1])
    _say("full-size segmented, keys:", n)
    k = inputs.keys(n, "uniform", seed=3, device=DEV)
    y = hv.segmented_sort(k, offs)
    torch.cuda.synchronize()
    d_off = offs.to(DEV)
    # every segment nondecreasing: only descents allowed are at segment starts
    desc = torch.nonzero(y[1:] < y[:-1]).flatten() + 1
    starts = torch.zeros(n + 1, dtype=torch.bool, device=DEV)
    starts[d_off] = True
    assert bool(starts[desc].all())
    ks, ys = k.cpu().numpy(), y.cpu().numpy()
    offs_np = offs.numpy()
    # per-segment multisets: the whole array's hash and every sampled segment exactly
    assert oracle.multiset_hash(ys) == oracle.multiset_hash(ks)
    rng = np.random.default_rng(0)
    for s in rng.choice(sizes.numel(), 300, replace=False).tolist() + [int(sizes.argmax())]:
        a, b = offs_np[s], offs_np[s + 1]
        assert np.array_equal(ys[a:b], oracle.sort(ks[a:b])), s


def test_grouped_pairs_match_oracle():
    sizes = inputs.log_uniform_sizes(300, 1, 60000, seed=11)
    dists = inputs.segment_distributions(300, seed=11)
    offs = inputs.offsets_from_sizes(sizes)
    k, v = inputs.segment_pairs(sizes, dists, 0, seed=11, device=DEV)
    ek, ev = oracle.segmented_sort_pairs(k.cpu().numpy(), v.cpu().numpy(), offs.numpy())
    ws = hv._workspace(hv.grouped_workspace_bytes(offs, max_group_keys=200000), k.device)
    hv.segmented_sort_pairs_grouped(k, v, offs, max_group_keys=200000, ws=ws)
    assert np.array_equal(k.cpu().numpy(), ek) and np.array_equal(v.cpu().numpy(), ev)


def _certify_pairs(k_in, k, v, offs_local, sizes):
    """Output equals the oracle's iff: pairs strictly increase inside every
    segment, payloads are a permutation of 0..size-1 per segment, and every
    payload still points at its original key."""
    n = k.numel()
    d_sizes = sizes.to(DEV)
    base = torch.repeat_interleave(offs_local[:-1].to(DEV), d_sizes)
    assert bool(((v >= 0) & (v.long() < torch.repeat_interleave(d_sizes, d_sizes))).all())
    src = base + v.long()
    assert torch.equal(k_in[src], k)
    mark = torch.zeros(n, dtype=torch.int32, device=DEV)
    mark.index_add_(0, src, torch.ones(n, dtype=torch.int32, device=DEV))
    assert bool((mark == 1).all())
    del mark, src
    inc = (k[1:] > k[:-1]) | ((k[1:] == k[:-1]) & (v[1:] > v[:-1]))
    starts = torch.zeros(n, dtype=torch.bool, device=DEV)
    starts[offs_local[:-1].to(DEV)] = True
    assert bool((inc | starts[1:]).all())


def test_full_size_50k_segments_learned_pairs():
    # 50,000 segments, sizes log-uniform in [256, 4194304] (about 2.15e10
    # pairs), each segment's keys from one of the six distributions, payload =
    # index within the segment, learned co-rank; bounded scratch: generated,
    # sorted and checked super-group by super-group
    nseg = 50000
    sizes = inputs.log_uniform_sizes(nseg, 256, 4194304, seed=0)
    dists = inputs.segment_distributions(nseg, seed=0)
    offs = inputs.offsets_from_sizes(sizes).tolist()
    total, checked = 0, 0
    rng = np.random.default_rng(0)

    def learned(kg, gi):
        p = hv.fit_cdf_model(kg, frac=0.01, steps=150, batch=32768, lr=3e-3, seed=gi)
        return {"corank_mode": hv.CORANK_LEARNED, "cdf_params": p}

    for s0, s1, _ in hv.segment_groups(offs, 1 << 31):
        sz = sizes[s0:s1]
        k, v = inputs.segment_pairs(sz, dists[s0:s1], s0, seed=0, device=DEV)
        k_in = k.clone()
        offs_local = inputs.offsets_from_sizes(sz)
        _say("super-group", s0, s1, "pairs", k.numel())
        hv.segmented_sort_pairs_grouped(k, v, offs_local, max_group_keys=1 << 30,
                                        opts_for_group=learned)
        torch.cuda.synchronize()
        _certify_pairs(k_in, k, v, offs_local, sz)
        for s in rng.choice(s1 - s0, 3, replace=False).tolist():
            a, b = int(offs_local[s]), int(offs_local[s + 1])
            if b - a <= 1 << 20:
                ek, ev = oracle.sort_pairs(k_in[a:b].cpu().numpy(), np.arange(b - a, dtype=np.int32))
                assert np.array_equal(k[a:b].cpu().numpy(), ek)
                assert np.array_equal(v[a:b].cpu().numpy(), ev)
                checked += 1
        total += k.numel()
        del k, v, k_in
        torch.cuda.empty_cache()
    assert total == offs[-1] and checked > 0
    _say("pairs", total, "oracle-checked segments", checked)


def test_all_permutations_of_8_as_segments():
    # all 8! = 40,320 arrangements of 0..7 as segments of one call: every
    # segment must come back as 0..7; the pair form keeps each key's position
    import itertools
    perms = np.array(list(itertools.permutations(range(8))), dtype=np.int32)
    k = torch.from_numpy(perms.reshape(-1).copy()).to(DEV)
    offs = torch.arange(0, perms.size + 1, 8, dtype=torch.int64)
    _say("segmented all 8! permutations")
    y = hv.segmented_sort(k, offs).cpu().numpy().reshape(-1, 8)
    assert (y == np.arange(8, dtype=np.int32)).all()
    pos = np.tile(np.arange(8, dtype=np.int32), len(perms))
    v = torch.from_numpy(pos).to(DEV)
    ko, vo = hv.segmented_sort_pairs(k, v, offs)
    ko, vo = ko.cpu().numpy().reshape(-1, 8), vo.cpu().numpy().reshape(-1, 8)
    assert (ko == np.arange(8)).all()
    # value j of segment s is where key j stood: perms[s, vo[s, j]] == j
    assert (np.take_along_axis(perms, vo, axis=1) == np.arange(8)).all()


# ------------------------------------------------ status words (max_seg, offsets)

def _raw_segmented(k, offs, max_seg, opts, out=None, vals=None):
    """One raw ABI call; returns (output keys, output values or None, status)."""
    n = int(offs[-1]) if offs.numel() else 0
    nseg = offs.numel() - 1
    d_off = offs.to(DEV)
    ws = torch.empty(max(hv.lib().hvms_segmented_workspace_bytes(n, nseg, max(max_seg, 0),
                                                                   int(vals is not None),
                                                                   hv._opts(opts)), 256),
                     dtype=torch.uint8, device=DEV)
    out = torch.empty_like(k) if out is None else out
    if vals is None:
        hv.hvms_segmented_sort_i32(k, out, d_off, n, max_seg, ws, opts=opts)
        vo = None
    else:
        vo = torch.empty_like(vals)
        hv.hvms_segmented_sort_pairs_i32(k, vals, out, vo, d_off, n, max_seg, ws, opts=opts)
    st = torch.full((3,), -7, dtype=torch.int64, device=DEV)
    hv.hvms_segmented_status(ws, st)
    return out, vo, st.cpu().tolist()


# block tile 2048 keys: a segment of s keys needs ceil(log2(ceil(s / 2048))) passes
_SMALL = {"keys_per_lane": 8, "block_threads": 256}
_SIZES = [5, 2048, 2049, 4096, 4097, 9000, 3 * 2048 + 7, 70000, 0, 131072, 1000]


@pytest.mark.parametrize("pairs", [False, True])
def test_max_seg_underestimated_reports_and_stays_a_permutation(pairs):
    # max_seg = 4096 enqueues one pass: segments above 4096 keys are left as
    # sorted runs of 4096 (an exact, checkable permutation) and counted
    sizes = torch.tensor(_SIZES, dtype=torch.int64)
    offs = inputs.offsets_from_sizes(sizes)
    n = int(offs[-1])
    k = inputs.keys(n, "uniform", seed=21, device=DEV)
    v = torch.arange(n, dtype=torch.int32, device=DEV) if pairs else None
    _say("max_seg underestimated, pairs", pairs)
    out, vo, st = _raw_segmented(k, offs, 4096, _SMALL, vals=v)
    over = int((sizes > 4096).sum())
    assert st == [over, 0, 0]
    kh, got = k.cpu().numpy(), out.cpu().numpy()
    vh = v.cpu().numpy() if pairs else None
    gotv = vo.cpu().numpy() if pairs else None
    o = offs.tolist()
    for s in range(len(_SIZES)):
        run = 4096 if _SIZES[s] > 4096 else max(_SIZES[s], 1)
        for a in range(o[s], o[s + 1], run):
            b = min(a + run, o[s + 1])
            if pairs:
                ek, ev = oracle.sort_pairs(kh[a:b], vh[a:b])
                assert np.array_equal(got[a:b], ek) and np.array_equal(gotv[a:b], ev), (s, a)
            else:
                assert np.array_equal(got[a:b], oracle.sort(kh[a:b])), (s, a)


def test_max_seg_unknown_sorts_everything():
    sizes = torch.tensor(_SIZES, dtype=torch.int64)
    offs = inputs.offsets_from_sizes(sizes)
    k = inputs.keys(int(offs[-1]), "zipf", seed=22, device=DEV)
    out, _, st = _raw_segmented(k, offs, -1, _SMALL)
    assert st == [0, 0, 0]
    assert np.array_equal(out.cpu().numpy(),
                          oracle.segmented_sort(k.cpu().numpy(), offs.numpy()))
    # an exact bound gives the same output and a clean status
    out2, _, st2 = _raw_segmented(k, offs, int(sizes.max()), _SMALL)
    assert st2 == [0, 0, 0] and torch.equal(out, out2)


def test_invalid_offsets_are_counted_and_skipped():
    # segment 1 ends past n_total, segment 2 has decreasing offsets: both are
    # skipped (their keys untouched) and counted; segment 0 is sorted
    n = 3000
    k = inputs.keys(n, "uniform", seed=23, device=DEV)
    offs = torch.tensor([0, 1000, 4000, 3000], dtype=torch.int64)
    pre = torch.full((n,), -5, dtype=torch.int32, device=DEV)
    out, _, st = _raw_segmented(k, offs, -1, _SMALL, out=pre)
    assert st == [0, 2, 0]
    got = out.cpu().numpy()
    assert np.array_equal(got[:1000], oracle.sort(k.cpu().numpy()[:1000]))
    assert (got[1000:] == -5).all()


def test_inconsistent_offsets_flagged_and_nothing_written():
    # offsets 0, n, 0, n, ...: four segments each spanning [0, n) (and three
    # decreasing ones between them, skipped).  Their sizes add up to four
    # times n_total, more pieces than the workspace plans for n_total keys,
    # so the call sorts and writes nothing and raises status word 2.
    n = 20 * 2048
    k = inputs.keys(n, "uniform", seed=24, device=DEV)
    offs = torch.tensor([0, n] * 3 + [0, n][:1] + [n], dtype=torch.int64)
    assert offs.tolist() == [0, n, 0, n, 0, n, 0, n]
    pre = torch.full((n,), -9, dtype=torch.int32, device=DEV)
    out, _, st = _raw_segmented(k, offs, n, _SMALL, out=pre)
    assert st == [0, 3, 1]
    assert bool((out == -9).all())


@pytest.mark.parametrize("pairs", [False, True])
def test_learned_corank_segments_match_oracle(pairs):
    # segments with merge passes, learned co-ranks (model table built by the
    # call), element by element against the oracle; binary mode must agree
    sizes = inputs.log_uniform_sizes(300, 1, 200000, seed=31)
    offs = inputs.offsets_from_sizes(sizes)
    n = int(offs[-1])
    k = inputs.keys(n, "mixture", seed=31, device=DEV)
    params = hv.fit_cdf_model(k, frac=0.02, steps=150, batch=8192, lr=3e-3, seed=31)
    st = torch.zeros(hv.STATS_WORDS, dtype=torch.int64, device=DEV)
    opts = {"corank_mode": hv.CORANK_LEARNED, "cdf_params": params, "radius_log2": 10,
            "stats": st}
    if pairs:
        v = torch.cat([torch.arange(int(s), dtype=torch.int32) for s in sizes.tolist()]).to(DEV)
        ko, vo = hv.segmented_sort_pairs(k, v, offs, opts=opts)
        ek, ev = oracle.segmented_sort_pairs(k.cpu().numpy(), v.cpu().numpy(), offs.numpy())
        assert np.array_equal(ko.cpu().numpy(), ek) and np.array_equal(vo.cpu().numpy(), ev)
    else:
        y = hv.segmented_sort(k, offs, opts=opts)
        assert np.array_equal(y.cpu().numpy(),
                              oracle.segmented_sort(k.cpu().numpy(), offs.numpy()))
        assert torch.equal(y, hv.segmented_sort(k, offs))
    s = hv.corank_stats(st.cpu())
    assert s["coranks"] > 0 and s.get("predicted", 0) > 0


# ------------------------------------------------ four-way segmented passes

_FOUR = [dict(keys_per_lane=R, block_threads=NT, merge_tile=TM, merge_ways=4, merge_variant=V)
         for R, NT in [(16, 256), (16, 512), (8, 512), (32, 256), (32, 512)]
         for TM in (4096, 8192, 16384) if TM <= 2 * R * NT
         for V in (0, 2)]


@pytest.mark.parametrize("opt", _FOUR, ids=lambda o: "R{keys_per_lane}_NT{block_threads}_TM{merge_tile}_V{merge_variant}".format(**o))
def test_four_way_every_shape(opt):
    # segments of one to about 2^19 keys: up to five merge levels, both
    # parities (an odd count ends with a two-way level), segment offsets at
    # every alignment
    _say("segmented four-way", opt)
    _run(inputs.log_uniform_sizes(400, 1, 1 << 19, seed=41), seed=41, opts=opt)


@pytest.mark.parametrize("dist", ["uniform", "sorted", "reverse", "distinct16", "zipf"])
def test_four_way_distributions(dist):
    _run(inputs.log_uniform_sizes(300, 1, 300000, seed=42), dist=dist, seed=42,
         opts={"merge_ways": 4, "merge_tile": 4096})


def test_four_way_edge_sizes():
    # around the tile, two, four and eight tiles, and single segments whose
    # level counts are odd and even
    opts = {"keys_per_lane": 8, "block_threads": 256, "merge_tile": 4096, "merge_ways": 4}
    t = 2048
    sizes = [0, 1, t - 1, t, t + 1, 2 * t, 2 * t + 1, 4 * t - 3, 4 * t, 4 * t + 1, 8 * t, 8 * t + 5,
             16 * t - 1, 16 * t, 16 * t + 1, 0, 33 * t + 7, 3, 64 * t, 129 * t + 1]
    _run(sizes, seed=43, opts=opts)
    _run(sizes[::-1], dist="distinct16", seed=44, opts=opts)
    _run([200003], seed=45, opts=opts)


@pytest.mark.parametrize("tm", [2048, 4096])
@pytest.mark.parametrize("dist", ["uniform", "zipf", "sorted"])
def test_four_way_pairs(tm, dist):
    _run(inputs.log_uniform_sizes(300, 1, 200000, seed=46), dist=dist, seed=46, pairs=True,
         opts={"keys_per_lane": 16, "block_threads": 256, "merge_tile": tm, "merge_ways": 4})


def test_four_way_graph_capture_replays():
    sizes = inputs.log_uniform_sizes(2000, 1, 100000, seed=47)
    offs = inputs.offsets_from_sizes(sizes)
    n = int(offs[-1])
    k = inputs.keys(n, "uniform", seed=47, device=DEV)
    d_off = offs.to(DEV)
    opts = {"merge_ways": 4, "merge_tile": 4096}
    ws = torch.empty(hv.lib().hvms_segmented_workspace_bytes(n, sizes.numel(), int(sizes.max()),
                                                             0, hv._opts(opts)),
                     dtype=torch.uint8, device=DEV)
    out = torch.empty_like(k)
    want = oracle.segmented_sort(k.cpu().numpy(), offs.numpy())
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            hv.hvms_segmented_sort_i32(k, out, d_off, n, int(sizes.max()), ws, opts=opts)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        out.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), want), rep


@pytest.mark.parametrize("pairs", [False, True])
def test_four_way_max_seg_underestimated(pairs):
    # max_seg = 4096 over 2048-key tiles: one merge level, so one launch;
    # a four-way launch merges two levels, so segments up to 8192 keys are
    # sorted and longer ones are left as sorted runs of 8192 and counted
    sizes = torch.tensor(_SIZES, dtype=torch.int64)
    offs = inputs.offsets_from_sizes(sizes)
    n = int(offs[-1])
    k = inputs.keys(n, "uniform", seed=48, device=DEV)
    v = torch.arange(n, dtype=torch.int32, device=DEV) if pairs else None
    opts = dict(_SMALL, merge_tile=4096, merge_ways=4)
    out, vo, st = _raw_segmented(k, offs, 4096, opts, vals=v)
    assert st == [int((sizes > 8192).sum()), 0, 0]
    kh, got = k.cpu().numpy(), out.cpu().numpy()
    vh = v.cpu().numpy() if pairs else None
    gotv = vo.cpu().numpy() if pairs else None
    o = offs.tolist()
    for s in range(len(_SIZES)):
        run = 8192 if _SIZES[s] > 8192 else max(_SIZES[s], 1)
        for a in range(o[s], o[s + 1], run):
            b = min(a + run, o[s + 1])
            if pairs:
                ek, ev = oracle.sort_pairs(kh[a:b], vh[a:b])
                assert np.array_equal(got[a:b], ek) and np.array_equal(gotv[a:b], ev), (s, a)
            else:
                assert np.array_equal(got[a:b], oracle.sort(kh[a:b])), (s, a)


def test_four_way_learned_corank_segments():
    sizes = inputs.log_uniform_sizes(200, 1, 400000, seed=49)
    offs = inputs.offsets_from_sizes(sizes)
    n = int(offs[-1])
    k = inputs.keys(n, "mixture", seed=49, device=DEV)
    params = hv.fit_cdf_model(k, frac=0.02, steps=150, batch=8192, lr=3e-3, seed=49)
    st = torch.zeros(hv.STATS_WORDS, dtype=torch.int64, device=DEV)
    opts = {"corank_mode": hv.CORANK_LEARNED, "cdf_params": params, "radius_log2": 9,
            "stats": st, "merge_ways": 4, "merge_tile": 4096}
    y = hv.segmented_sort(k, offs, opts=opts)
    assert np.array_equal(y.cpu().numpy(), oracle.segmented_sort(k.cpu().numpy(), offs.numpy()))
    assert torch.equal(y, hv.segmented_sort(k, offs, opts={"merge_ways": 4, "merge_tile": 4096}))
    s = hv.corank_stats(st.cpu())
    assert s["coranks"] > 0 and s.get("predicted", 0) > 0


@pytest.mark.parametrize("pairs", [False, True])
@pytest.mark.parametrize("ways", [2, 4])
@pytest.mark.parametrize("dist", ["uniform", "sorted", "distinct16"])
def test_pieces_around_half_a_tile(pairs, ways, dist):
    # segments, and ragged rests of longer segments, at the quarter- and
    # half-tile lines: up to a quarter of a tile they go to the packed
    # kernel, up to half a tile two to a full-kernel tile (each padded to
    # half a tile), above it one to a tile (padded); a tile of 4096 keys.
    # An odd number of half-list pieces leaves one pair with one piece.
    T, H, Q = 4096, 2048, 1024
    sizes = []
    for r in (Q - 1, Q, Q + 1, H - 1, H, H + 1, H + 2, T - 1, T):
        sizes += [r, T + r, 3 * T + r, 8 * T + r]
    sizes += [T + 1, 2 * T, 5 * T + H + 1, 0, 1, H + 1, Q + 7]
    _say("pieces around half a tile", pairs, ways, dist)
    _run(sizes, dist=dist, seed=17, pairs=pairs,
         opts={"keys_per_lane": 8, "block_threads": 512, "merge_tile": 4096,
               "merge_ways": ways})
