"""GPU parity of the sort path against the CPU oracle (bit-exact), through the
C ABI.  Networks are checked on every 0-1 input (0-1 principle)."""
import numpy as np
import pytest
import torch

import oracle
import oracle_parts
import paper_2409_03970_amd as hv
from paper_2409_03970_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _say(*a):
    print(*a, flush=True)


# ------------------------------------------------- 0-1 principle on the GPU

def _runs_from_bits(X, R):
    """All 2^X 0-1 inputs of X keys, one run each (X <= 16)."""
    q = torch.arange(1 << X, device=DEV, dtype=torch.int64)
    bits = (q[:, None] >> torch.arange(X, device=DEV)) & 1
    return bits.to(torch.int32).reshape(-1)


@pytest.mark.parametrize("R", [4, 8, 16])
def test_column_network_all_01_inputs(R):
    # runs of R keys = the per-lane network alone; every run must come out sorted
    _say("column network 0-1, R =", R)
    x = _runs_from_bits(R, R)
    y = hv.sort_runs(x, int(np.log2(R)), opts={"keys_per_lane": R, "block_threads": 256})
    torch.cuda.synchronize()
    runs = y.view(-1, R)
    ones = x.view(-1, R).sum(1)
    want = (torch.arange(R, device=DEV)[None, :] >= (R - ones)[:, None]).to(torch.int32)
    assert torch.equal(runs, want)


def test_column_network_32_random_01_inputs():
    g = torch.Generator(device=DEV)
    g.manual_seed(5)
    x = torch.randint(0, 2, (1 << 22,), generator=g, device=DEV, dtype=torch.int32)
    y = hv.sort_runs(x, 5, opts={"keys_per_lane": 32, "block_threads": 256})
    ones = x.view(-1, 32).sum(1)
    want = (torch.arange(32, device=DEV)[None, :] >= (32 - ones)[:, None]).to(torch.int32)
    assert torch.equal(y.view(-1, 32), want)


def _sorted_halves(X, device=DEV):
    """All (X/2 + 1)^2 0-1 runs of X keys whose halves are each sorted."""
    h = X // 2
    z1 = torch.arange(h + 1, device=device).repeat_interleave(h + 1)
    z2 = torch.arange(h + 1, device=device).repeat(h + 1)
    pos = torch.arange(h, device=device)[None, :]
    first = (pos >= z1[:, None]).to(torch.int32)
    second = (pos >= z2[:, None]).to(torch.int32)
    return torch.cat([first, second], 1).reshape(-1), z1 + z2


@pytest.mark.parametrize("R", [4, 8, 16])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_wave_merge_level_all_sorted_halves(R, k):
    # runs of X = R * 2^k: the levels below k keep the sorted halves as they
    # are, so level k sees every sorted-halves 0-1 input
    X = R << k
    _say("wave merge level", k, "R", R, "X", X)
    x, zeros = _sorted_halves(X)
    y = hv.sort_runs(x, int(np.log2(X)), opts={"keys_per_lane": R, "block_threads": 256})
    want = (torch.arange(X, device=DEV)[None, :] >= zeros[:, None]).to(torch.int32)
    assert torch.equal(y.view(-1, X), want)


@pytest.mark.parametrize("X", [2048, 4096, 8192])
def test_lds_merge_levels_sorted_halves(X):
    # LDS merge-path levels (not a network): a strided subset of the
    # sorted-halves inputs plus all extreme splits
    h = X // 2
    zs = sorted(set(list(range(0, h + 1, 97)) + [0, 1, 2, h - 2, h - 1, h]))
    z = torch.tensor(zs, device=DEV)
    z1 = z.repeat_interleave(len(zs))
    z2 = z.repeat(len(zs))
    pos = torch.arange(h, device=DEV)[None, :]
    x = torch.cat([(pos >= z1[:, None]), (pos >= z2[:, None])], 1).to(torch.int32).reshape(-1)
    y = hv.sort_runs(x, int(np.log2(X)), opts={"block_threads": 512})
    want = (torch.arange(X, device=DEV)[None, :] >= (z1 + z2)[:, None]).to(torch.int32)
    assert torch.equal(y.view(-1, X), want)


# ------------------------------------------------------ runs vs the oracle

@pytest.mark.parametrize("R,NT", [(16, 256), (16, 512), (8, 256), (32, 256), (16, 1024)])
def test_sort_runs_match_oracle(R, NT):
    n = 3 * R * NT + 77
    x = inputs.keys(n, "uniform", seed=R + NT, device=DEV)
    xs = x.cpu().numpy()
    for run_log2 in range(int(np.log2(R)), int(np.log2(R * NT)) + 1):
        _say("sort_runs", R, NT, run_log2)
        y = hv.sort_runs(x, run_log2, opts={"keys_per_lane": R, "block_threads": NT}).cpu().numpy()
        X = 1 << run_log2
        offs = np.append(np.arange(0, n, X), n)
        assert np.array_equal(y, oracle.segmented_sort(xs, offs))


# ----------------------------------------------------------- full sort

SIZES = [1, 2, 3, 15, 16, 17, 63, 64, 65, 100, 1023, 1024, 1025, 4095, 4096, 4097, 8191, 8192,
         8193, 12289, 65535, 65536, 65537, 100003, (1 << 20) + 3]


@pytest.mark.parametrize("n", SIZES)
def test_sort_matches_oracle_sizes(n):
    _say("sort n =", n)
    x = inputs.keys(n, "uniform", seed=n, device=DEV)
    y = hv.sort(x)
    assert np.array_equal(y.cpu().numpy(), oracle.sort(x.cpu().numpy()))


@pytest.mark.parametrize("dist", list(inputs.DISTRIBUTIONS) + ["mixture"])
@pytest.mark.parametrize("n", [777777, 1 << 21])
def test_sort_matches_oracle_distributions(dist, n):
    _say("sort", dist, n)
    x = inputs.keys(n, dist, seed=11, device=DEV)
    y = hv.sort(x)
    assert np.array_equal(y.cpu().numpy(), oracle.sort(x.cpu().numpy()))


@pytest.mark.parametrize("pattern", ["equal", "two_values", "extremes", "organ_pipe", "sawtooth",
                                     "negatives"])
def test_sort_adversarial(pattern):
    for n in (5, 4097, 300001):
        x = inputs.adversarial_keys(n, pattern, seed=2, device=DEV)
        y = hv.sort(x)
        assert np.array_equal(y.cpu().numpy(), oracle.sort(x.cpu().numpy())), (pattern, n)


def test_sort_in_place_and_input_untouched():
    x = inputs.keys(300007, "uniform", seed=3, device=DEV)
    ref = oracle.sort(x.cpu().numpy())
    keep = x.clone()
    y = hv.sort(x)
    assert torch.equal(x, keep)
    hv.sort(x, out=x)
    assert np.array_equal(x.cpu().numpy(), ref) and np.array_equal(y.cpu().numpy(), ref)


TUNINGS = [
    dict(keys_per_lane=R, block_threads=NT, merge_tile=TM, wave_levels=K + 1)
    for (R, NT) in [(8, 256), (8, 1024), (16, 256), (16, 512), (16, 1024), (32, 256), (32, 512),
                    (32, 1024)]
    for TM in (2048, 4096, 8192, 16384) if TM <= 2 * R * NT
    for K in (6, 3, 0)
]


@pytest.mark.parametrize("opt", TUNINGS, ids=lambda o: "R{keys_per_lane}_NT{block_threads}_TM{merge_tile}_K{wave_levels}".format(**o))
def test_sort_every_tuning(opt):
    n = 5 * opt["keys_per_lane"] * opt["block_threads"] + 12345
    x = inputs.keys(n, "zipf", seed=7, device=DEV)
    y = hv.sort(x, opts=opt)
    assert np.array_equal(y.cpu().numpy(), oracle.sort(x.cpu().numpy()))


def test_sort_on_a_side_stream():
    s = torch.cuda.Stream()
    x = inputs.keys(1 << 20, "uniform", seed=9, device=DEV)
    with torch.cuda.stream(s):
        y = hv.sort(x)
    s.synchronize()
    assert np.array_equal(y.cpu().numpy(), oracle.sort(x.cpu().numpy()))


# ------------------------------------------------------------- pairs

@pytest.mark.parametrize("n", [1, 17, 4097, 65537, 1000003])
@pytest.mark.parametrize("dist", ["uniform", "distinct16", "zipf", "reverse"])
def test_sort_pairs_match_oracle(n, dist):
    _say("pairs", n, dist)
    k = inputs.keys(n, dist, seed=n, device=DEV)
    v = torch.randint(-3, 3, (n,), device=DEV, dtype=torch.int32)
    ko, vo = hv.sort_pairs(k, v)
    ek, ev = oracle.sort_pairs(k.cpu().numpy(), v.cpu().numpy())
    assert np.array_equal(ko.cpu().numpy(), ek) and np.array_equal(vo.cpu().numpy(), ev)


@pytest.mark.parametrize("opt", [dict(keys_per_lane=R, block_threads=NT, merge_tile=TM)
                                 for R, NT in [(16, 256), (16, 512), (8, 1024), (32, 256), (16, 1024)]
                                 for TM in (2048, 4096, 8192) if TM <= 2 * R * NT])
def test_sort_pairs_every_tuning(opt):
    n = 3 * opt["keys_per_lane"] * opt["block_threads"] + 999
    k, v = inputs.pairs(n, "distinct16", seed=1, device=DEV)
    ko, vo = hv.sort_pairs(k, v, opts=opt)
    ek, ev = oracle.sort_pairs(k.cpu().numpy(), v.cpu().numpy())
    assert np.array_equal(ko.cpu().numpy(), ek) and np.array_equal(vo.cpu().numpy(), ev)


# ------------------------------------------------- merge pass and co-rank

@pytest.mark.parametrize("run", [4096, 8192, 65536])
@pytest.mark.parametrize("n_runs", [1, 2, 3, 7])
def test_merge_pass_matches_oracle(run, n_runs):
    n = run * n_runs - (run // 3 if n_runs > 1 else 0)
    x = inputs.keys(n, "distinct16", seed=run + n_runs, device=DEV).cpu().numpy()
    offs = np.append(np.arange(0, n, run), n)
    runs = oracle.segmented_sort(x, offs)
    y = hv.merge_pass(torch.from_numpy(runs).to(DEV), run).cpu().numpy()
    want = np.concatenate([oracle.merge(runs[a:min(a + run, n)], runs[min(a + run, n):min(a + 2 * run, n)])
                           for a in range(0, n, 2 * run)])
    assert np.array_equal(y, want)


@pytest.mark.parametrize("tm", [2048, 4096, 8192, 16384])
@pytest.mark.parametrize("variant", [2, 4])
@pytest.mark.parametrize("dist", ["uniform", "distinct16", "sorted"])
def test_merge_pass_serial_and_bitonic_mergers(tm, variant, dist):
    # the two per-thread mergers (serial, bitonic network in registers) at
    # VT = 8, 16, 16, 32 outputs per thread, ragged last pair
    run = 16384
    n = 5 * run + 4321
    x = inputs.keys(n, dist, seed=tm + variant, device=DEV).cpu().numpy()
    offs = np.append(np.arange(0, n, run), n)
    runs = oracle.segmented_sort(x, offs)
    y = hv.merge_pass(torch.from_numpy(runs).to(DEV), run,
                      opts={"merge_tile": tm, "merge_variant": variant,
                            "keys_per_lane": 32, "block_threads": 512}).cpu().numpy()
    want = np.concatenate([oracle.merge(runs[a:min(a + run, n)], runs[min(a + run, n):min(a + 2 * run, n)])
                           for a in range(0, n, 2 * run)])
    assert np.array_equal(y, want)


@pytest.mark.parametrize("tm", [2048, 8192, 16384])
def test_sort_with_bitonic_merger(tm):
    n = 3 * 16384 * 8 + 77
    x = inputs.keys(n, "zipf", seed=tm, device=DEV)
    y = hv.sort(x, opts={"keys_per_lane": 32, "block_threads": 512, "merge_tile": tm,
                         "merge_variant": 4})
    assert np.array_equal(y.cpu().numpy(), oracle.sort(x.cpu().numpy()))


@pytest.mark.parametrize("mode", [hv.CORANK_BINARY, hv.CORANK_LINEAR])
@pytest.mark.parametrize("seed", range(6))
def test_corank_all_diagonals_match_oracle(mode, seed):
    rng = np.random.default_rng(seed)
    m, k = int(rng.integers(0, 3000)), int(rng.integers(0, 3000))
    hi = int(rng.integers(1, 50))
    A = np.sort(rng.integers(0, hi, m)).astype(np.int32)
    B = np.sort(rng.integers(0, hi, k)).astype(np.int32)
    diag = np.arange(-1, m + k + 2, dtype=np.int64)
    got = hv.corank(torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV),
                    torch.from_numpy(diag).to(DEV), opts={"corank_mode": mode, "radius_log2": 3}).cpu().numpy()
    want = [oracle.corank(A, B, int(d)) for d in diag]
    assert got.tolist() == want


def test_corank_stats_count_probes():
    A = torch.arange(0, 2000000, 2, device=DEV, dtype=torch.int32)
    B = torch.arange(1, 2000000, 2, device=DEV, dtype=torch.int32)
    diag = torch.arange(1, 2000000, 1001, device=DEV, dtype=torch.int64)
    st = torch.zeros(hv.STATS_WORDS, dtype=torch.int64, device=DEV)
    got = hv.corank(A, B, diag, opts={"corank_mode": hv.CORANK_LINEAR, "radius_log2": 4, "stats": st})
    assert torch.equal(got, (diag + 1) // 2)
    s = st.cpu().tolist()
    assert s[0] == diag.numel() and s[2] == 0          # interleaved runs: prediction exact
    assert s[1] <= diag.numel() * 7                     # bracket check + log2(2 * 16) + 1


# ------------------------------------------------------- full-size check

def _full_check(x, y):
    xs, ys = x.cpu().numpy(), y.cpu().numpy()
    assert np.all(ys[1:] >= ys[:-1])
    assert oracle.multiset_hash(ys) == oracle.multiset_hash(xs)
    n = xs.size
    for p in [0, 1, n // 3, n // 2, n - 2, n - 1]:
        lt, le = oracle.count(xs, ys[p])
        assert lt <= p < le, p


_EXPECTED = {}


def expected_2p28(dist, seed=0):
    """(input on the host, oracle's sorted array) of the 2^28-key benchmark
    input of one distribution; kept for the tests that sort the same input."""
    key = (dist, seed)
    if key not in _EXPECTED:
        _EXPECTED.clear()
        xs = inputs.keys(1 << 28, dist, seed=seed, device=DEV).cpu().numpy()
        _EXPECTED[key] = (xs, oracle_parts.sort_in_parts(xs, parts=16, threads=16))
    return _EXPECTED[key]


@pytest.mark.parametrize("dist", inputs.DISTRIBUTIONS)
def test_full_size_2pow28(dist):
    # the benchmark's workload in its launch configuration (the tuned
    # options for 2^28 keys: four-way passes, seven merge launches over
    # runs up to 2^27), compared element by element with the oracle
    n = 1 << 28
    _say("full size", dist)
    xs, want = expected_2p28(dist)
    x = torch.from_numpy(xs).to(DEV)
    y = hv.sort(x)
    torch.cuda.synchronize()
    assert np.array_equal(y.cpu().numpy(), want)
    if dist == "uniform":    # the same input, two-way passes (the best two-way shape)
        from paper_2409_03970_amd import tune
        o2 = tune.tuned_options("sort", n, two_way=True)
        if o2:
            y = hv.sort(x, opts=o2)
            assert np.array_equal(y.cpu().numpy(), want)


def test_full_size_pairs_2pow28():
    # the key-value sort in its tuned launch shape for 2^28 pairs (four-way
    # passes); values are the input indices, so the (key, value) order is
    # unique: keys element by element against the oracle, values a
    # permutation that ascends within every run of equal keys and points
    # back at its key
    n = 1 << 28
    _say("full size pairs")
    xs, want = expected_2p28("uniform")
    k = torch.from_numpy(xs).to(DEV)
    v = torch.arange(n, dtype=torch.int32, device=DEV)
    ko, vo = hv.sort_pairs(k, v)
    torch.cuda.synchronize()
    assert np.array_equal(ko.cpu().numpy(), want)
    assert bool(torch.equal(k[vo.long()], ko))
    assert bool(((ko[1:] > ko[:-1]) | (vo[1:] > vo[:-1])).all())
    assert bool(torch.equal(torch.sort(vo).values, v))


@pytest.mark.parametrize("ways", [2, 4])
def test_beyond_2pow31_keys(ways):
    # more keys than a 32-bit index reaches (8.6 GB), ragged: every index,
    # tile count and co-rank path must be 64-bit
    n = (1 << 31) + 1003
    _say("beyond 2^31, ways", ways)
    x = inputs.keys(n, "uniform", seed=31, device=DEV)
    opts = {"keys_per_lane": 32, "block_threads": 512, "merge_tile": 8192, "merge_ways": ways}
    y = hv.sort(x, opts=opts)
    torch.cuda.synchronize()
    assert bool((y[1:] >= y[:-1]).all())
    del x
    torch.cuda.empty_cache()
    x = inputs.keys(n, "uniform", seed=31, device=DEV)   # the same input again
    _full_check(x, y)


@pytest.mark.parametrize("net", [1, 2])
def test_alternative_column_networks_all_01_inputs(net):
    # the Table 1 alternatives (odd-even 63, bitonic 80) through the real kernel
    x = _runs_from_bits(16, 16)
    y = hv.sort_runs(x, 4, opts={"keys_per_lane": 16, "block_threads": 256, "column_network": net})
    ones = x.view(-1, 16).sum(1)
    want = (torch.arange(16, device=DEV)[None, :] >= (16 - ones)[:, None]).to(torch.int32)
    assert torch.equal(y.view(-1, 16), want)


@pytest.mark.parametrize("net", [1, 2])
@pytest.mark.parametrize("NT", [256, 512, 1024])
def test_alternative_column_networks_full_sort(net, NT):
    n = 5 * 16 * NT + 777
    x = inputs.keys(n, "gaussian", seed=net, device=DEV)
    y = hv.sort(x, opts={"keys_per_lane": 16, "block_threads": NT, "column_network": net})
    assert np.array_equal(y.cpu().numpy(), oracle.sort(x.cpu().numpy()))


def test_sort_every_size_up_to_130():
    for n in range(1, 131):
        x = inputs.keys(n, "uniform", seed=1000 + n, device=DEV)
        y = hv.sort(x)
        assert np.array_equal(y.cpu().numpy(), oracle.sort(x.cpu().numpy())), n


@pytest.mark.parametrize("k", range(1, 25))
def test_sort_powers_of_two_and_neighbours(k):
    for n in ((1 << k) - 1, 1 << k, (1 << k) + 1):
        _say("sort n =", n)
        x = inputs.keys(n, "zipf", seed=k, device=DEV)
        y = hv.sort(x)
        assert np.array_equal(y.cpu().numpy(), oracle.sort(x.cpu().numpy())), n


# -------------------------------------------- presorted and reverse-sorted tiles

def _near_sorted(n, pos, seed, descending=False):
    """Sorted (or reverse-sorted) keys with the pair at pos swapped, so that
    exactly one adjacent pair breaks the order."""
    rng = np.random.default_rng(seed)
    x = np.sort(rng.integers(-2**31, 2**31, size=n, dtype=np.int64).astype(np.int32))
    if descending:
        x = x[::-1].copy()
    if pos is not None:
        x[pos], x[pos + 1] = x[pos + 1], x[pos]
    return x


@pytest.mark.parametrize("shape", [(16, 1024), (32, 512), (8, 256)])
@pytest.mark.parametrize("descending", [False, True])
def test_presorted_tiles_and_near_misses(shape, descending):
    R, NT = shape
    tile = R * NT
    opts = {"keys_per_lane": R, "block_threads": NT}
    # swaps: inside a lane's elements (64 apart), across lanes, across waves,
    # across tiles, at the tile's very start and end
    for pos in (None, 0, 5, 63, 64 * R - 1, 64 * R, 3 * 64 * R - 1, tile - 2, tile - 1,
                tile + 100, 2 * tile - 1):
        x = _near_sorted(4 * tile + 777, pos, seed=R + (pos or 0), descending=descending)
        _say("presorted", shape, descending, pos)
        y = hv.sort(torch.from_numpy(x).to(DEV), opts=opts).cpu().numpy()
        assert np.array_equal(y, np.sort(x)), pos
        # one tile only (the block stage is the whole sort)
        x1 = x[:tile]
        y1 = hv.sort(torch.from_numpy(x1.copy()).to(DEV), opts=opts).cpu().numpy()
        assert np.array_equal(y1, np.sort(x1)), pos


def test_presorted_ties_constants_and_mixed_tiles():
    rng = np.random.default_rng(5)
    tile = 16384
    parts = [np.full(tile, 7, np.int32),                                   # constant tile
             np.sort(rng.integers(0, 10, tile)).astype(np.int32),          # ties, ascending
             np.sort(rng.integers(0, 10, tile)).astype(np.int32)[::-1],    # ties, descending
             rng.integers(-2**31, 2**31, tile, dtype=np.int64).astype(np.int32),  # random
             np.arange(tile, 0, -1, dtype=np.int32),                       # strictly descending
             np.concatenate([np.arange(tile // 2), np.arange(tile // 2)]).astype(np.int32)]
    x = np.concatenate(parts)
    for opts in ({}, {"keys_per_lane": 32, "block_threads": 512, "merge_ways": 4}):
        y = hv.sort(torch.from_numpy(x).to(DEV), opts=opts).cpu().numpy()
        assert np.array_equal(y, np.sort(x))


@pytest.mark.parametrize("descending", [False, True])
def test_presorted_pairs_and_other_key_types(descending):
    n = 3 * 16384 + 5
    k = _near_sorted(n, None, seed=9, descending=descending)
    v = np.arange(n, dtype=np.int32)                    # ties in k keep pair order distinct
    ko, vo = hv.sort_pairs(torch.from_numpy(k).to(DEV), torch.from_numpy(v).to(DEV))
    ek, ev = oracle.sort_pairs(k, v)
    assert np.array_equal(ko.cpu().numpy(), ek) and np.array_equal(vo.cpu().numpy(), ev)
    # uint32 / float32 / 64-bit keys: the order is checked on the mapped keys
    u = np.sort(np.random.default_rng(1).integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32))
    u = u[::-1].copy() if descending else u
    yu = hv.sort_keys(torch.from_numpy(u.view(np.int32)).to(DEV).view(torch.uint32))
    assert np.array_equal(yu.view(torch.int32).cpu().numpy().view(np.uint32), oracle.sort_u32(u))
    f = np.sort(np.random.default_rng(2).standard_normal(n).astype(np.float32))
    f = f[::-1].copy() if descending else f
    yf = hv.sort_keys(torch.from_numpy(f).to(DEV))
    assert np.array_equal(yf.view(torch.int32).cpu().numpy(),
                          oracle.sort_f32(f).view(np.int32))
    d = np.sort(np.random.default_rng(3).standard_normal(16384))
    d = d[::-1].copy() if descending else d
    yd = hv.sort_keys(torch.from_numpy(d).to(DEV))          # full tiles read packed
    assert np.array_equal(yd.cpu().numpy().view(np.uint64), oracle.sort_f64(d).view(np.uint64))


# ----------------------------------------------- conveniences on a side stream

@pytest.mark.parametrize("shape", [(32, 512), (16, 512), (32, 256), (16, 1024)])
@pytest.mark.parametrize("order", ["descending_blocks", "ascending_blocks", "one_sided_ties"])
def test_lds_levels_exhausted_runs(shape, order):
    # tiles whose wave runs have disjoint key ranges (each run random inside,
    # so the tile is not presorted): at every LDS merge level one run of a
    # pair is exhausted part way, including at the tile's last element, the
    # read the branch-free serial merge clamps; ties between runs where the
    # A-first rule makes every share one-sided
    R, NT = shape
    tile, wave = R * NT, 64 * R
    n = 3 * tile + 4 * wave + 77
    rng = np.random.default_rng(R + NT)
    blk = np.arange(n) // wave
    if order == "descending_blocks":
        x = (1000 - blk) * 100000 + rng.integers(0, 100000, n)
    elif order == "ascending_blocks":
        x = blk * 100000 + rng.integers(0, 100000, n)
    else:
        x = np.where(blk % 2 == 0, 7, rng.integers(-5, 7, n))
    x = x.astype(np.int32)
    _say("exhausted runs", shape, order)
    y = hv.sort(torch.from_numpy(x).to(DEV), opts={"keys_per_lane": R, "block_threads": NT})
    assert np.array_equal(y.cpu().numpy(), oracle.sort(x))


def test_sort_on_side_stream_while_current_stream_allocates():
    # the convenience wrappers allocate their workspace for the stream the
    # kernels run on: memory freed when the call returns must not be handed
    # to work on the current stream while the side stream still sorts
    n = 1 << 24
    x = inputs.keys(n, "uniform", seed=77, device=DEV)
    want = oracle.sort(x.cpu().numpy())
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    for rep in range(3):
        y = hv.sort(x, stream=side)
        yk, yv = hv.sort_pairs(x, x, stream=side)
        # the current stream reuses whatever the allocator hands out, at once
        junk = [torch.full((n + 1024,), -1, dtype=torch.int32, device=DEV) for _ in range(6)]
        side.synchronize()
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy(), want), rep
        assert np.array_equal(yk.cpu().numpy(), want), rep
        del junk, y, yk, yv


# ------------------------------------------- four keys per lane (Table 2, R = 4)

@pytest.mark.parametrize("NT", [256, 512, 1024])
def test_four_keys_per_lane_sort(NT):
    for n, dist in ((3 * 4 * NT + 77, "uniform"), (200_003, "zipf"), (4 * NT, "reverse")):
        x = inputs.keys(n, dist, seed=NT + n, device=DEV)
        y = hv.sort(x, opts={"keys_per_lane": 4, "block_threads": NT})
        assert np.array_equal(y.cpu().numpy(), oracle.sort(x.cpu().numpy())), (NT, n, dist)
    x = inputs.keys(100_000, "gaussian", seed=3, device=DEV)
    for run_log2 in range(2, int(np.log2(4 * NT)) + 1):
        y = hv.sort_runs(x, run_log2, opts={"keys_per_lane": 4, "block_threads": NT}).cpu().numpy()
        xs = x.cpu().numpy()
        X = 1 << run_log2
        offs = np.append(np.arange(0, xs.size, X), xs.size).astype(np.int64)
        assert np.array_equal(y, oracle.segmented_sort(xs, offs)), run_log2


def test_four_keys_per_lane_rejected_for_pairs():
    k = torch.zeros(100000, dtype=torch.int32, device=DEV)
    with pytest.raises(hv.HvmsError):
        hv.sort_pairs(k, k.clone(), opts={"keys_per_lane": 4})
