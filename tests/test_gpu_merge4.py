"""GPU parity of the four-way merge passes (two merge levels per pass)
against the CPU oracle, bit-exact."""
import numpy as np
import pytest
import torch

import oracle
import paper_2409_03970_amd as hv
from paper_2409_03970_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _check(x, opts):
    y = hv.sort(x, opts=opts)
    assert np.array_equal(y.cpu().numpy(), oracle.sort(x.cpu().numpy())), opts


@pytest.mark.parametrize("tiles", [2, 3, 4, 5, 7, 8, 9, 16, 17, 33, 64])
@pytest.mark.parametrize("tm", [4096, 8192])
def test_four_way_level_counts_and_partial_groups(tiles, tm):
    # R16 x 256 threads: 4096-key block tiles; odd and even level counts,
    # groups with 1..3 runs at the end, ragged last run
    n = tiles * 4096 - (1000 if tiles > 2 else 0)
    x = inputs.keys(n, "uniform", seed=tiles, device=DEV)
    _check(x, {"keys_per_lane": 16, "block_threads": 256, "merge_tile": tm, "merge_ways": 4})


@pytest.mark.parametrize("tiles", [62, 63, 64, 65, 126, 127, 128, 190])
@pytest.mark.parametrize("dist", ["uniform", "sorted", "reverse", "distinct16"])
def test_four_way_tile_records_across_wave_boundaries(tiles, dist):
    # the co-rank kernel writes each tile's geometry record from its own
    # co-ranks and the next tile's (the next lane's; every 64-lane wave owns
    # 63 tiles): tile counts on both sides of multiples of 63, full and
    # ragged last tiles
    for ragged in (0, 777):
        n = tiles * 4096 - ragged
        x = inputs.keys(n, dist, seed=tiles, device=DEV)
        _check(x, {"keys_per_lane": 16, "block_threads": 256, "merge_tile": 4096, "merge_ways": 4})


@pytest.mark.parametrize("dist", list(inputs.DISTRIBUTIONS) + ["mixture"])
@pytest.mark.parametrize("mode", [hv.CORANK_BINARY, hv.CORANK_LINEAR])
def test_four_way_distributions(dist, mode):
    x = inputs.keys(3_000_007, dist, seed=3, device=DEV)
    _check(x, {"merge_ways": 4, "corank_mode": mode, "radius_log2": 9})


@pytest.mark.parametrize("pattern", ["equal", "two_values", "extremes", "negatives"])
def test_four_way_adversarial(pattern):
    x = inputs.adversarial_keys(1_000_003, pattern, seed=4, device=DEV)
    _check(x, {"merge_ways": 4, "merge_tile": 4096})


@pytest.mark.parametrize("shape", [(8, 1024), (16, 512), (16, 1024), (32, 256), (32, 512)])
def test_four_way_tile_shapes(shape):
    R, NT = shape
    x = inputs.keys(40 * R * NT + 12345, "zipf", seed=5, device=DEV)
    _check(x, {"keys_per_lane": R, "block_threads": NT, "merge_ways": 4})


@pytest.mark.parametrize("tm", [2048, 4096])
def test_four_way_pairs(tm):
    n = 2_000_003
    k = inputs.keys(n, "distinct16", seed=6, device=DEV)
    v = torch.randint(-5, 5, (n,), device=DEV, dtype=torch.int32)
    ko, vo = hv.sort_pairs(k, v, opts={"merge_ways": 4, "merge_tile": tm})
    ek, ev = oracle.sort_pairs(k.cpu().numpy(), v.cpu().numpy())
    assert np.array_equal(ko.cpu().numpy(), ek) and np.array_equal(vo.cpu().numpy(), ev)


@pytest.mark.parametrize("dist", ["uniform", "zipf"])
def test_four_way_full_size(dist):
    # 2^28 keys, four-way passes with the default tile shape (R = 16, 8192-key
    # block tiles: one two-way launch, then six four-way launches), element
    # by element against the oracle
    import oracle_parts
    n = 1 << 28
    x = inputs.keys(n, dist, seed=5, device=DEV)
    y = hv.sort(x, opts={"merge_ways": 4})
    torch.cuda.synchronize()
    want = oracle_parts.sort_in_parts(x.cpu().numpy(), parts=16, threads=16)
    assert np.array_equal(y.cpu().numpy(), want)


@pytest.mark.parametrize("offset", [1, 2, 3])
def test_four_way_requested_with_unaligned_output(offset):
    # an output that is not 16-byte aligned takes two-way passes (the
    # four-way kernel moves 16-byte chunks of the arrays it writes)
    n = 1_000_003
    x = inputs.keys(n, "uniform", seed=7 + offset, device=DEV)
    big = torch.empty(n + offset, dtype=torch.int32, device=DEV)
    y = big[offset:]
    assert y.data_ptr() % 16 != 0
    opts = {"merge_ways": 4, "merge_tile": 8192}
    ws = hv._workspace(hv.lib().hvms_sort_workspace_bytes(n, 0, hv._opts(opts)), x.device)
    hv.hvms_sort_i32(x, y, ws, opts=opts)
    assert np.array_equal(y.cpu().numpy(), oracle.sort(x.cpu().numpy()))
    k = inputs.keys(n, "distinct16", seed=8, device=DEV)
    v = torch.randint(-5, 5, (n,), device=DEV, dtype=torch.int32)
    vbig = torch.empty(n + offset, dtype=torch.int32, device=DEV)
    popts = {"merge_ways": 4, "merge_tile": 4096}
    ws = hv._workspace(hv.lib().hvms_sort_workspace_bytes(n, 1, hv._opts(popts)), x.device)
    ko = torch.empty_like(k)
    hv.hvms_sort_pairs_i32(k, v, ko, vbig[offset:], ws, opts=popts)
    ek, ev = oracle.sort_pairs(k.cpu().numpy(), v.cpu().numpy())
    assert np.array_equal(ko.cpu().numpy(), ek)
    assert np.array_equal(vbig[offset:].cpu().numpy(), ev)


@pytest.mark.parametrize("tiles", [2, 3, 4, 5, 8, 9, 17, 33])
def test_four_way_tile_16384(tiles):
    # R16 x 512 threads: 8192-key block tiles, four-way merge tiles of 16384
    n = tiles * 8192 - (777 if tiles > 2 else 0)
    x = inputs.keys(n, "zipf", seed=40 + tiles, device=DEV)
    _check(x, {"keys_per_lane": 16, "block_threads": 512, "merge_tile": 16384, "merge_ways": 4})


@pytest.mark.parametrize("dist", ["uniform", "mixture", "zipf", "sorted", "distinct16"])
def test_four_way_every_corank_mode_exact(dist):
    # the four-way co-ranks are selected in the runs directly in every mode;
    # the mode steers the two-way pass that an odd level count adds (9
    # levels here: one two-way pass, then four four-way passes)
    n = 3_000_017
    x = inputs.keys(n, dist, seed=12, device=DEV)
    want = oracle.sort(x.cpu().numpy())
    params = hv.fit_cdf_model(x, frac=0.02, steps=150, batch=8192, lr=3e-3, seed=12)
    counts = {}
    for mode in (hv.CORANK_BINARY, hv.CORANK_LINEAR, hv.CORANK_LEARNED):
        st = torch.zeros(hv.STATS_WORDS, dtype=torch.int64, device=DEV)
        y = hv.sort(x, opts={"keys_per_lane": 16, "block_threads": 512, "merge_ways": 4,
                             "corank_mode": mode, "cdf_params": params, "stats": st})
        assert np.array_equal(y.cpu().numpy(), want), mode
        counts[mode] = int(st[0])
    assert len(set(counts.values())) == 1
