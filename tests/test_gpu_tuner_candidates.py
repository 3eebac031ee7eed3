"""Every configuration the autotuner may pick, for each operation, sorts
bit-exactly (so a tuned choice can never change a result)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2409_03970_amd as hv
from paper_2409_03970_amd import inputs, tune

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _id(o):
    return "R{keys_per_lane}_NT{block_threads}_K{wave_levels}_TM{merge_tile}_V{merge_variant}_W{merge_ways}".format(**o)


@pytest.mark.parametrize("opt", tune.candidates("sort"), ids=_id)
def test_sort_candidate(opt):
    n = 5 * opt["keys_per_lane"] * opt["block_threads"] + 12345
    x = inputs.keys(n, "zipf", seed=3, device=DEV)
    y = hv.sort(x, opts=opt)
    assert np.array_equal(y.cpu().numpy(), oracle.sort(x.cpu().numpy()))


@pytest.mark.parametrize("opt", tune.candidates("sort_pairs"), ids=_id)
def test_sort_pairs_candidate(opt):
    n = 5 * opt["keys_per_lane"] * opt["block_threads"] + 777
    k = inputs.keys(n, "distinct16", seed=4, device=DEV)
    v = torch.randint(-9, 9, (n,), dtype=torch.int32, device=DEV)
    ko, vo = hv.sort_pairs(k, v, opts=opt)
    ek, ev = oracle.sort_pairs(k.cpu().numpy(), v.cpu().numpy())
    assert np.array_equal(ko.cpu().numpy(), ek) and np.array_equal(vo.cpu().numpy(), ev)


@pytest.mark.parametrize("opt", tune.candidates("segmented"), ids=_id)
def test_segmented_candidate(opt):
    sizes = inputs.log_uniform_sizes(300, 1, 3 * opt["keys_per_lane"] * opt["block_threads"],
                                     seed=5)
    offs = inputs.offsets_from_sizes(sizes)
    n = int(offs[-1])
    k = inputs.keys(n, "uniform", seed=6, device=DEV)
    y = hv.segmented_sort(k, offs, opts=opt)
    assert np.array_equal(y.cpu().numpy(), oracle.segmented_sort(k.cpu().numpy(), offs.numpy()))
