"""The two in-register mergers of Table 3 (hybrid and pure cross-lane) on the
GPU, through the C ABI: every pair of sorted runs of X keys merged into one
sorted run of 2X, element by element against the oracle, for every width,
both forms and repeated merges."""
import numpy as np
import pytest
import torch

import oracle
import paper_2409_03970_amd as hv
from paper_2409_03970_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _runs(n, X, dist, seed):
    """n keys of a distribution, each run of X sorted by the oracle."""
    x = inputs.keys(n, dist, seed=seed, device="cpu").numpy()
    offs = np.arange(0, n + 1, X, dtype=np.int64)
    return oracle.segmented_sort(x, offs)


@pytest.mark.parametrize("x_log2", [3, 4, 5])
@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("dist", ["uniform", "distinct16", "sorted", "reverse"])
def test_merge_runs_match_oracle(x_log2, form, dist):
    X = 1 << x_log2
    n = 256 * X * 37
    runs = _runs(n, X, dist, seed=x_log2 * 10 + form)
    offs2 = np.arange(0, n + 1, 2 * X, dtype=np.int64)
    want = oracle.segmented_sort(runs, offs2)
    d_in = torch.from_numpy(runs).to(DEV)
    for reps in (1, 3):
        out = torch.full_like(d_in, -1)
        hv.hvms_merge_runs_i32(d_in, out, x_log2, form, reps)
        assert np.array_equal(out.cpu().numpy(), want), reps


def test_merge_runs_all_01_sorted_halves():
    # every sorted-halves 0-1 input of 2X keys (X = 8: 81 of them), repeated
    # to fill 256 runs, both forms
    X = 8
    combos = [(a, b) for a in range(X + 1) for b in range(X + 1)]
    pos = np.arange(X)
    rows = [np.concatenate([pos >= a, pos >= b]).astype(np.int32)
            for a, b in (combos * 4)[:256]]
    x = np.concatenate(rows)
    want = np.concatenate([np.sort(r) for r in rows])
    for form in (0, 1):
        out = torch.empty(x.size, dtype=torch.int32, device=DEV)
        hv.hvms_merge_runs_i32(torch.from_numpy(x).to(DEV), out, 3, form)
        assert np.array_equal(out.cpu().numpy(), want), form


def test_merge_runs_argument_errors():
    x = torch.zeros(256 * 8 + 8, dtype=torch.int32, device=DEV)
    with pytest.raises(hv.HvmsError):
        hv.hvms_merge_runs_i32(x, x, 3, 0)           # not a multiple of 256 X
    y = torch.zeros(256 * 8, dtype=torch.int32, device=DEV)
    for bad in ((2, 0, 1), (6, 0, 1), (3, 2, 1), (3, 0, 0)):
        with pytest.raises(hv.HvmsError):
            hv.hvms_merge_runs_i32(y, y, *bad)
