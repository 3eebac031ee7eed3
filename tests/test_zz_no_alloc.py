"""The allocation-free sort entry point against the workspace one, through
the C ABI: bit-exact on consecutive calls (the second smaller than the
first, so stale scratch from the first call is present), every launch shape
it shares with hvms_sort_i32, and the size limit reported as an error."""
import numpy as np
import pytest
import torch

import oracle
import paper_2409_03970_amd as hv
from paper_2409_03970_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _with_ws(x, opts):
    y = torch.empty_like(x)
    ws = hv._workspace(hv.lib().hvms_sort_workspace_bytes(x.numel(), 0, hv._opts(opts)),
                       x.device)
    hv.hvms_sort_i32(x, y, ws, opts=opts)
    return y


@pytest.mark.parametrize("opts", [None,
                                  {"merge_ways": 4},
                                  {"keys_per_lane": 32, "block_threads": 512, "merge_ways": 4},
                                  {"keys_per_lane": 8, "block_threads": 256, "merge_tile": 2048}],
                         ids=["default", "four_way", "r32_four_way", "r8_tm2048"])
def test_noalloc_matches_workspace_sort_on_two_calls(opts):
    print("noalloc", opts, flush=True)
    for n, dist, seed in ((hv.SORT_NOALLOC_MAX_KEYS, "uniform", 1),
                          (3_000_017, "zipf", 2),
                          (200_003, "distinct16", 3)):
        x = inputs.keys(n, dist, seed=seed, device=DEV)
        y = torch.full_like(x, -1)
        hv.hvms_sort_i32_noalloc(x, y, opts=opts)
        ref = _with_ws(x, opts)
        torch.cuda.synchronize()
        assert torch.equal(y, ref), (n, dist)
        assert np.array_equal(y.cpu().numpy(), oracle.sort(x.cpu().numpy())), (n, dist)


def test_noalloc_small_in_place_and_empty():
    for n in (1, 17, 8192, 8193, 65537):
        x = inputs.keys(n, "reverse", seed=n, device=DEV)
        want = oracle.sort(x.cpu().numpy())
        hv.hvms_sort_i32_noalloc(x, x)                # in place
        assert np.array_equal(x.cpu().numpy(), want), n
    e = torch.empty(0, dtype=torch.int32, device=DEV)
    hv.hvms_sort_i32_noalloc(e, e)


def test_noalloc_rejects_sizes_beyond_its_scratch():
    n = hv.SORT_NOALLOC_MAX_KEYS + 1
    x = torch.zeros(n, dtype=torch.int32, device=DEV)
    y = torch.full_like(x, 5)
    with pytest.raises(hv.HvmsError) as e:
        hv.hvms_sort_i32_noalloc(x, y)
    assert e.value.status == -5
    torch.cuda.synchronize()
    assert bool((y == 5).all())            # nothing was enqueued


def test_noalloc_on_a_side_stream_and_in_a_graph():
    n = 1_000_003
    x = inputs.keys(n, "gaussian", seed=9, device=DEV)
    want = _with_ws(x, None)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    y = torch.empty_like(x)
    with torch.cuda.stream(s):
        hv.hvms_sort_i32_noalloc(x, y, stream=s)
    s.synchronize()
    assert torch.equal(y, want)
    # captured: no allocation inside the call, so the graph replays it as is
    y.fill_(0)
    g = torch.cuda.CUDAGraph()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            hv.hvms_sort_i32_noalloc(x, y, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        y.fill_(0)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, want), rep
        _with_ws(x[: n // 2], None)          # eager work between replays
