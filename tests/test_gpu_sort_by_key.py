"""GPU parity of the stable sort by key with 64-bit payloads against the
oracle, bit-exact, through the C ABI: heavy ties (where stability decides
the payload order), the int32 extremes, ragged sizes, the block-only path,
two-way and four-way passes, in-place keys, payload outputs that are only
8-byte aligned, payload dtypes int64 / uint64 / float64 (bit patterns,
NaNs included, come back unchanged), and 2^26 keys."""
import numpy as np
import pytest
import torch

import oracle
import paper_2409_03970_amd as hv

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _say(*a):
    print(*a, flush=True)


def _inputs(n, seed, ties):
    rng = np.random.default_rng(seed)
    if ties:
        k = rng.integers(-8, 8, size=n).astype(np.int32)
    else:
        k = rng.integers(-2**31, 2**31, size=n, dtype=np.int64).astype(np.int32)
    k[: n // 9] = rng.choice(np.array([-2**31, 2**31 - 1, 0], dtype=np.int32), size=n // 9)
    v = rng.integers(0, 2**64, size=n, dtype=np.uint64)
    return k, v


def _run(k, v, opts, vals_dtype=torch.int64, vout=None):
    kd = torch.from_numpy(k).to(DEV)
    vd = torch.from_numpy(v.view(np.int64)).to(DEV).view(vals_dtype)
    ko = torch.empty_like(kd)
    vo = torch.empty_like(vd) if vout is None else vout
    ws = hv._workspace(hv.lib().hvms_sort_by_key_workspace_bytes(k.size, hv._opts(opts)), kd.device)
    hv.hvms_sort_by_key_i32_p64(kd, vd, ko, vo, ws, opts=opts)
    torch.cuda.synchronize()
    return ko.cpu().numpy(), vo.view(torch.int64).cpu().numpy().view(np.uint64), kd, vd


SHAPES = [
    {},
    {"keys_per_lane": 8, "block_threads": 256, "merge_tile": 2048},
    {"keys_per_lane": 16, "block_threads": 1024, "merge_tile": 4096, "wave_levels": 5},
    {"keys_per_lane": 16, "block_threads": 512, "merge_tile": 8192, "merge_variant": 1},
    {"keys_per_lane": 16, "block_threads": 512, "merge_tile": 4096, "merge_ways": 4},
]


@pytest.mark.parametrize("ties", [True, False])
@pytest.mark.parametrize("n", [1, 7, 2048, 8193, 40000, 300007, (1 << 20) + 3])
@pytest.mark.parametrize("shape", range(len(SHAPES)))
def test_sort_by_key_matches_oracle(ties, n, shape):
    opts = SHAPES[shape]
    _say("sort_by_key", ties, n, opts)
    k, v = _inputs(n, seed=n + 13 * shape + ties, ties=ties)
    ko, vo, kd, vd = _run(k, v, opts)
    ek, ev = oracle.sort_by_key_p64(k, v)
    assert np.array_equal(ko, ek)
    assert np.array_equal(vo, ev)
    assert np.array_equal(kd.cpu().numpy(), k)        # inputs untouched
    assert np.array_equal(vd.view(torch.int64).cpu().numpy().view(np.uint64), v)


@pytest.mark.parametrize("dtype", [torch.int64, torch.uint64, torch.float64])
def test_payload_dtypes_bits_preserved(dtype):
    n = 100003
    k, v = _inputs(n, seed=21, ties=True)             # random bits: many float64 NaNs
    _say("sort_by_key dtype", dtype)
    ko, vo, _, _ = _run(k, v, {}, vals_dtype=dtype)
    ek, ev = oracle.sort_by_key_p64(k, v)
    assert np.array_equal(ko, ek) and np.array_equal(vo, ev)


@pytest.mark.parametrize("shape", [0, 4])
def test_payload_output_only_8_byte_aligned(shape):
    n = 300007
    k, v = _inputs(n, seed=22, ties=True)
    big = torch.empty(n + 1, dtype=torch.int64, device=DEV)
    vout = big[1:]
    assert vout.data_ptr() % 16 == 8
    _say("sort_by_key misaligned payload out", SHAPES[shape])
    ko, vo, _, _ = _run(k, v, SHAPES[shape], vout=vout)
    ek, ev = oracle.sort_by_key_p64(k, v)
    assert np.array_equal(ko, ek) and np.array_equal(vo, ev)


def test_keys_in_place():
    n = 1000003
    k, v = _inputs(n, seed=23, ties=True)
    kd = torch.from_numpy(k).to(DEV)
    vd = torch.from_numpy(v.view(np.int64)).to(DEV)
    _say("sort_by_key keys in place")
    _, vo = hv.sort_by_key(kd, vd, keys_out=kd)
    torch.cuda.synchronize()
    ek, ev = oracle.sort_by_key_p64(k, v)
    assert np.array_equal(kd.cpu().numpy(), ek)
    assert np.array_equal(vo.cpu().numpy().view(np.uint64), ev)


def test_full_size_2pow26():
    n = 1 << 26
    k, v = _inputs(n, seed=26, ties=False)
    kd = torch.from_numpy(k).to(DEV)
    vd = torch.from_numpy(v.view(np.int64)).to(DEV)
    _say("sort_by_key full 2^26")
    ko, vo = hv.sort_by_key(kd, vd)
    torch.cuda.synchronize()
    ek, ev = oracle.sort_by_key_p64(k, v)
    assert np.array_equal(ko.cpu().numpy(), ek)
    assert np.array_equal(vo.cpu().numpy().view(np.uint64), ev)
