"""GPU parity of the int64, uint64 and float64 key sorts against the oracle,
bit-exact, through the C ABI: random 64-bit patterns, keys that tie in the
high word and differ in the low word (with its top bit set and clear), the
extremes of each order (the largest element equals the padding value), the
IEEE 754 totalOrder special values, ragged sizes, the block-only path
(n <= one tile), two-way and four-way passes, odd and even pass counts,
outputs that are only 8-byte aligned, and in-place calls."""
import numpy as np
import pytest
import torch

import oracle
import paper_2409_03970_amd as hv

pytestmark = pytest.mark.gpu
DEV = "cuda"

KINDS = ["i64", "u64", "f64"]
_ENTRY = {"i64": "hvms_sort_i64", "u64": "hvms_sort_u64", "f64": "hvms_sort_f64"}
_NP = {"i64": np.int64, "u64": np.uint64, "f64": np.float64}


def _say(*a):
    print(*a, flush=True)


def _golden64(golden_dir):
    rows = []
    with open(f"{golden_dir}/f64_total_order.txt") as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append(int(line.split()[0], 16))
    return np.array(rows, dtype=np.uint64)


def _bits(n, kind, seed, golden):
    """Seeded uint64 bit patterns: a quarter uniform over all 2^64 patterns,
    a quarter sharing a few high words (ties decided by the low word), a
    quarter type-specific (normal floats / small integers), a quarter special
    values."""
    rng = np.random.default_rng(seed)
    x = rng.integers(0, 2**64, size=n, dtype=np.uint64)
    q = n // 4
    hi = rng.choice(np.array([0, 1, 0x7fffffff, 0x80000000, 0xffffffff, 0xbff00000],
                             dtype=np.uint64), size=q)
    lo = rng.choice(np.array([0, 1, 0x7fffffff, 0x80000000, 0x80000001, 0xffffffff],
                             dtype=np.uint64), size=q)
    x[q:2 * q] = (hi << np.uint64(32)) | lo
    if kind == "f64":
        x[2 * q:3 * q] = (rng.standard_normal(q) * 1e3).view(np.uint64)
        special = golden
    else:
        x[2 * q:3 * q] = rng.integers(-1000, 1000, size=q).astype(np.int64).view(np.uint64)
        special = np.array([0, 1, 2**63 - 1, 2**63, 2**64 - 1, 2**32 - 1, 2**32, 2**31],
                           dtype=np.uint64)
    x[3 * q:] = rng.choice(special, size=n - 3 * q)
    return rng.permutation(x)


def _dev(bits, kind):
    t = torch.from_numpy(bits.view(np.int64).copy()).to(DEV)
    if kind == "f64":
        return t.view(torch.float64)
    return t.view(torch.uint64) if kind == "u64" else t


def _host_bits(t):
    return t.view(torch.int64).cpu().numpy().view(np.uint64)


def _oracle(bits, kind):
    fn = {"i64": oracle.sort_i64, "u64": oracle.sort_u64, "f64": oracle.sort_f64}[kind]
    return fn(bits.view(_NP[kind])).view(np.uint64)


def _run(kind, x, y, opts):
    ws = hv._workspace(hv.lib().hvms_sort64_workspace_bytes(x.numel(), hv._opts(opts)), x.device)
    getattr(hv, _ENTRY[kind])(x, y, ws, opts=opts)


SHAPES = [
    {},                                                                      # defaults
    {"keys_per_lane": 8, "block_threads": 256, "merge_tile": 2048},
    {"keys_per_lane": 16, "block_threads": 1024, "merge_tile": 4096, "wave_levels": 5},
    {"keys_per_lane": 16, "block_threads": 512, "merge_tile": 8192, "merge_variant": 1},
    {"keys_per_lane": 16, "block_threads": 512, "merge_tile": 4096, "merge_ways": 4},
    {"keys_per_lane": 8, "block_threads": 256, "merge_tile": 2048, "merge_ways": 4},
    {"keys_per_lane": 32, "block_threads": 512, "merge_tile": 4096, "merge_variant": 3},
]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("n", [1, 7, 2048, 8192, 8193, 40000, 300007, (1 << 20) + 3])
@pytest.mark.parametrize("shape", range(len(SHAPES)))
def test_keys64_match_oracle(kind, n, shape, golden_dir):
    opts = SHAPES[shape]
    _say("sort64", kind, n, opts)
    bits = _bits(n, kind, seed=n + 31 * shape, golden=_golden64(golden_dir))
    x = _dev(bits, kind)
    y = torch.empty_like(x)
    _run(kind, x, y, opts)
    torch.cuda.synchronize()
    assert np.array_equal(_host_bits(y), _oracle(bits, kind))
    assert np.array_equal(_host_bits(x), bits)        # input untouched


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("shape", [0, 4])
def test_output_only_8_byte_aligned(kind, shape, golden_dir):
    # an output at an odd element offset is 8- but not 16-byte aligned: the
    # sort must take the two-way passes and the fallback kernel
    n = 300007
    opts = SHAPES[shape]
    _say("sort64 misaligned out", kind, n, opts)
    bits = _bits(n, kind, seed=99 + shape, golden=_golden64(golden_dir))
    x = _dev(bits, kind)
    big = torch.empty(n + 1, dtype=x.dtype, device=DEV)
    y = big[1:]
    assert y.data_ptr() % 16 == 8
    _run(kind, x, y, opts)
    torch.cuda.synchronize()
    assert np.array_equal(_host_bits(y), _oracle(bits, kind))


@pytest.mark.parametrize("kind", KINDS)
def test_in_place(kind, golden_dir):
    n = 1000003
    bits = _bits(n, kind, seed=5, golden=_golden64(golden_dir))
    x = _dev(bits, kind)
    _say("sort64 in place", kind, n)
    hv.sort_keys(x, out=x)
    torch.cuda.synchronize()
    assert np.array_equal(_host_bits(x), _oracle(bits, kind))


def test_f64_special_values_alone(golden_dir):
    want = _golden64(golden_dir)
    bits = np.random.default_rng(2).permutation(np.repeat(want, 1000))
    _say("sort64 f64 specials")
    y = hv.sort_keys(_dev(bits, "f64"))
    torch.cuda.synchronize()
    assert np.array_equal(_host_bits(y), np.repeat(want, 1000))


@pytest.mark.parametrize("kind", KINDS)
def test_full_size_2pow26(kind, golden_dir):
    # tuned shape, 2^26 keys (512 MiB): compared in full with the oracle
    n = 1 << 26
    bits = _bits(n, kind, seed=26, golden=_golden64(golden_dir))
    x = _dev(bits, kind)
    _say("sort64 full 2^26", kind)
    y = hv.sort_keys(x)
    torch.cuda.synchronize()
    assert np.array_equal(_host_bits(y), _oracle(bits, kind))
