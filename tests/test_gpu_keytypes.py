"""GPU parity of the uint32 and float32 key sorts (and their pair forms)
against the oracle, bit-exact, through the C ABI: random bit patterns (most
of them NaNs with random payloads), the IEEE 754 totalOrder special values,
ragged sizes, every tile shape class, the block-only path (n <= one tile),
two-way and four-way final passes, and in-place calls."""
import numpy as np
import pytest
import torch

import oracle
import paper_2409_03970_amd as hv

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _say(*a):
    print(*a, flush=True)


def _golden(golden_dir):
    rows = []
    with open(f"{golden_dir}/f32_total_order.txt") as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append(int(line.split()[0], 16))
    return np.array(rows, dtype=np.uint32)


def _bits(n, kind, seed, golden):
    """Seeded uint32 bit patterns: a third uniform over all 2^32 patterns, a
    third clustered (many ties), a third the special values."""
    rng = np.random.default_rng(seed)
    x = rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
    third = n // 3
    if kind == "f32":
        x[:third] = (rng.standard_normal(third) * 1e3).astype(np.float32).view(np.uint32)
    else:
        x[:third] = rng.integers(2**31 - 50, 2**31 + 50, size=third).astype(np.uint32)
    x[third:2 * third] = rng.choice(golden, size=third)
    return rng.permutation(x)


def _dev(bits, kind):
    t = torch.from_numpy(bits.view(np.int32).copy()).to(DEV)
    return t.view(torch.float32) if kind == "f32" else t.view(torch.uint32)


def _host_bits(t):
    return t.view(torch.int32).cpu().numpy().view(np.uint32)


def _oracle_keys(bits, kind):
    return (oracle.sort_f32(bits.view(np.float32)).view(np.uint32) if kind == "f32"
            else oracle.sort_u32(bits))


SHAPES = [
    {},                                                             # defaults
    {"keys_per_lane": 8, "block_threads": 256, "merge_tile": 4096},
    {"keys_per_lane": 32, "block_threads": 512, "merge_tile": 8192},
    {"keys_per_lane": 16, "block_threads": 1024, "merge_tile": 8192, "merge_variant": 1},
    {"keys_per_lane": 32, "block_threads": 512, "merge_tile": 8192, "merge_ways": 4},
]


@pytest.mark.parametrize("kind", ["u32", "f32"])
@pytest.mark.parametrize("n", [1, 7, 4096, 16384, 16385, 300007, (1 << 20) + 3])
@pytest.mark.parametrize("shape", range(len(SHAPES)))
def test_keys_match_oracle(kind, n, shape, golden_dir):
    opts = SHAPES[shape]
    _say("keytype sort", kind, n, opts)
    bits = _bits(n, kind, seed=n + 17 * shape, golden=_golden(golden_dir))
    x = _dev(bits, kind)
    y = torch.empty_like(x)
    ws = hv._workspace(hv.lib().hvms_sort_workspace_bytes(n, 0, hv._opts(opts)), x.device)
    (hv.hvms_sort_f32 if kind == "f32" else hv.hvms_sort_u32)(x, y, ws, opts=opts)
    torch.cuda.synchronize()
    assert np.array_equal(_host_bits(y), _oracle_keys(bits, kind))
    assert np.array_equal(_host_bits(x), bits)        # input untouched


@pytest.mark.parametrize("kind", ["u32", "f32"])
def test_in_place(kind, golden_dir):
    n = 1000003
    bits = _bits(n, kind, seed=5, golden=_golden(golden_dir))
    x = _dev(bits, kind)
    hv.sort_keys(x, out=x)
    torch.cuda.synchronize()
    assert np.array_equal(_host_bits(x), _oracle_keys(bits, kind))


@pytest.mark.parametrize("kind", ["u32", "f32"])
@pytest.mark.parametrize("n", [5, 3000, 70001, (1 << 19) + 1])
@pytest.mark.parametrize("shape", [0, 1, 4])
def test_pairs_match_oracle(kind, n, shape, golden_dir):
    opts = dict(SHAPES[shape])
    if opts.get("merge_ways") == 4:
        opts["merge_tile"] = 4096
    if opts.get("keys_per_lane") == 32:
        opts["keys_per_lane"] = 16
    _say("keytype pairs", kind, n, opts)
    rng = np.random.default_rng(n)
    bits = _bits(n, kind, seed=n + 1, golden=_golden(golden_dir))
    vals = rng.integers(-1000, 1000, size=n).astype(np.int32)
    k = _dev(bits, kind)
    v = torch.from_numpy(vals).to(DEV)
    ko, vo = torch.empty_like(k), torch.empty_like(v)
    ws = hv._workspace(hv.lib().hvms_sort_workspace_bytes(n, 1, hv._opts(opts)), k.device)
    fn = hv.hvms_sort_pairs_f32 if kind == "f32" else hv.hvms_sort_pairs_u32
    fn(k, v, ko, vo, ws, opts=opts)
    torch.cuda.synchronize()
    if kind == "f32":
        ek, ev = oracle.sort_pairs_f32(bits.view(np.float32), vals)
        ek = ek.view(np.uint32)
    else:
        ek, ev = oracle.sort_pairs_u32(bits, vals)
    assert np.array_equal(_host_bits(ko), ek)
    assert np.array_equal(vo.cpu().numpy(), ev)


def test_f32_special_values_alone(golden_dir):
    want = _golden(golden_dir)
    bits = np.random.default_rng(2).permutation(np.repeat(want, 1000))
    y = hv.sort_keys(_dev(bits, "f32"))
    torch.cuda.synchronize()
    assert np.array_equal(_host_bits(y), np.repeat(want, 1000))


def test_int32_path_unchanged_by_key_maps():
    # the int32 entry point and sort_keys on int32 agree with the oracle
    x = torch.randint(-2**31, 2**31 - 1, (1 << 20,), dtype=torch.int32, device=DEV)
    y = hv.sort_keys(x)
    torch.cuda.synchronize()
    assert np.array_equal(y.cpu().numpy(), oracle.sort(x.cpu().numpy()))


@pytest.mark.parametrize("kind", ["u32", "f32"])
def test_full_size_2pow26(kind, golden_dir):
    n = 1 << 26
    _say("keytype full size", kind, n)
    bits = _bits(n, kind, seed=26, golden=_golden(golden_dir))
    y = hv.sort_keys(_dev(bits, kind))
    torch.cuda.synchronize()
    assert np.array_equal(_host_bits(y), _oracle_keys(bits, kind))
