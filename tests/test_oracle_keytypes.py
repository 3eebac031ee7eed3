"""Pins of the oracle's uint32, float32, int64, uint64 and float64 sorts:
numpy's sort where its order is the same (integers; finite nonzero floats),
the IEEE 754 totalOrder sequences of special values
(tests/golden/f32_total_order.txt, f64_total_order.txt), and lexicographic
pair order against numpy's lexsort."""
import numpy as np
import pytest

import oracle


def _golden(golden_dir):
    rows = []
    with open(f"{golden_dir}/f32_total_order.txt") as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append(int(line.split()[0], 16))
    return np.array(rows, dtype=np.uint32)


@pytest.mark.parametrize("n", [0, 1, 2, 7, 1000, 100003])
def test_u32_matches_numpy(n):
    rng = np.random.default_rng(n)
    x = rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
    x[: n // 10] = rng.choice(np.array([0, 1, 2**31 - 1, 2**31, 2**32 - 1], dtype=np.uint32),
                             size=n // 10)
    assert np.array_equal(oracle.sort_u32(x), np.sort(x))


@pytest.mark.parametrize("n", [1, 5, 4097, 100003])
def test_f32_finite_nonzero_matches_numpy(n):
    rng = np.random.default_rng(7 + n)
    x = (rng.standard_normal(n) * 10.0 ** rng.integers(-30, 30, size=n)).astype(np.float32)
    x[x == 0] = 1.0
    got = oracle.sort_f32(x)
    assert np.array_equal(got.view(np.uint32), np.sort(x).view(np.uint32))


def test_f32_special_values_follow_total_order(golden_dir):
    want = _golden(golden_dir)
    rng = np.random.default_rng(3)
    for _ in range(20):
        x = rng.permutation(np.repeat(want, 3))
        got = oracle.sort_f32(x.view(np.float32)).view(np.uint32)
        assert np.array_equal(got, np.repeat(want, 3))


def test_f32_signed_zero_and_nan_placement():
    x = np.array([0.0, -0.0, np.nan, -np.nan, -np.inf, np.inf, 1.0, -1.0], dtype=np.float32)
    got = oracle.sort_f32(x).view(np.uint32)
    signs = got >> 31
    # negatives (sign set) first, and within them -NaN, -inf, -1, -0
    assert list(signs) == [1, 1, 1, 1, 0, 0, 0, 0]
    v = got.view(np.float32)
    assert np.isnan(v[0]) and v[1] == -np.inf and v[2] == -1.0 and v[3] == 0 and signs[3] == 1
    assert v[4] == 0 and signs[4] == 0 and v[5] == 1.0 and v[6] == np.inf and np.isnan(v[7])


@pytest.mark.parametrize("kind", ["u32", "f32"])
def test_pairs_lexicographic(kind):
    rng = np.random.default_rng(11)
    n = 20011
    if kind == "u32":
        k = rng.choice(np.array([0, 5, 2**31, 2**32 - 1], dtype=np.uint32), size=n)
        ko, vo = oracle.sort_pairs_u32(k, v := rng.integers(-50, 50, size=n).astype(np.int32))
        order = np.lexsort((v, k))
        assert np.array_equal(ko, k[order]) and np.array_equal(vo, v[order])
    else:
        k = rng.choice(np.array([-3.5, -1.0, 2.0, 1e30, -1e-30], dtype=np.float32), size=n)
        ko, vo = oracle.sort_pairs_f32(k, v := rng.integers(-50, 50, size=n).astype(np.int32))
        order = np.lexsort((v, k))
        assert np.array_equal(ko.view(np.uint32), k[order].view(np.uint32))
        assert np.array_equal(vo, v[order])


def test_pairs_f32_signed_zeros_order_by_sign_first():
    k = np.array([0.0, -0.0, 0.0, -0.0], dtype=np.float32)
    v = np.array([1, 2, -1, -2], dtype=np.int32)
    ko, vo = oracle.sort_pairs_f32(k, v)
    assert list(ko.view(np.uint32) >> 31) == [1, 1, 0, 0]
    assert list(vo) == [-2, 2, -1, 1]


# ------------------------------------------------------------- 64-bit keys

def _golden64(golden_dir):
    rows = []
    with open(f"{golden_dir}/f64_total_order.txt") as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append(int(line.split()[0], 16))
    return np.array(rows, dtype=np.uint64)


@pytest.mark.parametrize("n", [0, 1, 2, 9, 1000, 100003])
def test_i64_matches_numpy(n):
    rng = np.random.default_rng(100 + n)
    x = rng.integers(-2**63, 2**63, size=n, dtype=np.int64)
    # extremes, and keys equal in the high word that differ in the low word
    # (with the low word's top bit set and clear)
    special = np.array([-2**63, 2**63 - 1, -1, 0, 1, 2**31, 2**32 - 1, 2**32,
                        -2**32, -2**32 + 2**31, 5 * 2**32 + 2**31, 5 * 2**32 + 7], dtype=np.int64)
    x[: n // 5] = rng.choice(special, size=n // 5)
    assert np.array_equal(oracle.sort_i64(x), np.sort(x))


@pytest.mark.parametrize("n", [1, 7, 1000, 100003])
def test_u64_matches_numpy(n):
    rng = np.random.default_rng(200 + n)
    x = rng.integers(0, 2**64, size=n, dtype=np.uint64)
    special = np.array([0, 1, 2**63 - 1, 2**63, 2**64 - 1, 2**32, 2**63 + 2**31],
                       dtype=np.uint64)
    x[: n // 5] = rng.choice(special, size=n // 5)
    got = oracle.sort_u64(x)
    assert np.array_equal(got, np.sort(x))
    if n > 5:  # keys with the top bit set go last (a signed compare would put them first)
        assert got[-1] >= np.uint64(2**63) or not (x >= np.uint64(2**63)).any()


def test_i64_and_u64_orders_differ_on_top_bit():
    x = np.array([2**63, 1, 2**63 + 5, 3], dtype=np.uint64)
    assert list(oracle.sort_u64(x)) == [1, 3, 2**63, 2**63 + 5]
    assert list(oracle.sort_i64(x.view(np.int64)).view(np.uint64)) == [2**63, 2**63 + 5, 1, 3]


@pytest.mark.parametrize("n", [1, 5, 4097, 100003])
def test_f64_finite_nonzero_matches_numpy(n):
    rng = np.random.default_rng(300 + n)
    x = rng.standard_normal(n) * 10.0 ** rng.integers(-300, 300, size=n)
    x[x == 0] = 1.0
    got = oracle.sort_f64(x)
    assert np.array_equal(got.view(np.uint64), np.sort(x).view(np.uint64))


def test_f64_special_values_follow_total_order(golden_dir):
    want = _golden64(golden_dir)
    rng = np.random.default_rng(4)
    for _ in range(20):
        x = rng.permutation(np.repeat(want, 3))
        got = oracle.sort_f64(x.view(np.float64)).view(np.uint64)
        assert np.array_equal(got, np.repeat(want, 3))


def test_f64_golden_finite_values_ascend(golden_dir):
    # the fixture's finite entries, read as numbers, ascend (ties only at the
    # two zeros), which checks the fixture itself against arithmetic order
    want = _golden64(golden_dir).view(np.float64)
    fin = want[np.isfinite(want)]
    assert (np.diff(fin) >= 0).all() and (np.diff(fin) == 0).sum() == 1


# ----------------------------------------------- 64-bit payloads (stable)

@pytest.mark.parametrize("n", [0, 1, 2, 13, 1000, 100003])
def test_sort_by_key_p64_matches_numpy_stable_argsort(n):
    rng = np.random.default_rng(400 + n)
    k = rng.integers(-20, 20, size=n).astype(np.int32)          # many ties
    k[: n // 7] = rng.choice(np.array([-2**31, 2**31 - 1], dtype=np.int32), size=n // 7)
    v = rng.integers(0, 2**64, size=n, dtype=np.uint64)
    ko, vo = oracle.sort_by_key_p64(k, v)
    order = np.argsort(k, kind="stable")
    assert np.array_equal(ko, k[order]) and np.array_equal(vo, v[order])


def test_sort_by_key_p64_keeps_input_order_of_equal_keys():
    # payload = input position: within each key the payloads must ascend
    k = np.array([3, 1, 3, 2, 1, 3, 1], dtype=np.int32)
    v = np.arange(7, dtype=np.int64) * 10
    ko, vo = oracle.sort_by_key_p64(k, v)
    assert list(ko) == [1, 1, 1, 2, 3, 3, 3]
    assert list(vo) == [10, 40, 60, 30, 0, 20, 50]
    assert vo.dtype == np.int64


def test_sort_by_key_p64_brute_force_small():
    # every arrangement of a 6-element input with ties: the result is the
    # unique stable order
    import itertools
    base = [(2, 100), (0, 101), (2, 102), (1, 103), (0, 104), (2, 105)]
    for perm in itertools.permutations(range(6)):
        items = [base[i] for i in perm]
        k = np.array([a for a, _ in items], dtype=np.int32)
        v = np.array([b for _, b in items], dtype=np.uint64)
        ko, vo = oracle.sort_by_key_p64(k, v)
        want = sorted(items, key=lambda kv: kv[0])     # Python's sort is stable
        assert list(ko) == [a for a, _ in want] and list(vo) == [b for _, b in want]
