"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here retypes the oracle's own code: each check reaches the expected
value another way (a library routine, a counting construction, brute force
over all small inputs, a definition written as inequalities, or a property).
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_2409_03970_amd import inputs


def _np(t):
    return t.numpy()


# --------------------------------------------------------------- sort

@pytest.mark.parametrize("n", [0, 1, 2, 3, 17, 1000, 65537])
@pytest.mark.parametrize("dist", list(inputs.DISTRIBUTIONS) + ["mixture"])
def test_sort_equals_library_sort(n, dist):
    a = _np(inputs.keys(n, dist, seed=n))
    assert np.array_equal(oracle.sort(a), np.sort(a, kind="stable"))


@pytest.mark.parametrize("pattern", ["equal", "two_values", "extremes", "organ_pipe",
                                     "sawtooth", "negatives"])
@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 4097])
def test_sort_adversarial(pattern, n):
    a = _np(inputs.adversarial_keys(n, pattern, seed=3))
    assert np.array_equal(oracle.sort(a), np.sort(a))


@pytest.mark.parametrize("n", range(1, 9))
def test_sort_all_permutations(n):
    # every permutation of n distinct keys must come out as 0..n-1
    want = np.arange(n, dtype=np.int32)
    for p in itertools.permutations(range(n)):
        assert np.array_equal(oracle.sort(np.array(p, dtype=np.int32)), want)


@pytest.mark.parametrize("n", range(1, 8))
def test_sort_all_value_patterns_counting(n):
    # all n^n arrays over {0..n-1}, expected output by counting (no comparisons)
    for vals in itertools.product(range(n), repeat=n):
        a = np.array(vals, dtype=np.int32)
        want = np.repeat(np.arange(n, dtype=np.int32), np.bincount(a, minlength=n))
        assert np.array_equal(oracle.sort(a), want)


def test_sort_large_invariants():
    a = _np(inputs.keys(1 << 20, "uniform", seed=1))
    s = oracle.sort(a)
    assert np.all(s[1:] >= s[:-1])
    assert oracle.multiset_hash(s) == oracle.multiset_hash(a)


# --------------------------------------------------------------- pairs

@pytest.mark.parametrize("n", [0, 1, 5, 1000, 40000])
@pytest.mark.parametrize("dist", ["uniform", "distinct16", "zipf", "sorted"])
def test_pairs_equal_lexsort(n, dist):
    k = _np(inputs.keys(n, dist, seed=5))
    rng = np.random.default_rng(n)
    v = rng.integers(-50, 50, size=n, dtype=np.int32)   # ties in the payload too
    ok, ov = oracle.sort_pairs(k, v)
    order = np.lexsort((v, k))
    assert np.array_equal(ok, k[order]) and np.array_equal(ov, v[order])


def test_pairs_index_payload_is_stable_sort():
    k = _np(inputs.keys(10000, "distinct16", seed=9))
    v = np.arange(k.size, dtype=np.int32)
    ok, ov = oracle.sort_pairs(k, v)
    order = np.argsort(k, kind="stable")
    assert np.array_equal(ov, order) and np.array_equal(ok, k[order])


def test_pairs_all_permutations_small():
    for n in range(1, 7):
        base = [(x // 2, x % 3) for x in range(n)]
        want = sorted(base)
        for p in itertools.permutations(base):
            k = np.array([a for a, _ in p], dtype=np.int32)
            v = np.array([b for _, b in p], dtype=np.int32)
            ok, ov = oracle.sort_pairs(k, v)
            assert list(zip(ok.tolist(), ov.tolist())) == want


# ----------------------------------------------------------- segmented

def test_segmented_each_segment_sorted_and_rest_untouched():
    sizes = inputs.log_uniform_sizes(300, 1, 2000, seed=2)
    sizes[5] = 0
    sizes[17] = 0
    offs = inputs.offsets_from_sizes(sizes).numpy()
    total = int(offs[-1])
    k = _np(inputs.keys(total + 50, "uniform", seed=4))
    offs_inner = offs + 25          # 25 keys before and after are not in any segment
    out = oracle.segmented_sort(k, offs_inner)
    assert np.array_equal(out[:25], k[:25]) and np.array_equal(out[-25:], k[-25:])
    for s in range(sizes.numel()):
        a, b = offs_inner[s], offs_inner[s + 1]
        assert np.array_equal(out[a:b], np.sort(k[a:b]))


def test_segmented_pairs():
    sizes = inputs.log_uniform_sizes(100, 1, 500, seed=6)
    offs = inputs.offsets_from_sizes(sizes).numpy()
    k = _np(inputs.keys(int(offs[-1]), "distinct16", seed=6))
    v = np.concatenate([np.arange(s, dtype=np.int32) for s in sizes.tolist()])
    ok, ov = oracle.segmented_sort_pairs(k, v, offs)
    for s in range(sizes.numel()):
        a, b = offs[s], offs[s + 1]
        order = np.lexsort((v[a:b], k[a:b]))
        assert np.array_equal(ok[a:b], k[a:b][order]) and np.array_equal(ov[a:b], v[a:b][order])


def test_segmented_rejects_decreasing_offsets():
    with pytest.raises(ValueError):
        oracle.segmented_sort(np.zeros(10, np.int32), np.array([0, 5, 3, 10]))


# ------------------------------------------------------ merge / co-rank

def _tagged_first_d(A, B, d):
    # the A-first merge is Python's stable sort of (value, tag) with A tagged 0
    merged = sorted([(x, 0) for x in A] + [(x, 1) for x in B])
    return sum(1 for _, t in merged[:d] if t == 0)


def _corank_by_inequalities(A, B, d):
    # the unique i with A[i-1] <= B[j] and B[j-1] < A[i], j = d - i
    m, n = len(A), len(B)
    sols = []
    for i in range(max(0, d - n), min(d, m) + 1):
        j = d - i
        c1 = i == 0 or j == n or A[i - 1] <= B[j]
        c2 = j == 0 or i == m or B[j - 1] < A[i]
        if c1 and c2:
            sols.append(i)
    assert len(sols) == 1
    return sols[0]


@pytest.mark.parametrize("seed", range(40))
def test_corank_matches_definitions(seed):
    rng = np.random.default_rng(seed)
    m, n = int(rng.integers(0, 30)), int(rng.integers(0, 30))
    hi = int(rng.integers(1, 8))                 # few distinct values: many ties
    A = np.sort(rng.integers(0, hi, m)).astype(np.int32)
    B = np.sort(rng.integers(0, hi, n)).astype(np.int32)
    for d in range(m + n + 1):
        i = oracle.corank(A, B, d)
        assert i == _corank_by_inequalities(A.tolist(), B.tolist(), d)
        assert i == _tagged_first_d(A.tolist(), B.tolist(), d)
    assert oracle.corank(A, B, -1) == -1 and oracle.corank(A, B, m + n + 1) == -1


def test_merge_equals_sorted_concatenation():
    rng = np.random.default_rng(1)
    for _ in range(50):
        A = np.sort(rng.integers(-5, 5, rng.integers(0, 60))).astype(np.int32)
        B = np.sort(rng.integers(-5, 5, rng.integers(0, 60))).astype(np.int32)
        assert np.array_equal(oracle.merge(A, B), np.sort(np.concatenate([A, B])))


def test_corank_pairs_lexicographic():
    rng = np.random.default_rng(2)
    for _ in range(30):
        m, n = int(rng.integers(0, 20)), int(rng.integers(0, 20))
        Ak, Av = rng.integers(0, 3, m), rng.integers(0, 3, m)
        Bk, Bv = rng.integers(0, 3, n), rng.integers(0, 3, n)
        oa, ob = np.lexsort((Av, Ak)), np.lexsort((Bv, Bk))
        A = list(zip(Ak[oa].tolist(), Av[oa].tolist()))
        B = list(zip(Bk[ob].tolist(), Bv[ob].tolist()))
        for d in range(m + n + 1):
            got = oracle.corank_pairs(Ak[oa], Av[oa], Bk[ob], Bv[ob], d)
            assert got == _corank_by_inequalities(A, B, d)


# -------------------------------------------------------------- checks

def test_count_matches_numpy():
    a = _np(inputs.keys(5000, "distinct16", seed=1))
    for x in np.unique(a)[:5].tolist() + [-1, 2**31 - 1]:
        assert oracle.count(a, x) == (int(np.sum(a < x)), int(np.sum(a <= x)))


def test_multiset_hash_properties():
    a = _np(inputs.keys(10000, "uniform", seed=2))
    rng = np.random.default_rng(0)
    assert oracle.multiset_hash(rng.permutation(a)) == oracle.multiset_hash(a)
    b = a.copy()
    b[123] ^= 1
    assert oracle.multiset_hash(b) != oracle.multiset_hash(a)
    k, v = a.copy(), np.arange(a.size, dtype=np.int32)
    w = v.copy()
    w[[0, 1]] = w[[1, 0]]                        # payload moved to another key
    if k[0] != k[1]:
        assert oracle.multiset_hash_pairs(k, v) != oracle.multiset_hash_pairs(k, w)


# ------------------------------------------------------ network checks

def _table1(golden_dir):
    rows = {}
    with open(f"{golden_dir}/table1_comparators.txt") as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                n, bit, oe, lo, hi = map(int, line.split())
                rows[n] = (bit, oe, lo, hi)
    return rows


def _bitonic_by_definition(n):
    # textbook recursive bitonic sorter: sort halves in opposite directions,
    # then bitonic-merge; a descending comparator is (b, a)
    def merge(lo, cnt, up):
        out = []
        if cnt > 1:
            k = cnt // 2
            for i in range(lo, lo + k):
                out.append((i, i + k) if up else (i + k, i))
            out += merge(lo, k, up) + merge(lo + k, k, up)
        return out

    def srt(lo, cnt, up):
        if cnt <= 1:
            return []
        k = cnt // 2
        return srt(lo, k, True) + srt(lo + k, k, False) + merge(lo, cnt, up)
    return srt(0, n, True)


def test_checker_accepts_textbook_networks_with_table1_counts(golden_dir):
    rows = _table1(golden_dir)
    for n in (4, 8, 16):
        net = _bitonic_by_definition(n)
        assert len(net) == rows[n][0]
        assert oracle.network_failures01(net, n) == 0


def test_checker_rejects_broken_networks():
    net = _bitonic_by_definition(16)
    for drop in (0, 17, 40, len(net) - 1):
        broken = net[:drop] + net[drop + 1:]
        assert oracle.network_failures01(broken, 16) > 0
    # a reversed comparator breaks it too
    rev = list(net)
    rev[30] = (rev[30][1], rev[30][0])
    assert oracle.network_failures01(rev, 16) > 0
    # the empty network fails on exactly the unsorted inputs: 2^n - (n + 1)
    for n in (3, 5, 7):
        assert oracle.network_failures01([], n) == 2**n - (n + 1)


def test_merging_checker():
    p = q = 8
    # plain odd-even transposition over 16 wires merges anything given enough rounds
    rounds = [(i, i + 1) for r in range(16) for i in range(r % 2, 15, 2)]
    assert oracle.merging_network_failures01(rounds, p, q) == 0
    # a single pass of adjacent comparators does not merge two runs of 8
    assert oracle.merging_network_failures01([(i, i + 1) for i in range(15)], p, q) > 0
    # with no comparators exactly the inputs with a 1 in the first run before
    # a 0 in the second run fail: z1 < p and z2 > 0 -> p * q
    assert oracle.merging_network_failures01([], p, q) == p * q


def test_32_wire_checker_on_small_wire_count_is_consistent():
    # wires above the network's width are free: a 4-wire sorter on 6 wires fails
    net = _bitonic_by_definition(4)
    assert oracle.network_failures01(net, 4) == 0
    assert oracle.network_failures01(net, 6) > 0


def test_sort_in_parts_equals_oracle_sort():
    # the identity the full-size GPU tests use to run the oracle on several
    # host threads: sorting pieces and merging them gives oracle.sort's array
    import oracle_parts
    rng = np.random.default_rng(11)
    for n, parts in ((1 << 20, 8), (100003, 5), (17, 4), (1, 3), (0, 2)):
        for x in (rng.integers(-2**31, 2**31, n, dtype=np.int64).astype(np.int32),
                  rng.integers(0, 7, n).astype(np.int32)):
            assert np.array_equal(oracle_parts.sort_in_parts(x, parts), oracle.sort(x))


def test_std_sort_context_routine_sorts():
    # the library sort timed beside the oracle in the CPU baseline (context)
    rng = np.random.default_rng(12)
    for x in (rng.integers(-2**31, 2**31, 65537, dtype=np.int64).astype(np.int32),
              np.zeros(0, np.int32), np.full(9, 3, np.int32)):
        assert np.array_equal(oracle.std_sort(x), np.sort(x))
