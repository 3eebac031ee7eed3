"""The comparator networks the kernels use, checked with the oracle's
exhaustive 0-1 checker (Table 1 counts; the 0-1 principle)."""
import re

import pytest

import oracle
from paper_2409_03970_amd import netgen


def _table1(golden_dir):
    rows = {}
    with open(f"{golden_dir}/table1_comparators.txt") as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                n, bit, oe, lo, hi = map(int, line.split())
                rows[n] = (bit, oe, lo, hi)
    return rows


@pytest.mark.parametrize("n", [4, 8, 16, 32])
def test_generated_counts_match_table1(golden_dir, n):
    bit, oe, lo, hi = _table1(golden_dir)[n]
    assert len(netgen.bitonic(n)) == bit
    assert len(netgen.oddeven(n)) == oe


@pytest.mark.parametrize("n", [4, 8, 16])
def test_generated_symmetric_networks_sort(n):
    assert oracle.network_failures01(netgen.bitonic(n), n) == 0
    assert oracle.network_failures01(netgen.oddeven(n), n) == 0


def test_column_network_16_is_within_table1_asymmetric_range(golden_dir):
    bit, oe, lo, hi = _table1(golden_dir)[16]
    net = netgen.column_network(16)
    assert lo <= len(net) <= hi
    assert len(net) < oe < bit
    assert oracle.network_failures01(net, 16) == 0
    # depth: ten layers, each touching every wire at most once
    for layer in netgen.BEST16:
        wires = [w for c in layer for w in c]
        assert len(wires) == len(set(wires))
    assert len(netgen.BEST16) == 10


@pytest.mark.parametrize("R", [4, 8, 16])
def test_column_networks_sort_all_01_inputs(R):
    assert oracle.network_failures01(netgen.column_network(R), R) == 0


def test_column_network_32_sorts_all_01_inputs():
    # 2^32 inputs, bit-sliced: a few seconds
    net = netgen.column_network(32)
    assert len(net) == 191
    assert oracle.network_failures01(net, 32) == 0


@pytest.mark.parametrize("R", [4, 8, 16])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_wave_merge_levels_merge_all_sorted_halves(R, k):
    # the wave merge run for k levels (the levels below k re-sort each half,
    # the upper one descending) must merge every pair of sorted halves of
    # R * 2^k keys: the schedule the kernels run, as a comparator network
    comps = netgen.wave_merge(R, k)
    s = R << k
    # the levels act on disjoint runs of s keys; check the first and the last
    for base in (0, R * 64 - s):
        inside = [(a, b) for a, b in comps if base <= min(a, b) < base + s]
        assert all(base <= max(a, b) < base + s for a, b in inside)
        sub = [(a - base, b - base) for a, b in inside]
        assert oracle.merging_network_failures01(sub, s // 2, s // 2) == 0


@pytest.mark.parametrize("R", [8, 16])
def test_wave_merge_level_directions(R):
    # below the last level, blocks with lane bit k set come out descending:
    # the all-ascending merge of such a block must fail (the directions matter)
    comps = netgen.wave_merge(R, 2)
    flipped = [(min(a, b), max(a, b)) for a, b in comps]
    s = R << 2
    sub = [(a, b) for a, b in flipped if b < s]
    assert oracle.merging_network_failures01(sub, s // 2, s // 2) > 0


def test_lane_partners_cover_the_wave():
    # logical lane bits map one to one onto the six physical lane bits
    assert sorted(netgen.lane_partner(j) for j in range(6)) == [1, 2, 4, 8, 16, 32]


def _table(text, name):
    m = re.search(rf"{name}\[\d+\] = \{{([^}}]*)\}}", text)
    vals = [int(x) for x in m.group(1).replace(" ", "").split(",")]
    return list(zip(vals[::2], vals[1::2]))


def test_header_matches_generator():
    text = open(netgen.header_path()).read()
    assert text == netgen.render_header()
    for R in (4, 8, 16, 32):
        assert _table(text, f"HVMS_NET{R}") == netgen.column_network(R)


def test_header_ablation_networks(golden_dir):
    text = open(netgen.header_path()).read()
    bit, oe, lo, hi = _table1(golden_dir)[16]
    oe16, bt16 = _table(text, "HVMS_NET16_OE"), _table(text, "HVMS_NET16_BT")
    assert len(oe16) == oe and len(bt16) == bit
    assert oracle.network_failures01(oe16, 16) == 0
    assert oracle.network_failures01(bt16, 16) == 0
