"""The C ABI without a GPU: the library loads, exports every declared symbol,
and rejects bad arguments on the host before enqueueing anything."""
import ctypes
import os
import re

import pytest

import paper_2409_03970_amd as hv
import sys
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hvms.h")

pytestmark = pytest.mark.skipif(not os.path.exists(hv.LIB_PATH), reason="libhvms.so not built")

FAKE = ctypes.c_void_p(0x100000)       # never dereferenced: every call below fails validation


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(hvms_[a-z_0-9]+)\s*\(",
                                 text, re.M)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert len(names) >= 30
    L = hv.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(hv._SIGS), set(names) ^ set(hv._SIGS)


def test_python_names_match_c_names():
    for n in _declared():
        if n in ("hvms_status_string", "hvms_last_hip_error") or n.endswith("_workspace_bytes"):
            continue
        assert callable(getattr(hv, n)), n


def test_status_strings():
    L = hv.lib()
    assert L.hvms_status_string(0) == b"ok"
    for s in (-1, -2, -3, -4):
        assert L.hvms_status_string(s) != b"unknown status"


def test_workspace_queries():
    L = hv.lib()
    assert L.hvms_sort_workspace_bytes(0, 0, None) == 0
    assert L.hvms_sort_workspace_bytes(100, 0, None) == 0          # one tile needs none
    a = L.hvms_sort_workspace_bytes(1 << 20, 0, None)
    b = L.hvms_sort_workspace_bytes(1 << 21, 0, None)
    c = L.hvms_sort_workspace_bytes(1 << 20, 1, None)
    assert 4 * (1 << 20) <= a < b and c >= 8 * (1 << 20)
    assert a % 256 == 0 and c % 256 == 0
    assert L.hvms_sort_workspace_bytes(-1, 0, None) == -1
    o = hv.Options(keys_per_lane=7)
    assert L.hvms_sort_workspace_bytes(1000, 0, ctypes.byref(o)) == -4
    assert L.hvms_merge_workspace_bytes(1 << 20, 4096, None) > 0
    # 64-bit keys: two split buffer pairs (16 bytes per key) plus co-ranks
    w64 = L.hvms_sort64_workspace_bytes(1 << 20, None)
    assert w64 >= 16 * (1 << 20) and w64 % 256 == 0
    assert w64 > L.hvms_sort_workspace_bytes(1 << 20, 1, None)
    assert L.hvms_sort64_workspace_bytes(100, None) == 0
    assert L.hvms_sort64_workspace_bytes(-1, None) == -1
    # sort by key: indices (4 bytes per key) plus the key-value workspace
    assert L.hvms_sort_by_key_workspace_bytes(0, None) == 0
    assert L.hvms_sort_by_key_workspace_bytes(100, None) == 512
    assert (L.hvms_sort_by_key_workspace_bytes(1 << 20, None)
            == 4 * (1 << 20) + L.hvms_sort_workspace_bytes(1 << 20, 1, None))


def test_argument_errors_before_any_launch():
    L = hv.lib()
    assert L.hvms_sort_i32(None, None, -1, None, 0, None, None) == -1
    assert L.hvms_sort_i32(None, FAKE, 5, None, 0, None, None) == -1
    assert L.hvms_sort_i32(FAKE, FAKE, 0, None, 0, None, None) == 0          # n = 0: no-op
    # a multi-tile sort without workspace, with a short one, with a misaligned one
    assert L.hvms_sort_i32(FAKE, FAKE, 1 << 20, None, 0, None, None) == -2
    assert L.hvms_sort_i32(FAKE, FAKE, 1 << 20, FAKE, 16, None, None) == -2
    assert L.hvms_sort_i32(FAKE, FAKE, 1 << 20, ctypes.c_void_p(0x100004), 1 << 30, None, None) == -2
    bad = hv.Options(block_threads=300)
    assert L.hvms_sort_i32(FAKE, FAKE, 10, None, 0, None, ctypes.byref(bad)) == -4
    v4 = hv.Options(merge_variant=4)
    assert L.hvms_sort_i32(FAKE, FAKE, 1 << 20, None, 0, None, ctypes.byref(v4)) == -2  # accepted
    assert L.hvms_sort_pairs_i32(FAKE, FAKE, FAKE, FAKE, 10, None, 0, None, ctypes.byref(v4)) == -4
    assert L.hvms_sort_i32(FAKE, FAKE, 10, None, 0, None, ctypes.byref(hv.Options(merge_variant=5))) == -1
    learned_without_model = hv.Options(corank_mode=1)
    assert L.hvms_sort_i32(FAKE, FAKE, 10, None, 0, None, ctypes.byref(learned_without_model)) == -1
    assert L.hvms_sort_pairs_i32(FAKE, None, FAKE, FAKE, 3, None, 0, None, None) == -1
    for f in (L.hvms_sort_u32, L.hvms_sort_f32):
        assert f(None, FAKE, 5, None, 0, None, None) == -1
        assert f(FAKE, FAKE, 0, None, 0, None, None) == 0
        assert f(FAKE, FAKE, 1 << 20, None, 0, None, None) == -2
        assert f(FAKE, FAKE, 10, None, 0, None, ctypes.byref(bad)) == -4
    for f in (L.hvms_sort_pairs_u32, L.hvms_sort_pairs_f32):
        assert f(FAKE, None, FAKE, FAKE, 3, None, 0, None, None) == -1
        assert f(FAKE, FAKE, FAKE, FAKE, 1 << 20, FAKE, 16, None, None) == -2
    for f in (L.hvms_sort_i64, L.hvms_sort_u64, L.hvms_sort_f64):
        assert f(None, FAKE, 5, None, 0, None, None) == -1
        assert f(FAKE, FAKE, 0, None, 0, None, None) == 0
        assert f(FAKE, ctypes.c_void_p(0x100004), 5, None, 0, None, None) == -1   # not 8-aligned
        assert f(FAKE, FAKE, 1 << 20, None, 0, None, None) == -2
        assert f(FAKE, FAKE, 1 << 20, FAKE, 16, None, None) == -2
        assert f(FAKE, FAKE, 10, None, 0, None, ctypes.byref(bad)) == -4
        assert f(FAKE, FAKE, 10, None, 0, None, ctypes.byref(v4)) == -4       # keys-only merger
    f = L.hvms_sort_by_key_i32_p64
    V1, V2 = ctypes.c_void_p(0x200000), ctypes.c_void_p(0x300000)
    assert f(FAKE, None, FAKE, V2, 5, None, 0, None, None) == -1
    assert f(FAKE, V1, FAKE, V2, 0, None, 0, None, None) == 0
    assert f(FAKE, V1, FAKE, V2, -1, None, 0, None, None) == -1
    assert f(FAKE, V1, FAKE, V2, 2**31, None, 0, None, None) == -1         # int32 indices
    assert f(FAKE, V1, FAKE, ctypes.c_void_p(0x300004), 5, None, 0, None, None) == -1
    assert f(FAKE, V1, FAKE, V1, 5, None, 0, None, None) == -1             # payloads alias
    assert f(FAKE, V1, FAKE, ctypes.c_void_p(0x200000 + 8 * 4), 5, None, 0, None, None) == -1
    assert f(FAKE, V1, FAKE, V2, 5, None, 0, None, None) == -2             # needs workspace
    assert f(FAKE, V1, FAKE, V2, 10, None, 0, None, ctypes.byref(v4)) == -4
    assert L.hvms_sort_runs_i32(FAKE, FAKE, 100, 2, None, None) == -1        # run below R
    assert L.hvms_sort_runs_i32(FAKE, FAKE, 100, 20, None, None) == -1       # run above tile
    assert L.hvms_merge_pass_i32(FAKE, FAKE, 100, 3000, None, 0, None, None) == -1  # not 2^k
    assert L.hvms_corank_i32(None, 5, FAKE, 5, FAKE, 1, FAKE, None, None) == -1
    assert L.hvms_corank_i32(FAKE, 5, FAKE, 5, FAKE, 0, FAKE, None, None) == 0


def test_every_option_set_of_the_gpu_tests_is_accepted():
    import test_gpu_sort as g
    L = hv.lib()
    sets = list(g.TUNINGS) + [dict(keys_per_lane=R, block_threads=NT)
                              for R in (8, 16, 32) for NT in (256, 512, 1024)
                              if not (R == 32 and NT == 1024)]
    for o in sets:
        assert L.hvms_sort_workspace_bytes(1 << 20, 0, hv._opts(o)) >= 0, o
        assert L.hvms_sort_runs_i32(FAKE, FAKE, 0, 4 if o["keys_per_lane"] <= 16 else 5,
                                    None, hv._opts(o)) == 0, o


def test_segmented_workspace_and_errors():
    L = hv.lib()
    assert L.hvms_segmented_workspace_bytes(0, 0, 0, 0, None) == 0
    a = L.hvms_segmented_workspace_bytes(1 << 20, 100, 65536, 0, None)
    b = L.hvms_segmented_workspace_bytes(1 << 20, 100, 65536, 1, None)
    assert a >= 4 * (1 << 20) and b >= a + 4 * (1 << 20) and a % 256 == 0
    assert L.hvms_segmented_workspace_bytes(-1, 1, 1, 0, None) == -1
    # nseg == 0 and n_total == 0 are no-ops
    assert L.hvms_segmented_sort_i32(None, None, None, 0, 0, 0, None, 0, None, None) == 0
    # null offsets with segments, missing workspace, misaligned output
    assert L.hvms_segmented_sort_i32(FAKE, FAKE, None, 3, 100, 50, None, 0, None, None) == -1
    assert L.hvms_segmented_sort_i32(FAKE, FAKE, FAKE, 3, 100, 50, None, 0, None, None) == -2
    assert L.hvms_segmented_sort_i32(FAKE, ctypes.c_void_p(0x100004), FAKE, 3, 100, 50, FAKE,
                                     1 << 30, None, None) == -1
    assert L.hvms_segmented_sort_pairs_i32(FAKE, None, FAKE, FAKE, FAKE, 3, 100, 50, FAKE,
                                           1 << 30, None, None) == -1


def test_segmented_status_and_unknown_bound():
    L = hv.lib()
    # a negative max_seg means "no bound known": accepted, same workspace
    assert L.hvms_segmented_workspace_bytes(1 << 20, 100, -1, 0, None) == \
        L.hvms_segmented_workspace_bytes(1 << 20, 100, 65536, 0, None)
    # the status query rejects null and misaligned pointers on the host
    assert L.hvms_segmented_status(None, FAKE, None) == -1
    assert L.hvms_segmented_status(FAKE, None, None) == -1
    assert L.hvms_segmented_status(ctypes.c_void_p(0x100010), FAKE, None) == -1


def test_segmented_conveniences_refuse_invalid_offsets():
    import torch
    ok = hv._host_offsets(torch.tensor([0, 3, 3, 10], dtype=torch.int64), 10)
    assert ok.tolist() == [0, 3, 3, 10]
    for bad, n in (([0, 5, 4, 10], 10), ([-1, 5], 10), ([0, 11], 10)):
        with pytest.raises(ValueError):
            hv._host_offsets(torch.tensor(bad, dtype=torch.int64), n)
    with pytest.raises(ValueError):
        hv._host_offsets(torch.tensor([0, 5], dtype=torch.int32), 10)


def test_sort_noalloc_argument_errors():
    # host-side checks of the allocation-free sort, before any GPU call
    L = hv.lib()
    assert L.hvms_sort_i32_noalloc(None, None, 0, None, None) == 0
    assert L.hvms_sort_i32_noalloc(FAKE, FAKE, -1, None, None) == -1
    assert L.hvms_sort_i32_noalloc(None, FAKE, 5, None, None) == -1
    assert L.hvms_sort_i32_noalloc(FAKE, FAKE, hv.SORT_NOALLOC_MAX_KEYS + 1, None, None) == -5
    assert L.hvms_status_string(-5).decode().startswith("input larger")
    assert hv.SORT_NOALLOC_MAX_KEYS == 1 << 22
    text = open(HEADER).read()
    assert "#define HVMS_SORT_NOALLOC_MAX_KEYS (1 << 22)" in text


def test_cdf_param_count_matches_header_and_oracle():
    from oracle import mlp
    assert hv.hvms_cdf_param_count() == hv.CDF_PARAMS == mlp.N_PARAMS == 1153


def test_cdf_argument_errors():
    L = hv.lib()
    assert L.hvms_cdf_forward(FAKE, FAKE, FAKE, 0, None) == 0
    assert L.hvms_cdf_forward(None, FAKE, FAKE, 5, None) == -1
    assert L.hvms_cdf_workspace_bytes(4096) > 4096 * 4 * 132
    assert L.hvms_cdf_backward(FAKE, FAKE, FAKE, FAKE, FAKE, 0, FAKE, 1 << 30, None) == -1
    assert L.hvms_cdf_backward(FAKE, FAKE, FAKE, FAKE, FAKE, 100, None, 0, None) == -2
    assert L.hvms_cdf_adam_step(FAKE, FAKE, FAKE, FAKE, 0, 1e-3, 0.9, 0.999, 1e-8, None) == -1
    assert L.hvms_cdf_adam_step(FAKE, FAKE, FAKE, FAKE, 1, 1e-3, 1.0, 0.999, 1e-8, None) == -1
    assert L.hvms_cdf_train_workspace_bytes(0) == -1
    assert L.hvms_cdf_train(FAKE, FAKE, FAKE, FAKE, 0, 10, 1, 1e-3, 0, FAKE, 1 << 30, None) == -1
    assert L.hvms_cdf_sample_i32(FAKE, 0, 5, 1, FAKE, None) == -1
    assert L.hvms_cdf_sample_i32(FAKE, 10, 0, 1, FAKE, None) == 0


def test_stats_and_model_buffers_are_checked_before_any_call():
    import torch
    for bad in (torch.zeros(8, dtype=torch.int64), torch.zeros(136, dtype=torch.int32)):
        with pytest.raises(ValueError):
            hv._opts({"stats": bad})
    hv._opts({"stats": torch.zeros(hv.STATS_WORDS, dtype=torch.int64)})
    with pytest.raises(ValueError):
        hv._opts({"cdf_params": torch.zeros(100, dtype=torch.float32)})
    # the header's stats layout and the binding agree
    text = open(HEADER).read()
    assert re.search(r"HVMS_STATS_WORDS\s*=\s*%d" % hv.STATS_WORDS, text)
    assert re.search(r"HVMS_STAT_PROBE_HIST\s*=\s*8\b", text)
    assert re.search(r"HVMS_STAT_ERR_HIST\s*=\s*72\b", text)


def test_corank_stats_summary_percentiles():
    w = [0] * hv.STATS_WORDS
    w[0], w[1] = 100, 1000
    w[8 + 9], w[8 + 10], w[8 + 20] = 90, 9, 1          # probes: p99 -> 10
    w[2], w[3], w[4], w[5] = 5, 700, 300, 100
    w[72 + 0], w[72 + 3], w[72 + 9] = 50, 49, 1         # |err| bit lengths
    r = hv.corank_stats(w)
    assert r["probes_mean"] == 10.0 and r["probes_p99"] == 10
    assert r["abs_err_p99_at_most"] == 7 and r["max_err"] == 300
    assert r["fallback_rate"] == 0.05 and r["abs_err_mean"] == 7.0
    w[8 + 20] = 5                                       # 5 % at 20 probes: p99 -> 20
    assert hv.corank_stats(w)["probes_p99"] == 20


def test_grouped_sort_checks_a_caller_workspace_first():
    import torch
    offs = torch.tensor([0, 5000, 9000, 20000], dtype=torch.int64)
    need = hv.grouped_workspace_bytes(offs, max_group_keys=10000)
    assert need > 0
    k = torch.zeros(20000, dtype=torch.int32)
    with pytest.raises(ValueError):
        hv.segmented_sort_pairs_grouped(k, k.clone(), offs, max_group_keys=10000,
                                        ws=torch.empty(need - 1, dtype=torch.uint8))
