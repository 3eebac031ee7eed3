"""CPU oracle for the hybrid vectorized merge sort.  TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It never imports the product package and shares no code
with it.  The C part (oracle.c) is built with gcc into liboracle.so beside
this file; `build()` compiles it and `lib()` builds it on first use if it is
missing.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)


_CTX_SRC = os.path.join(_HERE, "std_sort.cpp")
_CTX_SO = os.path.join(_HERE, "libstdsort.so")
_ctx = None


def build():
    """Compile oracle.c with gcc (always, so edits are picked up), and the
    std::sort context routine with g++."""
    tmp = _SO + ".tmp"
    subprocess.run(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
                    _SRC, "-o", tmp], check=True)
    os.replace(tmp, _SO)
    tmp = _CTX_SO + ".tmp"
    subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-fPIC", "-shared",
                    _CTX_SRC, "-o", tmp], check=True)
    os.replace(tmp, _CTX_SO)


def std_sort(keys):
    """Context only: a copy of int32 keys sorted by the C++ library's
    std::sort (single thread).  Not an oracle: used to time the oracle against
    a common library sort on the same host."""
    global _ctx
    if _ctx is None:
        if not os.path.exists(_CTX_SO) or os.path.getmtime(_CTX_SO) < os.path.getmtime(_CTX_SRC):
            build()
        L = ctypes.CDLL(_CTX_SO)
        L.context_std_sort_i32.argtypes = [_i32p, ctypes.c_int64]
        L.context_std_sort_i32.restype = None
        _ctx = L
    a, p = _i32(np.array(keys, dtype=np.int32, copy=True))
    _ctx.context_std_sort_i32(p, a.size)
    return a


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_SO)
        L.oracle_sort_i32.argtypes = [_i32p, ctypes.c_int64]
        L.oracle_sort_pairs_i32.argtypes = [_i32p, _i32p, ctypes.c_int64]
        _u32p = ctypes.POINTER(ctypes.c_uint32)
        for name in ("oracle_sort_u32", "oracle_sort_f32"):
            getattr(L, name).argtypes = [_u32p, ctypes.c_int64]
        _u64p = ctypes.POINTER(ctypes.c_uint64)
        for name in ("oracle_sort_i64", "oracle_sort_u64", "oracle_sort_f64"):
            getattr(L, name).argtypes = [_u64p, ctypes.c_int64]
        L.oracle_sort_by_key_i32_p64.argtypes = [_i32p, _u64p, ctypes.c_int64]
        for name in ("oracle_sort_pairs_u32", "oracle_sort_pairs_f32"):
            getattr(L, name).argtypes = [_u32p, _i32p, ctypes.c_int64]
        L.oracle_segmented_sort_i32.argtypes = [_i32p, _i64p, ctypes.c_int64]
        L.oracle_segmented_sort_pairs_i32.argtypes = [_i32p, _i32p, _i64p, ctypes.c_int64]
        L.oracle_merge_i32.argtypes = [_i32p, ctypes.c_int64, _i32p, ctypes.c_int64, _i32p]
        L.oracle_merge_i32.restype = None
        L.oracle_corank_i32.argtypes = [_i32p, ctypes.c_int64, _i32p, ctypes.c_int64,
                                        ctypes.c_int64]
        L.oracle_corank_i32.restype = ctypes.c_int64
        L.oracle_corank_pairs_i32.argtypes = [_i32p, _i32p, ctypes.c_int64, _i32p, _i32p,
                                              ctypes.c_int64, ctypes.c_int64]
        L.oracle_corank_pairs_i32.restype = ctypes.c_int64
        L.oracle_count_i32.argtypes = [_i32p, ctypes.c_int64, ctypes.c_int32, _i64p, _i64p]
        L.oracle_count_i32.restype = None
        L.oracle_multiset_hash_i32.argtypes = [_i32p, ctypes.c_int64]
        L.oracle_multiset_hash_i32.restype = ctypes.c_uint64
        L.oracle_multiset_hash_pairs_i32.argtypes = [_i32p, _i32p, ctypes.c_int64]
        L.oracle_multiset_hash_pairs_i32.restype = ctypes.c_uint64
        L.oracle_network_failures01.argtypes = [_i32p, ctypes.c_int64, ctypes.c_int32]
        L.oracle_network_failures01.restype = ctypes.c_int64
        L.oracle_merging_network_failures01.argtypes = [_i32p, ctypes.c_int64, ctypes.c_int32,
                                                        ctypes.c_int32]
        L.oracle_merging_network_failures01.restype = ctypes.c_int64
        _lib = L
    return _lib


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_i32p)


def _i64(a):
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(_i64p)


def sort(keys):
    """Sorted copy of int32 keys."""
    a, p = _i32(np.array(keys, dtype=np.int32, copy=True))
    if lib().oracle_sort_i32(p, a.size) != 0:
        raise MemoryError("oracle sort failed")
    return a


def sort_pairs(keys, vals):
    """Copies of (keys, vals) sorted lexicographically by (key, val)."""
    k, pk = _i32(np.array(keys, dtype=np.int32, copy=True))
    v, pv = _i32(np.array(vals, dtype=np.int32, copy=True))
    assert k.size == v.size
    if lib().oracle_sort_pairs_i32(pk, pv, k.size) != 0:
        raise MemoryError("oracle pair sort failed")
    return k, v


def _bits(keys, dtype):
    """A uint32 copy of the keys' bit patterns (keys given as `dtype`)."""
    return np.ascontiguousarray(np.array(keys, dtype=dtype, copy=True).view(np.uint32))


def sort_u32(keys):
    """Sorted copy of uint32 keys (unsigned order)."""
    a = _bits(keys, np.uint32)
    if lib().oracle_sort_u32(a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), a.size) != 0:
        raise MemoryError("oracle sort failed")
    return a


def sort_f32(keys):
    """Sorted copy of float32 keys in IEEE 754 totalOrder (bit-exact: -0
    before +0, NaNs placed by sign and payload)."""
    a = _bits(keys, np.float32)
    if lib().oracle_sort_f32(a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), a.size) != 0:
        raise MemoryError("oracle sort failed")
    return a.view(np.float32)


def _sort64(fn, keys, dtype):
    a = np.ascontiguousarray(np.array(keys, dtype=dtype, copy=True).view(np.uint64))
    if fn(a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), a.size) != 0:
        raise MemoryError("oracle sort failed")
    return a.view(dtype)


def sort_i64(keys):
    """Sorted copy of int64 keys (signed order)."""
    return _sort64(lib().oracle_sort_i64, keys, np.int64)


def sort_u64(keys):
    """Sorted copy of uint64 keys (unsigned order)."""
    return _sort64(lib().oracle_sort_u64, keys, np.uint64)


def sort_f64(keys):
    """Sorted copy of float64 keys in IEEE 754 totalOrder (bit-exact: -0
    before +0, NaNs placed by sign and payload)."""
    return _sort64(lib().oracle_sort_f64, keys, np.float64)


def sort_by_key_p64(keys, vals):
    """Stable sort by int32 key carrying 64-bit payloads (any 8-byte dtype):
    copies (keys, vals) with keys nondecreasing, equal keys in input order."""
    k, pk = _i32(np.array(keys, dtype=np.int32, copy=True))
    v0 = np.array(vals, copy=True)
    assert v0.dtype.itemsize == 8 and v0.size == k.size
    v = np.ascontiguousarray(v0.view(np.uint64))
    if lib().oracle_sort_by_key_i32_p64(pk, v.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                        k.size) != 0:
        raise MemoryError("oracle sort by key failed")
    return k, v.view(v0.dtype)


def _sort_pairs_gen(fn, a, vals):
    v, pv = _i32(np.array(vals, dtype=np.int32, copy=True))
    assert a.size == v.size
    if fn(a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), pv, a.size) != 0:
        raise MemoryError("oracle pair sort failed")
    return a, v


def sort_pairs_u32(keys, vals):
    """(keys, vals) sorted by (unsigned key, signed value)."""
    return _sort_pairs_gen(lib().oracle_sort_pairs_u32, _bits(keys, np.uint32), vals)


def sort_pairs_f32(keys, vals):
    """(keys, vals) sorted by (key in IEEE 754 totalOrder, signed value)."""
    k, v = _sort_pairs_gen(lib().oracle_sort_pairs_f32, _bits(keys, np.float32), vals)
    return k.view(np.float32), v


def segmented_sort(keys, offsets):
    k, pk = _i32(np.array(keys, dtype=np.int32, copy=True))
    o, po = _i64(offsets)
    if lib().oracle_segmented_sort_i32(pk, po, o.size - 1) != 0:
        raise ValueError("oracle segmented sort failed (offsets not monotone?)")
    return k


def segmented_sort_pairs(keys, vals, offsets):
    k, pk = _i32(np.array(keys, dtype=np.int32, copy=True))
    v, pv = _i32(np.array(vals, dtype=np.int32, copy=True))
    o, po = _i64(offsets)
    if lib().oracle_segmented_sort_pairs_i32(pk, pv, po, o.size - 1) != 0:
        raise ValueError("oracle segmented pair sort failed")
    return k, v


def merge(A, B):
    a, pa = _i32(A)
    b, pb = _i32(B)
    out = np.empty(a.size + b.size, dtype=np.int32)
    lib().oracle_merge_i32(pa, a.size, pb, b.size, out.ctypes.data_as(_i32p))
    return out


def corank(A, B, d):
    a, pa = _i32(A)
    b, pb = _i32(B)
    return int(lib().oracle_corank_i32(pa, a.size, pb, b.size, int(d)))


def corank_pairs(Ak, Av, Bk, Bv, d):
    ak, pak = _i32(Ak)
    av, pav = _i32(Av)
    bk, pbk = _i32(Bk)
    bv, pbv = _i32(Bv)
    return int(lib().oracle_corank_pairs_i32(pak, pav, ak.size, pbk, pbv, bk.size, int(d)))


def count(a, x):
    """(#{a < x}, #{a <= x})."""
    arr, p = _i32(a)
    lt = ctypes.c_int64()
    le = ctypes.c_int64()
    lib().oracle_count_i32(p, arr.size, int(x), ctypes.byref(lt), ctypes.byref(le))
    return lt.value, le.value


def multiset_hash(a):
    arr, p = _i32(a)
    return int(lib().oracle_multiset_hash_i32(p, arr.size))


def multiset_hash_pairs(k, v):
    ka, pk = _i32(k)
    va, pv = _i32(v)
    return int(lib().oracle_multiset_hash_pairs_i32(pk, pv, ka.size))


def _comps(comparators):
    c = np.ascontiguousarray(np.asarray(comparators, dtype=np.int32).reshape(-1, 2))
    return c, c.ctypes.data_as(_i32p), c.shape[0]


def network_failures01(comparators, nwires):
    """How many of the 2^nwires 0-1 inputs the network leaves unsorted."""
    c, p, nc = _comps(comparators)
    return int(lib().oracle_network_failures01(p, nc, int(nwires)))


def merging_network_failures01(comparators, p_len, q_len):
    """How many of the sorted-halves 0-1 inputs the network leaves unsorted."""
    c, p, nc = _comps(comparators)
    return int(lib().oracle_merging_network_failures01(p, nc, int(p_len), int(q_len)))
