"""MI355X (gfx950) hybrid vectorized merge sort -- Python binding.

Thin ctypes marshalling over libhvms.so: every function named hvms_* below
calls the C entry point of the same name with device pointers taken from
torch tensors and the current HIP stream; all work runs in the library's HIP
kernels.  torch only provides device memory and streams.  Importing this
package does not load the library; the first call does, and raises if the
library has not been built (python -m paper_2409_03970_amd.build).
"""
import contextlib
import ctypes
import functools
import inspect
import os

import torch

__all__ = [
    "HvmsError", "Options", "lib", "CORANK_BINARY", "CORANK_LEARNED", "CORANK_LINEAR",
    "CDF_PARAMS", "STAT_NAMES", "STATS_WORDS", "corank_stats",
    "hvms_sort_i32", "hvms_sort_pairs_i32", "hvms_sort_runs_i32", "hvms_merge_pass_i32",
    "hvms_corank_i32", "hvms_segmented_sort_i32", "hvms_segmented_sort_pairs_i32",
    "hvms_cdf_forward", "hvms_cdf_backward", "hvms_cdf_adam_step", "hvms_cdf_train",
    "sort", "sort_pairs", "sort_runs", "merge_pass", "corank", "segmented_sort",
    "segmented_sort_pairs", "cdf_forward", "cdf_backward", "cdf_adam_step", "cdf_train",
    "hvms_cdf_sample_i32", "cdf_sample", "fit_cdf_model", "segmented_sort_pairs_grouped",
    "segment_groups", "grouped_workspace_bytes", "hvms_sort_u32", "hvms_sort_f32", "hvms_sort_pairs_u32",
    "hvms_sort_pairs_f32", "sort_keys", "sort_pairs_keys", "hvms_sort_i64", "hvms_sort_u64",
    "hvms_sort_f64", "hvms_sort_by_key_i32_p64", "sort_by_key", "hvms_segmented_status",
    "hvms_sort_i32_noalloc", "SORT_NOALLOC_MAX_KEYS", "hvms_merge_runs_i32",
    "hvms_cdf_param_count",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhvms.so")

CORANK_BINARY, CORANK_LEARNED, CORANK_LINEAR = 0, 1, 2
CDF_PARAMS = 1153
STAT_NAMES = ("coranks", "probes", "fallbacks", "abs_err_sum", "max_err", "predicted")
STATS_WORDS = 136        # words 8..71: probe histogram; 72..135: |error| bit-length histogram


def _quantile_bin(hist, q):
    """Smallest bin b with at least a fraction q of the histogram's mass in
    bins 0..b (None for an empty histogram)."""
    total = sum(hist)
    if total == 0:
        return None
    need, acc = q * total, 0
    for b, h in enumerate(hist):
        acc += h
        if acc >= need:
            return b
    return len(hist) - 1


def corank_stats(words):
    """Summary of a co-rank stats buffer (HVMS_STATS_WORDS uint64 words, as
    a list or tensor): counts, mean and 99th-percentile probes per co-rank,
    and over the co-ranks that used a prediction (learned / linear mode) the
    fallback rate, mean, 99th-percentile bound and max of
    |prediction - co-rank|.  The error percentile comes
    from the bit-length histogram, so it is reported as an upper bound
    (2^b - 1 for bin b)."""
    w = [int(v) for v in (words.tolist() if hasattr(words, "tolist") else words)]
    n = max(w[0], 1)
    ph, eh = w[8:72], w[72:136]
    r = {"coranks": w[0], "probes_mean": round(w[1] / n, 2),
         "probes_p99": _quantile_bin(ph, 0.99)}
    if w[5]:
        p = w[5]
        b = _quantile_bin(eh, 0.99)
        r.update(predicted=p, fallback_rate=round(w[2] / p, 4), abs_err_mean=round(w[3] / p, 1),
                 abs_err_p99_at_most=(1 << b) - 1, max_err=w[4])
    return r


class HvmsError(RuntimeError):
    def __init__(self, fn, status):
        msg = lib().hvms_status_string(status).decode()
        hip = lib().hvms_last_hip_error()
        super().__init__(f"{fn} failed: {msg} (status {status}, hip error {hip})")
        self.status = status


class Options(ctypes.Structure):
    """Mirror of hvms_options (0 / None keeps a field's default)."""
    _fields_ = [
        ("keys_per_lane", ctypes.c_int32),
        ("block_threads", ctypes.c_int32),
        ("wave_levels", ctypes.c_int32),
        ("merge_tile", ctypes.c_int32),
        ("corank_mode", ctypes.c_int32),
        ("radius_log2", ctypes.c_int32),
        ("cdf_params", ctypes.c_void_p),
        ("stats", ctypes.c_void_p),
        ("events", ctypes.POINTER(ctypes.c_void_p)),
        ("n_events", ctypes.c_int32),
        ("merge_variant", ctypes.c_int32),
        ("merge_occupancy", ctypes.c_int32),
        ("column_network", ctypes.c_int32),
        ("merge_ways", ctypes.c_int32),
    ]


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_sz = ctypes.c_size_t
_f32 = ctypes.c_float
_u64 = ctypes.c_uint64
_opt = ctypes.POINTER(Options)

_SIGS = {
    "hvms_status_string": ([_i32], ctypes.c_char_p),
    "hvms_last_hip_error": ([], _i32),
    "hvms_sort_workspace_bytes": ([_i64, _i32, _opt], _i64),
    "hvms_sort_i32": ([_vp, _vp, _i64, _vp, _sz, _vp, _opt], _i32),
    "hvms_sort_pairs_i32": ([_vp, _vp, _vp, _vp, _i64, _vp, _sz, _vp, _opt], _i32),
    "hvms_sort_runs_i32": ([_vp, _vp, _i64, _i32, _vp, _opt], _i32),
    "hvms_sort_u32": ([_vp, _vp, _i64, _vp, _sz, _vp, _opt], _i32),
    "hvms_sort_f32": ([_vp, _vp, _i64, _vp, _sz, _vp, _opt], _i32),
    "hvms_sort_pairs_u32": ([_vp, _vp, _vp, _vp, _i64, _vp, _sz, _vp, _opt], _i32),
    "hvms_sort_pairs_f32": ([_vp, _vp, _vp, _vp, _i64, _vp, _sz, _vp, _opt], _i32),
    "hvms_sort64_workspace_bytes": ([_i64, _opt], _i64),
    "hvms_sort_by_key_workspace_bytes": ([_i64, _opt], _i64),
    "hvms_sort_by_key_i32_p64": ([_vp, _vp, _vp, _vp, _i64, _vp, _sz, _vp, _opt], _i32),
    "hvms_sort_i64": ([_vp, _vp, _i64, _vp, _sz, _vp, _opt], _i32),
    "hvms_sort_u64": ([_vp, _vp, _i64, _vp, _sz, _vp, _opt], _i32),
    "hvms_sort_f64": ([_vp, _vp, _i64, _vp, _sz, _vp, _opt], _i32),
    "hvms_merge_workspace_bytes": ([_i64, _i64, _opt], _i64),
    "hvms_merge_pass_i32": ([_vp, _vp, _i64, _i64, _vp, _sz, _vp, _opt], _i32),
    "hvms_corank_i32": ([_vp, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _opt], _i32),
    "hvms_segmented_workspace_bytes": ([_i64, _i64, _i64, _i32, _opt], _i64),
    "hvms_segmented_sort_i32": ([_vp, _vp, _vp, _i64, _i64, _i64, _vp, _sz, _vp, _opt], _i32),
    "hvms_segmented_sort_pairs_i32": ([_vp, _vp, _vp, _vp, _vp, _i64, _i64, _i64, _vp, _sz, _vp,
                                       _opt], _i32),
    "hvms_cdf_forward": ([_vp, _vp, _vp, _i64, _vp], _i32),
    "hvms_cdf_workspace_bytes": ([_i64], _i64),
    "hvms_cdf_backward": ([_vp, _vp, _vp, _vp, _vp, _i64, _vp, _sz, _vp], _i32),
    "hvms_cdf_adam_step": ([_vp, _vp, _vp, _vp, _i32, _f32, _f32, _f32, _f32, _vp], _i32),
    "hvms_cdf_train_workspace_bytes": ([_i64], _i64),
    "hvms_cdf_train": ([_vp, _vp, _vp, _vp, _i64, _i64, _i32, _f32, _u64, _vp, _sz, _vp], _i32),
    "hvms_cdf_sample_i32": ([_vp, _i64, _i64, _u64, _vp, _vp], _i32),
    "hvms_segmented_status": ([_vp, _vp, _vp], _i32),
    "hvms_merge_runs_i32": ([_vp, _vp, _i64, _i32, _i32, _i32, _vp], _i32),
    "hvms_cdf_param_count": ([], _i64),
    "hvms_sort_i32_noalloc": ([_vp, _vp, _i64, _vp, _opt], _i32),
}

SORT_NOALLOC_MAX_KEYS = 1 << 22

_lib = None


def lib():
    """The loaded libhvms.so (raises if it was never built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2409_03970_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


# ------------------------------------------------------------------ helpers

def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return _vp(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _on(stream):
    """Context for the allocating conveniences: tensors they allocate (the
    workspace, temporaries, outputs) belong to the stream the library's
    kernels run on, so the caching allocator never hands that memory to
    other work before those kernels are done with it."""
    if stream is None:
        return contextlib.nullcontext()
    if not isinstance(stream, torch.cuda.Stream):
        stream = torch.cuda.ExternalStream(int(getattr(stream, "cuda_stream", stream)))
    return torch.cuda.stream(stream)


def _alloc_on_stream(fn):
    """Runs an allocating convenience inside _on(its `stream` argument)."""
    sig = inspect.signature(fn)

    @functools.wraps(fn)
    def wrapper(*args, **kwargs):
        with _on(sig.bind_partial(*args, **kwargs).arguments.get("stream")):
            return fn(*args, **kwargs)
    return wrapper


def _ptr(t, dtype=None, name="tensor"):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    return _vp(t.data_ptr())


def _opts(opts):
    if opts is None:
        return None
    if isinstance(opts, Options):
        return ctypes.byref(opts)
    o = Options()
    for k, v in opts.items():
        if k in ("cdf_params", "stats"):
            if k == "stats" and v is not None and (
                    v.element_size() != 8 or v.numel() < STATS_WORDS or not v.is_contiguous()):
                # the co-rank kernels write all STATS_WORDS words
                raise ValueError(f"stats must be a contiguous 64-bit tensor of at least "
                                 f"{STATS_WORDS} words")
            if k == "cdf_params" and v is not None and (
                    v.dtype != torch.float32 or v.numel() < CDF_PARAMS or not v.is_contiguous()):
                raise ValueError(f"cdf_params must be a contiguous float32 tensor of "
                                 f"{CDF_PARAMS} values")
            setattr(o, k, None if v is None else v.data_ptr())
        elif k == "events":
            # torch.cuda.Event objects (already recorded once, so they exist)
            arr = (ctypes.c_void_p * len(v))(*[e.cuda_event for e in v])
            o.events = ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p))
            o.n_events = len(v)
            o._keep = arr
        else:
            setattr(o, k, int(v))
    return ctypes.byref(o)


def _check(fn, status):
    if status != 0:
        raise HvmsError(fn, status)


def _workspace(nbytes, device):
    if nbytes < 0:
        raise HvmsError("workspace query", int(nbytes))
    if nbytes == 0:
        return None
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


def _wsargs(ws):
    if ws is None:
        return None, 0
    return _vp(ws.data_ptr()), ws.numel()


# ----------------------------------------------------- C entry points (1:1)

def hvms_sort_i32(d_in, d_out, ws=None, stream=None, opts=None):
    p, b = _wsargs(ws)
    _check("hvms_sort_i32", lib().hvms_sort_i32(
        _ptr(d_in, torch.int32, "in"), _ptr(d_out, torch.int32, "out"), d_in.numel(), p, b,
        _stream(stream), _opts(opts)))


def hvms_sort_i32_noalloc(d_in, d_out, stream=None, opts=None):
    """hvms_sort_i32 on the library's fixed per-device scratch (no workspace,
    no allocation; n <= SORT_NOALLOC_MAX_KEYS; calls overlapping on one GPU
    race)."""
    if d_in.numel() != d_out.numel():
        raise ValueError("in and out differ in length")
    _check("hvms_sort_i32_noalloc", lib().hvms_sort_i32_noalloc(
        _ptr(d_in, torch.int32, "in"), _ptr(d_out, torch.int32, "out"), d_in.numel(),
        _stream(stream), _opts(opts)))


def hvms_sort_pairs_i32(k_in, v_in, k_out, v_out, ws=None, stream=None, opts=None):
    assert k_in.numel() == v_in.numel() == k_out.numel() == v_out.numel()
    p, b = _wsargs(ws)
    _check("hvms_sort_pairs_i32", lib().hvms_sort_pairs_i32(
        _ptr(k_in, torch.int32), _ptr(v_in, torch.int32), _ptr(k_out, torch.int32),
        _ptr(v_out, torch.int32), k_in.numel(), p, b, _stream(stream), _opts(opts)))


# unsigned keys may come as torch.uint32 / uint64 or as signed bit patterns
_KEY_DTYPES = {"u32": (torch.uint32, torch.int32), "f32": (torch.float32,),
               "i64": (torch.int64,), "u64": (torch.uint64, torch.int64),
               "f64": (torch.float64,)}


def _kptr(t, kind, name):
    if t.dtype not in _KEY_DTYPES[kind]:
        raise ValueError(f"{name} must be one of {_KEY_DTYPES[kind]}, got {t.dtype}")
    return _ptr(t, None, name)


def hvms_sort_u32(d_in, d_out, ws=None, stream=None, opts=None):
    p, b = _wsargs(ws)
    _check("hvms_sort_u32", lib().hvms_sort_u32(
        _kptr(d_in, "u32", "in"), _kptr(d_out, "u32", "out"), d_in.numel(), p, b,
        _stream(stream), _opts(opts)))


def hvms_sort_f32(d_in, d_out, ws=None, stream=None, opts=None):
    p, b = _wsargs(ws)
    _check("hvms_sort_f32", lib().hvms_sort_f32(
        _kptr(d_in, "f32", "in"), _kptr(d_out, "f32", "out"), d_in.numel(), p, b,
        _stream(stream), _opts(opts)))


def _sort64(fn, kind, d_in, d_out, ws, stream, opts):
    assert d_in.numel() == d_out.numel()
    p, b = _wsargs(ws)
    _check(fn, getattr(lib(), fn)(
        _kptr(d_in, kind, "in"), _kptr(d_out, kind, "out"), d_in.numel(), p, b,
        _stream(stream), _opts(opts)))


def hvms_sort_i64(d_in, d_out, ws=None, stream=None, opts=None):
    _sort64("hvms_sort_i64", "i64", d_in, d_out, ws, stream, opts)


def hvms_sort_u64(d_in, d_out, ws=None, stream=None, opts=None):
    _sort64("hvms_sort_u64", "u64", d_in, d_out, ws, stream, opts)


def hvms_sort_f64(d_in, d_out, ws=None, stream=None, opts=None):
    _sort64("hvms_sort_f64", "f64", d_in, d_out, ws, stream, opts)


def hvms_sort_by_key_i32_p64(k_in, v_in, k_out, v_out, ws=None, stream=None, opts=None):
    assert k_in.numel() == v_in.numel() == k_out.numel() == v_out.numel()
    for t in (v_in, v_out):
        if t.element_size() != 8:
            raise ValueError(f"payloads must be 8-byte elements, got {t.dtype}")
    p, b = _wsargs(ws)
    _check("hvms_sort_by_key_i32_p64", lib().hvms_sort_by_key_i32_p64(
        _ptr(k_in, torch.int32), _ptr(v_in, None), _ptr(k_out, torch.int32), _ptr(v_out, None),
        k_in.numel(), p, b, _stream(stream), _opts(opts)))


def _sort_pairs_mapped(fn, kind, k_in, v_in, k_out, v_out, ws, stream, opts):
    assert k_in.numel() == v_in.numel() == k_out.numel() == v_out.numel()
    p, b = _wsargs(ws)
    _check(fn, getattr(lib(), fn)(
        _kptr(k_in, kind, "keys"), _ptr(v_in, torch.int32), _kptr(k_out, kind, "keys_out"),
        _ptr(v_out, torch.int32), k_in.numel(), p, b, _stream(stream), _opts(opts)))


def hvms_sort_pairs_u32(k_in, v_in, k_out, v_out, ws=None, stream=None, opts=None):
    _sort_pairs_mapped("hvms_sort_pairs_u32", "u32", k_in, v_in, k_out, v_out, ws, stream, opts)


def hvms_sort_pairs_f32(k_in, v_in, k_out, v_out, ws=None, stream=None, opts=None):
    _sort_pairs_mapped("hvms_sort_pairs_f32", "f32", k_in, v_in, k_out, v_out, ws, stream, opts)


def hvms_sort_runs_i32(d_in, d_out, run_log2, stream=None, opts=None):
    _check("hvms_sort_runs_i32", lib().hvms_sort_runs_i32(
        _ptr(d_in, torch.int32), _ptr(d_out, torch.int32), d_in.numel(), int(run_log2),
        _stream(stream), _opts(opts)))


def hvms_merge_runs_i32(d_in, d_out, x_log2, form, reps=1, stream=None):
    _check("hvms_merge_runs_i32", lib().hvms_merge_runs_i32(
        _ptr(d_in, torch.int32, "in"), _ptr(d_out, torch.int32, "out"), d_in.numel(),
        int(x_log2), int(form), int(reps), _stream(stream)))


def hvms_merge_pass_i32(d_in, d_out, run_len, ws=None, stream=None, opts=None):
    p, b = _wsargs(ws)
    _check("hvms_merge_pass_i32", lib().hvms_merge_pass_i32(
        _ptr(d_in, torch.int32), _ptr(d_out, torch.int32), d_in.numel(), int(run_len), p, b,
        _stream(stream), _opts(opts)))


def hvms_corank_i32(a, b, diag, out, stream=None, opts=None):
    _check("hvms_corank_i32", lib().hvms_corank_i32(
        _ptr(a, torch.int32), a.numel(), _ptr(b, torch.int32), b.numel(),
        _ptr(diag, torch.int64), diag.numel(), _ptr(out, torch.int64), _stream(stream),
        _opts(opts)))


def hvms_segmented_sort_i32(d_in, d_out, d_offsets, n_total, max_seg, ws=None, stream=None,
                            opts=None):
    p, b = _wsargs(ws)
    _check("hvms_segmented_sort_i32", lib().hvms_segmented_sort_i32(
        _ptr(d_in, torch.int32), _ptr(d_out, torch.int32), _ptr(d_offsets, torch.int64),
        d_offsets.numel() - 1, int(n_total), int(max_seg), p, b, _stream(stream), _opts(opts)))


def hvms_segmented_sort_pairs_i32(k_in, v_in, k_out, v_out, d_offsets, n_total, max_seg,
                                  ws=None, stream=None, opts=None):
    p, b = _wsargs(ws)
    _check("hvms_segmented_sort_pairs_i32", lib().hvms_segmented_sort_pairs_i32(
        _ptr(k_in, torch.int32), _ptr(v_in, torch.int32), _ptr(k_out, torch.int32),
        _ptr(v_out, torch.int32), _ptr(d_offsets, torch.int64), d_offsets.numel() - 1,
        int(n_total), int(max_seg), p, b, _stream(stream), _opts(opts)))


def hvms_segmented_status(ws, status, stream=None):
    """Enqueue the copy of the status words of the last segmented call on
    workspace ws into status (int64 device tensor of at least 3 entries)."""
    if status.numel() < 3:
        raise ValueError("status needs 3 int64 entries")
    _check("hvms_segmented_status", lib().hvms_segmented_status(
        _ptr(ws, None, "ws"), _ptr(status, torch.int64, "status"), _stream(stream)))


def hvms_cdf_param_count():
    return int(lib().hvms_cdf_param_count())


def hvms_cdf_forward(params, x, y, stream=None):
    _check("hvms_cdf_forward", lib().hvms_cdf_forward(
        _ptr(params, torch.float32), _ptr(x, torch.float32), _ptr(y, torch.float32), x.numel(),
        _stream(stream)))


def hvms_cdf_backward(params, x, t, grad, loss, ws=None, stream=None):
    p, b = _wsargs(ws)
    _check("hvms_cdf_backward", lib().hvms_cdf_backward(
        _ptr(params, torch.float32), _ptr(x, torch.float32), _ptr(t, torch.float32),
        _ptr(grad, torch.float32), _ptr(loss, torch.float32), x.numel(), p, b, _stream(stream)))


def hvms_cdf_adam_step(params, m, v, grad, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                       stream=None):
    _check("hvms_cdf_adam_step", lib().hvms_cdf_adam_step(
        _ptr(params, torch.float32), _ptr(m, torch.float32), _ptr(v, torch.float32),
        _ptr(grad, torch.float32), int(step), lr, beta1, beta2, eps, _stream(stream)))


def hvms_cdf_train(params, m, v, sorted_keys, batch, steps, lr, seed, ws=None, stream=None):
    p, b = _wsargs(ws)
    _check("hvms_cdf_train", lib().hvms_cdf_train(
        _ptr(params, torch.float32), _ptr(m, torch.float32), _ptr(v, torch.float32),
        _ptr(sorted_keys, torch.int32), sorted_keys.numel(), int(batch), int(steps), lr,
        int(seed) & 0xFFFFFFFFFFFFFFFF, p, b, _stream(stream)))


def hvms_cdf_sample_i32(keys, m, seed, out, stream=None):
    _check("hvms_cdf_sample_i32", lib().hvms_cdf_sample_i32(
        _ptr(keys, torch.int32), keys.numel(), int(m), int(seed) & 0xFFFFFFFFFFFFFFFF,
        _ptr(out, torch.int32), _stream(stream)))


# -------------------------------------------------- allocating conveniences

def _auto(op, n, opts):
    """Explicit options win; otherwise the autotuner's cached entry, if any."""
    if opts is not None:
        return opts
    from . import tune
    return tune.tuned_options(op, n)


@_alloc_on_stream
def sort(keys, out=None, opts=None, stream=None):
    """Sorted copy of an int32 device tensor (out may be keys: in place)."""
    opts = _auto("sort", keys.numel(), opts)
    if out is None:
        out = torch.empty_like(keys)
    ws = _workspace(lib().hvms_sort_workspace_bytes(keys.numel(), 0, _opts(opts)), keys.device)
    hvms_sort_i32(keys, out, ws, stream, opts)
    return out


@_alloc_on_stream
def sort_pairs(keys, vals, keys_out=None, vals_out=None, opts=None, stream=None):
    opts = _auto("sort_pairs", keys.numel(), opts)
    keys_out = torch.empty_like(keys) if keys_out is None else keys_out
    vals_out = torch.empty_like(vals) if vals_out is None else vals_out
    ws = _workspace(lib().hvms_sort_workspace_bytes(keys.numel(), 1, _opts(opts)), keys.device)
    hvms_sort_pairs_i32(keys, vals, keys_out, vals_out, ws, stream, opts)
    return keys_out, vals_out


_SORT64 = {torch.int64: hvms_sort_i64, torch.uint64: hvms_sort_u64,
           torch.float64: hvms_sort_f64}


@_alloc_on_stream
def sort_keys(keys, out=None, opts=None, stream=None):
    """Sorted copy of a device tensor of int32, uint32 (torch.uint32), float32
    (IEEE 754 totalOrder), int64, uint64 (torch.uint64) or float64 keys; out
    may be keys (in place)."""
    if keys.dtype == torch.int32:
        return sort(keys, out, opts, stream)
    fn64 = _SORT64.get(keys.dtype)
    if fn64 is not None:
        # 64-bit keys run on the key-value kernels: their tuning applies
        opts = _auto("sort_pairs", keys.numel(), opts)
        out = torch.empty_like(keys) if out is None else out
        ws = _workspace(lib().hvms_sort64_workspace_bytes(keys.numel(), _opts(opts)),
                        keys.device)
        fn64(keys, out, ws, stream, opts)
        return out
    fn = {torch.uint32: hvms_sort_u32, torch.float32: hvms_sort_f32}.get(keys.dtype)
    if fn is None:
        raise ValueError(f"unsupported key dtype {keys.dtype}")
    opts = _auto("sort", keys.numel(), opts)
    out = torch.empty_like(keys) if out is None else out
    ws = _workspace(lib().hvms_sort_workspace_bytes(keys.numel(), 0, _opts(opts)), keys.device)
    fn(keys, out, ws, stream, opts)
    return out


@_alloc_on_stream
def sort_pairs_keys(keys, vals, keys_out=None, vals_out=None, opts=None, stream=None):
    """sort_pairs for int32, uint32 (torch.uint32) or float32 keys with int32
    values, lexicographic (key, value)."""
    if keys.dtype == torch.int32:
        return sort_pairs(keys, vals, keys_out, vals_out, opts, stream)
    fn = {torch.uint32: hvms_sort_pairs_u32, torch.float32: hvms_sort_pairs_f32}.get(keys.dtype)
    if fn is None:
        raise ValueError(f"unsupported key dtype {keys.dtype}")
    opts = _auto("sort_pairs", keys.numel(), opts)
    keys_out = torch.empty_like(keys) if keys_out is None else keys_out
    vals_out = torch.empty_like(vals) if vals_out is None else vals_out
    ws = _workspace(lib().hvms_sort_workspace_bytes(keys.numel(), 1, _opts(opts)), keys.device)
    fn(keys, vals, keys_out, vals_out, ws, stream, opts)
    return keys_out, vals_out


@_alloc_on_stream
def sort_by_key(keys, vals, keys_out=None, vals_out=None, opts=None, stream=None):
    """Stable sort of int32 keys carrying 64-bit payloads (vals: any 8-byte
    dtype); equal keys keep their input order.  keys_out may be keys."""
    opts = _auto("sort_pairs", keys.numel(), opts)
    keys_out = torch.empty_like(keys) if keys_out is None else keys_out
    vals_out = torch.empty_like(vals) if vals_out is None else vals_out
    ws = _workspace(lib().hvms_sort_by_key_workspace_bytes(keys.numel(), _opts(opts)),
                    keys.device)
    hvms_sort_by_key_i32_p64(keys, vals, keys_out, vals_out, ws, stream, opts)
    return keys_out, vals_out


@_alloc_on_stream
def sort_runs(keys, run_log2, out=None, opts=None, stream=None):
    out = torch.empty_like(keys) if out is None else out
    hvms_sort_runs_i32(keys, out, run_log2, stream, opts)
    return out


@_alloc_on_stream
def merge_pass(keys, run_len, out=None, opts=None, stream=None):
    out = torch.empty_like(keys) if out is None else out
    ws = _workspace(lib().hvms_merge_workspace_bytes(keys.numel(), int(run_len), _opts(opts)),
                    keys.device)
    hvms_merge_pass_i32(keys, out, run_len, ws, stream, opts)
    return out


@_alloc_on_stream
def corank(a, b, diag, opts=None, stream=None):
    out = torch.empty(diag.numel(), dtype=torch.int64, device=a.device)
    hvms_corank_i32(a, b, diag, out, stream, opts)
    return out


def _host_offsets(offsets, n_keys):
    """Offsets on the host, checked: nondecreasing, within [0, n_keys].  The
    library skips invalid segments (and counts them, see
    hvms_segmented_status); the conveniences refuse them instead."""
    off_host = offsets.cpu()
    if off_host.numel():
        if off_host.dtype != torch.int64:
            raise ValueError(f"offsets must be int64, got {off_host.dtype}")
        if int(off_host[0]) < 0 or int(off_host[-1]) > n_keys or \
                bool((off_host[1:] < off_host[:-1]).any()):
            raise ValueError("offsets must be nondecreasing and within [0, number of keys]")
    return off_host


@_alloc_on_stream
def segmented_sort(keys, offsets, max_seg=None, out=None, opts=None, stream=None):
    """offsets: int64 tensor of nseg+1 entries (host or device)."""
    opts = _auto("segmented", keys.numel(), opts)
    out = torch.empty_like(keys) if out is None else out
    off_host = _host_offsets(offsets, keys.numel())
    nseg = off_host.numel() - 1
    n_total = int(off_host[-1]) if nseg >= 0 and off_host.numel() else 0
    if max_seg is None:
        max_seg = int((off_host[1:] - off_host[:-1]).max()) if nseg > 0 else 0
    d_off = offsets.to(keys.device) if not offsets.is_cuda else offsets
    ws = _workspace(lib().hvms_segmented_workspace_bytes(n_total, nseg, max_seg, 0, _opts(opts)),
                    keys.device)
    hvms_segmented_sort_i32(keys, out, d_off, n_total, max_seg, ws, stream, opts)
    return out


@_alloc_on_stream
def segmented_sort_pairs(keys, vals, offsets, max_seg=None, opts=None, stream=None):
    opts = _auto("segmented_pairs", keys.numel(), opts)
    ko, vo = torch.empty_like(keys), torch.empty_like(vals)
    off_host = _host_offsets(offsets, keys.numel())
    nseg = off_host.numel() - 1
    n_total = int(off_host[-1]) if off_host.numel() else 0
    if max_seg is None:
        max_seg = int((off_host[1:] - off_host[:-1]).max()) if nseg > 0 else 0
    d_off = offsets.to(keys.device) if not offsets.is_cuda else offsets
    ws = _workspace(lib().hvms_segmented_workspace_bytes(n_total, nseg, max_seg, 1, _opts(opts)),
                    keys.device)
    hvms_segmented_sort_pairs_i32(keys, vals, ko, vo, d_off, n_total, max_seg, ws, stream, opts)
    return ko, vo


def segment_groups(off_host, max_group_keys):
    """Consecutive segment ranges [s0, s1) whose keys (from off[s0] rounded
    down to a multiple of 4, so every group's arrays stay 16-byte aligned)
    fit max_group_keys; a single larger segment forms its own group."""
    groups, nseg, s0 = [], len(off_host) - 1, 0
    while s0 < nseg:
        base = off_host[s0] & ~3
        s1 = s0 + 1
        while s1 < nseg and off_host[s1 + 1] - base <= max_group_keys:
            s1 += 1
        groups.append((s0, s1, base))
        s0 = s1
    return groups


def grouped_workspace_bytes(offsets, max_group_keys=1 << 30, opts=None):
    """Workspace bytes segmented_sort_pairs_grouped needs for these offsets."""
    off_host = offsets.cpu().tolist() if hasattr(offsets, "cpu") else list(offsets)
    groups = segment_groups(off_host, max_group_keys)
    sizes = [off_host[i + 1] - off_host[i] for i in range(len(off_host) - 1)]
    max_seg = max(sizes) if sizes else 0
    gmax = max((off_host[s1] - base for s0, s1, base in groups), default=0)
    smax = max((s1 - s0 for s0, s1, base in groups), default=0)
    return lib().hvms_segmented_workspace_bytes(gmax, smax, max_seg, 1,
                                                _opts(opts if opts is not None else {}))


@_alloc_on_stream
def segmented_sort_pairs_grouped(keys, vals, offsets, max_group_keys=1 << 30, opts=None,
                                 stream=None, opts_for_group=None, ws=None):
    """In-place segmented pair sort with bounded scratch: the segments are
    sorted group by group (each group one batched call), so the workspace
    holds scratch for one group instead of the whole array.  opts_for_group,
    if given, is called as opts_for_group(keys_view, group_index) and returns
    the options of that group's call (e.g. a CDF model trained on it).  ws:
    an optional preallocated uint8 device tensor of at least
    grouped_workspace_bytes(offsets, max_group_keys, opts) bytes (else one is
    allocated here)."""
    off_host = offsets.cpu().tolist()
    d_off = offsets.to(keys.device) if not offsets.is_cuda else offsets
    groups = segment_groups(off_host, max_group_keys)
    sizes = [off_host[i + 1] - off_host[i] for i in range(len(off_host) - 1)]
    max_seg = max(sizes) if sizes else 0
    gmax = max((off_host[s1] - base for s0, s1, base in groups), default=0)
    smax = max((s1 - s0 for s0, s1, base in groups), default=0)
    o0 = opts if opts is not None else {}
    need = lib().hvms_segmented_workspace_bytes(gmax, smax, max_seg, 1, _opts(o0))
    if ws is None:
        ws = _workspace(need, keys.device)
    elif ws.numel() < need:
        raise ValueError(f"workspace of {ws.numel()} bytes, {need} needed")
    for gi, (s0, s1, base) in enumerate(groups):
        n_g = off_host[s1] - base
        kg = keys[base:base + n_g]
        vg = vals[base:base + n_g]
        sub = d_off[s0:s1 + 1] - base
        og = opts_for_group(kg, gi) if opts_for_group else opts
        hvms_segmented_sort_pairs_i32(kg, vg, kg, vg, sub, n_g, max(sizes[s0:s1]), ws,
                                      stream, og)
    return keys, vals


@_alloc_on_stream
def cdf_forward(params, x, stream=None):
    y = torch.empty_like(x)
    hvms_cdf_forward(params, x, y, stream)
    return y


@_alloc_on_stream
def cdf_backward(params, x, t, stream=None):
    grad = torch.empty(CDF_PARAMS, dtype=torch.float32, device=x.device)
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    ws = _workspace(lib().hvms_cdf_workspace_bytes(x.numel()), x.device)
    hvms_cdf_backward(params, x, t, grad, loss, ws, stream)
    return float(loss.item()), grad


def cdf_adam_step(params, m, v, grad, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                  stream=None):
    hvms_cdf_adam_step(params, m, v, grad, step, lr, beta1, beta2, eps, stream)


@_alloc_on_stream
def cdf_sample(keys, m, seed=0, stream=None):
    out = torch.empty(int(m), dtype=torch.int32, device=keys.device)
    hvms_cdf_sample_i32(keys, m, seed, out, stream)
    return out


@_alloc_on_stream
def fit_cdf_model(keys, frac=0.01, steps=400, batch=65536, lr=1e-3, seed=0, init=None,
                  stream=None):
    """The learned part end to end on the device: draw frac * n keys, sort the
    sample with this library's sort, train the CDF model on it with the
    library's forward/backward/Adam kernels.  Returns the fp32 parameters."""
    from . import inputs
    m = max(2, int(keys.numel() * frac))
    sample = cdf_sample(keys, m, seed, stream)
    sample = sort(sample, out=sample, stream=stream)
    params = (inputs.mlp_init(seed) if init is None else init).to(keys.device).contiguous()
    cdf_train(params, sample, batch=min(batch, m), steps=steps, lr=lr, seed=seed, stream=stream)
    return params


@_alloc_on_stream
def cdf_train(params, sorted_keys, batch=65536, steps=500, lr=1e-3, seed=0, stream=None):
    """Trains params (in place) on a sorted sample; returns (params, m, v)."""
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    ws = _workspace(lib().hvms_cdf_train_workspace_bytes(int(batch)), params.device)
    hvms_cdf_train(params, m, v, sorted_keys, batch, steps, lr, seed, ws, stream)
    return params, m, v
