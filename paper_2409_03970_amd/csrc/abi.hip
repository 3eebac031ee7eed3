// C ABI: argument validation, workspace layout, tuning resolution and the
// enqueue order of the sort's kernels.  No device memory is allocated here.
#include <stdint.h>
#include <string.h>

#include <mutex>

#include "hvms.h"
#include "hvms_internal.h"

using namespace hvms;

namespace {

thread_local int g_last_hip = 0;

}  // namespace

void hvms::set_last_hip_error(int e) { g_last_hip = e; }

namespace {

int hip_status(hipError_t e)
{
    if (e == hipSuccess)
        return HVMS_OK;
    g_last_hip = (int)e;
    return e == hipErrorInvalidValue ? HVMS_ERR_UNSUPPORTED : HVMS_ERR_HIP;
}

int ilog2_exact(int64_t x)
{
    int l = 0;
    while (((int64_t)1 << l) < x)
        ++l;
    return l;
}

int64_t align256(int64_t b) { return (b + 255) & ~(int64_t)255; }

struct Cfg {
    int R, NT, K, TM, variant, occupancy, net, ways;
    CorankOpts co;
    void *const *events;
    int n_events;
};

void trace(const Cfg &c, int idx, hipStream_t s)
{
    if (c.events && idx < c.n_events && c.events[idx])
        (void)hipEventRecord((hipEvent_t)c.events[idx], s);
}

int resolve(const hvms_options *o, bool pairs, Cfg &c)
{
    c.R = (o && o->keys_per_lane) ? o->keys_per_lane : 16;
    c.NT = (o && o->block_threads) ? o->block_threads : (pairs ? 512 : 512);
    c.K = (o && o->wave_levels) ? o->wave_levels - 1 : 6;
    c.TM = (o && o->merge_tile) ? o->merge_tile : (pairs ? 4096 : 8192);
    if (!(o && o->merge_tile) && c.TM > 2 * c.R * c.NT)
        c.TM = 2 * c.R * c.NT;
    c.ways = (o && o->merge_ways) ? o->merge_ways : 2;
    if (c.ways != 2 && c.ways != 4)
        return HVMS_ERR_INVALID_ARG;
    c.net = o ? o->column_network : 0;
    if (c.net < 0 || c.net > 2 || (c.net != 0 && (c.R != 16 || pairs)))
        return c.net < 0 || c.net > 2 ? HVMS_ERR_INVALID_ARG : HVMS_ERR_UNSUPPORTED;
    c.variant = o ? o->merge_variant : 0;
    c.occupancy = o ? o->merge_occupancy : 0;
    if (c.variant < 0 || c.variant > 4 || c.occupancy < 0 || c.occupancy > 32)
        return HVMS_ERR_INVALID_ARG;
    if (c.variant == 4 && pairs)  // the bitonic register merge is built for keys
        return HVMS_ERR_UNSUPPORTED;
    c.co.mode = o ? o->corank_mode : HVMS_CORANK_BINARY;
    c.co.radius_log2 = (o && o->radius_log2) ? o->radius_log2 : 12;
    c.co.cdf = o ? o->cdf_params : nullptr;
    c.co.stats = o ? o->stats : nullptr;
    c.events = o ? o->events : nullptr;
    c.n_events = o ? o->n_events : 0;
    if (c.K < 0 || c.K > 6 || c.co.radius_log2 < 0 || c.co.radius_log2 > 40)
        return HVMS_ERR_INVALID_ARG;
    if (c.co.mode < HVMS_CORANK_BINARY || c.co.mode > HVMS_CORANK_LINEAR)
        return HVMS_ERR_INVALID_ARG;
    if (c.co.mode == HVMS_CORANK_LEARNED && !c.co.cdf)
        return HVMS_ERR_INVALID_ARG;
    if (!block_sort_supported(c.R, c.NT, pairs) || !merge_tile_supported(c.TM, pairs))
        return HVMS_ERR_UNSUPPORTED;
    if (c.ways == 4 && !merge4_supported(c.TM, pairs))
        return HVMS_ERR_UNSUPPORTED;
    if ((int64_t)c.TM > 2 * (int64_t)c.R * c.NT)
        return HVMS_ERR_UNSUPPORTED;
    return HVMS_OK;
}

struct SortWs {
    int64_t scratch_k, scratch_v, alt_k, alt_v, coranks, records, table, total;
};

// packed: a 64-bit key sort, whose passes ping-pong between two split
// (key, value) buffer pairs in the workspace, since the caller's arrays hold
// the packed form.
SortWs sort_ws_layout(int64_t n, bool pairs, const Cfg &c, bool packed = false)
{
    SortWs w{};
    const int64_t tile = (int64_t)c.R * c.NT;
    if (n <= tile)
        return w;
    w.scratch_k = 0;
    int64_t off = align256(n * 4);
    if (pairs) {
        w.scratch_v = off;
        off += align256(n * 4);
    }
    if (packed) {
        w.alt_k = off;
        off += align256(n * 4);
        w.alt_v = off;
        off += align256(n * 4);
    }
    const int64_t ntiles = (n + c.TM - 1) / c.TM;
    w.coranks = off;  // one int64 per tile
    off += align256((ntiles + 2) * 8);
    if (c.ways == 4) {  // four-way passes: one window-geometry record per tile
        w.records = off;
        off += align256((ntiles + 2) * (int64_t)merge4_record_bytes());
    }
    // the learned co-rank's model, sampled once per sort (reserved in every
    // mode, so one workspace serves calls that switch co-rank modes)
    w.table = off;
    off += kCdfTableBytes;
    w.total = off;
    return w;
}

int check_ws(void *ws, size_t bytes, int64_t need)
{
    if (need == 0)
        return HVMS_OK;
    if (!ws || (int64_t)bytes < need || ((uintptr_t)ws & 255))
        return HVMS_ERR_WORKSPACE;
    return HVMS_OK;
}

// km: the key map of a uint32 / float32 / 64-bit sort, applied as the keys
// are loaded by the block stage and undone as the last launch stores them;
// km.packed: kin and kout are packed 64-bit key arrays (pairs must be set).
int run_sort(bool pairs, const int32_t *kin, const int32_t *vin, int32_t *kout, int32_t *vout,
             int64_t n, void *ws, hipStream_t s, const Cfg &c, KeyMap km = {})
{
    const int64_t tile = (int64_t)c.R * c.NT;
    const int lanes_log2 = ilog2_exact(c.NT);  // levels from R-runs to the tile
    const int K = c.K;
    const int lds_levels = lanes_log2 - K;
    if (n <= tile)
        return hip_status(
            launch_block_sort(c.R, c.NT, pairs, kin, vin, kout, vout, n, K, lds_levels, false, s,
                              c.net, km, km));

    const SortWs w = sort_ws_layout(n, pairs, c, km.packed);
    char *base = (char *)ws;
    int32_t *sk = (int32_t *)(base + w.scratch_k);
    int32_t *sv = pairs ? (int32_t *)(base + w.scratch_v) : nullptr;
    int64_t *cr = (int64_t *)(base + w.coranks);
    CorankOpts co = c.co;
    if (co.mode == HVMS_CORANK_LEARNED) {
        co.table = (const float *)(base + w.table);
        const int st0 = hip_status(launch_cdf_table(co.cdf, (float *)(base + w.table), s));
        if (st0)
            return st0;
    }
    // the passes alternate between (ak, av) and (sk, sv); the last one
    // writes the caller's arrays, in packed form for a 64-bit key sort
    int32_t *ak = km.packed ? (int32_t *)(base + w.alt_k) : kout;
    int32_t *av = km.packed ? (int32_t *)(base + w.alt_v) : vout;

    // Four-way passes move 16-byte chunks of the arrays they read and write:
    // a caller's output that is not 16-byte aligned takes two-way passes,
    // whose launcher has a fallback for it.
    const bool out_aligned =
        (uintptr_t)kout % 16 == 0 && (!pairs || km.packed || (uintptr_t)vout % 16 == 0);
    const int64_t nb = (n + tile - 1) / tile;
    const int P = ilog2_exact(nb);  // merge levels
    const int P4 = c.ways == 4 && out_aligned ? P / 2 : 0;  // four-way passes (two levels each)
    const int P2 = P - 2 * P4;                               // two-way passes (first)
    const int passes = P2 + P4;
    int32_t *dk = (passes % 2 == 0) ? ak : sk;
    int32_t *dv = (passes % 2 == 0) ? av : sv;
    trace(c, 0, s);
    int st = hip_status(
        launch_block_sort(c.R, c.NT, pairs, kin, vin, dk, dv, n, K, lds_levels, false, s,
                          c.net, km, passes == 0 ? km : KeyMap{}));
    if (st)
        return st;
    trace(c, 1, s);
    int64_t run = tile;
    for (int p = 0; p < passes; ++p) {
        int32_t *ok = (dk == ak) ? sk : ak;
        int32_t *ov = (dk == ak) ? sv : av;
        if (p == passes - 1) {
            ok = kout;
            ov = km.packed ? nullptr : vout;
        }
        if (p >= P2) {
            st = hip_status(launch_merge4_corank(c.TM, pairs, dk, dv, n, run, base + w.records,
                                                 co, s));
            if (st)
                return st;
            trace(c, 2 + 2 * p, s);
            st = hip_status(launch_merge4_pass(c.TM, pairs, dk, dv, ok, ov, n, run,
                                               base + w.records, c.occupancy, s,
                                               p == passes - 1 ? km : KeyMap{}));
            if (st)
                return st;
            trace(c, 3 + 2 * p, s);
            dk = ok;
            dv = ov;
            run *= 4;
            continue;
        }
        st = hip_status(launch_pass_corank(pairs, dk, dv, n, run, c.TM, cr, co, s));
        if (st)
            return st;
        trace(c, 2 + 2 * p, s);
        st = hip_status(launch_merge_pass(c.TM, pairs, dk, dv, ok, ov, n, run, cr, c.variant,
                                          c.occupancy, s, p == passes - 1 ? km : KeyMap{}));
        if (st)
            return st;
        trace(c, 3 + 2 * p, s);
        dk = ok;
        dv = ov;
        run *= 2;
    }
    return HVMS_OK;
}

}  // namespace

extern "C" {

const char *hvms_status_string(int status)
{
    switch (status) {
    case HVMS_OK: return "ok";
    case HVMS_ERR_INVALID_ARG: return "invalid argument";
    case HVMS_ERR_WORKSPACE: return "workspace missing, too small or misaligned";
    case HVMS_ERR_HIP: return "HIP runtime error";
    case HVMS_ERR_UNSUPPORTED: return "unsupported tuning value";
    case HVMS_ERR_TOO_LARGE: return "input larger than the fixed scratch of this entry point";
    default: return "unknown status";
    }
}

int hvms_last_hip_error(void) { return g_last_hip; }

int64_t hvms_sort_workspace_bytes(int64_t n, int32_t pairs, const hvms_options *opt)
{
    Cfg c;
    if (n < 0)
        return HVMS_ERR_INVALID_ARG;
    const int st = resolve(opt, pairs != 0, c);
    if (st)
        return st;
    return sort_ws_layout(n, pairs != 0, c).total;
}

int hvms_sort_i32(const int32_t *d_in, int32_t *d_out, int64_t n, void *d_ws, size_t ws_bytes,
                  void *stream, const hvms_options *opt)
{
    if (n < 0 || (n > 0 && (!d_in || !d_out)))
        return HVMS_ERR_INVALID_ARG;
    Cfg c;
    int st = resolve(opt, false, c);
    if (st)
        return st;
    if (n == 0)
        return HVMS_OK;
    st = check_ws(d_ws, ws_bytes, sort_ws_layout(n, false, c).total);
    if (st)
        return st;
    return run_sort(false, d_in, nullptr, d_out, nullptr, n, d_ws, (hipStream_t)stream, c);
}

}  // extern "C"

// Scratch of hvms_sort_i32_noalloc: one fixed array per device.  In host
// code its name stands for a host-side shadow, never the device address, so
// every use below goes through the address hipGetSymbolAddress returns for
// the current device.
static __device__ __align__(256) unsigned char scratch[HVMS_SORT_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
void *g_scratch_ptr[64];  // per device, filled on its first call

// this device's copy of the array, looked up once per device
int scratch_for_current_device(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_status(e);
    if (dev < 0 || dev >= 64)
        return HVMS_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return hip_status(e);
        if (!p || ((uintptr_t)p & 255))
            return HVMS_ERR_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return HVMS_OK;
}

}  // namespace

extern "C" {

int hvms_sort_i32_noalloc(const int32_t *d_in, int32_t *d_out, int64_t n, void *stream,
                          const hvms_options *opt)
{
    if (n < 0 || (n > 0 && (!d_in || !d_out)))
        return HVMS_ERR_INVALID_ARG;
    Cfg c;
    int st = resolve(opt, false, c);
    if (st)
        return st;
    if (n > HVMS_SORT_NOALLOC_MAX_KEYS)
        return HVMS_ERR_TOO_LARGE;
    if (n == 0)
        return HVMS_OK;
    const int64_t need = sort_ws_layout(n, false, c).total;
    if (need > (int64_t)HVMS_SORT_NOALLOC_SCRATCH_BYTES)
        return HVMS_ERR_TOO_LARGE;
    void *ws = nullptr;
    if (need > 0) {
        st = scratch_for_current_device(&ws);
        if (st)
            return st;
    }
    return run_sort(false, d_in, nullptr, d_out, nullptr, n, ws, (hipStream_t)stream, c);
}

int hvms_sort_pairs_i32(const int32_t *d_keys_in, const int32_t *d_vals_in, int32_t *d_keys_out,
                        int32_t *d_vals_out, int64_t n, void *d_ws, size_t ws_bytes,
                        void *stream, const hvms_options *opt)
{
    if (n < 0 || (n > 0 && (!d_keys_in || !d_vals_in || !d_keys_out || !d_vals_out)))
        return HVMS_ERR_INVALID_ARG;
    Cfg c;
    int st = resolve(opt, true, c);
    if (st)
        return st;
    if (n == 0)
        return HVMS_OK;
    st = check_ws(d_ws, ws_bytes, sort_ws_layout(n, true, c).total);
    if (st)
        return st;
    return run_sort(true, d_keys_in, d_vals_in, d_keys_out, d_vals_out, n, d_ws,
                    (hipStream_t)stream, c);
}

}  // extern "C"

namespace {

KeyMap key_map_of(int kind)  // 1 uint32, 2 float32
{
    KeyMap m;
    if (kind == 1)
        m.um = (int32_t)0x80000000u;
    else
        m.fm = 0x7fffffff;
    return m;
}

int sort_keys_mapped(const void *d_in, void *d_out, int64_t n, void *d_ws, size_t ws_bytes,
                     void *stream, const hvms_options *opt, int kind)
{
    if (n < 0 || (n > 0 && (!d_in || !d_out)))
        return HVMS_ERR_INVALID_ARG;
    Cfg c;
    int st = resolve(opt, false, c);
    if (st)
        return st;
    if (n == 0)
        return HVMS_OK;
    st = check_ws(d_ws, ws_bytes, sort_ws_layout(n, false, c).total);
    if (st)
        return st;
    return run_sort(false, (const int32_t *)d_in, nullptr, (int32_t *)d_out, nullptr, n, d_ws,
                    (hipStream_t)stream, c, key_map_of(kind));
}

int sort_pairs_mapped(const void *d_keys_in, const int32_t *d_vals_in, void *d_keys_out,
                      int32_t *d_vals_out, int64_t n, void *d_ws, size_t ws_bytes, void *stream,
                      const hvms_options *opt, int kind)
{
    if (n < 0 || (n > 0 && (!d_keys_in || !d_vals_in || !d_keys_out || !d_vals_out)))
        return HVMS_ERR_INVALID_ARG;
    Cfg c;
    int st = resolve(opt, true, c);
    if (st)
        return st;
    if (n == 0)
        return HVMS_OK;
    st = check_ws(d_ws, ws_bytes, sort_ws_layout(n, true, c).total);
    if (st)
        return st;
    return run_sort(true, (const int32_t *)d_keys_in, d_vals_in, (int32_t *)d_keys_out,
                    d_vals_out, n, d_ws, (hipStream_t)stream, c, key_map_of(kind));
}

KeyMap key_map64_of(int kind)  // 0 int64, 1 uint64, 2 float64
{
    KeyMap m;
    m.packed = true;
    if (kind == 1) {
        m.um = (int32_t)0x80000000u;
    } else if (kind == 2) {
        m.fm = 0x7fffffff;
        m.fl = -1;
    }
    return m;
}

int sort_keys64(const void *d_in, void *d_out, int64_t n, void *d_ws, size_t ws_bytes,
                void *stream, const hvms_options *opt, int kind)
{
    if (n < 0 || (n > 0 && (!d_in || !d_out)))
        return HVMS_ERR_INVALID_ARG;
    if (n > 0 && (((uintptr_t)d_in | (uintptr_t)d_out) & 7))  // 64-bit elements
        return HVMS_ERR_INVALID_ARG;
    Cfg c;
    int st = resolve(opt, true, c);
    if (st)
        return st;
    if (n == 0)
        return HVMS_OK;
    st = check_ws(d_ws, ws_bytes, sort_ws_layout(n, true, c, true).total);
    if (st)
        return st;
    return run_sort(true, (const int32_t *)d_in, nullptr, (int32_t *)d_out, nullptr, n, d_ws,
                    (hipStream_t)stream, c, key_map64_of(kind));
}

}  // namespace

extern "C" {

int64_t hvms_sort64_workspace_bytes(int64_t n, const hvms_options *opt)
{
    Cfg c;
    if (n < 0)
        return HVMS_ERR_INVALID_ARG;
    const int st = resolve(opt, true, c);
    if (st)
        return st;
    return sort_ws_layout(n, true, c, true).total;
}

int hvms_sort_i64(const int64_t *d_in, int64_t *d_out, int64_t n, void *d_ws, size_t ws_bytes,
                  void *stream, const hvms_options *opt)
{
    return sort_keys64(d_in, d_out, n, d_ws, ws_bytes, stream, opt, 0);
}

int hvms_sort_u64(const uint64_t *d_in, uint64_t *d_out, int64_t n, void *d_ws, size_t ws_bytes,
                  void *stream, const hvms_options *opt)
{
    return sort_keys64(d_in, d_out, n, d_ws, ws_bytes, stream, opt, 1);
}

int hvms_sort_f64(const double *d_in, double *d_out, int64_t n, void *d_ws, size_t ws_bytes,
                  void *stream, const hvms_options *opt)
{
    return sort_keys64(d_in, d_out, n, d_ws, ws_bytes, stream, opt, 2);
}

int64_t hvms_sort_by_key_workspace_bytes(int64_t n, const hvms_options *opt)
{
    Cfg c;
    if (n < 0)
        return HVMS_ERR_INVALID_ARG;
    const int st = resolve(opt, true, c);
    if (st)
        return st;
    if (n == 0)
        return 0;
    return align256(n * 4) + sort_ws_layout(n, true, c).total;
}

int hvms_sort_by_key_i32_p64(const int32_t *d_keys_in, const uint64_t *d_vals_in,
                             int32_t *d_keys_out, uint64_t *d_vals_out, int64_t n, void *d_ws,
                             size_t ws_bytes, void *stream, const hvms_options *opt)
{
    if (n < 0 || n > INT32_MAX ||
        (n > 0 && (!d_keys_in || !d_vals_in || !d_keys_out || !d_vals_out)))
        return HVMS_ERR_INVALID_ARG;
    if (n > 0 && (((uintptr_t)d_vals_in | (uintptr_t)d_vals_out) & 7))
        return HVMS_ERR_INVALID_ARG;
    // the payload pass reads d_vals_in in permuted order: no overlap allowed
    const uintptr_t vi = (uintptr_t)d_vals_in, vo = (uintptr_t)d_vals_out;
    if (n > 0 && vi < vo + (uintptr_t)n * 8 && vo < vi + (uintptr_t)n * 8)
        return HVMS_ERR_INVALID_ARG;
    Cfg c;
    int st = resolve(opt, true, c);
    if (st)
        return st;
    if (n == 0)
        return HVMS_OK;
    const int64_t idx_bytes = align256(n * 4);
    st = check_ws(d_ws, ws_bytes, idx_bytes + sort_ws_layout(n, true, c).total);
    if (st)
        return st;
    int32_t *idx = (int32_t *)d_ws;
    KeyMap km;
    km.iota = true;
    st = run_sort(true, d_keys_in, nullptr, d_keys_out, idx, n, (char *)d_ws + idx_bytes,
                  (hipStream_t)stream, c, km);
    if (st)
        return st;
    return hip_status(launch_gather_u64(idx, d_vals_in, d_vals_out, n, (hipStream_t)stream));
}

int hvms_sort_u32(const uint32_t *d_in, uint32_t *d_out, int64_t n, void *d_ws, size_t ws_bytes,
                  void *stream, const hvms_options *opt)
{
    return sort_keys_mapped(d_in, d_out, n, d_ws, ws_bytes, stream, opt, 1);
}

int hvms_sort_f32(const float *d_in, float *d_out, int64_t n, void *d_ws, size_t ws_bytes,
                  void *stream, const hvms_options *opt)
{
    return sort_keys_mapped(d_in, d_out, n, d_ws, ws_bytes, stream, opt, 2);
}

int hvms_sort_pairs_u32(const uint32_t *d_keys_in, const int32_t *d_vals_in, uint32_t *d_keys_out,
                        int32_t *d_vals_out, int64_t n, void *d_ws, size_t ws_bytes,
                        void *stream, const hvms_options *opt)
{
    return sort_pairs_mapped(d_keys_in, d_vals_in, d_keys_out, d_vals_out, n, d_ws, ws_bytes,
                             stream, opt, 1);
}

int hvms_sort_pairs_f32(const float *d_keys_in, const int32_t *d_vals_in, float *d_keys_out,
                        int32_t *d_vals_out, int64_t n, void *d_ws, size_t ws_bytes,
                        void *stream, const hvms_options *opt)
{
    return sort_pairs_mapped(d_keys_in, d_vals_in, d_keys_out, d_vals_out, n, d_ws, ws_bytes,
                             stream, opt, 2);
}

int hvms_sort_runs_i32(const int32_t *d_in, int32_t *d_out, int64_t n, int32_t run_log2,
                       void *stream, const hvms_options *opt)
{
    if (n < 0 || (n > 0 && (!d_in || !d_out)))
        return HVMS_ERR_INVALID_ARG;
    Cfg c;
    int st = resolve(opt, false, c);
    if (st)
        return st;
    const int r_log2 = ilog2_exact(c.R);
    const int tile_log2 = r_log2 + ilog2_exact(c.NT);
    if (run_log2 < r_log2 || run_log2 > tile_log2)
        return HVMS_ERR_INVALID_ARG;
    if (n == 0)
        return HVMS_OK;
    const int levels = run_log2 - r_log2;
    const int K = levels < c.K ? levels : c.K;
    const bool blocked = run_log2 < tile_log2;
    return hip_status(launch_block_sort(c.R, c.NT, false, d_in, nullptr, d_out, nullptr, n, K,
                                        levels - K, blocked, (hipStream_t)stream, c.net));
}

int64_t hvms_merge_workspace_bytes(int64_t n, int64_t run_len, const hvms_options *opt)
{
    Cfg c;
    if (n < 0 || run_len <= 0)
        return HVMS_ERR_INVALID_ARG;
    const int st = resolve(opt, false, c);
    if (st)
        return st;
    return align256(((n + c.TM - 1) / c.TM + 1) * 8);
}

int hvms_merge_pass_i32(const int32_t *d_in, int32_t *d_out, int64_t n, int64_t run_len,
                        void *d_ws, size_t ws_bytes, void *stream, const hvms_options *opt)
{
    if (n < 0 || (n > 0 && (!d_in || !d_out)) || run_len <= 0 || (run_len & (run_len - 1)))
        return HVMS_ERR_INVALID_ARG;
    Cfg c;
    int st = resolve(opt, false, c);
    if (st)
        return st;
    if (2 * run_len < c.TM)
        return HVMS_ERR_INVALID_ARG;
    if (n == 0)
        return HVMS_OK;
    st = check_ws(d_ws, ws_bytes, hvms_merge_workspace_bytes(n, run_len, opt));
    if (st)
        return st;
    int64_t *cr = (int64_t *)d_ws;
    hipStream_t s = (hipStream_t)stream;
    st = hip_status(launch_pass_corank(false, d_in, nullptr, n, run_len, c.TM, cr, c.co, s));
    if (st)
        return st;
    return hip_status(launch_merge_pass(c.TM, false, d_in, nullptr, d_out, nullptr, n, run_len,
                                       cr, c.variant, c.occupancy, s));
}

int hvms_corank_i32(const int32_t *d_a, int64_t m, const int32_t *d_b, int64_t k,
                    const int64_t *d_diag, int64_t count, int64_t *d_out, void *stream,
                    const hvms_options *opt)
{
    if (m < 0 || k < 0 || count < 0 || (m > 0 && !d_a) || (k > 0 && !d_b) ||
        (count > 0 && (!d_diag || !d_out)))
        return HVMS_ERR_INVALID_ARG;
    Cfg c;
    const int st = resolve(opt, false, c);
    if (st)
        return st;
    if (count == 0)
        return HVMS_OK;
    return hip_status(launch_corank_list(d_a, m, d_b, k, d_diag, count, d_out, c.co,
                                         (hipStream_t)stream));
}

int64_t hvms_segmented_workspace_bytes(int64_t n_total, int64_t nseg, int64_t max_seg,
                                       int32_t pairs, const hvms_options *opt)
{
    if (n_total < 0 || nseg < 0)
        return HVMS_ERR_INVALID_ARG;
    Cfg c;
    const int st = resolve(opt, pairs != 0, c);
    if (st)
        return st;
    if (nseg == 0)
        return 0;
    return seg_layout(n_total, nseg, c.R, c.NT, c.TM, pairs != 0, c.ways).total;
}

static int run_segmented(const int32_t *kin, const int32_t *vin, int32_t *kout, int32_t *vout,
                         const int64_t *off, int64_t nseg, int64_t n_total, int64_t max_seg,
                         void *ws, size_t ws_bytes, void *stream, const hvms_options *opt)
{
    const bool pairs = vin != nullptr;
    if (nseg < 0 || n_total < 0 || (nseg > 0 && !off) || nseg >= (1ll << 31))
        return HVMS_ERR_INVALID_ARG;
    if (n_total > 0 && (!kin || !kout || (pairs && (!vin || !vout))))
        return HVMS_ERR_INVALID_ARG;
    Cfg c;
    int st = resolve(opt, pairs, c);
    if (st)
        return st;
    if (!segmented_supported(c.R, c.NT, pairs))
        return HVMS_ERR_UNSUPPORTED;
    if (nseg == 0 || n_total == 0)
        return HVMS_OK;
    // the merge passes move 16-byte chunks of the output and scratch arrays
    if (((uintptr_t)kout & 15) || (pairs && ((uintptr_t)vout & 15)))
        return HVMS_ERR_INVALID_ARG;
    st = check_ws(ws, ws_bytes, seg_layout(n_total, nseg, c.R, c.NT, c.TM, pairs, c.ways).total);
    if (st)
        return st;
    const int64_t tile = (int64_t)c.R * c.NT;
    SegArgs a;
    a.kin = kin;
    a.vin = vin;
    a.kout = kout;
    a.vout = vout;
    a.off = off;
    a.nseg = nseg;
    a.n_total = n_total;
    // a negative max_seg: no bound known, enqueue the passes a segment of
    // all n_total keys would need (passes with no tiles cost a few empty
    // launches)
    const int64_t bound = max_seg < 0 ? n_total : max_seg;
    const int levels = bound > tile ? ilog2_exact((bound + tile - 1) / tile) : 0;
    // four-way: one launch per two merge levels (a segment with an odd
    // count merges its last level two-way)
    a.ways = c.ways;
    a.passes = c.ways == 4 ? (levels + 1) / 2 : levels;
    a.R = c.R;
    a.NT = c.NT;
    a.K = c.K;
    a.TM = c.TM;
    if (c.variant == 4)
        return HVMS_ERR_UNSUPPORTED;
    a.variant = c.variant;
    a.occupancy = c.occupancy;
    a.co = c.co;
    a.ws = ws;
    if (a.passes > 0 && n_total < 16)
        return HVMS_ERR_INVALID_ARG;
    return hip_status(launch_segmented(a, (hipStream_t)stream));
}

int hvms_segmented_status(const void *d_ws, int64_t *d_status, void *stream)
{
    if (!d_ws || !d_status || ((uintptr_t)d_ws & 255))
        return HVMS_ERR_INVALID_ARG;
    return hip_status(launch_seg_status(d_ws, d_status, (hipStream_t)stream));
}

int hvms_segmented_sort_i32(const int32_t *d_in, int32_t *d_out, const int64_t *d_offsets,
                            int64_t nseg, int64_t n_total, int64_t max_seg, void *d_ws,
                            size_t ws_bytes, void *stream, const hvms_options *opt)
{
    if (nseg > 0 && n_total > 0 && (!d_in || !d_out))
        return HVMS_ERR_INVALID_ARG;
    return run_segmented(d_in, nullptr, d_out, nullptr, d_offsets, nseg, n_total, max_seg, d_ws,
                         ws_bytes, stream, opt);
}

int hvms_segmented_sort_pairs_i32(const int32_t *d_keys_in, const int32_t *d_vals_in,
                                  int32_t *d_keys_out, int32_t *d_vals_out,
                                  const int64_t *d_offsets, int64_t nseg, int64_t n_total,
                                  int64_t max_seg, void *d_ws, size_t ws_bytes, void *stream,
                                  const hvms_options *opt)
{
    if (nseg > 0 && n_total > 0 && (!d_keys_in || !d_vals_in || !d_keys_out || !d_vals_out))
        return HVMS_ERR_INVALID_ARG;
    return run_segmented(d_keys_in, d_vals_in, d_keys_out, d_vals_out, d_offsets, nseg, n_total,
                         max_seg, d_ws, ws_bytes, stream, opt);
}

}  // extern "C"
