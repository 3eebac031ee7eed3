// Internal launcher interface between the C ABI (abi.hip) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hvms {

// abi.hip: the hipError_t reported by hvms_last_hip_error (thread-local)
void set_last_hip_error(int e);

// What happens to elements at the boundary of a sort: as they are first
// loaded (block stage) and as they are finally stored (last launch).
//
// Key map: an order-preserving map of another key type onto signed order,
// its own inverse.  32-bit keys: key ^ (((key >> 31) & fm) | um); uint32:
// um = sign bit; float32: fm = 0x7fffffff (IEEE 754 totalOrder of the bit
// patterns); int32: both 0 (identity).  Pair elements map their key the
// same way.  64-bit keys are pair elements (high word = key, low word =
// value with its sign bit flipped, see common.h), and the map of the whole
// 64-bit word is x ^ (((x >> 63) & (fm:fl)) | (um:0)): uint64 um = sign bit,
// float64 fm = 0x7fffffff and fl = 0xffffffff.
//
// packed: the array on that side holds 64-bit elements at the key pointer
// (an int64 / uint64 / float64 key array) instead of separate key and value
// int32 arrays; the sort's intermediate buffers stay split.
// iota (input side, pairs): each element's value is its index in the input;
// no value array is read (a stable sort by key).
struct KeyMap {
    int32_t um = 0, fm = 0, fl = 0;
    bool packed = false, iota = false;
};

struct CorankOpts {
    int mode;
    int radius_log2;
    const float *cdf;
    unsigned long long *stats;
    const float *table = nullptr;  // learned mode: the model sampled (cdf_lookup)
};

// mlp.hip: the model sampled at 2^16 + 1 points (HVMS_CDF_TABLE_BYTES)
constexpr int64_t kCdfTableBytes = ((int64_t)((1 << 16) + 1) * 4 + 255) & ~(int64_t)255;
hipError_t launch_cdf_table(const float *params, float *table, hipStream_t s);

// block_sort.hip
bool block_sort_supported(int R, int NT, bool pairs);
hipError_t launch_block_sort(int R, int NT, bool pairs, const int32_t *kin, const int32_t *vin,
                             int32_t *kout, int32_t *vout, int64_t n, int wave_levels,
                             int lds_levels, bool blocked, hipStream_t s, int net = 0,
                             KeyMap xin = {}, KeyMap xout = {});

// payload.hip: dst[i] = src[idx[i]] for 64-bit payloads
hipError_t launch_gather_u64(const int32_t *idx, const uint64_t *src, uint64_t *dst, int64_t n,
                             hipStream_t s);

// merge.hip
bool merge_tile_supported(int tm, bool pairs);
hipError_t launch_pass_corank(bool pairs, const int32_t *kin, const int32_t *vin, int64_t n,
                              int64_t run, int64_t tm, int64_t *cr, const CorankOpts &o,
                              hipStream_t s);
// variant: 0 default (= 2), 1 one tile per workgroup, 2 persistent pipelined,
// 3 persistent pipelined with XCD-grouped tiles; occupancy: workgroups per CU
// of the persistent grid (0 = as many as fit).
hipError_t launch_merge_pass(int tm, bool pairs, const int32_t *kin, const int32_t *vin,
                             int32_t *kout, int32_t *vout, int64_t n, int64_t run,
                             const int64_t *cr, int variant, int occupancy, hipStream_t s,
                             KeyMap xout = {});
int device_cus();

// merge4.hip: four-way passes (co-rank records by selection in the four
// runs of each group, pipelined merge); rec: one record per tile
// (merge4_record_bytes) with room for two more
bool merge4_supported(int tm, bool pairs);
size_t merge4_record_bytes();
hipError_t launch_merge4_corank(int tm, bool pairs, const int32_t *kin, const int32_t *vin,
                                int64_t n, int64_t run, void *rec, const CorankOpts &o,
                                hipStream_t s);
hipError_t launch_merge4_pass(int tm, bool pairs, const int32_t *kin, const int32_t *vin,
                              int32_t *kout, int32_t *vout, int64_t n, int64_t run,
                              const void *rec, int occupancy, hipStream_t s, KeyMap xout = {});
// segmented four-way pass over the four-way tiles of map (count read from
// the control block): co-ranks and records, then the merge
struct SegMap;
hipError_t launch_seg_merge4(int tm, bool pairs, const SegMap &map, int64_t run, void *rec,
                             int64_t *obase, int64_t max_tiles, int64_t n_total,
                             unsigned long long *stats, int occupancy, hipStream_t s);
hipError_t launch_corank_list(const int32_t *a, int64_t m, const int32_t *b, int64_t k,
                              const int64_t *diag, int64_t count, int64_t *out,
                              const CorankOpts &o, hipStream_t s);

// ablation.hip: one in-register merge level of sorted runs of 2^x_log2 keys
hipError_t launch_merge_runs(const int32_t *in, int32_t *out, int64_t n, int x_log2, int form,
                             int reps, hipStream_t s);

constexpr int ilog2_const(int x) { return x <= 1 ? 0 : 1 + ilog2_const(x / 2); }

inline int ceil_log2_host(int64_t x)
{
    int l = 0;
    while (((int64_t)1 << l) < x)
        ++l;
    return l;
}

// segmented.hip
struct SegLayout {
    int64_t ctrl, pieces, fulls, tiles, cr, rec, obase, passes, table, scr_k, scr_v, total,
        max_tiles,
        max_pieces, max_full, max_half;
};
SegLayout seg_layout(int64_t n_total, int64_t nseg, int R, int NT, int TM, bool pairs,
                     int ways = 2);

struct SegArgs {
    const int32_t *kin, *vin;  // vin == nullptr: keys only
    int32_t *kout, *vout;
    const int64_t *off;
    int64_t nseg, n_total;
    int passes;                // merge launches the largest segment needs
    int ways;                  // 2: two-way passes; 4: four-way (two levels per launch)
    int R, NT, K, TM, variant, occupancy;
    CorankOpts co;
    void *ws;
};
bool segmented_supported(int R, int NT, bool pairs);
hipError_t launch_segmented(const SegArgs &a, hipStream_t s);
// the status words of the last segmented call on workspace ws
hipError_t launch_seg_status(const void *ws, int64_t *out, hipStream_t s);

}  // namespace hvms
