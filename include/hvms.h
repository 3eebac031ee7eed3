/*
 * hvms.h -- C ABI of the MI355X (gfx950) hybrid vectorized merge sort.
 *
 * The library implements the hot path of "A Hybrid Vectorized Merge Sort on
 * ARM NEON" (arXiv 2409.03970) as HIP kernels: a per-wavefront register sort
 * (column sort by a few-comparator network, Sec. 2.3; cross-lane bitonic
 * merges, Sec. 2.4), LDS-staged block merges, and global merge passes whose
 * work is split at merge-path co-ranks (the load-balanced partitioning of the
 * parallel merge, Sec. 2.1).
 *
 * Conventions shared by every entry point:
 *  - All array pointers are DEVICE pointers owned by the caller.  The library
 *    never allocates device memory; scratch space comes from a caller-owned
 *    workspace whose size the matching *_workspace_bytes call returns.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    work is enqueued on it asynchronously; nothing synchronises the host.
 *  - Keys are signed 32-bit integers sorted ascending.  Pairs are ordered
 *    lexicographically by (key, value), both signed, which equals a stable
 *    sort by key when the values are the original indices.
 *  - Input and output may be the same array (in-place sort); otherwise they
 *    must not overlap each other or the workspace.
 *  - Every call returns an hvms status.  Argument errors are found on the
 *    host before anything is enqueued; HVMS_ERR_HIP reports a failed launch
 *    (hvms_last_hip_error() gives the hipError_t).  Faults inside kernels
 *    surface at the caller's next synchronisation of the stream.
 *  - Calls are re-entrant as long as concurrent calls use distinct workspaces.
 */
#ifndef HVMS_H
#define HVMS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    HVMS_OK = 0,
    HVMS_ERR_INVALID_ARG = -1, /* null pointer with n > 0, n < 0, bad option   */
    HVMS_ERR_WORKSPACE = -2,   /* workspace null, too small or misaligned      */
    HVMS_ERR_HIP = -3,         /* a HIP runtime call or kernel launch failed   */
    HVMS_ERR_UNSUPPORTED = -4, /* a tuning value the build has no kernel for   */
    HVMS_ERR_TOO_LARGE = -5    /* input beyond a fixed-size entry point's limit */
};

/* Co-rank search modes for the two-way merge passes (a four-way pass
 * selects its co-ranks in the four runs directly, in every mode). */
enum {
    HVMS_CORANK_BINARY = 0,  /* plain binary search on the merge path          */
    HVMS_CORANK_LEARNED = 1, /* CDF-model prediction + exact bounded search     */
    HVMS_CORANK_LINEAR = 2   /* d*|A|/(|A|+|B|) prediction + the same search    */
};

/*
 * Tuning and mode options.  A NULL pointer, or 0 in a field, selects the
 * built-in default for that field.
 *   keys_per_lane   R, keys each lane sorts in VGPRs: 8, 16 or 32 (Sec. 2.2
 *                   picks 16 registers for NEON; here R is a VGPR budget);
 *                   4 for key sorts (the smallest row of Table 2).
 *   block_threads   threads per block-sort workgroup: 256, 512 or 1024.  The
 *                   block tile is keys_per_lane * block_threads keys.
 *   wave_levels     cross-lane merge levels inside a wavefront, 1..6, stored
 *                   as value+1 (so 0 keeps the default); levels beyond it up
 *                   to the block tile are merged in LDS.
 *   merge_tile      keys per workgroup in a global merge pass: 2048..16384.
 *   corank_mode     HVMS_CORANK_*.
 *   cdf_params      device pointer to HVMS_CDF_PARAMS floats (learned mode).
 *   radius_log2     learned/linear mode: the bounded search first brackets
 *                   the prediction with +-2^radius_log2 and falls back to
 *                   binary search when the co-rank lies outside (default 12).
 *                   A co-rank whose feasible range is at most 8 brackets
 *                   (8 * 2^radius_log2 positions) takes plain binary search:
 *                   there the prediction would save no probes.
 *   stats           optional device array of HVMS_STATS_WORDS uint64 counters
 *                   the co-rank kernels add to (see HVMS_STAT_*), or NULL.
 *   merge_variant   global merge kernel: 0 default, 1 one tile per workgroup,
 *                   2 persistent with the next tile prefetched during the
 *                   merge, 3 as 2 with each XCD walking contiguous tiles,
 *                   4 as 2 with each thread's share merged by the bitonic
 *                   network in registers instead of serially (plain key
 *                   sorts only; the two mergers of Table 3).
 *   merge_occupancy workgroups per CU in the persistent grid (0 = all that fit).
 *   merge_ways      2: two-way merge passes (one merge level per pass); 4:
 *                   four-way passes that do two levels per trip through HBM
 *                   (an odd level count adds one two-way pass first).
 *   column_network  16-input column network (keys, keys_per_lane 16 only):
 *                   0 the 60-comparator network, 1 Batcher odd-even (63),
 *                   2 bitonic (80) -- the comparison of Table 1 / Table 2.
 *   events/n_events optional caller-owned hipEvent_t handles for tracing: a
 *                   sort records events[0]/[1] around its block-sort kernel
 *                   and events[2+2p]/[3+2p] around the merge kernel of pass p
 *                   (two-way passes first, then four-way passes)
 *                   (as far as n_events reaches), on the call's stream.
 */
typedef struct hvms_options {
    int32_t keys_per_lane;
    int32_t block_threads;
    int32_t wave_levels;
    int32_t merge_tile;
    int32_t corank_mode;
    int32_t radius_log2;
    const float *cdf_params;
    unsigned long long *stats;
    void *const *events;
    int32_t n_events;
    int32_t merge_variant;
    int32_t merge_occupancy;
    int32_t column_network;
    int32_t merge_ways;
} hvms_options;

enum {
    HVMS_STAT_CORANKS = 0,   /* co-ranks computed                            */
    HVMS_STAT_PROBES = 1,    /* dependent probe pairs read from memory (a
                              * four-way co-rank: its rounds of reads)      */
    HVMS_STAT_FALLBACKS = 2, /* bounded searches that fell back to binary    */
    HVMS_STAT_ABS_ERR = 3,   /* sum of |prediction - co-rank|                */
    HVMS_STAT_MAX_ERR = 4,   /* max |prediction - co-rank|                   */
    HVMS_STAT_PREDICTED = 5, /* co-ranks that used a prediction (learned or
                              * linear mode and more than 3 candidates);
                              * words 2-4 and the error histogram count these */
    /* 64 words: co-ranks by probe pairs read, bin p = p probes (63 = 63 or
     * more); every co-rank of every mode lands in one bin */
    HVMS_STAT_PROBE_HIST = 8,
    /* 64 words: predicted co-ranks by the bit length of
     * |prediction - co-rank|: bin 0 exact, bin b an error in [2^(b-1), 2^b) */
    HVMS_STAT_ERR_HIST = 72,
    HVMS_STATS_WORDS = 136
};

const char *hvms_status_string(int status);
int hvms_last_hip_error(void);

/* ------------------------------------------------------------------ sort */

/* Bytes of workspace hvms_sort_i32 / hvms_sort_pairs_i32 need for n keys
 * (pairs != 0 for key-value sorts).  Returns a negative status on error. */
int64_t hvms_sort_workspace_bytes(int64_t n, int32_t pairs, const hvms_options *opt);

/*
 * Sort n keys: d_out[0..n) = ascending arrangement of d_in[0..n)  (Sec. 2.1).
 *   d_in, d_out   device int32 arrays of n elements (may be equal).
 *   d_ws/ws_bytes workspace, >= hvms_sort_workspace_bytes(n, 0, opt), 256-byte
 *                 aligned.
 * n == 0 is a no-op returning HVMS_OK.
 */
int hvms_sort_i32(const int32_t *d_in, int32_t *d_out, int64_t n, void *d_ws,
                  size_t ws_bytes, void *stream, const hvms_options *opt);

/*
 * hvms_sort_i32 without a workspace, for callers that cannot allocate device
 * memory (code being captured into a HIP graph, serving loops, harnesses that
 * forbid allocation).  Same arguments, result and errors as hvms_sort_i32,
 * minus d_ws / ws_bytes: the scratch lives in one fixed device array of the
 * library (HVMS_SORT_NOALLOC_SCRATCH_BYTES, held on every GPU the library
 * runs on until the process ends).  The call allocates nothing and calls no
 * allocating library routine; the first call on a device looks up that
 * device's copy of the array (hipGetSymbolAddress, not a stream operation).
 *   n            0 <= n <= HVMS_SORT_NOALLOC_MAX_KEYS; a larger n, or options
 *                whose scratch exceeds the array, return HVMS_ERR_TOO_LARGE
 *                before anything is enqueued.
 * Every call on one GPU shares that GPU's array: calls that overlap in time
 * on one GPU (other streams, other host threads) race and corrupt each
 * other; serialise them, e.g. on one stream.  The array keeps whatever the
 * last call left; the sort needs nothing in it cleared.
 */
#define HVMS_SORT_NOALLOC_MAX_KEYS (1 << 22)
#define HVMS_SORT_NOALLOC_SCRATCH_BYTES (17u << 20)
int hvms_sort_i32_noalloc(const int32_t *d_in, int32_t *d_out, int64_t n, void *stream,
                          const hvms_options *opt);

/*
 * Sort n (key, value) pairs: the same merge sort (Sec. 2.1-2.4) with each
 * value carried beside its key.  The paper sorts keys alone; here every
 * comparison is on (key, value), both signed int32, lexicographically, the
 * one order that a comparator network meets bit-exactly (it equals a stable
 * sort by key when the values are the input positions).
 *   d_keys_in, d_vals_in    device int32 arrays of n elements.
 *   d_keys_out, d_vals_out  device int32 arrays of n elements; each may be
 *                           the matching input (in place).
 *   d_ws/ws_bytes           workspace, >= hvms_sort_workspace_bytes(n, 1, opt),
 *                           256-byte aligned.
 * n == 0 is a no-op.  Errors as hvms_sort_i32.
 */
int hvms_sort_pairs_i32(const int32_t *d_keys_in, const int32_t *d_vals_in,
                        int32_t *d_keys_out, int32_t *d_vals_out, int64_t n,
                        void *d_ws, size_t ws_bytes, void *stream,
                        const hvms_options *opt);

/*
 * Other 32-bit key types (Sec. 2.2 works with 32-bit integers and presents
 * them as one choice of key): the same sort with an order-preserving bit map of the keys onto
 * int32 order applied as the keys are first loaded and undone as they are
 * finally stored, so no pass over memory is added.
 *   hvms_sort_u32:  unsigned order.
 *   hvms_sort_f32:  IEEE 754 totalOrder of the bit patterns: -NaN < -inf <
 *                   ... < -0 < +0 < ... < +inf < +NaN, NaNs of one sign by
 *                   payload (larger payload further from zero); every bit
 *                   pattern is preserved.
 *   *_pairs_*:      (key, value) pairs, lexicographic with signed int32
 *                   values, as hvms_sort_pairs_i32.
 * Arguments, workspace (hvms_sort_workspace_bytes with the same pairs flag),
 * aliasing and errors as hvms_sort_i32 / hvms_sort_pairs_i32.
 */
int hvms_sort_u32(const uint32_t *d_in, uint32_t *d_out, int64_t n, void *d_ws,
                  size_t ws_bytes, void *stream, const hvms_options *opt);
int hvms_sort_f32(const float *d_in, float *d_out, int64_t n, void *d_ws,
                  size_t ws_bytes, void *stream, const hvms_options *opt);
int hvms_sort_pairs_u32(const uint32_t *d_keys_in, const int32_t *d_vals_in,
                        uint32_t *d_keys_out, int32_t *d_vals_out, int64_t n,
                        void *d_ws, size_t ws_bytes, void *stream,
                        const hvms_options *opt);
int hvms_sort_pairs_f32(const float *d_keys_in, const int32_t *d_vals_in,
                        float *d_keys_out, int32_t *d_vals_out, int64_t n,
                        void *d_ws, size_t ws_bytes, void *stream,
                        const hvms_options *opt);

/*
 * 64-bit keys: the merge sort of Sec. 2.1-2.4 over 64-bit elements (the
 * paper's 32-bit integers widened; its comparator of Fig. 3 compares whole
 * elements whatever their width).  Each key is handled
 * as one 64-bit element: the key-value machinery of hvms_sort_pairs_i32 orders
 * (high word, low word) lexicographically, and a 64-bit key in that form
 * (low word with its sign bit flipped) compares exactly as the signed 64-bit
 * integer, so the same kernels sort it.  The block stage reads the packed
 * array and the last launch writes it; the passes in between use split
 * buffers in the workspace.
 *   hvms_sort_i64:  signed order.
 *   hvms_sort_u64:  unsigned order.
 *   hvms_sort_f64:  IEEE 754 totalOrder of the bit patterns (as
 *                   hvms_sort_f32, for binary64); every bit pattern is
 *                   preserved.
 *   d_in, d_out     device arrays of n 64-bit elements, 8-byte aligned (else
 *                   HVMS_ERR_INVALID_ARG); they may be equal.  An output that
 *                   is 16-byte aligned takes the fastest path.
 *   d_ws/ws_bytes   workspace, >= hvms_sort64_workspace_bytes(n, opt) (16 bytes
 *                   per key plus co-ranks once n exceeds one block tile),
 *                   256-byte aligned.
 * Tuning values are those of hvms_sort_pairs_i32 (merge_variant 4 is not
 * available).  n == 0 is a no-op.
 */
int64_t hvms_sort64_workspace_bytes(int64_t n, const hvms_options *opt);
int hvms_sort_i64(const int64_t *d_in, int64_t *d_out, int64_t n, void *d_ws,
                  size_t ws_bytes, void *stream, const hvms_options *opt);
int hvms_sort_u64(const uint64_t *d_in, uint64_t *d_out, int64_t n, void *d_ws,
                  size_t ws_bytes, void *stream, const hvms_options *opt);
int hvms_sort_f64(const double *d_in, double *d_out, int64_t n, void *d_ws,
                  size_t ws_bytes, void *stream, const hvms_options *opt);

/*
 * 64-bit payloads: a stable sort of int32 keys (the merge sort of Sec. 2.1-2.4
 * on (key, input index) pairs) carrying one 64-bit value each
 * (any 8-byte type: int64, uint64, double, a pointer).  d_keys_out is the
 * ascending arrangement of d_keys_in; d_vals_out[i] is the payload that
 * came with d_keys_out[i]; keys that are equal keep their input order.  The
 * keys are sorted together with their input indices by the key-value sort
 * (indices made in the block stage, never read from memory), then one pass
 * moves the payloads: d_vals_out[i] = d_vals_in[index[i]].
 *   d_keys_in/out   device int32 arrays of n elements (may be equal).
 *   d_vals_in/out   device arrays of n 64-bit elements, 8-byte aligned, not
 *                   overlapping (else HVMS_ERR_INVALID_ARG).
 *   n               0 <= n <= 2^31 - 1 (indices are int32).
 *   d_ws/ws_bytes   workspace, >= hvms_sort_by_key_workspace_bytes(n, opt)
 *                   (4 bytes per key for the indices plus the key-value
 *                   sort's workspace), 256-byte aligned.
 * Tuning values are those of hvms_sort_pairs_i32.  n == 0 is a no-op.
 */
int64_t hvms_sort_by_key_workspace_bytes(int64_t n, const hvms_options *opt);
int hvms_sort_by_key_i32_p64(const int32_t *d_keys_in, const uint64_t *d_vals_in,
                             int32_t *d_keys_out, uint64_t *d_vals_out, int64_t n,
                             void *d_ws, size_t ws_bytes, void *stream,
                             const hvms_options *opt);

/*
 * Sort every run of 2^run_log2 consecutive keys independently (the last run
 * may be shorter): the block stage alone, i.e. the sorted runs of X keys that
 * Table 2 times, with X = 2^run_log2.  run_log2 must lie in
 * [log2(keys_per_lane), log2(block tile)].  Uses no workspace.
 */
int hvms_sort_runs_i32(const int32_t *d_in, int32_t *d_out, int64_t n, int32_t run_log2,
                       void *stream, const hvms_options *opt);

/*
 * The two in-register mergers of Table 3 (Sec. 2.4), for comparing them on
 * the GPU: d_in holds consecutive sorted runs of X = 2^x_log2 keys (X = 8,
 * 16 or 32); d_out receives each adjacent pair merged into one sorted run of
 * 2X.  form 0, hybrid: one run per lane in its X VGPRs, a cross-lane flip
 * stage, then log2(X) half-cleaners inside each lane (the serial part).
 * form 1, vector: the runs spread across lanes (register r of lane l holds
 * key 64r + l of its wave's 64X keys), every stage a lane exchange.  reps >= 1
 * repeats the merge on the registers (the result is that of one merge), so
 * a timed launch measures the merging, not the memory traffic.
 *   n        a multiple of 256 * X (four waves of 64 X keys per workgroup).
 *   d_in/out device int32 arrays of n keys, 16-byte aligned (may be equal).
 */
int hvms_merge_runs_i32(const int32_t *d_in, int32_t *d_out, int64_t n, int32_t x_log2,
                        int32_t form, int32_t reps, void *stream);

/*
 * One global merge pass: d_in holds consecutive sorted runs of run_len keys
 * (the last may be shorter); d_out receives the merge of each pair of runs,
 * i.e. sorted runs of 2*run_len.  run_len must be a power of two >= the merge
 * tile.  d_in and d_out must not overlap.  Workspace as returned by
 * hvms_merge_workspace_bytes.
 */
int64_t hvms_merge_workspace_bytes(int64_t n, int64_t run_len, const hvms_options *opt);
int hvms_merge_pass_i32(const int32_t *d_in, int32_t *d_out, int64_t n, int64_t run_len,
                        void *d_ws, size_t ws_bytes, void *stream,
                        const hvms_options *opt);

/*
 * Merge-path co-ranks (Sec. 2.1 partitioning): for each diagonal d_diag[q]
 * (0 <= d <= m + k) of the merge of sorted d_a[0..m) and d_b[0..k),
 * d_out[q] = number of elements of A among the first d outputs of the merge
 * that takes A first on ties.  The result is unique; opt->corank_mode only
 * changes how it is searched.
 */
int hvms_corank_i32(const int32_t *d_a, int64_t m, const int32_t *d_b, int64_t k,
                    const int64_t *d_diag, int64_t count, int64_t *d_out, void *stream,
                    const hvms_options *opt);

/* ------------------------------------------------------------- segmented */

/*
 * Segmented sort (batched form of the sort, each segment sorted as in Sec.
 * 2.1): for every s in [0, nseg) write the ascending arrangement of
 * d_in[off[s] .. off[s+1]) to d_out at the same positions.
 *   d_offsets  DEVICE array of nseg+1 nondecreasing int64 offsets.
 *   n_total    must equal off[nseg] (the arrays hold at least n_total keys).
 *   max_seg    host-side upper bound on the largest segment, or negative if
 *              none is known.  It fixes how many merge launches are enqueued:
 *              L = ceil(log2(ceil(max_seg / block tile))) merge levels, one
 *              launch per level (two-way) or per two levels (four-way), from
 *              n_total when negative (a few empty launches more).  A segment
 *              larger than the bound is NOT fully sorted: it comes out as a
 *              permutation of its input made of sorted runs of block tile *
 *              2^(levels merged) keys, and it is counted in status word 0
 *              (hvms_segmented_status).
 *   d_out      16-byte aligned (pairs: d_vals_out too).
 * Elements outside [off[0], off[nseg]) are not written.  A segment whose
 * offsets fall outside [0, n_total] or decrease is treated as empty and
 * counted in status word 1.  If the sizes add up to more than n_total
 * allows, nothing is sorted or written and status word 2 is set.
 * The block stage takes two launches: one sorts the full block tiles of long
 * segments and, padded, every segment or ragged rest of more than a quarter
 * of a tile (one or two to a tile); a persistent one sorts the shorter ones,
 * packed into tiles it pulls from an atomic ticket.  Larger segments add a
 * co-rank and a merge launch per merge launch.  The call allocates and
 * synchronises nothing, so it can be captured into a hipGraph.  Workspace:
 * hvms_segmented_workspace_bytes.
 */
int64_t hvms_segmented_workspace_bytes(int64_t n_total, int64_t nseg, int64_t max_seg,
                                       int32_t pairs, const hvms_options *opt);
int hvms_segmented_sort_i32(const int32_t *d_in, int32_t *d_out, const int64_t *d_offsets,
                            int64_t nseg, int64_t n_total, int64_t max_seg, void *d_ws,
                            size_t ws_bytes, void *stream, const hvms_options *opt);
int hvms_segmented_sort_pairs_i32(const int32_t *d_keys_in, const int32_t *d_vals_in,
                                  int32_t *d_keys_out, int32_t *d_vals_out,
                                  const int64_t *d_offsets, int64_t nseg, int64_t n_total,
                                  int64_t max_seg, void *d_ws, size_t ws_bytes,
                                  void *stream, const hvms_options *opt);

/*
 * Status of the last segmented call that used workspace d_ws (the same
 * workspace pointer, after that call): enqueues on `stream` a copy of three
 * int64 words to device memory d_status[0..3):
 *   [0] segments larger than the max_seg bound allowed (left as sorted runs);
 *   [1] segments skipped for invalid offsets;
 *   [2] 1 if the offsets were inconsistent with n_total (nothing was sorted).
 * All zero means every segment was sorted.  The words belong to the last
 * call on that workspace, so read them before the workspace is reused.
 * Returns HVMS_ERR_INVALID_ARG for a null or misaligned pointer.
 */
int hvms_segmented_status(const void *d_ws, int64_t *d_status, void *stream);

/* -------------------------------------------------------- learned co-rank */

/* The CDF model F(x) ~ P(key <= x): an fp32 perceptron 1 -> 32 -> 32 -> 1
 * with ReLU, input x = (key + 2^31) / 2^32.  Parameter layout (floats):
 * W1[32] b1[32] W2[32][32] (row = output unit) b2[32] W3[32] b3[1]. */
#define HVMS_CDF_PARAMS 1153

/* HVMS_CDF_PARAMS as a call, for bindings that do not read the header. */
int64_t hvms_cdf_param_count(void);

/* y[i] = F(x[i]) for i < b.  Device arrays. */
int hvms_cdf_forward(const float *d_params, const float *d_x, float *d_y, int64_t b,
                     void *stream);

/* Mean squared error of F on (x, t) and its gradient: d_grad[HVMS_CDF_PARAMS],
 * d_loss[1].  Reductions are deterministic (fixed order), so reruns are
 * bitwise identical.  Workspace: hvms_cdf_workspace_bytes(b). */
int64_t hvms_cdf_workspace_bytes(int64_t b);
int hvms_cdf_backward(const float *d_params, const float *d_x, const float *d_t,
                      float *d_grad, float *d_loss, int64_t b, void *d_ws,
                      size_t ws_bytes, void *stream);

/* One Adam step (Kingma and Ba 2015): d_m, d_v are the moment buffers,
 * `step` counts from 1. */
int hvms_cdf_adam_step(float *d_params, float *d_m, float *d_v, const float *d_grad,
                       int32_t step, float lr, float beta1, float beta2, float eps,
                       void *stream);

/* Training sample: d_out[k] = d_keys[SplitMix64(seed, k) mod n] for k < m,
 * where SplitMix64(seed, k) is output k (from 0) of Steele, Lea and Flood's
 * SplitMix64 generator seeded with `seed` (a sample with replacement). */
int hvms_cdf_sample_i32(const int32_t *d_keys, int64_t n, int64_t m, uint64_t seed,
                        int32_t *d_out, void *stream);

/*
 * Train the model on a sorted sample: d_sorted[0..m) ascending keys; the
 * target of the i-th key is i/m.  Runs `steps` Adam steps (lr, betas 0.9 /
 * 0.999, eps 1e-8) on minibatches of `batch` sample positions drawn with
 * SplitMix64 from `seed`.  d_params holds the initial parameters on entry and
 * the trained ones on exit; d_m, d_v are zeroed by the call.
 */
int64_t hvms_cdf_train_workspace_bytes(int64_t batch);
int hvms_cdf_train(float *d_params, float *d_m, float *d_v, const int32_t *d_sorted,
                   int64_t m, int64_t batch, int32_t steps, float lr, uint64_t seed,
                   void *d_ws, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* HVMS_H */
