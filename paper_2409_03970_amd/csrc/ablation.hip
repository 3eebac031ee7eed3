// The in-register merge of Table 3 on the GPU: every pair of adjacent sorted
// runs of X keys (X = 8, 16, 32) becomes one sorted run of 2X, in one of the
// two forms the paper compares (Sec. 2.4):
//   hybrid (form 0): the blocked layout of the block stage, lane l holding
//     one run of X consecutive keys in its X VGPRs.  A flip stage pairs lanes
//     l and l ^ 1 (register r with X - 1 - r, by a DPP quad permute), then
//     log2(X) half-cleaners run inside each lane: the serial part.
//   vector (form 1): a striped layout, register r of lane l holding key
//     64 r + l, so a run of 2X keys lies across 2X lanes of one register and
//     all log2(2X) stages are lane exchanges: the flip with lane
//     l ^ (2X - 1), then half-cleaners with lane l ^ d, d = X/2 .. 1 (DPP
//     where a control exists, else ds_swizzle / ds_bpermute).
// Each wave merges 64 X keys; `reps` repeats the merge on the registers (a
// merged run is again two sorted halves, so every repetition is a full
// merge and the result equals one), which makes the in-register work, not
// memory, the cost of a timed launch.
#include "common.h"
#include "hvms.h"
#include "hvms_internal.h"

namespace hvms {

namespace {

// v from lane (lane ^ M), any M < 64
template <int M> __device__ __forceinline__ int32_t lane_xor(int32_t v)
{
    if constexpr (M == 1 || M == 2 || M == 4 || M == 8)
        return xlane32<M>(v);
    else if constexpr (M == 3)
        return __builtin_amdgcn_update_dpp(0, v, 0x1B, 0xF, 0xF, true);   // quad_perm 3,2,1,0
    else if constexpr (M == 7)
        return __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, true);  // row_half_mirror
    else if constexpr (M == 15)
        return __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, true);  // row_mirror
    else if constexpr (M == 16)
        return __builtin_amdgcn_ds_swizzle(v, 0x401F);
    else if constexpr (M == 31)
        return __builtin_amdgcn_ds_swizzle(v, 0x7C1F);
    else
        return __builtin_amdgcn_ds_bpermute((lane_id() ^ M) << 2, v);
}

template <int X, int D>
__device__ __forceinline__ void vector_half_cleaners(int32_t (&v)[X], int lane)
{
    if constexpr (D >= 1) {
        const int32_t sel = keep_selector((lane & D) != 0);
#pragma unroll
        for (int r = 0; r < X; ++r)
            v[r] = keep_sel(v[r], lane_xor<D>(v[r]), sel);
        vector_half_cleaners<X, D / 2>(v, lane);
    }
}

template <int X, int FORM>
__global__ __launch_bounds__(256) void merge_runs_kernel(const int32_t *__restrict__ in,
                                                         int32_t *__restrict__ out, int reps)
{
    const int lane = threadIdx.x & 63;
    const int64_t base = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * (64 * X);
    int32_t v[X];
    if constexpr (FORM == 0) {
#pragma unroll
        for (int q = 0; q < X; q += 4) {
            const int4 c = *(const int4 *)(in + base + (int64_t)X * lane + q);
            v[q] = c.x;
            v[q + 1] = c.y;
            v[q + 2] = c.z;
            v[q + 3] = c.w;
        }
    } else {
#pragma unroll
        for (int r = 0; r < X; ++r)
            v[r] = in[base + 64 * r + lane];
    }
    for (int rep = 0; rep < reps; ++rep) {
        if constexpr (FORM == 0) {
            const int32_t sel = keep_selector((lane & 1) != 0);
            int32_t p[X];
#pragma unroll
            for (int r = 0; r < X; ++r)
                p[r] = xlane32<1>(v[X - 1 - r]);
#pragma unroll
            for (int r = 0; r < X; ++r)
                v[r] = keep_sel(v[r], p[r], sel);
            inlane_half_cleaners<X, X / 2>(v, DirSel<int32_t>(false));
        } else {
            const int32_t sel = keep_selector((lane & X) != 0);
#pragma unroll
            for (int r = 0; r < X; ++r)
                v[r] = keep_sel(v[r], lane_xor<2 * X - 1>(v[r]), sel);
            vector_half_cleaners<X, X / 2>(v, lane);
        }
    }
    if constexpr (FORM == 0) {
#pragma unroll
        for (int q = 0; q < X; q += 4)
            *(int4 *)(out + base + (int64_t)X * lane + q) =
                make_int4(v[q], v[q + 1], v[q + 2], v[q + 3]);
    } else {
#pragma unroll
        for (int r = 0; r < X; ++r)
            out[base + 64 * r + lane] = v[r];
    }
}

template <int X, int FORM>
hipError_t launch_mr(const int32_t *in, int32_t *out, int64_t n, int reps, hipStream_t s)
{
    const int64_t blocks = n / (256 * X);  // four waves of 64 X keys each
    hipLaunchKernelGGL((merge_runs_kernel<X, FORM>), dim3((unsigned)blocks), dim3(256), 0, s, in,
                       out, reps);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_merge_runs(const int32_t *in, int32_t *out, int64_t n, int x_log2, int form,
                             int reps, hipStream_t s)
{
#define HVMS_MR(XX)                                                                   \
    if (x_log2 == ilog2_const(XX))                                                    \
        return form == 0 ? launch_mr<XX, 0>(in, out, n, reps, s)                      \
                         : launch_mr<XX, 1>(in, out, n, reps, s);
    HVMS_MR(8)
    HVMS_MR(16)
    HVMS_MR(32)
#undef HVMS_MR
    return hipErrorInvalidValue;
}

}  // namespace hvms

using namespace hvms;

extern "C" int hvms_merge_runs_i32(const int32_t *d_in, int32_t *d_out, int64_t n,
                                   int32_t x_log2, int32_t form, int32_t reps, void *stream)
{
    if (x_log2 < 3 || x_log2 > 5 || form < 0 || form > 1 || reps < 1 || n < 0)
        return HVMS_ERR_INVALID_ARG;
    if (n % (256LL << x_log2) != 0 || (n > 0 && (!d_in || !d_out)))
        return HVMS_ERR_INVALID_ARG;
    if (((uintptr_t)d_in | (uintptr_t)d_out) & 15)
        return HVMS_ERR_INVALID_ARG;
    if (n == 0)
        return HVMS_OK;
    const hipError_t e = launch_merge_runs(d_in, d_out, n, x_log2, form, reps, (hipStream_t)stream);
    if (e != hipSuccess) {
        set_last_hip_error((int)e);
        return HVMS_ERR_HIP;
    }
    return HVMS_OK;
}
