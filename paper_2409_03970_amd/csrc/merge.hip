// Global merge passes (steps a5-a6): merge-path co-ranks, then a pass that
// streams pairs of sorted runs through LDS.
//
// Pass with run length L: output tile g covers [g*TM, (g+1)*TM) of the
// result; it lies inside one merge pair (TM divides 2L).  Its first output is
// diagonal d = g*TM - pair_base of that pair, and the tile needs the co-rank
// of d and of the next tile's diagonal (the parallel merge's segmentation
// points, Sec. 2.1).  A co-rank kernel computes them for all tiles; the merge
// kernel then loads exactly its A window and B window (TM elements together)
// into LDS, each thread finds its own co-rank inside LDS and merges VT
// elements serially, and the tile leaves through LDS in coalesced order.
#include "hvms_internal.h"
#include "merge_common.h"

namespace hvms {

// Co-ranks of the first diagonal of every output tile of a merge pass.
// In learned mode the block first takes the model's CDF (table lookup, or
// the network without a table) at the four run endpoints of each of its
// pairs (at most 64: a pair has 2*run/tm >= 1 tiles), one per thread and
// round, so every co-rank of a pair shares them.
template <typename T>
__global__ __launch_bounds__(64) void pass_corank_kernel(PlainMap map, int64_t run, int64_t tm,
                                                          int64_t *__restrict__ cr, CorankCtl c)
{
    __shared__ float4 F[256];
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // (only where the runs are long enough for a prediction: see find_corank)
    if (c.mode == 1 && run > ((int64_t)8 << c.radius_log2)) {  // block-uniform
        const int64_t q0 = (int64_t)blockIdx.x * blockDim.x;
        const int64_t qlast = q0 + blockDim.x - 1 < map.ntiles - 1 ? q0 + blockDim.x - 1 : map.ntiles - 1;
        const int64_t p0 = q0 * tm / (2 * run), p1 = qlast * tm / (2 * run);
        const int np = (int)(p1 - p0 + 1);
        for (int e = threadIdx.x; e < 4 * np; e += blockDim.x) {
            const int64_t pb = (p0 + e / 4) * 2 * run;
            const int64_t alen = run < map.n - pb ? run : map.n - pb;
            const int64_t rest = map.n - pb - run;
            const int64_t blen = rest <= 0 ? 0 : (rest < run ? rest : run);
            const int w = e & 3;
            int64_t idx = w == 0 ? pb : w == 1 ? pb + alen - 1 : w == 2 ? pb + run : pb + run + blen - 1;
            if (w >= 2 && blen == 0)
                idx = pb + alen - 1;
            const int32_t key = map.ik[idx];
            ((float *)&F[e / 4])[w] =
                c.table ? cdf_lookup(c.table, key) : cdf_eval(c.cdf, key_to_unit(key));
        }
        __syncthreads();
        c.pair_cdf = F;
        c.pair_first = p0;
    }
    if (q < map.ntiles)
        tile_corank<T>(map, q, run, tm, cr, c);
}

// Co-ranks of arbitrary diagonals of two arrays (keys only).
__global__ __launch_bounds__(256) void corank_list_kernel(const int32_t *__restrict__ a, int64_t m,
                                                          const int32_t *__restrict__ b, int64_t k,
                                                          const int64_t *__restrict__ diag,
                                                          int64_t count, int64_t *__restrict__ out,
                                                          CorankCtl c)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count)
        return;
    const int64_t d = diag[q];
    if (d < 0 || d > m + k) {
        out[q] = -1;
        return;
    }
    auto A = [=](int64_t i) { return a[i]; };
    auto B = [=](int64_t i) { return b[i]; };
    out[q] = find_corank<int32_t>(c, A, B, A, B, m, k, d);
}

// ------------------------------------------------------------ merge pass

template <int NT, int VT, typename T, bool PK = false>
__global__ __launch_bounds__(NT) void merge_pass_kernel(const int32_t *__restrict__ kin,
                                                        const int32_t *__restrict__ vin,
                                                        int32_t *__restrict__ kout,
                                                        int32_t *__restrict__ vout, int64_t n,
                                                        int64_t run, const int64_t *__restrict__ cr,
                                                        KeyMap xout)
{
    constexpr int TM = NT * VT;
    __shared__ T S[TM];
    const int t = threadIdx.x;
    const int64_t g = blockIdx.x;
    const int64_t o0 = g * TM;
    const int64_t o1 = o0 + TM < n ? o0 + TM : n;
    const int64_t pb = o0 & ~(2 * run - 1);
    const int64_t alen = run < n - pb ? run : n - pb;
    const int64_t rest = n - pb - run;
    const int64_t blen = rest <= 0 ? 0 : (rest < run ? rest : run);
    const int64_t d0 = o0 - pb, d1 = o1 - pb;
    // Co-ranks are clamped to their feasible ranges and to i0 <= i1 <= i0 +
    // cnt, so every window below stays inside its run even if the input runs
    // were not sorted (garbage out, never an access out of bounds).
    auto clampc = [&](int64_t i, int64_t d) {
        const int64_t lo = d > blen ? d - blen : 0, hi = d < alen ? d : alen;
        return i < lo ? lo : (i > hi ? hi : i);
    };
    const int64_t i0 = clampc(cr[g], d0);
    int64_t i1 = clampc(d1 == alen + blen ? alen : cr[g + 1], d1);
    i1 = i1 < i0 ? i0 : (i1 > i0 + (d1 - d0) ? i0 + (d1 - d0) : i1);
    const int acnt = (int)(i1 - i0);
    const int cnt = (int)(d1 - d0);
    const int bcnt = cnt - acnt;
    const int64_t j0 = d0 - i0;

    const int64_t abase = pb + i0, bbase = pb + run + j0 - acnt;
#pragma unroll
    for (int k = 0; k < VT; ++k) {
        const int idx = t + NT * k;
        if (idx < cnt)
            S[idx] = load_elem<T>(kin, vin, idx < acnt ? abase + idx : bbase + idx);
    }
    __syncthreads();

    const int diag = t * VT < cnt ? t * VT : cnt;
    const LdsPlain<T> SV{S, 0};
    const int i = lds_corank(SV, acnt, acnt, bcnt, diag);
    T out[VT];
    serial_merge<VT>(SV, acnt, acnt, bcnt, i, diag - i, out);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < VT; ++k)
        S[t * VT + k] = out[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < VT; ++k) {
        const int idx = t + NT * k;
        if (idx < cnt)
            store_elem<T, PK>(kout, vout, o0 + idx, map_elem(S[idx], xout));
    }
}

// ------------------------------------------- persistent, pipelined merge pass

template <int NT, int VT, typename T, bool BIT = false, bool PK = false>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(merge_waves_per_simd<T, VT>())))
void merge_pass_pipe_kernel(PlainMap map, int64_t run, const int64_t *__restrict__ cr,
                            int xcd_group, KeyMap xout)
{
    merge_pipe_body<NT, VT, T, PlainMap, BIT, PK>(map, run, cr, map.n, xcd_group, xout);
}

// ------------------------------------------------------------- launchers

static CorankCtl make_ctl(const CorankOpts &o)
{
    CorankCtl c;
    c.mode = o.mode;
    c.radius_log2 = o.radius_log2;
    c.cdf = o.cdf;
    c.stats = o.stats;
    c.pair_cdf = nullptr;
    c.pair_first = 0;
    c.table = o.table;
    return c;
}

hipError_t launch_pass_corank(bool pairs, const int32_t *kin, const int32_t *vin, int64_t n,
                              int64_t run, int64_t tm, int64_t *cr, const CorankOpts &o,
                              hipStream_t s)
{
    const CorankCtl ctl = make_ctl(o);
    PlainMap map;
    map.ik = kin;
    map.iv = pairs ? vin : nullptr;
    map.ok = nullptr;
    map.ov = nullptr;
    map.n = n;
    map.ntiles = (n + tm - 1) / tm;
    const unsigned blocks = (unsigned)((map.ntiles + 63) / 64);
    if (pairs)
        hipLaunchKernelGGL(pass_corank_kernel<int64_t>, dim3(blocks), dim3(64), 0, s, map, run,
                           tm, cr, ctl);
    else
        hipLaunchKernelGGL(pass_corank_kernel<int32_t>, dim3(blocks), dim3(64), 0, s, map, run,
                           tm, cr, ctl);
    return hipGetLastError();
}

hipError_t launch_corank_list(const int32_t *a, int64_t m, const int32_t *b, int64_t k,
                              const int64_t *diag, int64_t count, int64_t *out,
                              const CorankOpts &o, hipStream_t s)
{
    const unsigned blocks = (unsigned)((count + 255) / 256);
    hipLaunchKernelGGL(corank_list_kernel, dim3(blocks), dim3(256), 0, s, a, m, b, k, diag, count,
                       out, make_ctl(o));
    return hipGetLastError();
}

bool merge_tile_supported(int tm, bool pairs)
{
    return tm == 2048 || tm == 4096 || tm == 8192 || (tm == 16384 && !pairs);
}

template <int NT, int VT, typename T>
static hipError_t launch_mp(const int32_t *kin, const int32_t *vin, int32_t *kout, int32_t *vout,
                            int64_t n, int64_t run, const int64_t *cr, hipStream_t s, KeyMap xout)
{
    const int64_t ntiles = (n + NT * VT - 1) / (NT * VT);
    if constexpr (sizeof(T) == 8) {
        if (xout.packed) {
            hipLaunchKernelGGL((merge_pass_kernel<NT, VT, T, true>), dim3((unsigned)ntiles),
                               dim3(NT), 0, s, kin, vin, kout, vout, n, run, cr, xout);
            return hipGetLastError();
        }
    } else if (xout.packed) {
        return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL((merge_pass_kernel<NT, VT, T>), dim3((unsigned)ntiles), dim3(NT), 0, s,
                       kin, vin, kout, vout, n, run, cr, xout);
    return hipGetLastError();
}

int device_cus()
{
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return 256;
    if (!cus[dev]) {
        int c = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            c <= 0)
            c = 256;
        cus[dev] = c;
    }
    return cus[dev];
}

template <int NT, int VT, typename T, bool BIT = false, bool PK = false>
static hipError_t launch_mpp1(const int32_t *kin, const int32_t *vin, int32_t *kout,
                              int32_t *vout, int64_t n, int64_t run, const int64_t *cr,
                              int occupancy, bool xcd, hipStream_t s, KeyMap xout)
{
    const int64_t ntiles = (n + NT * VT - 1) / (NT * VT);
    int occ = occupancy;
    if (occ <= 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &occ, (const void *)merge_pass_pipe_kernel<NT, VT, T, BIT, PK>, NT, 0) !=
                hipSuccess ||
            occ <= 0)
            occ = 1;
    }
    int64_t grid = (int64_t)device_cus() * occ;
    if (grid > ntiles)
        grid = ntiles;
    if (xcd)
        grid = ((grid + 7) / 8) * 8;
    PlainMap map;
    map.ik = kin;
    map.iv = vin;
    map.ok = kout;
    map.ov = vout;
    map.n = n;
    map.ntiles = ntiles;
    hipLaunchKernelGGL((merge_pass_pipe_kernel<NT, VT, T, BIT, PK>), dim3((unsigned)grid), dim3(NT),
                       0, s, map, run, cr, xcd ? 1 : 0, xout);
    return hipGetLastError();
}

// xout.packed (the last pass of a 64-bit key sort) selects the instance that
// stores packed 64-bit elements
template <int NT, int VT, typename T, bool BIT = false>
static hipError_t launch_mpp(const int32_t *kin, const int32_t *vin, int32_t *kout, int32_t *vout,
                             int64_t n, int64_t run, const int64_t *cr, int occupancy, bool xcd,
                             hipStream_t s, KeyMap xout)
{
    if constexpr (sizeof(T) == 8) {
        if (xout.packed)
            return launch_mpp1<NT, VT, T, BIT, true>(kin, vin, kout, vout, n, run, cr, occupancy,
                                                     xcd, s, xout);
    } else if (xout.packed) {
        return hipErrorInvalidValue;
    }
    return launch_mpp1<NT, VT, T, BIT>(kin, vin, kout, vout, n, run, cr, occupancy, xcd, s, xout);
}

hipError_t launch_merge_pass(int tm, bool pairs, const int32_t *kin, const int32_t *vin,
                             int32_t *kout, int32_t *vout, int64_t n, int64_t run,
                             const int64_t *cr, int variant, int occupancy, hipStream_t s,
                             KeyMap xout)
{
    // The pipelined kernel moves 16-byte chunks: it needs 16-byte aligned
    // arrays and at least 16 elements; anything else takes the simple kernel.
    const bool aligned = ((uintptr_t)kin % 16 == 0) && ((uintptr_t)kout % 16 == 0) &&
                         (!pairs || (((uintptr_t)vin % 16 == 0) &&
                                     (xout.packed || (uintptr_t)vout % 16 == 0)));
    if (variant == 4 && !pairs && aligned && n >= 16) {  // bitonic register merge (keys)
        switch (tm) {
        case 2048:
            return launch_mpp<256, 8, int32_t, true>(kin, vin, kout, vout, n, run, cr, occupancy, false, s, xout);
        case 4096:
            return launch_mpp<256, 16, int32_t, true>(kin, vin, kout, vout, n, run, cr, occupancy, false, s, xout);
        case 8192:
            return launch_mpp<512, 16, int32_t, true>(kin, vin, kout, vout, n, run, cr, occupancy, false, s, xout);
        case 16384:
            return launch_mpp<512, 32, int32_t, true>(kin, vin, kout, vout, n, run, cr, occupancy, false, s, xout);
        }
        return hipErrorInvalidValue;
    }
    if (variant != 1 && aligned && n >= 16) {
        const bool xcd = variant == 3;
        switch (tm) {
        case 2048:
            return pairs ? launch_mpp<256, 8, int64_t>(kin, vin, kout, vout, n, run, cr, occupancy, xcd, s, xout)
                         : launch_mpp<256, 8, int32_t>(kin, vin, kout, vout, n, run, cr, occupancy, xcd, s, xout);
        case 4096:
            return pairs ? launch_mpp<256, 16, int64_t>(kin, vin, kout, vout, n, run, cr, occupancy, xcd, s, xout)
                         : launch_mpp<256, 16, int32_t>(kin, vin, kout, vout, n, run, cr, occupancy, xcd, s, xout);
        case 8192:
            return pairs ? launch_mpp<512, 16, int64_t>(kin, vin, kout, vout, n, run, cr, occupancy, xcd, s, xout)
                         : launch_mpp<512, 16, int32_t>(kin, vin, kout, vout, n, run, cr, occupancy, xcd, s, xout);
        case 16384:
            if (!pairs)
                return launch_mpp<512, 32, int32_t>(kin, vin, kout, vout, n, run, cr, occupancy, xcd, s, xout);
            break;
        }
        return hipErrorInvalidValue;
    }
    switch (tm) {
    case 2048:
        return pairs ? launch_mp<256, 8, int64_t>(kin, vin, kout, vout, n, run, cr, s, xout)
                     : launch_mp<256, 8, int32_t>(kin, vin, kout, vout, n, run, cr, s, xout);
    case 4096:
        return pairs ? launch_mp<256, 16, int64_t>(kin, vin, kout, vout, n, run, cr, s, xout)
                     : launch_mp<256, 16, int32_t>(kin, vin, kout, vout, n, run, cr, s, xout);
    case 8192:
        return pairs ? launch_mp<512, 16, int64_t>(kin, vin, kout, vout, n, run, cr, s, xout)
                     : launch_mp<512, 16, int32_t>(kin, vin, kout, vout, n, run, cr, s, xout);
    case 16384:
        if (!pairs)
            return launch_mp<512, 32, int32_t>(kin, vin, kout, vout, n, run, cr, s, xout);
        break;
    }
    return hipErrorInvalidValue;
}

}  // namespace hvms
