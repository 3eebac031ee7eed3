// Device building blocks shared by the sort kernels (gfx950, wave64).
//
// Element types: int32_t for keys, and int64_t for (key, value) pairs packed
// as (key << 32) | (value ^ 0x80000000), whose signed 64-bit order is the
// lexicographic (key, value) order with both halves signed.  The pad value
// for ragged tiles is the maximum of the order (INT32_MAX, or the pair
// (INT32_MAX, INT32_MAX)); a real element equal to it is bit-identical, so
// dropping the trailing pads is exact.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hvms_internal.h"
#include "networks.h"

namespace hvms {

template <typename T> struct Traits;
template <> struct Traits<int32_t> {
    static constexpr int32_t kMax = 0x7fffffff;
};
template <> struct Traits<int64_t> {
    static constexpr int64_t kMax = 0x7fffffffffffffffll;
};

__device__ __forceinline__ int64_t pack_pair(int32_t k, int32_t v)
{
    return (int64_t)(((uint64_t)(uint32_t)k << 32) | (uint64_t)((uint32_t)v ^ 0x80000000u));
}
__device__ __forceinline__ int32_t pair_key(int64_t p) { return (int32_t)((uint64_t)p >> 32); }
__device__ __forceinline__ int32_t pair_val(int64_t p)
{
    return (int32_t)((uint32_t)(uint64_t)p ^ 0x80000000u);
}

// Element i of a key array, or of a key/value array pair, as type T.  PK:
// the 64-bit elements sit packed at k (a 64-bit key array; v unused).  IOTA:
// the value is the index i itself (v unused; i < 2^31).
template <typename T, bool PK = false, bool IOTA = false>
__device__ __forceinline__ T load_elem(const int32_t *__restrict__ k,
                                       const int32_t *__restrict__ v, int64_t i)
{
    if constexpr (sizeof(T) == 4)
        return k[i];
    else if constexpr (PK)
        return ((const int64_t *)k)[i];
    else if constexpr (IOTA)
        return pack_pair(k[i], (int32_t)i);
    else
        return pack_pair(k[i], v[i]);
}
template <typename T, bool PK = false>
__device__ __forceinline__ void store_elem(int32_t *__restrict__ k, int32_t *__restrict__ v,
                                           int64_t i, T x)
{
    if constexpr (sizeof(T) == 4) {
        k[i] = x;
    } else if constexpr (PK) {
        ((int64_t *)k)[i] = x;
    } else {
        k[i] = pair_key(x);
        v[i] = pair_val(x);
    }
}

// Buffer resource over `bytes` bytes from p: raw layout (stride 0, no
// format conversion; the gfx9 descriptor's third word).  An access through
// it adds a 32-bit VGPR byte offset, a wave-uniform SGPR offset and an
// immediate to the base, so the unrolled loads and stores of a tile need no
// 64-bit address arithmetic per element.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(const void *p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes,
                                             0x00020000);
}

// One tile's elements through buffer resources: int32 keys, or key/value
// pairs in two int32 arrays (packed 64-bit arrays and index values keep
// load_elem / store_elem).  Offsets are in elements: vo per lane, so
// wave-uniform.
template <typename T> struct TileIO {
    __amdgpu_buffer_rsrc_t k, v;
    __device__ __forceinline__ TileIO(const int32_t *kb, const int32_t *vb, int n)
        : k(raw_rsrc(kb, 4u * (uint32_t)n)), v(raw_rsrc(sizeof(T) == 8 ? vb : kb, 4u * (uint32_t)n))
    {
    }
    __device__ __forceinline__ T load(int vo, int so) const
    {
        const int32_t x = __builtin_amdgcn_raw_buffer_load_b32(k, 4 * vo, 4 * so, 0);
        if constexpr (sizeof(T) == 4)
            return x;
        else
            return pack_pair(x, __builtin_amdgcn_raw_buffer_load_b32(v, 4 * vo, 4 * so, 0));
    }
    __device__ __forceinline__ void store(int vo, int so, T x) const
    {
        if constexpr (sizeof(T) == 4) {
            __builtin_amdgcn_raw_buffer_store_b32(x, k, 4 * vo, 4 * so, 0);
        } else {
            __builtin_amdgcn_raw_buffer_store_b32(pair_key(x), k, 4 * vo, 4 * so, 0);
            __builtin_amdgcn_raw_buffer_store_b32(pair_val(x), v, 4 * vo, 4 * so, 0);
        }
    }
};

// Key maps (see KeyMap): the element with its key mapped; pads are never
// mapped, so the callers apply these to real elements only.
__device__ __forceinline__ bool key_map_on(KeyMap m) { return (m.um | m.fm | m.fl) != 0; }
__device__ __forceinline__ int32_t key_map(int32_t b, KeyMap m)
{
    return b ^ (((b >> 31) & m.fm) | m.um);
}
template <typename T> __device__ __forceinline__ T map_elem(T x, KeyMap m)
{
    if constexpr (sizeof(T) == 4) {
        return key_map(x, m);
    } else {
        const int64_t f = (int64_t)(((uint64_t)(uint32_t)m.fm << 32) | (uint32_t)m.fl);
        const int64_t u = (int64_t)((uint64_t)(uint32_t)m.um << 32);
        return x ^ (((x >> 63) & f) | u);
    }
}

// ---------------------------------------------------------------- comparators

// In-lane compare-exchange: a <- min, b <- max.  Keys: v_min_i32 + v_max_i32;
// pairs: one 64-bit compare and four selects (the branch-free "conditional
// select" comparator of Fig. 3b).
template <typename T> __device__ __forceinline__ void cmpx(T &a, T &b)
{
    if constexpr (sizeof(T) == 4) {
        const T lo = a < b ? a : b;
        const T hi = a < b ? b : a;
        a = lo;
        b = hi;
    } else {
        const bool s = b < a;
        const T lo = s ? b : a;
        const T hi = s ? a : b;
        a = lo;
        b = hi;
    }
}

// Cross-lane half of a compare-exchange: this lane keeps the min of its value
// and its partner's (upper == false) or the max (upper == true).
//
// Keys take a per-stage selector instead (keep_sel): the median of
// (v, p, sel) with sel = INT32_MAX keeps the max and sel = INT32_MIN the min,
// one v_med3_i32 per element.  The selector is hidden from the optimizer
// (an empty asm with a register operand, no instruction), which would
// otherwise turn the median back into min + max + select.
__device__ __forceinline__ int32_t keep_selector(bool upper)
{
    int32_t sel = upper ? 0x7fffffff : (int32_t)0x80000000;
    asm volatile("" : "+v"(sel));
    return sel;
}
__device__ __forceinline__ int32_t keep_sel(int32_t v, int32_t p, int32_t sel)
{
    const int32_t mn = v < p ? v : p;
    const int32_t mx = v < p ? p : v;
    const int32_t m = mn > sel ? mn : sel;
    return mx < m ? mx : m;
}
template <typename T> __device__ __forceinline__ T keep(T v, T p, bool upper)
{
    if constexpr (sizeof(T) == 4) {
        const T mn = v < p ? v : p;
        const T mx = v < p ? p : v;
        return upper ? mx : mn;
    } else {
        const bool s = p < v;
        return (s != upper) ? p : v;
    }
}

// ------------------------------------------------------------ lane exchange

__device__ __forceinline__ int lane_id()
{
    return (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Value of v held by lane (lane ^ M), for the partners the merge levels
// reach this way: DPP quad permutes (xor 1, 2) and row rotate by 8 (xor 8
// inside a 16-lane row), ds_swizzle in bit-mask mode for xor 4.  (xor 16
// and 32 go through lane_swap below.)
template <int M> __device__ __forceinline__ int32_t xlane32(int32_t v)
{
    static_assert(M == 1 || M == 2 || M == 4 || M == 8, "no single-operation exchange");
    // update_dpp with every row and bank enabled and bound_ctrl set
    if constexpr (M == 1)
        return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, true);  // quad_perm 1,0,3,2
    else if constexpr (M == 2)
        return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, true);  // quad_perm 2,3,0,1
    else if constexpr (M == 4)
        return __builtin_amdgcn_ds_swizzle(v, 0x101F);                    // xor 4
    else
        return __builtin_amdgcn_update_dpp(0, v, 0x128, 0xF, 0xF, true); // row_ror:8
}

template <int M, typename T> __device__ __forceinline__ T xlane(T v)
{
    if constexpr (sizeof(T) == 4) {
        return xlane32<M>(v);
    } else {
        const int32_t lo = xlane32<M>((int32_t)(uint32_t)(uint64_t)v);
        const int32_t hi = xlane32<M>((int32_t)((uint64_t)v >> 32));
        return (T)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
    }
}

// ------------------------------------------------ per-lane column sort (a2)

// Each lane sorts the R values it holds with the network table for R
// (Sec. 2.3): 60 comparators at R = 16, Batcher's odd-even sort otherwise.
// NET selects the 16-input alternatives of the Table 1 ablation: 1 = Batcher
// odd-even (63 comparators), 2 = bitonic (80).
template <int R, typename T, int NET = 0> __device__ __forceinline__ void column_sort(T (&v)[R])
{
    if constexpr (R == 16 && NET == 1) {
#pragma unroll
        for (int c = 0; c < HVMS_NET16_OE_SIZE; ++c)
            cmpx(v[HVMS_NET16_OE[2 * c]], v[HVMS_NET16_OE[2 * c + 1]]);
    } else if constexpr (R == 16 && NET == 2) {
#pragma unroll
        for (int c = 0; c < HVMS_NET16_BT_SIZE; ++c)
            cmpx(v[HVMS_NET16_BT[2 * c]], v[HVMS_NET16_BT[2 * c + 1]]);
    } else if constexpr (R == 16) {
#pragma unroll
        for (int c = 0; c < HVMS_NET16_SIZE; ++c)
            cmpx(v[HVMS_NET16[2 * c]], v[HVMS_NET16[2 * c + 1]]);
    } else if constexpr (R == 8) {
#pragma unroll
        for (int c = 0; c < HVMS_NET8_SIZE; ++c)
            cmpx(v[HVMS_NET8[2 * c]], v[HVMS_NET8[2 * c + 1]]);
    } else if constexpr (R == 32) {
#pragma unroll
        for (int c = 0; c < HVMS_NET32_SIZE; ++c)
            cmpx(v[HVMS_NET32[2 * c]], v[HVMS_NET32[2 * c + 1]]);
    } else {
        static_assert(R == 4, "unsupported keys per lane");
#pragma unroll
        for (int c = 0; c < HVMS_NET4_SIZE; ++c)
            cmpx(v[HVMS_NET4[2 * c]], v[HVMS_NET4[2 * c + 1]]);
    }
}

// ------------------------------------- cross-lane bitonic merge levels (a3)
//
// Layout: logical lane l holds elements R*l .. R*l + R-1 of the wavefront's
// tile in v[0..R).  Merge level K turns sorted runs of R*2^(K-1) (2^(K-1)
// adjacent logical lanes) into runs of R*2^K.  The runs alternate in
// direction, as in Batcher's bitonic sort: level K leaves the run of logical
// lanes with bit K set in descending order (ascending at the last level), so
// the two runs level K merges form a bitonic sequence and every stage is a
// half-cleaner.  Level 1 merges the ascending columns of the column sort
// instead, and starts with the flip stage (element e against e ^ (2R - 1):
// lane l ^ 1, register R-1-r).  The cross-lane half-cleaners (partner lane
// l ^ 2^j, same register) are the vector part of the hybrid merger of Sec.
// 2.4; the in-lane ones at distances R/2 .. 1 its serial part.
//
// Logical lane bits 0..5 sit at physical lane bits 0, 1, 3, 4, 5, 2.  The
// partners of the five most used bits are then reached by VALU operations
// only: DPP quad permutes (physical xor 1, 2), DPP row rotate by 8 (xor 8)
// and the gfx950 lane swaps v_permlane16_swap / v_permlane32_swap (xor 16,
// xor 32).  Logical bit 5, used once (the first stage of level 6), is
// physical xor 4: ds_swizzle.  Which element a lane holds never matters to
// the column sort; the loads and stores around the merge use logical_lane.

__device__ __forceinline__ int logical_lane(int p)
{
    return (p & 3) | (((p >> 3) & 7) << 2) | (((p >> 2) & 1) << 5);
}
constexpr int lane_phys_bit(int j)
{
    return j == 0 ? 0 : j == 1 ? 1 : j == 2 ? 3 : j == 3 ? 4 : j == 4 ? 5 : 2;
}

// In-lane compare-exchange in the direction `desc` (per lane): keys as two
// medians with opaque selectors (the same two VALU operations as min + max),
// pairs as one 64-bit compare and four selects.
template <typename T> struct DirSel;
template <> struct DirSel<int32_t> {
    int32_t lo, hi;  // selector of the element kept at the lower / higher index
    __device__ __forceinline__ explicit DirSel(bool desc)
        : lo(keep_selector(desc)), hi(keep_selector(!desc)) {}
};
template <> struct DirSel<int64_t> {
    bool desc;
    __device__ __forceinline__ explicit DirSel(bool d) : desc(d) {}
};

template <typename T> __device__ __forceinline__ void cmpx_dir(T &a, T &b, const DirSel<T> &d)
{
    if constexpr (sizeof(T) == 4) {
        const T lo = keep_sel(a, b, d.lo);
        const T hi = keep_sel(a, b, d.hi);
        a = lo;
        b = hi;
    } else {
        const bool s = (b < a) != d.desc;
        const T lo = s ? b : a;
        const T hi = s ? a : b;
        a = lo;
        b = hi;
    }
}

template <int R, int D, typename T>
__device__ __forceinline__ void inlane_half_cleaners(T (&v)[R], const DirSel<T> &d)
{
    if constexpr (D >= 1) {
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (!(r & D))
                cmpx_dir(v[r], v[r + D], d);
        inlane_half_cleaners<R, D / 2>(v, d);
    }
}

// v_permlane{16,32}_swap on (x, y): x keeps its rows (16 lanes) or halves
// (32 lanes) with the bit clear and takes y's there; y takes x's others.  So
// at every lane q, (x', y') is the pair {lane q, lane q ^ M} of x when q's
// bit is clear and of y when it is set, the lower lane's element in x'.
template <int M> __device__ __forceinline__ void lane_swap(int32_t &x, int32_t &y)
{
    static_assert(M == 16 || M == 32, "lane swaps exist for xor 16 and 32");
    if constexpr (M == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(x, y, false, false);
        x = (int32_t)r[0];
        y = (int32_t)r[1];
    } else {
        const auto r = __builtin_amdgcn_permlane32_swap(x, y, false, false);
        x = (int32_t)r[0];
        y = (int32_t)r[1];
    }
}
template <int M> __device__ __forceinline__ void lane_swap(int64_t &x, int64_t &y)
{
    int32_t xl = (int32_t)(uint32_t)(uint64_t)x, xh = (int32_t)((uint64_t)x >> 32);
    int32_t yl = (int32_t)(uint32_t)(uint64_t)y, yh = (int32_t)((uint64_t)y >> 32);
    lane_swap<M>(xl, yl);
    lane_swap<M>(xh, yh);
    x = (int64_t)(((uint64_t)(uint32_t)xh << 32) | (uint32_t)xl);
    y = (int64_t)(((uint64_t)(uint32_t)yh << 32) | (uint32_t)yl);
}

// Cross-lane half-cleaner on logical bit J with direction `desc`: the lane
// whose bit J is clear keeps the min (the max when descending).
template <int R, int J, typename T>
__device__ __forceinline__ void cross_half_cleaner(T (&v)[R], int lane, bool desc)
{
    constexpr int PB = lane_phys_bit(J);
    constexpr int M = 1 << PB;
    if constexpr (M == 16 || M == 32) {
        // registers in pairs: swap so that each lane holds one lane pair of
        // one register (lower element in the first), compare-exchange in
        // place, swap back.  The direction is the same for both lanes of a
        // pair (it depends on a higher bit), so each lane uses its own.
        const DirSel<T> d(desc);
#pragma unroll
        for (int r = 0; r < R; r += 2) {
            lane_swap<M>(v[r], v[r + 1]);
            cmpx_dir(v[r], v[r + 1], d);
            lane_swap<M>(v[r], v[r + 1]);
        }
    } else {
        const bool upper = (((lane >> PB) & 1) != 0) != desc;  // keeps the max
        if constexpr (sizeof(T) == 4) {
            const int32_t sel = keep_selector(upper);
#pragma unroll
            for (int r = 0; r < R; ++r)
                v[r] = keep_sel(v[r], xlane<M>(v[r]), sel);
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r)
                v[r] = keep(v[r], xlane<M>(v[r]), upper);
        }
    }
}

template <int R, int J, typename T>
__device__ __forceinline__ void cross_half_cleaners(T (&v)[R], int lane, bool desc)
{
    if constexpr (J >= 0) {
        cross_half_cleaner<R, J>(v, lane, desc);
        cross_half_cleaners<R, J - 1>(v, lane, desc);
    }
}

// Level K of `levels`: descending output for the runs whose logical lanes
// have bit K set, unless this is the last level.
template <int R, int K, typename T>
__device__ __forceinline__ void wave_merge_level(T (&v)[R], int lane, int levels)
{
    const bool desc = K < levels && ((lane >> lane_phys_bit(K < 6 ? K : 0)) & 1) != 0;
    if constexpr (K == 1) {
        // flip stage between the ascending columns of lanes l and l ^ 1
        const bool upper = ((lane & 1) != 0) != desc;
        T p[R];
#pragma unroll
        for (int r = 0; r < R; ++r)
            p[r] = xlane<1>(v[R - 1 - r]);
        if constexpr (sizeof(T) == 4) {
            const int32_t sel = keep_selector(upper);
#pragma unroll
            for (int r = 0; r < R; ++r)
                v[r] = keep_sel(v[r], p[r], sel);
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r)
                v[r] = keep(v[r], p[r], upper);
        }
    } else {
        cross_half_cleaners<R, K - 1>(v, lane, desc);
    }
    inlane_half_cleaners<R, R / 2>(v, DirSel<T>(desc));
}

template <int R, typename T> __device__ __forceinline__ void wave_merge(T (&v)[R], int lane, int levels)
{
    if (levels >= 1) wave_merge_level<R, 1>(v, lane, levels);
    if (levels >= 2) wave_merge_level<R, 2>(v, lane, levels);
    if (levels >= 3) wave_merge_level<R, 3>(v, lane, levels);
    if (levels >= 4) wave_merge_level<R, 4>(v, lane, levels);
    if (levels >= 5) wave_merge_level<R, 5>(v, lane, levels);
    if (levels >= 6) wave_merge_level<R, 6>(v, lane, levels);
}

// ------------------------------------------------------- merge path (a4-a6)

// LDS views.  LdsPlain indexes an array directly.  LdsSkew inserts 16 bytes
// after every 16 elements, so that lanes writing or reading R consecutive
// elements each (stride R elements) hit distinct banks: with R = 16 int32
// the lane stride becomes 80 bytes and the 16 lanes of one ds_write_b128
// pass cover all 64 banks once.
template <typename T> struct LdsPlain {
    T *S;
    int base;
    __device__ __forceinline__ T &operator[](int i) const { return S[base + i]; }
    static constexpr int size(int n) { return n; }
};
template <typename T> struct LdsSkew {
    T *S;
    int base;
    static constexpr int kPad = 16 / (int)sizeof(T);
    __device__ __forceinline__ static int pos(int i) { return i + (i >> 4) * kPad; }
    __device__ __forceinline__ T &operator[](int i) const { return S[pos(base + i)]; }
    static constexpr int size(int n) { return n + (n / 16) * kPad; }
};

// Co-rank of diagonal d in the merge of S[0..alen) and S[boff..boff+blen):
// the number of elements taken from the first run among the first d outputs
// of the merge that takes the first run on ties.
// Writes a row of VT elements at position o of a skewed LDS array (o a
// multiple of 16 bytes' worth of elements, the array's base 0): 16-byte
// stores when the whole row is valid (consecutive threads' rows then fall in
// distinct banks), else the first lim elements one by one.
template <int VT, typename T>
__device__ __forceinline__ void put_row(const LdsSkew<T> &W, int o, const T (&v)[VT], int lim)
{
    constexpr int E = 16 / (int)sizeof(T);
    typedef T Vec __attribute__((ext_vector_type(E)));
    if (lim >= VT) {
#pragma unroll
        for (int q = 0; q < VT; q += E) {
            Vec x;
#pragma unroll
            for (int e = 0; e < E; ++e)
                x[e] = v[q + e];
            *(Vec *)&W[o + q] = x;
        }
    } else {
#pragma unroll
        for (int k = 0; k < VT; ++k)
            if (k < lim)
                W[o + k] = v[k];
    }
}

template <typename V>
__device__ __forceinline__ int lds_corank(const V &S, int alen, int boff, int blen, int d)
{
    int lo = d > blen ? d - blen : 0;
    int hi = d < alen ? d : alen;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (S[boff + d - 1 - mid] < S[mid])
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// Serial merge of VT outputs starting at positions (i, j) of the two runs in
// S (first run at 0, second at boff); one LDS read per output.
template <int VT, typename V, typename T>
__device__ __forceinline__ void serial_merge(const V &S, int alen, int boff, int blen, int i, int j,
                                             T (&out)[VT])
{
    T a = S[i < alen ? i : (alen > 0 ? alen - 1 : 0)];
    T b = S[boff + (j < blen ? j : (blen > 0 ? blen - 1 : 0))];
#pragma unroll
    for (int k = 0; k < VT; ++k) {
        const bool takeB = (j < blen) && (i >= alen || b < a);
        out[k] = takeB ? b : a;
        i += takeB ? 0 : 1;
        j += takeB ? 1 : 0;
        int ia = i < alen ? i : alen - 1;
        int ib = j < blen ? j : blen - 1;
        int addr = takeB ? boff + (ib < 0 ? 0 : ib) : (ia < 0 ? 0 : ia);
        const T nx = S[addr];
        a = takeB ? a : nx;
        b = takeB ? nx : b;
    }
}

// The serial merge of the block stage's LDS levels: runs A = [base, base +
// run) and B = [base + run, base + 2 run) of a skewed tile of TILE elements,
// R outputs from co-ranks (i, j).  Branch-free: a run counts as exhausted
// once its next position reaches its end (the value read there is never
// used); the next position read is clamped to the tile's last element, the
// only read that could leave the array (A's end is B's start).
template <int R, int TILE, typename T>
__device__ __forceinline__ void merge_pair_rows(const T *S, int base, int run, int i, int j,
                                                T (&out)[R])
{
    int pa = base + i, pb = base + run + j;
    const int aend = base + run, bend = base + 2 * run;
    T a = S[LdsSkew<T>::pos(pa)];
    T b = S[LdsSkew<T>::pos(pb < TILE - 1 ? pb : TILE - 1)];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const bool takeB = (pb < bend) & ((pa >= aend) | (b < a));
        out[k] = takeB ? b : a;
        if (k + 1 < R) {
            pa += takeB ? 0 : 1;
            pb += takeB ? 1 : 0;
            int r = takeB ? pb : pa;
            r = r < TILE - 1 ? r : TILE - 1;
            const T nx = S[LdsSkew<T>::pos(r)];
            a = takeB ? a : nx;
            b = takeB ? nx : b;
        }
    }
}

// serial_merge without index clamps, for callers whose LDS array extends at
// least one element past the end of either run: a run counts as exhausted
// once its next position reaches its end (the value read there is never
// used), so the loop is branch-free.
template <int VT, typename V, typename T>
__device__ __forceinline__ void serial_merge_open(const V &S, int alen, int boff, int blen, int i,
                                                  int j, T (&out)[VT])
{
    int pa = i, pb = boff + j;
    const int bend = boff + blen;
    T a = S[pa], b = S[pb];
#pragma unroll
    for (int k = 0; k < VT; ++k) {
        const bool takeB = (pb < bend) & ((pa >= alen) | (b < a));
        out[k] = takeB ? b : a;
        if (k + 1 < VT) {
            pa += takeB ? 0 : 1;
            pb += takeB ? 1 : 0;
            const T nx = S[takeB ? pb : pa];
            a = takeB ? a : nx;
            b = takeB ? nx : b;
        }
    }
}

// VT consecutive elements from position i of an LDS view.
//
// int32 runs of VT <= 16 are read as the VT/4 + 1 16-byte chunks that cover
// them, then shifted in registers by i mod 4.  Threads whose runs start
// about VT/2 elements apart (a merge-path share per thread) would meet up to
// 8-way bank conflicts element by element, and up to 16-way inside runs of
// equal keys (where the tie rule makes every share one-sided); 16-byte reads
// meet at most 2-way.  Both views keep 16-byte chunks contiguous (the skewed
// one pads every four chunks).  Reads up to 3 elements past i + VT - 1.
__device__ __forceinline__ const int4 *lds_chunk(const LdsPlain<int32_t> &S, int c)
{
    return (const int4 *)(S.S + 4 * c);
}
__device__ __forceinline__ const int4 *lds_chunk(const LdsSkew<int32_t> &S, int c)
{
    return (const int4 *)(S.S + 4 * c + LdsSkew<int32_t>::kPad * (c >> 2));
}
template <int VT, typename View>
__device__ __forceinline__ void load_run_chunks(const View &S, int i, int32_t (&x)[VT])
{
    const int p = S.base + i;
    const int c0 = p >> 2, sh = p & 3;
    int32_t w[VT + 4];
#pragma unroll
    for (int c = 0; c < VT / 4 + 1; ++c) {
        const int4 v = *lds_chunk(S, c0 + c);
        w[4 * c] = v.x;
        w[4 * c + 1] = v.y;
        w[4 * c + 2] = v.z;
        w[4 * c + 3] = v.w;
    }
    // the shift as bitwise selects on opaque masks (left as selects, the
    // compiler turns them into an indexed array in scratch)
    int32_t m0 = -(sh & 1), m1 = -((sh >> 1) & 1);
    asm volatile("" : "+v"(m0), "+v"(m1));
#pragma unroll
    for (int k = 0; k < VT; ++k) {
        const int32_t lo = (w[k + 1] & m0) | (w[k] & ~m0);
        const int32_t hi = (w[k + 3] & m0) | (w[k + 2] & ~m0);
        x[k] = (hi & m1) | (lo & ~m1);
    }
}

// Other element types and widths: in the skewed view a run of VT <= 16
// crosses at most one 16-element row, whose padding shifts the elements
// after the crossing by one pad: each element's address is one of two bases
// plus a constant offset.
template <int VT, typename T>
__device__ __forceinline__ void load_run(const LdsPlain<T> &S, int i, T (&x)[VT])
{
    if constexpr (sizeof(T) == 4 && VT <= 16) {
        load_run_chunks<VT>(S, i, x);
    } else {
#pragma unroll
        for (int k = 0; k < VT; ++k)
            x[k] = S[i + k];
    }
}
template <int VT, typename T>
__device__ __forceinline__ void load_run(const LdsSkew<T> &S, int i, T (&x)[VT])
{
    if constexpr (sizeof(T) == 4 && VT <= 16) {
        load_run_chunks<VT>(S, i, x);
    } else if constexpr (VT <= 16) {
        const int p = S.base + i;
        // bit k of cross: element k lies past the end of p's row
        uint32_t cross = 0xffffu << (16 - (p & 15));
        asm("" : "+v"(cross));
        const T *p0 = S.S + LdsSkew<T>::pos(p);
#pragma unroll
        for (int k = 0; k < VT; ++k) {
            // the bit stays opaque, so that its address takes one bit
            // extract and one shift-add
            uint32_t bit = __builtin_amdgcn_ubfe(cross, k, 1);
            asm("" : "+v"(bit));
            x[k] = p0[k + LdsSkew<T>::kPad * (int)bit];
        }
    } else {
#pragma unroll
        for (int k = 0; k < VT; ++k)
            x[k] = S[i + k];
    }
}

// The same VT outputs as serial_merge without a dependent LDS read per
// output (the hybrid bitonic merge of Sec. 2.4 applied to one thread's share
// of a merge path): both runs' next VT elements are read at once (positions
// past a run's end read as the pad value), the flip stage of a bitonic merge
// keeps the VT smallest of the 2VT as a bitonic sequence, and log2(VT)
// half-cleaner stages sort it.  Exact because the element order is total on
// bit patterns (equal elements are identical, and the pad is the maximum).
// Reads S up to VT + 2 positions past each run's end (VT - 1 for 64-bit
// elements): the caller's LDS array must extend that far.
// MASK = false: the caller guarantees that the VT - 1 positions after each
// run hold the maximum of the order (sentinels), so no read needs a mask.
template <int VT, bool MASK = true, typename V, typename T>
__device__ __forceinline__ void reg_merge(const V &S, int alen, int boff, int blen, int i, int j,
                                          T (&out)[VT])
{
    T b[VT], xa[VT], yb[VT];
    load_run<VT>(S, i, xa);
#pragma unroll
    for (int k = 0; k < VT; ++k)
        out[k] = (!MASK || i + k < alen) ? xa[k] : Traits<T>::kMax;
    // the second run's reads after the first run's (fewer live registers)
    asm volatile("" ::: "memory");
    load_run<VT>(S, boff + j, yb);
#pragma unroll
    for (int k = 0; k < VT; ++k)
        b[k] = (!MASK || j + k < blen) ? yb[k] : Traits<T>::kMax;
#pragma unroll
    for (int k = 0; k < VT; ++k) {
        const T y = b[VT - 1 - k];
        out[k] = y < out[k] ? y : out[k];
    }
#pragma unroll
    for (int h = VT / 2; h >= 1; h >>= 1)
#pragma unroll
        for (int k = 0; k < VT; ++k)
            if (!(k & h))
                cmpx(out[k], out[k + h]);
}

// Steps a2-a4 on one tile: v holds each lane's R values (for runs shorter
// than the tile: elements R*lane .. R*lane+R-1 of its wave's slice); sorts
// the columns, runs `wave_levels` cross-lane merge levels, writes the runs to
// the skewed LDS tile in order and merges them `lds_levels` more times in
// LDS.  On return (after a barrier) element p of the tile's sorted runs is at
// LdsSkew position p of S.
template <int R, int NT, typename T, int NET = 0>
__device__ __forceinline__ void sort_tile_core(T *S, T (&v)[R], int t, int wave_levels,
                                               int lds_levels)
{
    const int lane = t & 63;
    const int wave = t >> 6;
    column_sort<R, T, NET>(v);
    wave_merge<R>(v, lane, wave_levels);

    const LdsSkew<T> W{S, wave * (64 * R) + logical_lane(lane) * R};
#pragma unroll
    for (int r = 0; r < R; ++r)
        W[r] = v[r];
    __syncthreads();

    int run = R << wave_levels;
    for (int l = 0; l < lds_levels; ++l, run *= 2) {
        const int o0 = t * R;
        const int base = o0 & ~(2 * run - 1);
        const int d = o0 - base;
        const LdsSkew<T> P{S, base};
        const int i = lds_corank(P, run, run, run, d);
        T out[R];
        merge_pair_rows<R, R * NT>(S, base, run, i, d - i, out);
        __syncthreads();
        const LdsSkew<T> O{S, o0};
#pragma unroll
        for (int k = 0; k < R; ++k)
            O[k] = out[k];
        __syncthreads();
    }
}

// ------------------------------------------- presorted tiles (block stage)

// Lane (lane + 1)'s value, and lane 0's for lane 63 (its caller replaces it).
template <typename T> __device__ __forceinline__ T from_next_lane(T v, int lane)
{
    const int src = ((lane + 1) & 63) << 2;
    if constexpr (sizeof(T) == 4) {
        return __builtin_amdgcn_ds_bpermute(src, v);
    } else {
        const int lo = __builtin_amdgcn_ds_bpermute(src, (int)(uint32_t)(uint64_t)v);
        const int hi = __builtin_amdgcn_ds_bpermute(src, (int)((uint64_t)v >> 32));
        return (T)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
    }
}

template <typename T> __device__ __forceinline__ T lane_value(T v, int src_lane)
{
    if constexpr (sizeof(T) == 4) {
        return __builtin_amdgcn_readlane(v, src_lane);
    } else {
        const int lo = __builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)v, src_lane);
        const int hi = __builtin_amdgcn_readlane((int)((uint64_t)v >> 32), src_lane);
        return (T)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
    }
}

// Order of a full tile as loaded (lane l holds elements l, l + 64, ... of its
// wave's slice): 1 nondecreasing, 2 nonincreasing (and not constant), 0
// neither.  A cheap in-lane test (elements 64 apart) rules out most tiles;
// waves that pass it compare lane neighbours, then the waves' boundary
// elements are compared through S (free before the sort; one barrier, and a
// second one when the sort follows).  Block-uniform result.
template <int R, int NT, typename T>
__device__ __forceinline__ int tile_order(T *S, const T (&v)[R], int lane, int wave)
{
    constexpr int W = NT / 64;
    bool up = true, down = true;
#pragma unroll
    for (int j = 0; j + 1 < R; ++j) {
        up = up && !(v[j + 1] < v[j]);
        down = down && !(v[j] < v[j + 1]);
    }
    up = __builtin_amdgcn_ballot_w64(!up) == 0;  // wave-uniform from here
    down = __builtin_amdgcn_ballot_w64(!down) == 0;
    if (up || down) {
#pragma unroll
        for (int j = 0; j < R; ++j) {
            T nx = from_next_lane(v[j], lane);
            if (j + 1 < R)
                nx = lane == 63 ? lane_value(v[j + 1], 0) : nx;
            const bool last = j + 1 == R && lane == 63;  // the wave's last element
            up = up && (last || !(nx < v[j]));
            down = down && (last || !(v[j] < nx));
        }
        up = __builtin_amdgcn_ballot_w64(!up) == 0;
        down = __builtin_amdgcn_ballot_w64(!down) == 0;
    }
    if (lane == 0) {
        S[4 * wave + 0] = up ? 1 : 0;
        S[4 * wave + 1] = down ? 1 : 0;
        S[4 * wave + 2] = v[0];
    }
    if (lane == 63)
        S[4 * wave + 3] = v[R - 1];
    __syncthreads();
    bool bu = true, bd = true;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        bu = bu && S[4 * w] != 0;
        bd = bd && S[4 * w + 1] != 0;
        if (w + 1 < W) {
            const T last = S[4 * w + 3], first = S[4 * (w + 1) + 2];
            bu = bu && !(first < last);
            bd = bd && !(last < first);
        }
    }
    return bu ? 1 : (bd ? 2 : 0);
}

}  // namespace hvms
