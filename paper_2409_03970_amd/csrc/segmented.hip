// Batched segmented sort: many arrays of uneven sizes, sorted by one
// persistent launch for everything up to the block tile, plus merge passes
// for the segments larger than it (steps a1-a6 applied per segment, a8).
//
// Plan (all kernels on the caller's stream; no memset, no allocation, no host
// synchronisation, so the whole call can be captured into a hipGraph):
//  1. init:     zero the control block.
//  2. count:    each segment gets a size class.  A segment longer than TILE
//               keys is cut into its full TILE-key pieces and a ragged rest,
//               and needs P_s = ceil(log2(pieces)) merge levels.  A segment
//               of at most TILE keys, or a rest, of s keys goes to the
//               full-piece list if s > TILE/2 (padded), to the half list if
//               s > TILE/4 (two to a tile), else to bucket X = max(R,
//               2^ceil(log2 s)) of the packed kernel.  Counts are reduced in
//               LDS, then added to the control block once per workgroup.
//  3. plan:     one workgroup turns counts into list bases, task numbers
//               (a task packs TILE/X pieces of one bucket into one tile) and
//               the tile count of every merge pass.
//  4. scatter:  pieces go to their lists; the merge tiles of large segments
//               go to a tile list ordered by P_s descending, so the tiles of
//               pass p are a prefix of it.
//  5. block:    the full-piece kernel sorts the full list (one piece per
//               workgroup) and the half list (two per workgroup); the packed
//               kernel, persistent, pulls tasks with an atomic ticket, largest
//               buckets first: a task gathers its pieces into LDS (padded
//               with the maximum), sorts every run of X in place (column
//               sort, cross-lane levels, LDS merges), and scatters them back.
//               Short segments go straight to the output, pieces of large
//               segments to output or scratch by the parity of their merge
//               launches.
//  6. passes:   for p < P_max: co-ranks of pass p's tiles, then the
//               persistent pipelined merge over the same tile list.  With
//               four-way passes a segment takes ceil(L_s / 2) launches for
//               its L_s merge levels: launch p merges groups of four runs of
//               TILE * 4^p for the segments with at least two levels left
//               (the front of pass p's tiles) and pairs of such runs for the
//               segments with one level left (the rest).
#include "hvms.h"
#include "hvms_internal.h"
#include "merge_common.h"

namespace hvms {

namespace {

constexpr int kMaxBuckets = 16;
constexpr int kMaxP = 48;

// control block layout (int64 words)
enum : int {
    C_CNT = 0,                      // pieces per bucket
    C_CUR = C_CNT + kMaxBuckets,    // scatter cursors per bucket
    C_BASE = C_CUR + kMaxBuckets,   // first piece of each bucket
    C_TASK = C_BASE + kMaxBuckets,  // first task of each bucket
    C_NTASK = C_TASK + kMaxBuckets, // total tasks
    C_TICKET,                       // task ticket counter
    C_OVER,                         // segments with P_s above the enqueued passes
    C_SKIP,                         // segments skipped: offsets outside [0, n_total] or decreasing
    C_BAD,                          // 1: offsets inconsistent with n_total, nothing sorted
    C_FULL,                         // full-list pieces (a tile, or padded: more than half a tile)
    C_FCUR,                         // scatter cursor of the full-piece list
    C_HALF,                         // half-list pieces (more than a quarter, at most half a tile)
    C_HCUR,                         // scatter cursor of the half list
    C_LCNT = 80,                    // large segments with P_s == P
    C_TCNT = C_LCNT + kMaxP,        // merge tiles of those segments
    C_TCUR = C_TCNT + kMaxP,        // tile-list cursors per P
    C_TBASE = C_TCUR + kMaxP,       // tile-list base per P
    C_PASS = C_TBASE + kMaxP,       // tiles of pass p
    C_PASSF = C_PASS + kMaxP,       // four-way passes: the four-way tiles of pass p
    C_WORDS = C_PASSF + kMaxP
};

struct Piece {
    int64_t off;  // absolute index of the first key
    int32_t len;  // keys (<= X of its bucket)
    int32_t dst;  // 0: output, 1: scratch
};

__device__ __forceinline__ int ceil_log2(int64_t x)
{
    int l = 0;
    while (((int64_t)1 << l) < x)
        ++l;
    return l;
}

struct SegParams {
    const int64_t *off;
    int64_t nseg, n_total;
    int64_t max_pieces, max_tiles, max_full, max_half;  // list capacities in the workspace
    int tile_log2, r_log2, nb;  // nb = buckets = tile_log2 - r_log2 + 1
    int passes;                 // merge launches enqueued by the host
    int ways;                   // 2 or 4 runs merged per launch
    int64_t tm;
};

// Merge launches of a segment with L merge levels.
__device__ __forceinline__ int launches_of(const SegParams &P, int L)
{
    return P.ways == 4 ? (L + 1) >> 1 : L;
}

// Where a piece (a segment of at most a tile, or a longer segment's ragged
// rest) of len keys is sorted: 2 the full-piece list (more than half a tile,
// padded), 1 the half list (more than a quarter: two per full-kernel tile,
// each padded to half a tile), 0 the packed kernel's bucket of its size.
__device__ __forceinline__ int piece_class(int64_t len, int64_t tile)
{
    return 2 * len > tile ? 2 : (4 * len > tile ? 1 : 0);
}

__device__ __forceinline__ int bucket_of(const SegParams &P, int64_t size)
{
    const int l = ceil_log2(size);
    return (l < P.r_log2 ? P.r_log2 : l) - P.r_log2;
}

__global__ void seg_init_kernel(unsigned long long *ctrl)
{
    for (int i = threadIdx.x; i < C_WORDS; i += blockDim.x)
        ctrl[i] = 0;
}

__global__ __launch_bounds__(256) void seg_count_kernel(SegParams P, unsigned long long *ctrl)
{
    __shared__ unsigned long long cnt[kMaxBuckets], lcnt[kMaxP], tcnt[kMaxP], over, skip, full,
        half;
    for (int i = threadIdx.x; i < kMaxP; i += blockDim.x) {
        lcnt[i] = 0;
        tcnt[i] = 0;
        if (i < kMaxBuckets)
            cnt[i] = 0;
    }
    if (threadIdx.x == 0) {
        over = 0;
        skip = 0;
        full = 0;
        half = 0;
    }
    __syncthreads();
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < P.nseg) {
        // a segment outside [0, n_total], or with decreasing offsets, is
        // treated as empty and counted
        const int64_t a = P.off[s], e = P.off[s + 1];
        const bool valid = a >= 0 && e <= P.n_total && e >= a;
        const int64_t size = valid ? e - a : 0;
        if (!valid)
            atomicAdd(&skip, 1ull);
        if (size > 0) {
            const int64_t tile = (int64_t)1 << P.tile_log2;
            // full pieces go to the full-piece list, the segment itself (at
            // most a tile) or a longer one's ragged rest where piece_class says
            const int64_t nfull = size > tile ? size / tile : 0, rest = size - nfull * tile;
            const int cls = piece_class(rest, tile);
            if (nfull || cls == 2)
                atomicAdd(&full, (unsigned long long)(nfull + (cls == 2 ? 1 : 0)));
            if (cls == 1)
                atomicAdd(&half, 1ull);
            else if (cls == 0 && rest)
                atomicAdd(&cnt[bucket_of(P, rest)], 1ull);
            if (size > tile) {
                const int64_t np = (size + tile - 1) / tile;
                const int ps = ceil_log2(np);
                atomicAdd(&lcnt[ps], 1ull);
                atomicAdd(&tcnt[ps], (unsigned long long)((size + P.tm - 1) / P.tm));
                if (launches_of(P, ps) > P.passes)
                    atomicAdd(&over, 1ull);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (over)
            atomicAdd(&ctrl[C_OVER], over);
        if (skip)
            atomicAdd(&ctrl[C_SKIP], skip);
        if (full)
            atomicAdd(&ctrl[C_FULL], full);
        if (half)
            atomicAdd(&ctrl[C_HALF], half);
    }
    for (int i = threadIdx.x; i < kMaxP; i += blockDim.x) {
        if (lcnt[i])
            atomicAdd(&ctrl[C_LCNT + i], lcnt[i]);
        if (tcnt[i])
            atomicAdd(&ctrl[C_TCNT + i], tcnt[i]);
        if (i < kMaxBuckets && cnt[i])
            atomicAdd(&ctrl[C_CNT + i], cnt[i]);
    }
}

__global__ __launch_bounds__(64) void seg_plan_kernel(SegParams P, unsigned long long *ctrl)
{
    // one wave: the counts are read once into LDS, the prefix sums over the
    // (at most 48) pass counts are taken by one thread each
    __shared__ unsigned long long cnt[kMaxBuckets], tcnt[kMaxP];
    __shared__ int bad;
    const int t = threadIdx.x;
    if (t < kMaxBuckets)
        cnt[t] = t < P.nb ? ctrl[C_CNT + t] : 0;
    if (t < kMaxP)
        tcnt[t] = ctrl[C_TCNT + t];
    __syncthreads();
    if (t == 0) {
        unsigned long long pieces = 0, tiles_total = 0;
        for (int b = 0; b < P.nb; ++b)
            pieces += cnt[b];
        for (int p = 0; p < kMaxP; ++p)
            tiles_total += tcnt[p];
        bad = pieces > (unsigned long long)P.max_pieces ||
              tiles_total > (unsigned long long)P.max_tiles ||
              ctrl[C_FULL] > (unsigned long long)P.max_full ||
              ctrl[C_HALF] > (unsigned long long)P.max_half;
    }
    __syncthreads();
    if (bad) {
        // inconsistent offsets / n_total: leave every task and pass empty,
        // keep the counts of the status words and raise the flag
        const unsigned long long over = ctrl[C_OVER], skip = ctrl[C_SKIP];
        __syncthreads();
        for (int i = t; i < C_WORDS; i += blockDim.x)
            ctrl[i] = 0;
        __syncthreads();
        if (t == 0) {
            ctrl[C_OVER] = over;
            ctrl[C_SKIP] = skip;
            ctrl[C_BAD] = 1;
        }
        return;
    }
    if (t == 0) {
        unsigned long long base = 0, task = 0;
        for (int b = P.nb - 1; b >= 0; --b) {  // largest bucket first
            const unsigned long long slots = (unsigned long long)1
                                             << (P.tile_log2 - (P.r_log2 + b));
            ctrl[C_BASE + b] = base;
            ctrl[C_TASK + b] = task;
            base += cnt[b];
            task += (cnt[b] + slots - 1) / slots;
        }
        ctrl[C_NTASK] = task;
    }
    if (t < kMaxP) {
        // tile list ordered by merge levels L descending: base of L = t.
        // Two-way pass t covers the segments with L_s > t, a prefix of the
        // list; four-way pass p those with L_s > 2p, of which the ones with
        // L_s > 2p + 1 (four-way tiles) come first
        unsigned long long above = 0;
        for (int q = t + 1; q < kMaxP; ++q)
            above += tcnt[q];
        if (t >= 1)
            ctrl[C_TBASE + t] = above;
        if (P.ways == 4)
            ctrl[((t & 1) ? C_PASSF : C_PASS) + (t >> 1)] = above;
        else
            ctrl[C_PASS + t] = above;
    }
}

__global__ __launch_bounds__(256) void seg_scatter_kernel(SegParams P, unsigned long long *ctrl,
                                                          Piece *pieces, Piece *fulls,
                                                          Piece *halves, int2 *tiles,
                                                          int32_t *passes)
{
    __shared__ unsigned long long cnt[kMaxBuckets], bbase[kMaxBuckets], tcnt[kMaxP], tbase[kMaxP];
    __shared__ unsigned long long fcnt, fbase, hcnt, hbase;
    for (int i = threadIdx.x; i < kMaxP; i += blockDim.x) {
        tcnt[i] = 0;
        if (i < kMaxBuckets)
            cnt[i] = 0;
    }
    if (threadIdx.x == 0) {
        fcnt = 0;
        hcnt = 0;
    }
    __syncthreads();
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tile = (int64_t)1 << P.tile_log2;
    int64_t size = 0, nfull = 0, nt = 0, o = 0, rest = 0;
    int b = -1, ps = 0;
    bool ragged = false;  // the segment, or its rest, is a padded full-list piece
    bool halfp = false;   // ... or a half-list piece
    unsigned long long mine = 0, tmine = 0, fmine = 0, hmine = 0;
    if (s < P.nseg) {
        o = P.off[s];
        const int64_t e = P.off[s + 1];
        size = (o >= 0 && e <= P.n_total && e >= o) ? e - o : 0;
        if (size > 0) {
            nfull = size > tile ? size / tile : 0;
            rest = size - nfull * tile;
            const int cls = piece_class(rest, tile);
            ragged = cls == 2;
            halfp = cls == 1;
            b = (rest && cls == 0) ? bucket_of(P, rest) : -1;
            if (size > tile) {
                ps = ceil_log2((size + tile - 1) / tile);
                nt = (size + P.tm - 1) / P.tm;
                tmine = atomicAdd(&tcnt[ps], (unsigned long long)nt);
            }
            if (nfull || ragged)
                fmine = atomicAdd(&fcnt, (unsigned long long)(nfull + (ragged ? 1 : 0)));
            if (halfp)
                hmine = atomicAdd(&hcnt, 1ull);
            if (b >= 0)
                mine = atomicAdd(&cnt[b], 1ull);
        }
        // a segment needing more passes than are enqueued runs the enqueued
        // ones (and is counted in C_OVER): its pieces start where that pass
        // count lands them in the output
        const int ls = launches_of(P, ps);
        passes[s] = ls < P.passes ? ls : P.passes;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kMaxP; i += blockDim.x) {
        if (tcnt[i])
            tbase[i] = ctrl[C_TBASE + i] + atomicAdd(&ctrl[C_TCUR + i], tcnt[i]);
        if (i < kMaxBuckets && cnt[i])
            bbase[i] = ctrl[C_BASE + i] + atomicAdd(&ctrl[C_CUR + i], cnt[i]);
    }
    if (threadIdx.x == 0 && fcnt)
        fbase = atomicAdd(&ctrl[C_FCUR], fcnt);
    if (threadIdx.x == 0 && hcnt)
        hbase = atomicAdd(&ctrl[C_HCUR], hcnt);
    __syncthreads();
    const int lsd = launches_of(P, ps);
    const int dst = ((lsd < P.passes ? lsd : P.passes) & 1) ? 1 : 0;
    if (b >= 0 && bbase[b] + mine < (unsigned long long)P.max_pieces) {
        // the segment itself, or the ragged rest after its full pieces
        Piece pc;
        pc.off = o + nfull * tile;
        pc.len = (int32_t)(size - nfull * tile);
        pc.dst = dst;
        pieces[bbase[b] + mine] = pc;
    }
    const int64_t nlist = nfull + (ragged ? 1 : 0);
    for (int64_t i = 0; i < nlist && fbase + fmine + i < (unsigned long long)P.max_full; ++i) {
        Piece pc;
        pc.off = o + i * tile;
        pc.len = (int32_t)(i < nfull ? tile : rest);
        pc.dst = dst;
        fulls[fbase + fmine + i] = pc;
    }
    if (halfp && hbase + hmine < (unsigned long long)P.max_half) {
        Piece pc;
        pc.off = o + nfull * tile;
        pc.len = (int32_t)rest;
        pc.dst = dst;
        halves[hbase + hmine] = pc;
    }
    if (nt) {
        const int64_t tf = tbase[ps] + tmine;
        for (int64_t j = 0; j < nt && tf + j < P.max_tiles; ++j)
            tiles[tf + j] = make_int2((int)s, (int)j);
    }
}

// The full pieces of long segments: a tile of exactly R * NT keys each, sorted
// like a tile of the plain block stage (strided register loads, the
// presorted-tile test, column sort, in-register merge levels, LDS merge
// levels), one workgroup per entry of the full-piece list.  R and NT are
// chosen for the tile size (R = 32 where it fits), independent of the packed
// kernel's, which must also serve tiny segments.  The list also holds the
// segments and ragged rests of more than half a tile: such a piece is padded
// with the maximum of the order and sorted whole, and its first len outputs
// are stored (a workgroup-uniform branch; the packed kernel at its smaller R
// sorts a tile about half as fast).  The workgroups past the full list take
// the half list two pieces at a time: each padded to half a tile, sorted with
// one LDS merge level less, so the two halves stay independent runs.
template <int R, int NT, typename T>
__global__ __launch_bounds__(NT) void seg_full_kernel(int wave_levels, int lds_levels,
                                                      const unsigned long long *ctrl,
                                                      const Piece *__restrict__ fulls,
                                                      const Piece *__restrict__ halves,
                                                      const int32_t *__restrict__ ik,
                                                      const int32_t *__restrict__ iv,
                                                      int32_t *__restrict__ ok,
                                                      int32_t *__restrict__ ov,
                                                      int32_t *__restrict__ sk,
                                                      int32_t *__restrict__ sv)
{
    constexpr int TILE = R * NT;
    __shared__ __attribute__((aligned(16))) T S[LdsSkew<T>::size(TILE)];
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int64_t nfull = (int64_t)ctrl[C_FULL];
    if ((int64_t)blockIdx.x >= nfull) {  // two half-list pieces
        constexpr int HT = TILE / 2;
        const int64_t nhalf = (int64_t)ctrl[C_HALF];
        const int64_t h = 2 * ((int64_t)blockIdx.x - nfull);
        if (h >= nhalf)
            return;
        const Piece p0 = halves[h];
        Piece p1 = p0;
        p1.len = 0;
        if (h + 1 < nhalf)
            p1 = halves[h + 1];
        // waves 0 .. NT/128 - 1 hold the first half, the others the second
        const bool second = wave >= NT / 128;
        const int64_t off = second ? p1.off : p0.off;
        const int len = second ? p1.len : p0.len;
        const int rel = (wave & (NT / 128 - 1)) * (64 * R) + lane;
        T v[R];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int p = rel + 64 * j;
            v[j] = p < len ? load_elem<T>(ik + off, sizeof(T) == 8 ? iv + off : nullptr, p)
                           : Traits<T>::kMax;
        }
        sort_tile_core<R, NT>(S, v, t, wave_levels, lds_levels - 1);
        const T *zt = S + LdsSkew<T>::pos(t);
        constexpr int ZS = LdsSkew<T>::size(NT);
#pragma unroll
        for (int j = 0; j < R; ++j) {
            // element t + NT*j: the second half from j = R/2 on (uniform)
            const bool sj = NT * j >= HT;
            const int64_t po = sj ? p1.off : p0.off;
            const int pl = sj ? p1.len : p0.len;
            const bool scr = (sj ? p1.dst : p0.dst) != 0;
            const int e = t + NT * j - (sj ? HT : 0);
            if (e < pl)
                store_elem<T>((scr ? sk : ok) + po, sizeof(T) == 8 ? (scr ? sv : ov) + po : nullptr,
                              e, zt[ZS * j]);
        }
        return;
    }
    {
        const int64_t q = blockIdx.x;  // one piece per workgroup
        const Piece pc = fulls[q];
        // the piece's arrays from its first key on: 32-bit indices below
        const int32_t *pk = ik + pc.off;
        const int32_t *pv = sizeof(T) == 8 ? iv + pc.off : nullptr;
        int32_t *dk = (pc.dst ? sk : ok) + pc.off;
        int32_t *dv = sizeof(T) == 8 ? (pc.dst ? sv : ov) + pc.off : nullptr;
        if (pc.len != TILE) {  // workgroup-uniform: a padded piece
            const int len = pc.len;
            const int rel = wave * (64 * R) + lane;
            T v[R];
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int p = rel + 64 * j;
                v[j] = p < len ? load_elem<T>(pk, pv, p) : Traits<T>::kMax;
            }
            sort_tile_core<R, NT>(S, v, t, wave_levels, lds_levels);
            const T *zt = S + LdsSkew<T>::pos(t);
            constexpr int ZS = LdsSkew<T>::size(NT);
#pragma unroll
            for (int j = 0; j < R; ++j)
                if (t + NT * j < len)
                    store_elem<T>(dk, dv, t + NT * j, zt[ZS * j]);
            return;
        }
        // buffer loads and stores: a lane offset plus a wave-uniform one
        const TileIO<T> in(pk, pv, TILE), out(dk, dv, TILE);
        const int wb = __builtin_amdgcn_readfirstlane(wave) * (64 * R);
        T v[R];
#pragma unroll
        for (int j = 0; j < R; ++j)
            v[j] = in.load(lane, wb + 64 * j);
        const int ord = tile_order<R, NT, T>(S, v, lane, wave);
        if (ord != 0) {  // block-uniform: stored as loaded, or reversed
            const int rel = wave * (64 * R) + lane;
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int p = rel + 64 * j;
                store_elem<T>(dk, dv, ord == 1 ? p : TILE - 1 - p, v[j]);
            }
        } else {
            __syncthreads();  // S is the sort's from here
            // level counts as arguments (not constants), as in the plain
            // block stage: unrolled LDS levels cost registers
            sort_tile_core<R, NT>(S, v, t, wave_levels, lds_levels);
            // element t + NT*j sits at a constant distance from element t
            const T *zt = S + LdsSkew<T>::pos(t);
            constexpr int ZS = LdsSkew<T>::size(NT);
#pragma unroll
            for (int j = 0; j < R; ++j)
                out.store(t, NT * j, zt[ZS * j]);
        }
    }
}

// Persistent block stage: one packed task per iteration.
// Register target of the segmented block stage: at R = 8 (keys) it fits 64
// VGPRs, which keeps two 1024-thread workgroups per CU; one register over
// that allocation step halves the occupancy.
template <int R, typename T> constexpr int seg_block_waves_per_simd()
{
    return (R <= 8 && sizeof(T) == 4) ? 8 : 1;
}

template <int R, int NT, typename T>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(seg_block_waves_per_simd<R, T>())))
void seg_block_kernel(SegParams P, unsigned long long *ctrl,
                                                       const Piece *__restrict__ pieces,
                                                       const int32_t *__restrict__ ik,
                                                       const int32_t *__restrict__ iv,
                                                       int32_t *__restrict__ ok,
                                                       int32_t *__restrict__ ov,
                                                       int32_t *__restrict__ sk,
                                                       int32_t *__restrict__ sv, int wave_max)
{
    constexpr int TILE = R * NT;
    __shared__ __attribute__((aligned(16))) T S[LdsSkew<T>::size(TILE)];
    const LdsSkew<T> Z{S, 0};
    __shared__ int64_t s_off[NT];
    __shared__ int32_t s_len[NT], s_dst[NT];
    __shared__ unsigned long long s_ticket;
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const unsigned long long ntask = ctrl[C_NTASK];

    for (;;) {
        if (t == 0)
            s_ticket = atomicAdd(&ctrl[C_TICKET], 1ull);
        __syncthreads();
        const unsigned long long ticket = s_ticket;
        if (ticket >= ntask)
            break;
        int b = P.nb - 1;
        while (b > 0 && ctrl[C_TASK + b - 1] <= ticket)
            --b;
        const int xlog = P.r_log2 + b;
        const int slots = 1 << (P.tile_log2 - xlog);
        const unsigned long long first = ctrl[C_BASE + b] + (ticket - ctrl[C_TASK + b]) * slots;
        const unsigned long long avail = ctrl[C_CNT + b] - (ticket - ctrl[C_TASK + b]) * slots;
        const int npieces = (int)(avail < (unsigned long long)slots ? avail : (unsigned long long)slots);
        if (t < npieces) {
            const Piece pc = pieces[first + t];
            s_off[t] = pc.off;
            s_len[t] = pc.len;
            s_dst[t] = pc.dst;
        }
        __syncthreads();

        // gather: slot i of X keys holds piece i, padded with the maximum
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int p = t + NT * k;
            const int slot = p >> xlog, j = p & ((1 << xlog) - 1);
            T x = Traits<T>::kMax;
            if (slot < npieces && j < s_len[slot])
                x = load_elem<T>(ik, iv, s_off[slot] + j);
            Z[p] = x;
        }
        __syncthreads();
        T v[R];
        const LdsSkew<T> W{S, wave * (64 * R) + logical_lane(lane) * R};
#pragma unroll
        for (int r = 0; r < R; ++r)
            v[r] = W[r];
        __syncthreads();
        const int levels = xlog - P.r_log2;
        const int K = levels < wave_max ? levels : wave_max;
        sort_tile_core<R, NT>(S, v, t, K, levels - K);

#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int p = t + NT * k;
            const int slot = p >> xlog, j = p & ((1 << xlog) - 1);
            if (slot < npieces && j < s_len[slot]) {
                const bool scr = s_dst[slot] != 0;
                store_elem<T>(scr ? sk : ok, scr ? sv : ov, s_off[slot] + j, Z[p]);
            }
        }
        __syncthreads();
    }
}

// One wave per workgroup, one tile per lane.  In learned mode the model's
// CDF at a pair's four run endpoints is taken once per pair and wave, by the
// pair's first lane, and handed to the pair's other lanes.
template <typename T>
__global__ __launch_bounds__(64) void seg_corank_kernel(SegMap map, int64_t run, int64_t tm,
                                                         int64_t *__restrict__ cr, CorankCtl c)
{
    const int lane = threadIdx.x;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + lane;
    const bool valid = q < map.count();
    if (c.mode != 1 || run <= ((int64_t)8 << c.radius_log2)) {  // no prediction (find_corank)
        if (valid)
            tile_corank<T>(map, q, run, tm, cr, c);
        return;
    }
    // the pair of this tile: segment and pair base (the run pair index)
    int seg = -1;
    int64_t pb = -1;
    TileRef r{};
    PairGeo P{};
    if (valid) {
        r = map.at(q);
        P = pair_geo(r, tm, run);
        seg = map.entry(q).x;
        pb = P.pb;
    }
    const int prev = (lane + 63) & 63;
    const int pseg = __builtin_amdgcn_ds_bpermute(prev << 2, seg);
    const int pl = __builtin_amdgcn_ds_bpermute(prev << 2, (int)(uint32_t)pb);
    const int ph = __builtin_amdgcn_ds_bpermute(prev << 2, (int)(pb >> 32));
    const int64_t ppb = (int64_t)(uint32_t)pl | ((int64_t)ph << 32);
    const bool leader = valid && (lane == 0 || pseg != seg || ppb != pb);
    float4 f = make_float4(0.f, 0.f, 0.f, 0.f);
    if (leader && P.alen > 0) {
        const int32_t *ak = r.ik + r.base + P.pb;
        f = pair_cdf_of(c, ak, P.alen, ak + run, P.blen);
    }
    // each lane's leader: the highest leader lane at or below it
    const uint64_t lm = __builtin_amdgcn_ballot_w64(leader);
    const uint64_t below = lm & (lane == 63 ? ~0ull : ((2ull << lane) - 1));
    const int src = below ? 63 - __builtin_clzll(below) : lane;
    float4 g;
    g.x = __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(f.x)));
    g.y = __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(f.y)));
    g.z = __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(f.z)));
    g.w = __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(f.w)));
    if (valid)
        tile_corank<T>(map, q, run, tm, cr, c, &g);
}

template <int NT, int VT, typename T>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(merge_waves_per_simd<T, VT>())))
void seg_merge_kernel(SegMap map, int64_t run,
                                                       const int64_t *__restrict__ cr,
                                                       int64_t n_abs, int xcd_group)
{
    merge_pipe_body<NT, VT, T>(map, run, cr, n_abs, xcd_group);
}

int64_t a256(int64_t b) { return (b + 255) & ~(int64_t)255; }

__global__ void seg_status_kernel(const unsigned long long *ctrl, int64_t *out)
{
    if (threadIdx.x == 0) {
        out[0] = (int64_t)ctrl[C_OVER];
        out[1] = (int64_t)ctrl[C_SKIP];
        out[2] = (int64_t)ctrl[C_BAD];
    }
}

}  // namespace

hipError_t launch_seg_status(const void *ws, int64_t *out, hipStream_t s)
{
    hipLaunchKernelGGL(seg_status_kernel, dim3(1), dim3(64), 0, s,
                       (const unsigned long long *)ws, out);
    return hipGetLastError();
}

SegLayout seg_layout(int64_t n_total, int64_t nseg, int R, int NT, int TM, bool pairs, int ways)
{
    SegLayout L{};
    const int64_t tile = (int64_t)R * NT;
    const int64_t max_pieces = nseg + 2 * (n_total / tile) + 2;
    // full pieces and padded pieces of more than half a tile, all disjoint;
    // the half list: pieces of more than a quarter of a tile
    const int64_t max_full = 2 * (n_total / tile) + 2;
    const int64_t max_half = 4 * (n_total / tile) + 2;
    const int64_t max_tiles = n_total / TM + n_total / tile + 2;
    int64_t o = 0;
    L.ctrl = o;
    o += a256(C_WORDS * 8);
    L.pieces = o;
    o += a256(max_pieces * (int64_t)sizeof(Piece));
    L.fulls = o;  // the full list, then the half list
    o += a256((max_full + max_half) * (int64_t)sizeof(Piece));
    L.tiles = o;
    o += a256(max_tiles * 8);
    L.cr = o;
    o += a256((max_tiles + 1) * 8);
    if (ways == 4) {  // four-way tiles: a window-geometry record and an output index each
        L.rec = o;
        o += a256((max_tiles + 1) * (int64_t)merge4_record_bytes());
        L.obase = o;
        o += a256((max_tiles + 1) * 8);
    }
    L.passes = o;
    o += a256(nseg * 4);
    L.table = o;  // the learned co-rank's model table (used in learned mode)
    o += kCdfTableBytes;
    L.scr_k = o;
    o += a256(n_total * 4);
    L.scr_v = o;
    if (pairs)
        o += a256(n_total * 4);
    L.total = o;
    L.max_tiles = max_tiles;
    L.max_pieces = max_pieces;
    L.max_full = max_full;
    L.max_half = max_half;
    return L;
}

template <int R, int NT, typename T>
static hipError_t launch_seg_block(const SegParams &P, unsigned long long *ctrl, const Piece *pieces,
                                   const int32_t *ik, const int32_t *iv, int32_t *ok, int32_t *ov,
                                   int32_t *sk, int32_t *sv, int wave_max, hipStream_t s)
{
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void *)seg_block_kernel<R, NT, T>,
                                                     NT, 0) != hipSuccess ||
        occ <= 0)
        occ = 1;
    const unsigned grid = (unsigned)(device_cus() * occ);
    hipLaunchKernelGGL((seg_block_kernel<R, NT, T>), dim3(grid), dim3(NT), 0, s, P, ctrl, pieces,
                       ik, iv, ok, ov, sk, sv, wave_max);
    return hipGetLastError();
}

template <int NT, int VT, typename T>
static hipError_t launch_seg_merge(const SegMap &map, int64_t run, const int64_t *cr,
                                   int64_t n_abs, int64_t max_tiles, int occupancy, bool xcd,
                                   hipStream_t s)
{
    int occ = occupancy;
    if (occ <= 0 &&
        (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void *)seg_merge_kernel<NT, VT, T>,
                                                      NT, 0) != hipSuccess ||
         occ <= 0))
        occ = 1;
    int64_t grid = (int64_t)device_cus() * occ;
    if (grid > max_tiles)
        grid = max_tiles;
    if (xcd)
        grid = ((grid + 7) / 8) * 8;
    hipLaunchKernelGGL((seg_merge_kernel<NT, VT, T>), dim3((unsigned)grid), dim3(NT), 0, s, map,
                       run, cr, n_abs, xcd ? 1 : 0);
    return hipGetLastError();
}

template <int R, int NT, typename T>
static hipError_t launch_seg_full(const unsigned long long *ctrl, const Piece *fulls,
                                  int64_t max_full, int64_t max_half, const SegArgs &a,
                                  int32_t *sk, int32_t *sv, hipStream_t s)
{
    // one workgroup per possible full-list piece and per possible pair of
    // half-list pieces; those past the counts exit
    const int64_t grid = max_full + (max_half + 1) / 2;
    const int lanes_log2 = NT == 256 ? 8 : NT == 512 ? 9 : 10;
    hipLaunchKernelGGL((seg_full_kernel<R, NT, T>), dim3((unsigned)grid), dim3(NT), 0, s, 6,
                       lanes_log2 - 6, ctrl, fulls, fulls + max_full, a.kin, a.vin, a.kout, a.vout,
                       sk, sv);
    return hipGetLastError();
}

// The full-piece kernel's shape for a tile of `tile` keys: 32 keys per lane
// where the tile has at least 256 lanes of them, else fewer.
static hipError_t launch_seg_full_any(int64_t tile, bool pairs, const unsigned long long *ctrl,
                                      const Piece *fulls, int64_t max_full, int64_t max_half,
                                      const SegArgs &a, int32_t *sk, int32_t *sv, hipStream_t s)
{
    if (pairs) {
        switch (tile) {
        case 2048: return launch_seg_full<8, 256, int64_t>(ctrl, fulls, max_full, max_half, a, sk, sv, s);
        case 4096: return launch_seg_full<16, 256, int64_t>(ctrl, fulls, max_full, max_half, a, sk, sv, s);
        case 8192: return launch_seg_full<16, 512, int64_t>(ctrl, fulls, max_full, max_half, a, sk, sv, s);
        case 16384: return launch_seg_full<16, 1024, int64_t>(ctrl, fulls, max_full, max_half, a, sk, sv, s);
        }
    } else {
        switch (tile) {
        case 2048: return launch_seg_full<8, 256, int32_t>(ctrl, fulls, max_full, max_half, a, sk, sv, s);
        case 4096: return launch_seg_full<16, 256, int32_t>(ctrl, fulls, max_full, max_half, a, sk, sv, s);
        case 8192: return launch_seg_full<32, 256, int32_t>(ctrl, fulls, max_full, max_half, a, sk, sv, s);
        case 16384: return launch_seg_full<32, 512, int32_t>(ctrl, fulls, max_full, max_half, a, sk, sv, s);
        }
    }
    return hipErrorInvalidValue;
}

static hipError_t launch_seg_block_any(int R, int NT, bool pairs, const SegParams &P,
                                       unsigned long long *ctrl, const Piece *pieces, const SegArgs &a,
                                       int32_t *sk, int32_t *sv, hipStream_t s)
{
#define HVMS_SB(RR, NN)                                                                         \
    if (R == RR && NT == NN)                                                                    \
        return pairs ? launch_seg_block<RR, NN, int64_t>(P, ctrl, pieces, a.kin, a.vin, a.kout, \
                                                         a.vout, sk, sv, a.K, s)                 \
                     : launch_seg_block<RR, NN, int32_t>(P, ctrl, pieces, a.kin, a.vin, a.kout, \
                                                         a.vout, sk, sv, a.K, s);
    HVMS_SB(16, 256)
    HVMS_SB(16, 512)
    if (R == 16 && NT == 1024 && !pairs)  // the pair tile plus piece table exceeds LDS
        return launch_seg_block<16, 1024, int32_t>(P, ctrl, pieces, a.kin, a.vin, a.kout, a.vout,
                                                   sk, sv, a.K, s);
    HVMS_SB(8, 256)
    HVMS_SB(8, 512)
    HVMS_SB(8, 1024)
    HVMS_SB(32, 256)
    HVMS_SB(32, 512)
#undef HVMS_SB
    return hipErrorInvalidValue;
}

bool segmented_supported(int R, int NT, bool pairs)
{
    const long tile = (long)R * NT;
    const long lds = (pairs ? LdsSkew<int64_t>::size(tile) * 8 : LdsSkew<int32_t>::size(tile) * 4) +
                     (long)NT * 16 + 8;
    return block_sort_supported(R, NT, pairs) && lds <= 163840 && !(R == 32 && NT == 1024) &&
           R != 4;
}

hipError_t launch_segmented(const SegArgs &a, hipStream_t s)
{
    const bool pairs = a.vin != nullptr;
    const int64_t tile = (int64_t)a.R * a.NT;
    const int tile_log2 = ceil_log2_host(tile), r_log2 = ceil_log2_host(a.R);
    const SegLayout L = seg_layout(a.n_total, a.nseg, a.R, a.NT, a.TM, pairs, a.ways);
    SegParams P;
    P.off = a.off;
    P.nseg = a.nseg;
    P.n_total = a.n_total;
    P.max_pieces = L.max_pieces;
    P.max_tiles = L.max_tiles;
    P.max_full = L.max_full;
    P.max_half = L.max_half;
    P.tile_log2 = tile_log2;
    P.r_log2 = r_log2;
    P.nb = tile_log2 - r_log2 + 1;
    P.passes = a.passes;
    P.ways = a.ways;
    P.tm = a.TM;
    char *ws = (char *)a.ws;
    unsigned long long *ctrl = (unsigned long long *)(ws + L.ctrl);
    Piece *pieces = (Piece *)(ws + L.pieces);
    Piece *fulls = (Piece *)(ws + L.fulls);
    int2 *tiles = (int2 *)(ws + L.tiles);
    int64_t *cr = (int64_t *)(ws + L.cr);
    int32_t *passes = (int32_t *)(ws + L.passes);
    int32_t *sk = (int32_t *)(ws + L.scr_k);
    int32_t *sv = pairs ? (int32_t *)(ws + L.scr_v) : nullptr;

    hipLaunchKernelGGL(seg_init_kernel, dim3(1), dim3(256), 0, s, ctrl);
    const unsigned sb = (unsigned)((a.nseg + 255) / 256);
    hipLaunchKernelGGL(seg_count_kernel, dim3(sb), dim3(256), 0, s, P, ctrl);
    hipLaunchKernelGGL(seg_plan_kernel, dim3(1), dim3(64), 0, s, P, ctrl);
    hipLaunchKernelGGL(seg_scatter_kernel, dim3(sb), dim3(256), 0, s, P, ctrl, pieces, fulls,
                       fulls + L.max_full, tiles, passes);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;

    e = launch_seg_full_any(tile, pairs, ctrl, fulls, L.max_full, L.max_half, a, sk, sv, s);
    if (e != hipSuccess)
        return e;
    e = launch_seg_block_any(a.R, a.NT, pairs, P, ctrl, pieces, a, sk, sv, s);
    if (e != hipSuccess)
        return e;
    float *table = (float *)(ws + L.table);
    if (a.co.mode == HVMS_CORANK_LEARNED && a.passes > 0) {
        e = launch_cdf_table(a.co.cdf, table, s);
        if (e != hipSuccess)
            return e;
    }

    // co-ranks then merge over the two-way tiles of a map (run: the runs it
    // merges in pairs)
    auto two_way = [&](const SegMap &map, int64_t run, const CorankCtl &c) -> hipError_t {
        const unsigned cb = (unsigned)((L.max_tiles + 63) / 64);
        if (pairs)
            hipLaunchKernelGGL(seg_corank_kernel<int64_t>, dim3(cb), dim3(64), 0, s, map, run,
                               (int64_t)a.TM, cr, c);
        else
            hipLaunchKernelGGL(seg_corank_kernel<int32_t>, dim3(cb), dim3(64), 0, s, map, run,
                               (int64_t)a.TM, cr, c);
        hipError_t e2 = hipGetLastError();
        if (e2 != hipSuccess)
            return e2;
        const bool xcd = a.variant == 3;
        switch (a.TM) {
        case 2048:
            return pairs ? launch_seg_merge<256, 8, int64_t>(map, run, cr, a.n_total, L.max_tiles, a.occupancy, xcd, s)
                         : launch_seg_merge<256, 8, int32_t>(map, run, cr, a.n_total, L.max_tiles, a.occupancy, xcd, s);
        case 4096:
            return pairs ? launch_seg_merge<256, 16, int64_t>(map, run, cr, a.n_total, L.max_tiles, a.occupancy, xcd, s)
                         : launch_seg_merge<256, 16, int32_t>(map, run, cr, a.n_total, L.max_tiles, a.occupancy, xcd, s);
        case 8192:
            return pairs ? launch_seg_merge<512, 16, int64_t>(map, run, cr, a.n_total, L.max_tiles, a.occupancy, xcd, s)
                         : launch_seg_merge<512, 16, int32_t>(map, run, cr, a.n_total, L.max_tiles, a.occupancy, xcd, s);
        case 16384:
            return pairs ? hipErrorInvalidValue
                         : launch_seg_merge<512, 32, int32_t>(map, run, cr, a.n_total, L.max_tiles, a.occupancy, xcd, s);
        }
        return hipErrorInvalidValue;
    };

    for (int p = 0; p < a.passes; ++p) {
        SegMap map;
        map.outk = a.kout;
        map.outv = a.vout;
        map.scrk = sk;
        map.scrv = sv;
        map.off = a.off;
        map.tiles = tiles;
        map.passes = passes;
        map.pass_tiles = (const int64_t *)(ctrl + C_PASS);
        map.first_tiles = nullptr;
        map.p = p;
        CorankCtl c;
        c.mode = a.co.mode;
        c.radius_log2 = a.co.radius_log2;
        c.cdf = a.co.cdf;
        c.stats = a.co.stats;
        c.pair_cdf = nullptr;
        c.pair_first = 0;
        c.table = a.co.mode == HVMS_CORANK_LEARNED ? table : nullptr;
        if (a.ways != 4) {
            e = two_way(map, tile << p, c);
            if (e != hipSuccess)
                return e;
            continue;
        }
        // four-way launch p: runs of TILE * 4^p; first the four-way tiles
        // (their co-rank records, then the merge), then the two-way tiles of
        // the segments with one level left
        const int64_t run = tile << (2 * p);
        SegMap m4 = map;
        m4.pass_tiles = (const int64_t *)(ctrl + C_PASSF);
        e = launch_seg_merge4(a.TM, pairs, m4, run, ws + L.rec, (int64_t *)(ws + L.obase),
                              L.max_tiles, a.n_total, c.stats, a.occupancy, s);
        if (e != hipSuccess)
            return e;
        SegMap m2 = map;
        m2.first_tiles = (const int64_t *)(ctrl + C_PASSF);
        e = two_way(m2, run, c);
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace hvms
