// Four-way merge pass: two merge levels per trip through HBM.
//
// A pass with run length L merges every group of four consecutive runs
// A, B, C, D into one run of 4L: the output is (A merge B) merge (C merge D),
// each merge taking its first operand on ties, i.e. the order (key, run).
// Output tile g covers [g*TM, (g+1)*TM) of its group.  Its windows follow from
// three co-ranks of its first diagonal d: x = number of X = A(+)B elements
// among the first d outputs of X (+) Y (Y = C(+)D), a = co-rank of x in A(+)B,
// c = co-rank of d - x in C(+)D.  X and Y are never stored.  The three
// follow from the shares of A, B, C and D among the group's d smallest
// elements, which the co-rank kernel selects in the four runs directly
// (select4: one round of independent reads per halving of a stride, no
// nested searches).  The co-rank kernel turns the co-ranks of a tile's
// first and next diagonals into the
// tile's window geometry, one 64-byte record per tile, so that the merge
// kernel's waves do no 64-bit geometry arithmetic of their own.  The merge
// kernel loads the four windows (TM elements together), merges A with B and
// C with D in LDS, then the two results, and writes a full tile from
// registers (each thread's outputs are consecutive) and the array's ragged
// last tile through LDS with coalesced stores.
#include "hvms_internal.h"
#include "merge_common.h"

namespace hvms {

namespace {

// One virtual run V = P (+) Q of two sorted arrays (P first on ties).
struct VRun {
    const int32_t *pk, *pv, *qk, *qv;
    int64_t np, nq;
};

struct Quad {
    int64_t x, a, c;  // co-ranks of a tile's first diagonal
};

template <typename T> struct Group {
    VRun X, Y;
    int64_t gb;  // absolute index of the group's first element
};

template <typename T>
__device__ __forceinline__ Group<T> group_of(const int32_t *k, const int32_t *v, int64_t n,
                                             int64_t run, int64_t gq)
{
    Group<T> G;
    G.gb = gq * 4 * run;
    int64_t len[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t s = G.gb + r * run;
        len[r] = s >= n ? 0 : (n - s < run ? n - s : run);
    }
    const int32_t *vb = v ? v + G.gb : nullptr;
    G.X.pk = k + G.gb;
    G.X.pv = vb;
    G.X.qk = k + G.gb + run;
    G.X.qv = vb ? vb + run : nullptr;
    G.X.np = len[0];
    G.X.nq = len[1];
    G.Y.pk = k + G.gb + 2 * run;
    G.Y.pv = vb ? vb + 2 * run : nullptr;
    G.Y.qk = k + G.gb + 3 * run;
    G.Y.qv = vb ? vb + 3 * run : nullptr;
    G.Y.np = len[2];
    G.Y.nq = len[3];
    return G;
}

// Selection among four windows of the runs A, B, C, D (window r holds the
// elements [0, W_r) of its run from some base on): how many elements of each
// window are among the D smallest of their union, in the order of the
// four-way merge, (key, run) for keys and (key, value, run) for pairs.  Past
// its end a window reads as a sentinel, after every element, sentinels of
// different windows ordered by r.  Keys become one 64-bit word
// (key << 2 | r); a pair keeps its key, run and a pointer to its value, read
// only when two keys tie.
template <typename T> struct SelE;
template <> struct SelE<int32_t> {
    int64_t w;
};
template <> struct SelE<int64_t> {
    int32_t key, r;
    const int32_t *vp;  // nullptr: the sentinel
};
__device__ __forceinline__ bool sel_less(const SelE<int32_t> &a, const SelE<int32_t> &b)
{
    return a.w < b.w;
}
__device__ __forceinline__ bool sel_less(const SelE<int64_t> &a, const SelE<int64_t> &b)
{
    if (!a.vp || !b.vp)
        return !b.vp && (a.vp || a.r < b.r);
    if (a.key != b.key)
        return a.key < b.key;
    const int32_t va = *a.vp, vb = *b.vp;
    if (va != vb)
        return va < vb;
    return a.r < b.r;
}
template <typename T> struct SelWin {
    const int32_t *k, *v;  // the window's first element
    int64_t W;
    __device__ __forceinline__ SelE<T> sentinel(int r) const
    {
        if constexpr (sizeof(T) == 8)
            return SelE<T>{0, r, nullptr};
        else
            return SelE<T>{((int64_t)1 << 40) | r};
    }
    __device__ __forceinline__ SelE<T> at(int r, int64_t j) const
    {
        if (j >= W)
            return sentinel(r);
        if constexpr (sizeof(T) == 8)
            return SelE<T>{k[j], r, v + j};
        else
            return SelE<T>{((int64_t)k[j] << 2) | r};
    }
};

// Counts (w_0..w_3) of the D smallest elements of four windows (D at most
// the sum of their widths).  Stride halving: at stride s the samples of a
// window are its elements at positions j*s - 1, and the selection at that
// stride is the floor(D / s) smallest samples (w_r of them in window r, the
// first w_r of its samples); at s = 1 that is the answer.  From stride 2s
// to s, every selected sample brings the sample before it, and outside
// those only the sample after each window's last selected one (its
// candidate c_r) can lie below the largest selected sample y, so the
// samples up to y are the 2 * old count plus the candidates below y; the
// new count floor(D / s) is within one of twice the old one, so at most
// three of them go again (the largest first) or the smallest candidate
// joins.  Each level reads the four candidates and the sample before each
// window's top together (the top's replacement after a removal), so a
// level costs one round of independent loads; a second removal from one
// window (rare) reads one more.  About log2(width) + 1 rounds in all,
// against log2(width)^2 / 2 for the nested bisection.
// Strides below which the sample before a window's top is read ahead with
// the candidates: there it shares a cache line with the top.  At larger
// strides reading it ahead doubles the lines a level fetches, and the kernel
// is bound by those line fetches; a removal then reads it when needed.
constexpr int64_t kSelReadAhead = 32;
template <typename T>
__device__ __forceinline__ void select4(const SelWin<T> (&S)[4], int64_t D, int64_t (&w)[4],
                                        unsigned &probes)
{
    using E = SelE<T>;
    int64_t mw = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        w[r] = 0;
        mw = S[r].W > mw ? S[r].W : mw;
    }
    const int lgL = mw <= 1 ? 0 : 64 - __builtin_clzll((uint64_t)(mw - 1));
    E top[4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
        top[r] = S[r].sentinel(r);
    for (int lg = lgL; lg >= 0; --lg) {
        const int64_t s = (int64_t)1 << lg;
        const int64_t tn = D >> lg;
        int64_t b2[4];
        E c[4], p[4], ot[4];
        bool any = false, ld = false;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            b2[r] = 2 * w[r];
            w[r] = b2[r];
            ot[r] = top[r];
            const int64_t jc = (b2[r] + 1) * s - 1, jp = (b2[r] - 1) * s - 1;
            c[r] = S[r].at(r, jc);
            p[r] = (b2[r] > 0 && s < kSelReadAhead) ? S[r].at(r, jp) : S[r].sentinel(r);
            ld |= jc < S[r].W || (b2[r] > 0 && s < kSelReadAhead && jp < S[r].W);
            any |= b2[r] > 0;
        }
        probes += ld ? 1u : 0u;
        int64_t cnt = 0;
        if (any) {
            E y = S[0].sentinel(0);
            bool have = false;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (w[r] > 0 && (!have || sel_less(y, top[r]))) {
                    y = top[r];
                    have = true;
                }
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (sel_less(c[r], y)) {
                    w[r] += 1;
                    top[r] = c[r];
                }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
            cnt += w[r];
        for (; cnt > tn; --cnt) {  // at most three times
            int rm = -1;
            E m = S[0].sentinel(0);
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (w[r] > 0 && (rm < 0 || sel_less(m, top[r]))) {
                    rm = r;
                    m = top[r];
                }
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (r == rm) {
                    w[r] -= 1;
                    const int64_t q = w[r] - b2[r];
                    if (w[r] > 0) {
                        if (q == 0)
                            top[r] = ot[r];
                        else if (q == -1 && s < kSelReadAhead)
                            top[r] = p[r];
                        else {
                            ++probes;
                            top[r] = S[r].at(r, w[r] * s - 1);
                        }
                    }
                }
        }
        for (; cnt < tn; ++cnt) {  // one candidate, or up to four at the first level
            int ra = -1;
            E m = S[0].sentinel(0);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                // past the candidate only the first level gets here, where
                // the next sample lies past the window: a sentinel
                const E nx = w[r] == b2[r] ? c[r] : S[r].sentinel(r);
                if (ra < 0 || sel_less(nx, m)) {
                    ra = r;
                    m = nx;
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (r == ra) {
                    w[r] += 1;
                    top[r] = m;
                }
        }
    }
}

// Co-ranks (x, a, c) of diagonal d of X (+) Y: the shares of A, B, C and D
// among the d smallest elements of the group, selected in the four whole
// runs (x = a + b: X's share).
// When the four runs' ranges do not overlap in run order (presorted input)
// or in reverse run order (reverse-sorted input, or each run one value), the
// merge is their concatenation in that order and the shares follow from d
// directly: one round of reads of the runs' end elements (shared by all
// tiles of a group) instead of the selection.
template <typename T>
__device__ __forceinline__ Quad quad_corank(const Group<T> &G, int64_t d, unsigned &probes)
{
    SelWin<T> S[4];
    S[0] = SelWin<T>{G.X.pk, G.X.pv, G.X.np};
    S[1] = SelWin<T>{G.X.qk, G.X.qv, G.X.nq};
    S[2] = SelWin<T>{G.Y.pk, G.Y.pv, G.Y.np};
    S[3] = SelWin<T>{G.Y.qk, G.Y.qv, G.Y.nq};
    using E = SelE<T>;
    E first[4], last[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        first[r] = S[r].at(r, 0);  // an empty run's reads are sentinels (no load)
        last[r] = S[r].W > 0 ? S[r].at(r, S[r].W - 1) : S[r].sentinel(r);
    }
    ++probes;
    bool up = true, down = true, hu = false, hd = false;
    E lu = first[0], ld = first[0];
#pragma unroll
    for (int r = 0; r < 4; ++r)  // every element of an earlier run before every later one
        if (S[r].W > 0) {
            if (hu)
                up = up && sel_less(lu, first[r]);
            lu = last[r];
            hu = true;
        }
#pragma unroll
    for (int r = 3; r >= 0; --r)  // ... or of a later run before every earlier one
        if (S[r].W > 0) {
            if (hd)
                down = down && sel_less(ld, first[r]);
            ld = last[r];
            hd = true;
        }
    int64_t w[4];
    if (up || down) {
        int64_t rem = d;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int r = up ? k : 3 - k;
            int64_t take = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (q == r)
                    take = rem < S[q].W ? rem : S[q].W;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (q == r)
                    w[q] = take;
            rem -= take;
        }
    } else {
        select4<T>(S, d, w, probes);
    }
    return Quad{w[0] + w[1], w[0], w[2]};
}

struct Tile4 {
    int64_t gb, o0;       // group start (absolute), first output (group-relative)
    int64_t al[4];        // absolute index of the first chunk of each window
    int cnt, nx;          // outputs; of them from X = A (+) B
    int len[4], off[4];   // window lengths, offset of window start in its first chunk
    int nch[4], base[4];  // chunks per window, LDS index of window element 0
};

// Window geometry of tile g from the co-ranks of its first and next
// diagonals, clamped so that every window stays inside its run and the four
// lengths add up to the tile even if the runs were not sorted.  abs0: the
// absolute index of the sequence's first element (a segment's offset; 0 for
// a whole array), so that chunks are aligned in absolute index.
template <typename T>
__device__ __forceinline__ Tile4 tile4_geo(const Group<T> &G, int64_t run, int64_t tm, int64_t g,
                                           Quad q0, Quad q1, int64_t abs0 = 0)
{
    Tile4 t;
    const int64_t nA = G.X.np, nB = G.X.nq, nC = G.Y.np, nD = G.Y.nq;
    const int64_t nx = nA + nB, ny = nC + nD;
    t.gb = G.gb;
    t.o0 = g * tm - G.gb;
    const int64_t d0 = t.o0;
    const int64_t d1 = d0 + tm < nx + ny ? d0 + tm : nx + ny;
    if (d1 == nx + ny) {
        q1.x = nx;
        q1.a = nA;
        q1.c = nC;
    }
    auto cl = [](int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); };
    const int64_t x0 = cl(q0.x, d0 > ny ? d0 - ny : 0, d0 < nx ? d0 : nx);
    int64_t x1 = cl(q1.x, d1 > ny ? d1 - ny : 0, d1 < nx ? d1 : nx);
    x1 = cl(x1, x0, x0 + (d1 - d0));
    const int64_t a0 = cl(q0.a, x0 > nB ? x0 - nB : 0, x0 < nA ? x0 : nA);
    int64_t a1 = cl(q1.a, x1 > nB ? x1 - nB : 0, x1 < nA ? x1 : nA);
    a1 = cl(a1, a0, a0 + (x1 - x0));
    const int64_t y0 = d0 - x0, y1 = d1 - x1;
    const int64_t c0 = cl(q0.c, y0 > nD ? y0 - nD : 0, y0 < nC ? y0 : nC);
    int64_t c1 = cl(q1.c, y1 > nD ? y1 - nD : 0, y1 < nC ? y1 : nC);
    c1 = cl(c1, c0, c0 + (y1 - y0));
    const int64_t start[4] = {abs0 + G.gb + a0, abs0 + G.gb + run + (x0 - a0),
                              abs0 + G.gb + 2 * run + c0, abs0 + G.gb + 3 * run + (y0 - c0)};
    const int64_t len[4] = {a1 - a0, (x1 - a1) - (x0 - a0), c1 - c0, (y1 - c1) - (y0 - c0)};
    t.cnt = (int)(d1 - d0);
    t.nx = (int)(x1 - x0);
    int chunks = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        t.al[r] = start[r] & ~(int64_t)3;
        t.off[r] = (int)(start[r] - t.al[r]);
        t.len[r] = (int)len[r];
        t.nch[r] = len[r] ? (t.off[r] + t.len[r] + 3) >> 2 : 0;
        t.base[r] = 4 * chunks + t.off[r];
        chunks += t.nch[r];
    }
    return t;
}


// A tile's window geometry as the merge kernel reads it: one 64-byte record
// per tile, written by the co-rank kernel, so that the merge kernel's waves
// do no 64-bit geometry arithmetic of their own.  w: len0 | len1 << 16,
// len2 | len3 << 16, base0 | base1 << 16, base2 | base3 << 16, c1 | c2 << 16,
// c3 | nc << 16 (c_r: first chunk of window r, nc: chunks in all), cnt, nx.
struct TileRec {
    int64_t dl[4];  // chunk c of window r starts at absolute index 4c + dl[r]
    uint32_t w[8];
};

// The record as the merge kernel holds it (wave-uniform); ob: a segmented
// tile's first output index, with bit 62 set when the segment's data sits
// in scratch (read scratch, write the output arrays)
struct TileW {
    int64_t dl[4];
    int cnt, nx;
    int len[4], base[4];
    int c1, c2, c3, nc;
    int64_t ob;
};
static_assert(sizeof(TileRec) == 64, "one 64-byte record per tile");

__device__ __forceinline__ TileRec tile_rec_of(const Tile4 &t)
{
    TileRec r;
    const int c1 = t.nch[0], c2 = c1 + t.nch[1], c3 = c2 + t.nch[2], nc = c3 + t.nch[3];
    r.dl[0] = t.al[0];
    r.dl[1] = t.al[1] - 4 * c1;
    r.dl[2] = t.al[2] - 4 * c2;
    r.dl[3] = t.al[3] - 4 * c3;
    r.w[0] = (uint32_t)t.len[0] | ((uint32_t)t.len[1] << 16);
    r.w[1] = (uint32_t)t.len[2] | ((uint32_t)t.len[3] << 16);
    r.w[2] = (uint32_t)t.base[0] | ((uint32_t)t.base[1] << 16);
    r.w[3] = (uint32_t)t.base[2] | ((uint32_t)t.base[3] << 16);
    r.w[4] = (uint32_t)c1 | ((uint32_t)c2 << 16);
    r.w[5] = (uint32_t)c3 | ((uint32_t)nc << 16);
    r.w[6] = (uint32_t)t.cnt;
    r.w[7] = (uint32_t)t.nx;
    return r;
}

// One wave per workgroup; lane l searches the co-ranks of tile 63 * wave +
// l, and lanes 0..62 each write their tile's record, taking the next
// tile's co-ranks from the next lane (lane 63 searches the first tile of
// the following wave for lane 62, so every wave has all it needs).
template <typename T>
__global__ __launch_bounds__(64) void quad_corank_kernel(const int32_t *__restrict__ kin,
                                                          const int32_t *__restrict__ vin,
                                                          int64_t n, int64_t run, int64_t tm,
                                                          int64_t ntiles, int lg4run,
                                                          TileRec *__restrict__ out,
                                                          unsigned long long *stats)
{
    const int l = threadIdx.x;
    const int64_t g = (int64_t)blockIdx.x * 63 + l;
    Quad q{0, 0, 0};
    Group<T> G{};
    if (g < ntiles) {
        const int64_t o0 = g * tm;
        G = group_of<T>(kin, vin, n, run, o0 >> lg4run);
        unsigned probes = 0;
        q = quad_corank<T>(G, o0 - G.gb, probes);
        if (stats && l < 63) {
            atomicAdd(stats + 0, 1ull);
            atomicAdd(stats + 1, (unsigned long long)probes);
            atomicAdd(stats + 8 + (probes < 63 ? probes : 63), 1ull);
        }
    }
    // the next tile's co-ranks (for the array's last tile they are unused:
    // its end is its group's end)
    auto next = [&](int64_t v) {
        const int a = ((l + 1) & 63) << 2;
        const int lo = __builtin_amdgcn_ds_bpermute(a, (int)(uint32_t)v);
        const int hi = __builtin_amdgcn_ds_bpermute(a, (int)(v >> 32));
        return (int64_t)(uint32_t)lo | ((int64_t)hi << 32);
    };
    Quad q1;
    q1.x = next(q.x);
    q1.a = next(q.a);
    q1.c = next(q.c);
    if (l < 63 && g < ntiles)
        out[g] = tile_rec_of(tile4_geo<T>(G, run, tm, g, q, q1));
}

// The same for the four-way tiles of a segmented pass: tile q of the list is
// tile j of its segment.  Each record's chunk bases are absolute;
// obase[q] is the tile's first output index, bit 62 marking a segment whose
// data sits in scratch.
template <typename T>
__global__ __launch_bounds__(64) void seg_quad_corank_kernel(SegMap map, int64_t run, int64_t tm,
                                                              int lg4run,
                                                              TileRec *__restrict__ out,
                                                              int64_t *__restrict__ obase,
                                                              unsigned long long *stats)
{
    const int l = threadIdx.x;
    const int64_t q = (int64_t)blockIdx.x * 63 + l;
    const int64_t cnt = map.count();
    Quad qd{0, 0, 0};
    Group<T> G{};
    int64_t base = 0, o0 = 0;
    int j = 0;
    bool odd = false;
    if (q < cnt) {
        const int2 e = map.entry(q);
        base = map.off[e.x];
        const int64_t len = map.off[e.x + 1] - base;
        j = e.y;
        odd = ((map.passes[e.x] - map.p) & 1) != 0;
        const int32_t *ik = odd ? map.scrk : map.outk;
        const int32_t *iv = odd ? map.scrv : map.outv;
        o0 = (int64_t)j * tm;
        G = group_of<T>(ik + base, iv ? iv + base : nullptr, len, run, o0 >> lg4run);
        unsigned probes = 0;
        qd = quad_corank<T>(G, o0 - G.gb, probes);
        if (stats && l < 63) {
            atomicAdd(stats + 0, 1ull);
            atomicAdd(stats + 1, (unsigned long long)probes);
            atomicAdd(stats + 8 + (probes < 63 ? probes : 63), 1ull);
        }
    }
    // the next tile's co-ranks (used only when it is the next tile of the
    // same group, which is then the next entry of the list)
    auto next = [&](int64_t v) {
        const int a = ((l + 1) & 63) << 2;
        const int lo = __builtin_amdgcn_ds_bpermute(a, (int)(uint32_t)v);
        const int hi = __builtin_amdgcn_ds_bpermute(a, (int)(v >> 32));
        return (int64_t)(uint32_t)lo | ((int64_t)hi << 32);
    };
    Quad q1;
    q1.x = next(qd.x);
    q1.a = next(qd.a);
    q1.c = next(qd.c);
    if (l < 63 && q < cnt) {
        out[q] = tile_rec_of(tile4_geo<T>(G, run, tm, j, qd, q1, base));
        obase[q] = (base + o0) | ((int64_t)odd << 62);
    }
}

// VT consecutive outputs of one thread from registers to absolute index e
// (a multiple of 4), as 16-byte stores; pairs are split into the key and
// value arrays, or stored whole when the output is packed (PK).
template <int VT, typename T, bool PK>
__device__ __forceinline__ void store_run(int32_t *__restrict__ k, int32_t *__restrict__ v,
                                          int64_t e, const T (&x)[VT])
{
#pragma unroll
    for (int q = 0; q < VT; q += 4) {
        if constexpr (sizeof(T) == 4) {
            *(int4 *)(k + e + q) = make_int4(x[q], x[q + 1], x[q + 2], x[q + 3]);
        } else if constexpr (PK) {
            typedef int64_t V2 __attribute__((ext_vector_type(2)));
            V2 *o = (V2 *)((int64_t *)k + e + q);
            o[0] = V2{x[q], x[q + 1]};
            o[1] = V2{x[q + 2], x[q + 3]};
        } else {
            *(int4 *)(k + e + q) =
                make_int4(pair_key(x[q]), pair_key(x[q + 1]), pair_key(x[q + 2]), pair_key(x[q + 3]));
            *(int4 *)(v + e + q) =
                make_int4(pair_val(x[q]), pair_val(x[q + 1]), pair_val(x[q + 2]), pair_val(x[q + 3]));
        }
    }
}

// PK: the output is one packed 64-bit array at kout (the last pass of a
// 64-bit key sort).  SEG: the four-way tiles of a segmented pass: their
// count is read from *seg_count, and each tile's record comes with its first
// output index and the side its segment's data sits on (obase): kin/vin are
// then the output arrays and scrk/scrv the scratch ones, read or written per
// tile, and a tile whose first output is not 16-byte aligned leaves through
// LDS with chunk-aligned stores.
template <int NT, int VT, typename T, bool PK = false, bool SEG = false>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void merge4_pipe_kernel(const int32_t *__restrict__ kin,
                                                         const int32_t *__restrict__ vin,
                                                         int32_t *__restrict__ kout,
                                                         int32_t *__restrict__ vout, int64_t n,
                                                         int64_t run, const TileRec *__restrict__ rec,
                                                         int64_t ntiles, int lg4run, KeyMap xout,
                                                         const int64_t *__restrict__ obase,
                                                         int32_t *scrk, int32_t *scrv,
                                                         const int64_t *seg_count)
{
    constexpr int TM = NT * VT;
    constexpr int CH = VT / 4 + 1;  // chunk slots per thread: TM/4 + 6 chunks at most
    // S: the four windows (TM elements, up to 24 of chunk alignment, and
    // up to VT + 2 read past a window's end by reg_merge); M: the level-1
    // output in the skewed layout, so that rows of VT written by consecutive
    // threads fall in distinct banks (its 8 spare slots: the reads past Y's
    // sentinels)
    __shared__ __attribute__((aligned(16))) T S[TM + 32 + VT];
    __shared__ __attribute__((aligned(16))) T M[LdsSkew<T>::size(TM + 2 * VT + 8)];
    const int t = threadIdx.x;
    const int64_t first = blockIdx.x, step = gridDim.x;
    const int64_t last = SEG ? *seg_count : ntiles;
    if (first >= last)
        return;

    // tile g's record: one 32-bit word per lane 0..15 (a vector load, so
    // that waiting for it never waits for LDS traffic), and for a segmented
    // tile its output index in lanes 16 and 17
    const uint32_t *words = (const uint32_t *)rec;
    auto load_rec = [&](int64_t g) -> uint32_t {
        if constexpr (SEG) {
            const int l = t & 31;
            if (l >= 16)
                return l < 18 ? ((const uint32_t *)obase)[2 * g + (l & 1)] : 0u;
        }
        return words[g * 16 + (t & 15)];
    };
    auto geo_of = [&](uint32_t rv) {
        auto rl = [&](int lane) { return (uint32_t)__builtin_amdgcn_readlane((int)rv, lane); };
        TileW w;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            w.dl[r] = (int64_t)((uint64_t)rl(2 * r) | ((uint64_t)rl(2 * r + 1) << 32));
        const uint32_t l01 = rl(8), l23 = rl(9), b01 = rl(10), b23 = rl(11), c12 = rl(12),
                       c3n = rl(13);
        w.len[0] = (int)(l01 & 0xffff);
        w.len[1] = (int)(l01 >> 16);
        w.len[2] = (int)(l23 & 0xffff);
        w.len[3] = (int)(l23 >> 16);
        w.base[0] = (int)(b01 & 0xffff);
        w.base[1] = (int)(b01 >> 16);
        w.base[2] = (int)(b23 & 0xffff);
        w.base[3] = (int)(b23 >> 16);
        w.c1 = (int)(c12 & 0xffff);
        w.c2 = (int)(c12 >> 16);
        w.c3 = (int)(c3n & 0xffff);
        w.nc = (int)(c3n >> 16);
        w.cnt = (int)rl(14);
        w.nx = (int)rl(15);
        w.ob = SEG ? (int64_t)((uint64_t)rl(16) | ((uint64_t)rl(17) << 32)) : 0;
        return w;
    };
    // a tile's input and output arrays, and its first output index.  The
    // choice between two arrays is made in integer arithmetic (a mask):
    // a select of pointers is turned by the compiler into a table in
    // scratch memory.
    auto pick = [](const void *a, const void *b, bool use_b) -> uintptr_t {
        const uintptr_t m = (uintptr_t)0 - (uintptr_t)use_b;
        return (uintptr_t)a ^ (((uintptr_t)a ^ (uintptr_t)b) & m);
    };
    auto src_k = [=](const TileW &G) -> const int32_t * {
        return SEG ? (const int32_t *)pick(kin, scrk, (G.ob >> 62) & 1) : kin;
    };
    auto src_v = [=](const TileW &G) -> const int32_t * {
        return SEG ? (const int32_t *)pick(vin, scrv, (G.ob >> 62) & 1) : vin;
    };
    auto dst_k = [=](const TileW &G) -> int32_t * {
        return SEG ? (int32_t *)pick(kout, scrk, !((G.ob >> 62) & 1)) : kout;
    };
    auto dst_v = [=](const TileW &G) -> int32_t * {
        return SEG ? (int32_t *)pick(vout, scrv, !((G.ob >> 62) & 1)) : vout;
    };
    auto out0 = [](const TileW &G, int64_t g) -> int64_t {
        return SEG ? (G.ob & ~((int64_t)1 << 62)) : g * TM;
    };

    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int64_t e_tail = n & ~(int64_t)3;
    const bool has_tail = (n & 3) != 0;
    auto chunk_elem = [&](const TileW &G, int c) -> int64_t {
        const int64_t d = c < G.c1 ? G.dl[0] : c < G.c2 ? G.dl[1] : c < G.c3 ? G.dl[2] : G.dl[3];
        return d + 4 * c;
    };
    auto total_chunks = [](const TileW &G) { return G.nc; };
    Chunk<T> pf[CH];
    auto prefetch = [&](const TileW &G) {
        const int nc = total_chunks(G);
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            if (NT * q + 64 * wave < nc) {
                const int c = t + NT * q;
                int64_t e = c < nc ? chunk_elem(G, c) : 0;
                e = (has_tail && e == e_tail) ? e_tail - 4 : e;
                pf[q] = load_chunk<T>(src_k(G), src_v(G), e);
            }
        }
    };

    // records stay undecoded in a VGPR until their tile comes up (rc: this
    // tile, rn: the next); the prefetch decodes only what it needs, so no
    // second decoded tile is held in scalar registers across the loop
    int64_t g = first;
    uint32_t rc = load_rec(g);
    prefetch(geo_of(rc));
    uint32_t rn = g + step < last ? load_rec(g + step) : 0;

    for (;;) {
        const TileW cur = geo_of(rc);
        // no barrier needed here: S was last read by level 1 of the previous
        // tile, and a barrier has followed it since
        const int nc = total_chunks(cur);
        // a full tile has at least TM/4 chunks: its first VT/4 slots need no
        // per-lane check (wave-uniform)
        const bool full = cur.cnt == TM;
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            const int c = t + NT * q;
            if ((full && q < VT / 4) || c < nc) {
                if (has_tail && chunk_elem(cur, c) == e_tail)
                    fix_tail<T>(pf[q], src_k(cur), src_v(cur), e_tail, n);
                put_chunk<T>(S, c, pf[q]);
            }
        }
        lds_barrier();

        const int64_t gn = g + step;
        const bool more = gn < last;
        const uint32_t rnext = rn;
        if (more) {
            prefetch(geo_of(rn));
            rn = gn + step < last ? load_rec(gn + step) : 0;
        }

        // a tile fed by one window only: no merging (tile-uniform branch)
        // (constant indices only: a runtime index would put cur in scratch)
        const int src = cur.len[0] == cur.cnt   ? cur.base[0]
                        : cur.len[1] == cur.cnt ? cur.base[1]
                        : cur.len[2] == cur.cnt ? cur.base[2]
                        : cur.len[3] == cur.cnt ? cur.base[3]
                                                : -1;
        if (src >= 0) {
            const int64_t o = out0(cur, g);
            const int sh = (int)(o & 3);
            if (full)  // constant count: no end checks
                copy_run<NT, CH, T, PK>(LdsPlain<T>{S, 0}, src, sh, dst_k(cur), dst_v(cur),
                                        o - sh, TM, t, xout);
            else
                copy_run<NT, CH, T, PK>(LdsPlain<T>{S, 0}, src, sh, dst_k(cur), dst_v(cur),
                                        o - sh, cur.cnt, t, xout);
            lds_barrier();  // the next tile's chunks overwrite S
            if (!more)
                break;
            g = gn;
            rc = rnext;
            continue;
        }

        // level 1: X = A (+) B into M[0, nx), Y = C (+) D into M[nx + VT,
        // cnt + VT), with VT sentinels (the maximum of the order) after each,
        // so that level 2 reads past either run's end without masks.
        // Thread t produces outputs [t*VT, t*VT + VT) of X followed by Y.
        // The row that crosses nx is cut at nx: its thread merges only the
        // X part, and the head of Y (fewer than VT outputs, from co-rank 0)
        // is computed by wave 0, one output per lane, so no thread runs two
        // merges while the others wait at the barrier.
        const int nxw = cur.nx, nyw = cur.cnt - cur.nx;
        {
            const int o = t * VT;
            if (full || o < cur.cnt) {
                const bool isx = o < nxw;
                const int diag = isx ? o : o - nxw;
                const int alen = isx ? cur.len[0] : cur.len[2];
                const int blen = isx ? cur.len[1] : cur.len[3];
                const int abase = isx ? cur.base[0] : cur.base[2];
                const int boff = (isx ? cur.base[1] : cur.base[3]) - abase;
                const LdsPlain<T> P{S, abase};
                const int i = lds_corank(P, alen, boff, blen, diag);
                T v[VT];
                reg_merge<VT>(P, alen, boff, blen, i, diag - i, v);
                const LdsSkew<T> MW{M, 0};
                // in a full tile only the row crossing nx is short, and the
                // register merge filled its slots past the X part with the
                // maximum of the order, the value the sentinel slots there
                // receive anyway: store every row whole
                if (full)
                    put_row<VT>(MW, isx ? o : o + VT, v, VT);
                else
                    put_row<VT>(MW, isx ? o : o + VT, v, (isx ? nxw : cur.cnt) - o);
            }
            // the head of Y in the row that crosses nx: outputs [0, hy) of
            // C (+) D; lane k finds output k by its co-rank (at most
            // log2(VT) + 1 steps) and one comparison
            const int os = nxw - nxw % VT;  // first output of the crossing row
            const int hy = (nxw % VT != 0 && nyw > 0)
                               ? (os + VT < cur.cnt ? os + VT : cur.cnt) - nxw
                               : 0;
            // wave 0: its lanes search the shortest diagonals, so it has
            // the slack to take this on before the barrier
            if (hy > 0 && (t >> 6) == 0) {  // wave-uniform
                const int k = t & 63;
                if (k < hy) {
                    const LdsPlain<T> Q{S, cur.base[2]};
                    const int dq = cur.base[3] - cur.base[2];
                    const int i = lds_corank(Q, cur.len[2], dq, cur.len[3], k);
                    const int j = k - i;
                    // both reads stay inside S (windows are followed by
                    // their chunk padding and VT spare slots)
                    const T cv = Q[i], dv = Q[dq + j];
                    const bool fromC = i < cur.len[2] && (j >= cur.len[3] || !(dv < cv));
                    const LdsSkew<T> MW{M, 0};
                    MW[nxw + VT + k] = fromC ? cv : dv;
                }
            }
            if (t < 2 * VT) {  // sentinels at [nx, nx + VT) and [cnt + VT, cnt + 2 VT)
                const LdsSkew<T> MW{M, 0};
                MW[t < VT ? nxw + t : cur.cnt + t] = Traits<T>::kMax;
            }
        }
        lds_barrier();

        // level 2: X (+) Y, reads past the runs' ends land on sentinels
        const LdsSkew<T> MX{M, 0};
        const int diag = t * VT < cur.cnt ? t * VT : cur.cnt;
        const int i = lds_corank(MX, nxw, nxw + VT, nyw, diag);
        T out[VT];
        reg_merge<VT, false>(MX, nxw, nxw + VT, nyw, i, diag - i, out);
        if (key_map_on(xout)) {  // wave-uniform: the last pass of a uint32 / float32 sort
#pragma unroll
            for (int k = 0; k < VT; ++k)
                out[k] = map_elem(out[k], xout);
        }
        // Every tile but the ragged last one of the array is full: each
        // thread's VT outputs are consecutive in the output, and it stores
        // them from registers (16-byte stores; a tile starts at a multiple
        // of TM).  No LDS is written after level 2, so neither barrier of
        // the staged copy is needed: the next tile writes S (last read
        // before this tile's second barrier) and then, after its first
        // barrier, M.  A ragged tile stages its rows in M (skewed) and
        // copies out the first cnt outputs.
        const int64_t o = out0(cur, g);
        if (full && (o & 3) == 0) {
            store_run<VT, T, PK>(dst_k(cur), dst_v(cur), o + diag, out);
        } else if (!SEG) {
            lds_barrier();
            put_row<VT>(MX, diag, out, cur.cnt - diag);
            lds_barrier();
            copy_out<NT, CH, T, PK>(MX, kout, vout, g * TM, cur.cnt, t);
        } else {  // a segmented tile not aligned to 16 bytes, or ragged
            lds_barrier();
            put_row<VT>(MX, diag, out, cur.cnt - diag);
            lds_barrier();
            const int sh = (int)(o & 3);
            copy_run<NT, CH, T, PK>(MX, 0, sh, dst_k(cur), dst_v(cur), o - sh, cur.cnt, t,
                                    xout);
        }
        if (!more)
            break;
        g = gn;
        rc = rnext;
    }
}

}  // namespace

// log2 of a power of two
static int ilog2_pow2(int64_t x)
{
    int l = 0;
    while (((int64_t)1 << l) < x)
        ++l;
    return l;
}

bool merge4_supported(int tm, bool pairs)
{
    return pairs ? (tm == 2048 || tm == 4096) : (tm == 4096 || tm == 8192 || tm == 16384);
}

size_t merge4_record_bytes() { return sizeof(TileRec); }

template <typename T>
static hipError_t launch_quad_corank(const int32_t *kin, const int32_t *vin, int64_t n,
                                     int64_t run, int64_t tm, void *rec,
                                     unsigned long long *stats, hipStream_t s)
{
    const int64_t ntiles = (n + tm - 1) / tm;
    // one thread per tile, one wave per workgroup: the tiles' selections
    // spread over all CUs (256-thread workgroups left half of them idle at
    // 2^28 keys and measured 3 % slower per sort)
    hipLaunchKernelGGL(quad_corank_kernel<T>, dim3((unsigned)((ntiles + 62) / 63)), dim3(64), 0,
                       s, kin, vin, n, run, tm, ntiles, ilog2_pow2(4 * run), (TileRec *)rec,
                       stats);
    return hipGetLastError();
}

template <int NT, int VT, typename T, bool PK>
static hipError_t launch_m4_1(const int32_t *kin, const int32_t *vin, int32_t *kout,
                              int32_t *vout, int64_t n, int64_t run, const void *rec,
                              int occupancy, hipStream_t s, KeyMap xout)
{
    const int64_t ntiles = (n + NT * VT - 1) / (NT * VT);
    int occ = occupancy;
    if (occ <= 0 &&
        (hipOccupancyMaxActiveBlocksPerMultiprocessor(
             &occ, (const void *)merge4_pipe_kernel<NT, VT, T, PK>, NT, 0) != hipSuccess ||
         occ <= 0))
        occ = 1;
    int64_t grid = (int64_t)device_cus() * occ;
    if (grid > ntiles)
        grid = ntiles;
    hipLaunchKernelGGL((merge4_pipe_kernel<NT, VT, T, PK>), dim3((unsigned)grid), dim3(NT), 0, s,
                       kin, vin, kout, vout, n, run, (const TileRec *)rec, ntiles, ilog2_pow2(4 * run),
                       xout, nullptr, nullptr, nullptr, nullptr);
    return hipGetLastError();
}

template <int NT, int VT, typename T>
static hipError_t launch_m4(const int32_t *kin, const int32_t *vin, int32_t *kout, int32_t *vout,
                            int64_t n, int64_t run, const void *rec, int occupancy, hipStream_t s,
                            KeyMap xout)
{
    if constexpr (sizeof(T) == 8) {
        if (xout.packed)
            return launch_m4_1<NT, VT, T, true>(kin, vin, kout, vout, n, run, rec, occupancy, s,
                                                xout);
    } else if (xout.packed) {
        return hipErrorInvalidValue;
    }
    return launch_m4_1<NT, VT, T, false>(kin, vin, kout, vout, n, run, rec, occupancy, s, xout);
}

hipError_t launch_merge4_corank(int tm, bool pairs, const int32_t *kin, const int32_t *vin,
                                int64_t n, int64_t run, void *rec, const CorankOpts &o,
                                hipStream_t s)
{
    // runs are powers of two (the kernels find a tile's group by a shift)
    if (!merge4_supported(tm, pairs) || run <= 0 || (run & (run - 1)) != 0 || (2 * run) % tm != 0)
        return hipErrorInvalidValue;
    return pairs ? launch_quad_corank<int64_t>(kin, vin, n, run, tm, rec, o.stats, s)
                 : launch_quad_corank<int32_t>(kin, nullptr, n, run, tm, rec, o.stats, s);
}

hipError_t launch_merge4_pass(int tm, bool pairs, const int32_t *kin, const int32_t *vin,
                              int32_t *kout, int32_t *vout, int64_t n, int64_t run,
                              const void *rec, int occupancy, hipStream_t s, KeyMap xout)
{
    if (run <= 0 || (run & (run - 1)) != 0 || (2 * run) % tm != 0)
        return hipErrorInvalidValue;
    switch (tm) {
    case 2048:
        return pairs ? launch_m4<256, 8, int64_t>(kin, vin, kout, vout, n, run, rec, occupancy, s, xout)
                     : hipErrorInvalidValue;
    case 4096:  // pairs: 512 threads x 8 (64-bit LDS tiles: the VGPRs of 8 outputs keep
                // four waves per SIMD, as many as the tile's LDS allows)
        return pairs ? launch_m4<512, 8, int64_t>(kin, vin, kout, vout, n, run, rec, occupancy, s, xout)
                     : launch_m4<256, 16, int32_t>(kin, vin, kout, vout, n, run, rec, occupancy, s, xout);
    case 8192:
        return pairs ? hipErrorInvalidValue
                     : launch_m4<512, 16, int32_t>(kin, vin, kout, vout, n, run, rec, occupancy, s, xout);
    case 16384:
        return pairs ? hipErrorInvalidValue
                     : launch_m4<1024, 16, int32_t>(kin, vin, kout, vout, n, run, rec, occupancy, s, xout);
    }
    return hipErrorInvalidValue;
}

template <int NT, int VT, typename T>
static hipError_t launch_m4_seg(const SegMap &map, int64_t n_total, int64_t run, const void *rec,
                                const int64_t *obase, int64_t max_tiles, int occupancy,
                                hipStream_t s)
{
    int occ = occupancy;
    if (occ <= 0 &&
        (hipOccupancyMaxActiveBlocksPerMultiprocessor(
             &occ, (const void *)merge4_pipe_kernel<NT, VT, T, false, true>, NT, 0) != hipSuccess ||
         occ <= 0))
        occ = 1;
    int64_t grid = (int64_t)device_cus() * occ;
    if (grid > max_tiles)
        grid = max_tiles;
    if (grid < 1)
        grid = 1;
    hipLaunchKernelGGL((merge4_pipe_kernel<NT, VT, T, false, true>), dim3((unsigned)grid), dim3(NT),
                       0, s, map.outk, map.outv, map.outk, map.outv, n_total, run,
                       (const TileRec *)rec, (int64_t)0, ilog2_pow2(4 * run), KeyMap{}, obase,
                       map.scrk, map.scrv, map.pass_tiles + map.p);
    return hipGetLastError();
}

hipError_t launch_seg_merge4(int tm, bool pairs, const SegMap &map, int64_t run, void *rec,
                             int64_t *obase, int64_t max_tiles, int64_t n_total,
                             unsigned long long *stats, int occupancy, hipStream_t s)
{
    if (!merge4_supported(tm, pairs) || run <= 0 || (run & (run - 1)) != 0 || (2 * run) % tm != 0 ||
        max_tiles <= 0)
        return hipErrorInvalidValue;
    const unsigned qb = (unsigned)((max_tiles + 62) / 63);
    const int lg = ilog2_pow2(4 * run);
    if (pairs)
        hipLaunchKernelGGL(seg_quad_corank_kernel<int64_t>, dim3(qb), dim3(64), 0, s, map, run,
                           (int64_t)tm, lg, (TileRec *)rec, obase, stats);
    else
        hipLaunchKernelGGL(seg_quad_corank_kernel<int32_t>, dim3(qb), dim3(64), 0, s, map, run,
                           (int64_t)tm, lg, (TileRec *)rec, obase, stats);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    switch (tm) {
    case 2048:
        return launch_m4_seg<256, 8, int64_t>(map, n_total, run, rec, obase, max_tiles, occupancy, s);
    case 4096:
        return pairs ? launch_m4_seg<512, 8, int64_t>(map, n_total, run, rec, obase, max_tiles, occupancy, s)
                     : launch_m4_seg<256, 16, int32_t>(map, n_total, run, rec, obase, max_tiles, occupancy, s);
    case 8192:
        return launch_m4_seg<512, 16, int32_t>(map, n_total, run, rec, obase, max_tiles, occupancy, s);
    case 16384:
        return launch_m4_seg<1024, 16, int32_t>(map, n_total, run, rec, obase, max_tiles, occupancy, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace hvms
