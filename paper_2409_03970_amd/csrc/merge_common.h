// Device code shared by the plain and the segmented merge passes: the
// merge-path co-rank search (plain binary search, or a model / linear
// prediction corrected by an exact bounded search), the geometry of an
// output tile, 16-byte chunk I/O, and the persistent pipelined merge body,
// all parameterised by a tile map that says where each output tile lives.
#pragma once

#include <type_traits>

#include "common.h"
#include "mlp_common.h"

namespace hvms {

// ------------------------------------------------------------ co-rank search

struct CorankCtl {
    int mode;          // HVMS_CORANK_*
    int radius_log2;   // bracket half-width for the bounded search
    const float *cdf;  // model parameters (learned mode)
    unsigned long long *stats;
    // learned mode: model values at the four run endpoints of each merge
    // pair (F(A[0]), F(A[m-1]), F(B[0]), F(B[k-1])), indexed by pair number
    // and shared by the pair's co-ranks; nullptr = evaluate in place
    const float4 *pair_cdf;
    int64_t pair_first;  // pair number of pair_cdf[0]
    // learned mode: the model sampled (cdf_lookup), or nullptr = evaluate it
    const float *table;
};

// P(i) := A[i] <= B[d-1-i]  (A-first merge takes A[i] before B[d-1-i]).  The
// co-rank is the first i in [lo, hi) where P is false, or hi.
template <typename T, typename FA, typename FB>
__device__ __forceinline__ int64_t binary_corank(FA A, FB B, int64_t d, int64_t lo, int64_t hi,
                                                 unsigned &probes)
{
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        ++probes;
        if (B(d - 1 - mid) < A(mid))
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// Prediction of the co-rank of diagonal d for runs A (m) and B (k).
//  linear:  d * m / (m + k);
//  learned: the model maps both runs' key ranges onto its CDF axis; inside
//           its range each run is taken as spread like the model's CDF, i.e.
//           its count below level u is m * clamp((u - fa0) / (fa1 - fa0)).
//           The level u* where the two counts add up to d gives the
//           prediction m * ramp_A(u*) (the breakpoints make this exact for
//           runs with disjoint key ranges).
template <typename FA, typename FB>
__device__ int64_t predict_corank(const CorankCtl &c, FA Akey, FB Bkey, int64_t m, int64_t k,
                                  int64_t d, const float4 *pre)
{
    if (c.mode != 1 || m == 0 || k == 0)
        return (int64_t)((double)d * (double)m / (double)(m + k));
    float fa0, fa1, fb0, fb1;
    if (pre) {
        fa0 = pre->x;
        fa1 = pre->y;
        fb0 = pre->z;
        fb1 = pre->w;
    } else if (c.table) {
        fa0 = cdf_lookup(c.table, Akey(0));
        fa1 = cdf_lookup(c.table, Akey(m - 1));
        fb0 = cdf_lookup(c.table, Bkey(0));
        fb1 = cdf_lookup(c.table, Bkey(k - 1));
    } else {
        fa0 = cdf_eval(c.cdf, key_to_unit(Akey(0)));
        fa1 = cdf_eval(c.cdf, key_to_unit(Akey(m - 1)));
        fb0 = cdf_eval(c.cdf, key_to_unit(Bkey(0)));
        fb1 = cdf_eval(c.cdf, key_to_unit(Bkey(k - 1)));
    }
    if (!(fa1 > fa0)) fa1 = fa0 + 1e-7f;
    if (!(fb1 > fb0)) fb1 = fb0 + 1e-7f;
    // total count at level u: piecewise linear, nondecreasing; find u* by
    // walking the sorted breakpoints.
    auto count = [&](float u, double &ca) {
        const double ra = fminf(fmaxf((u - fa0) / (fa1 - fa0), 0.0f), 1.0f);
        const double rb = fminf(fmaxf((u - fb0) / (fb1 - fb0), 0.0f), 1.0f);
        ca = ra * (double)m;
        return ca + rb * (double)k;
    };
    float bp[4] = {fa0, fa1, fb0, fb1};
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 3 - a; ++b)
            if (bp[b + 1] < bp[b]) {
                const float tmp = bp[b];
                bp[b] = bp[b + 1];
                bp[b + 1] = tmp;
            }
    double ca_prev = 0.0, tot_prev = count(bp[0], ca_prev);
    double pred = ca_prev;
    for (int q = 1; q < 4; ++q) {
        double ca;
        const double tot = count(bp[q], ca);
        if (tot >= (double)d) {
            const double w = tot > tot_prev ? ((double)d - tot_prev) / (tot - tot_prev) : 0.0;
            pred = ca_prev + w * (ca - ca_prev);
            break;
        }
        ca_prev = ca;
        tot_prev = tot;
        pred = ca;
    }
    return (int64_t)(pred + 0.5);
}

template <typename T, typename FA, typename FB, typename KA, typename KB>
__device__ int64_t find_corank(const CorankCtl &c, FA A, FB B, KA Akey, KB Bkey, int64_t m,
                               int64_t k, int64_t d, const float4 *pre = nullptr)
{
    const int64_t lo = d > k ? d - k : 0;
    const int64_t hi = d < m ? d : m;
    unsigned probes = 0, fallback = 0;
    int64_t res, pred = 0;
    // predict only where the bracket is a small part of the feasible range:
    // the prediction's reads and the two bracket tests cost about as much as
    // the three bisection steps they can save against a range of 8 brackets
    const bool predicted = c.mode != 0 && hi - lo > ((int64_t)8 << c.radius_log2);
    if (!predicted) {
        res = binary_corank<T>(A, B, d, lo, hi, probes);
    } else {
        pred = predict_corank(c, Akey, Bkey, m, k, d, pre);
        pred = pred < lo ? lo : (pred > hi ? hi : pred);
        const int64_t r = (int64_t)1 << c.radius_log2;
        const int64_t L = pred - r > lo ? pred - r : lo;
        const int64_t H = pred + r < hi ? pred + r : hi;
        // co-rank >= L  iff  L == lo or P(L-1);   co-rank <= H  iff  H == hi or !P(H)
        const bool okL = L == lo || !(B(d - L) < A(L - 1));
        const bool okH = H == hi || (B(d - 1 - H) < A(H));
        ++probes;
        if (okL && okH) {
            res = binary_corank<T>(A, B, d, L, H, probes);
        } else {
            fallback = 1;
            res = okL ? binary_corank<T>(A, B, d, H + 1, hi, probes)
                      : binary_corank<T>(A, B, d, lo, L - 1 > lo ? L - 1 : lo, probes);
        }
    }
    if (c.stats) {
        const unsigned long long err =
            (unsigned long long)(res > pred ? res - pred : pred - res);
        atomicAdd(c.stats + 0, 1ull);
        atomicAdd(c.stats + 1, (unsigned long long)probes);
        atomicAdd(c.stats + 8 + (probes < 63 ? probes : 63), 1ull);
        if (predicted) {
            atomicAdd(c.stats + 5, 1ull);
            atomicAdd(c.stats + 2, (unsigned long long)fallback);
            atomicAdd(c.stats + 3, err);
            atomicMax(c.stats + 4, err);
            const int bits = err ? 64 - __clzll((long long)err) : 0;
            atomicAdd(c.stats + 72 + (bits < 63 ? bits : 63), 1ull);
        }
    }
    return res;
}

// ------------------------------------------------------------ tile maps
//
// A tile map enumerates the output tiles of one merge pass.  Tile q belongs to
// a sequence (the whole array, or one segment) that starts at absolute index
// `base` of the arrays and holds `n` elements as sorted runs of `run`; `g` is
// the tile's index inside its sequence.  src/dst are absolute array pointers.

struct TileRef {
    int64_t base, n, g;
    const int32_t *ik, *iv;
    int32_t *ok, *ov;
};

struct PlainMap {
    const int32_t *ik, *iv;
    int32_t *ok, *ov;
    int64_t n, ntiles;
    __device__ __forceinline__ int64_t count() const { return ntiles; }
    __device__ __forceinline__ TileRef at(int64_t q) const
    {
        TileRef r;
        r.base = 0;
        r.n = n;
        r.g = q;
        r.ik = ik;
        r.iv = iv;
        r.ok = ok;
        r.ov = ov;
        return r;
    }
};

// Segmented pass p: tile list entries (segment, tile in segment); a
// segment's data sits in scratch or in the output depending on the parity of
// the passes it still has to run, so that its last pass writes the output.
// first_tiles (optional): the pass's tiles start at list position
// first_tiles[p] (a segmented four-way pass's two-way tiles follow its
// four-way ones).
struct SegMap {
    int32_t *outk, *outv, *scrk, *scrv;
    const int64_t *off;
    const int2 *tiles;
    const int32_t *passes;
    const int64_t *pass_tiles;
    const int64_t *first_tiles;
    int p;
    __device__ __forceinline__ int64_t first() const { return first_tiles ? first_tiles[p] : 0; }
    __device__ __forceinline__ int64_t count() const { return pass_tiles[p] - first(); }
    __device__ __forceinline__ int2 entry(int64_t q) const { return tiles[q + first()]; }
    __device__ __forceinline__ TileRef at(int64_t q) const
    {
        const int2 e = entry(q);
        TileRef r;
        r.base = off[e.x];
        r.n = off[e.x + 1] - r.base;
        r.g = e.y;
        const bool odd = (passes[e.x] - p) & 1;
        r.ik = odd ? scrk : outk;
        r.iv = odd ? scrv : outv;
        r.ok = odd ? outk : scrk;
        r.ov = odd ? outv : scrv;
        return r;
    }
};

// Pair geometry of a tile: pair base pb, run lengths alen/blen, diagonals.
struct PairGeo {
    int64_t pb, alen, blen, d0, d1, o0;
};

__device__ __forceinline__ PairGeo pair_geo(const TileRef &r, int64_t tm, int64_t run)
{
    PairGeo P;
    P.o0 = r.g * tm;
    const int64_t o1 = P.o0 + tm < r.n ? P.o0 + tm : r.n;
    P.pb = P.o0 & ~(2 * run - 1);
    P.alen = run < r.n - P.pb ? run : r.n - P.pb;
    const int64_t rest = r.n - P.pb - run;
    P.blen = rest <= 0 ? 0 : (rest < run ? rest : run);
    P.d0 = P.o0 - P.pb;
    P.d1 = o1 - P.pb;
    return P;
}

// A (key, value) element of two int32 arrays, compared without forming it:
// keys first, values only where the keys tie (the order of pack_pair: both
// words signed), so a co-rank probe on key-value runs reads 8 bytes, not 16,
// unless the keys are equal.
struct LazyPair {
    const int32_t *k, *v;
    int64_t i;
};
__device__ __forceinline__ bool operator<(const LazyPair &x, const LazyPair &y)
{
    const int32_t a = x.k[x.i], b = y.k[y.i];
    if (a != b)
        return a < b;
    return x.v[x.i] < y.v[y.i];
}

// The model's CDF at the first and last keys of a pair's runs A and B (the
// learned prediction's inputs, shared by every tile of the pair).
__device__ __forceinline__ float4 pair_cdf_of(const CorankCtl &c, const int32_t *ak, int64_t alen,
                                              const int32_t *bk, int64_t blen)
{
    auto f = [&](int32_t k) {
        return c.table ? cdf_lookup(c.table, k) : cdf_eval(c.cdf, key_to_unit(k));
    };
    const int32_t a0 = ak[0], a1 = ak[alen - 1];
    const int32_t b0 = blen ? bk[0] : a1, b1 = blen ? bk[blen - 1] : a1;
    return make_float4(f(a0), f(a1), f(b0), f(b1));
}

// Co-rank of a tile's first diagonal (one thread per tile).  pre: the pair's
// CDF values (pair_cdf_of), or nullptr.
template <typename T, typename Map>
__device__ __forceinline__ void tile_corank(const Map &map, int64_t q, int64_t run, int64_t tm,
                                            int64_t *__restrict__ cr, const CorankCtl &c,
                                            const float4 *pair_pre = nullptr)
{
    const TileRef r = map.at(q);
    const PairGeo P = pair_geo(r, tm, run);
    if (P.d0 == 0 || P.blen == 0) {
        cr[q] = P.d0 < P.alen ? P.d0 : P.alen;
        return;
    }
    const int32_t *ak = r.ik + r.base + P.pb, *bk = ak + run;
    const int32_t *av = r.iv ? r.iv + r.base + P.pb : nullptr;
    const int32_t *bv = av ? av + run : nullptr;
    auto Ak = [=](int64_t i) { return ak[i]; };
    auto Bk = [=](int64_t i) { return bk[i]; };
    // pairs start at multiples of 2 * run from the sequence start
    const float4 *pre = pair_pre ? pair_pre
                        : c.pair_cdf ? c.pair_cdf + (P.pb / (2 * run) - c.pair_first) : nullptr;
    if constexpr (sizeof(T) == 8) {
        auto A = [=](int64_t i) { return LazyPair{ak, av, i}; };
        auto B = [=](int64_t i) { return LazyPair{bk, bv, i}; };
        cr[q] = find_corank<T>(c, A, B, Ak, Bk, P.alen, P.blen, P.d0, pre);
    } else {
        auto A = [=](int64_t i) { return ak[i]; };
        auto B = [=](int64_t i) { return bk[i]; };
        cr[q] = find_corank<T>(c, A, B, Ak, Bk, P.alen, P.blen, P.d0, pre);
    }
}

// ------------------------------------------- persistent, pipelined merge pass
//
// Each workgroup walks a sequence of tiles and overlaps HBM with LDS work:
// while tile g is merged out of LDS, the A and B windows of its next tile
// are already in flight into registers (16-byte loads of the 4-element
// chunks, aligned in absolute index, that cover each window), and the
// co-ranks of the tile after that are loaded too.  Barriers fence LDS only,
// so the prefetch stays in flight across them.

__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

struct TileGeo {
    TileRef r;
    int64_t o0;     // first output index of the tile (sequence-relative)
    int64_t a_al;   // absolute index of the first chunk of the A window
    int64_t b_al;   // absolute index of the first chunk of the B window
    int cnt;        // outputs in the tile
    int acnt, bcnt; // window lengths
    int a_off;      // A window start - a_al
    int nA, nB;     // chunks covering the A and B windows
    int b_base;     // LDS index of B element 0
    int shift;      // (absolute first output) % 4: LDS offset of output 0
};

__device__ __forceinline__ TileGeo tile_geo(const TileRef &r, int64_t tm, int64_t run, int64_t c0,
                                            int64_t c1)
{
    TileGeo G;
    const PairGeo P = pair_geo(r, tm, run);
    auto clampc = [&](int64_t i, int64_t d) {
        const int64_t lo = d > P.blen ? d - P.blen : 0, hi = d < P.alen ? d : P.alen;
        return i < lo ? lo : (i > hi ? hi : i);
    };
    // Co-ranks are clamped to their feasible ranges and to i0 <= i1 <= i0 +
    // cnt, so every window stays inside its run even if the runs were not
    // sorted (garbage out, never an access out of bounds).
    const int64_t i0 = clampc(c0, P.d0);
    int64_t i1 = clampc(P.d1 == P.alen + P.blen ? P.alen : c1, P.d1);
    i1 = i1 < i0 ? i0 : (i1 > i0 + (P.d1 - P.d0) ? i0 + (P.d1 - P.d0) : i1);
    G.r = r;
    G.o0 = P.o0;
    G.cnt = (int)(P.d1 - P.d0);
    G.acnt = (int)(i1 - i0);
    G.bcnt = G.cnt - G.acnt;
    const int64_t abeg = r.base + P.pb + i0, bbeg = r.base + P.pb + run + (P.d0 - i0);
    G.a_al = abeg & ~(int64_t)3;
    G.b_al = bbeg & ~(int64_t)3;
    G.a_off = (int)(abeg - G.a_al);
    const int b_off = (int)(bbeg - G.b_al);
    G.nA = G.acnt ? (G.a_off + G.acnt + 3) >> 2 : 0;
    G.nB = G.bcnt ? (b_off + G.bcnt + 3) >> 2 : 0;
    G.b_base = 4 * G.nA + b_off;
    G.shift = (int)((r.base + P.o0) & 3);
    return G;
}

template <typename T> struct Chunk;
template <> struct Chunk<int32_t> {
    int4 k;
};
template <> struct Chunk<int64_t> {
    int4 k, v;
};

// The 4 elements at absolute index e (e % 4 == 0), one 16-byte load per
// array.  Callers keep e + 4 <= n_abs; the single ragged chunk at the end of
// an array whose length is not a multiple of 4 is patched by fix_tail.
template <typename T>
__device__ __forceinline__ Chunk<T> load_chunk(const int32_t *__restrict__ k,
                                               const int32_t *__restrict__ v, int64_t e)
{
    Chunk<T> c;
    c.k = *(const int4 *)(k + e);
    if constexpr (sizeof(T) == 8)
        c.v = *(const int4 *)(v + e);
    return c;
}

template <typename T>
__device__ __forceinline__ void fix_tail(Chunk<T> &c, const int32_t *__restrict__ k,
                                         const int32_t *__restrict__ v, int64_t e, int64_t n_abs)
{
    int kk[4], vv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        kk[q] = e + q < n_abs ? k[e + q] : 0x7fffffff;
        if constexpr (sizeof(T) == 8)
            vv[q] = e + q < n_abs ? v[e + q] : 0x7fffffff;
    }
    c.k = make_int4(kk[0], kk[1], kk[2], kk[3]);
    if constexpr (sizeof(T) == 8)
        c.v = make_int4(vv[0], vv[1], vv[2], vv[3]);
}

template <typename T> __device__ __forceinline__ void put_chunk(T *S, int c, const Chunk<T> &x)
{
    if constexpr (sizeof(T) == 4) {
        *(int4 *)(S + 4 * c) = x.k;
    } else {
        S[4 * c + 0] = pack_pair(x.k.x, x.v.x);
        S[4 * c + 1] = pack_pair(x.k.y, x.v.y);
        S[4 * c + 2] = pack_pair(x.k.z, x.v.z);
        S[4 * c + 3] = pack_pair(x.k.w, x.v.w);
    }
}

// n_abs: length of the arrays (for the ragged last chunk).  Arrays must be
// 16-byte aligned.
// Coalesced copy of the first cnt elements of a skewed LDS array to global
// index abs0 (a multiple of 4): thread t moves 16-byte chunks t, t + NT, ...
// The ragged last chunk is read like the others (its 4 slots exist in W) and
// only its stores are guarded, so it needs no addresses of its own.
template <int NT, int CH, typename T, bool PK = false>
__device__ __forceinline__ void copy_out(const LdsSkew<T> &W, int32_t *__restrict__ k,
                                         int32_t *__restrict__ v, int64_t abs0, int cnt, int t)
{
    constexpr int E = 16 / (int)sizeof(T);
    typedef T Vec __attribute__((ext_vector_type(E)));
#pragma unroll
    for (int q = 0; q < CH; ++q) {
        const int c = t + NT * q;
        if (4 * c >= cnt)
            continue;
        const int64_t e = abs0 + 4 * c;
        // W[4c] is 16-byte aligned in the skewed layout
        T x[4];
#pragma unroll
        for (int h = 0; h < 4; h += E) {
            const Vec y = *(const Vec *)&W[4 * c + h];
#pragma unroll
            for (int u = 0; u < E; ++u)
                x[h + u] = y[u];
        }
        if (4 * c + 4 <= cnt) {
            if constexpr (sizeof(T) == 4) {
                *(int4 *)(k + e) = make_int4(x[0], x[1], x[2], x[3]);
            } else if constexpr (PK) {
                typedef int64_t V2 __attribute__((ext_vector_type(2)));
                V2 *o = (V2 *)((int64_t *)k + e);
                o[0] = V2{x[0], x[1]};
                o[1] = V2{x[2], x[3]};
            } else {
                *(int4 *)(k + e) =
                    make_int4(pair_key(x[0]), pair_key(x[1]), pair_key(x[2]), pair_key(x[3]));
                *(int4 *)(v + e) =
                    make_int4(pair_val(x[0]), pair_val(x[1]), pair_val(x[2]), pair_val(x[3]));
            }
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (4 * c + u < cnt)
                    store_elem<T, PK>(k, v, e + u, x[u]);
        }
    }
}

// A tile whose outputs all come from one window (runs with disjoint key
// ranges, as in presorted input) is that window in order: copy it from
// position src of the staged windows.  Output x (0 <= x < cnt) goes to
// absolute index abs0 + shift + x, abs0 a multiple of 4; thread t moves
// 16-byte output chunks t, t + NT, ... and the ragged chunks at both ends
// element by element.  Applies the last pass's key map.  Reads stay inside
// the window: Z[src .. src + cnt).
template <int NT, int CH, typename T, bool PK, typename View>
__device__ __forceinline__ void copy_run(const View &Z, int src, int shift,
                                         int32_t *__restrict__ k, int32_t *__restrict__ v,
                                         int64_t abs0, int cnt, int t, KeyMap xout)
{
#pragma unroll
    for (int q = 0; q < CH; ++q) {
        const int c = t + NT * q;
        const int x0 = 4 * c - shift;  // output index of the chunk's first slot
        if (x0 >= cnt)
            continue;
        const int64_t e = abs0 + 4 * c;
        if (x0 >= 0 && x0 + 4 <= cnt) {
            T x[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                x[u] = Z[src + x0 + u];
            if (key_map_on(xout)) {  // wave-uniform: the last pass of a mapped sort
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    x[u] = map_elem(x[u], xout);
            }
            if constexpr (sizeof(T) == 4) {
                *(int4 *)(k + e) = make_int4(x[0], x[1], x[2], x[3]);
            } else if constexpr (PK) {
                typedef int64_t V2 __attribute__((ext_vector_type(2)));
                V2 *o = (V2 *)((int64_t *)k + e);
                o[0] = V2{x[0], x[1]};
                o[1] = V2{x[2], x[3]};
            } else {
                *(int4 *)(k + e) =
                    make_int4(pair_key(x[0]), pair_key(x[1]), pair_key(x[2]), pair_key(x[3]));
                *(int4 *)(v + e) =
                    make_int4(pair_val(x[0]), pair_val(x[1]), pair_val(x[2]), pair_val(x[3]));
            }
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (x0 + u >= 0 && x0 + u < cnt)
                    store_elem<T, PK>(k, v, e + u, map_elem(Z[src + x0 + u], xout));
        }
    }
}

// Register targets of the merge kernels: waves per SIMD that they fit
// without spilling (keys 4, or 2 at VT = 32; pairs 3).  A register over an
// allocation step costs a whole wave, so the target is stated, not left to
// the allocator.
template <typename T, int VT> constexpr int merge_waves_per_simd()
{
    return sizeof(T) == 8 ? 3 : (VT <= 16 ? 4 : 2);
}

// BIT: each thread merges its merge-path share with the bitonic network in
// registers (reg_merge) instead of the serial merge (the two mergers of
// Table 3; the serial one is the default).  PK: the output is one packed
// 64-bit array at the key pointer (the last pass of a 64-bit key sort).
template <int NT, int VT, typename T, typename Map, bool BIT = false, bool PK = false>
__device__ __forceinline__ void merge_pipe_body(const Map &map, int64_t run,
                                                const int64_t *__restrict__ cr, int64_t n_abs,
                                                int xcd_group, KeyMap xout = {})
{
    constexpr int TM = NT * VT;
    constexpr int CH = VT / 4 + 1;  // chunk slots per thread: TM/4 + 3 chunks at most
    // The windows: TM elements plus up to 6 of chunk alignment (plus VT - 1
    // read past a window's end by reg_merge), in the skewed layout: threads
    // whose shares lie VT apart (runs of equal keys, presorted input) then
    // hit 4-way instead of 16-way bank conflicts, and 16-byte chunks stay
    // aligned.  At VT = 32 the padding would cost the second workgroup per
    // CU, so that tile stays plain.
    constexpr bool SKEW = VT <= 16;
    using View = std::conditional_t<SKEW, LdsSkew<T>, LdsPlain<T>>;
    constexpr int SN = TM + 16 + (BIT ? VT : 0);
    __shared__ __attribute__((aligned(16))) T S[SKEW ? LdsSkew<T>::size(SN) : SN];
    const View Z{S, 0};
    const int t = threadIdx.x;
    const int64_t ntiles = map.count();

    // Tile order: plain round robin over workgroups, or (xcd_group) the
    // workgroups of one XCD (blockIdx % 8 when dispatch is round robin over
    // 8 XCDs) walk one contiguous eighth of the tiles, so neighbouring tiles
    // share window-boundary cache lines in that XCD's L2.
    int64_t first, step, last;
    if (xcd_group) {
        const int64_t nx = 8, x = blockIdx.x % nx, slot = blockIdx.x / nx;
        const int64_t slots = gridDim.x / nx;
        const int64_t per = (ntiles + nx - 1) / nx;
        first = x * per + slot;
        step = slots;
        last = (x + 1) * per < ntiles ? (x + 1) * per : ntiles;
    } else {
        first = blockIdx.x;
        step = gridDim.x;
        last = ntiles;
    }
    if (first >= last)
        return;

    // co-ranks of a tile and of its successor, as vector loads in lanes 0
    // and 1, so that waiting for them never waits for LDS traffic
    auto load_cr = [&](int64_t g) -> int64_t {
        const int64_t idx = g + (t & 1);
        return cr[idx < ntiles ? idx : ntiles - 1];
    };
    auto geo_of = [&](int64_t g, int64_t crv) {
        const int64_t c0 = (int64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)crv, 0) |
                           ((int64_t)__builtin_amdgcn_readlane((int)(crv >> 32), 0) << 32);
        const int64_t c1 = (int64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)crv, 1) |
                           ((int64_t)__builtin_amdgcn_readlane((int)(crv >> 32), 1) << 32);
        return tile_geo(map.at(g), TM, run, c0, c1);
    };

    // Chunk c of a tile: A chunks first, then B chunks.  Slots are guarded
    // per wavefront (uniform branch) and every lane loads from an in-bounds
    // address, so no two loads write the same registers on different paths
    // and the whole prefetch stays in flight.
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int64_t e_tail = n_abs & ~(int64_t)3;   // start of the ragged chunk
    const bool has_tail = (n_abs & 3) != 0;
    auto chunk_elem = [&](const TileGeo &G, int c) -> int64_t {
        return c < G.nA ? G.a_al + 4 * c : G.b_al + 4 * (c - G.nA);
    };
    Chunk<T> pf[CH];
    auto prefetch = [&](const TileGeo &G) {
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            if (NT * q + 64 * wave < G.nA + G.nB) {
                const int c = t + NT * q;
                int64_t e = c < G.nA + G.nB ? chunk_elem(G, c) : 0;
                e = (has_tail && e == e_tail) ? e_tail - 4 : e;
                pf[q] = load_chunk<T>(G.r.ik, G.r.iv, e);
            }
        }
    };

    int64_t g = first;
    TileGeo cur = geo_of(g, load_cr(g));
    prefetch(cur);
    int64_t crn = g + step < last ? load_cr(g + step) : 0;

    for (;;) {
        lds_barrier();  // the previous tile's store has read S
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            const int c = t + NT * q;
            if (c < cur.nA + cur.nB) {
                if (has_tail && chunk_elem(cur, c) == e_tail)
                    fix_tail<T>(pf[q], cur.r.ik, cur.r.iv, e_tail, n_abs);
                put_chunk<T>(&Z[4 * c], 0, pf[q]);
            }
        }
        lds_barrier();

        const int64_t gn = g + step;
        const bool more = gn < last;
        TileGeo nxt;
        if (more) {
            nxt = geo_of(gn, crn);
            prefetch(nxt);
            crn = gn + step < last ? load_cr(gn + step) : 0;
        }

        const View A{S, cur.a_off};
        const int boff = cur.b_base - cur.a_off;
        const int diag = t * VT < cur.cnt ? t * VT : cur.cnt;
        const int i = lds_corank(A, cur.acnt, boff, cur.bcnt, diag);
        T out[VT];
        if constexpr (BIT)
            reg_merge<VT>(A, cur.acnt, boff, cur.bcnt, i, diag - i, out);
        else  // windows are followed by chunk padding: reads one past stay in S
            serial_merge_open<VT>(A, cur.acnt, boff, cur.bcnt, i, diag - i, out);
        // the last pass of a uint32 / float32 sort maps the keys back: keys in
        // registers here, pairs where the packed pairs are split for the
        // store (each keeps the 16-byte stores and the register budget)
        if constexpr (sizeof(T) == 4) {
            if (key_map_on(xout)) {  // wave-uniform
#pragma unroll
                for (int k = 0; k < VT; ++k)
                    out[k] = map_elem(out[k], xout);
            }
        }
        lds_barrier();
#pragma unroll
        for (int k = 0; k < VT; ++k)
            Z[cur.shift + t * VT + k] = out[k];
        lds_barrier();

        // LDS index x holds output x - shift, i.e. absolute index
        // abs0 + x with abs0 = base + o0 - shift (a multiple of 4).
        const int64_t abs0 = cur.r.base + cur.o0 - cur.shift;
        const int end = cur.shift + cur.cnt;
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            const int c = t + NT * q;
            if (4 * c >= end)
                continue;
            const int64_t e = abs0 + 4 * c;
            if (4 * c >= cur.shift && 4 * c + 4 <= end) {
                if constexpr (sizeof(T) == 4) {
                    *(int4 *)(cur.r.ok + e) = *(const int4 *)&Z[4 * c];
                } else if constexpr (PK) {
                    typedef int64_t V2 __attribute__((ext_vector_type(2)));
                    V2 x0 = *(const V2 *)&Z[4 * c], x1 = *(const V2 *)&Z[4 * c + 2];
                    if (key_map_on(xout)) {  // wave-uniform
                        x0 = V2{map_elem(x0.x, xout), map_elem(x0.y, xout)};
                        x1 = V2{map_elem(x1.x, xout), map_elem(x1.y, xout)};
                    }
                    V2 *o = (V2 *)((int64_t *)cur.r.ok + e);
                    o[0] = x0;
                    o[1] = x1;
                } else {
                    const T x0 = Z[4 * c], x1 = Z[4 * c + 1], x2 = Z[4 * c + 2], x3 = Z[4 * c + 3];
                    int4 kk = make_int4(pair_key(x0), pair_key(x1), pair_key(x2), pair_key(x3));
                    *(int4 *)(cur.r.ov + e) =
                        make_int4(pair_val(x0), pair_val(x1), pair_val(x2), pair_val(x3));
                    if (key_map_on(xout))  // wave-uniform
                        kk = make_int4(key_map(kk.x, xout), key_map(kk.y, xout),
                                       key_map(kk.z, xout), key_map(kk.w, xout));
                    *(int4 *)(cur.r.ok + e) = kk;
                }
            } else {
#pragma unroll
                for (int q2 = 0; q2 < 4; ++q2)
                    if (4 * c + q2 >= cur.shift && 4 * c + q2 < end)
                        store_elem<T, PK>(cur.r.ok, cur.r.ov, e + q2,
                                          sizeof(T) == 8 ? map_elem(Z[4 * c + q2], xout)
                                                         : Z[4 * c + q2]);
            }
        }
        if (!more)
            break;
        g = gn;
        cur = nxt;
    }
}

}  // namespace hvms
