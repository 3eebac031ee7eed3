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
#include "common.h"
#include "hvms_internal.h"

namespace hvms {

// ------------------------------------------------------------ co-rank search

struct CorankCtl {
    int mode;          // HVMS_CORANK_*
    int radius_log2;   // bracket half-width for the bounded search
    const float *cdf;  // model parameters (learned mode)
    unsigned long long *stats;
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

// CDF model forward in fp32: 1 -> 32 -> 32 -> 1 with ReLU.
__device__ float cdf_eval(const float *__restrict__ p, float x)
{
    const float *W1 = p, *b1 = p + 32, *W2 = p + 64, *b2 = p + 64 + 1024, *W3 = p + 64 + 1024 + 32;
    const float b3 = p[64 + 1024 + 64];
    float h1[32];
#pragma unroll
    for (int u = 0; u < 32; ++u)
        h1[u] = fmaxf(fmaf(W1[u], x, b1[u]), 0.0f);
    float y = b3;
#pragma unroll 4
    for (int o = 0; o < 32; ++o) {
        float z = b2[o];
#pragma unroll
        for (int u = 0; u < 32; ++u)
            z = fmaf(W2[o * 32 + u], h1[u], z);
        y = fmaf(W3[o], fmaxf(z, 0.0f), y);
    }
    return y;
}

__device__ __forceinline__ float key_to_unit(int32_t k)
{
    return (float)((double)k + 2147483648.0) * (1.0f / 4294967296.0f);
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
                                  int64_t d)
{
    if (c.mode != 1 || m == 0 || k == 0)
        return (int64_t)((double)d * (double)m / (double)(m + k));
    float fa0 = cdf_eval(c.cdf, key_to_unit(Akey(0)));
    float fa1 = cdf_eval(c.cdf, key_to_unit(Akey(m - 1)));
    float fb0 = cdf_eval(c.cdf, key_to_unit(Bkey(0)));
    float fb1 = cdf_eval(c.cdf, key_to_unit(Bkey(k - 1)));
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
                               int64_t k, int64_t d)
{
    const int64_t lo = d > k ? d - k : 0;
    const int64_t hi = d < m ? d : m;
    unsigned probes = 0, fallback = 0;
    int64_t res, pred = 0;
    if (c.mode == 0 || hi - lo <= 2) {
        res = binary_corank<T>(A, B, d, lo, hi, probes);
    } else {
        pred = predict_corank(c, Akey, Bkey, m, k, d);
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
        if (c.mode != 0) {
            atomicAdd(c.stats + 2, (unsigned long long)fallback);
            atomicAdd(c.stats + 3, err);
            atomicMax(c.stats + 4, err);
        }
    }
    return res;
}

// Co-ranks of the first diagonal of every output tile of a merge pass.
template <typename T>
__global__ __launch_bounds__(256) void pass_corank_kernel(const int32_t *__restrict__ kin,
                                                          const int32_t *__restrict__ vin,
                                                          int64_t n, int64_t run, int64_t tm,
                                                          int64_t ntiles, int64_t *__restrict__ cr,
                                                          CorankCtl c)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ntiles)
        return;
    const int64_t o0 = g * tm;
    const int64_t pb = o0 & ~(2 * run - 1);
    const int64_t alen = run < n - pb ? run : n - pb;
    const int64_t rest = n - pb - run;
    const int64_t blen = rest <= 0 ? 0 : (rest < run ? rest : run);
    const int64_t d = o0 - pb;
    if (d == 0 || blen == 0) {
        cr[g] = d < alen ? d : alen;
        return;
    }
    const int32_t *ak = kin + pb, *bk = kin + pb + run;
    const int32_t *av = vin ? vin + pb : nullptr, *bv = vin ? vin + pb + run : nullptr;
    auto A = [=](int64_t i) { return load_elem<T>(ak, av, i); };
    auto B = [=](int64_t i) { return load_elem<T>(bk, bv, i); };
    auto Ak = [=](int64_t i) { return ak[i]; };
    auto Bk = [=](int64_t i) { return bk[i]; };
    cr[g] = find_corank<T>(c, A, B, Ak, Bk, alen, blen, d);
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

template <int NT, int VT, typename T>
__global__ __launch_bounds__(NT) void merge_pass_kernel(const int32_t *__restrict__ kin,
                                                        const int32_t *__restrict__ vin,
                                                        int32_t *__restrict__ kout,
                                                        int32_t *__restrict__ vout, int64_t n,
                                                        int64_t run, const int64_t *__restrict__ cr)
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
    const int i = lds_corank(S, acnt, acnt, bcnt, diag);
    T out[VT];
    serial_merge<VT>(S, acnt, acnt, bcnt, i, diag - i, out);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < VT; ++k)
        S[t * VT + k] = out[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < VT; ++k) {
        const int idx = t + NT * k;
        if (idx < cnt)
            store_elem<T>(kout, vout, o0 + idx, S[idx]);
    }
}

// ------------------------------------------- persistent, pipelined merge pass
//
// Same tiles and co-ranks as merge_pass_kernel, but each workgroup walks a
// sequence of tiles and overlaps HBM with LDS work: while tile g is merged
// out of LDS, the A and B windows of its next tile are already in flight
// into registers (16-byte loads of the 4-element chunks that cover each
// window), and the co-ranks of the tile after that are loaded too.  Barriers
// fence LDS only, so the prefetch stays in flight across them.

__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

struct TileGeo {
    int64_t o0;     // first output index of the tile
    int64_t a_al;   // A window start, rounded down to a 4-element chunk
    int64_t b_al;   // B window start, rounded down
    int cnt;        // outputs in the tile
    int acnt, bcnt; // window lengths
    int a_off;      // A window start - a_al
    int nA, nB;     // chunks covering the A and B windows
    int b_base;     // LDS index of B element 0
};

__device__ __forceinline__ TileGeo tile_geo(int64_t g, int64_t tm, int64_t n, int64_t run,
                                            int64_t c0, int64_t c1)
{
    TileGeo G;
    const int64_t o0 = g * tm;
    const int64_t o1 = o0 + tm < n ? o0 + tm : n;
    const int64_t pb = o0 & ~(2 * run - 1);
    const int64_t alen = run < n - pb ? run : n - pb;
    const int64_t rest = n - pb - run;
    const int64_t blen = rest <= 0 ? 0 : (rest < run ? rest : run);
    const int64_t d0 = o0 - pb, d1 = o1 - pb;
    auto clampc = [&](int64_t i, int64_t d) {
        const int64_t lo = d > blen ? d - blen : 0, hi = d < alen ? d : alen;
        return i < lo ? lo : (i > hi ? hi : i);
    };
    const int64_t i0 = clampc(c0, d0);
    int64_t i1 = clampc(d1 == alen + blen ? alen : c1, d1);
    i1 = i1 < i0 ? i0 : (i1 > i0 + (d1 - d0) ? i0 + (d1 - d0) : i1);
    G.o0 = o0;
    G.cnt = (int)(d1 - d0);
    G.acnt = (int)(i1 - i0);
    G.bcnt = G.cnt - G.acnt;
    const int64_t abeg = pb + i0, bbeg = pb + run + (d0 - i0);
    G.a_al = abeg & ~(int64_t)3;
    G.b_al = bbeg & ~(int64_t)3;
    G.a_off = (int)(abeg - G.a_al);
    const int b_off = (int)(bbeg - G.b_al);
    G.nA = G.acnt ? (G.a_off + G.acnt + 3) >> 2 : 0;
    G.nB = G.bcnt ? (b_off + G.bcnt + 3) >> 2 : 0;
    G.b_base = 4 * G.nA + b_off;
    return G;
}

template <typename T> struct Chunk;
template <> struct Chunk<int32_t> {
    int4 k;
};
template <> struct Chunk<int64_t> {
    int4 k, v;
};

// Chunk of the 4 elements starting at e (e % 4 == 0) with one 16-byte load
// per array.  The caller keeps e + 4 <= n; the single ragged chunk at the end
// of an array whose length is not a multiple of 4 is patched by fix_tail.
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
                                         const int32_t *__restrict__ v, int64_t e, int64_t n)
{
    int kk[4], vv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        kk[q] = e + q < n ? k[e + q] : 0x7fffffff;
        if constexpr (sizeof(T) == 8)
            vv[q] = e + q < n ? v[e + q] : 0x7fffffff;
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

template <int NT, int VT, typename T>
__global__ __launch_bounds__(NT) void merge_pass_pipe_kernel(
    const int32_t *__restrict__ kin, const int32_t *__restrict__ vin, int32_t *__restrict__ kout,
    int32_t *__restrict__ vout, int64_t n, int64_t run, const int64_t *__restrict__ cr,
    int64_t ntiles, int xcd_group)
{
    constexpr int TM = NT * VT;
    constexpr int CH = VT / 4 + 1;  // chunk slots per thread: TM/4 + 2 chunks at most
    __shared__ __attribute__((aligned(16))) T S[TM + 16];
    const int t = threadIdx.x;

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

    // co-ranks of a tile, as vector loads (lanes 0 and 1) so that waiting for
    // them never waits for LDS traffic
    auto load_cr = [&](int64_t g) -> int64_t {
        const int64_t idx = g + (t & 1);
        return cr[idx < ntiles ? idx : ntiles - 1];
    };
    auto geo_of = [&](int64_t g, int64_t crv) {
        const int64_t c0 = __builtin_amdgcn_readlane((int)(uint32_t)crv, 0) |
                           ((int64_t)__builtin_amdgcn_readlane((int)(crv >> 32), 0) << 32);
        const int64_t c1 = __builtin_amdgcn_readlane((int)(uint32_t)crv, 1) |
                           ((int64_t)__builtin_amdgcn_readlane((int)(crv >> 32), 1) << 32);
        return tile_geo(g, TM, n, run, c0, c1);
    };
    // Chunk c of a tile: A chunks first, then B chunks.  Slots are guarded
    // per wavefront (uniform branch) and every lane loads from an in-bounds
    // address, so no two loads ever write the same registers on different
    // paths and the prefetch stays in flight.
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int64_t e_tail = n & ~(int64_t)3;   // start of the ragged chunk
    const bool has_tail = (n & 3) != 0;
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
                pf[q] = load_chunk<T>(kin, vin, e);
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
                    fix_tail<T>(pf[q], kin, vin, e_tail, n);
                put_chunk<T>(S, c, pf[q]);
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

        const T *A = S + cur.a_off;
        const int boff = cur.b_base - cur.a_off;
        const int diag = t * VT < cur.cnt ? t * VT : cur.cnt;
        const int i = lds_corank(A, cur.acnt, boff, cur.bcnt, diag);
        T out[VT];
        serial_merge<VT>(A, cur.acnt, boff, cur.bcnt, i, diag - i, out);
        lds_barrier();
#pragma unroll
        for (int k = 0; k < VT; ++k)
            S[t * VT + k] = out[k];
        lds_barrier();

#pragma unroll
        for (int q = 0; q < VT / 4; ++q) {
            const int c = t + NT * q;
            const int64_t e = cur.o0 + 4 * c;
            if (4 * c >= cur.cnt)
                continue;
            if (4 * c + 4 <= cur.cnt) {
                if constexpr (sizeof(T) == 4) {
                    *(int4 *)(kout + e) = *(const int4 *)(S + 4 * c);
                } else {
                    const T x0 = S[4 * c], x1 = S[4 * c + 1], x2 = S[4 * c + 2], x3 = S[4 * c + 3];
                    *(int4 *)(kout + e) =
                        make_int4(pair_key(x0), pair_key(x1), pair_key(x2), pair_key(x3));
                    *(int4 *)(vout + e) =
                        make_int4(pair_val(x0), pair_val(x1), pair_val(x2), pair_val(x3));
                }
            } else {
#pragma unroll
                for (int q2 = 0; q2 < 4; ++q2)
                    if (4 * c + q2 < cur.cnt)
                        store_elem<T>(kout, vout, e + q2, S[4 * c + q2]);
            }
        }
        if (!more)
            break;
        g = gn;
        cur = nxt;
    }
}

// ------------------------------------------------------------- launchers

static CorankCtl make_ctl(const CorankOpts &o)
{
    CorankCtl c;
    c.mode = o.mode;
    c.radius_log2 = o.radius_log2;
    c.cdf = o.cdf;
    c.stats = o.stats;
    return c;
}

hipError_t launch_pass_corank(bool pairs, const int32_t *kin, const int32_t *vin, int64_t n,
                              int64_t run, int64_t tm, int64_t *cr, const CorankOpts &o,
                              hipStream_t s)
{
    const int64_t ntiles = (n + tm - 1) / tm;
    const unsigned blocks = (unsigned)((ntiles + 255) / 256);
    if (pairs)
        hipLaunchKernelGGL(pass_corank_kernel<int64_t>, dim3(blocks), dim3(256), 0, s, kin, vin,
                           n, run, tm, ntiles, cr, make_ctl(o));
    else
        hipLaunchKernelGGL(pass_corank_kernel<int32_t>, dim3(blocks), dim3(256), 0, s, kin,
                           nullptr, n, run, tm, ntiles, cr, make_ctl(o));
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
                            int64_t n, int64_t run, const int64_t *cr, hipStream_t s)
{
    const int64_t ntiles = (n + NT * VT - 1) / (NT * VT);
    hipLaunchKernelGGL((merge_pass_kernel<NT, VT, T>), dim3((unsigned)ntiles), dim3(NT), 0, s,
                       kin, vin, kout, vout, n, run, cr);
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

template <int NT, int VT, typename T>
static hipError_t launch_mpp(const int32_t *kin, const int32_t *vin, int32_t *kout, int32_t *vout,
                             int64_t n, int64_t run, const int64_t *cr, int occupancy, bool xcd,
                             hipStream_t s)
{
    const int64_t ntiles = (n + NT * VT - 1) / (NT * VT);
    int occ = occupancy;
    if (occ <= 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &occ, (const void *)merge_pass_pipe_kernel<NT, VT, T>, NT, 0) != hipSuccess ||
            occ <= 0)
            occ = 1;
    }
    int64_t grid = (int64_t)device_cus() * occ;
    if (grid > ntiles)
        grid = ntiles;
    if (xcd)
        grid = ((grid + 7) / 8) * 8;
    hipLaunchKernelGGL((merge_pass_pipe_kernel<NT, VT, T>), dim3((unsigned)grid), dim3(NT), 0, s,
                       kin, vin, kout, vout, n, run, cr, ntiles, xcd ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_merge_pass(int tm, bool pairs, const int32_t *kin, const int32_t *vin,
                             int32_t *kout, int32_t *vout, int64_t n, int64_t run,
                             const int64_t *cr, int variant, int occupancy, hipStream_t s)
{
    // The pipelined kernel moves 16-byte chunks: it needs 16-byte aligned
    // arrays and at least 16 elements; anything else takes the simple kernel.
    const bool aligned = ((uintptr_t)kin % 16 == 0) && ((uintptr_t)kout % 16 == 0) &&
                         (!pairs || (((uintptr_t)vin % 16 == 0) && ((uintptr_t)vout % 16 == 0)));
    if (variant != 1 && aligned && n >= 16) {
        const bool xcd = variant == 3;
        switch (tm) {
        case 2048:
            return pairs ? launch_mpp<256, 8, int64_t>(kin, vin, kout, vout, n, run, cr, occupancy, xcd, s)
                         : launch_mpp<256, 8, int32_t>(kin, vin, kout, vout, n, run, cr, occupancy, xcd, s);
        case 4096:
            return pairs ? launch_mpp<256, 16, int64_t>(kin, vin, kout, vout, n, run, cr, occupancy, xcd, s)
                         : launch_mpp<256, 16, int32_t>(kin, vin, kout, vout, n, run, cr, occupancy, xcd, s);
        case 8192:
            return pairs ? launch_mpp<512, 16, int64_t>(kin, vin, kout, vout, n, run, cr, occupancy, xcd, s)
                         : launch_mpp<512, 16, int32_t>(kin, vin, kout, vout, n, run, cr, occupancy, xcd, s);
        case 16384:
            if (!pairs)
                return launch_mpp<512, 32, int32_t>(kin, vin, kout, vout, n, run, cr, occupancy, xcd, s);
            break;
        }
        return hipErrorInvalidValue;
    }
    switch (tm) {
    case 2048:
        return pairs ? launch_mp<256, 8, int64_t>(kin, vin, kout, vout, n, run, cr, s)
                     : launch_mp<256, 8, int32_t>(kin, vin, kout, vout, n, run, cr, s);
    case 4096:
        return pairs ? launch_mp<256, 16, int64_t>(kin, vin, kout, vout, n, run, cr, s)
                     : launch_mp<256, 16, int32_t>(kin, vin, kout, vout, n, run, cr, s);
    case 8192:
        return pairs ? launch_mp<512, 16, int64_t>(kin, vin, kout, vout, n, run, cr, s)
                     : launch_mp<512, 16, int32_t>(kin, vin, kout, vout, n, run, cr, s);
    case 16384:
        if (!pairs)
            return launch_mp<512, 32, int32_t>(kin, vin, kout, vout, n, run, cr, s);
        break;
    }
    return hipErrorInvalidValue;
}

}  // namespace hvms
