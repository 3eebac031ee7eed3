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

hipError_t launch_merge_pass(int tm, bool pairs, const int32_t *kin, const int32_t *vin,
                             int32_t *kout, int32_t *vout, int64_t n, int64_t run,
                             const int64_t *cr, hipStream_t s)
{
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
