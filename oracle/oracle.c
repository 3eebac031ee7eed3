/*
 * oracle.c -- plain, slow, obviously correct CPU reference for the results of
 * the hybrid vectorized merge sort ("A Hybrid Vectorized Merge Sort on ARM
 * NEON", arXiv 2409.03970).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or helper
 * with the HIP library.
 *
 * What the method computes has a plain definition (Sec. 2.1: sort N 32-bit
 * integers; the in-register sort, vectorized merge and parallel merge only
 * change how fast that result is reached), so the oracle is that definition
 * written out:
 *   - sort:           the nondecreasing arrangement of the input multiset,
 *                     signed 32-bit order;
 *   - sort of pairs:  the nondecreasing arrangement in lexicographic
 *                     (key, value) order, both signed;
 *   - other key types: the same with the type's own order (uint32/uint64
 *                     unsigned, float32/float64 IEEE 754 totalOrder,
 *                     int64 signed);
 *   - sort by key:    int32 keys with 64-bit payloads, keys nondecreasing,
 *                     equal keys in input order (stable);
 *   - segmented:      the above applied to each segment independently;
 *   - co-rank:        the number of elements of A among the first d outputs
 *                     of the merge of sorted A and B that takes A first on
 *                     ties (the partition point of the parallel merge of
 *                     Sec. 2.1);
 *   - 0-1 checks:     a comparator network sorts (merges) every input iff it
 *                     sorts (merges) every 0-1 input (Knuth's 0-1
 *                     principle), so the checks enumerate all such inputs.
 *
 * The sort is a top-down merge sort with one auxiliary buffer that takes the
 * left element on ties (stable); recursion depth is at most 63.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ keys */

static void msort_keys(int32_t *a, int32_t *aux, int64_t lo, int64_t hi)
{
    if (hi - lo < 2)
        return;
    int64_t mid = lo + (hi - lo) / 2;
    msort_keys(a, aux, lo, mid);
    msort_keys(a, aux, mid, hi);
    int64_t i = lo, j = mid, k = lo;
    while (i < mid && j < hi) {
        if (a[j] < a[i])
            aux[k++] = a[j++];
        else
            aux[k++] = a[i++];
    }
    while (i < mid)
        aux[k++] = a[i++];
    while (j < hi)
        aux[k++] = a[j++];
    memcpy(a + lo, aux + lo, (size_t)(hi - lo) * sizeof(int32_t));
}

/* Sorts a[0..n) ascending.  Returns 0, or -1 if n < 0 or memory runs out. */
int oracle_sort_i32(int32_t *a, int64_t n)
{
    if (n < 0)
        return -1;
    if (n < 2)
        return 0;
    int32_t *aux = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!aux)
        return -1;
    msort_keys(a, aux, 0, n);
    free(aux);
    return 0;
}

/* ----------------------------------------------------------------- pairs */

static int pair_less(int32_t ka, int32_t va, int32_t kb, int32_t vb)
{
    return ka < kb || (ka == kb && va < vb);
}

static void msort_pairs(int32_t *k, int32_t *v, int32_t *auxk, int32_t *auxv,
                        int64_t lo, int64_t hi)
{
    if (hi - lo < 2)
        return;
    int64_t mid = lo + (hi - lo) / 2;
    msort_pairs(k, v, auxk, auxv, lo, mid);
    msort_pairs(k, v, auxk, auxv, mid, hi);
    int64_t i = lo, j = mid, o = lo;
    while (i < mid && j < hi) {
        if (pair_less(k[j], v[j], k[i], v[i])) {
            auxk[o] = k[j];
            auxv[o++] = v[j++];
        } else {
            auxk[o] = k[i];
            auxv[o++] = v[i++];
        }
    }
    while (i < mid) {
        auxk[o] = k[i];
        auxv[o++] = v[i++];
    }
    while (j < hi) {
        auxk[o] = k[j];
        auxv[o++] = v[j++];
    }
    memcpy(k + lo, auxk + lo, (size_t)(hi - lo) * sizeof(int32_t));
    memcpy(v + lo, auxv + lo, (size_t)(hi - lo) * sizeof(int32_t));
}

/* Sorts the pairs (k[i], v[i]) lexicographically. */
int oracle_sort_pairs_i32(int32_t *k, int32_t *v, int64_t n)
{
    if (n < 0)
        return -1;
    if (n < 2)
        return 0;
    int32_t *auxk = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *auxv = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!auxk || !auxv) {
        free(auxk);
        free(auxv);
        return -1;
    }
    msort_pairs(k, v, auxk, auxv, 0, n);
    free(auxk);
    free(auxv);
    return 0;
}

/* ------------------------------------------- unsigned and float32 keys */

/*
 * Other 32-bit key types, each with the order written out directly:
 *   - uint32: unsigned order;
 *   - float32: the totalOrder predicate of IEEE 754-2008 (5.10) on the bit
 *     patterns: negative values (sign bit set) before positive ones; among
 *     positives the larger magnitude field (exponent and fraction read as
 *     one unsigned integer) is larger, among negatives it is smaller.  So
 *     -NaN < -inf < ... < -0 < +0 < ... < +inf < +NaN, NaNs ordered by
 *     payload.
 * Pairs carry a signed int32 value and order lexicographically (key, value).
 * The merge sort is the same top-down stable merge sort as above, with the
 * key comparison passed in.
 */
typedef int (*less32_fn)(uint32_t, uint32_t);

static int less_u32(uint32_t a, uint32_t b) { return a < b; }

static int less_f32_total(uint32_t a, uint32_t b)
{
    uint32_t sa = a >> 31, sb = b >> 31;
    if (sa != sb)
        return sa > sb;
    uint32_t ma = a & 0x7fffffffu, mb = b & 0x7fffffffu;
    return sa ? ma > mb : ma < mb;
}

static int gpair_less(less32_fn less, uint32_t ka, int32_t va, uint32_t kb, int32_t vb)
{
    if (less(ka, kb))
        return 1;
    if (less(kb, ka))
        return 0;
    return va < vb;
}

/* v may be NULL (keys only) */
static void msort_gen(less32_fn less, uint32_t *k, int32_t *v, uint32_t *auxk, int32_t *auxv,
                      int64_t lo, int64_t hi)
{
    if (hi - lo < 2)
        return;
    int64_t mid = lo + (hi - lo) / 2;
    msort_gen(less, k, v, auxk, auxv, lo, mid);
    msort_gen(less, k, v, auxk, auxv, mid, hi);
    int64_t i = lo, j = mid, o = lo;
    while (i < mid || j < hi) {
        int take_j;
        if (i == mid)
            take_j = 1;
        else if (j == hi)
            take_j = 0;
        else
            take_j = v ? gpair_less(less, k[j], v[j], k[i], v[i]) : less(k[j], k[i]);
        int64_t src = take_j ? j++ : i++;
        auxk[o] = k[src];
        if (v)
            auxv[o] = v[src];
        ++o;
    }
    memcpy(k + lo, auxk + lo, (size_t)(hi - lo) * sizeof(uint32_t));
    if (v)
        memcpy(v + lo, auxv + lo, (size_t)(hi - lo) * sizeof(int32_t));
}

static int sort_gen(less32_fn less, uint32_t *k, int32_t *v, int64_t n)
{
    if (n < 0)
        return -1;
    if (n < 2)
        return 0;
    uint32_t *auxk = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    int32_t *auxv = v ? (int32_t *)malloc((size_t)n * sizeof(int32_t)) : NULL;
    if (!auxk || (v && !auxv)) {
        free(auxk);
        free(auxv);
        return -1;
    }
    msort_gen(less, k, v, auxk, auxv, 0, n);
    free(auxk);
    free(auxv);
    return 0;
}

int oracle_sort_u32(uint32_t *k, int64_t n) { return sort_gen(less_u32, k, NULL, n); }
int oracle_sort_f32(uint32_t *bits, int64_t n) { return sort_gen(less_f32_total, bits, NULL, n); }
int oracle_sort_pairs_u32(uint32_t *k, int32_t *v, int64_t n)
{
    return sort_gen(less_u32, k, v, n);
}
int oracle_sort_pairs_f32(uint32_t *bits, int32_t *v, int64_t n)
{
    return sort_gen(less_f32_total, bits, v, n);
}

/* ------------------------------------------------------------ 64-bit keys */

/*
 * 64-bit keys, with the order written out for each type:
 *   - int64: signed order;
 *   - uint64: unsigned order;
 *   - float64: IEEE 754-2008 totalOrder (5.10) on the binary64 bit patterns,
 *     by the same rule as float32 above: sign bit set first; magnitudes (the
 *     63 bits below the sign, read as one unsigned integer) ascending among
 *     positives and descending among negatives.
 * Same stable top-down merge sort, on 64-bit words.
 */
typedef int (*less64_fn)(uint64_t, uint64_t);

static int less_i64(uint64_t a, uint64_t b) { return (int64_t)a < (int64_t)b; }

static int less_u64(uint64_t a, uint64_t b) { return a < b; }

static int less_f64_total(uint64_t a, uint64_t b)
{
    uint64_t sa = a >> 63, sb = b >> 63;
    if (sa != sb)
        return sa > sb;
    uint64_t ma = a & 0x7fffffffffffffffull, mb = b & 0x7fffffffffffffffull;
    return sa ? ma > mb : ma < mb;
}

static void msort64(less64_fn less, uint64_t *k, uint64_t *aux, int64_t lo, int64_t hi)
{
    if (hi - lo < 2)
        return;
    int64_t mid = lo + (hi - lo) / 2;
    msort64(less, k, aux, lo, mid);
    msort64(less, k, aux, mid, hi);
    int64_t i = lo, j = mid, o = lo;
    while (i < mid || j < hi) {
        int take_j;
        if (i == mid)
            take_j = 1;
        else if (j == hi)
            take_j = 0;
        else
            take_j = less(k[j], k[i]);
        aux[o++] = take_j ? k[j++] : k[i++];
    }
    memcpy(k + lo, aux + lo, (size_t)(hi - lo) * sizeof(uint64_t));
}

static int sort64(less64_fn less, uint64_t *k, int64_t n)
{
    if (n < 0)
        return -1;
    if (n < 2)
        return 0;
    uint64_t *aux = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    if (!aux)
        return -1;
    msort64(less, k, aux, 0, n);
    free(aux);
    return 0;
}

int oracle_sort_i64(uint64_t *k, int64_t n) { return sort64(less_i64, k, n); }
int oracle_sort_u64(uint64_t *k, int64_t n) { return sort64(less_u64, k, n); }
int oracle_sort_f64(uint64_t *bits, int64_t n) { return sort64(less_f64_total, bits, n); }

/* ------------------------------------------------------ 64-bit payloads */

/*
 * Stable sort by key with a 64-bit payload: the keys in nondecreasing signed
 * order, each payload moved with its key, equal keys in their input order.
 * The merge sort compares keys only and takes the left element on ties,
 * which is what makes it stable.
 */
static void msort_bykey(int32_t *k, uint64_t *v, int32_t *auxk, uint64_t *auxv, int64_t lo,
                        int64_t hi)
{
    if (hi - lo < 2)
        return;
    int64_t mid = lo + (hi - lo) / 2;
    msort_bykey(k, v, auxk, auxv, lo, mid);
    msort_bykey(k, v, auxk, auxv, mid, hi);
    int64_t i = lo, j = mid, o = lo;
    while (i < mid || j < hi) {
        int take_j;
        if (i == mid)
            take_j = 1;
        else if (j == hi)
            take_j = 0;
        else
            take_j = k[j] < k[i];
        int64_t src = take_j ? j++ : i++;
        auxk[o] = k[src];
        auxv[o] = v[src];
        ++o;
    }
    memcpy(k + lo, auxk + lo, (size_t)(hi - lo) * sizeof(int32_t));
    memcpy(v + lo, auxv + lo, (size_t)(hi - lo) * sizeof(uint64_t));
}

int oracle_sort_by_key_i32_p64(int32_t *k, uint64_t *v, int64_t n)
{
    if (n < 0)
        return -1;
    if (n < 2)
        return 0;
    int32_t *auxk = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    uint64_t *auxv = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    if (!auxk || !auxv) {
        free(auxk);
        free(auxv);
        return -1;
    }
    msort_bykey(k, v, auxk, auxv, 0, n);
    free(auxk);
    free(auxv);
    return 0;
}

/* ------------------------------------------------------------- segmented */

/* Segment s is k[offs[s] .. offs[s+1]); offsets must be nondecreasing. */
int oracle_segmented_sort_i32(int32_t *k, const int64_t *offs, int64_t nseg)
{
    for (int64_t s = 0; s < nseg; ++s) {
        if (offs[s + 1] < offs[s])
            return -1;
        if (oracle_sort_i32(k + offs[s], offs[s + 1] - offs[s]) != 0)
            return -1;
    }
    return 0;
}

int oracle_segmented_sort_pairs_i32(int32_t *k, int32_t *v, const int64_t *offs,
                                    int64_t nseg)
{
    for (int64_t s = 0; s < nseg; ++s) {
        if (offs[s + 1] < offs[s])
            return -1;
        if (oracle_sort_pairs_i32(k + offs[s], v + offs[s], offs[s + 1] - offs[s]) != 0)
            return -1;
    }
    return 0;
}

/* ----------------------------------------------------- merge and co-rank */

/* out[0..m+n) = merge of sorted A and B, taking A first on ties. */
void oracle_merge_i32(const int32_t *A, int64_t m, const int32_t *B, int64_t n,
                      int32_t *out)
{
    int64_t i = 0, j = 0, o = 0;
    while (i < m && j < n)
        out[o++] = (B[j] < A[i]) ? B[j++] : A[i++];
    while (i < m)
        out[o++] = A[i++];
    while (j < n)
        out[o++] = B[j++];
}

/* Number of elements of A among the first d outputs of that merge, found by
 * running the merge for d steps.  Returns -1 when d is outside [0, m+n]. */
int64_t oracle_corank_i32(const int32_t *A, int64_t m, const int32_t *B, int64_t n,
                          int64_t d)
{
    if (d < 0 || d > m + n)
        return -1;
    int64_t i = 0, j = 0;
    for (int64_t step = 0; step < d; ++step) {
        if (i < m && (j >= n || !(B[j] < A[i])))
            ++i;
        else
            ++j;
    }
    return i;
}

int64_t oracle_corank_pairs_i32(const int32_t *Ak, const int32_t *Av, int64_t m,
                                const int32_t *Bk, const int32_t *Bv, int64_t n,
                                int64_t d)
{
    if (d < 0 || d > m + n)
        return -1;
    int64_t i = 0, j = 0;
    for (int64_t step = 0; step < d; ++step) {
        if (i < m && (j >= n || !pair_less(Bk[j], Bv[j], Ak[i], Av[i])))
            ++i;
        else
            ++j;
    }
    return i;
}

/* ------------------------------------------------------ counting checks */

/* For a value x: *lt = #{a[i] < x}, *le = #{a[i] <= x}.  The p-th output of
 * the sort equals x exactly when lt <= p < le, which checks one sampled
 * output against the input without sorting it. */
void oracle_count_i32(const int32_t *a, int64_t n, int32_t x, int64_t *lt, int64_t *le)
{
    int64_t l = 0, e = 0;
    for (int64_t i = 0; i < n; ++i) {
        l += a[i] < x;
        e += a[i] <= x;
    }
    *lt = l;
    *le = e;
}

/* SplitMix64 finaliser (Steele, Lea, Flood 2014) used as a mixing function. */
static uint64_t mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Order-independent multiset hash: sum of mix64(key) modulo 2^64. */
uint64_t oracle_multiset_hash_i32(const int32_t *a, int64_t n)
{
    uint64_t h = 0;
    for (int64_t i = 0; i < n; ++i)
        h += mix64((uint64_t)(uint32_t)a[i]);
    return h;
}

/* Same for pairs, mixing key and value together. */
uint64_t oracle_multiset_hash_pairs_i32(const int32_t *k, const int32_t *v, int64_t n)
{
    uint64_t h = 0;
    for (int64_t i = 0; i < n; ++i)
        h += mix64(((uint64_t)(uint32_t)k[i] << 32) | (uint64_t)(uint32_t)v[i]);
    return h;
}

/* --------------------------------------------------- 0-1 network checks */

/* A network is a list of comparators (a, b): after it, wire a holds the
 * minimum and wire b the maximum of the two.  On 0-1 values min is AND and
 * max is OR, so 64 inputs are evaluated at once, one per bit of a word. */
static void apply_network01(uint64_t *w, const int32_t *comps, int64_t ncomp)
{
    for (int64_t c = 0; c < ncomp; ++c) {
        int32_t a = comps[2 * c], b = comps[2 * c + 1];
        uint64_t lo = w[a] & w[b], hi = w[a] | w[b];
        w[a] = lo;
        w[b] = hi;
    }
}

/* Bits of the inputs that end unsorted (a 1 on wire i above a 0 on i+1). */
static uint64_t unsorted01(const uint64_t *w, int32_t nwires)
{
    uint64_t bad = 0;
    for (int32_t i = 0; i + 1 < nwires; ++i)
        bad |= w[i] & ~w[i + 1];
    return bad;
}

static int popcount64(uint64_t x)
{
    int c = 0;
    while (x) {
        x &= x - 1;
        ++c;
    }
    return c;
}

/* Number of the 2^nwires 0-1 inputs that the network leaves unsorted
 * (0 means it is a sorting network).  1 <= nwires <= 32; -1 on bad args. */
int64_t oracle_network_failures01(const int32_t *comps, int64_t ncomp, int32_t nwires)
{
    if (nwires < 1 || nwires > 32)
        return -1;
    for (int64_t c = 0; c < 2 * ncomp; ++c)
        if (comps[c] < 0 || comps[c] >= nwires)
            return -1;
    /* Input x sets wire i to bit i of x.  Within a block of 64 consecutive
     * x the low six bits run through all patterns. */
    static const uint64_t low_bits[6] = {
        0xAAAAAAAAAAAAAAAAull, 0xCCCCCCCCCCCCCCCCull, 0xF0F0F0F0F0F0F0F0ull,
        0xFF00FF00FF00FF00ull, 0xFFFF0000FFFF0000ull, 0xFFFFFFFF00000000ull};
    uint64_t total = 1ull << nwires;
    uint64_t valid = nwires >= 6 ? ~0ull : ((1ull << total) - 1);
    int64_t failures = 0;
    uint64_t w[32];
    for (uint64_t base = 0; base < total; base += 64) {
        for (int32_t i = 0; i < nwires; ++i)
            w[i] = i < 6 ? low_bits[i] : (((base >> i) & 1) ? ~0ull : 0ull);
        apply_network01(w, comps, ncomp);
        failures += popcount64(unsorted01(w, nwires) & valid);
    }
    return failures;
}

/* Number of inputs, among the (p+1)(q+1) 0-1 inputs whose wires [0, p) and
 * [p, p+q) are each sorted, that the network leaves unsorted.  By the 0-1
 * principle a network that passes merges any two sorted runs of lengths p
 * and q.  Returns -1 on bad arguments. */
int64_t oracle_merging_network_failures01(const int32_t *comps, int64_t ncomp,
                                          int32_t p, int32_t q)
{
    if (p < 0 || q < 0 || p + q < 1)
        return -1;
    int32_t nw = p + q;
    for (int64_t c = 0; c < 2 * ncomp; ++c)
        if (comps[c] < 0 || comps[c] >= nw)
            return -1;
    uint64_t *w = (uint64_t *)malloc((size_t)nw * sizeof(uint64_t));
    if (!w)
        return -1;
    int64_t total = (int64_t)(p + 1) * (q + 1), failures = 0;
    for (int64_t base = 0; base < total; base += 64) {
        memset(w, 0, (size_t)nw * sizeof(uint64_t));
        uint64_t valid = 0;
        for (int s = 0; s < 64 && base + s < total; ++s) {
            int64_t id = base + s;
            int32_t z1 = (int32_t)(id / (q + 1)); /* zeros in the first run  */
            int32_t z2 = (int32_t)(id % (q + 1)); /* zeros in the second run */
            valid |= 1ull << s;
            for (int32_t i = z1; i < p; ++i)
                w[i] |= 1ull << s;
            for (int32_t i = z2; i < q; ++i)
                w[p + i] |= 1ull << s;
        }
        apply_network01(w, comps, ncomp);
        failures += popcount64(unsorted01(w, nw) & valid);
    }
    free(w);
    return failures;
}
