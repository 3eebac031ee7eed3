// Block sort: steps a1-a4 of the sort (Sec. 2.1-2.4).
//
// One workgroup of NT threads sorts a tile of R * NT elements:
//   a1  each wavefront loads 64 * R consecutive elements, lane l taking
//       elements l, l + 64, ... (every load instruction reads 256 contiguous
//       bytes; the column sort does not care which elements a lane holds);
//   a2  each lane sorts its R values in VGPRs with the column network;
//   a3  `wave_levels` cross-lane bitonic merge levels turn the 64 sorted
//       columns into runs of R * 2^wave_levels (the transpose + row merge of
//       the in-register sort, done in place by lane exchanges);
//   a4  the runs go to LDS in blocked order and `lds_levels` merge-path
//       levels merge them further, each thread producing R outputs by a
//       serial merge from its co-rank;
// then the tile is written back with coalesced stores.  Ragged tiles are
// padded with the maximum of the order.  PKM (64-bit elements only): bit 0,
// the input is one packed 64-bit array at kin; bit 1, so is the output;
// bit 2, each value is the element's input index (vin is not read).
#include "common.h"
#include "hvms_internal.h"

namespace hvms {

template <int R, int NT, typename T, int NET = 0, int PKM = 0>
__global__ __launch_bounds__(NT) void block_sort_kernel(const int32_t *__restrict__ kin,
                                                        const int32_t *__restrict__ vin,
                                                        int32_t *__restrict__ kout,
                                                        int32_t *__restrict__ vout, int64_t n,
                                                        int wave_levels, int lds_levels,
                                                        bool blocked, KeyMap xin, KeyMap xout)
{
    constexpr int TILE = R * NT;
    constexpr bool PI = (PKM & 1) != 0, PO = (PKM & 2) != 0, IO = (PKM & 4) != 0;
    __shared__ __attribute__((aligned(16))) T S[LdsSkew<T>::size(TILE)];
    const LdsSkew<T> Z{S, 0};
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int64_t tile0 = (int64_t)blockIdx.x * TILE;
    const int64_t wave0 = tile0 + (int64_t)wave * (64 * R);

    T v[R];
    if (blocked) {
        // Runs shorter than the tile must be consecutive input elements, so
        // lane l needs elements R*l .. R*l+R-1 of its wave's slice: stage the
        // tile through LDS with coalesced loads, then read it back blocked.
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int64_t g = tile0 + t + NT * j;
            Z[t + NT * j] =
                g < n ? map_elem(load_elem<T, PI, IO>(kin, vin, g), xin) : Traits<T>::kMax;
        }
        __syncthreads();
        const LdsSkew<T> W{S, wave * (64 * R) + logical_lane(lane) * R};
#pragma unroll
        for (int r = 0; r < R; ++r)
            v[r] = W[r];
        __syncthreads();
    } else if (tile0 + TILE <= n) {
        if constexpr (!PI && !IO) {
            // buffer loads: a lane offset plus a wave-uniform one per element
            const TileIO<T> io(kin + tile0, vin ? vin + tile0 : nullptr, TILE);
            const int wb = __builtin_amdgcn_readfirstlane(wave) * (64 * R);
#pragma unroll
            for (int j = 0; j < R; ++j)
                v[j] = io.load(lane, wb + 64 * j);
        } else {
#pragma unroll
            for (int j = 0; j < R; ++j)
                v[j] = load_elem<T, PI, IO>(kin, vin, wave0 + 64 * j + lane);
        }
        if (key_map_on(xin)) {  // wave-uniform
#pragma unroll
            for (int j = 0; j < R; ++j)
                v[j] = map_elem(v[j], xin);
        }
        // a presorted tile is stored as loaded, a reverse-sorted one reversed
        // (exact: equal elements are identical); block-uniform branches
        const int ord = tile_order<R, NT, T>(S, v, lane, wave);
        if (ord != 0) {
            const int64_t rel = (int64_t)wave * (64 * R) + lane;
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int64_t p = rel + 64 * j;
                store_elem<T, PO>(kout, vout, tile0 + (ord == 1 ? p : TILE - 1 - p),
                                  map_elem(v[j], xout));
            }
            return;
        }
        __syncthreads();  // S is the sort's from here
    } else {
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int64_t g = wave0 + 64 * j + lane;
            v[j] = g < n ? map_elem(load_elem<T, PI, IO>(kin, vin, g), xin) : Traits<T>::kMax;
        }
    }

    sort_tile_core<R, NT, T, NET>(S, v, t, wave_levels, lds_levels);

    if (tile0 + TILE <= n && !PO) {
        // element t + NT*j of the tile sits at a constant distance from
        // element t in the skewed layout (NT is a multiple of 16)
        const TileIO<T> io(kout + tile0, vout ? vout + tile0 : nullptr, TILE);
        const T *zt = S + LdsSkew<T>::pos(t);
        constexpr int ZS = LdsSkew<T>::size(NT);
        if (!key_map_on(xout)) {
#pragma unroll
            for (int j = 0; j < R; ++j)
                io.store(t, NT * j, zt[ZS * j]);
        } else {
#pragma unroll
            for (int j = 0; j < R; ++j)
                io.store(t, NT * j, map_elem(zt[ZS * j], xout));
        }
    } else if (tile0 + TILE <= n && !key_map_on(xout)) {
#pragma unroll
        for (int j = 0; j < R; ++j)
            store_elem<T, PO>(kout, vout, tile0 + t + NT * j, Z[t + NT * j]);
    } else if (tile0 + TILE <= n) {
#pragma unroll
        for (int j = 0; j < R; ++j)
            store_elem<T, PO>(kout, vout, tile0 + t + NT * j, map_elem(Z[t + NT * j], xout));
    } else {
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int64_t g = tile0 + t + NT * j;
            if (g < n)
                store_elem<T, PO>(kout, vout, g, map_elem(Z[t + NT * j], xout));
        }
    }
}

template <int R, int NT, typename T, int NET = 0, int PKM = 0>
static hipError_t launch_bs1(const int32_t *kin, const int32_t *vin, int32_t *kout, int32_t *vout,
                             int64_t n, int wave_levels, int lds_levels, bool blocked,
                             hipStream_t s, KeyMap xin, KeyMap xout)
{
    const int64_t tiles = (n + R * NT - 1) / (R * NT);
    hipLaunchKernelGGL((block_sort_kernel<R, NT, T, NET, PKM>), dim3((unsigned)tiles), dim3(NT), 0,
                       s, kin, vin, kout, vout, n, wave_levels, lds_levels, blocked, xin, xout);
    return hipGetLastError();
}

// Packed 64-bit arrays: a packed input with split output (the block stage
// of a longer sort) or packed on both sides (a sort of one tile).  Index
// values: the block stage of a stable sort by key.
template <int R, int NT, typename T, int NET = 0>
static hipError_t launch_bs(const int32_t *kin, const int32_t *vin, int32_t *kout, int32_t *vout,
                            int64_t n, int wave_levels, int lds_levels, bool blocked,
                            hipStream_t s, KeyMap xin, KeyMap xout)
{
    const int pkm = (xin.packed ? 1 : 0) | (xout.packed ? 2 : 0) | (xin.iota ? 4 : 0);
    if (pkm == 0)
        return launch_bs1<R, NT, T, NET>(kin, vin, kout, vout, n, wave_levels, lds_levels,
                                         blocked, s, xin, xout);
    if constexpr (sizeof(T) == 8) {
        switch (pkm) {
        case 1:
            return launch_bs1<R, NT, T, NET, 1>(kin, vin, kout, vout, n, wave_levels, lds_levels,
                                                blocked, s, xin, xout);
        case 3:
            return launch_bs1<R, NT, T, NET, 3>(kin, vin, kout, vout, n, wave_levels, lds_levels,
                                                blocked, s, xin, xout);
        case 4:
            return launch_bs1<R, NT, T, NET, 4>(kin, vin, kout, vout, n, wave_levels, lds_levels,
                                                blocked, s, xin, xout);
        }
    }
    return hipErrorInvalidValue;
}

bool block_sort_supported(int R, int NT, bool pairs)
{
    const bool r_ok = R == 8 || R == 16 || R == 32 || (R == 4 && !pairs);
    const bool nt_ok = NT == 256 || NT == 512 || NT == 1024;
    const long tile = (long)R * NT;
    const long lds = pairs ? LdsSkew<int64_t>::size(tile) * 8 : LdsSkew<int32_t>::size(tile) * 4;
    return r_ok && nt_ok && lds <= 163840;
}

hipError_t launch_block_sort(int R, int NT, bool pairs, const int32_t *kin, const int32_t *vin,
                             int32_t *kout, int32_t *vout, int64_t n, int wave_levels,
                             int lds_levels, bool blocked, hipStream_t s, int net, KeyMap xin,
                             KeyMap xout)
{
    if (net != 0) {  // the 16-input network ablation: keys, R = 16 only
        if (R != 16 || pairs || (net != 1 && net != 2))
            return hipErrorInvalidValue;
#define HVMS_BSN(NN)                                                                               \
    if (NT == NN)                                                                                  \
        return net == 1 ? launch_bs<16, NN, int32_t, 1>(kin, vin, kout, vout, n, wave_levels,     \
                                                        lds_levels, blocked, s, xin, xout)                   \
                        : launch_bs<16, NN, int32_t, 2>(kin, vin, kout, vout, n, wave_levels,     \
                                                        lds_levels, blocked, s, xin, xout);
        HVMS_BSN(256)
        HVMS_BSN(512)
        HVMS_BSN(1024)
#undef HVMS_BSN
        return hipErrorInvalidValue;
    }
#define HVMS_BS(RR, NN)                                                                         \
    if (R == RR && NT == NN) {                                                                  \
        if (pairs)                                                                              \
            return launch_bs<RR, NN, int64_t>(kin, vin, kout, vout, n, wave_levels, lds_levels, \
                                              blocked, s, xin, xout);                                               \
        return launch_bs<RR, NN, int32_t>(kin, vin, kout, vout, n, wave_levels, lds_levels, \
                                          blocked, s, xin, xout);                                         \
    }
    HVMS_BS(16, 256)
    HVMS_BS(16, 512)
    HVMS_BS(16, 1024)
    HVMS_BS(8, 256)
    HVMS_BS(8, 512)
    HVMS_BS(8, 1024)
    HVMS_BS(32, 256)
    HVMS_BS(32, 512)
    if (R == 4 && !pairs) {  // the smallest row of Table 2 (keys only)
        if (NT == 256)
            return launch_bs<4, 256, int32_t>(kin, vin, kout, vout, n, wave_levels, lds_levels,
                                              blocked, s, xin, xout);
        if (NT == 512)
            return launch_bs<4, 512, int32_t>(kin, vin, kout, vout, n, wave_levels, lds_levels,
                                              blocked, s, xin, xout);
        if (NT == 1024)
            return launch_bs<4, 1024, int32_t>(kin, vin, kout, vout, n, wave_levels, lds_levels,
                                               blocked, s, xin, xout);
    }
    if (R == 32 && NT == 1024 && !pairs)
        return launch_bs<32, 1024, int32_t>(kin, vin, kout, vout, n, wave_levels, lds_levels,
                                            blocked, s, xin, xout);
#undef HVMS_BS
    return hipErrorInvalidValue;
}

}  // namespace hvms
