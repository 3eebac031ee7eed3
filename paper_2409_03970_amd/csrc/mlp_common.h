// Device side of the learned key-CDF model shared by the training kernels
// and the co-rank predictor: the fp32 forward pass, the key -> unit-interval
// map and the counter-based SplitMix64 generator.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hvms {

// Parameter layout (floats): W1[32] b1[32] W2[32][32] (row = output unit)
// b2[32] W3[32] b3.  F(x) = W3 . relu(W2 relu(W1 x + b1) + b2) + b3.
__device__ __forceinline__ float cdf_eval(const float *__restrict__ p, float x)
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

// The model sampled at 2^16 + 1 points of the unit interval (one launch per
// sort): F at a key is then the linear interpolation between the two table
// entries around it, two loads from a 256 KiB table instead of a 1153-weight
// evaluation.  An approximation of the model used only for predictions,
// which the exact search corrects.
constexpr int kCdfTableSteps = 1 << 16;

__device__ __forceinline__ float cdf_lookup(const float *__restrict__ table, int32_t k)
{
    const uint32_t u = (uint32_t)k ^ 0x80000000u;  // key + 2^31
    const uint32_t hi = u >> 16;
    const float f = (float)(u & 0xffffu) * (1.0f / 65536.0f);
    const float a = table[hi], b = table[hi + 1];
    return fmaf(f, b - a, a);
}

// key -> (key + 2^31) / 2^32, rounded once to fp32.
__device__ __forceinline__ float key_to_unit(int32_t k)
{
    return (float)(((double)k + 2147483648.0) * (1.0 / 4294967296.0));
}

// Output number `counter` (from 0) of a SplitMix64 generator seeded with
// `seed`: the finaliser applied to seed + (counter + 1) * 0x9E3779B97F4A7C15.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t counter)
{
    uint64_t z = seed + (counter + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace hvms
