// 64-bit payloads of a stable sort by key: after the keys have been sorted
// together with their input indices (the key-value sort with index values),
// one pass moves each payload to its key's place: dst[i] = src[idx[i]].
// Reads of idx and writes of dst are coalesced 16-byte accesses (4 indices,
// then 2 x 2 payloads per thread) when dst is 16-byte aligned; the payload
// reads follow the permutation.
#include "common.h"
#include "hvms_internal.h"

namespace hvms {

template <bool VEC>
__global__ __launch_bounds__(256) void gather_u64_kernel(const int32_t *__restrict__ idx,
                                                         const uint64_t *__restrict__ src,
                                                         uint64_t *__restrict__ dst, int64_t n)
{
    const int64_t i0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
    if (VEC && i0 + 4 <= n) {
        const int4 q = *(const int4 *)(idx + i0);
        typedef uint64_t V2 __attribute__((ext_vector_type(2)));
        V2 *o = (V2 *)(dst + i0);
        o[0] = V2{src[q.x], src[q.y]};
        o[1] = V2{src[q.z], src[q.w]};
    } else {
        const int64_t i1 = i0 + 4 < n ? i0 + 4 : n;
        for (int64_t i = i0; i < i1; ++i)
            dst[i] = src[idx[i]];
    }
}

hipError_t launch_gather_u64(const int32_t *idx, const uint64_t *src, uint64_t *dst, int64_t n,
                             hipStream_t s)
{
    // idx is a workspace buffer (256-byte aligned); dst is the caller's
    if (n <= 0)
        return hipSuccess;
    if ((uintptr_t)idx % 16)
        return hipErrorInvalidValue;
    const int64_t blocks = (n + 1023) / 1024;
    if ((uintptr_t)dst % 16 == 0)
        hipLaunchKernelGGL(gather_u64_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, s, idx,
                           src, dst, n);
    else
        hipLaunchKernelGGL(gather_u64_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, s,
                           idx, src, dst, n);
    return hipGetLastError();
}

}  // namespace hvms
