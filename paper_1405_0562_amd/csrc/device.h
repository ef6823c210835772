// Device helpers shared by the HIP translation units of libsfa.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace sfa_dev {

// Copies n16 16-byte words from global memory to LDS; each thread has U
// loads in flight before it waits, so the copy costs one memory latency per
// U * blockDim.x words instead of one per word.  Indices past the end are
// clamped to the last word (a repeated copy of the same value), which keeps
// the loads unconditional and the staging array in registers.  The copy
// starts at word `rot` (mod n16), so blocks that stage the same table at the
// same time spread their requests over different memory channels.
template <int U = 8>
__device__ __forceinline__ void copy16(uint4 *dst, const uint4 *__restrict__ src, uint32_t n16, uint32_t rot = 0) {
    for (uint32_t base = threadIdx.x; base < n16; base += U * blockDim.x) {
        uint4 r[U];
        uint32_t j[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t i = min(base + u * blockDim.x, n16 - 1) + rot;
            j[u] = i >= n16 ? i - n16 : i;
            r[u] = src[j[u]];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) dst[j[u]] = r[u];
    }
}

}  // namespace sfa_dev
