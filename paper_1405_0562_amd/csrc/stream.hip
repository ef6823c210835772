// Streaming-read reference: the HBM read rate a kernel that only reads the
// input reaches on the same buffer, reported beside the matcher's rate as a
// second denominator next to the 8 TB/s peak.  Not a matching step.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <string>

#include "internal.h"

namespace {

constexpr uint32_t kReadBlock = 256;
constexpr int kMaxDevices = 64;
constexpr int kReadUnroll = 16;         // 16-byte loads in flight per thread

// The grid sweeps the input front to back: on each iteration block b reads
// the 64 KiB tile (iteration * blocks + b), so the blocks together cover one
// contiguous window.  Within a tile, consecutive lanes read consecutive
// 16-byte words (one load instruction of a wave covers 1 KiB) and each
// thread has kReadUnroll loads in flight before it uses any.  The XOR of all
// words (and of the tail bytes) is folded into *out, so no load can be
// dropped; each block adds one atomic (atomics on one address serialise,
// so the grid is kept to two blocks per CU).
__global__ __launch_bounds__(kReadBlock) void k_stream_read(const uint4 *in, uint64_t words, const uint8_t *tail,
                                                           uint32_t tail_bytes, uint32_t *out) {
    constexpr uint64_t tile = (uint64_t)kReadBlock * kReadUnroll;   // words per tile
    uint32_t acc = 0;
    uint64_t base = (uint64_t)blockIdx.x * tile;
    for (; base + tile <= words; base += (uint64_t)gridDim.x * tile) {
        uint4 r[kReadUnroll];
#pragma unroll
        for (int u = 0; u < kReadUnroll; ++u) r[u] = in[base + u * kReadBlock + threadIdx.x];
#pragma unroll
        for (int u = 0; u < kReadUnroll; ++u) acc ^= r[u].x ^ r[u].y ^ r[u].z ^ r[u].w;
    }
    if (base < words) {                     // the last, partial tile
        for (uint64_t i = base + threadIdx.x; i < words; i += kReadBlock) {
            const uint4 r = in[i];
            acc ^= r.x ^ r.y ^ r.z ^ r.w;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x < tail_bytes) acc ^= tail[threadIdx.x];
    for (int o = 32; o > 0; o >>= 1) acc ^= __shfl_xor(acc, o);
    __shared__ uint32_t s_wave[kReadBlock / 64];
    if ((threadIdx.x & 63) == 0) s_wave[threadIdx.x / 64] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t x = 0;
#pragma unroll
        for (uint32_t w = 0; w < kReadBlock / 64; ++w) x ^= s_wave[w];
        atomicXor(out, x);
    }
}

}  // namespace

extern "C" sfa_status sfa_stream_read(const uint8_t *d_in, uint64_t n, uint32_t *d_out, void *stream) {
    if (!d_out || (n && !d_in)) return sfa_fail(SFA_ERR_INVALID_ARG, "null argument");
    if ((uintptr_t)d_in & 15) return sfa_fail(SFA_ERR_INVALID_ARG, "input must be 16-byte aligned");
    if (n == 0) return SFA_OK;
    // CU count per device, queried once (the attribute query costs tens of
    // microseconds, more than the kernel on small inputs)
    static std::atomic<int> cu_count[kMaxDevices];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return sfa_fail(SFA_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return sfa_fail(SFA_ERR_INVALID_ARG, "device index out of range");
    int cus = cu_count[dev].load(std::memory_order_relaxed);
    if (cus == 0) {
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return sfa_fail(SFA_ERR_HIP, std::string("device query: ") + hipGetErrorString(e));
        cu_count[dev].store(cus, std::memory_order_relaxed);
    }
    const uint64_t words = n / 16;
    const uint32_t tail = (uint32_t)(n % 16);
    // two blocks per CU, fewer for short inputs (one tile each at least)
    const uint64_t tile = (uint64_t)kReadBlock * kReadUnroll;
    const uint64_t tiles = (words + tile - 1) / tile;
    const uint32_t blocks = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)cus * 2, tiles));
    hipLaunchKernelGGL(k_stream_read, dim3(blocks), dim3(kReadBlock), 0, (hipStream_t)stream, (const uint4 *)d_in,
                       words, d_in + words * 16, tail, d_out);
    e = hipGetLastError();
    if (e != hipSuccess) return sfa_fail(SFA_ERR_HIP, std::string("k_stream_read: ") + hipGetErrorString(e));
    return SFA_OK;
}
