// micro.hip -- microbenchmarks that measure the ceilings the raster's kernels are held against:
// HBM streaming bandwidth (a plain copy with 16-byte accesses) and the throughput of FP32 global
// atomic adds in the access patterns the backward's gradient flush issues. Measurement only: no
// step of the method runs here.
#include "device.hpp"
#include "internal.hpp"

namespace gsr {

// Grid-stride copy of n16 16-byte words: each wave instruction moves 1 KB, coalesced.
__global__ __launch_bounds__(256) void k_micro_copy(const uint4* __restrict__ src,
                                                    uint4* __restrict__ dst, size_t n16) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        dst[i] = src[i];
}

// per x GS_MICRO_THREADS FP32 atomic adds into slots[0 .. nslots) (nslots a power of two), each
// thread `per` of them:
//   MODE 0 (GS_MICRO_ATOMIC_SPREAD): add k of thread t goes to slot (t + k T) mod nslots with T
//     the thread count: consecutive lanes hit consecutive words, as the tile flush's slot-by-slot
//     adds do, and the address walks the whole buffer; the old value is not returned;
//   MODE 1 (GS_MICRO_ATOMIC_SPREAD_RETURN): the same with the old value returned and consumed,
//     as the compensated flush's first add;
//   MODE 2 (GS_MICRO_ATOMIC_WAVE_SAME): all lanes of a wave add to one word per instruction (the
//     per-fragment atomics of the naive reduction when one splat covers the wave).
// One instance per mode, so that each compiles to its own form of the atomic (with one kernel,
// the returning form served both the returning and the non-returning mode).
// The values added are exact in FP32 (1/64), so the slots' sums are checkable.
template <int MODE>
__global__ __launch_bounds__(256) void k_micro_atomic(float* __restrict__ slots, uint32_t mask,
                                                      int per, float* __restrict__ sink) {
    const uint32_t T = gridDim.x * blockDim.x;
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    float acc = 0.f;
    for (int k = 0; k < per; ++k) {
        uint32_t i;
        if constexpr (MODE == 2) i = ((t >> 6) + (uint32_t)k * (T >> 6)) & mask;
        else i = (t + (uint32_t)k * T) & mask;
        if constexpr (MODE == 1) acc += unsafeAtomicAdd(slots + i, 1.0f / 64.0f);
        else unsafeAtomicAdd(slots + i, 1.0f / 64.0f);
    }
    if (MODE == 1 && acc == -1.0f) sink[0] = acc;      // keeps the returned values live
}

hipError_t launch_micro_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
    const size_t n16 = bytes / 16;
    if (n16 == 0) return hipSuccess;
    const size_t blocks = (n16 + 255) / 256 < 256 * 64 ? (n16 + 255) / 256 : 256 * 64;
    hipLaunchKernelGGL(k_micro_copy, dim3((unsigned)blocks), dim3(256), 0, s,
                       (const uint4*)src, (uint4*)dst, n16);
    return hipGetLastError();
}

hipError_t launch_micro_atomic(float* slots, size_t nslots, int per, int mode, hipStream_t s) {
    if (per == 0) return hipSuccess;
    const dim3 g(GS_MICRO_THREADS / 256), b(256);
    const uint32_t mask = (uint32_t)(nslots - 1);
    if (mode == 0) hipLaunchKernelGGL(k_micro_atomic<0>, g, b, 0, s, slots, mask, per, slots);
    else if (mode == 1) hipLaunchKernelGGL(k_micro_atomic<1>, g, b, 0, s, slots, mask, per, slots);
    else hipLaunchKernelGGL(k_micro_atomic<2>, g, b, 0, s, slots, mask, per, slots);
    return hipGetLastError();
}

}  // namespace gsr
